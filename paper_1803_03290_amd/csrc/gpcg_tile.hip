// The tile kernel of the batched "N-1" contingency PCG (gfx950, wave64, FP64).
//
// Layout.  Scenarios are grouped S to a tile; one wavefront carries its S
// scenario columns through the preconditioned CG of Section III.A.  Its 64
// lanes are R x S with R = 64 / S: lane = rs * S + sc treats scenario column
// sc and row slot rs.  Per wavefront the workspace holds four vectors: delta
// (the change of state from the base case) and p, interleaved as pairs
// {delta, p} per (row, column) because only the product sweep touches them
// and always together; r; and w, which holds in turn y (the forward-solve
// result), z (the backward-solve result) and q = A_c p (a row's z is last
// read as a look-ahead row, before the product writes its q).  Each is
// (n_r + 1) x S row-major (row n_r is scratch), so a wave touching one row
// of a vector reads S contiguous doubles, and every matrix entry it reads is
// shared by the S columns.  r and w are separate vectors rather than pairs:
// the backward and product sweeps touch only one of the two, and a half-pair
// access moves the whole pair's cache lines (on the 10,000-bus grid the
// separate vectors cut the sweeps' memory traffic by about a fifth and were
// 9 % faster at block 8).
//
// The outage of branch c = (f, t) is applied as a rank-1 correction of the
// shared base matrix: A_c = A - b_c u u^T with u = e_f - e_t (Section IV.B:
// four entries change), so no per-scenario matrix exists.  Islanded buses
// (a DFS pre-order interval of the bridge's far side) are held at zero.
//
// The triangular solves run through a schedule of steps of R independent
// rows each; values the next rows depend on are kept in an LDS ring of
// 2^k rows x S columns, sized on the host so that no live value is
// overwritten.
#include "gpcg_device.h"

#include <algorithm>
#include <climits>

namespace gpcg {
namespace {

// ---------------------------------------------------------------------------
// Sweeps.  Each sweep walks its program step by step through a register
// pipeline: a step's row record is loaded H = 2D steps ahead, its vector rows
// D steps ahead and its matrix entries ahead of those (shared by every wave,
// they sit in L1/L2; vector-memory counters retire in order, so the wait for
// a step's entries also waits for every older load).  A step first consumes
// its pipeline slots and then refills them with later steps, so no register
// is copied, no load waits on another load still in flight, and a step only
// waits on the LDS ring that carries the dependencies between rows.
//
// The entries and the row record of a step serve the S column lanes of
// each row slot alike.  Where a step's block (its entry chunks, then the
// records of a later step, packed so on the host) fits two loads per lane
// (S >= 4; the triangular sweeps at S = 2 too), each chunk is loaded once:
// lane l loads chunk l of the block, writes it to a per-wave LDS staging
// area, and every lane reads its slot's entries and record back from
// there, the entries LA steps before their step and the record one step
// before its vector rows are loaded.  This cuts the vector-memory
// instructions and lane traffic of the program data by the factor S (they
// had been the larger part of the sweeps' vector-memory work); LDS,
// otherwise lightly used, carries the copies.  Smaller blocks load each
// slot's record and entries per lane directly.
// Vector-memory counters complete in order, so the loop has no branches
// around loads and stores: idle slots read and write the tile's scratch row
// (row n_r; it holds r = 0 and p = 0, and q = 0 when the forward sweep reads
// it) and the ring's trash row, and padding entries are real zero entries
// pointing at the ring's zero row.
//
// A tile stores the pairs {delta, p}, r and w, each row-major with S
// columns: a wave's access to one vector row is S contiguous doubles (or
// pairs), and every sweep reads only the vectors it needs.  Vector bases are
// wave-uniform (scalar registers); a step computes one 32-bit offset for all
// of them (twice it for the pairs).
constexpr int kEntAheadTri = 8;    // steps the triangular solves load entries ahead (per-lane loads)
constexpr int kStageAheadTri = 8;  // steps a staged block is loaded before its LDS copy (triangular solves)
constexpr int kEntAheadProd = 2;  // steps the product loads entries ahead (direct form)

// The step index as a vector register the compiler cannot see through.
// Without it a wave-uniform index makes the loaded row id uniform too, and
// the compiler copies it to a scalar register right after the load, which
// waits for every load in flight.
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ double ring_at(const double *ring, int byte_off) {
    return *(const double *)((const char *)ring + byte_off);
}

__device__ __forceinline__ void ring_put(double *ring, int byte_off, double v) {
    *(double *)((char *)ring + byte_off) = v;
}

// A step's K entry records for this lane's slot, in 3 K / 4 sixteen-byte
// chunks: K / 2 chunks of two values each, then K / 4 chunks of four ring
// byte offsets.  Chunk c of every slot of a step is stored contiguously, so
// each chunk is one coalesced 16-byte load into an aligned register group.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef int ivec4 __attribute__((ext_vector_type(4)));

// Access-policy bits of the sweeps (see Tile).
constexpr int kStreamVec = 1, kGlobalVec = 2;

// A load of program data (records, entry chunks) under the same policy:
// with kGlobalVec through a global-memory pointer, as a native vector type
// (the 16-byte records are class objects, which do not load through one).
template <int NT, class V>
__device__ __forceinline__ V pload(const V *a) {
    if constexpr ((NT & kGlobalVec) != 0) {
        if constexpr (sizeof(V) == 16 && alignof(V) >= 16) {
            const ivec4 w = *(const __attribute__((address_space(1))) ivec4 *)a;
            V v;
            __builtin_memcpy(&v, &w, 16);
            return v;
        } else {
            return *(const __attribute__((address_space(1))) V *)a;
        }
    } else {
        return *a;
    }
}

template <int K>
struct Ents {
    static_assert(K % 4 == 0, "entry records come in 16-byte chunks");
    dvec2 v[K / 2];
    int4 o[K / 4];
    __device__ __forceinline__ double val(int j) const { return v[j / 2][j % 2]; }
    __device__ __forceinline__ int off(int j) const {
        const int4 &w = o[j / 4];
        return (j % 4 == 0) ? w.x : (j % 4 == 1) ? w.y : (j % 4 == 2) ? w.z : w.w;
    }
};

// Loads of a step's records through a slot pointer: the step's chunk 0 of
// slot rs (program base + (step * 3K/4) * R + rs), formed once per unrolled
// iteration so that every step's loads use constant offsets from it.
template <int S, int K>
__device__ __forceinline__ const int4 *ent_slot(const Program &g, int s, int rs) {
    constexpr int R = kWave / S;
    return g.ent + (size_t)s * (3 * K / 4) * R + rs;
}

template <int S, int K, int NT>
__device__ __forceinline__ void load_ents(Ents<K> &E, const int4 *p) {
    constexpr int R = kWave / S;
#pragma unroll
    for (int c = 0; c < K / 2; ++c) E.v[c] = pload<NT>((const dvec2 *)(p + c * R));
#pragma unroll
    for (int c = 0; c < K / 4; ++c) E.o[c] = pload<NT>(p + (K / 2 + c) * R);
}

// A step's ring values and entry values, gathered before the step's refill
// loads are issued so that the LDS reads are in flight meanwhile.
template <int K>
struct Gath {
    double r[K], v[K];
};

template <int K>
__device__ __forceinline__ void gather(Gath<K> &G, const Ents<K> &E, const double *ring, int lane_off) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
        G.r[j] = ring_at(ring, E.off(j) + lane_off);
        G.v[j] = E.val(j);
    }
}

// sum_j v_j * ring[col_j]
template <int K>
__device__ __forceinline__ double gdot(const Gath<K> &G) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) acc += G.v[j] * G.r[j];
    return acc;
}

// ---- staged blocks ---------------------------------------------------------
// A block of NB chunks (a step's NC = C R entry chunks, then R row records of
// a later step), loaded once each: load i of lane l takes chunk
// (i kWave + l) mod NB, so NL loads cover the block (lanes past NB repeat
// chunks of the same block and write them to unused staging rows).
// The staging area holds NL kWave chunks; a wave writes it and reads it back
// in program order, and its LDS instructions complete in order, so one area
// per wave serves every step.
template <int S, int K>
struct Stage {
    static constexpr int R = kWave / S, C = 3 * K / 4, NC = C * R;  // entry chunks of a step
    static constexpr int NB = stage_chunks(S, K);                    // block: entries, then R records
    static constexpr int NL = (NB + kWave - 1) / kWave;
    static constexpr bool kOn = staged(S, K);
};

// the chunks of a block lane l loads: i kWave + l, wrapped into the block
template <int S, int K>
struct StageLane {
    int j[Stage<S, K>::NL];
    __device__ __forceinline__ explicit StageLane(int lane) {
#pragma unroll
        for (int i = 0; i < Stage<S, K>::NL; ++i) j[i] = (i * kWave + lane) % Stage<S, K>::NB;
    }
};

template <int S, int K, int NT>
__device__ __forceinline__ void raw_load(ivec4 *q, const int4 *step_base, const StageLane<S, K> &L) {
#pragma unroll
    for (int i = 0; i < Stage<S, K>::NL; ++i) q[i] = pload<NT>((const ivec4 *)(step_base + L.j[i]));
}

template <int S, int K>
__device__ __forceinline__ void raw_put(int4 *stage, const ivec4 *q, int lane) {
#pragma unroll
    for (int i = 0; i < Stage<S, K>::NL; ++i) ((ivec4 *)stage)[i * kWave + lane] = q[i];
}

// entries of slot rs from the staging area (chunk c of slot rs at c R + rs)
template <int S, int K>
__device__ __forceinline__ void stage_read(Ents<K> &E, const int4 *stage, int rs) {
    constexpr int R = kWave / S;
#pragma unroll
    for (int c = 0; c < K / 2; ++c) E.v[c] = *(const dvec2 *)(stage + c * R + rs);
#pragma unroll
    for (int c = 0; c < K / 4; ++c) E.o[c] = stage[(K / 2 + c) * R + rs];
}

// A tile's vectors, each (n_r + 1) rows x S columns (row n_r is scratch):
// the {delta, p} pairs at xp, r, and w (y, then z, then q).  NT holds the
// policy bits of the sweeps' accesses: kStreamVec, the non-temporal hint
// on the vectors (below); kGlobalVec, vector and program accesses through
// global-memory pointers (the batch kernel reads its bases from a parameter
// array in memory, so the compiler cannot prove them global and would issue
// flat instructions, which also count against the LDS wait counter; the
// batch ran 2 % faster with the vectors cast, 7 % with the programs too).
template <int NT>
struct Tile {
    double *xp, *r, *w;
    double *v[kVectors];
    int nr;
    bool idle;  // this lane's column holds no scenario: the sweeps touch only its scratch row
};

// byte offset of (row, column sc) inside any vector of a tile (idle slots
// name the scratch row n_r)
template <int S, int NT>
__device__ __forceinline__ unsigned row_off(const Tile<NT> &T, int row, int sc) {
    return ((unsigned)row * S + sc) * 8u;
}

// the same inside the sweeps: a column without a scenario reads and writes
// its scratch row only (one cache line, so the finished columns of a wave
// cost no memory traffic while the others finish)
template <int S, int NT>
__device__ __forceinline__ unsigned sweep_off(const Tile<NT> &T, int row, int sc) {
    return ((unsigned)(T.idle ? T.nr : row) * S + sc) * 8u;
}

// Cache policy of the vector accesses.  A row of a vector is next touched
// one sweep later, after the wave has streamed through the whole vector and
// the other waves through theirs; where that is more than the Infinity
// Cache holds (4.3 GB on the 10,000-bus grid at block 16) no cache keeps
// it, and with kStreamVec the accesses carry the non-temporal hint,
// which leaves L2 to the matrix and factor entries that every wave reads
// (there: 0.47 TB less read traffic per launch and 3.7 % faster; the hint
// on loads or on stores alone made no difference).  The hint also streams
// the scratch row that idle columns write at every step, so it pays only
// while few columns idle.  The host takes it when the vectors exceed the
// Infinity Cache and the queue is ranked by an iteration record (idle
// overhead near 1.0), the ordinary policy otherwise (the first solve,
// ranked by the analytic key, sweeps about 1.3 times the busy columns and
// took 1.91 s instead of 1.57 s with the hint).
template <int NT, class V>
__device__ __forceinline__ V vload(const V *a) {
    if constexpr ((NT & kGlobalVec) != 0) {
        const __attribute__((address_space(1))) V *g = (const __attribute__((address_space(1))) V *)a;
        if constexpr ((NT & kStreamVec) != 0) return __builtin_nontemporal_load(g);
        else return *g;
    } else {
        if constexpr ((NT & kStreamVec) != 0) return __builtin_nontemporal_load(a);
        else return *a;
    }
}

template <int NT, class V>
__device__ __forceinline__ void vstore(V v, V *a) {
    if constexpr ((NT & kGlobalVec) != 0) {
        __attribute__((address_space(1))) V *g = (__attribute__((address_space(1))) V *)a;
        if constexpr ((NT & kStreamVec) != 0) __builtin_nontemporal_store(v, g);
        else *g = v;
    } else {
        if constexpr ((NT & kStreamVec) != 0) __builtin_nontemporal_store(v, a);
        else *a = v;
    }
}

// the pair {delta, p} at the element offset off of the other vectors
template <int NT>
__device__ __forceinline__ dvec2 xp_get(const Tile<NT> &T, unsigned off) {
    return vload<NT>((const dvec2 *)((const char *)T.xp + 2 * off));
}

template <int NT>
__device__ __forceinline__ void xp_put(const Tile<NT> &T, unsigned off, double x, double pv) {
    dvec2 w;
    w.x = x;
    w.y = pv;
    vstore<NT>(w, (dvec2 *)((char *)T.xp + 2 * off));
}

// r and w (y / z / q) at the element offset off, each in its own vector
template <int NT>
__device__ __forceinline__ dvec2 ry_get(const Tile<NT> &T, unsigned off) {
    dvec2 v;
    v.x = vload<NT>((const double *)((const char *)T.r + off));
    v.y = vload<NT>((const double *)((const char *)T.w + off));
    return v;
}

template <int NT>
__device__ __forceinline__ void ry_put(const Tile<NT> &T, unsigned off, double r, double y) {
    vstore<NT>(r, (double *)((char *)T.r + off));
    vstore<NT>(y, (double *)((char *)T.w + off));
}

template <int NT>
__device__ __forceinline__ double y_get(const Tile<NT> &T, unsigned off) {
    return vload<NT>((const double *)((const char *)T.w + off));
}

template <int NT>
__device__ __forceinline__ void y_put(const Tile<NT> &T, unsigned off, double y) {
    vstore<NT>(y, (double *)((char *)T.w + off));
}

// Programs end with kPadSteps idle steps, more than the deepest prefetch
// reads past the last real step, so the loads need neither a clamp nor a
// branch that would wait for them.
template <int S>
__device__ __forceinline__ const int4 *head_slot(const Program &g, int s, int rs) {
    constexpr int R = kWave / S;
    return g.rec + (size_t)s * R + rs;
}
// ---- triangular sweeps -----------------------------------------------------
// Consecutive steps of a triangular solve may depend on each other through
// the ring, so a step is split in two.  Part A is the chain: finish the ring
// dot product, form the row's value, write it to the ring and issue the next
// step's ring reads.  Part B holds the rest of the step (stores, the next
// step's right-hand side and carry, refills)
// and is issued while those reads are in flight.  The right-hand side enters
// as (rhs - carry) - dot, one subtraction on the chain.

// ring byte addresses of a step's entries for this lane
template <int K>
__device__ __forceinline__ void ring_addr(int (&a)[K], const Ents<K> &E, int lane_off) {
#pragma unroll
    for (int j = 0; j < K; ++j) a[j] = E.off(j) + lane_off;
}

template <int K>
__device__ __forceinline__ void ring_read(double (&r)[K], const int (&a)[K], const double *ring) {
#pragma unroll
    for (int j = 0; j < K; ++j) r[j] = ring_at(ring, a[j]);
}

// sum_j v_j * ring[col_j] as a pairwise tree (short dependency chain)
template <int K>
__device__ __forceinline__ double tree_dot(const double (&r)[K], const Ents<K> &E) {
    double acc[K / 2];
#pragma unroll
    for (int j = 0; j < K / 2; ++j)
        acc[j] = __builtin_fma(E.val(2 * j + 1), r[2 * j + 1], E.val(2 * j) * r[2 * j]);
#pragma unroll
    for (int w = 1; w < K / 2; w <<= 1)
#pragma unroll
        for (int j = 0; j + w < K / 2; j += 2 * w) acc[j] += acc[j + w];
    return acc[0];
}

// ---- forward: r -= alpha q, ||r||^2, y = L^-1 r, y' D^-1 y -----------------
// Its records are packed like the backward solve's, so that 1 / U_ii rides
// in them: with factors U = D L^T, y' D^-1 y = r' (L U)^-1 r = r'z.
struct FwdVec {
    double r, q;
};

template <int S, int NT>
__device__ __forceinline__ void fwd_vec(FwdVec &v, const int4 &h, const Tile<NT> &T, int sc) {
    const unsigned o = sweep_off<S>(T, h.x & kBwdRowMask, sc);  // packed record (see the backward solve)
    const dvec2 rq = ry_get(T, o);  // r and q (q sits where y and z were)
    v.r = rq.x;
    v.q = rq.y;
}

template <int S, int D, int NT>
__device__ __forceinline__ dvec2 fwd_sweep_direct(const Program &g, double *ring, const Tile<NT> &T, int rs, int sc,
                                                   double alpha) {
    constexpr int H = 2 * D, E = kEntAheadTri, K = kEntTri;
    static_assert(H % E == 0 && E >= 3, "entry slots must tile the unrolled loop");
    static_assert(2 * H - 1 <= kPadSteps, "prefetch past the last step must stay in the padding");
    constexpr int R = kWave / S, KE = K, C = 3 * K / 4;
    const int z0 = opaque(0);
    const int lane_off = sc * 8;
    if (rs == 0) ring_put(ring, g.ring * S * 8 + lane_off, 0.0);
    double rr = 0.0, carry = 0.0, rho = 0.0;
    int4 hq[H];
    FwdVec vq[D];
    Ents<K> eq[E];
    const int4 *hb0 = head_slot<S>(g, z0, rs);
#pragma unroll
    for (int d = 0; d < H; ++d) hq[d] = hb0[d * R];
#pragma unroll
    for (int d = 0; d < D; ++d) fwd_vec<S>(vq[d], hq[d], T, sc);
#pragma unroll
    for (int d = 0; d < E; ++d) load_ents<S, K, NT>(eq[d], ent_slot<S, K>(g, z0, rs) + d * C * R);
    int ga[K];
    double G[K];
    ring_addr(ga, eq[0], lane_off);
    ring_read(G, ga, ring);
    double r = vq[0].r - alpha * vq[0].q;  // step 0's residual row
    double rc = r;                         // ... minus its carry
    fwd_vec<S>(vq[0], hq[D], T, sc);
    for (int s0 = 0; s0 < g.steps; s0 += H) {
        const int sb = opaque(s0);  // step base: every address below is a constant offset from it
        const int4 *hb = head_slot<S>(g, sb, rs);
        const int4 *eb = ent_slot<S, KE>(g, sb, rs);
#pragma unroll
        for (int d = 0; d < H; ++d) {
            const int4 h = hq[d];
            // A
            const double dot = tree_dot(G, eq[d % E]);
            const double y = rc - dot;
            ring_put(ring, (int)(((unsigned)h.x >> kBwdRowBits) * (S * 8)) + lane_off, y);
            ring_addr(ga, eq[(d + 1) % E], lane_off);
            ring_read(G, ga, ring);
            __builtin_amdgcn_sched_barrier(0);
            // B
            {
                const unsigned o = sweep_off<S>(T, h.x & kBwdRowMask, sc);
                const bool cont = ((unsigned)h.y >> kBwdRowBits) == 2u;
                // a continuation's partial y is not stored: the scratch row's
                // w is read back as q by later idle slots of this sweep
                ry_put(T, o, r, cont ? 0.0 : y);
                rr = __builtin_fma(r, r, rr);
                // y' D^-1 y: 1 / U_ii is 0 for idle and continuation slots
                rho = __builtin_fma(y * __hiloint2double(h.w, h.z), y, rho);  // idle slots hold the scratch row's r = 0
                carry = cont ? carry + dot : 0.0;
                const FwdVec v = vq[(d + 1) % D];
                r = v.r - alpha * v.q;
                rc = r - carry;
            }
            load_ents<S, K, NT>(eq[d % E], eb + (d + E) * C * R);
            fwd_vec<S>(vq[(d + 1) % D], hq[(d + 1 + D) % H], T, sc);
            hq[d] = pload<NT>(hb + (d + H) * R);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    dvec2 out;
    out.x = rr;
    out.y = rho;
    return out;
}

template <int S, int D, int NT>
__device__ __forceinline__ dvec2 fwd_sweep_staged(const Program &g, double *ring, int4 *stage, const Tile<NT> &T,
                                                   int rs, int sc, double alpha) {
    constexpr int H = 2 * D, EQ = kStageAheadTri, K = kEntTri;
    using St = Stage<S, K>;
    constexpr int R = St::R, NC = St::NC, NB = St::NB, NL = St::NL;
    constexpr int NE = 4, LA = kStageLookTri;  // entry register slots; entries read from LDS LA steps ahead of use
    static_assert(H % EQ == 0 && H % NE == 0 && EQ >= 1, "entry slots must tile the unrolled loop");
    static_assert(2 * H - 1 <= kPadSteps && H - 1 + LA + EQ + 1 <= kPadSteps,
                  "prefetch past the last step must stay in the padding");
    static_assert(D == kPrefetchTri && LA + stage_rec_ahead(true) == D + 2 && D + 3 <= H,
                  "a block's records are those of step d + D + 2, read at step d (host packing)");
    static_assert(NE >= LA, "an entry slot is refilled only after its step has read it");
    const int lane = threadIdx.x;
    const StageLane<S, K> L(lane);
    const int z0 = opaque(0);
    const int lane_off = sc * 8;
    if (rs == 0) ring_put(ring, g.ring * S * 8 + lane_off, 0.0);
    double rr = 0.0, carry = 0.0, rho = 0.0;
    int4 hq[H];
    FwdVec vq[D];
    ivec4 q[EQ][NL];   // raw chunks of steps LA .. LA + EQ - 1 ahead
    Ents<K> eq[NE];    // entries of steps d .. d + LA
    const int4 *hb0 = head_slot<S>(g, z0, rs);
    const int4 *qb0 = g.ent + (size_t)z0 * NB;
#pragma unroll
    for (int d = 0; d < D + 2; ++d) hq[d] = hb0[d * R];  // later records arrive with the staged blocks
#pragma unroll
    for (int d = 0; d < D; ++d) fwd_vec<S>(vq[d], hq[d], T, sc);
#pragma unroll
    for (int d = 0; d < LA; ++d) {
        raw_load<S, K, NT>(q[0], qb0 + d * NB, L);
        raw_put<S, K>(stage, q[0], lane);
        stage_read<S, K>(eq[d], stage, rs);
    }
#pragma unroll
    for (int d = 0; d < EQ; ++d) raw_load<S, K, NT>(q[(d + LA) % EQ], qb0 + (d + LA) * NB, L);
    int ga[K];
    double G[K];
    ring_addr(ga, eq[0], lane_off);
    ring_read(G, ga, ring);
    double r = vq[0].r - alpha * vq[0].q;  // step 0's residual row
    double rc = r;                         // ... minus its carry
    fwd_vec<S>(vq[0], hq[D], T, sc);
    for (int s0 = 0; s0 < g.steps; s0 += H) {
        const int sb = opaque(s0);  // step base: every address below is a constant offset from it
        const int4 *qb = g.ent + (size_t)sb * NB;
#pragma unroll
        for (int d = 0; d < H; ++d) {
            const int4 h = hq[d];
            // A
            const double dot = tree_dot(G, eq[d % NE]);
            const double y = rc - dot;
            ring_put(ring, (int)(((unsigned)h.x >> kBwdRowBits) * (S * 8)) + lane_off, y);
            ring_addr(ga, eq[(d + 1) % NE], lane_off);
            ring_read(G, ga, ring);
            __builtin_amdgcn_sched_barrier(0);
            // B
            {
                const unsigned o = sweep_off<S>(T, h.x & kBwdRowMask, sc);
                const bool cont = ((unsigned)h.y >> kBwdRowBits) == 2u;
                ry_put(T, o, r, cont ? 0.0 : y);
                rr = __builtin_fma(r, r, rr);
                // y' D^-1 y: 1 / U_ii is 0 for idle and continuation slots
                rho = __builtin_fma(y * __hiloint2double(h.w, h.z), y, rho);
                carry = cont ? carry + dot : 0.0;
                const FwdVec v = vq[(d + 1) % D];
                r = v.r - alpha * v.q;
                rc = r - carry;
            }
            // step d + LA: raw chunks to LDS, its entries back into the slot
            // step d - 1 used; then the raw slot takes step d + LA + EQ
            raw_put<S, K>(stage, q[(d + LA) % EQ], lane);
            stage_read<S, K>(eq[(d + LA) % NE], stage, rs);
            hq[(d + D + 2) % H] = stage[NC + rs];  // the record of step (d + D + 2)
            raw_load<S, K, NT>(q[(d + LA) % EQ], qb + (d + LA + EQ) * NB, L);
            fwd_vec<S>(vq[(d + 1) % D], hq[(d + 1 + D) % H], T, sc);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    dvec2 out;
    out.x = rr;
    out.y = rho;
    return out;
}

// returns {||r||^2, y' D^-1 y} of this lane's rows
template <int S, int D, int NT>
__device__ __forceinline__ dvec2 fwd_sweep(const Program &g, double *ring, int4 *stage, const Tile<NT> &T, int rs,
                                           int sc, double alpha) {
    if constexpr (Stage<S, kEntTri>::kOn)
        return fwd_sweep_staged<S, D>(g, ring, stage, T, rs, sc, alpha);
    else
        return fwd_sweep_direct<S, D>(g, ring, T, rs, sc, alpha);
}

// ---- backward: z = U^-1 y, islanded rows zeroed on output, r'z ------------
// Its records are packed: {row | slot << 20, pre | (aux + 1) << 20, 1 / U_ii}.
__device__ __forceinline__ int bwd_row(const int4 &h) { return h.x & kBwdRowMask; }
__device__ __forceinline__ int bwd_pre(const int4 &h) { return h.y & kBwdRowMask; }
__device__ __forceinline__ bool bwd_cont(const int4 &h) { return ((unsigned)h.y >> kBwdRowBits) == 2u; }
__device__ __forceinline__ double bwd_dinv(const int4 &h) { return __hiloint2double(h.w, h.z); }
template <int S>
__device__ __forceinline__ int bwd_own(const int4 &h) {
    return (int)(((unsigned)h.x >> kBwdRowBits) * (S * 8));
}

struct BwdVec {
    double y, r;
};

// RZ: the sweep forms r'z (reads r); else only y
template <int S, bool RZ, int NT>
__device__ __forceinline__ void bwd_vec(BwdVec &v, const int4 &h, const Tile<NT> &T, int sc) {
    const unsigned o = sweep_off<S>(T, bwd_row(h), sc);
    if constexpr (RZ) {
        const dvec2 ry = ry_get(T, o);
        v.y = ry.y;
        v.r = ry.x;
    } else {
        v.y = y_get(T, o);
        v.r = 0.0;
    }
}
template <int S, int D, bool RZ, int NT>
__device__ __forceinline__ double bwd_sweep_direct(const Program &g, double *ring, const Tile<NT> &T, int rs, int sc,
                                                   int lo, int hi) {
    constexpr int H = 2 * D, E = kEntAheadTri, K = kEntTri;
    static_assert(H % E == 0 && E >= 3, "entry slots must tile the unrolled loop");
    static_assert(2 * H - 1 <= kPadSteps, "prefetch past the last step must stay in the padding");
    constexpr int R = kWave / S, KE = K, C = 3 * K / 4;
    const int z0 = opaque(0);
    const int lane_off = sc * 8;
    if (rs == 0) ring_put(ring, g.ring * S * 8 + lane_off, 0.0);
    double rz = 0.0, carry = 0.0;
    int4 hq[H];
    BwdVec vq[D];
    Ents<K> eq[E];
    const int4 *hb0 = head_slot<S>(g, z0, rs);
#pragma unroll
    for (int d = 0; d < H; ++d) hq[d] = hb0[d * R];
#pragma unroll
    for (int d = 0; d < D; ++d) bwd_vec<S, RZ>(vq[d], hq[d], T, sc);
#pragma unroll
    for (int d = 0; d < E; ++d) load_ents<S, K, NT>(eq[d], ent_slot<S, K>(g, z0, rs) + d * C * R);
    int ga[K];
    double G[K];
    ring_addr(ga, eq[0], lane_off);
    ring_read(G, ga, ring);
    double yc = vq[0].y, dv = bwd_dinv(hq[0]), r = vq[0].r;  // step 0's row
    bwd_vec<S, RZ>(vq[0], hq[D], T, sc);
    for (int s0 = 0; s0 < g.steps; s0 += H) {
        const int sb = opaque(s0);  // step base: every address below is a constant offset from it
        const int4 *hb = head_slot<S>(g, sb, rs);
        const int4 *eb = ent_slot<S, KE>(g, sb, rs);
#pragma unroll
        for (int d = 0; d < H; ++d) {
            const int4 h = hq[d];
            // A
            const double dot = tree_dot(G, eq[d % E]);
            const double z = (yc - dot) * dv;
            ring_put(ring, bwd_own<S>(h) + lane_off, z);
            ring_addr(ga, eq[(d + 1) % E], lane_off);
            ring_read(G, ga, ring);
            __builtin_amdgcn_sched_barrier(0);
            // B
            {
                const int row = bwd_row(h);
                const double zm = in_interval(bwd_pre(h), lo, hi) ? 0.0 : z;
                y_put(T, sweep_off<S>(T, row, sc), zm);
                rz = __builtin_fma(r, zm, rz);  // idle slots: r = 0 and 1/U_ii = 0
                carry = bwd_cont(h) ? carry + dot : 0.0;
                const BwdVec v = vq[(d + 1) % D];
                yc = v.y - carry;
                dv = bwd_dinv(hq[(d + 1) % H]);
                r = v.r;
            }
            load_ents<S, K, NT>(eq[d % E], eb + (d + E) * C * R);
            bwd_vec<S, RZ>(vq[(d + 1) % D], hq[(d + 1 + D) % H], T, sc);
            hq[d] = pload<NT>(hb + (d + H) * R);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    return rz;
}

template <int S, int D, bool RZ, int NT>
__device__ __forceinline__ double bwd_sweep_staged(const Program &g, double *ring, int4 *stage, const Tile<NT> &T,
                                                   int rs, int sc, int lo, int hi) {
    constexpr int H = 2 * D, EQ = kStageAheadTri, K = kEntTri;
    using St = Stage<S, K>;
    constexpr int R = St::R, NC = St::NC, NB = St::NB, NL = St::NL;
    constexpr int NE = 4, LA = kStageLookTri;
    static_assert(H % EQ == 0 && H % NE == 0 && EQ >= 1, "entry slots must tile the unrolled loop");
    static_assert(2 * H - 1 <= kPadSteps && H - 1 + LA + EQ + 1 <= kPadSteps,
                  "prefetch past the last step must stay in the padding");
    static_assert(D == kPrefetchTri && LA + stage_rec_ahead(true) == D + 2 && D + 3 <= H,
                  "a block's records are those of step d + D + 2, read at step d (host packing)");
    static_assert(NE >= LA, "an entry slot is refilled only after its step has read it");
    const int lane = threadIdx.x;
    const StageLane<S, K> L(lane);
    const int z0 = opaque(0);
    const int lane_off = sc * 8;
    if (rs == 0) ring_put(ring, g.ring * S * 8 + lane_off, 0.0);
    double rz = 0.0, carry = 0.0;
    int4 hq[H];
    BwdVec vq[D];
    ivec4 q[EQ][NL];
    Ents<K> eq[NE];
    const int4 *hb0 = head_slot<S>(g, z0, rs);
    const int4 *qb0 = g.ent + (size_t)z0 * NB;
#pragma unroll
    for (int d = 0; d < D + 2; ++d) hq[d] = hb0[d * R];  // later records arrive with the staged blocks
#pragma unroll
    for (int d = 0; d < D; ++d) bwd_vec<S, RZ>(vq[d], hq[d], T, sc);
#pragma unroll
    for (int d = 0; d < LA; ++d) {
        raw_load<S, K, NT>(q[0], qb0 + d * NB, L);
        raw_put<S, K>(stage, q[0], lane);
        stage_read<S, K>(eq[d], stage, rs);
    }
#pragma unroll
    for (int d = 0; d < EQ; ++d) raw_load<S, K, NT>(q[(d + LA) % EQ], qb0 + (d + LA) * NB, L);
    int ga[K];
    double G[K];
    ring_addr(ga, eq[0], lane_off);
    ring_read(G, ga, ring);
    double yc = vq[0].y, dv = bwd_dinv(hq[0]), r = vq[0].r;  // step 0's row
    bwd_vec<S, RZ>(vq[0], hq[D], T, sc);
    for (int s0 = 0; s0 < g.steps; s0 += H) {
        const int sb = opaque(s0);
        const int4 *qb = g.ent + (size_t)sb * NB;
#pragma unroll
        for (int d = 0; d < H; ++d) {
            const int4 h = hq[d];
            // A
            const double dot = tree_dot(G, eq[d % NE]);
            const double z = (yc - dot) * dv;
            ring_put(ring, bwd_own<S>(h) + lane_off, z);
            ring_addr(ga, eq[(d + 1) % NE], lane_off);
            ring_read(G, ga, ring);
            __builtin_amdgcn_sched_barrier(0);
            // B
            {
                const int row = bwd_row(h);
                const double zm = in_interval(bwd_pre(h), lo, hi) ? 0.0 : z;
                y_put(T, sweep_off<S>(T, row, sc), zm);
                rz = __builtin_fma(r, zm, rz);
                carry = bwd_cont(h) ? carry + dot : 0.0;
                const BwdVec v = vq[(d + 1) % D];
                yc = v.y - carry;
                dv = bwd_dinv(hq[(d + 1) % H]);
                r = v.r;
            }
            raw_put<S, K>(stage, q[(d + LA) % EQ], lane);
            stage_read<S, K>(eq[(d + LA) % NE], stage, rs);
            hq[(d + D + 2) % H] = stage[NC + rs];  // the record of step (d + D + 2)
            raw_load<S, K, NT>(q[(d + LA) % EQ], qb + (d + LA + EQ) * NB, L);
            bwd_vec<S, RZ>(vq[(d + 1) % D], hq[(d + 1 + D) % H], T, sc);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    return rz;
}

template <int S, int D, bool RZ, int NT>
__device__ __forceinline__ double bwd_sweep(const Program &g, double *ring, int4 *stage, const Tile<NT> &T, int rs,
                                            int sc, int lo, int hi) {
    if constexpr (Stage<S, kEntTri>::kOn)
        return bwd_sweep_staged<S, D, RZ>(g, ring, stage, T, rs, sc, lo, hi);
    else
        return bwd_sweep_direct<S, D, RZ>(g, ring, T, rs, sc, lo, hi);
}

// ---- product: on the look-ahead row delta += alpha p_old and p = z + beta
// p_old (into the ring and memory); on the current row q = A_c p from the
// ring with the outaged branch shielded, and p'q.  Natural row order.
struct ProdVec {
    double z, p, x;
};

template <int S, int NT>
__device__ __forceinline__ void prod_vec(ProdVec &v, const int4 &h, const Tile<NT> &T, int sc) {
    const unsigned o = sweep_off<S>(T, h.w, sc);  // look-ahead row (or the scratch row)
    v.z = y_get(T, o);
    const dvec2 xp = xp_get(T, o);
    v.x = xp.x;
    v.p = xp.y;
}

template <int S, int D, int NT>
__device__ __forceinline__ double prod_sweep_direct(const Program &g, double *ring, const Tile<NT> &T, int rs, int sc,
                                             double alpha, double beta, bool done, int lo, int hi, int ic, int jc,
                                             double bc) {
    constexpr int H = 2 * D, E = kEntAheadProd;
    static_assert(2 * H - 1 <= kPadSteps && E <= H, "prefetch past the last step must stay in the padding");
    constexpr int R = kWave / S, KE = kEntProd, C = 3 * kEntProd / 4;
    const int z0 = opaque(0);
    const int lane_off = sc * 8;
    const int wm = g.ring - 1;
    const int zero = g.ring * S * 8;
    const int trash = (g.ring + 1) * S * 8;
    if (rs == 0) ring_put(ring, zero + lane_off, 0.0);
    const int ic_off = ((ic >= 0) ? (ic & wm) * S * 8 : zero) + lane_off;
    const int jc_off = ((jc >= 0) ? (jc & wm) * S * 8 : zero) + lane_off;
    double pq = 0.0, carry = 0.0;
    int4 hq[H];
    ProdVec vq[D];
    Ents<kEntProd> eq[E];
    const int4 *hb0 = head_slot<S>(g, z0, rs);
#pragma unroll
    for (int d = 0; d < H; ++d) hq[d] = hb0[d * R];
#pragma unroll
    for (int d = 0; d < D; ++d) prod_vec<S>(vq[d], hq[d], T, sc);
#pragma unroll
    for (int d = 0; d < E; ++d) load_ents<S, kEntProd, NT>(eq[d], ent_slot<S, kEntProd>(g, z0, rs) + d * C * R);
    for (int s0 = 0; s0 < g.steps; s0 += H) {
        const int sb = opaque(s0);  // step base: every address below is a constant offset from it
        const int4 *hb = head_slot<S>(g, sb, rs);
        const int4 *eb = ent_slot<S, KE>(g, sb, rs);
#pragma unroll
        for (int d = 0; d < H; ++d) {
            const int4 h = hq[d];
            const ProdVec v = vq[d % D];
            // look-ahead row: pending solution update and new direction (its
            // ring write must precede this step's reads)
            const unsigned lo_ = sweep_off<S>(T, h.w, sc);
            const double pn = done ? v.p : v.z + beta * v.p;
            ring_put(ring, ((h.w < T.nr) ? (h.w & wm) * S * 8 : trash) + lane_off, pn);
            Gath<kEntProd> G;
            gather(G, eq[d % E], ring, lane_off);
            const double pf = ring_at(ring, ic_off), pt = ring_at(ring, jc_off);
            const double pown = ring_at(ring, h.y + lane_off);
            prod_vec<S>(vq[d % D], hq[(d + D) % H], T, sc);
            load_ents<S, kEntProd, NT>(eq[d % E], eb + (d + E) * C * R);
            hq[d] = pload<NT>(hb + (d + H) * R);
            {
                xp_put(T, lo_, v.x + alpha * v.p, pn);
                const double dot = gdot(G);
                const bool cont = h.z == -2;
                double qv = carry + dot;
                carry = cont ? carry + dot : 0.0;
                const double dpc = pf - pt;
                qv += (h.x == ic) ? -bc * dpc : ((h.x == jc) ? bc * dpc : 0.0);
                // a continuation's partial sum is not stored, so the scratch
                // row's q, as the forward sweep reads it, is exactly zero
                // (and with it its r); islanded rows are zero
                if (in_interval(h.z, lo, hi)) qv = 0.0;
                qv = cont ? 0.0 : qv;
                y_put(T, sweep_off<S>(T, h.x, sc), qv);  // z of this row was read as a look-ahead row
                pq = __builtin_fma(pown, qv, pq);  // idle slots read pown from the zero row
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    return pq;
}

template <int S, int D, int NT>
__device__ __forceinline__ double prod_sweep_staged(const Program &g, double *ring, int4 *stage, const Tile<NT> &T,
                                                    int rs, int sc, double alpha, double beta, bool done, int lo,
                                                    int hi, int ic, int jc, double bc) {
    constexpr int H = 2 * D, K = kEntProd;
    using St = Stage<S, K>;
    constexpr int R = St::R, NC = St::NC, NB = St::NB, NL = St::NL;
    constexpr int NE = 2, LA = kStageLookProd, EQ = 2;  // entry slots, LDS read-ahead, raw-load distance
    static_assert(H % EQ == 0 && H % NE == 0, "entry slots must tile the unrolled loop");
    static_assert(2 * H - 1 <= kPadSteps && H - 1 + LA + EQ + 1 <= kPadSteps,
                  "prefetch past the last step must stay in the padding");
    static_assert(D == kPrefetchProd && LA + stage_rec_ahead(false) == D + 1 && D + 2 <= H,
                  "a block's records are those of step d + D + 1, read at step d (host packing)");
    static_assert(NE >= LA, "an entry slot is refilled only after its step has read it");
    const int lane = threadIdx.x;
    const StageLane<S, K> L(lane);
    const int z0 = opaque(0);
    const int lane_off = sc * 8;
    const int wm = g.ring - 1;
    const int zero = g.ring * S * 8;
    const int trash = (g.ring + 1) * S * 8;
    if (rs == 0) ring_put(ring, zero + lane_off, 0.0);
    const int ic_off = ((ic >= 0) ? (ic & wm) * S * 8 : zero) + lane_off;
    const int jc_off = ((jc >= 0) ? (jc & wm) * S * 8 : zero) + lane_off;
    double pq = 0.0, carry = 0.0;
    int4 hq[H];
    ProdVec vq[D];
    ivec4 q[EQ][NL];
    Ents<K> eq[NE];
    const int4 *hb0 = head_slot<S>(g, z0, rs);
    const int4 *qb0 = g.ent + (size_t)z0 * NB;
#pragma unroll
    for (int d = 0; d < D + 1; ++d) hq[d] = hb0[d * R];  // later records arrive with the staged blocks
#pragma unroll
    for (int d = 0; d < D; ++d) prod_vec<S>(vq[d], hq[d], T, sc);
#pragma unroll
    for (int d = 0; d < LA; ++d) {
        raw_load<S, K, NT>(q[0], qb0 + d * NB, L);
        raw_put<S, K>(stage, q[0], lane);
        stage_read<S, K>(eq[d], stage, rs);
    }
#pragma unroll
    for (int d = 0; d < EQ; ++d) raw_load<S, K, NT>(q[(d + LA) % EQ], qb0 + (d + LA) * NB, L);
    for (int s0 = 0; s0 < g.steps; s0 += H) {
        const int sb = opaque(s0);  // step base: every address below is a constant offset from it
        const int4 *qb = g.ent + (size_t)sb * NB;
#pragma unroll
        for (int d = 0; d < H; ++d) {
            const int4 h = hq[d];
            const ProdVec v = vq[d % D];
            // look-ahead row: pending solution update and new direction (its
            // ring write must precede this step's reads)
            const unsigned lo_ = sweep_off<S>(T, h.w, sc);
            const double pn = done ? v.p : v.z + beta * v.p;
            ring_put(ring, ((h.w < T.nr) ? (h.w & wm) * S * 8 : trash) + lane_off, pn);
            Gath<K> G;
            gather(G, eq[d % NE], ring, lane_off);
            const double pf = ring_at(ring, ic_off), pt = ring_at(ring, jc_off);
            const double pown = ring_at(ring, h.y + lane_off);
            prod_vec<S>(vq[d % D], hq[(d + D) % H], T, sc);
            // step d + LA: raw chunks to LDS, its entries into the slot this
            // step's gather has read; the raw slot takes step d + LA + EQ
            raw_put<S, K>(stage, q[(d + LA) % EQ], lane);
            stage_read<S, K>(eq[(d + LA) % NE], stage, rs);
            hq[(d + D + 1) % H] = stage[NC + rs];  // the record of step (d + D + 1)
            raw_load<S, K, NT>(q[(d + LA) % EQ], qb + (d + LA + EQ) * NB, L);

            {
                xp_put(T, lo_, v.x + alpha * v.p, pn);
                const double dot = gdot(G);
                const bool cont = h.z == -2;
                double qv = carry + dot;
                carry = cont ? carry + dot : 0.0;
                const double dpc = pf - pt;
                qv += (h.x == ic) ? -bc * dpc : ((h.x == jc) ? bc * dpc : 0.0);
                // a continuation's partial sum is not stored, so the scratch
                // row's q, as the forward sweep reads it, is exactly zero
                // (and with it its r); islanded rows are zero
                if (in_interval(h.z, lo, hi)) qv = 0.0;
                qv = cont ? 0.0 : qv;
                y_put(T, sweep_off<S>(T, h.x, sc), qv);  // z of this row was read as a look-ahead row
                pq = __builtin_fma(pown, qv, pq);  // idle slots read pown from the zero row
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    return pq;
}

template <int S, int D, int NT>
__device__ __forceinline__ double prod_sweep(const Program &g, double *ring, int4 *stage, const Tile<NT> &T, int rs,
                                             int sc, double alpha, double beta, bool done, int lo, int hi, int ic,
                                             int jc, double bc) {
    if constexpr (Stage<S, kEntProd>::kOn)
        return prod_sweep_staged<S, D>(g, ring, stage, T, rs, sc, alpha, beta, done, lo, hi, ic, jc, bc);
    else
        return prod_sweep_direct<S, D>(g, ring, T, rs, sc, alpha, beta, done, lo, hi, ic, jc, bc);
}

// delta += alpha p over every row (the update the product sweep would have
// made next, applied once the tile stops)
template <int S, int NT>
__device__ __forceinline__ void final_update(const Tile<NT> &T, int rs, int sc, double alpha) {
    constexpr int R = kWave / S;
    for (int i = rs; i < T.nr; i += R) {
        const unsigned o = sweep_off<S>(T, i, sc);
        const dvec2 xp = xp_get(T, o);
        xp_put(T, o, xp.x + alpha * xp.y, xp.y);
    }
}

// ---------------------------------------------------------------------------
// Persistent waves.  Every wavefront of the launch owns one workspace slot
// (the four vectors of S columns) and pulls scenarios from an atomic queue:
// whenever a column has stopped (and its last step length has reached
// delta), the column writes its results and takes the next scenario, so no
// lane sweeps a finished column while scenarios are left.  The iteration
// itself is per column: its own step count, alpha, rho and stop decision;
// the sweeps are shared by the S columns, so every matrix and factor entry a
// wave reads still serves S scenarios.

// One column's scenario (the same in the R lanes of the column).
struct Col {
    int scen = -1;  // scenario index; -1: the column holds none
    int ic = -1, jc = -1, lo = 0, hi = 0;  // outaged branch's reduced rows, island interval
    double bc = 0.0;                       // its susceptance
    double bb = 0.0;                       // ||b_M||^2
    double gfac = 0.0;                     // re-dispatch factor dP / S_gen
    bool island = false, nogen = false, bad = false;
    int status = kConverged;
    int k = 0;  // step-length updates applied so far
};

// Take scenario `scen` into this lane's column when `take` (column-uniform):
// island interval, re-dispatch (Section IV.C) and the correction-form start
// r0 = (P' - P)_M + (P - A theta_b)_M + b_c (theta_b,f - theta_b,t) u_M
// from the base state, or r0 = b_M for per-scenario right-hand sides and for
// the zero start; delta = p = q = 0.  Every lane runs the loops and the
// column sums (the butterflies need the whole wave); only taking columns
// touch memory.  Returns the column's squared residual norm.
template <int S, int NT>
__device__ __forceinline__ double column_init(const PcgParams &p, const Tile<NT> &T, int rs, int sc, bool take, int scen,
                                              Col &col) {
    constexpr int R = kWave / S;
    const int nr = p.n_r;
    Col c{};
    int oc = -1;
    if (take) {
        c.scen = scen;
        oc = p.outages[scen];
        c.bad = oc < -1 || oc >= p.m;
        if (c.bad) oc = -1;
        if (oc >= 0) {
            c.ic = p.br_from[oc] - 1;
            c.jc = p.br_to[oc] - 1;
            c.bc = p.br_b[oc];
            c.lo = p.isl_lo[oc];
            c.hi = p.isl_hi[oc];
        }
        if (c.bad) {
            c.lo = 0;
            c.hi = INT_MAX;
        }
        c.island = c.hi > c.lo;
    }
    const bool cols = p.rhs_cols != nullptr;
    double rr = 0.0, bb = 0.0;
    if (cols) {
        const double *b = p.rhs_cols + (size_t)(take ? scen : 0) * p.rhs_ld;
        for (int i = rs; i < nr; i += R) {
            if (take) {
                const double r0 = !in_interval(p.pre_row[i], c.lo, c.hi) ? b[caller_bus(p.bus_map, i + 1)] : 0.0;
                rr += r0 * r0;
                const unsigned o = row_off<S>(T, i, sc);
                xp_put(T, o, 0.0, 0.0);
                ry_put(T, o, r0, 0.0);  // q = 0
            }
        }
        bb = rr;
    } else {
        double dP = 0.0, Sg = 0.0;
        for (int i = rs; i < nr; i += R) {
            if (take) {
                const double Pk = p.rhs[caller_bus(p.bus_map, i + 1)];
                if (in_interval(p.pre_row[i], c.lo, c.hi))
                    dP += Pk;
                else if (Pk > 0.0)
                    Sg += Pk;
            }
        }
        dP = col_sum<S>(dP);
        Sg = col_sum<S>(Sg);
        c.nogen = c.island && !(Sg > 0.0);
        c.gfac = (p.kind == 0 && c.island && !c.bad && !c.nogen) ? dP / Sg : 0.0;
        const double thf = (c.ic >= 0) ? p.theta_b[c.ic + 1] : 0.0;
        const double tht = (c.jc >= 0) ? p.theta_b[c.jc + 1] : 0.0;
        const double corr = c.bc * (thf - tht);
        for (int i = rs; i < nr; i += R) {
            if (take) {
                double r0 = 0.0;
                if (!in_interval(p.pre_row[i], c.lo, c.hi)) {
                    const double Pk = p.rhs[caller_bus(p.bus_map, i + 1)];
                    const double dPk = (c.gfac != 0.0 && Pk > 0.0) ? Pk * c.gfac : 0.0;
                    const double b = Pk + dPk;
                    if (p.zero_start) {
                        r0 = b;
                    } else {
                        r0 = dPk + p.rho_b[i];
                        if (i == c.ic) r0 += corr;
                        if (i == c.jc) r0 -= corr;
                    }
                    bb += b * b;
                }
                rr += r0 * r0;
                const unsigned o = row_off<S>(T, i, sc);
                xp_put(T, o, 0.0, 0.0);
                ry_put(T, o, r0, 0.0);  // q = 0
            }
        }
    }
    rr = col_sum<S>(rr);
    bb = col_sum<S>(bb);
    if (take) {
        c.bb = bb;
        c.status = c.bad ? kBadOutage
                         : ((!__builtin_isfinite(rr) || !__builtin_isfinite(bb)) ? kNonfinite : kConverged);
        col = c;
    }
    return rr;
}

// Write a stopped column's results: x = theta_b + delta (or delta alone for
// per-scenario right-hand sides and the zero start) on the main system, 0 on
// islanded buses and at the slack; its step count, status and re-dispatch
// factor.  Only retiring columns touch memory.
template <int S, int NT>
__device__ __forceinline__ void column_retire(const PcgParams &p, const Tile<NT> &T, int rs, int sc, bool retire,
                                              const Col &c) {
    constexpr int R = kWave / S;
    if (!retire) return;
    double *x = p.x_out + (size_t)c.scen * p.n_bus;
    for (int i = rs; i < p.n_r; i += R) {
        double v = 0.0;
        if (!in_interval(p.pre_row[i], c.lo, c.hi))
            v = (p.add_base ? p.theta_b[i + 1] : 0.0) + xp_get(T, row_off<S>(T, i, sc)).x;
        x[caller_bus(p.bus_map, i + 1)] = v;
    }
    if (rs == 0) {
        x[0] = 0.0;
        int st = c.status;
        if (st == kConverged && c.island) st = (p.kind == 0 && c.nogen) ? kIslandedNoGen : kConvergedIslanded;
        p.iters_out[c.scen] = c.k;
        p.status_out[c.scen] = st;
        p.gfac_out[c.scen] = c.gfac;
    }
}

// Retire every stopped column and refill the free ones from the queue, until
// every column is busy or the queue is empty.  A column whose new scenario
// stops at once (a bad id, a start that already meets the stop test) is
// retired and refilled in the next pass of the loop.
template <int S, int NT>
__device__ __forceinline__ void refill(const PcgParams &p, const Tile<NT> &T, int rs, int sc, Col &col, bool &done,
                                       double &alpha, double &rho, bool &drained) {
    const int lane = threadIdx.x;
    for (;;) {
        const bool retire = col.scen >= 0 && done;
        if (__any(retire)) column_retire<S>(p, T, rs, sc, retire, col);
        if (retire) col.scen = -1;
        if (drained) return;
        const bool want = col.scen < 0;
        const unsigned long long wmask = __ballot(want && rs == 0);  // lanes 0 .. S-1 carry rs == 0
        if (wmask == 0ull) return;
        int base = 0;
        if (lane == 0) base = atomicAdd(p.queue, __popcll(wmask));
        base = __shfl(base, 0);
        const int j = base + __popcll(wmask & ((1ull << sc) - 1ull));
        const bool take = want && j < p.n_out;
        if (base + __popcll(wmask) >= p.n_out) drained = true;
        if (!__any(take)) return;
        const int scen = take ? (p.order ? p.order[p.n_out - 1 - j] : j) : 0;
        const double rr = column_init<S>(p, T, rs, sc, take, scen, col);
        if (take) {
            done = col.status != kConverged || rr <= p.tol2 * col.bb;
            alpha = 0.0;
            rho = 0.0;
        }
        if (!__any(take && done)) return;
    }
}

// The PCG of every scenario this wave takes (Section III.A), in correction
// form from the base state (Section III.B), with the base-case ILU(0)
// preconditioner (Section IV.B).  Per iteration: forward sweep (r -= alpha q,
// ||r||^2, y = L^-1 r, and r'z = y' D^-1 y when the factors have the form
// U = D L^T), stop test, backward sweep (z = P_M U^-1 y; r'z here for other
// factors), beta, product sweep (delta += alpha p_old, p = z + beta p, q = A_c p with
// the outaged branch shielded, p'q), alpha.  Returns the iterations the wave
// ran (sweeps of its columns, counting stopped ones).
template <int S, int D, int DP, int NT>
__device__ __forceinline__ long long pcg_wave(const PcgParams &p, int wave, double *ring) {
    const int lane = threadIdx.x;
    const int sc = lane % S;
    const int rs = lane / S;
    Tile<NT> T;
    for (int v = 0; v < kVectors; ++v) T.v[v] = p.ws + (size_t)wave * p.ws_slot + (size_t)v * vec_stride(p.n_r, S);
    T.xp = T.v[0];
    T.r = T.v[2];
    T.w = T.v[3];
    T.nr = p.n_r;
    T.idle = false;
    // entry staging after the rings (the launch sizes LDS for the largest)
    const int ring_rows = max(p.fwd.ring, max(p.bwd.ring, p.prod.ring));
    int4 *stage = (int4 *)((char *)ring + ((((size_t)ring_rows + 2) * S * 8 + 15) & ~(size_t)15));
    if (rs == 0) {  // the scratch row holds zeros for idle slots
        const unsigned o = row_off<S>(T, p.n_r, sc);
        xp_put(T, o, 0.0, 0.0);
        ry_put(T, o, 0.0, 0.0);
    }
    Col col;
    bool done = true, drained = false;
    double alpha = 0.0, rho = 0.0;
    refill<S>(p, T, rs, sc, col, done, alpha, rho, drained);
    T.idle = col.scen < 0;
    long long sweeps = 0;
    while (__any(col.scen >= 0)) {
        __syncthreads();
        ++sweeps;
        // ---- forward sweep: r -= alpha q, y = L^-1 r ----------------------
        const dvec2 fr = fwd_sweep<S, D>(p.fwd, ring, stage, T, rs, sc, alpha);
        double rrp = fr.x;
        __syncthreads();
        rrp = col_sum<S>(rrp);
        if (col.scen >= 0 && !done) {
            if (col.k > 0) {
                if (!__builtin_isfinite(rrp)) {
                    done = true;
                    col.status = kNonfinite;
                } else if (rrp <= p.tol2 * col.bb) {
                    done = true;
                }
            }
            if (!done && col.k >= p.max_iter) {
                col.status = kMaxIter;
                done = true;
            }
        }
        if (__all(done)) {
            // every column stopped: the last step length has not reached
            // delta yet; then hand the columns back
            final_update<S>(T, rs, sc, alpha);
            alpha = 0.0;
            refill<S>(p, T, rs, sc, col, done, alpha, rho, drained);
            T.idle = col.scen < 0;
            continue;
        }

        // ---- backward sweep: z = P_M U^-1 y, rho = r'z ---------------------
        double rz;
        if (p.sym) {  // r'z = y' D^-1 y from the forward sweep
            (void)bwd_sweep<S, D, false>(p.bwd, ring, stage, T, rs, sc, col.lo, col.hi);
            rz = col_sum<S>(fr.y);
        } else {
            rz = col_sum<S>(bwd_sweep<S, D, true>(p.bwd, ring, stage, T, rs, sc, col.lo, col.hi));
        }
        __syncthreads();
        const double beta = (col.k == 0 || done) ? 0.0 : rz / rho;
        rho = rz;

        // ---- p = z + beta p and q = A_c p (outaged branch shielded), p'q ---
        const double sigma = col_sum<S>(
            prod_sweep<S, DP>(p.prod, ring, stage, T, rs, sc, alpha, beta, done, col.lo, col.hi, col.ic, col.jc,
                              col.bc));
        __syncthreads();
        if (!done) {
            if (!__builtin_isfinite(sigma) || !__builtin_isfinite(rho)) {
                done = true;
                col.status = kNonfinite;
            } else if (!(sigma > 0.0)) {
                done = true;
                col.status = kBreakdown;
            } else {
                alpha = rho / sigma;
                ++col.k;
            }
        }
        if (done) alpha = 0.0;  // a stopped column's delta is complete after this product sweep
        if (__any(col.scen >= 0 && done)) {
            refill<S>(p, T, rs, sc, col, done, alpha, rho, drained);
            T.idle = col.scen < 0;
        }
    }
    return sweeps;
}

// Work-group b (one wavefront) is persistent wave b; NT: the non-temporal
// vector accesses (kStreamVec).
template <int S, int D, int DP, bool NT>
__global__ void __launch_bounds__(kWave) pcg_wave_kernel(PcgParams p) {
    extern __shared__ double ring[];
    const long long n = pcg_wave<S, D, DP, NT ? kStreamVec : 0>(p, blockIdx.x, ring);
    if (p.sweeps && threadIdx.x == 0) atomicAdd(p.sweeps, (unsigned long long)n);
}

// Several grids (the uneven batch): every wave works through the grids in
// the caller's order (heaviest first), each until that grid's queue is
// empty and its own columns have stopped, so waves done with a large grid
// move on to the smaller ones while the others finish.  Its vector and
// program accesses go through global-memory pointers (kGlobalVec).
template <int S, int D, int DP, bool NT>
__global__ void __launch_bounds__(kWave) pcg_multi_kernel(const PcgParams *grids, int n_grids) {
    extern __shared__ double ring[];
    long long n = 0;
    for (int g = 0; g < n_grids; ++g) {
        const PcgParams &p = grids[g];
        n += pcg_wave<S, D, DP, (NT ? kStreamVec : 0) | kGlobalVec>(p, blockIdx.x, ring);
        __syncthreads();
    }
    if (grids[0].sweeps && threadIdx.x == 0) atomicAdd(grids[0].sweeps, (unsigned long long)n);
}

// Queue counters (and the sweep counter) back to zero before a launch; a
// kernel rather than a memory set, so that graph replays see it too.
__global__ void queue_reset_kernel(const PcgParams *grids, int n_grids, int32_t *queue, unsigned long long *sweeps) {
    const int t = threadIdx.x;
    if (grids) {
        for (int g = t; g < n_grids; g += blockDim.x) {
            *grids[g].queue = 0;
            if (grids[g].sweeps) *grids[g].sweeps = 0ull;
        }
    } else if (t == 0) {
        *queue = 0;
        if (sweeps) *sweeps = 0ull;
    }
}

}  // namespace

// ---------------------------------------------------------------------------

template <int S>
static hipError_t launch_wave_s(const PcgParams &prm, int n_waves, size_t lds, bool stream, hipStream_t st) {
    auto kern = pcg_wave_kernel<S, kPrefetchTri, kPrefetchProd, false>;
    if constexpr (S > 1) {  // one column per wave (the base-case solve) has no idle columns to ease
        if (stream) kern = pcg_wave_kernel<S, kPrefetchTri, kPrefetchProd, true>;
    }
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(kWave), 0, st, (const PcgParams *)nullptr, 0, prm.queue,
                       prm.sweeps);
    hipLaunchKernelGGL(kern, dim3(n_waves), dim3(kWave), lds, st, prm);
    return hipGetLastError();
}

template <int S>
static hipError_t launch_multi_s(const PcgParams *grids, int n_grids, int n_waves, size_t lds, bool stream,
                                 hipStream_t st) {
    auto kern = pcg_multi_kernel<S, kPrefetchTri, kPrefetchProd, false>;
    if constexpr (S > 1) {
        if (stream) kern = pcg_multi_kernel<S, kPrefetchTri, kPrefetchProd, true>;
    }
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(kWave), 0, st, grids, n_grids, (int32_t *)nullptr,
                       (unsigned long long *)nullptr);
    hipLaunchKernelGGL(kern, dim3(n_waves), dim3(kWave), lds, st, grids, n_grids);
    return hipGetLastError();
}

template <int S>
static int max_waves_s(size_t lds) {
    int per_cu = 0, cu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    // the smaller occupancy of the two cache-policy forms (they differ in the hint only)
    const void *kerns[2] = {(const void *)pcg_wave_kernel<S, kPrefetchTri, kPrefetchProd, false>,
                            (const void *)pcg_wave_kernel<S, kPrefetchTri, kPrefetchProd, S != 1>};
    int best = INT_MAX;
    for (const void *kern : kerns) {
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kWave, lds) != hipSuccess) return 0;
        best = std::min(best, per_cu);
    }
    return best * cu;
}

static size_t ring_lds(int ring_rows, int S) {
    // ring rows plus the zero row and the trash row of idle slots, then the
    // entry staging area (16-byte aligned)
    return (((size_t)(ring_rows + 2) * S * sizeof(double) + 15) & ~(size_t)15) + (size_t)kStageChunks * 16;
}

int pcg_max_waves(int S, int ring_rows) {
    const size_t lds = ring_lds(ring_rows, S);
    switch (S) {
        case 1: return max_waves_s<1>(lds);
        case 2: return max_waves_s<2>(lds);
        case 4: return max_waves_s<4>(lds);
        case 8: return max_waves_s<8>(lds);
        case 16: return max_waves_s<16>(lds);
        case 32: return max_waves_s<32>(lds);
        case 64: return max_waves_s<64>(lds);
        default: return 0;
    }
}

hipError_t launch_pcg_multi(const PcgParams *grids, int n_grids, int S, int n_waves, int ring_rows, bool stream,
                            hipStream_t st) {
    if (n_waves <= 0 || n_grids <= 0) return hipSuccess;
    const size_t lds = ring_lds(ring_rows, S);
    switch (S) {
        case 1: return launch_multi_s<1>(grids, n_grids, n_waves, lds, stream, st);
        case 2: return launch_multi_s<2>(grids, n_grids, n_waves, lds, stream, st);
        case 4: return launch_multi_s<4>(grids, n_grids, n_waves, lds, stream, st);
        case 8: return launch_multi_s<8>(grids, n_grids, n_waves, lds, stream, st);
        case 16: return launch_multi_s<16>(grids, n_grids, n_waves, lds, stream, st);
        case 32: return launch_multi_s<32>(grids, n_grids, n_waves, lds, stream, st);
        case 64: return launch_multi_s<64>(grids, n_grids, n_waves, lds, stream, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pcg(const PcgParams &prm, int S, int n_waves, int ring_rows, bool stream, hipStream_t st) {
    if (n_waves <= 0) return hipSuccess;
    const size_t lds = ring_lds(ring_rows, S);
    switch (S) {
        case 1: return launch_wave_s<1>(prm, n_waves, lds, stream, st);
        case 2: return launch_wave_s<2>(prm, n_waves, lds, stream, st);
        case 4: return launch_wave_s<4>(prm, n_waves, lds, stream, st);
        case 8: return launch_wave_s<8>(prm, n_waves, lds, stream, st);
        case 16: return launch_wave_s<16>(prm, n_waves, lds, stream, st);
        case 32: return launch_wave_s<32>(prm, n_waves, lds, stream, st);
        case 64: return launch_wave_s<64>(prm, n_waves, lds, stream, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gpcg
