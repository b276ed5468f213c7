// Internal declarations shared by the host side (gpcg_host.cpp) and the
// device kernels (gpcg_tile.hip, gpcg_kernels.hip) of the batched contingency
// PCG library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gpcg.h"

namespace gpcg {

constexpr int kWave = 64;     // gfx950 wavefront width
constexpr int kVectors = 4;   // per wave: pairs {delta, p} (two vectors), r, w (y, z, then q); (n_r + 1) x S each
// doubles per vector of a tile: (n_r + 1) rows x S columns, rounded up to
// even so that every vector, and every {delta, p} pair, is 16-byte aligned
constexpr size_t vec_stride(int n_r, int S) { return ((size_t)(n_r + 1) * S + 1) / 2 * 2; }
constexpr int kLdsBudget = 80 * 1024;  // bytes of LDS ring per wavefront (two waves fit one CU)

enum Status : int32_t {
    kConverged = 0,
    kMaxIter = 1,
    kBreakdown = 2,
    kNonfinite = 3,
    kConvergedIslanded = 4,
    kIslandedNoGen = 5,
    kBadOutage = 6,
};

// Matrix entries per row slot of a step: triangular solves and the product.
// Longer rows are split on the host into continuation segments placed in
// the same slot of the steps just before the row's own step; the lane
// carries their partial sums.
constexpr int kPadSteps = 32;  // idle steps appended to every program (>= the deepest prefetch)
constexpr int kEntTri = 4;
constexpr int kEntProd = 8;

// Prefetch depths of the sweeps: vector rows are loaded D steps ahead of
// their step (triangular solves, product).
constexpr int kPrefetchTri = 8;
constexpr int kPrefetchProd = 6;

// Staged programs (blocks of 4 scenarios or more).  A step's entry chunks
// and, behind them, the R row records of a later step form one block of
// 16-byte chunks that a wave loads once, one chunk per lane, and hands to
// its lanes through a per-wave LDS staging area.  The entries are read from
// there kStageLook steps before their step runs; the records ride
// stage_rec_ahead() steps ahead of the block's own step, so that each
// record arrives one step before its vector rows are loaded.
constexpr int kStageChunks = 2 * kWave;  // chunks of a wave's staging area
constexpr int kStageLookTri = 3;
constexpr int kStageLookProd = 2;
constexpr int stage_chunks(int S, int K) { return (3 * K / 4 + 1) * (kWave / S); }
constexpr bool staged(int S, int K) { return stage_chunks(S, K) <= kStageChunks; }
constexpr int stage_rec_ahead(bool tri) {
    return tri ? kPrefetchTri + 2 - kStageLookTri : kPrefetchProd + 1 - kStageLookProd;
}

// A sweep program: the steps one wavefront walks, R row slots per step, each
// slot with a fixed number K of packed matrix entries (padding entries carry
// value 0 and point at the ring's zero row).
//   rec[s * R + rs] = {row, own, pre, aux}:
//     row: the row finished in this slot (n_r, the scratch row, when the
//          slot is idle or holds a continuation segment);
//     own: LDS byte offset of that row's ring slot for column 0 (the trash
//          row when row is -1; the zero row for idle product slots);
//     pre: pre-order number of the row's bus (-1 when none; -2 marks a
//          continuation segment of the product);
//     aux: triangular solves: 1 for a continuation segment, else 0 (-1 idle);
//          product: the look-ahead row whose direction is updated, or n_r.
//   entries of slot rs of step s, in 3K/4 sixteen-byte chunks
//     ent[(s * 3K/4 + c) * R + rs]: chunks c < K/2 hold the values of
//     entries 2c and 2c + 1 (doubles), chunks K/2 + c' the LDS byte offsets
//     of the ring slots (for column 0) of entries 4c' .. 4c' + 3;
//   The forward solve's records use the backward solve's packed form too
//   (its 1 / U_ii weights y_i^2 in r'z = y' D^-1 y).
//   Staged programs (staged(S, K)) store ent as blocks of stage_chunks(S, K)
//   chunks per step instead: the 3K/4 R entry chunks above, then the R
//   records of step s + stage_rec_ahead(tri) (the last padding step's past
//   the end); rec keeps every step's records for the first steps a sweep
//   reads directly.
//   The backward solve packs its records instead (kBwdRowBits-bit row and
//   pre-order fields), so that 1 / U_ii rides in the same 16-byte load:
//     rec[s * R + rs] = {row | slot << 20, pre | (aux + 1) << 20, 1 / U_ii}:
//     slot: the ring slot index of own (own = slot * S * 8); pre: 2^20 - 1
//     when none; 1 / U_ii: 0 for idle and continuation slots.
struct Program {
    const int4 *rec;
    const int4 *ent;
    int steps, ring;
};
constexpr int kBwdRowBits = 20;                      // row and pre-order fields of the backward records
constexpr int kBwdRowMask = (1 << kBwdRowBits) - 1;  // also the "none" pre-order number
constexpr int kBwdMaxRing = 2048;                    // ring rows of the backward solve (slot + 2 < 2^12)

// Buses are numbered internally in the order of the reduced rows: row i is
// internal bus i + 1, the slack is 0.  bus_map (device, n_bus; NULL when the
// caller's numbering is the internal one) turns an internal bus into the
// caller's bus, which numbers every bus-indexed array the caller passes or
// receives.
__host__ __device__ __forceinline__ int caller_bus(const int32_t *bus_map, int k) { return bus_map ? bus_map[k] : k; }

// Everything one launch of the persistent PCG kernel needs.  All pointers
// are device memory.  Reduced row i is internal bus i + 1.
struct PcgParams {
    int n_r, n_bus, m, kind;
    const int32_t *bus_map;  // internal bus -> caller's bus (NULL: the same)
    Program fwd;   // y = L^-1 r  (rows in a dependency-respecting order)
    Program bwd;   // z = U^-1 y
    Program prod;  // p = z + beta p, delta += alpha p_old, q = A_c p (natural order, R rows per step)
    // branch table; br_b = 1 / x
    const int32_t *br_from, *br_to;
    const double *br_b;
    // DFS pre-order number of the bus of each reduced row; island interval per branch
    const int32_t *pre_row;
    const int32_t *isl_lo, *isl_hi;
    // base state and its double-double residual for this right-hand side
    const double *theta_b;  // n_bus, slack 0
    const double *rho_b;    // n_r: rhs - A theta_b
    const double *rhs;      // n_bus, caller's numbering
    // per-scenario right-hand sides (NULL: rhs above with the warm start):
    // scenario j solves A_c x = rhs_cols[j * rhs_ld + bus] (caller's bus)
    // from x = 0, with no re-dispatch
    const double *rhs_cols;
    int rhs_ld;
    int zero_start;  // 1: start from x = 0 (r0 = P'_M), the result is theta itself
    // 1: the factors have the form U = D L^T (M = L U symmetric), so r'z is
    // summed in the forward sweep as y' D^-1 y and the backward sweep does not
    // read r; 0: r'z in the backward sweep
    int sym;
    // scenarios: queue position j takes scenario order[n_out - 1 - j] (the
    // order sorted by expected work, taken from its heavy end; NULL: j)
    const int32_t *outages;
    const int32_t *order;
    int n_out;
    int32_t *queue;                // next queue position (zeroed before the launch)
    unsigned long long *sweeps;    // NULL, or the sum over waves of the iterations each ran
    double tol2;
    int max_iter;
    // workspace: wave w owns ws + w * ws_slot: pairs {delta, p}, r, w,
    // kVectors x (n_r + 1) rows x S
    double *ws;
    size_t ws_slot;
    // results, written when a column stops: x = (theta_b if add_base) + delta
    // on the main system [n_out x n_bus, caller's numbering], steps, status,
    // re-dispatch factor
    double *x_out;
    int add_base;
    int32_t *iters_out, *status_out;
    double *gfac_out;
};

// Outputs formed after the PCG launch from the angles it wrote: island
// flags, flows, true residuals.
struct OutParams {
    int n_r, n_bus, m, kind, n_out;
    const int32_t *bus_map;            // internal bus -> caller's bus (NULL: the same)
    const int32_t *cbr_from, *cbr_to;  // branch endpoints in the caller's numbering (flows)
    const int32_t *a_rowptr, *a_col;
    const double *a_val;
    const int32_t *br_from, *br_to;
    const double *br_x, *br_b;
    const int32_t *pre_bus;  // n_bus, by internal bus
    const int32_t *isl_lo, *isl_hi;
    const double *theta_b, *rhs;  // theta_b internal, rhs caller's numbering
    const double *rhs_cols;  // per-scenario right-hand sides (then x = delta, no base state added)
    int rhs_ld;
    int add_base;  // 1: x = theta_b + delta (warm start from the base state)
    const int32_t *outages;
    const int32_t *status;
    const double *gfac;
    const double *x_out;
    double *flows_out, *resid_out;
    uint8_t *island_out;
};

// The stand-alone product reads A through a per-chunk copy laid out on the
// host once per chunk height ch: chunk k holds max_nnz entries at
// k * max_nnz (values; columns as row offsets from the chunk's lowest read
// row max(0, k ch - bw); padding has value 0 and offset 0), ch + 1 row
// pointers relative to the chunk's first entry at k (ch + 1), and the ch
// rows' pre-order numbers at k ch.  No staging load then depends on another.
struct SpmmParams {
    int n_r, m, ncols;
    const double *c_val;
    const int32_t *c_col, *c_rp, *c_pre;
    const int32_t *br_from, *br_to;
    const double *br_b;
    const int32_t *isl_lo, *isl_hi;
    const int32_t *outages;
    const double *p;
    double *q, *pq;
};

// Branch-overload loss L = sum_e softplus(kappa (|f_e| / F_e - 1)) of every
// scenario and its gradients by the adjoint method: with s_e = dL/df_e and
// g = dL/dtheta = D^T s (D: flows as a map of the angles), the adjoint
// lambda solves A_c[M,M] lambda_M = g_M; then
//   dL/dx_e = -s_e f_e / x_e + (lambda_f - lambda_t)(theta_f - theta_t) / x_e^2
// (0 for the outaged branch), and dL/dP = (dP'/dP)^T lambda through the
// re-dispatch.  Scenario-major arrays: theta, lambda, g [n_out * n_bus],
// flows and dL/dx [n_out * m].
struct OverloadParams {
    int n_bus, m, n_out;
    double kappa;
    const int32_t *br_from, *br_to;
    const double *br_x;
    const int32_t *inc_ptr, *inc_br;  // branches incident to each bus (CSR over buses)
    const int32_t *pre_bus;
    const int32_t *isl_lo, *isl_hi;
    const int32_t *outages;
    const double *P, *F;  // injections [n_bus], flow limits [m]
    const double *theta, *flows, *lambda;
    double *g, *loss, *grad_p, *grad_x;
};

// Fast-decoupled power flow of every outage (Section II, eqs. (1)-(5)) on a
// lossless, tap-free network with bus shunts: per outer iteration a P-theta
// half (B'_c dtheta = dP / V) and a Q-V half (B''_c dV = dQ / V), each a
// batched solve with a right-hand side per scenario.  State theta, V and the
// right-hand sides are scenario-major [n_out * n_bus].
struct FdpfParams {
    int n_bus, m, n_out;
    const int32_t *br_from, *br_to;
    const double *br_b;
    const int32_t *inc_ptr, *inc_br;
    const int32_t *pre_bus, *isl_lo, *isl_hi;
    const int32_t *outages;
    const double *P, *Q;     // specified injections [n_bus]
    const double *diag_bpp;  // B'' diagonal by bus: sum of 1/x at the bus + its shunt
    const double *theta0, *V0;
    double *theta, *V, *rhs;
    const double *dx;
    double *gfac;                     // per scenario: re-dispatch factor
    int32_t *nogen;                   // per scenario: islanded with no main generator
    int32_t *iters, *status;          // accumulated over the half-iterations
    const int32_t *it_step, *st_step;  // the last half-iteration's solve
};

// Launchers (launch_pcg in gpcg_tile.hip, the rest in gpcg_kernels.hip).  They
// return hipSuccess or the launch error.
// n_waves persistent wavefronts (each with a workspace slot) over one queue;
// the queue and sweep counters are reset by a kernel launched first.
// stream: the sweeps' vector accesses carry the non-temporal hint (for a
// queue ranked by an iteration record, where few columns idle; S > 1).
hipError_t launch_pcg(const PcgParams &prm, int S, int n_waves, int ring_rows, bool stream, hipStream_t st);
// several grids in one launch: grids (device, n_grids entries, heaviest
// first) share the workspace slots; ring_rows = the largest ring of any grid
hipError_t launch_pcg_multi(const PcgParams *grids, int n_grids, int S, int n_waves, int ring_rows, bool stream,
                            hipStream_t st);
// wavefronts of the PCG kernel at block S that fit the device at once
int pcg_max_waves(int S, int ring_rows);
hipError_t launch_outputs(const OutParams &prm, hipStream_t st);
// rho = rhs - A theta_b (theta_b internal; rhs by bus_map, NULL: internal)
hipError_t launch_base_residual(int n_r, const int32_t *rowptr, const int32_t *col, const double *val,
                                const double *theta_b, const double *rhs, const int32_t *bus_map, double *rho,
                                hipStream_t st);
// theta_b[k] += x[k] for the buses k >= 1
hipError_t launch_base_accumulate(int n_bus, double *theta_b, const double *x, hipStream_t st);
// q = A_c p over ncols / S tiles of n_r x S (bw: bandwidth of A).  Rows are
// cut into chunks of ch (a multiple of 256 / S that spmm_chunk_fits accepts)
// and chunks into segments of nseg, one work-group per (tile, segment);
// max_nnz: the most entries of A in one chunk.  partial:
// f64[n_segments * ncols] scratch for the p'q column sums (NULL when prm.pq
// is NULL).
constexpr size_t kSpmmLdsBudget = 40 * 1024;  // LDS per work-group the host aims for (at least four per CU)
constexpr int kSpmmMaxChunk = 80;  // rows per chunk beyond which more work-groups per CU pay more than longer chunks
size_t spmm_lds_bytes(int S, int bw, int ch, int max_nnz);
bool spmm_chunk_fits(int S, int ch, int max_nnz);
hipError_t launch_spmm_partial(const SpmmParams &prm, int S, int bw, int ch, int nseg, int max_nnz, double *partial,
                               hipStream_t st);
hipError_t launch_sumsq(int n, const double *v, double *out, hipStream_t st);
// seed g = dL/dtheta and the per-scenario loss (after the forward solve)
hipError_t launch_overload_seed(const OverloadParams &prm, hipStream_t st);
// dL/dP and dL/dx from theta, flows and lambda (after the adjoint solve)
hipError_t launch_overload_grads(const OverloadParams &prm, hipStream_t st);
// fast-decoupled power flow: 0 start from (theta0, V0) and re-dispatch;
// 1 mismatch of half h into rhs; 2 state += dx for half h and accumulate
// the solve's iterations and status; 3 islands to theta = 0, V = 1
hipError_t launch_fdpf(const FdpfParams &prm, int phase, int half, hipStream_t st);
// per scenario: branches with |f| > F, the largest |f| / F and its branch
hipError_t launch_screen(int n_out, int m, const double *flows, const double *F, int32_t *count, double *worst,
                         int32_t *worst_branch, hipStream_t st);
// out[j] = sum_r w[r] a[r * lda + j]
hipError_t launch_weighted_rows(int n_rows, int n_cols, const double *a, int lda, const double *w, double *out,
                                hipStream_t st);

// The library's fixed device scratch: a file-scope device array of
// kStaticScratchBytes on every GPU the library runs on, for the solve entry
// point that allocates nothing.  static_scratch() returns its address on the
// current device, looked up with hipGetSymbolAddress once per device and
// kept (the array's name is not a device address in host code).
constexpr size_t kStaticScratchBytes = GPCG_NOALLOC_SCRATCH_BYTES;
hipError_t static_scratch(void **ptr);

// Rank scenarios by expected PCG work, ascending (the queue takes them from
// the heavy end): by the iterations each outage took in this context's
// previous solve (hist, indexed c + 1; -1 = none; NULL: no records), and
// outages without a record first, islanding ones before the others, each by
// the base-case flow of the outaged branch.  Writes order[] (scenario of each
// rank) and pos[] (its inverse).  temp / temp_bytes: scratch from
// sort_temp_bytes().
size_t sort_temp_bytes(int n);
hipError_t launch_order(int n, const int32_t *outages, int m, const int32_t *br_from, const int32_t *br_to,
                        const double *br_b, const int32_t *isl_lo, const int32_t *isl_hi, const double *theta_b,
                        const int32_t *hist, uint32_t *keys, uint32_t *keys_sorted, int32_t *iota, int32_t *order,
                        int32_t *pos, void *temp, size_t temp_bytes, hipStream_t st);
// hist[outages[s] + 1] = iters[s] for the valid outages
hipError_t launch_record_iters(int n, const int32_t *outages, int m, const int32_t *iters, int32_t *hist,
                               hipStream_t st);

}  // namespace gpcg
