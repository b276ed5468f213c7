// Device kernels of the batched "N-1" contingency PCG other than the tile
// kernel: outputs and true residuals, the base-case helpers, the stand-alone
// outage-corrected product and the scenario ordering (gfx950, FP64).
#include "gpcg_device.h"

#include <algorithm>
#include <climits>
#include <hipcub/hipcub.hpp>
#include <mutex>
#include <type_traits>

namespace gpcg {
namespace {

// ---------------------------------------------------------------------------
// double-double helpers (Dekker 1971; Ogita, Rump, Oishi 2005): error-free
// sum and product, used where a residual must be formed without cancellation
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
#pragma clang fp contract(off)
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) += a * b
__device__ __forceinline__ void dd_fma(double &hi, double &lo, double a, double b) {
#pragma clang fp contract(off)
    const double p = a * b;
    const double pe = __builtin_fma(a, b, -p);
    double s, e;
    two_sum(hi, p, s, e);
    hi = s;
    lo += e + pe;
}

// ---------------------------------------------------------------------------
// Island flags of each scenario (the angles themselves are written by the
// PCG kernel when a scenario stops).
__global__ void island_out_kernel(OutParams p) {
    const int s = blockIdx.x;
    const int k = blockIdx.y * blockDim.x + threadIdx.x;
    if (k >= p.n_bus) return;
    const int c = p.outages[s];
    const bool bad = c < -1 || c >= p.m;
    int lo = 0, hi = 0;
    if (!bad && c >= 0) {
        lo = p.isl_lo[c];
        hi = p.isl_hi[c];
    }
    const bool in = (k > 0) && in_interval(p.pre_bus[k], lo, hi);  // k: internal bus
    p.island_out[(size_t)s * p.n_bus + caller_bus(p.bus_map, k)] = in ? 1 : 0;
}

// Branch flows (theta_f - theta_t) / x_e; the outaged branch carries 0 and
// branches inside an island see two zero angles.
__global__ void flows_out_kernel(OutParams p) {
    const int s = blockIdx.x;
    const int e = blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= p.m) return;
    const int c = p.outages[s];
    const double *th = p.x_out + (size_t)s * p.n_bus;
    double f = 0.0;
    if (e != c && c >= -1 && c < p.m) f = (th[p.cbr_from[e]] - th[p.cbr_to[e]]) / p.br_x[e];
    p.flows_out[(size_t)s * p.m + e] = f;
}

// True relative residual ||P'_M - A_c theta_M|| / ||P'_M|| of the returned
// angles (or ||b_M - A_c x_M|| / ||b_M|| for per-scenario right-hand sides),
// each row's residual formed in double-double.
__global__ void __launch_bounds__(256) resid_kernel(OutParams p) {
    __shared__ double sh_r[256], sh_b[256];
    const int s = blockIdx.x;
    const int c0 = p.outages[s];
    const bool bad = c0 < -1 || c0 >= p.m;
    const int c = bad ? -1 : c0;
    int ic = -1, jc = -1, lo = 0, hi = 0;
    double bc = 0.0;
    if (c >= 0) {
        ic = p.br_from[c] - 1;
        jc = p.br_to[c] - 1;
        bc = p.br_b[c];
        lo = p.isl_lo[c];
        hi = p.isl_hi[c];
    }
    const double gfac = p.gfac[s];
    const double *th = p.x_out + (size_t)s * p.n_bus;
    const int32_t *bm = p.bus_map;
    const double thf = (ic >= 0) ? th[caller_bus(bm, ic + 1)] : 0.0;
    const double tht = (jc >= 0) ? th[caller_bus(bm, jc + 1)] : 0.0;
    double rr = 0.0, bb = 0.0;
    if (!bad) {
        for (int i = threadIdx.x; i < p.n_r; i += blockDim.x) {
            if (in_interval(p.pre_bus[i + 1], lo, hi)) continue;
            const int k = caller_bus(bm, i + 1);
            const double Pk = p.rhs_cols ? p.rhs_cols[(size_t)s * p.rhs_ld + k] : p.rhs[k];
            const double b = Pk + ((gfac != 0.0 && Pk > 0.0) ? Pk * gfac : 0.0);
            double h = b, l = 0.0;
            for (int e = p.a_rowptr[i]; e < p.a_rowptr[i + 1]; ++e)
                dd_fma(h, l, -p.a_val[e], th[caller_bus(bm, p.a_col[e] + 1)]);
            if (i == ic) {
                dd_fma(h, l, bc, thf);
                dd_fma(h, l, -bc, tht);
            }
            if (i == jc) {
                dd_fma(h, l, -bc, thf);
                dd_fma(h, l, bc, tht);
            }
            const double r = h + l;
            rr += r * r;
            bb += b * b;
        }
    }
    sh_r[threadIdx.x] = rr;
    sh_b[threadIdx.x] = bb;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sh_r[threadIdx.x] += sh_r[threadIdx.x + w];
            sh_b[threadIdx.x] += sh_b[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nb = sqrt(sh_b[0]), nr = sqrt(sh_r[0]);
        p.resid_out[s] = nb > 0.0 ? nr / nb : nr;
    }
}

// rho = rhs - A theta_b per reduced row, in double-double, rounded once
// (theta_b by internal bus, rhs by the caller's).
__global__ void base_residual_kernel(int n_r, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                     const double *__restrict__ val, const double *__restrict__ theta_b,
                                     const double *__restrict__ rhs, const int32_t *__restrict__ bus_map,
                                     double *__restrict__ rho) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_r) return;
    double h = rhs[caller_bus(bus_map, i + 1)], l = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) dd_fma(h, l, -val[e], theta_b[col[e] + 1]);
    rho[i] = h + l;
}

// theta_b += x over the buses other than the slack
__global__ void base_accumulate_kernel(int n_bus, double *theta_b, const double *x) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 1 && k < n_bus) theta_b[k] += x[k];
}

__global__ void __launch_bounds__(256) sumsq_kernel(int n, const double *v, double *out) {
    __shared__ double sh[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a += v[i] * v[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// ---------------------------------------------------------------------------
// Stand-alone outage-corrected product q = A_c p over many tiles.  The rows
// are cut into chunks of ch and the chunks into segments of nseg; one
// work-group streams one segment of one tile.  Its LDS holds a ring of
// W = ch + 2 bw rows of p (the chunk and the band of A on either side) and
// the chunk's slice of A.  While it forms q for chunk k from LDS, the loads
// of chunk k + 1 (its ch new rows of p, its slice of A, its row pointers)
// are in flight in registers; they are written to LDS once chunk k is done.
// Work-groups are handed to the XCDs in turn (block b runs on XCD b mod 8);
// the grid is numbered so that the segments of one tile follow each other
// on one XCD, and the bw halo rows two segments share come from its L2.
constexpr int kSpmmThreads = 256;
constexpr int kXcds = 8;
constexpr int kSpmmLoadsP = 4;  // 16-byte (8-byte when S = 1) loads of p per thread per chunk
constexpr int kSpmmLoadsA = 4;  // entries of A per thread per chunk
constexpr int kSpmmLoadsR = 2;  // row pointers per thread per chunk

// a native two-double vector (kept in registers, unlike the HIP struct type)
typedef double dvec2 __attribute__((ext_vector_type(2)));

template <int S>
struct SpmmStage {
    using V = typename std::conditional<S % 2 == 0, dvec2, double>::type;
    static constexpr int W = sizeof(V) / sizeof(double);
    V vp[kSpmmLoadsP];
    double va[kSpmmLoadsA];
    int vc[kSpmmLoadsA], vr[kSpmmLoadsR], vpre[kSpmmLoadsR];
    int lo = 0, np = 0;
};

// Issue the loads of p rows [lo, hi) and of chunk k's copy of A (entries,
// row pointers, pre-order numbers).  None depends on another, so all are in
// flight together and nothing waits on them until they are committed.
template <int S>
__device__ __forceinline__ void spmm_fetch(SpmmStage<S> &st, const SpmmParams &p, const double *P, int lo, int hi,
                                           int k, int ch, int max_nnz, int tid, bool rows_only) {
    using V = typename SpmmStage<S>::V;
    const V *src = (const V *)(P + (size_t)lo * S);
    st.lo = lo;
    st.np = (hi - lo) * S / SpmmStage<S>::W;
#pragma unroll
    for (int j = 0; j < kSpmmLoadsP; ++j) {
        const int t = j * kSpmmThreads + tid;
        if (t < st.np) st.vp[j] = __builtin_nontemporal_load(&src[t]);  // streamed once
    }
    if (rows_only) return;
    const size_t e0 = (size_t)k * max_nnz;
#pragma unroll
    for (int j = 0; j < kSpmmLoadsA; ++j) {
        const int t = j * kSpmmThreads + tid;
        if (t < max_nnz) {
            st.va[j] = p.c_val[e0 + t];
            st.vc[j] = p.c_col[e0 + t];
        }
    }
#pragma unroll
    for (int j = 0; j < kSpmmLoadsR; ++j) {
        const int t = j * kSpmmThreads + tid;
        if (t <= ch) st.vr[j] = p.c_rp[(size_t)k * (ch + 1) + t];
        if (t < ch) st.vpre[j] = p.c_pre[(size_t)k * ch + t];
    }
}

// Write fetched p rows into the ring and (unless rows_only) the chunk's A
// into the chunk buffers, with the ring slot of every entry's column
// resolved here once.  Row r lives in ring slot r mod Wr; base_slot is the
// slot of the chunk's lowest read row, and every row the chunk touches lies
// within Wr rows of it.
template <int S>
__device__ __forceinline__ void spmm_commit(const SpmmStage<S> &st, double *ring, double *lval, int *lcol, int *lrp,
                                            int *lpre, int Wr, int lo_slot, int base_slot, int ch, int max_nnz,
                                            int tid, bool rows_only) {
    constexpr int VW = SpmmStage<S>::W;
#pragma unroll
    for (int j = 0; j < kSpmmLoadsP; ++j) {
        const int t = j * kSpmmThreads + tid;
        if (t < st.np) {
            const int e = t * VW;  // first double of this load within the rows
            int slot = lo_slot + e / S;
            if (slot >= Wr) slot -= Wr;
            *(typename SpmmStage<S>::V *)(ring + (size_t)slot * S + e % S) = st.vp[j];
        }
    }
    if (rows_only) return;
#pragma unroll
    for (int j = 0; j < kSpmmLoadsA; ++j) {
        const int t = j * kSpmmThreads + tid;
        if (t < max_nnz) {
            int slot = st.vc[j] + base_slot;
            if (slot >= Wr) slot -= Wr;
            lval[t] = st.va[j];
            lcol[t] = slot * S;
        }
    }
#pragma unroll
    for (int j = 0; j < kSpmmLoadsR; ++j) {
        const int t = j * kSpmmThreads + tid;
        if (t <= ch) lrp[t] = st.vr[j];
        if (t < ch) lpre[t] = st.vpre[j];
    }
}

template <int S>
__global__ void __launch_bounds__(kSpmmThreads)
    spmm_kernel(SpmmParams p, int bw, int ch, int nseg, int n_segs, int max_nnz, double *partial) {
    extern __shared__ double lds[];
    constexpr int RS = kSpmmThreads / S;  // row slots
    const int tid = threadIdx.x;
    const int sc = tid % S, rs = tid / S;
    const int n_tiles = p.ncols / S;
    const int b = blockIdx.x;
    const int tile = (b / kXcds / n_segs) * kXcds + b % kXcds;
    const int seg = (b / kXcds) % n_segs;
    if (tile >= n_tiles) return;  // whole work-group
    const int col = tile * S + sc;
    const int nr = p.n_r;
    const int Wr = ch + 2 * bw;  // ring rows
    const int k0 = seg * nseg;
    const int k1 = min((nr + ch - 1) / ch, k0 + nseg);
    const double *P = p.p + (size_t)tile * nr * S;
    double *Q = p.q + (size_t)tile * nr * S;
    double *ring = lds;
    double *lval = ring + (size_t)Wr * S;
    int *lcol = (int *)(lval + max_nnz);
    int *lrp = lcol + max_nnz;
    int *lpre = lrp + ch + 1;

    const int c = p.outages[col];
    int ic = -1, jc = -1, lo = 0, hi = 0;
    double bc = 0.0;
    if (c >= 0 && c < p.m) {
        ic = p.br_from[c] - 1;
        jc = p.br_to[c] - 1;
        bc = p.br_b[c];
        lo = p.isl_lo[c];
        hi = p.isl_hi[c];
    }
    const double dpc = ((ic >= 0) ? P[(size_t)ic * S + sc] : 0.0) - ((jc >= 0) ? P[(size_t)jc * S + sc] : 0.0);

    // prologue: the rows before the first chunk's new rows, in passes
    SpmmStage<S> st;
    const int c0s = k0 * ch;
    {
        const int w0 = max(0, c0s - bw), w1 = min(nr, c0s + bw);
        const int per = kSpmmLoadsP * kSpmmThreads * SpmmStage<S>::W / S;  // rows per pass
        for (int r = w0; r < w1; r += per) {
            spmm_fetch(st, p, P, r, min(w1, r + per), k0, ch, max_nnz, tid, true);
            spmm_commit(st, ring, lval, lcol, lrp, lpre, Wr, r % Wr, 0, ch, max_nnz, tid, true);
        }
        spmm_fetch(st, p, P, w1, min(nr, c0s + ch + bw), k0, ch, max_nnz, tid, false);
    }
    double pq = 0.0;
    for (int k = k0; k < k1; ++k) {
        const int c0 = k * ch, c1 = min(nr, c0 + ch);
        const int base = max(0, c0 - bw);  // lowest row chunk k reads
        const int bslot = base % Wr;
        spmm_commit(st, ring, lval, lcol, lrp, lpre, Wr, st.lo % Wr, bslot, ch, max_nnz, tid, false);
        __syncthreads();
        if (k + 1 < k1)
            spmm_fetch(st, p, P, min(nr, c1 + bw), min(nr, c1 + ch + bw), k + 1, ch, max_nnz, tid, false);
        for (int i = c0 + rs; i < c1; i += RS) {
            const int b0 = lrp[i - c0], b1 = lrp[i - c0 + 1];
            double q = 0.0;
            for (int e = b0; e < b1; ++e) q += lval[e] * ring[lcol[e] + sc];
            if (i == ic) q -= bc * dpc;
            if (i == jc) q += bc * dpc;
            if (in_interval(lpre[i - c0], lo, hi)) q = 0.0;
            __builtin_nontemporal_store(q, &Q[(size_t)i * S + sc]);  // q is not read back here
            int slot = bslot + (i - base);
            if (slot >= Wr) slot -= Wr;
            pq += ring[(size_t)slot * S + sc] * q;
        }
        __syncthreads();
    }
    if (!partial) return;  // whole work-group
    // column sums of p'q over the row slots, in a fixed order
    ring[tid] = pq;
    __syncthreads();
    if (tid < S) {
        double a = 0.0;
        for (int k = 0; k < RS; ++k) a += ring[k * S + sc];
        partial[(size_t)seg * p.ncols + col] = a;
    }
}

__global__ void spmm_pq_reduce_kernel(int ncols, int chunks, const double *partial, double *pq) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    double a = 0.0;
    for (int k = 0; k < chunks; ++k) a += partial[(size_t)k * ncols + col];
    pq[col] = a;
}

// ---------------------------------------------------------------------------
// Branch-overload loss and its adjoint gradients (see OverloadParams).

__device__ __forceinline__ double softplus(double z) { return fmax(z, 0.0) + log1p(exp(-fabs(z))); }

__device__ __forceinline__ double sigmoid(double z) {
    const double e = exp(-fabs(z));
    return z >= 0.0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
}

// s_e = dL/df_e = sigma(z) kappa sign(f_e) / F_e, z = kappa (|f_e| / F_e - 1);
// 0 where the flow is exactly 0 (the outaged branch, island branches)
__device__ __forceinline__ double flow_seed(const OverloadParams &p, const double *f, int e) {
    const double fe = f[e], Fe = p.F[e];
    if (fe == 0.0) return 0.0;
    const double z = p.kappa * (fabs(fe) / Fe - 1.0);
    return sigmoid(z) * p.kappa * (fe > 0.0 ? 1.0 : -1.0) / Fe;
}

// g_k = sum over branches e at bus k of +-s_e / x_e (+ at the from end)
__global__ void overload_seed_kernel(OverloadParams p) {
    const int s = blockIdx.x;
    const int k = blockIdx.y * blockDim.x + threadIdx.x;
    if (k >= p.n_bus) return;
    const double *f = p.flows + (size_t)s * p.m;
    double g = 0.0;
    for (int t = p.inc_ptr[k]; t < p.inc_ptr[k + 1]; ++t) {
        const int e = p.inc_br[t];
        const double v = flow_seed(p, f, e) / p.br_x[e];
        g += (p.br_from[e] == k) ? v : -v;
    }
    p.g[(size_t)s * p.n_bus + k] = g;
}

// per-scenario loss, summed over the branches in a fixed order
__global__ void __launch_bounds__(256) overload_loss_kernel(OverloadParams p) {
    __shared__ double sh[256];
    const int s = blockIdx.x;
    const double *f = p.flows + (size_t)s * p.m;
    double L = 0.0;
    for (int e = threadIdx.x; e < p.m; e += blockDim.x) L += softplus(p.kappa * (fabs(f[e]) / p.F[e] - 1.0));
    sh[threadIdx.x] = L;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) p.loss[s] = sh[0];
}

__global__ void overload_grad_x_kernel(OverloadParams p) {
    const int s = blockIdx.x;
    const int e = blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= p.m) return;
    const int c = p.outages[s];
    double d = 0.0;
    if (e != c && c >= -1 && c < p.m) {
        const double *th = p.theta + (size_t)s * p.n_bus;
        const double *la = p.lambda + (size_t)s * p.n_bus;
        const double *f = p.flows + (size_t)s * p.m;
        const int a = p.br_from[e], b = p.br_to[e];
        const double x = p.br_x[e];
        d = -flow_seed(p, f, e) * f[e] / x + (la[a] - la[b]) * (th[a] - th[b]) / (x * x);
    }
    p.grad_x[(size_t)s * p.m + e] = d;
}

// dL/dP_k through the re-dispatch of Section IV.C: with islanded power
// dP = sum_I P, main generators G (non-slack, P > 0), S = sum_G P and
// T = sum_G lambda P:  lambda_k on M \ G;  lambda_k (1 + dP/S) - T dP / S^2
// on G;  T / S on I.  Without generators (or without an island) it is
// lambda on M and 0 on I.  The slack's injection is not an input.
__global__ void __launch_bounds__(256) overload_grad_p_kernel(OverloadParams p) {
    __shared__ double sh[3][256];
    const int s = blockIdx.x;
    const int c = p.outages[s];
    const bool bad = c < -1 || c >= p.m;
    int lo = 0, hi = 0;
    if (!bad && c >= 0) {
        lo = p.isl_lo[c];
        hi = p.isl_hi[c];
    }
    const double *la = p.lambda + (size_t)s * p.n_bus;
    double dP = 0.0, S = 0.0, T = 0.0;
    for (int k = 1 + threadIdx.x; k < p.n_bus; k += blockDim.x) {
        const double Pk = p.P[k];
        if (in_interval(p.pre_bus[k], lo, hi)) {
            dP += Pk;
        } else if (Pk > 0.0) {
            S += Pk;
            T += la[k] * Pk;
        }
    }
    sh[0][threadIdx.x] = dP;
    sh[1][threadIdx.x] = S;
    sh[2][threadIdx.x] = T;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int v = 0; v < 3; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
        __syncthreads();
    }
    dP = sh[0][0];
    S = sh[1][0];
    T = sh[2][0];
    const bool redis = hi > lo && S > 0.0;
    for (int k = threadIdx.x; k < p.n_bus; k += blockDim.x) {
        double d = 0.0;
        if (k > 0 && !bad) {
            const double Pk = p.P[k];
            if (in_interval(p.pre_bus[k], lo, hi))
                d = redis ? T / S : 0.0;
            else if (redis && Pk > 0.0)
                d = la[k] * (1.0 + dP / S) - T * dP / (S * S);
            else
                d = la[k];
        }
        p.grad_p[(size_t)s * p.n_bus + k] = d;
    }
}

// ---------------------------------------------------------------------------
// Fast-decoupled power flow (see FdpfParams).

__device__ __forceinline__ bool fdpf_island(const FdpfParams &p, int c, int k) {
    return c >= 0 && in_interval(p.pre_bus[k], p.isl_lo[c], p.isl_hi[c]);
}

__global__ void fdpf_start_kernel(FdpfParams p) {
    const int s = blockIdx.x;
    const int k = blockIdx.y * blockDim.x + threadIdx.x;
    if (k >= p.n_bus) return;
    const size_t o = (size_t)s * p.n_bus + k;
    p.theta[o] = k ? p.theta0[k] : 0.0;
    p.V[o] = k ? p.V0[k] : 1.0;
}

// re-dispatch factor of each scenario (Section IV.C) and its no-generator
// flag; clears the accumulated iterations and status
__global__ void __launch_bounds__(256) fdpf_redispatch_kernel(FdpfParams p) {
    __shared__ double sh[2][256];
    const int s = blockIdx.x;
    const int c = p.outages[s];
    const bool ok = c >= 0 && c < p.m;
    double dP = 0.0, S = 0.0;
    for (int k = 1 + threadIdx.x; k < p.n_bus; k += blockDim.x) {
        const double Pk = p.P[k];
        if (ok && fdpf_island(p, c, k))
            dP += Pk;
        else if (Pk > 0.0)
            S += Pk;
    }
    sh[0][threadIdx.x] = dP;
    sh[1][threadIdx.x] = S;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool island = ok && p.isl_hi[c] > p.isl_lo[c];
        p.gfac[s] = (island && sh[1][0] > 0.0) ? sh[0][0] / sh[1][0] : 0.0;
        p.nogen[s] = (island && !(sh[1][0] > 0.0)) ? 1 : 0;
        p.iters[s] = 0;
        p.status[s] = (c < -1 || c >= p.m) ? kBadOutage : kConverged;
    }
}

// rhs = (specified - taken) / V at every main-system load bus, 0 elsewhere
//   half 0: P_k = sum_e V_k V_j b_e sin(theta_k - theta_j)
//   half 1: Q_k = V_k^2 (sum_e b_e + b_sh,k) - sum_e V_k V_j b_e cos(theta_k - theta_j)
// over the branches e = (k, j) in service (the outaged one is skipped).
__global__ void fdpf_mismatch_kernel(FdpfParams p, int half) {
    const int s = blockIdx.x;
    const int k = blockIdx.y * blockDim.x + threadIdx.x;
    if (k >= p.n_bus) return;
    const int c = p.outages[s];
    const size_t o = (size_t)s * p.n_bus + k;
    if (k == 0 || c < -1 || c >= p.m || fdpf_island(p, c, k)) {
        p.rhs[o] = 0.0;
        return;
    }
    const double *th = p.theta + (size_t)s * p.n_bus;
    const double *V = p.V + (size_t)s * p.n_bus;
    const double tk = th[k], vk = V[k];
    double acc = 0.0, cut = 0.0;
    for (int t = p.inc_ptr[k]; t < p.inc_ptr[k + 1]; ++t) {
        const int e = p.inc_br[t];
        if (e == c) {
            cut += p.br_b[e];
            continue;
        }
        const int j = (p.br_from[e] == k) ? p.br_to[e] : p.br_from[e];
        const double w = vk * V[j] * p.br_b[e];
        const double d = tk - th[j];
        acc += half ? -w * cos(d) : w * sin(d);
    }
    double r;
    if (half == 0) {
        const double Pk = p.P[k];
        const double g = p.gfac[s];
        const double spec = (g != 0.0 && Pk > 0.0) ? Pk + Pk * g : Pk;
        r = spec - acc;
    } else {
        const double taken = vk * vk * (p.diag_bpp[k] - cut) + acc;
        r = p.Q[k] - taken;
    }
    p.rhs[o] = r / vk;
}

// state += the half-iteration's correction; accumulate its solve's work
__global__ void fdpf_update_kernel(FdpfParams p, int half) {
    const int s = blockIdx.x;
    const int k = blockIdx.y * blockDim.x + threadIdx.x;
    if (k >= p.n_bus) return;
    const size_t o = (size_t)s * p.n_bus + k;
    if (half == 0)
        p.theta[o] += p.dx[o];
    else
        p.V[o] += p.dx[o];
    if (k == 0) {
        p.iters[s] += p.it_step[s];
        const int a = p.status[s], b = p.st_step[s];
        const bool fail_b = b == kMaxIter || b == kBreakdown || b == kNonfinite;
        const bool fail_a = a == kMaxIter || a == kBreakdown || a == kNonfinite || a == kBadOutage;
        if (!fail_a && (fail_b || a == kConverged)) p.status[s] = b;
    }
}

// islanded buses (and every bus of a bad outage id) report theta = 0, V = 1
__global__ void fdpf_finish_kernel(FdpfParams p) {
    const int s = blockIdx.x;
    const int k = blockIdx.y * blockDim.x + threadIdx.x;
    if (k >= p.n_bus) return;
    const int c = p.outages[s];
    const size_t o = (size_t)s * p.n_bus + k;
    if (c < -1 || c >= p.m || fdpf_island(p, c, k)) {
        p.theta[o] = 0.0;
        p.V[o] = 1.0;
    }
    if (k == 0 && p.nogen[s] && p.status[s] == kConvergedIslanded) p.status[s] = kIslandedNoGen;
}

// Overload screening: per scenario the count of |f_e| > F_e, the largest
// loading |f_e| / F_e and the lowest branch index that reaches it.
__global__ void __launch_bounds__(256) screen_kernel(int m, const double *flows, const double *F, int32_t *count,
                                                     double *worst, int32_t *worst_branch) {
    __shared__ int sc[256];
    __shared__ double sw[256];
    __shared__ int sb[256];
    const int s = blockIdx.x;
    const double *f = flows + (size_t)s * m;
    int n = 0, wb = -1;
    double w = 0.0;
    for (int e = threadIdx.x; e < m; e += blockDim.x) {
        const double a = fabs(f[e]);
        if (a > F[e]) ++n;
        const double l = a / F[e];
        if (l > w) {  // e increases within a thread: the first maximum wins
            w = l;
            wb = e;
        }
    }
    sc[threadIdx.x] = n;
    sw[threadIdx.x] = w;
    sb[threadIdx.x] = wb;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const int t = threadIdx.x + o;
            sc[threadIdx.x] += sc[t];
            if (sw[t] > sw[threadIdx.x] || (sw[t] == sw[threadIdx.x] && sb[t] >= 0 &&
                                            (sb[threadIdx.x] < 0 || sb[t] < sb[threadIdx.x]))) {
                sw[threadIdx.x] = sw[t];
                sb[threadIdx.x] = sb[t];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        count[s] = sc[0];
        worst[s] = sw[0];
        worst_branch[s] = sb[0];
    }
}

// out[j] = sum_r w[r] a[r * lda + j], rows summed in order (deterministic)
__global__ void weighted_rows_kernel(int n_rows, int n_cols, const double *a, int lda, const double *w,
                                     double *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_cols) return;
    double acc = 0.0;
    for (int r = 0; r < n_rows; ++r) acc += w[r] * a[(size_t)r * lda + j];
    out[j] = acc;
}

// Sort key of a scenario (the queue hands out the largest keys first).  An
// outage solved before by this context is ranked by the iterations it took
// then (hist[c + 1]); one without such a record ranks above all of those,
// and among themselves such outages go islanding first, then by the base
// flow on the outaged branch (the start residual of a non-islanding outage
// is that flow across the branch).
__global__ void order_keys_kernel(int n, const int32_t *outages, int m, const int32_t *br_from, const int32_t *br_to,
                                  const double *br_b, const int32_t *isl_lo, const int32_t *isl_hi,
                                  const double *theta_b, const int32_t *hist, uint32_t *keys, int32_t *iota) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int c = outages[j];
    uint32_t key = 0;
    if (c < -1 || c >= m) {
        key = 0u;  // nothing to solve: last
    } else if (hist && hist[c + 1] >= 0) {
        key = (uint32_t)min(hist[c + 1], (1 << 20) - 1) << 10;
    } else if (c >= 0) {
        const float f = (float)fabs(br_b[c] * (theta_b[br_from[c]] - theta_b[br_to[c]]));
        key = 0x80000000u | (isl_hi[c] > isl_lo[c] ? 0x40000000u : 0u) | (__float_as_uint(f) >> 2);
    } else {
        key = 0x80000000u;
    }
    keys[j] = key;
    iota[j] = j;
}

// hist[c + 1] = the iterations scenario s took (its outage c), for the
// next solve's ranking
__global__ void record_iters_kernel(int n, const int32_t *outages, int m, const int32_t *iters, int32_t *hist) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int c = outages[j];
    if (c >= -1 && c < m) hist[c + 1] = iters[j];
}

__global__ void order_inverse_kernel(int n, const int32_t *order, int32_t *pos) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) pos[order[j]] = j;
}
}  // namespace


// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free solve.  Each GPU holds its own
// copy until the process ends; every call on a GPU shares it.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

size_t sort_temp_bytes(int n) {
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                             (const int32_t *)nullptr, (int32_t *)nullptr, n);
    return bytes;
}

hipError_t launch_order(int n, const int32_t *outages, int m, const int32_t *br_from, const int32_t *br_to,
                        const double *br_b, const int32_t *isl_lo, const int32_t *isl_hi, const double *theta_b,
                        const int32_t *hist, uint32_t *keys, uint32_t *keys_sorted, int32_t *iota, int32_t *order,
                        int32_t *pos, void *temp, size_t temp_bytes, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(order_keys_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, outages, m, br_from, br_to, br_b,
                       isl_lo, isl_hi, theta_b, hist, keys, iota);
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_sorted, iota, order, n, 0, 32, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(order_inverse_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, order, pos);
    return hipGetLastError();
}

hipError_t launch_record_iters(int n, const int32_t *outages, int m, const int32_t *iters, int32_t *hist,
                               hipStream_t st) {
    if (n <= 0 || !hist) return hipSuccess;
    hipLaunchKernelGGL(record_iters_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, outages, m, iters, hist);
    return hipGetLastError();
}

hipError_t launch_outputs(const OutParams &prm, hipStream_t st) {
    if (prm.n_out <= 0) return hipSuccess;
    const int tb = 256;
    if (prm.island_out)
        hipLaunchKernelGGL(island_out_kernel, dim3(prm.n_out, (prm.n_bus + tb - 1) / tb), dim3(tb), 0, st, prm);
    if (prm.flows_out)
        hipLaunchKernelGGL(flows_out_kernel, dim3(prm.n_out, (prm.m + tb - 1) / tb), dim3(tb), 0, st, prm);
    if (prm.resid_out) hipLaunchKernelGGL(resid_kernel, dim3(prm.n_out), dim3(256), 0, st, prm);
    return hipGetLastError();
}

hipError_t launch_base_residual(int n_r, const int32_t *rowptr, const int32_t *col, const double *val,
                                const double *theta_b, const double *rhs, const int32_t *bus_map, double *rho,
                                hipStream_t st) {
    if (n_r <= 0) return hipSuccess;
    hipLaunchKernelGGL(base_residual_kernel, dim3((n_r + 255) / 256), dim3(256), 0, st, n_r, rowptr, col, val, theta_b,
                       rhs, bus_map, rho);
    return hipGetLastError();
}

hipError_t launch_base_accumulate(int n_bus, double *theta_b, const double *x, hipStream_t st) {
    if (n_bus <= 1) return hipSuccess;
    hipLaunchKernelGGL(base_accumulate_kernel, dim3((n_bus + 255) / 256), dim3(256), 0, st, n_bus, theta_b, x);
    return hipGetLastError();
}

hipError_t launch_sumsq(int n, const double *v, double *out, hipStream_t st) {
    hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(256), 0, st, n, v, out);
    return hipGetLastError();
}

hipError_t launch_overload_seed(const OverloadParams &prm, hipStream_t st) {
    if (prm.n_out <= 0) return hipSuccess;
    const int tb = 256;
    hipLaunchKernelGGL(overload_seed_kernel, dim3(prm.n_out, (prm.n_bus + tb - 1) / tb), dim3(tb), 0, st, prm);
    hipLaunchKernelGGL(overload_loss_kernel, dim3(prm.n_out), dim3(256), 0, st, prm);
    return hipGetLastError();
}

hipError_t launch_overload_grads(const OverloadParams &prm, hipStream_t st) {
    if (prm.n_out <= 0) return hipSuccess;
    const int tb = 256;
    if (prm.grad_x)
        hipLaunchKernelGGL(overload_grad_x_kernel, dim3(prm.n_out, (prm.m + tb - 1) / tb), dim3(tb), 0, st, prm);
    if (prm.grad_p) hipLaunchKernelGGL(overload_grad_p_kernel, dim3(prm.n_out), dim3(256), 0, st, prm);
    return hipGetLastError();
}

hipError_t launch_fdpf(const FdpfParams &prm, int phase, int half, hipStream_t st) {
    if (prm.n_out <= 0) return hipSuccess;
    const int tb = 256;
    const dim3 grid(prm.n_out, (prm.n_bus + tb - 1) / tb);
    switch (phase) {
        case 0:
            hipLaunchKernelGGL(fdpf_start_kernel, grid, dim3(tb), 0, st, prm);
            hipLaunchKernelGGL(fdpf_redispatch_kernel, dim3(prm.n_out), dim3(256), 0, st, prm);
            break;
        case 1: hipLaunchKernelGGL(fdpf_mismatch_kernel, grid, dim3(tb), 0, st, prm, half); break;
        case 2: hipLaunchKernelGGL(fdpf_update_kernel, grid, dim3(tb), 0, st, prm, half); break;
        case 3: hipLaunchKernelGGL(fdpf_finish_kernel, grid, dim3(tb), 0, st, prm); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_screen(int n_out, int m, const double *flows, const double *F, int32_t *count, double *worst,
                         int32_t *worst_branch, hipStream_t st) {
    if (n_out <= 0) return hipSuccess;
    hipLaunchKernelGGL(screen_kernel, dim3(n_out), dim3(256), 0, st, m, flows, F, count, worst, worst_branch);
    return hipGetLastError();
}

hipError_t launch_weighted_rows(int n_rows, int n_cols, const double *a, int lda, const double *w, double *out,
                                hipStream_t st) {
    if (n_cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(weighted_rows_kernel, dim3((n_cols + 255) / 256), dim3(256), 0, st, n_rows, n_cols, a, lda, w,
                       out);
    return hipGetLastError();
}

template <int S>
static hipError_t launch_spmm_s(const SpmmParams &prm, int bw, int ch, int nseg, int max_nnz, double *partial,
                                hipStream_t st) {
    const int n_tiles = prm.ncols / S;
    const int n_chunks = (prm.n_r + ch - 1) / ch;
    const int n_segs = (n_chunks + nseg - 1) / nseg;
    const size_t lds = spmm_lds_bytes(S, bw, ch, max_nnz);
    auto kern = spmm_kernel<S>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int groups = (n_tiles + kXcds - 1) / kXcds;
    hipLaunchKernelGGL(kern, dim3((unsigned)(groups * kXcds * n_segs)), dim3(kSpmmThreads), lds, st, prm, bw, ch,
                       nseg, n_segs, max_nnz, partial);
    if (partial && prm.pq)
        hipLaunchKernelGGL(spmm_pq_reduce_kernel, dim3((prm.ncols + 255) / 256), dim3(256), 0, st, prm.ncols,
                           n_segs, partial, prm.pq);
    return hipGetLastError();
}

size_t spmm_lds_bytes(int S, int bw, int ch, int max_nnz) {
    return (size_t)(ch + 2 * bw) * S * sizeof(double) + (size_t)max_nnz * (sizeof(double) + sizeof(int)) +
           (size_t)(2 * ch + 1) * sizeof(int);
}

bool spmm_chunk_fits(int S, int ch, int max_nnz) {
    const int vw = (S % 2 == 0) ? 2 : 1;
    return ch >= kSpmmThreads / S && ch % (kSpmmThreads / S) == 0 && ch * S <= kSpmmLoadsP * kSpmmThreads * vw &&
           max_nnz <= kSpmmLoadsA * kSpmmThreads && ch + 1 <= kSpmmLoadsR * kSpmmThreads;
}

hipError_t launch_spmm_partial(const SpmmParams &prm, int S, int bw, int ch, int nseg, int max_nnz, double *partial,
                               hipStream_t st) {
    if (!spmm_chunk_fits(S, ch, max_nnz) || nseg < 1) return hipErrorInvalidValue;
    switch (S) {
        case 1: return launch_spmm_s<1>(prm, bw, ch, nseg, max_nnz, partial, st);
        case 2: return launch_spmm_s<2>(prm, bw, ch, nseg, max_nnz, partial, st);
        case 4: return launch_spmm_s<4>(prm, bw, ch, nseg, max_nnz, partial, st);
        case 8: return launch_spmm_s<8>(prm, bw, ch, nseg, max_nnz, partial, st);
        case 16: return launch_spmm_s<16>(prm, bw, ch, nseg, max_nnz, partial, st);
        case 32: return launch_spmm_s<32>(prm, bw, ch, nseg, max_nnz, partial, st);
        case 64: return launch_spmm_s<64>(prm, bw, ch, nseg, max_nnz, partial, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gpcg
