// Device kernels of the batched "N-1" contingency PCG (gfx950, wave64, FP64).
//
// Layout.  Scenarios are grouped S to a tile; one wavefront owns one tile and
// carries it through the whole preconditioned CG of Section III.A.  Its 64
// lanes are R x S with R = 64 / S: lane = rs * S + sc treats scenario column
// sc and row slot rs.  Every per-scenario vector of a tile is stored
// row-interleaved, element (row i, column sc) at i * S + sc, so one row of S
// columns is S contiguous doubles: a wave touching a row for all its columns
// issues one contiguous S * 8-byte access, and every CSR / factor entry it
// reads is shared by the S columns.
//
// Per tile the workspace holds five vectors: delta (the change of state
// from the base case), r, p, q = A_c p, and y / z (the forward-solve result,
// overwritten by the backward-solve result).
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
#include "gpcg_internal.h"

#include <climits>

namespace gpcg {
namespace {

template <int S>
__device__ __forceinline__ double col_sum(double v) {
    // butterfly over the R lanes of one column; every lane gets the same
    // bits because each addition is commutative
#pragma unroll
    for (int off = S; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ bool in_interval(int v, int lo, int hi) { return v >= lo && v < hi; }

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
// The tile kernel: init, then PCG iterations until every column stops.
template <int S>
__global__ void __launch_bounds__(kWave) pcg_tile_kernel(PcgParams p) {
    constexpr int R = kWave / S;
    extern __shared__ double ring[];
    const int lane = threadIdx.x;
    const int sc = lane % S;
    const int rs = lane / S;
    const int tile = blockIdx.x + p.tile0;
    const int scen = tile * S + sc;
    const bool valid = scen < p.n_out;
    const int nr = p.n_r;
    const size_t vs = (size_t)nr * S;
    double *X = p.ws + (size_t)tile * kVectors * vs;
    double *Rv = X + vs;
    double *Pv = Rv + vs;
    double *Qv = Pv + vs;
    double *Yv = Qv + vs;

    // ---- per-column outage data -------------------------------------------
    int c = valid ? p.outages[scen] : -1;
    const bool bad = valid && (c < -1 || c >= p.m);
    if (bad) c = -1;
    int ic = -1, jc = -1, lo = 0, hi = 0;
    double bc = 0.0;
    if (c >= 0) {
        ic = p.br_from[c] - 1;
        jc = p.br_to[c] - 1;
        bc = p.br_b[c];
        lo = p.isl_lo[c];
        hi = p.isl_hi[c];
    }
    if (bad) {
        lo = 0;
        hi = INT_MAX;
    }
    const bool island = hi > lo;

    // ---- re-dispatch (Section IV.C): islanded power over main generators --
    double dP = 0.0, Sg = 0.0;
    for (int i = rs; i < nr; i += R) {
        const double Pk = p.rhs[i + 1];
        if (in_interval(p.pre_row[i], lo, hi))
            dP += Pk;
        else if (Pk > 0.0)
            Sg += Pk;
    }
    dP = col_sum<S>(dP);
    Sg = col_sum<S>(Sg);
    const bool nogen = island && !(Sg > 0.0);
    const double gfac = (p.kind == 0 && island && !bad && !nogen) ? dP / Sg : 0.0;

    // ---- correction-form start from the base state --------------------------
    // r0 = (P' - P)_M + (P - A theta_b)_M + b_c (theta_b,f - theta_b,t) u_M
    const double thf = (ic >= 0) ? p.theta_b[ic + 1] : 0.0;
    const double tht = (jc >= 0) ? p.theta_b[jc + 1] : 0.0;
    const double corr = bc * (thf - tht);
    double rr = 0.0, bb = 0.0;
    for (int i = rs; i < nr; i += R) {
        double r0 = 0.0;
        if (!in_interval(p.pre_row[i], lo, hi)) {
            const double Pk = p.rhs[i + 1];
            const double dPk = (gfac != 0.0 && Pk > 0.0) ? Pk * gfac : 0.0;
            r0 = dPk + p.rho_b[i];
            if (i == ic) r0 += corr;
            if (i == jc) r0 -= corr;
            const double b = Pk + dPk;
            bb += b * b;
        }
        rr += r0 * r0;
        const size_t o = (size_t)i * S + sc;
        X[o] = 0.0;
        Rv[o] = r0;
        Pv[o] = 0.0;
        Qv[o] = 0.0;
    }
    rr = col_sum<S>(rr);
    bb = col_sum<S>(bb);

    int status = kConverged;
    int iters = 0;
    bool done;
    if (!valid) {
        done = true;
    } else if (bad) {
        done = true;
        status = kBadOutage;
    } else if (!__builtin_isfinite(rr) || !__builtin_isfinite(bb)) {
        done = true;
        status = kNonfinite;
    } else {
        done = rr <= p.tol2 * bb;
    }
    __syncthreads();

    double alpha = 0.0, rho = 0.0;
    for (int k = 0;; ++k) {
        // ---- forward sweep: delta += alpha p, r -= alpha q, y = L^-1 r ----
        double rrp = 0.0;
        const bool upd = alpha != 0.0;
        for (int s = 0; s < p.steps_f; ++s) {
            const int row = (R == 1) ? s : p.sched_f[s * R + rs];
            if (row >= 0) {
                const size_t o = (size_t)row * S + sc;
                double r = Rv[o];
                if (upd) {
                    X[o] += alpha * Pv[o];
                    r -= alpha * Qv[o];
                    Rv[o] = r;
                }
                rrp += r * r;
                double y = r;
                const int e1 = p.l_rowptr[row + 1];
                for (int e = p.l_rowptr[row]; e < e1; ++e)
                    y -= p.l_val[e] * ring[(p.l_col[e] & p.wmask_f) * S + sc];
                ring[(row & p.wmask_f) * S + sc] = y;
                Yv[o] = y;
            }
        }
        __syncthreads();
        rrp = col_sum<S>(rrp);
        if (k > 0 && !done) {
            iters = k;
            if (!__builtin_isfinite(rrp)) {
                done = true;
                status = kNonfinite;
            } else if (rrp <= p.tol2 * bb) {
                done = true;
            }
        }
        if (__all(done)) break;
        if (k >= p.max_iter) {
            if (!done) {
                status = kMaxIter;
                done = true;
            }
            break;
        }

        // ---- backward sweep: z = P_M U^-1 y, rho = r'z ---------------------
        double rzp = 0.0;
        for (int s = 0; s < p.steps_b; ++s) {
            const int row = (R == 1) ? (nr - 1 - s) : p.sched_b[s * R + rs];
            if (row >= 0) {
                const size_t o = (size_t)row * S + sc;
                double z = Yv[o];
                const int e1 = p.u_rowptr[row + 1];
                for (int e = p.u_rowptr[row]; e < e1; ++e)
                    z -= p.u_val[e] * ring[(p.u_col[e] & p.wmask_b) * S + sc];
                z *= p.u_invdiag[row];
                ring[(row & p.wmask_b) * S + sc] = z;
                const double zm = in_interval(p.pre_row[row], lo, hi) ? 0.0 : z;
                Yv[o] = zm;
                rzp += Rv[o] * zm;
            }
        }
        __syncthreads();
        const double rz = col_sum<S>(rzp);
        double beta = (k == 0 || done) ? 0.0 : rz / rho;
        rho = rz;

        // ---- new direction p = z + beta p ----------------------------------
        if (!done) {
            for (int i = rs; i < nr; i += R) {
                const size_t o = (size_t)i * S + sc;
                Pv[o] = Yv[o] + beta * Pv[o];
            }
        }
        __syncthreads();

        // ---- q = A_c p with the outaged branch shielded; sigma = p'q -------
        const double dpc = ((ic >= 0) ? Pv[(size_t)ic * S + sc] : 0.0) - ((jc >= 0) ? Pv[(size_t)jc * S + sc] : 0.0);
        double pqp = 0.0;
        for (int i = rs; i < nr; i += R) {
            double q = 0.0;
            const int e1 = p.a_rowptr[i + 1];
            for (int e = p.a_rowptr[i]; e < e1; ++e) q += p.a_val[e] * Pv[(size_t)p.a_col[e] * S + sc];
            if (i == ic) q -= bc * dpc;
            if (i == jc) q += bc * dpc;
            if (in_interval(p.pre_row[i], lo, hi)) q = 0.0;
            const size_t o = (size_t)i * S + sc;
            Qv[o] = q;
            pqp += Pv[o] * q;
        }
        __syncthreads();
        const double sigma = col_sum<S>(pqp);
        if (!done) {
            if (!__builtin_isfinite(sigma) || !__builtin_isfinite(rho)) {
                done = true;
                status = kNonfinite;
            } else if (!(sigma > 0.0)) {
                done = true;
                status = kBreakdown;
            } else {
                alpha = rho / sigma;
            }
        }
        if (done) alpha = 0.0;
    }

    if (valid && rs == 0) {
        int st = status;
        if (st == kConverged && island) st = (p.kind == 0 && nogen) ? kIslandedNoGen : kConvergedIslanded;
        p.iters_out[scen] = iters;
        p.status_out[scen] = st;
        p.gfac_out[scen] = gfac;
    }
}

// ---------------------------------------------------------------------------
// Outputs: theta = theta_b + delta on the main system, 0 on islands and at
// the slack; island flags.
__global__ void theta_out_kernel(OutParams p) {
    const int s = blockIdx.x;
    const int k = blockIdx.y * blockDim.x + threadIdx.x;
    if (k >= p.n_bus) return;
    int c = p.outages[s];
    const bool bad = c < -1 || c >= p.m;
    int lo = 0, hi = 0;
    if (!bad && c >= 0) {
        lo = p.isl_lo[c];
        hi = p.isl_hi[c];
    }
    const bool in = (k > 0) && in_interval(p.pre_bus[k], lo, hi);
    double th = 0.0;
    if (k > 0 && !in && !bad) {
        const int tile = s / p.S, sc = s % p.S;
        th = p.theta_b[k] + p.ws[(size_t)tile * kVectors * p.n_r * p.S + (size_t)(k - 1) * p.S + sc];
    }
    p.x_out[(size_t)s * p.n_bus + k] = th;
    if (p.island_out) p.island_out[(size_t)s * p.n_bus + k] = in ? 1 : 0;
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
    if (e != c && c >= -1 && c < p.m) f = (th[p.br_from[e]] - th[p.br_to[e]]) / p.br_x[e];
    p.flows_out[(size_t)s * p.m + e] = f;
}

// True relative residual ||P'_M - A_c theta_M|| / ||P'_M|| of the returned
// angles, each row's residual formed in double-double.
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
    const double thf = (ic >= 0) ? th[ic + 1] : 0.0, tht = (jc >= 0) ? th[jc + 1] : 0.0;
    double rr = 0.0, bb = 0.0;
    if (!bad) {
        for (int i = threadIdx.x; i < p.n_r; i += blockDim.x) {
            if (in_interval(p.pre_bus[i + 1], lo, hi)) continue;
            const double Pk = p.rhs[i + 1];
            const double b = Pk + ((gfac != 0.0 && Pk > 0.0) ? Pk * gfac : 0.0);
            double h = b, l = 0.0;
            for (int e = p.a_rowptr[i]; e < p.a_rowptr[i + 1]; ++e) dd_fma(h, l, -p.a_val[e], th[p.a_col[e] + 1]);
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

// rho = rhs - A theta_b per reduced row, in double-double, rounded once.
__global__ void base_residual_kernel(int n_r, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                     const double *__restrict__ val, const double *__restrict__ theta_b,
                                     const double *__restrict__ rhs, double *__restrict__ rho) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_r) return;
    double h = rhs[i + 1], l = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) dd_fma(h, l, -val[e], theta_b[col[e] + 1]);
    rho[i] = h + l;
}

__global__ void base_accumulate_kernel(int n_r, double *theta_b, const double *delta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_r) theta_b[i + 1] += delta[i];
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
// Stand-alone outage-corrected product q = A_c p over many tiles.  A wave
// takes a chunk of rows of one tile; the blocks of one tile are placed on
// the same XCD (work-groups are dealt to the 8 XCDs round-robin) so that the
// neighbour rows one wave reads were fetched into that XCD's L2 by another.
constexpr int kSpmmRows = 64;  // rows per wave
constexpr int kXcd = 8;

template <int S>
__global__ void __launch_bounds__(256) spmm_kernel(SpmmParams p, int chunks, int n_tiles, double *partial) {
    constexpr int R = kWave / S;
    const int xcd = blockIdx.x % kXcd;
    const int idx = blockIdx.x / kXcd;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int chunk = (idx % ((chunks + 3) / 4)) * 4 + wave;
    const int tile = (idx / ((chunks + 3) / 4)) * kXcd + xcd;
    if (tile >= n_tiles || chunk >= chunks) return;
    const int sc = lane % S, rs = lane / S;
    const int col = tile * S + sc;
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
    const size_t vs = (size_t)p.n_r * S;
    const double *P = p.p + (size_t)tile * vs;
    double *Q = p.q + (size_t)tile * vs;
    const double dpc = ((ic >= 0) ? P[(size_t)ic * S + sc] : 0.0) - ((jc >= 0) ? P[(size_t)jc * S + sc] : 0.0);
    double pq = 0.0;
    const int r0 = chunk * kSpmmRows, r1 = min(p.n_r, r0 + kSpmmRows);
    for (int i = r0 + rs; i < r1; i += R) {
        double q = 0.0;
        const int e1 = p.a_rowptr[i + 1];
        for (int e = p.a_rowptr[i]; e < e1; ++e) q += p.a_val[e] * P[(size_t)p.a_col[e] * S + sc];
        if (i == ic) q -= bc * dpc;
        if (i == jc) q += bc * dpc;
        if (in_interval(p.pre_row[i], lo, hi)) q = 0.0;
        Q[(size_t)i * S + sc] = q;
        pq += P[(size_t)i * S + sc] * q;
    }
    pq = col_sum<S>(pq);
    if (partial && rs == 0) partial[(size_t)chunk * p.ncols + col] = pq;
}

__global__ void spmm_pq_reduce_kernel(int ncols, int chunks, const double *partial, double *pq) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    double a = 0.0;
    for (int k = 0; k < chunks; ++k) a += partial[(size_t)k * ncols + col];
    pq[col] = a;
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_pcg(const PcgParams &prm, int S, int n_tiles, int ring_rows, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    const size_t lds = (size_t)ring_rows * S * sizeof(double);
    dim3 grid(n_tiles), block(kWave);
    switch (S) {
        case 1: hipLaunchKernelGGL(pcg_tile_kernel<1>, grid, block, lds, st, prm); break;
        case 2: hipLaunchKernelGGL(pcg_tile_kernel<2>, grid, block, lds, st, prm); break;
        case 4: hipLaunchKernelGGL(pcg_tile_kernel<4>, grid, block, lds, st, prm); break;
        case 8: hipLaunchKernelGGL(pcg_tile_kernel<8>, grid, block, lds, st, prm); break;
        case 16: hipLaunchKernelGGL(pcg_tile_kernel<16>, grid, block, lds, st, prm); break;
        case 32: hipLaunchKernelGGL(pcg_tile_kernel<32>, grid, block, lds, st, prm); break;
        case 64: hipLaunchKernelGGL(pcg_tile_kernel<64>, grid, block, lds, st, prm); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_outputs(const OutParams &prm, hipStream_t st) {
    if (prm.n_out <= 0) return hipSuccess;
    const int tb = 256;
    hipLaunchKernelGGL(theta_out_kernel, dim3(prm.n_out, (prm.n_bus + tb - 1) / tb), dim3(tb), 0, st, prm);
    if (prm.flows_out)
        hipLaunchKernelGGL(flows_out_kernel, dim3(prm.n_out, (prm.m + tb - 1) / tb), dim3(tb), 0, st, prm);
    if (prm.resid_out) hipLaunchKernelGGL(resid_kernel, dim3(prm.n_out), dim3(256), 0, st, prm);
    return hipGetLastError();
}

hipError_t launch_base_residual(int n_r, const int32_t *rowptr, const int32_t *col, const double *val,
                                const double *theta_b, const double *rhs, double *rho, hipStream_t st) {
    if (n_r <= 0) return hipSuccess;
    hipLaunchKernelGGL(base_residual_kernel, dim3((n_r + 255) / 256), dim3(256), 0, st, n_r, rowptr, col, val, theta_b,
                       rhs, rho);
    return hipGetLastError();
}

hipError_t launch_base_accumulate(int n_r, double *theta_b, const double *delta, hipStream_t st) {
    if (n_r <= 0) return hipSuccess;
    hipLaunchKernelGGL(base_accumulate_kernel, dim3((n_r + 255) / 256), dim3(256), 0, st, n_r, theta_b, delta);
    return hipGetLastError();
}

hipError_t launch_sumsq(int n, const double *v, double *out, hipStream_t st) {
    hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(256), 0, st, n, v, out);
    return hipGetLastError();
}

int spmm_chunks(int n_r) { return (n_r + kSpmmRows - 1) / kSpmmRows; }

hipError_t launch_spmm_partial(const SpmmParams &prm, int S, double *partial, hipStream_t st) {
    const int n_tiles = prm.ncols / S;
    const int chunks = (prm.n_r + kSpmmRows - 1) / kSpmmRows;
    const int groups = (chunks + 3) / 4;
    const int tile_rounds = (n_tiles + kXcd - 1) / kXcd;
    dim3 grid((unsigned)(tile_rounds * groups * kXcd)), block(256);
    switch (S) {
        case 1: hipLaunchKernelGGL(spmm_kernel<1>, grid, block, 0, st, prm, chunks, n_tiles, partial); break;
        case 2: hipLaunchKernelGGL(spmm_kernel<2>, grid, block, 0, st, prm, chunks, n_tiles, partial); break;
        case 4: hipLaunchKernelGGL(spmm_kernel<4>, grid, block, 0, st, prm, chunks, n_tiles, partial); break;
        case 8: hipLaunchKernelGGL(spmm_kernel<8>, grid, block, 0, st, prm, chunks, n_tiles, partial); break;
        case 16: hipLaunchKernelGGL(spmm_kernel<16>, grid, block, 0, st, prm, chunks, n_tiles, partial); break;
        case 32: hipLaunchKernelGGL(spmm_kernel<32>, grid, block, 0, st, prm, chunks, n_tiles, partial); break;
        case 64: hipLaunchKernelGGL(spmm_kernel<64>, grid, block, 0, st, prm, chunks, n_tiles, partial); break;
        default: return hipErrorInvalidValue;
    }
    if (partial && prm.pq)
        hipLaunchKernelGGL(spmm_pq_reduce_kernel, dim3((prm.ncols + 255) / 256), dim3(256), 0, st, prm.ncols, chunks,
                           partial, prm.pq);
    return hipGetLastError();
}

}  // namespace gpcg
