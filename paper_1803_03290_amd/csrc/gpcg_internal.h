// Internal declarations shared by the host side (gpcg_host.cpp) and the
// device kernels (gpcg_kernels.hip) of the batched contingency PCG library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpcg {

constexpr int kWave = 64;     // gfx950 wavefront width
constexpr int kVectors = 5;   // per tile: delta, r, p, q, y/z
constexpr int kLdsBudget = 64 * 1024;  // bytes of ring per wavefront (two waves fit one CU)

enum Status : int32_t {
    kConverged = 0,
    kMaxIter = 1,
    kBreakdown = 2,
    kNonfinite = 3,
    kConvergedIslanded = 4,
    kIslandedNoGen = 5,
    kBadOutage = 6,
};

// Everything one launch of the tile kernel needs.  All pointers are device
// memory.  Reduced row i is bus i + 1.
struct PcgParams {
    int n_r, n_bus, m, kind;
    // base matrix A (reduced, CSR)
    const int32_t *a_rowptr, *a_col;
    const double *a_val;
    // strictly lower factor L (unit diagonal implied)
    const int32_t *l_rowptr, *l_col;
    const double *l_val;
    // strictly upper part of U, and 1 / diag(U)
    const int32_t *u_rowptr, *u_col;
    const double *u_val, *u_invdiag;
    // branch table; br_b = 1 / x
    const int32_t *br_from, *br_to;
    const double *br_b;
    // DFS pre-order number of the bus of each reduced row; island interval per branch
    const int32_t *pre_row;
    const int32_t *isl_lo, *isl_hi;
    // triangular-solve schedules: steps x R row ids (-1 = idle slot)
    const int32_t *sched_f, *sched_b;
    int steps_f, steps_b;
    int wmask_f, wmask_b;  // ring rows - 1 (ring rows are a power of two)
    // base state and its double-double residual for this right-hand side
    const double *theta_b;  // n_bus, slack 0
    const double *rho_b;    // n_r: rhs - A theta_b
    const double *rhs;      // n_bus
    // scenarios
    const int32_t *outages;
    int n_out;
    int tile0;  // first tile of this launch (plain mode launches one tile at a time)
    double tol2;
    int max_iter;
    double *ws;  // tiles x kVectors x n_r x S
    int32_t *iters_out, *status_out;
    double *gfac_out;  // per scenario: re-dispatch factor dP / S_gen (0 when none)
};

struct OutParams {
    int n_r, n_bus, m, kind, S, n_out;
    const int32_t *a_rowptr, *a_col;
    const double *a_val;
    const int32_t *br_from, *br_to;
    const double *br_x, *br_b;
    const int32_t *pre_bus;  // n_bus
    const int32_t *isl_lo, *isl_hi;
    const double *theta_b, *rhs;
    const int32_t *outages;
    const double *ws;
    const int32_t *status;
    const double *gfac;
    double *x_out, *flows_out, *resid_out;
    uint8_t *island_out;
};

struct SpmmParams {
    int n_r, m, ncols;
    const int32_t *a_rowptr, *a_col;
    const double *a_val;
    const int32_t *br_from, *br_to;
    const double *br_b;
    const int32_t *pre_row, *isl_lo, *isl_hi;
    const int32_t *outages;
    const double *p;
    double *q, *pq;
};

// Launchers (gpcg_kernels.hip).  They return hipSuccess or the launch error.
hipError_t launch_pcg(const PcgParams &prm, int S, int n_tiles, int ring_rows, hipStream_t st);
hipError_t launch_outputs(const OutParams &prm, hipStream_t st);
hipError_t launch_base_residual(int n_r, const int32_t *rowptr, const int32_t *col, const double *val,
                                const double *theta_b, const double *rhs, double *rho, hipStream_t st);
hipError_t launch_base_accumulate(int n_r, double *theta_b, const double *delta, hipStream_t st);
// q = A_c p over ncols / S tiles; partial: f64[spmm_chunks(n_r) * ncols]
// scratch for the p'q column sums (NULL when prm.pq is NULL).
int spmm_chunks(int n_r);
hipError_t launch_spmm_partial(const SpmmParams &prm, int S, double *partial, hipStream_t st);
hipError_t launch_sumsq(int n, const double *v, double *out, hipStream_t st);

}  // namespace gpcg
