/*
 * gpcg.h - C ABI of the MI355X (gfx950) batched PCG library for "N-1"
 * contingency screening with a base-case ILU preconditioner
 * (Zhao, Yuan, Liu, Grinberg, arXiv 1803.03290).
 *
 * What the library computes.  For a lossless, tap-free grid with bus 0 as
 * the slack, the fast-decoupled susceptance system (B' of eq. 4, or B'' of
 * eq. 5) loses one branch per scenario; Section IV.B notes that only four
 * entries of the matrix change.  Every scenario is solved by preconditioned
 * conjugate gradient (Section III) started from the base-case state
 * (Section III.B, last paragraph) and preconditioned by the incomplete LU
 * factors of the unmodified base-case matrix (Section IV.B, eqs. 6-7).
 * Outages that island part of the grid are found by an exact integer bridge
 * pass; the islanded buses are held at zero and, for B', their power is
 * re-dispatched proportionally over the remaining main-system generators
 * (Section IV.C).
 *
 * Conventions shared by every entry point.
 *  - Bus 0 is the slack.  The reduced system drops it, so n_r = n_bus - 1.
 *    Its rows are the non-slack buses in a row order: bus k + 1 in row k,
 *    or the order of a permutation (gpcg_options.perm, or the library's own
 *    reverse Cuthill-McKee order with gpcg_options.reorder).  A banded row
 *    order makes the ILU(0) preconditioner much stronger and is what the
 *    kernels' LDS windows need.  Matrices (A, L, U) are in row order; every
 *    array indexed by bus (injections, angles, island flags, ...) is in the
 *    caller's bus numbering whatever the row order; arrays indexed by
 *    branch follow the caller's branch table.
 *  - Matrices are CSR with int32 indices, column indices sorted within
 *    each row, FP64 values.
 *  - "host" pointers are ordinary CPU memory and are only read during the
 *    call.  "device" pointers are HIP device memory on the context's GPU
 *    (for example torch tensors); the library never frees them.
 *  - Every function returns GPCG_OK (0) or a negative GPCG_E_* code and
 *    never lets a C++ exception escape; gpcg_last_error() then holds a
 *    message for the calling thread.
 *  - Solves are asynchronous on the context's stream: device outputs are
 *    valid once that stream has been synchronised.
 *  - A context must not be used by two threads at once; distinct contexts
 *    are independent.
 */
#ifndef GPCG_H
#define GPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define GPCG_OK 0
#define GPCG_E_ARG (-1)         /* bad argument: null pointer, size, id out of range */
#define GPCG_E_HIP (-2)         /* a HIP runtime call failed */
#define GPCG_E_NOMEM (-3)       /* host or device allocation failed */
#define GPCG_E_PATTERN (-4)     /* CSR or factor pattern is malformed */
#define GPCG_E_PIVOT (-5)       /* zero or negative pivot in a factor */
#define GPCG_E_UNSUPPORTED (-6) /* the grid or block width exceeds a kernel limit */

/* ---- per-scenario outcome (status_out) -------------------------------- */
#define GPCG_CONVERGED 0           /* ||r|| <= tol ||b|| reached */
#define GPCG_MAX_ITER 1            /* stopped at max_iter */
#define GPCG_BREAKDOWN 2           /* p'Ap <= 0: the operator is not positive definite */
#define GPCG_NONFINITE 3           /* NaN or Inf met (for example in the injections) */
#define GPCG_CONVERGED_ISLANDED 4  /* converged; part of the grid islanded and was re-dispatched */
#define GPCG_ISLANDED_NO_GEN 5     /* converged; islanded, but no main-system generator: the slack absorbs */
#define GPCG_BAD_OUTAGE 6          /* outage id outside [-1, m): nothing solved, outputs zero */

/* ---- system kinds ----------------------------------------------------- */
#define GPCG_KIND_BP 0  /* B' (P-theta, eq. 4): re-dispatch islanded power, branch flows available */
#define GPCG_KIND_BPP 1 /* B'' (Q-V, eq. 5): islanded rows zeroed, no re-dispatch, no flows */

typedef struct gpcg_context *gpcg_t;
typedef struct gpcg_batch *gpcg_batch_t;

/* A CSR matrix in host memory. */
typedef struct {
    int32_t n;             /* rows (= columns) */
    int32_t nnz;           /* stored entries */
    const int32_t *rowptr; /* n + 1 */
    const int32_t *col;    /* nnz, sorted within each row */
    const double *val;     /* nnz */
} gpcg_csr;

/* Solver options (all fields may be zero: then defaults apply). */
typedef struct {
    int32_t kind;          /* GPCG_KIND_BP (default) or GPCG_KIND_BPP */
    int32_t block;         /* scenarios per tile, one of 1,2,4,8,16,32,64; 0 = 64 */
    int32_t base_max_iter; /* iterations per base-case solve step; 0 = 20000 */
    int32_t lookahead;     /* rows the triangular-solve scheduler may look ahead; 0 = 256 */
    int32_t zero_start;    /* 1: every scenario starts from x0 = 0 (the listing of Section III.A)
                              instead of the base state (Section III.B); 0 = base state */
    int32_t reorder;       /* 1: A is given in bus order (row k = bus k + 1) and L, U are NULL;
                              gpcg_setup orders the rows by gpcg_rcm, permutes A and forms the
                              ILU(0) itself (Section IV.B) */
    const int32_t *perm;   /* host, n_bus - 1 entries, or NULL: perm[k] is the bus held in row k
                              (each bus 1 .. n_bus - 1 once); A, L, U are then in that row order */
} gpcg_options;

/* Context facts, for logging and for the roofline accounting. */
typedef struct {
    int32_t n_bus, m, n_r;
    int32_t nnz_a, nnz_l, nnz_u;
    int32_t bandwidth;  /* max |i - j| over the pattern of A */
    int32_t block;      /* S: scenarios per tile */
    int32_t rows_per_step; /* R = 64 / S: rows a wavefront treats per step */
    int32_t ring_fwd, ring_bwd; /* LDS ring rows of the forward / backward solves */
    int32_t steps_fwd, steps_bwd; /* schedule steps of the forward / backward solves */
    int32_t n_bridges;
    int32_t base_iters; /* PCG iterations spent on the base-case solve (all refinement steps) */
    double base_resid;  /* relative residual of the base-case state, double-double */
    int32_t sym_factors; /* 1: U = diag(U) L^T to 1e-12 (M = L U symmetric, as for the ILU(0) of
                            A and the Jacobi pair): r'z is formed as y' D^-1 y in the forward
                            sweep; 0: as r'z in the backward sweep */
} gpcg_info;

/* Message describing the last error of the calling thread ("" if none). */
const char *gpcg_last_error(void);

/* ---- host-side preparation (no GPU involved) --------------------------- */

/*
 * Reduced susceptance matrix of the grid: sum over branches of
 * (1/x_e) u_e u_e^T with u_e = e_from - e_to (B' of eq. 4), plus diag(shunt)
 * when shunt != NULL (B'' of eq. 5, reactor sign), with the slack row and
 * column dropped.  Parallel branches add up.
 *   from, to, x: host, m entries; 0 <= from, to < n_bus, from != to, x > 0.
 *   shunt: host, n_bus entries, or NULL.
 *   perm: host, n_bus - 1 entries, or NULL: rows in that order (row k =
 *     bus perm[k]), else row k = bus k + 1.
 *   rowptr: host output, n_bus entries (n_r + 1).
 *   col, val: host outputs with room for cap entries; cap >= n_bus - 1 + 2m
 *   always suffices.  *nnz_out receives the entry count.
 * Every entry is the exact sum of its terms (each branch's 1/x rounded to
 * FP64, the shunt) rounded once, so the result does not depend on the
 * order of the branch table.  Errors: GPCG_E_ARG (bad branch, bad perm,
 * capacity).
 */
int gpcg_assemble(int32_t n_bus, int32_t m, const int32_t *from, const int32_t *to, const double *x,
                  const double *shunt, const int32_t *perm, int32_t *rowptr, int32_t *col, double *val, int32_t cap,
                  int32_t *nnz_out);

/*
 * Reverse Cuthill-McKee order of the non-slack buses (the graph of the
 * reduced system: branches at the slack left out), a banded row order for
 * gpcg_options.perm.  Every connected piece starts at its bus of least
 * degree, a breadth-first search appends each bus's unvisited neighbours by
 * increasing degree (ties by bus number), and the sequence is reversed.  perm: host output, n_bus - 1 entries (buses 1 .. n_bus - 1).
 * All pointers are host memory.  Errors: GPCG_E_ARG (bad branch).
 */
int gpcg_rcm(int32_t n_bus, int32_t m, const int32_t *from, const int32_t *to, int32_t *perm);

/*
 * Zero-fill incomplete LU of A (Saad, Iterative Methods for Sparse Linear
 * Systems, Alg. 10.4), the preconditioner of Section IV.B: L strictly lower
 * with unit diagonal implied, U upper with the diagonal, such that (I+L)U
 * equals A on the pattern of A.  All pointers are host memory;
 * l_rowptr / u_rowptr have n + 1 entries, l_col / l_val / u_col / u_val room
 * for A->nnz entries.  Counts go to *nnz_l, *nnz_u.
 * Errors: GPCG_E_PATTERN (unsorted row or missing diagonal),
 * GPCG_E_PIVOT (a zero pivot).
 */
int gpcg_ilu0(const gpcg_csr *A, int32_t *l_rowptr, int32_t *l_col, double *l_val, int32_t *nnz_l,
              int32_t *u_rowptr, int32_t *u_col, double *u_val, int32_t *nnz_u);

/*
 * Exact integer topology pass (the islanding detection of Section IV.C):
 * depth-first search from the slack, low-link bridge test keyed by branch
 * id (so parallel branches are never bridges).  All pointers are host
 * memory:
 *   is_bridge: m entries, 1 when removing the branch disconnects the grid;
 *   pre: n_bus entries, depth-first pre-order number of each bus (slack 0);
 *   subtree: n_bus entries, size of each bus's DFS subtree;
 *   island_lo, island_hi: m entries; the buses cut off from the slack by a
 *     bridge c are exactly those with island_lo[c] <= pre[bus] < island_hi[c]
 *     (lo == hi == 0 for other branches).
 * Error GPCG_E_ARG when the grid is not connected.
 */
int gpcg_topology(int32_t n_bus, int32_t m, const int32_t *from, const int32_t *to, uint8_t *is_bridge,
                  int32_t *pre, int32_t *subtree, int32_t *island_lo, int32_t *island_hi);

/* ---- contexts ------------------------------------------------------------ */

/*
 * Create a context on the current HIP device: upload the reduced matrix A
 * (B' or B'') and its factors L (strictly lower, unit diagonal implied) and
 * U (upper with diagonal) - normally the ILU(0) of A, but any factors with
 * the same shapes are accepted, e.g. an exact LU - plus the branch table,
 * run the topology pass and the triangular-solve scheduling, and fix the
 * base state theta_b used as the start of every scenario (Section III.B):
 *   - theta_base != NULL: host, n_bus entries (slack entry ignored);
 *   - otherwise theta_b solves A theta = base_rhs on the device by PCG with
 *     iterative refinement whose residual is formed in double-double.
 * Row order (see the conventions above): A, L, U in bus order (opt NULL or
 * perm NULL), in opt->perm's order, or, with opt->reorder, A in bus order
 * and L = U = NULL: the library orders the rows by gpcg_rcm.  L and U may
 * be NULL without reorder too: the library then forms the ILU(0) of A in
 * the given row order.  Every bus-indexed input and output of the context
 * stays in the caller's numbering.
 * base_rhs: host, n_bus entries (slack entry ignored); required when
 * theta_base is NULL, ignored otherwise.
 * stream: a hipStream_t (NULL = the null stream) on which every later
 * operation of the context is enqueued.
 * Errors: GPCG_E_ARG (fewer than two buses, a branch out of range, a bad
 * perm, perm with reorder, only one of L and U), GPCG_E_UNSUPPORTED (2^20 - 1
 * buses or more, or a row order whose bandwidth needs a larger LDS window
 * than one wavefront may hold at this block: pass perm or reorder).
 * On error *out is NULL and nothing is leaked.
 */
int gpcg_setup(gpcg_t *out, int32_t n_bus, int32_t m, const int32_t *br_from, const int32_t *br_to,
               const double *br_x, const gpcg_csr *A, const gpcg_csr *L, const gpcg_csr *U,
               const double *base_rhs, const double *theta_base, const gpcg_options *opt, void *stream);

/* Free a context and its device memory (NULL is ignored). */
void gpcg_destroy(gpcg_t h);

/* Fill *info with the context's sizes and set-up results. */
int gpcg_get_info(gpcg_t h, gpcg_info *info);

/* Copy the topology pass results into host arrays of m entries (is_bridge)
 * and n_bus entries (theta_base: the base state by the caller's bus, slack
 * entry 0). Either pointer may be NULL. */
int gpcg_get_base(gpcg_t h, uint8_t *is_bridge, double *theta_base);

/* The bridge flags of the integer topology pass (Section IV.C: removing a
 * bridge islands part of the grid): is_bridge, host, m entries. */
int gpcg_bridge_flags(gpcg_t h, uint8_t *is_bridge);

/* The context's row order: perm[k] = the caller's bus held in reduced row
 * k; host, n_bus - 1 entries.  (A stand-alone gpcg_spmm works in rows.) */
int gpcg_get_perm(gpcg_t h, int32_t *perm);

/*
 * Solve n_out outage scenarios (the hot path).  Scenario s takes branch
 * outages[s] out (-1: no outage, the base case itself).  The scenarios are
 * batched S to a tile: one wavefront carries S scenario columns through the
 * whole PCG, so every sweep reads the shared matrix and factor entries once
 * for S right-hand sides.
 *
 *   outages:    device int32[n_out], -1 <= outages[s] < m.
 *   rhs:        device f64[n_bus]: P for B' (slack entry ignored), or the
 *               B'' right-hand side.  Scenario s solves
 *               A_c theta = rhs' on its main rows, where rhs' is rhs after
 *               re-dispatch (B') or with islanded entries zeroed (B'').
 *   tol:        stop when ||r_k||_2 <= tol ||rhs'_M||_2 (recursive residual).
 *   max_iter:   per scenario, >= 1.
 *   x_out:      device f64[n_out * n_bus], scenario-major: angles (B') or
 *               magnitude corrections (B''); 0 at the slack and on islands.
 *   flows_out:  device f64[n_out * m] or NULL; B' only: (theta_from -
 *               theta_to) / x_e, 0 on the outaged branch and inside islands.
 *   iters_out:  device int32[n_out]: step-length updates taken.
 *   status_out: device int32[n_out]: GPCG_CONVERGED ... GPCG_ISLANDED_NO_GEN.
 *   island_out: device uint8[n_out * n_bus] or NULL: 1 on islanded buses.
 *   resid_out:  device f64[n_out] or NULL: true relative residual
 *               ||rhs'_M - A_c theta_M|| / ||rhs'_M|| of the returned
 *               theta, formed in double-double.
 * The scenarios are handed out by an atomic queue to persistent wavefronts
 * (as many as fit the device at once, at most one per S scenarios), each
 * with S scenario columns; a column that stops writes its results and takes
 * the next scenario, heaviest expected work first: an outage this context
 * has solved before is ranked by the iterations it took then, others first
 * (the context keeps one iteration record per outage id and start mode).
 * The order changes no result: every scenario's arithmetic is the same in
 * any column.  Once the context has an iteration record and the workspace
 * exceeds 256 MB (more than the Infinity Cache holds), the sweeps stream
 * their vectors past the caches (a cache hint; the results are the same).
 * Workspace (4 (n_r + 1) S doubles per wavefront) is owned by
 * the context and grows on demand.  Errors: GPCG_E_ARG for NULL required pointers, n_out < 0,
 * max_iter < 1, or flows requested from a B'' context.  Outage ids are read
 * on the device only: an id outside [-1, m) gives that scenario status
 * GPCG_BAD_OUTAGE and zero outputs, the other scenarios are unaffected.
 */
int gpcg_solve_contingencies(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs, double tol,
                             int32_t max_iter, double *x_out, double *flows_out, int32_t *iters_out,
                             int32_t *status_out, uint8_t *island_out, double *resid_out);

/*
 * gpcg_solve_contingencies without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, kernels and results as
 * gpcg_solve_contingencies (bit for bit); its workspace (the re-dispatch
 * factors and the scenario ordering's buffers, about 28 bytes per scenario,
 * then the wavefronts' vectors, 4 (n_r + 1) S doubles each) is carved from
 * a fixed device array of GPCG_NOALLOC_SCRATCH_BYTES that the library holds
 * on every GPU it runs on until the process ends, instead of the context's
 * own growable workspace.  When fewer wavefronts fit than the ordinary
 * solve would run, fewer run (e.g. 255 instead of 700 for the 2,000-bus
 * grid at block 4), each taking more scenarios from the queue.
 *   Limit: a call whose per-scenario buffers and one wavefront's vectors do
 *   not fit fails with GPCG_E_UNSUPPORTED before anything is enqueued (more
 *   than about two million scenarios, or a grid of more than about 30,000
 *   buses at block 64; split the list, or use a smaller block).
 *   Sharing: every call on one GPU uses the same array, from any context, and
 *   the array keeps the last call's contents (nothing in it needs to start at
 *   zero).  Calls that overlap on one GPU (on different streams or threads)
 *   race on it; order them on one stream.  gpcg_get_order after such a call
 *   reads the order from the array, so it must come before the next one.
 */
#define GPCG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int gpcg_solve_contingencies_noalloc(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs, double tol,
                                     int32_t max_iter, double *x_out, double *flows_out, int32_t *iters_out,
                                     int32_t *status_out, uint8_t *island_out, double *resid_out);

/*
 * The batched solve with a right-hand side of its own for every scenario,
 * as the adjoint of a screening loss and the half-iterations of the
 * fast-decoupled power flow need (Section III: eqs. (4)-(5) solved for a
 * given mismatch; adjoint systems for the gradients).  Scenario j solves
 * A_c[M,M] x_M = b_j|M by the same batched PCG with the base-case ILU(0)
 * preconditioner, starting from x = 0; there is no base state and no
 * re-dispatch, islanded buses and the slack get x = 0.
 *   rhs_cols   device f64[n_out * ld], b_j at rhs_cols + j * ld indexed by
 *              bus (the slack's entry is ignored); ld >= n_bus.
 *   x_out      device f64[n_out * n_bus] (scenario-major).
 *   iters_out, status_out, island_out (nullable), resid_out (nullable,
 *              ||b_M - A_c x_M|| / ||b_M|| in double-double): as for
 *              gpcg_solve_contingencies; an islanding outage reports
 *              GPCG_CONVERGED_ISLANDED (never GPCG_ISLANDED_NO_GEN).
 * Errors: GPCG_E_ARG for NULL pointers, ld < n_bus, max_iter < 1 or a bad
 * tol.  Asynchronous on the context's stream, like the other solves.
 */
int gpcg_solve_rhs(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs_cols, int32_t ld, double tol,
                   int32_t max_iter, double *x_out, int32_t *iters_out, int32_t *status_out, uint8_t *island_out,
                   double *resid_out);

/*
 * Smooth branch-overload screening loss of every outage and its gradients
 * by the adjoint method.  The screening quantity is the post-outage branch
 * flow (Section IV: flows of the re-dispatched solution); per scenario
 *     L = sum_e softplus(kappa (|f_e| / F_e - 1)),
 * with caller-given limits F_e (held constant).  The gradients with respect
 * to the bus injections P and the branch reactances x come from one adjoint
 * solve per scenario, A_c[M,M] lambda_M = (dL/dtheta)_M, run by the same
 * batched PCG with the same symmetric base-case ILU(0) preconditioner; the
 * forward angles are recomputed by this call (no iterate is stored).
 *   dL/dx_e = -s_e f_e / x_e + (lambda_f - lambda_t)(theta_f - theta_t) / x_e^2
 *             (s_e = dL/df_e; 0 for the outaged branch),
 *   dL/dP   = (dP'/dP)^T lambda through the re-dispatch of Section IV.C
 *             (0 for the slack's injection).
 * At f_e = 0 the derivative of |f_e| is taken as 0.
 *   rhs          device f64[n_bus]: injections P (slack entry ignored).
 *   flow_limit   device f64[m]: F_e > 0.
 *   loss_out     device f64[n_out].
 *   grad_p_out   device f64[n_out * n_bus] or NULL; grad_x_out device
 *                f64[n_out * m] or NULL (both NULL: loss only, no adjoint).
 *   iters_out, status_out  device int32[2 * n_out]: the forward solve's in
 *                the first n_out, the adjoint solve's in the next n_out
 *                (written only when a gradient is asked for).
 * The context must be a B' context built with these reactances.  Errors:
 * GPCG_E_ARG for NULL pointers, a B'' context or kappa <= 0.  Asynchronous
 * on the context's stream; the workspace (four n_out x n_bus or n_out x m
 * f64 arrays) is kept by the context.
 */
int gpcg_overload_gradients(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs,
                            const double *flow_limit, double kappa, double tol, int32_t max_iter, double *loss_out,
                            double *grad_p_out, double *grad_x_out, int32_t *iters_out, int32_t *status_out);

/*
 * out[j] = sum_r w[r] a[r * lda + j] on the context's stream, rows summed in
 * order: the weighted sum of per-scenario gradient rows that a caller's
 * reverse-mode differentiation needs (not a step of the paper's method).
 * a: device f64[n_rows * lda], lda >= n_cols; w: device f64[n_rows];
 * out: device f64[n_cols].  GPCG_E_ARG for bad sizes or NULL pointers.
 */
int gpcg_weighted_rows(gpcg_t h, int32_t n_rows, int32_t n_cols, const double *a, int32_t lda, const double *w,
                       double *out);

/*
 * Fast-decoupled AC power flow of every outage (Section II, eqs. (1)-(5)):
 * n_outer iterations, each a P-theta half (B'_c dtheta = dP / V, then
 * theta += dtheta) and a Q-V half with the updated angles (B''_c dV = dQ / V,
 * then V += dV), every half a batched PCG solve with one right-hand side
 * per scenario and the base-case ILU(0) of its matrix.  The network is
 * lossless and tap-free (branch reactances only) with bus shunts b_sh; the
 * injections it takes are
 *   P_k = sum_j V_k V_j sin(theta_k - theta_j) / x_kj,
 *   Q_k = V_k^2 (sum_j 1 / x_kj + b_sh,k) - sum_j V_k V_j cos(theta_k - theta_j) / x_kj,
 * over the branches in service.  The slack (bus 0) holds theta = 0, V = 1;
 * every other bus is a load bus with the specified P and Q.  Islanded buses
 * are left out of every equation and reported as theta = 0, V = 1; the
 * islanded active power is re-dispatched as in the DC screening
 * (Section IV.C).
 *   bp, bpp      a B' context and a B'' context (with the shunts on its
 *                diagonal) of the same grid on the same device and stream.
 *   P, Q         device f64[n_bus] specified injections (slack ignored).
 *   theta0, V0   device f64[n_bus], the state every scenario starts from
 *                (a flat start, or the base case's state).
 *   theta_out, V_out  device f64[n_out * n_bus] (scenario-major).
 *   iters_out    device int32[n_out]: PCG iterations over all halves.
 *   status_out   device int32[n_out]: the first failure of any half, else
 *                GPCG_CONVERGED(_ISLANDED) or GPCG_ISLANDED_NO_GEN.
 * The power-flow iteration itself is not checked for convergence: the
 * caller picks n_outer.  Errors: GPCG_E_ARG for NULL pointers, swapped or
 * mismatched contexts, n_outer < 1.  Asynchronous on the shared stream.
 */
int gpcg_fdpf(gpcg_t bp, gpcg_t bpp, int32_t n_out, const int32_t *outages, const double *P, const double *Q,
              const double *theta0, const double *V0, int32_t n_outer, double tol, int32_t max_iter,
              double *theta_out, double *V_out, int32_t *iters_out, int32_t *status_out);

/*
 * Overload screening of solved scenarios (Section IV: the post-outage
 * branch flows are the screening quantity): per scenario, the number of
 * branches with |f_e| > F_e, the largest loading |f_e| / F_e and the branch
 * that carries it (the lowest index among equals).
 *   flows        device f64[n_out * m], e.g. flows_out of a solve.
 *   flow_limit   device f64[m], F_e > 0.
 *   count_out    device int32[n_out]; worst_out device f64[n_out];
 *   worst_branch_out device int32[n_out] (-1 when every flow is 0).
 * GPCG_E_ARG for NULL pointers.  Asynchronous on the context's stream.
 */
int gpcg_screen_overloads(gpcg_t h, int32_t n_out, const double *flows, const double *flow_limit,
                          int32_t *count_out, double *worst_out, int32_t *worst_branch_out);

/*
 * Batches of grids (the uneven multi-grid workload).  A batch fixes, for
 * n_ctx contexts of different grids on one device and stream, their scenario
 * lists, right-hand sides and output buffers (arrays of n_ctx device
 * pointers, given in host arrays), one tile shape for all - block size S and
 * the triangular schedules' look-ahead window (lookahead rows; 0 = each
 * context's own) - tol and max_iter.  Its solve is the batched PCG of
 * gpcg_solve_contingencies for every grid in ONE persistent launch: every
 * wavefront works through the grids heaviest first, taking scenarios from
 * each grid's queue until it is empty, so waves done with a large grid move
 * on to the smaller ones; the launch is captured once in a HIP graph
 * together with each grid's base-state residual and output kernels.
 *   gpcg_batch_create  builds the batch (schedules for S, its own
 *                      workspace and scenario queues per grid), runs one
 *                      solve eagerly, captures the graph;
 *   gpcg_batch_run     ranks each grid's queue, then replays the graph
 *                      (reads the current contents of the input buffers,
 *                      overwrites the outputs).
 * Each solve ranks a grid's queue as gpcg_solve_contingencies does, by the
 * iterations each outage took in the context's previous solve, batch or
 * single (the ranking runs on the batch's stream before the graph), and
 * the graph records this solve's iterations for the next.
 *   gpcg_batch_destroy frees the batch (the contexts must outlive it).
 * flows_out and resid_out may be NULL (or hold NULL entries).  The batch
 * works on a stream of its own ordered after and before the contexts'
 * stream by events, so callers synchronise on the contexts' stream as for a
 * solve.  Errors as for gpcg_solve_contingencies, plus GPCG_E_ARG when the
 * contexts do not share a device and a stream.
 */
int gpcg_batch_create(gpcg_batch_t *out, int32_t n_ctx, const gpcg_t *ctxs, int32_t block, int32_t lookahead,
                      const int32_t *n_outs,
                      const int32_t *const *outages, const double *const *rhs, double tol, int32_t max_iter,
                      double *const *x_out, double *const *flows_out, int32_t *const *iters_out,
                      int32_t *const *status_out, double *const *resid_out);
int gpcg_batch_run(gpcg_batch_t b);
void gpcg_batch_destroy(gpcg_batch_t b);

/*
 * The tile-shape search of the batch autotuner: for each candidate k, block
 * cand[k] and look-ahead window cand_look[k] (cand_look may be NULL: each
 * context's own window), a batch of the same inputs is built and its solve
 * timed (one warm-up, then reps solves, HIP events); ms_out[k] =
 * milliseconds per solve.  Outputs go to scratch buffers.  The caller keeps
 * the best shape (and may cache it per grid set).
 */
int gpcg_batch_tune(int32_t n_ctx, const gpcg_t *ctxs, const int32_t *n_outs, const int32_t *const *outages,
                    const double *const *rhs, double tol, int32_t max_iter, int32_t n_cand, const int32_t *cand,
                    const int32_t *cand_look, int32_t reps, double *ms_out);

/*
 * The same computation with the plain per-scenario PCG: one scenario at a
 * time (S = 1): a single wavefront takes the scenarios one after the other,
 * with its 64 lanes spread over rows instead of scenarios.  Same arguments
 * and results as gpcg_solve_contingencies; this is the baseline the batched
 * form is measured against.
 */
int gpcg_solve_plain(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs, double tol,
                     int32_t max_iter, double *x_out, double *flows_out, int32_t *iters_out, int32_t *status_out,
                     uint8_t *island_out, double *resid_out);

/*
 * One outage-corrected sparse matrix product on its own: q = A_c p for
 * ncols scenario columns, with the outaged branch's coupling removed per
 * column (the edge "shielding" of the GPCG listing in Section III.B) and
 * islanded rows zeroed, plus pq[j] = p_j' q_j.  p and q are device f64
 * blocks in the context's row order (gpcg_get_perm) and tile-interleaved:
 * element (row i, column j) sits at ((j / S) * n_r + i) * S + j % S with
 * S = the context's block; ncols must be a multiple of S.
 * outages: device int32[ncols].  pq: device f64[ncols] or NULL.
 */
int gpcg_spmm(gpcg_t h, int32_t ncols, const int32_t *outages, const double *p, double *q, double *pq);

/*
 * Queue order of the last batched solve: order[j] is the scenario the queue
 * handed out j-th.  Scenarios are ranked by expected work (the iterations
 * the outage took in this context's previous solve; without one, islanding
 * outages, then the base-case flow of the outaged branch) and handed out
 * from the heaviest, so that the last ones to finish are short.  order:
 * host int32[n_out] (n_out of that call).  Synchronises the context's
 * stream.
 */
int gpcg_get_order(gpcg_t h, int32_t n_out, int32_t *order);

/*
 * Work of the last solve's PCG launch, for roofline accounting: *waves =
 * the persistent wavefronts it ran, *wave_iterations = the PCG iterations
 * summed over them (each wavefront iteration sweeps the matrix and factor
 * entries once for its S columns).  Synchronises the context's stream.
 */
int gpcg_get_sweeps(gpcg_t h, int32_t *waves, int64_t *wave_iterations);

/*
 * Kernel timing.  With timing enabled, every solve records a HIP event on
 * the context's stream right before its first PCG kernel launch and one
 * right after its last, so the interval covers the PCG kernel(s) only (not
 * the base residual or output kernels).  gpcg_get_timing waits for the
 * second event of the last solve and returns the interval in milliseconds.
 */
int gpcg_set_timing(gpcg_t h, int enable);
int gpcg_get_timing(gpcg_t h, double *pcg_ms);

#ifdef __cplusplus
}
#endif

#endif /* GPCG_H */
