/*
 * pdhcg.h -- C ABI of the MI355X restarted-PDHG solver for conic convex QP.
 *
 * Problem (paper, introduction, eq. cqp):
 *     minimise  1/2 <x, Q x> + <c, x>   subject to  A x = b,  x in K,
 * with Q = P + R^T D R (implementation section, "General Quadratic
 * Objective") and K a Cartesian product of free, nonnegative, second-order
 * (v, t), rotated second-order (v, s, t), exponential (r, s, t) and 3-D power
 * (x, y, z; exponent alpha) blocks (implementation section, cone list).
 *
 * The implementation form of the same section (eq. solver-input) is also
 * accepted: two-sided row bounds l <= A x <= u and box blocks [l^x, u^x].
 *
 * Method (implementation section): primal-first PDHG operator whose primal
 * step is the conic proximal subproblem (eq. prox-subproblem), solved by one
 * diagonal-metric projection when Q is diagonal (eq. diagonal-q-metric) or by
 * Jacobi-preconditioned projected Barzilai-Borwein iterations
 * (eq. jacobi-bb-step) otherwise; reflected-Halpern epochs (eq. rh-update)
 * or averaged epochs (Alg. 1); adaptive restart (eq. practical-restart-rule);
 * PID primal weight (eq. pid-weight); rescaling (Section "Problem
 * Rescaling"); termination on relative KKT residuals of the unscaled
 * candidate.
 *
 * Conventions
 *  - settings.memory_kind says where the caller's arrays live: with
 *    PDHCG_MEM_HOST (default) every pointer of pdhcg_problem and the
 *    x0/y0/x/y/s arguments of the solve calls is a host pointer; with
 *    PDHCG_MEM_DEVICE each is a device pointer on the current device (the
 *    data of torch CUDA tensors, say).  The library deep-copies problem data
 *    during setup; the caller keeps ownership of every buffer it passes and
 *    may free it after the call returns.  Handles (pdhcg_handle) are opaque,
 *    owned by the library, freed by pdhcg_free.
 *  - Device memory of a handle comes from hipMalloc, or from the caller's
 *    allocator when settings.dev_alloc / dev_free are set (a caching
 *    allocator such as torch's).
 *  - Matrices are CSR with int64 row pointers (length rows+1, starting at 0,
 *    nondecreasing) and int32 column indices in [0, cols); duplicates are
 *    summed; columns need not be sorted.
 *  - Cone blocks must tile 0..n-1 contiguously in increasing start order.
 *  - Functions return PDHCG_OK (0) or a negative error code; nothing throws
 *    across the ABI and nothing aborts.  Solver outcomes are reported in
 *    pdhcg_result.status.
 *  - A handle is not thread-safe; use one handle per host thread.  All device
 *    work is issued on settings.stream (a hipStream_t passed as void*; NULL
 *    means the null stream).
 */
#ifndef PDHCG_H
#define PDHCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes (function return values) ---------------------------- */
#define PDHCG_OK        0
#define PDHCG_E_ARG    -1   /* null pointer, count < 1, bad setting value     */
#define PDHCG_E_SHAPE  -2   /* n < 1, m < 0, r < 0 or inconsistent sizes      */
#define PDHCG_E_CSR    -3   /* bad row pointer or column index out of range   */
#define PDHCG_E_CONE   -4   /* blocks do not tile 0..n-1, bad dim or alpha    */
#define PDHCG_E_NONSYM -5   /* P not symmetric or D not symmetric             */
#define PDHCG_E_MEM    -6   /* host or device allocation failed               */
#define PDHCG_E_HIP    -7   /* a HIP runtime call failed                      */
#define PDHCG_E_STATE  -8   /* call not valid for this handle                 */
#define PDHCG_E_NOTRACE -9  /* trace requested but not recorded               */

/* ---- solver status (pdhcg_result.status) ----------------------------- */
#define PDHCG_OPTIMAL     1
#define PDHCG_MAX_ITER    2
#define PDHCG_TIME_LIMIT  3
#define PDHCG_NUMERICAL   4   /* NaN/Inf detected in the iterates            */
#define PDHCG_ABORTED     5   /* device-side grid barrier timed out          */

/* ---- cone types ------------------------------------------------------- */
#define PDHCG_CONE_FREE   0
#define PDHCG_CONE_NONNEG 1
#define PDHCG_CONE_SOC    2   /* (v, t): ||v|| <= t, dim >= 1                 */
#define PDHCG_CONE_RSOC   3   /* (v, s, t): ||v||^2 <= 2 s t, s,t >= 0, dim>=2 */
#define PDHCG_CONE_EXP    4   /* (r, s, t): cl{s > 0, s e^{r/s} <= t}, dim 3  */
#define PDHCG_CONE_POW    5   /* (x, y, z): x^a y^(1-a) >= |z|, dim 3,
                                 alpha in (0, 1)                              */
#define PDHCG_CONE_BOX    6   /* x_i in [x_lo_i, x_hi_i] on each coordinate of
                                 the block (the box set of eq. solver-input;
                                 bounds from pdhcg_problem.x_lo / x_hi)      */
#define PDHCG_CONE_EXP1   7   /* (z, s, t) with s fixed at 1 and e^z <= t, dim
                                 3: an exponential-cone block whose middle
                                 coordinate is fixed at one, as in the Fisher
                                 experiment (Section "Large-Scale Fisher
                                 Equilibrium"); a convex set, not a cone    */

/* ---- enumerations in settings ---------------------------------------- */
#define PDHCG_MEM_HOST    0   /* caller arrays are host memory                */
#define PDHCG_MEM_DEVICE  1   /* caller arrays are device memory              */
#define PDHCG_SCHEME_RH   0   /* reflected-Halpern epochs (eq. rh-update)     */
#define PDHCG_SCHEME_AVG  1   /* averaged epochs of Alg. 1                    */
#define PDHCG_INNER_JACOBI 0  /* eq. jacobi-bb-step                           */
#define PDHCG_INNER_EUCLID 1  /* eq. bb-step                                  */
#define PDHCG_SCALE_BLOCK 0   /* cone-preserving block scaling
                                 (eq. cone-preserving-scaling): one common
                                 factor per cone block, S_j K_j = K_j       */
#define PDHCG_SCALE_CONE  1   /* rescaled-cone mode: coordinatewise factors
                                 (eq. cone-scaling-candidates) on SOC, RSOC,
                                 EXP and POW blocks, which become S_j K_j
                                 and are projected through
                                 eq. scaling-induced-metric; EXP1 blocks keep
                                 one common factor (their set is not a cone)*/
#define PDHCG_ORDER_CALLER -1 /* device coordinate order (settings.interleave):
                                 the caller's                                */
#define PDHCG_ORDER_AUTO   0  /* DEGREE where it applies (see interleave)    */
#define PDHCG_ORDER_CONES  1  /* cone blocks interleaved with FREE/R+        */
#define PDHCG_ORDER_DEGREE 2  /* columns by nonzero count, dealt to ranges   */
#define PDHCG_PREC_FP64   0
#define PDHCG_PREC_FP32   1   /* FP32 copies of A, A^T, P, R for the bulk
                                 sweeps (A^T y, P u, R u, A w; FP32 products
                                 and row sums); FP64 iterates, reductions,
                                 restart and KKT checks (checks use the FP64
                                 data) and cone root-finding; then an FP64
                                 polish (single problems only)              */

typedef struct {
    int32_t n;                    /* primal dimension                         */
    int32_t m;                    /* number of equality rows (may be 0)       */
    /* A: m x n CSR */
    const int64_t* A_rowptr;      /* m+1                                      */
    const int32_t* A_col;         /* A_nnz                                    */
    const double*  A_val;         /* A_nnz                                    */
    const double*  b;             /* m                                        */
    const double*  c;             /* n                                        */
    /* P: n x n symmetric sparse part of Q, full storage, CSR; nullable       */
    const int64_t* P_rowptr;
    const int32_t* P_col;
    const double*  P_val;
    /* R: r x n row-major dense factor and D: r x r symmetric; nullable      */
    int32_t        r;
    const double*  R;
    const double*  D;             /* NULL with R != NULL means D = I          */
    /* cone blocks */
    int32_t        nblocks;
    const int32_t* cone_type;     /* PDHCG_CONE_*                             */
    const int32_t* cone_start;
    const int32_t* cone_dim;
    const double*  cone_alpha;    /* read for POW blocks only; nullable       */
    /* implementation form (eq. solver-input), all nullable:
     * row_lo, row_hi (m): row_lo <= A x <= row_hi replaces A x = b (b may
     *   then be NULL); -INFINITY / +INFINITY mark absent endpoints, equal
     *   endpoints an equality; both or neither must be given;
     * x_lo, x_hi (n): bounds of the coordinates of PDHCG_CONE_BOX blocks
     *   (read there only; required when such a block exists).
     * Invalid: NaN, lo > hi, a lower endpoint +INFINITY or an upper
     * endpoint -INFINITY (PDHCG_E_ARG).                                      */
    const double*  row_lo;
    const double*  row_hi;
    const double*  x_lo;
    const double*  x_hi;
} pdhcg_problem;

typedef void* (*pdhcg_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*pdhcg_free_fn)(void* ptr, void* stream, void* ctx);

/* Opaque solver handle: the scaled instances on the device, their step
 * sizes and solver state.                                                   */
typedef struct pdhcg_handle pdhcg_handle;

typedef struct {
    /* termination */
    double  tol;                  /* relative KKT tolerance (default 1e-6)    */
    int64_t max_iter;             /* outer PDHG evaluations (default 1e6)     */
    double  time_limit;           /* seconds (default 3600)                   */
    int32_t check_every;          /* restart / KKT check period (default 64)  */
    /* scheme */
    int32_t scheme;               /* PDHCG_SCHEME_* (default RH)              */
    double  rho;                  /* reflection coefficient in [1/2, 1] (1)   */
    int32_t avg_epoch;            /* T of Alg. 1 (default 64)                 */
    /* inner solve (general Q) */
    int32_t inner;                /* PDHCG_INNER_* (default JACOBI)           */
    int32_t fixed_inner;          /* >0: exactly that many inner steps        */
    int32_t j_max;                /* inner step cap (default 500)             */
    double  eps_in0, gamma_in, eps_min;   /* (1e-3, 5e-4, 1e-9)              */
    /* restart and primal weight */
    double  beta_s, beta_n, beta_a;       /* (0.2, 0.8, 0.36)                 */
    double  pid_beta_i, pid_kp, pid_ki, pid_kd;  /* (0.3, 0.99, 0.01, 0)     */
    /* rescaling */
    int32_t scaling;              /* master switch (default 1)                */
    int32_t ruiz_iters;           /* default 10                               */
    int32_t pock_chambolle;       /* default 1                                */
    double  pc_alpha;             /* default 1                                */
    int32_t bound_objective;      /* default 1                                */
    /* step size */
    int32_t power_iters;          /* default 128                              */
    double  a_norm;               /* >0 overrides the power iteration         */
    double  omega0;               /* >0 overrides the initial primal weight   */
    /* execution */
    int32_t precision;            /* PDHCG_PREC_* (default FP64)              */
    int32_t trace_iters;          /* record the first k outer iterations      */
    int32_t block_dim;            /* 0 = auto                                 */
    int32_t grid_dim;             /* 0 = auto; 1 runs the single-workgroup
                                     variant, whose arithmetic is that of a
                                     batch solve of the same instance        */
    int32_t lanes_at;             /* lanes per row of A^T / P (0 = auto)      */
    int32_t lanes_a;              /* lanes per row of A (0 = auto)            */
    int32_t host_poll;            /* outer iterations per launch (default 512)*/
    void*   stream;               /* hipStream_t                              */
    int32_t verbose;              /* bit 0: a progress line on stderr per
                                     launch (at most every 5 s) in
                                     pdhcg_solve                             */
    int32_t time_kernels;         /* 1: time every solver launch with HIP
                                     events on `stream` (result.kernel_s)     */
    int32_t autotune;             /* batches: 1 = choose the lanes-per-row
                                     mapping of the A and A^T products by
                                     timing candidate mappings at setup;
                                     0 = the rule of single problems (fewest
                                     dependent memory round trips per pass).
                                     Ignored for single problems.            */
    int32_t tune_iters;           /* outer iterations per autotuner probe (64)*/
    double  fp32_tol;             /* PDHCG_PREC_FP32: tolerance of the FP32
                                     phase; the FP64 polish then restarts at
                                     its candidate and runs to tol
                                     (<= 0: 10 * tol)                         */
    int32_t interleave;           /* PDHCG_ORDER_*: the device's coordinate
                                     order (inputs, outputs, traces and
                                     scalings stay in the caller's order).
                                     CONES: cone blocks interleaved with the
                                     FREE/R+ coordinates, so every workgroup
                                     gets a mix of both kinds of work.
                                     DEGREE (cone-free problems): columns
                                     sorted by their count of nonzeros in A,
                                     the longest (at least 1/8 of a 1/512
                                     share of A's and P's nonzeros, and
                                     4096) first, the rest dealt in turn
                                     to the ranges of 512 left beside the
                                     head's workgroups.
                                     AUTO (default): DEGREE for cone-free
                                     problems with n >= 2^20 whose longest
                                     column holds at least 64 times the mean
                                     count, else the caller's order.
                                     CALLER: the caller's order.             */
    int32_t cone_scaling;         /* PDHCG_SCALE_* (default BLOCK)            */
    int32_t memory_kind;          /* PDHCG_MEM_* of the caller's problem
                                     arrays, warm starts and outputs
                                     (default HOST)                           */
    /* device allocator (both or neither; default NULL = hipMalloc/hipFree):
     * dev_alloc(bytes, stream, ctx) returns device memory on the current
     * device usable on `stream` (settings.stream) or NULL on failure
     * (PDHCG_E_MEM); dev_free(ptr, stream, ctx) releases it.  Called during
     * pdhcg_setup, the solve calls (buffers created on first use) and
     * pdhcg_free, on the calling thread.                                    */
    pdhcg_alloc_fn dev_alloc;
    pdhcg_free_fn  dev_free;
    void*          alloc_ctx;
} pdhcg_settings;

typedef struct {
    int32_t status;               /* PDHCG_OPTIMAL ... PDHCG_ABORTED          */
    int64_t iterations;           /* outer PDHG evaluations                   */
    int64_t inner_iterations;     /* projected-BB steps summed over all       */
    int64_t restarts;
    double  rel_primal, rel_dual, rel_gap;
    double  primal_obj, dual_obj;
    double  setup_s, solve_s;
    double  omega;                /* final primal weight                      */
    double  a_norm;               /* ||A^||_2 used for the step size          */
    /* caller-allocated outputs (host or device memory per
       settings.memory_kind), nullable: x[n], y[m], s[n] (dual slack
       s = Qx + c - A^T y of the original problem at the returned x, y)      */
    double* x;
    double* y;
    double* s;
    /* device time of the solver launches (settings.time_kernels = 1) */
    double  kernel_s;
    int64_t kernel_launches;
    int32_t grid_dim;             /* workgroups of the solver launch          */
    int32_t block_dim;            /* threads per workgroup                    */
    int64_t polish_iterations;    /* FP32 mode: outer iterations of the FP64
                                     polish (included in `iterations`)      */
} pdhcg_result;

/* Per-iteration record for parity checks, in the library's scaled space
 * (x^ = S_x x / nu_b, y^ = y / (nu_c S_y); the scale vectors are returned by
 * pdhcg_get_scaling).  Arrays are caller-allocated host buffers of length
 * count*n (x, wx) and count*m (y, wy), count*1 for the scalars; iteration k
 * occupies the k-th slice.  x, y: Halpern state before the evaluation;
 * wx, wy: PDHG candidate.                                                   */
typedef struct {
    int32_t count;                /* in: slices provided; out: recorded       */
    double* x;  double* y;  double* wx;  double* wy;
    double* tau; double* sigma; double* omega; double* eps_in;
    int32_t* inner; int32_t* restart; int32_t* check; double* E;
} pdhcg_trace;

/* Fill *s with the defaults of the paper's Table practical-defaults and the
 * library's readings (check_every 64, J_max 500, 128 power iterations).
 * Returns PDHCG_E_ARG if s is NULL.                                          */
int pdhcg_default_settings(pdhcg_settings* s);

/* Validate `count` problems, rescale them (Section "Problem Rescaling"),
 * build A^T, estimate ||A^||_2 (eq. practical-stepsizes), upload everything
 * to the current HIP device and return a handle in *out.  count > 1 prepares
 * a batch for pdhcg_solve_batch.  On error *out is left NULL.
 * The host part runs on up to 16 threads (fewer if the environment variable
 * PDHCG_HOST_THREADS says so); its result does not depend on their number. */
int pdhcg_setup(const pdhcg_problem* probs, int32_t count,
                const pdhcg_settings* s, pdhcg_handle** out);

/* Solve the single problem of handle h (count == 1) with the restarted
 * PDHG method of the implementation section: evaluations of the PDHG
 * operator (eq. theory-pdhg-map) whose primal step is the conic proximal
 * subproblem (eq. prox-subproblem), reflected-Halpern epochs (eq. rh-update;
 * or averaged epochs of Alg. 1 with settings.scheme), adaptive restarts
 * (eq. practical-restart-rule) with the PID primal weight (eq. pid-weight),
 * until the relative KKT residuals of the unscaled candidate (eq. kkt-cqp)
 * are within settings.tol, or max_iter / time_limit.  Starts from the
 * optional warm start (x0[n], y0[m], original space, memory_kind memory;
 * NULL means zero).  Fills *res (status, counters, residuals, objectives,
 * timings) and, when non-NULL, res->x, res->y and the dual slack res->s,
 * all computed on the device.  Returns PDHCG_E_STATE for a batch handle,
 * PDHCG_E_HIP when a device call fails (status is then unset).             */
int pdhcg_solve(pdhcg_handle* h, const double* x0, const double* y0, pdhcg_result* res);

/* Solve every problem of a batch handle (count > 1 at setup) in one
 * persistent launch, replayed from a HIP graph: each workgroup takes the next
 * instance from a device queue (largest first) and runs the whole restarted
 * PDHG method on it with that instance's own step sizes, primal weight,
 * restarts and inner tolerance, then takes the next.  Every instance runs to
 * its own termination (tol, max_iter); settings.time_limit bounds the whole
 * launch (instances still running then report PDHCG_TIME_LIMIT).
 * x0s/y0s: NULL or host arrays of `count` pointers (each may be NULL;
 * original space; each pointing to memory_kind memory).  res: array of `count` results; their x/y/s pointers may be set.
 * kernel_s of res[0] holds the device time of the launch; setup_s and
 * solve_s are those of the whole batch.  For a single-problem handle this is
 * pdhcg_solve on res[0].                                                     */
int pdhcg_solve_batch(pdhcg_handle* h, const double* const* x0s, const double* const* y0s,
                      pdhcg_result* res);

/* Copy the recorded iterations of instance `inst` into *t.  Requires
 * settings.trace_iters > 0 at setup; PDHCG_E_NOTRACE otherwise.             */
int pdhcg_get_trace(pdhcg_handle* h, int32_t inst, pdhcg_trace* t);

/* Copy the scaling of instance `inst`: Sx[n], Sy[m] (nullable) and the
 * bound/objective factors nu_b, nu_c (nullable); also eta and omega0.       */
int pdhcg_get_scaling(pdhcg_handle* h, int32_t inst, double* Sx, double* Sy,
                      double* nu_b, double* nu_c, double* eta, double* omega0);

/* Diagnostics of a PDHCG_NUMERICAL status on the current device: *count =
 * number of cone projections of the last solve (or batch) whose
 * root-finding failed; rec[0..7] = the first one's (cone type, r[0..2],
 * metric m[0..2], alpha), zeros when *count is 0.  Reads device memory; call
 * after the solve has returned.                                            */
int pdhcg_last_cone_failure(double* rec, int64_t* count);

/* Diagnostic (not on the solve path): project `count` blocks of one cone
 * type with the same device routines the solver uses, so they can be
 * compared with an independent implementation.  Appendix C gives the
 * projections: the closed forms onto R+, SOC and RSOC, the root of h_M for
 * EXP and the bisection of Prop. power-cone-bisection for POW, all in the
 * diagonal metric of eq. metric-block-projection,
 *     Pi^M_K(r) = argmin_{u in K} 1/2 ||u - r||_M^2,  M = diag(metric).
 * type: PDHCG_CONE_* except BOX; dim: coordinates per block (RSOC >= 2,
 * EXP/POW/EXP1 3).
 * r, out: count*dim doubles, block after block, in the coordinate order of
 * the cone list (host pointers, caller-owned).  metric: count*dim positive
 * entries, or NULL for the Euclidean projection; a block whose metric is
 * constant takes the Euclidean formula, as in the solver.  alpha: count
 * exponents in (0, 1), POW only (nullable otherwise).  Root-finding failures
 * give NaN in out (see pdhcg_last_cone_failure).  Runs on the null stream
 * and returns when out is filled.  Errors: PDHCG_E_ARG (bad type, sizes,
 * null pointers, metric <= 0), PDHCG_E_CONE (dim, alpha), PDHCG_E_MEM,
 * PDHCG_E_HIP.                                                            */
int pdhcg_project_cones(int32_t type, int32_t dim, int64_t count, const double* alpha,
                        const double* r, const double* metric, double* out);

/* pdhcg_project_cones for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same projections with DEVICE pointers, issued
 * asynchronously on `stream` (hipStream_t as void*, NULL = null stream), no
 * allocation, no memset and no host synchronisation.  r, out: count*dim
 * doubles; metric: count*dim or NULL; alpha: count (POW) -- all device
 * memory owned by the caller.  The per-block flags (metric constant on the
 * block) go to a static device array of the library, one per device, held
 * until the process ends: count may not exceed 4,194,304 blocks
 * (PDHCG_E_ARG otherwise).  Every call on a device writes that device's
 * array, so calls that overlap on one device (different streams, threads)
 * race; serialise them.  Metric and alpha values are not checked (invalid
 * ones give NaN).  Errors: PDHCG_E_ARG, PDHCG_E_CONE, PDHCG_E_HIP.         */
int pdhcg_project_cones_noalloc(int32_t type, int32_t dim, int64_t count, const double* alpha,
                                const double* r, const double* metric, double* out, void* stream);

/* Release every host and device resource of h (NULL is a no-op).          */
void pdhcg_free(pdhcg_handle* h);

/* Static description of an error code or status.                          */
const char* pdhcg_strerror(int code);

/* Library version string.                                                  */
const char* pdhcg_version(void);

/* ---- learned warm start ------------------------------------------------
 * A ReLU multilayer perceptron, dims[0] -> dims[1] -> ... -> dims[layers],
 * trained on (instance parameters -> primal-dual solution) pairs produced by
 * the solver itself; its prediction seeds pdhcg_solve, which still runs to
 * the same tolerance.  The paper has no learned component: the network is
 * this library's own (Z_l = H_{l-1} W_l + b_l, H_l = relu(Z_l) below the
 * output layer, mean-squared-error loss, Adam).  Matrix products run on the
 * matrix cores with BF16 operands (input, weights, activations and backward
 * signals rounded to nearest-even BF16) and FP32 accumulation; master
 * weights, biases, gradients and Adam moments are FP32.
 *
 * Pointers named x, y in forward/train_step are DEVICE pointers (row-major
 * batch x dims[0] inputs, batch x dims[layers] targets/outputs, FP32), e.g.
 * the data of torch CUDA tensors; parameters and gradients are exchanged
 * through HOST pointers.  W of layer l is dims[l] x dims[l+1] row-major.
 * All work is issued on `stream`.  Handles are not thread-safe.            */
typedef struct {
    double lr, beta1, beta2, eps;       /* e.g. 1e-3, 0.9, 0.999, 1e-8      */
} pdhcg_adam;

/* Allocate a network (weights zero) for batches of up to max_batch rows.
 * Errors: PDHCG_E_ARG (null/invalid sizes), PDHCG_E_SHAPE (a dim < 1),
 * PDHCG_E_MEM, PDHCG_E_HIP.                                               */
int pdhcg_mlp_create(int32_t layers, const int32_t* dims, int32_t max_batch,
                     void* stream, void** out);
/* Set the FP32 weights (host, dims[l] x dims[l+1]) and bias (host, dims[l+1])
 * of layer l; resets that layer's Adam moments and the step count.         */
int pdhcg_mlp_set_params(void* h, int32_t layer, const float* W, const float* b);
/* Copy layer l's FP32 weights / bias to host buffers (each nullable).      */
int pdhcg_mlp_get_params(void* h, int32_t layer, float* W, float* b);
/* y (device, batch x dims[layers]) = network(x) (device, batch x dims[0]).  */
int pdhcg_mlp_forward(void* h, const float* x, int32_t batch, float* y);
/* One step on the batch (x, y): forward, loss, backward, and an Adam update
 * when opt is non-NULL (opt = NULL computes the gradients only; read them
 * with pdhcg_mlp_get_grads).  *loss (host, nullable) receives the mean
 * squared error of the forward pass before the update.                     */
int pdhcg_mlp_train_step(void* h, const float* x, const float* y, int32_t batch,
                         const pdhcg_adam* opt, double* loss);
/* Copy layer l's gradients of the last train step (host, nullable).        */
int pdhcg_mlp_get_grads(void* h, int32_t layer, float* dW, float* db);
/* Release the network (NULL is a no-op).                                   */
void pdhcg_mlp_free(void* h);

#ifdef __cplusplus
}
#endif
#endif /* PDHCG_H */
