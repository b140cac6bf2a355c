/*
 * symnmf.h - C ABI of the MI355X (gfx950) SymNMF hot path.
 *
 * Problem (paper section "Symmetric Non-negative Matrix Factorization",
 * eq. symnmf): given a dense symmetric non-negative S (n x n), find
 * H >= 0 (n x k, k << n) minimising f(H) = ||S - H H^T||_F^2.  Every step
 * works in the trace-identity form (eq. trace_loss)
 *     f(H) = ||S||_F^2 - 2 tr(H^T S H) + ||H^T H||_F^2,
 *     grad f = 4 (H (H^T H) - S H),
 * so no n x n intermediate is ever formed: each iteration streams S once
 * (or the sampled part of it) against H.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All sizes are int64_t.  Matrices are row-major.  "device" pointers are
 *   HIP device allocations owned by the caller unless stated otherwise.
 * - Every call is enqueued on the context's HIP stream and returns without
 *   waiting, except where a description says it synchronises (calls that
 *   hand back host scalars).
 * - Nothing throws across the ABI.  A non-zero symnmf_status is returned and
 *   symnmf_last_error() describes it.  Invalid arguments are rejected before
 *   any kernel is launched (SYMNMF_EINVAL); a non-finite value detected in a
 *   reduction is SYMNMF_ENUMERIC.
 * - S storage (symnmf_S): rows_pad = rows rounded up to 256, ld = n rounded up
 *   to 256; padding is zero.  FP64 S is row-major with leading dimension ld.
 *   FP32 / BF16 / FP8 S are stored in 256 x 256 tiles, tile (R, C) at element
 *   offset (R * ld/256 + C) * 65536; inside a tile the elements follow the
 *   order the S.H stream reads them: [wave w 0..3][sub-step s][row group g
 *   0..3][lane l 0..63][E], E = 16 bytes / element size, lane l holding row
 *   64 w + 16 g + l%16 and columns 4E s + E (l/16) + e.  FP8 S also keeps the
 *   per-row-panel scales and the FP32 diagonal after the matrix in the same
 *   buffer.
 * - H buffers handed to the library are n x k, contiguous k.
 * - A context is not thread safe; use one per host thread.
 */
#ifndef SYMNMF_H
#define SYMNMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SYMNMF_OK = 0,
    SYMNMF_EINVAL = 1,       /* bad argument, shape or state                    */
    SYMNMF_ENOMEM = 2,       /* device allocation failed / buffer too small     */
    SYMNMF_EDEVICE = 3,      /* HIP runtime error                               */
    SYMNMF_ENUMERIC = 4,     /* non-finite value in a reduction                 */
    SYMNMF_ENOTCONV = 5,     /* solve_to_tol hit max_iter before the stop rule  */
    SYMNMF_EUNSUPPORTED = 6  /* valid request the library does not implement   */
} symnmf_status;

/* Storage type of S.  The paper runs fp32; BF16 and FP8 storage are an
 * addition (the paper leaves half precision open in its numerical
 * consideration paragraph).  FP64 is kept for exact parity runs. */
typedef enum {
    SYMNMF_S_FP32 = 0,
    SYMNMF_S_BF16 = 1,       /* round-to-nearest-even                            */
    SYMNMF_S_FP8 = 2,        /* OCP E4M3, per-row-panel scale, exact unit diag   */
    SYMNMF_S_FP64 = 3
} symnmf_sdtype;

typedef enum {
    SYMNMF_ABS_CORR = 0,     /* |Pearson correlation| (appendix, correlation construction) */
    SYMNMF_TPDM = 1          /* empirical tail pairwise dependence (section "Empirical Estimation") */
} symnmf_skind;

/* Solver families of appendix "Detailed Algorithm Descriptions": family 3
 * (AdaGrad to Block-SVRG) and family 6 (ADMM). */
typedef enum {
    SYMNMF_ADAGRAD = 0,
    SYMNMF_RMSPROP = 1,
    SYMNMF_PIECEWISE_ADAGRAD = 2,
    SYMNMF_ROW_SVRG = 3,
    SYMNMF_BLOCK_SVRG = 4,   /* Block-SVRG AdaptGrow */
    SYMNMF_ADMM = 5,         /* eqs. admm_H, admm_W, admm_U; the iterate is W, the
                                dual U starts at 0; projected form only */
    SYMNMF_ADAM = 6,         /* family 3: bias-corrected first and second moments
                                (beta1, beta2), step eta m^ / (sqrt(v^) + eps) */
    SYMNMF_NADAM = 7,        /* Adam with the look-ahead b1 m^ + (1 - b1) g / (1 - b1^t) */
    SYMNMF_ADAN = 8,         /* Xie et al. 2023: averages of g (beta1), of g - g_prev
                                (beta2) and of (g + beta2 (g - g_prev))^2 (beta3),
                                bias-corrected; the first difference is 0 */
    SYMNMF_MU = 9            /* family 1, dampened multiplicative update
                                H <- H (1 + SH / (H H^T H + eps)) / 2 (eps: fp32
                                machine epsilon in the paper); no eta, no softplus form */
} symnmf_method;

typedef struct symnmf_ctx symnmf_ctx;
typedef struct symnmf_state symnmf_state;

/* Parameters of S construction. */
typedef struct {
    int32_t kind;            /* symnmf_skind                                     */
    int32_t dtype;           /* symnmf_sdtype of the stored S                    */
    int64_t n;               /* instruments = columns of X                       */
    int64_t T;               /* samples = rows of X (T >= 2)                     */
    int64_t row0;            /* first row of S to build (0 for the full matrix)  */
    int64_t rows;            /* rows to build: n for the full matrix, fewer for a row panel */
    double q;                /* TPDM: exceedance fraction, n_exc = floor(q T) >= 1 */
    int32_t lower_tail;      /* TPDM: 1 = lower tail (transform -X), 0 = upper   */
    int32_t raw_marginals;   /* TPDM: 0 = rank transform to Pareto(2) margins;
                              * 1 = X used as given (it must already have
                              * Pareto-type margins and be >= 0 in the chosen
                              * tail orientation), the construction of the
                              * appendix's benchmark matrices               */
    int64_t fp8_panel_rows;  /* FP8: rows per scale panel (>= 1)                 */
} symnmf_sbuild_params;

/* Descriptor of a stored S (or of a row panel of S).  Filled by
 * symnmf_build_S / symnmf_S_load; the caller owns the memory at ``data``. */
typedef struct {
    void* data;              /* device: rows_pad x ld elements of dtype           */
    float* panel_scale;      /* device: FP8 scales (stored code = S * scale), else NULL */
    float* diag;             /* device: FP8 S_ii of every panel row (codes hold 0 there), else NULL */
    int64_t n, row0, rows, ld, rows_pad, fp8_panel_rows;
    int32_t dtype, kind;
    double fro2;             /* ||S||_F^2 before storage rounding (FP64 sum)      */
    double fro2_stored;      /* ||S_stored||_F^2, what the solver's objective uses */
    double sum;              /* sum of the entries before storage rounding        */
    double mean;             /* sum / (rows * n)                                  */
} symnmf_S;

/* Solver parameters.  Readings of values the paper leaves open are listed
 * with the fields; defaults come from symnmf_params_default(). */
typedef struct {
    int32_t method;          /* symnmf_method                                    */
    int32_t softplus;        /* 1: H = softplus(Theta), optimiser on Theta (eq. logspace_grad) */
    double eta;              /* learning rate                                     */
    double eps;              /* added outside the square root                     */
    double alpha;            /* RMSprop EMA factor                                */
    double mu;               /* RMSprop momentum                                  */
    double c;                /* Piecewise: reset scale c                          */
    double c_r;              /* Piecewise: reset only while KKT > c_r * tau_g     */
    double eps_med;          /* Piecewise: median(g^2) floor                      */
    double row_frac;         /* Row-SVRG: |I| / n                                 */
    double phi0;             /* Block-SVRG: initial entry coverage phi_0          */
    double c_grow;           /* Block-SVRG: grow only while KKT > c_grow * tau_g  */
    int64_t grow_checks;     /* Block-SVRG: consecutive stagnating checks to grow */
    int64_t snapshot_s;      /* SVRG snapshot period s (full step at t = 0 mod s) */
    int64_t block_rows;      /* SVRG row-block size, a multiple of 256            */
    int32_t independent_blocks; /* Block-SVRG: 1 = independent I and J, 0 = J = I */
    int32_t reserved0;
    int64_t delta;           /* check interval (eq. obj_stag), multiple of snapshot_s for SVRG */
    int64_t warmup;          /* stagnation test suppressed for t < warmup         */
    int64_t max_iter;
    double tau_E;            /* loss gate (eq. loss_gate)                         */
    double tau_g_inf;        /* KKT gate tau_g^inf (eq. kkt_scaled)               */
    double n_ref;            /* n_ref of eq. kkt_scaled                           */
    double tau_stag;         /* stagnation tolerance (eq. obj_stag)               */
    uint64_t seed;           /* key of the index-set sampler                      */
    double rho;              /* ADMM consensus penalty rho > 0                    */
    double beta1;            /* Adam / NAdam / Adan: decay of the gradient average (0.9) */
    double beta2;            /* Adam / NAdam: second-moment decay (0.999); Adan: decay of
                                the gradient-difference average (0.92 in Xie et al.) */
    double beta3;            /* Adan: second-moment decay (0.99)                   */
} symnmf_params;

/* Statistics of one iteration, of the iterate H_t that the step read. */
typedef struct {
    int64_t t;
    double f;                /* f(H_t) on the stored S (NaN on sub-sampled steps) */
    double E;                /* f / ||S_stored||_F^2                              */
    double kkt;              /* ||grad_proj f(H_t)||_F / (n k) (eq. kkt_stop)     */
    double stag;             /* (E_{t-delta} - E_t) / E_0 at checks, else NaN     */
    double phi;              /* Block-SVRG coverage when the step ran (1 for other  */
                             /*   methods; a snapshot step also reports it)       */
    double wall_ms;          /* host wall time since the state was created        */
    int32_t full;            /* 1: the step read all of S                         */
    int32_t reset_fired;     /* Piecewise reset applied after this step           */
    int32_t converged;       /* stop rule (eq. conv_and) satisfied at this check  */
    int32_t nonfinite;       /* non-finite gradient entries seen                   */
} symnmf_stats;

int32_t symnmf_abi_version(void);
void symnmf_params_default(symnmf_params* p);

/* Create a context bound to HIP device ``device`` and stream ``hip_stream``
 * (a hipStream_t; NULL = the null stream).  Allocates nothing on the device. */
symnmf_status symnmf_create(symnmf_ctx** ctx, int32_t device, void* hip_stream);
void symnmf_destroy(symnmf_ctx* ctx);

/* Device scratch.  The calls that need temporary device buffers (S build and
 * load, objective, median, sketch, canonical coordinates, warm start,
 * subspace error, K-means, silhouette, spectral diagnostic) take them from a
 * pool held by the context; the state and the network objects own their own
 * workspace instead.  symnmf_set_workspace(ctx, dev, bytes) makes the pool a
 * caller-owned device buffer: the library then allocates nothing for these
 * calls, and a call that needs more than ``bytes`` returns ENOMEM (its message
 * gives the size; the *_workspace queries below give it beforehand).  With no
 * workspace attached (the default, or after symnmf_set_workspace(ctx, NULL,
 * 0)) the pool takes device memory with hipMalloc when a call needs more than
 * it holds and keeps it until symnmf_destroy, so a call no larger than an
 * earlier one on the same context allocates nothing.  Buffers are carved in
 * stack order and reused by the next call at once (calls on a context run in
 * its stream's order); set_workspace synchronises the stream and fails with
 * EINVAL while a call is using the pool.  The caller keeps an attached buffer
 * alive until it is detached or the context is destroyed. */
symnmf_status symnmf_set_workspace(symnmf_ctx* ctx, void* dev, int64_t bytes);
/* Bytes the pool holds (attached or allocated) and the number of blocks the
 * pool has taken from hipMalloc since the context was created. */
symnmf_status symnmf_workspace_info(symnmf_ctx* ctx, int64_t* held, int64_t* allocs);
const char* symnmf_last_error(const symnmf_ctx* ctx);

/* Bytes of the buffer a stored S (rows x n, dtype) needs, scales included. */
int64_t symnmf_S_bytes(int64_t rows, int64_t n, int32_t dtype, int64_t fp8_panel_rows);

/* Element offset (in elements of dtype) of panel row r, column c inside the
 * data of a stored S with leading dimension ld (host only; -1 if out of range). */
int64_t symnmf_S_offset(int64_t r, int64_t c, int64_t rows_pad, int64_t ld, int32_t dtype);

/* Build S (or rows [row0, row0+rows) of S) from the returns panel X.
 * X: device, T x n float32 row-major (samples x instruments), read only.
 * |corr| (appendix, correlation construction): columns centred and scaled to
 *   unit norm in FP64, S = |Z^T Z| by an MFMA GEMM, S_ii = 1.
 * TPDM (section "Empirical Estimation"): per-column ranks (ties to the lower
 *   sample), Pareto(2) margins x = (1 - r/(T+1))^-1/2, FP64 radial norms, the
 *   floor(qT) largest kept (ties to the lower sample), angular rows Omega,
 *   S = D^-1/2 Omega^T Omega D^-1/2 by the same GEMM, S_ii = 1.  With
 *   raw_marginals the rank step is skipped and the polar transform is taken
 *   of (+-)X itself (appendix "Benchmark Data Generation", TPDM construction).
 * The GEMM accumulates in FP32: FP32 storage multiplies on the FP32 matrix
 * cores; BF16 / FP8 storage splits the operand into two bf16 planes
 * (z = h + m, products h h + h m + m h, relative error ~2^-16 before the
 * storage rounding); FP64 storage uses FP64 FMAs.  The stored S is exactly
 * symmetric in every format.
 * buf: device, >= symnmf_S_bytes(...) bytes, caller owned.  Scratch comes from
 * the context pool (symnmf_build_S_workspace bytes).  Synchronises (fills the FP64
 * sums of ``out``).  EINVAL: T < 2, n < 1, bad row range, zero-variance
 * column, floor(qT) < 1, raw_marginals not 0/1, a raw-marginal X < 0 in the
 * tail orientation.  EUNSUPPORTED: the rank transform with T > 32768.
 * ENUMERIC: X holds a NaN or an infinity. */
/* Scratch bytes symnmf_build_S needs for these parameters (the standardised
 * or angular operand Z, FP64 sums, FP8 panel maxima, the TPDM rank workspace
 * and the bf16 operand planes), or -1 for invalid parameters. */
int64_t symnmf_build_S_workspace(const symnmf_sbuild_params* p);
symnmf_status symnmf_build_S(symnmf_ctx* ctx, const float* X, const symnmf_sbuild_params* p,
                             void* buf, int64_t buf_bytes, symnmf_S* out);

/* Store a given dense S panel (device, rows x n row-major, float32 or float64
 * when src_is_f64) in ``dtype`` - e.g. a planted S = H* H*^T.  Same storage
 * and sums as symnmf_build_S.  Synchronises. */
symnmf_status symnmf_S_load(symnmf_ctx* ctx, const void* src, int32_t src_is_f64, int64_t n,
                            int64_t row0, int64_t rows, int32_t dtype, int64_t fp8_panel_rows,
                            void* buf, int64_t buf_bytes, symnmf_S* out);

/* Initial factor (section "Initialization and seeds"): H_ij = u_ij * sqrt(mean(S)/k),
 * u_ij = 2^-24 * (top 24 bits of SplitMix64 output number i*k+j of key ``seed``).
 * H: device n x k float32.  Uses S->mean. */
symnmf_status symnmf_init_H(symnmf_ctx* ctx, const symnmf_S* S, int64_t k, uint64_t seed, float* H);

/* Solver state for S and rank k.  H0: device n x k (float32, or float64 when
 * h0_is_f64; FP64 storage of S runs the whole iteration in FP64 and needs
 * an FP64 H0).  The state owns its device workspace (iterates H_t and H_{t+1},
 * optimiser buffers, snapshot gradient, reduction partials) and frees it in
 * symnmf_state_destroy.  1 <= k <= 64.  For a row panel (rows < n) the state
 * updates the panel's rows of H and keeps the other rows fixed. */
symnmf_status symnmf_state_create(symnmf_ctx* ctx, const symnmf_S* S, int64_t k,
                                  const symnmf_params* p, const void* H0, int32_t h0_is_f64,
                                  symnmf_state** st);
void symnmf_state_destroy(symnmf_state* st);

/* One solver iteration t -> t+1 (appendix family 3 rules; Piecewise resets,
 * phi growth and the stop rule live in symnmf_solve_to_tol).  Reads H_t,
 * forms g_t = grad f(H_t) from S H_t (or its sampled blocks), updates the
 * optimiser state, writes H_{t+1}, and reduces in FP64 the statistics of H_t.
 * ADMM (family 6): the iterate is the feasible factor W; the step forms
 * (2 W^T W + rho I)^-1 from the FP64 Gram of W_t, then H, W_{t+1} and U from
 * S W_t (eqs. admm_H, admm_W, admm_U); the statistics are those of W_t.
 * ``out`` NULL: nothing waits; otherwise the call synchronises and fills it. */
symnmf_status symnmf_step(symnmf_ctx* ctx, const symnmf_S* S, symnmf_state* st, symnmf_stats* out);

/* Copy a state buffer to ``dst`` (device, n x k elements of the state's
 * precision: float32, or float64 for FP64 S).  which: 0 = current iterate,
 * 1 = previous iterate, 2 = accumulator G (RMSprop v), 3 = RMSprop momentum
 * (ADMM: the scaled dual U), 4 = Theta (softplus), 5 = snapshot gradient mu,
 * 6 = gradient of the last step, 7 = Adan average of gradient differences,
 * 8 = Adan previous gradient.  For Adam / NAdam / Adan, 2 holds the second
 * moment and 3 the gradient average. */
symnmf_status symnmf_state_read(symnmf_ctx* ctx, symnmf_state* st, int32_t which, void* dst);
/* Host copy of the statistics of the last step (synchronises). */
symnmf_status symnmf_state_stats(symnmf_ctx* ctx, symnmf_state* st, symnmf_stats* out);
/* Block-SVRG coverage phi (0 < phi <= 1). */
symnmf_status symnmf_state_set_phi(symnmf_state* st, double phi);

/* Control state of the check-time rules (appendix "Detailed Algorithm
 * Descriptions": Piecewise AdaGrad's accumulator resets, Block-SVRG
 * AdaptGrow's coverage growth), as left by the last check. */
typedef struct {
    int64_t t;               /* iterations taken                                   */
    double phi;              /* Block-SVRG coverage of the next sampled step       */
    int64_t stag_run;        /* consecutive stagnating checks counted for growth   */
    int64_t pw_resets;       /* Piecewise resets applied so far                    */
    int32_t pw_enabled;      /* 0 once a reset was refused for lack of progress     */
    int32_t pw_cooling;      /* 1 after a reset: stagnation waits for sum(G) to     */
                             /*   reach pw_cool_target                             */
    double pw_cool_target;   /* twice sum(G) right after the last reset            */
    double pw_E_reset;       /* E at the last reset                                */
} symnmf_control;
/* Host copy of the control state (no device work). */
symnmf_status symnmf_state_control(symnmf_ctx* ctx, symnmf_state* st, symnmf_control* out);
/* Statistics of the check iterations (t = 0 mod delta) evaluated so far by
 * symnmf_solve_to_tol, symnmf_solve_trace or the ladder, in order, with the
 * decisions taken at each (stag, reset_fired, converged, and phi, the coverage
 * the checked step used).  Copies min(count, cap) records to ``out`` (host)
 * and the number of records to *count.  No device work. */
symnmf_status symnmf_state_checks(symnmf_ctx* ctx, symnmf_state* st, symnmf_stats* out, int64_t cap,
                                  int64_t* count);

/* f(H) and E = f/||S_stored||^2 for any H (device n x k, float32 or float64),
 * the measure every result is compared by.  S H is accumulated in FP64: for FP32/BF16/FP8 storage
 * with float32 H and k in {16, 32} the MFMA products are summed in FP32 within
 * each 256-column chunk and in FP64 across chunks; otherwise every product is
 * accumulated in FP64.  The trace and Gram terms are FP64.  Synchronises. */
/* Scratch bytes of symnmf_objective for this S and rank (-1: bad argument). */
int64_t symnmf_objective_workspace(const symnmf_ctx* ctx, const symnmf_S* S, int64_t k, int32_t h_is_f64);
symnmf_status symnmf_objective(symnmf_ctx* ctx, const symnmf_S* S, const void* H, int32_t h_is_f64,
                               int64_t k, double* f, double* E);

/* Iterate until the stop rule (eq. conv_and, checked every delta steps)
 * certifies an iterate, or (f_target > 0) f(H_t) <= f_target (1 + rel_tol),
 * or max_iter.  Applies Piecewise resets and Block-SVRG growth at checks.
 * Copies the certified iterate H_t (or the last one) to H_out (device, may be
 * NULL).  Returns SYMNMF_OK when a stop condition was met, SYMNMF_ENOTCONV
 * when max_iter was reached.  Synchronises at every check. */
symnmf_status symnmf_solve_to_tol(symnmf_ctx* ctx, const symnmf_S* S, symnmf_state* st,
                                  double f_target, double rel_tol, symnmf_stats* final_stats,
                                  void* H_out);

/* Trace of a solve: ``steps`` iterations with every rule of symnmf_solve_to_tol
 * applied at the checks (stop-rule statistics, Piecewise resets, Block-SVRG
 * growth) but without stopping when the stop rule certifies an iterate.
 * After every save_every-th iteration the current iterate is copied to the
 * next slot of H_save (device, slots x n x k of the state's precision,
 * slots >= steps / save_every) and ms_out[slot] (host) receives the time from
 * the start of the call to that copy, from HIP events on the context stream.
 * *certified_at (may be NULL) receives the first t the stop rule certified,
 * or -1.  Synchronises at every check.  ENUMERIC on a non-finite gradient. */
symnmf_status symnmf_solve_trace(symnmf_ctx* ctx, const symnmf_S* S, symnmf_state* st, int64_t steps,
                                 int64_t save_every, void* H_save, int64_t slots, double* ms_out,
                                 int64_t* certified_at);

/* Precision ladder (not in the paper, whose discussion of numerical
 * considerations leaves reduced-precision storage open): the solver iterates
 * on the rounded problem min ||S_q - H H^T||^2, whose minimiser differs from
 * that of S by a term of the order of the rounding of S, so on FP8 storage
 * the objective on S stalls above a tight tolerance.  The ladder iterates on
 * the low-precision storage while it makes progress and then continues on a
 * second, more precise storage of the same matrix.
 *
 * symnmf_state_rebind: point the state at S (another storage of the matrix
 * the state was created for: same n, row0, rows and padding; FP64 storage for
 * an FP64 state only, else EINVAL).  The iterate, the optimiser buffers and
 * t are kept; the stream launch shape and the image / partial buffers follow
 * the new storage type (grown when needed; synchronises); the stagnation
 * reference of the stop rule restarts because E is measured on the stored
 * matrix.  Later calls must pass S.
 *
 * symnmf_solve_trace_ladder: symnmf_solve_trace that starts on S_lo (the
 * state's storage) and rebinds the state to S_hi at the first check (t a
 * multiple of delta, t >= warmup) whose stagnation measure
 * (E_{t-delta} - E_t) / E_0 is below tau_switch (>= 0); *switched_at
 * (may be NULL) receives that t or -1.  *certified_at only counts
 * certifications on S_hi.  The state is left bound to the storage of the last
 * step. */
symnmf_status symnmf_state_rebind(symnmf_ctx* ctx, symnmf_state* st, const symnmf_S* S);
symnmf_status symnmf_solve_trace_ladder(symnmf_ctx* ctx, const symnmf_S* S_lo, const symnmf_S* S_hi,
                                        symnmf_state* st, int64_t steps, int64_t save_every, void* H_save,
                                        int64_t slots, double* ms_out, double tau_switch, int64_t* certified_at,
                                        int64_t* switched_at);

/* Subspace error of two factors (solutions are defined up to column
 * permutation and scaling): ||P_A - P_B||_F / sqrt(2k) with P_X the orthogonal
 * projector onto the column span of X, from ||P_A - P_B||_F^2 =
 * 2k - 2 ||Q_A^T Q_B||_F^2 and Q_X = X (X^T X)^-1/2; only k x k FP64 work
 * after the products A^T A, B^T B, A^T B.  A, B: device n x k float32.
 * ENUMERIC when a factor is rank deficient.  Synchronises. */
/* Scratch bytes of symnmf_subspace_error (-1: bad argument). */
int64_t symnmf_subspace_error_workspace(int64_t n, int64_t k);
symnmf_status symnmf_subspace_error(symnmf_ctx* ctx, const float* A, const float* B, int64_t n, int64_t k,
                                    double* out);

/* Lower median (element floor((m-1)/2) in sorted order) of g_i^2 over a device
 * float32 array of m values, by radix selection on the bit patterns.
 * Synchronises; the result goes to *out. */
symnmf_status symnmf_median_sq(symnmf_ctx* ctx, const float* g, int64_t m, float* out);
/* Scratch bytes of symnmf_median_sq. */
int64_t symnmf_median_workspace(void);

/* The same lower median of g_i^2 for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): no allocation, no synchronisation.  The result goes to
 * out_dev[0] (device, one double holding the float32 value) on the context's
 * stream.  Working memory is a fixed 4096-byte array of the library on each
 * GPU (held until the process ends), cleared by the call's own kernels, so
 * calls that overlap on one GPU (several streams or threads) race on it and
 * must be serialised by the caller.  m <= 2^32 - 1 (32-bit histogram counts),
 * else EINVAL; EDEVICE if the array's address could not be found on this
 * device when the context was created. */
symnmf_status symnmf_median_sq_noalloc(symnmf_ctx* ctx, const float* g, int64_t m, double* out_dev);

/* Piecewise AdaGrad accumulator recalibration G_i <- max(c g_i^2, c median(g^2))
 * with g the gradient of the state's last step (appendix, Piecewise AdaGrad).
 * Synchronises; *median_out (may be NULL) receives median(g^2). */
symnmf_status symnmf_piecewise_reset(symnmf_ctx* ctx, symnmf_state* st, double c, float* median_out);

/* The index-set sampler of the stochastic variants (host only): m distinct
 * block indices of [0, nblocks), sorted, by a partial Fisher-Yates shuffle
 * driven by SplitMix64 keyed by (seed, 2t + stream). */
void symnmf_sample_blocks(uint64_t seed, int64_t t, int32_t stream, int64_t nblocks, int64_t m,
                          int32_t* out);

/* Plain grid-stride copy of ``bytes`` (a multiple of 16) from src to dst
 * (device): a kernel of known traffic, for calibrating hardware byte counters
 * against the S.H stream.  Asynchronous. */
symnmf_status symnmf_probe_copy(symnmf_ctx* ctx, const void* src, void* dst, int64_t bytes);

/* Plain read of ``bytes`` (a multiple of 16) from src (device) by 2048
 * persistent work-groups (fewer when sink_words / 4 is smaller) with 16-byte
 * nontemporal loads: the read-bandwidth ceiling the S.H stream competes
 * against.  sink: device, sink_words 32-bit words (>= 4) receiving one folded
 * word per wave.  Asynchronous. */
symnmf_status symnmf_probe_read(symnmf_ctx* ctx, const void* src, void* sink, int64_t sink_words, int64_t bytes);

/* HIP-event timing of the kernels a step launches, on the context's stream.
 * Reading (ms_out / launches_out non-NULL, 5 entries each: 0 = S.H stream,
 * 1 = fused update, 2 = finalize, 3 = plan of a sub-sampled step, 4 = H
 * chunk images for the MFMA stream)
 * synchronises and returns the summed milliseconds and launch counts since the
 * last call; every call then clears the record and sets profiling on or off
 * (enable).  Off by default; timing adds two events per kernel. */
symnmf_status symnmf_profile(symnmf_ctx* ctx, int32_t enable, double* ms_out, int64_t* launches_out);

/* Device self-check of the FP8 -> BF16 conversion instruction the FP8 stream
 * relies on: the number of finite E4M3 codes it decodes differently from the
 * format definition (0 expected), or -1 on a HIP error.  Synchronises. */
int32_t symnmf_selfcheck_fp8(symnmf_ctx* ctx);

/* ------------------------------------------------------------------------
 * Learned warm start.  Not part of the paper's method (its only learned
 * solver is trained per instance and, the paper notes, its weights do not
 * carry over between matrices of different spectral structure).  A per-row
 * sketch of S is mapped to canonical coordinates that do not depend on the
 * random sketch basis or on the column order of the solution, and a small MLP
 * maps every row's coordinates to an initial row of H:
 *   1. Y = S Omega, Omega n x w standard normal (Box-Muller on SplitMix64);
 *   2. top-k eigenpairs of Y^T Y: Z = Y V_k Lambda_k^-1/2; successive
 *      projection (Gillis & Vavasis 2014) picks k anchor rows of Z; rows in
 *      the anchor basis C = Z Z[anchors]^-1, zero-padded to w columns;
 *   3. MLP w -> h -> h -> k, exact GELU x Phi(x), softplus output;
 *   4. H0 = alpha A with alpha^2 = tr(A^T S A) / ||A^T A||_F^2.
 * Training minimises a column-permutation invariant Gram loss (through the
 * trace identity ||A A^T - B B^T||^2 = ||A^T A||^2 - 2 ||A^T B||^2 + ||B^T B||^2,
 * no m x m matrix) against solved factors B with AdamW (Loshchilov & Hutter
 * 2019).
 * ------------------------------------------------------------------------ */
typedef struct symnmf_mlp symnmf_mlp;

typedef struct {
    double lr, beta1, beta2, eps, weight_decay;   /* AdamW; decay on W1..W3 only */
} symnmf_adamw;

/* Parameters of the network as one float32 vector, in this order:
 * W1 (h x w), W2 (h x h), W3 (k x h) row-major (y = W x + b), b1 (h), b2 (h),
 * b3 (k).  Returns the count, or -1 for sizes outside 1..64 (w, k) and
 * 1..1024 (h). */
int64_t symnmf_mlp_param_count(int64_t width, int64_t hidden, int64_t k);

/* Initial parameters (device, symnmf_mlp_param_count floats): layer l = 0, 1, 2
 * gets W_l = G / sqrt(fan_in) with G the standard normals of the sketch
 * generator (same definition as Omega in symnmf_sketch) keyed 4 seed + 1 + l,
 * element (r, c) at counter index r * fan_in + c; biases 0.  Asynchronous. */
symnmf_status symnmf_mlp_init(symnmf_ctx* ctx, int64_t width, int64_t hidden, int64_t k, uint64_t seed,
                              float* params);

/* Network with parameters ``params`` (device, symnmf_mlp_param_count floats,
 * copied) and zero AdamW state.  Owns its device memory (parameters, BF16
 * weight copies, gradients, moments, activations grown to the largest row
 * count seen), freed by symnmf_mlp_destroy. */
symnmf_status symnmf_mlp_create(symnmf_ctx* ctx, int64_t width, int64_t hidden, int64_t k, const float* params,
                                symnmf_mlp** out);
void symnmf_mlp_destroy(symnmf_mlp* mlp);

/* Copy to ``dst`` (device, symnmf_mlp_param_count floats): which 0 = parameters,
 * 1 = gradient of the last training step, 2 = AdamW first moment, 3 = second
 * moment.  Asynchronous. */
symnmf_status symnmf_mlp_read(symnmf_ctx* ctx, const symnmf_mlp* mlp, int32_t which, float* dst);
/* Output form of the network: residual = 0, A = softplus(z) (the default);
 * residual = 1, A = max(C + z, 0) with C the first k columns of the network
 * input (the canonical coordinates) and z the last layer's output, so the
 * network learns a correction to the network-free start max(C, 0) and
 * reproduces it exactly when the last layer is zero.  Applies to
 * symnmf_mlp_forward, symnmf_mlp_train_step and symnmf_warm_start.  EINVAL
 * for residual not in {0, 1} or k > width. */
symnmf_status symnmf_mlp_set_output(symnmf_ctx* ctx, symnmf_mlp* mlp, int32_t residual);
/* Grow the network's activation buffers (part of the network object's
 * workspace, freed by symnmf_mlp_destroy) to ``rows`` rows for inference, and
 * with ``training`` also for symnmf_mlp_train_step, so that later calls of at
 * most that many rows allocate nothing. */
symnmf_status symnmf_mlp_reserve(symnmf_ctx* ctx, symnmf_mlp* mlp, int64_t rows, int32_t training);
/* Replace the parameters (device floats) and clear the AdamW state and step
 * count.  Asynchronous. */
symnmf_status symnmf_mlp_write(symnmf_ctx* ctx, symnmf_mlp* mlp, const float* params);

/* A (m x k, device float32) = network(X) for X (m x w, device float32).
 * bf16_weights: multiply by the BF16-rounded weights (inference form, FP32
 * activations and accumulation); 0: the FP32 weights.  Asynchronous. */
symnmf_status symnmf_mlp_forward(symnmf_ctx* ctx, symnmf_mlp* mlp, const float* X, int64_t m,
                                 int32_t bf16_weights, float* A);

/* One training step on one instance: forward with the FP32 weights on X
 * (m x w), loss against the target B (m x k, device float32), backward, one
 * AdamW update.  loss_kind 0: L = ||A A^T - B B^T||_F^2 / ||B^T B||_F^2;
 * 1: the scale-free form L = 1 - ||A^T B||^4 / (||A^T A||^2 ||B^T B||^2), the
 * residual of the best scalar multiple of A A^T (the warm start rescales A
 * anyway).  *loss (may be NULL) receives L at the parameters before the
 * update.  Synchronises (the k x k products are read back). */
symnmf_status symnmf_mlp_train_step(symnmf_ctx* ctx, symnmf_mlp* mlp, const float* X, const float* B, int64_t m,
                                    const symnmf_adamw* opt, int32_t loss_kind, double* loss);

/* Y (rows x width, device float32 row-major) = S_panel Omega with
 * Omega_ij = sqrt(-2 ln(1 - u)) cos(2 pi v), u and v the top 53 bits of
 * SplitMix64 outputs 2e and 2e + 1 (e = i * width + j) of key omega_seed,
 * scaled by 2^-53.  1 <= width <= 64.  Runs the S.H stream once.
 * Scratch from the context pool (symnmf_sketch_workspace).  Synchronises. */
symnmf_status symnmf_sketch(symnmf_ctx* ctx, const symnmf_S* S, uint64_t omega_seed, int64_t width, float* Y);
/* Scratch bytes of symnmf_sketch (-1: bad argument). */
int64_t symnmf_sketch_workspace(const symnmf_ctx* ctx, const symnmf_S* S, int64_t width);

/* Canonical coordinates of the rows of a sketch Y (n x w, device float32):
 * X (n x w, device float32) = [C, 0] with C = Z Z[anchors]^-1 (step 2 above;
 * C is the same for any signs and order of the eigenvectors).  anchors
 * (device int64, k entries, may be NULL) receives the anchor rows in
 * selection order.  1 <= k <= w <= 64, n >= w.  ENUMERIC when Y^T Y has a
 * non-positive eigenvalue among the k largest or the anchor rows are linearly
 * dependent.  Synchronises. */
/* Scratch bytes of symnmf_canonical (-1: bad argument). */
int64_t symnmf_canonical_workspace(int64_t n, int64_t width, int64_t k);
symnmf_status symnmf_canonical(symnmf_ctx* ctx, const float* Y, int64_t n, int64_t width, int64_t k, float* X,
                               int64_t* anchors);

/* Warm start of the full matrix (S->rows == n): sketch with omega_seed and the
 * network's width, canonical coordinates, network with BF16 weights (mlp
 * non-NULL) or the coordinates themselves clipped at zero (mlp NULL: the
 * network-free ablation), then the alpha rescaling; H0: device n x k float32.
 * The network's k must equal k.  Synchronises. */
/* Scratch bytes of symnmf_warm_start (-1: bad argument): the sketch and the
 * coordinates, plus the largest of the sketch, canonical and objective scratch
 * used one after another (the network's activations are its own workspace,
 * symnmf_mlp_reserve). */
int64_t symnmf_warm_start_workspace(const symnmf_ctx* ctx, const symnmf_S* S, int64_t width, int64_t k);
symnmf_status symnmf_warm_start(symnmf_ctx* ctx, const symnmf_S* S, symnmf_mlp* mlp, int64_t width, int64_t k,
                                uint64_t omega_seed, float* H0);

/* ------------------------------------------------------------------------
 * Spherical K-means on the rows of S (paper section "Clustering": spherical
 * K-means as constrained SymNMF, Theorem snmf_spkmeans, and the computational
 * comparison with table tab:kmeans).  The points are the rows s_i of the
 * full stored S (S->rows == n; a row panel is EUNSUPPORTED) scaled to unit
 * length, s^_i = s_i / ||s_i||; a centroid is the normalised sum of its
 * members; the objective is J = sum_i (1 - cos(s^_i, c_{label_i})).  Every
 * product with S runs the S.H stream with an n x K factor in slices of at
 * most 64 columns; because S is symmetric,
 *     cos(s^_i, c_k) = (S C)_ik / ||s_i||   and
 *     sum_{j in k} s^_j = (S W)_{:,k},  W_jk = [label_j = k] / ||s_j||.
 * (FP8 storage with per-row-panel scales is symmetric only up to one
 * quantisation step; both products then use the stored rows.)  Centroids,
 * weights and products are FP64 for FP64 storage and FP32 otherwise; the
 * argmax is taken on the products in that precision, ties to the lowest
 * cluster index; J and the silhouette are summed in FP64.
 * Readings of what the paper leaves open: Forgy seeding (K distinct rows by
 * a partial Fisher-Yates shuffle, Knuth's Algorithm P, on 53-bit uniforms of
 * SplitMix64 keyed by the seed: for i = 0..K-1 swap positions i and
 * i + floor(u_i (n - i))); a cluster left without members keeps its previous
 * centroid.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t iters;           /* (centroid update, assignment) pairs after the first assignment */
    double J0;               /* objective of the first assignment (seed centroids) */
    double J;                /* objective of the returned labels                   */
    double wall_ms;          /* host wall time of the whole call                   */
    int64_t changed;         /* labels changed by the last assignment              */
    int32_t converged;       /* the stop rule fired within max_iter                */
    int32_t empty;           /* clusters without members at the end                */
} symnmf_kmeans_stats;

/* The Forgy seed rows symnmf_kmeans draws for (seed, n, K), in draw order
 * (host only, no GPU needed): out (host int64, K entries).  Returns EINVAL
 * unless 1 <= K <= n. */
symnmf_status symnmf_kmeans_seed_rows(uint64_t seed, int64_t n, int64_t K, int64_t* out);

/* k-means++ seed rows (Arthur & Vassilvitskii 2007) on the unit rows of the
 * stored S, for symnmf_kmeans's init_rows: the first is row floor(u_0 n);
 * seed i is the smallest j with sum_{l <= j} d_l > u_i sum_l d_l, where
 * d_l = min over the seeds so far of max(1 - cos(s^_l, s^_seed), 0) (the
 * squared distance of unit vectors up to the factor 2; 0 at the seeds) and
 * u_i is the i-th 53-bit uniform of SplitMix64 keyed by seed; when every d_l
 * is 0 the lowest unchosen row is taken.  One S pass per seed (FP64 sums of
 * d in a fixed order).  rows: host int64, K entries in draw order.
 * 1 <= K <= n.  Synchronises. */
symnmf_status symnmf_kmeans_seed_pp(symnmf_ctx* ctx, const symnmf_S* S, int64_t K, uint64_t seed, int64_t* rows);

/* ||s_i|| for every row (norms: device FP64, n entries), one pass over S
 * with FP64 sums.  EINVAL when a row is zero (it has no direction).
 * Synchronises. */
symnmf_status symnmf_row_norms(symnmf_ctx* ctx, const symnmf_S* S, double* norms);

/* Lloyd's assignment step: labels (device int32, n) = argmax_k cos(s^_i, c_k)
 * for the centroids C (device, n x K row-major, column k = c_k, unit length;
 * FP64 for FP64 storage, FP32 otherwise); best (device, same type, n
 * entries, may be NULL) receives the winning cosine; *J the objective.
 * 1 <= K <= n.  Synchronises. */
symnmf_status symnmf_kmeans_assign(symnmf_ctx* ctx, const symnmf_S* S, const void* C, int64_t K, int32_t* labels,
                                   void* best, double* J);

/* Lloyd's update step: C (device, n x K row-major, type as above) = the
 * normalised sums of the unit rows of every cluster of labels (device int32,
 * n entries in [-1, K); -1 = in no cluster).  A cluster without members
 * keeps its column of C_prev (device, same layout; NULL: zeros).  C may
 * equal C_prev.  Synchronises. */
symnmf_status symnmf_kmeans_centroids(symnmf_ctx* ctx, const symnmf_S* S, const int32_t* labels, int64_t K,
                                      const void* C_prev, void* C);

/* Spherical K-means (Lloyd) from K seed rows: init_rows (host int64, K
 * distinct rows) or, when NULL, the Forgy draw of `seed`.  Iterates
 * (centroid update, assignment) until J_{t-1} - J_t < tol J_{t-1} (or
 * J_{t-1} = 0) or max_iter pairs (the paper stops at a relative drop of
 * 1e-4).  labels: device int32, n entries; C (may be NULL): device n x K,
 * type as above, the last centroids.  stats (may be NULL).  ENOTCONV when
 * max_iter ends the run (labels, C and stats are still written).  The
 * n x K factors and the partials are scratch from the context pool.
 * Synchronises (once per iteration, to read J). */
symnmf_status symnmf_kmeans(symnmf_ctx* ctx, const symnmf_S* S, int64_t K, uint64_t seed, const int64_t* init_rows,
                            double tol, int64_t max_iter, int32_t* labels, void* C, symnmf_kmeans_stats* stats);

/* Spectral diagnostic of the collapse of angular clustering (section
 * "Clustering", eq. angular_collapse; table tab:spectral): lambda_1 of S by
 * power iteration from the normalised all-ones vector (S >= 0, so its Perron
 * vector is non-negative) until the Rayleigh quotient changes by at most
 * tol relative or max_iter passes; tr(S); r_eff = tr(S) / lambda_1;
 * collapse = (||S||_F^2 - lambda_1^2) / ||S||_F^2, the norm-weighted mean of
 * sin^2 of the angle between the rows and u_1, bounded by (r_eff - 1)^2 for
 * PSD S; collapse_rows = (||S||_F^2 - ||S u||^2) / ||S||_F^2, the same mean
 * evaluated from the rows with the computed u (equal to collapse when u is
 * exact).  ||S||_F^2 is S->fro2_stored.  Every output pointer (host) may be
 * NULL; u1 (device float32, n entries, may be NULL) receives the unit
 * vector.  One S pass per iteration.  ENUMERIC if S u vanishes.
 * Synchronises. */
symnmf_status symnmf_spectral(symnmf_ctx* ctx, const symnmf_S* S, int64_t max_iter, double tol, double* lambda1,
                              double* trace, double* r_eff, double* collapse, double* collapse_rows, int64_t* iters,
                              float* u1);

/* Mean silhouette of the partition labels (device int32, n entries in
 * [0, K)) under the cosine distance d(i, j) = 1 - cos(s^_i, s^_j)
 * (Rousseeuw 1987): a(i) = (n_a - s^_i . m_a) / (n_a - 1) and
 * b(i) = min over other non-empty clusters c of 1 - s^_i . m_c / n_c with
 * m_c the sum of the unit rows of cluster c, s(i) = (b - a) / max(a, b), and
 * s(i) = 0 in a singleton.  Two passes over S (M = S W, then S M).  EINVAL
 * with fewer than two non-empty clusters.  Synchronises. */
symnmf_status symnmf_silhouette(symnmf_ctx* ctx, const symnmf_S* S, const int32_t* labels, int64_t K, double* sil);

#ifdef __cplusplus
}
#endif
#endif /* SYMNMF_H */
