/*
 * tvi.h -- C ABI of the time-vectorized backward-Euler library for MI355X
 * (gfx950).  Plain C: no C++ types, no exceptions cross this boundary.
 *
 * The library integrates batches of ODE systems  dy/dt = h(y, t; p)  with
 * backward Euler (Section 2.2, Eq. backward-euler) and computes the adjoint
 * gradient of a loss of the computed trajectory (Appendix A).  Instead of
 * stepping one time step at a time it solves a chunk of steps of a series at
 * once (Section 2.3, Eq. batched-backward-euler): every Newton iteration
 * assembles the residuals and n x n diagonal blocks D_j = I - dt_j j_j of
 * the chunk Jacobian for all steps of the chunk in one pass and solves the
 * block lower-bidiagonal system (sub-diagonal blocks -I) by parallel cyclic
 * reduction (Section 3.2) inside one wavefront; the adjoint solves the
 * transposed, block upper-bidiagonal system the same way (Appendix A.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.  Every array argument is a DEVICE pointer to memory the caller
 *   owns (for example a contiguous torch tensor); the library keeps no
 *   pointer after a call returns.  Arrays are row-major and series-major.
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Work is
 *   enqueued on it and the call returns without waiting: results, and the
 *   per-series status codes, are ready once the stream reaches them.
 * Errors.  Arguments are checked on the host before anything is enqueued; a
 *   negative tvi_status is returned synchronously and nothing is launched.
 *   A launch failure returns TVI_EHIP.  Per-series outcomes (converged, not
 *   converged, singular block, non-finite value) are written to the device
 *   array `status[B]` asynchronously.
 * Precision.  TVI_F64 keeps everything in IEEE double.  TVI_F32 stores the
 *   inputs and outputs in float; the linear, Van der Pol and Robertson models
 *   still evaluate the residual, the blocks, their inverses and the
 *   reduction in double (stiff problems), the MLP model computes in float.
 *
 * Layouts
 * -------
 *   y0       [B][n]
 *   times    uniform grid: [N+1], shared by every series;
 *            ragged series: the points of series b at times[offsets[b] .. offsets[b+1]-1]
 *   offsets  NULL (uniform grid) or int64 point offsets [B+1] (device), offsets[0] = 0;
 *            series b has N_b = offsets[b+1] - offsets[b] - 1 >= 0 steps
 *   params   per series [B][P], or one shared [P] (model.params_shared)
 *   y        trajectory, uniform: [B][N+1][n]; ragged: [offsets[B]][n];
 *            the first point of each series is its y0
 *   ckpt     chunk-boundary checkpoints, always double, [B][K][n] with
 *            K = ceil(N / chunk) + 1: ckpt[b][c] = y of series b at step c * chunk
 *            (c * chunk <= N_b); entry ceil(N_b / chunk) is the final state
 *   g        dL/dy in the layout of y
 *   dLdp     [B][P], or [P] for shared parameters
 *   dLdy0    [B][n]
 *
 * Models and parameter vectors P
 *   TVI_LINEAR     h = A y,  n in {2, 3, 4}, p = A [n][n] (P = n^2)
 *   TVI_VANDERPOL  n = 2, h = (y2, mu (1 - y1^2) y2 - y1), p = (mu)
 *   TVI_ROBERTSON  n = 3, rate constants 0.04 s1, 3e7 s2 (on y2^2), 1e4 s3 (on y2 y3),
 *                  p = (s1, s2, s3)
 *   TVI_MLP        neural ODE (Section 5.1.4 without forcing): n = 8, hidden = 64,
 *                  h = W3 tanh(W2 tanh(W1 y + b1) + b2) + b3, one shared
 *                  p = (W1[64][8], b1[64], W2[64][64], b2[64], W3[8][64], b3[8]) (P = 5256);
 *                  computed in float on MFMA (bf16x3 products for h)
 *   TVI_CHABOCHE   Chaboche viscoplasticity (Section 5.1.1), n = 2 + nu with nu = 1..5
 *                  backstresses (nu >= 3: one step per lane, backward Euler, analytic
 *                  Jacobian, no learned start; TVI_EUNSUPPORTED otherwise): state (sigma, K, X_1..X_nu), s = sigma - sum X,
 *                  a = (|s| - K - sigma0)/eta, ep = <a>^n sign(s),
 *                  h = (E (edot(t) - ep), tau (K_inf - K) |ep|, 2/3 C_i ep - gamma_i X_i |ep|),
 *                  edot(t) = edot_a sin(2 pi t / T),
 *                  p = (E, n, eta, sigma0, K_inf, tau, C_1..C_nu, gamma_1..gamma_nu, edot_a, T)
 *                  (P = 8 + 2 nu); the hardening rate carries |ep| (the model's standard form);
 *                  TVI_F64 only
 *   TVI_NEURON     the coupled-neuron model (Section 5.1.1) with nu = n / 4 = 1 or 2 neurons,
 *                  state (V_i, m_i, h_i, n_i) per neuron: dV_i/dt = (-g_Na m^3 h (V_i - E_Na)
 *                  - g_K n^4 (V_i - E_K) - g_L (V_i - E_L) + I_a sin(2 pi t / T_i)
 *                  + g_C sum_j (V_i - V_j)) / C_i, dx/dt = (x_inf - x)/tau_x,
 *                  p = (C, g_Na, E_Na, g_K, E_K, g_L, E_L, m_inf, tau_m, h_inf, tau_h, n_inf,
 *                  tau_n, g_C, T) per neuron, then I_a (P = 15 nu + 1); TVI_F64 only; two
 *                  neurons: one step per lane, backward Euler, analytic Jacobian; 3 to 10
 *                  neurons (n = 12..40): the block solver
 *   TVI_MDS        the mass-damper-spring chain (Section 5.1.1) of nu = n / 2 units, n even,
 *                  2 <= n <= 40, state (d_1, v_1, ..., d_nu, v_nu):
 *                  dd_i/dt = v_i, dv_i/dt = [K_i (d_{i+1} - d_i) + C_i (v_{i+1} - v_i)
 *                  - K_{i-1} (d_i - d_{i-1}) - C_{i-1} (v_i - v_{i-1})] / M_i + f_i(t),
 *                  position nu + 1 the wall (d = v = 0), no i - 1 terms for the first unit,
 *                  f_1 = f_a sin(2 pi t / T), f_i = 0 otherwise;
 *                  p = (K_1..K_nu, C_1..C_nu, M_1..M_nu, f_a, T) (P = 3 nu + 2); block solver
 *   TVI_FNODE      the forced neural ODE (Section 5.1.1), 1 <= n <= 40: x = (y, f_a sin(2 pi t / T)),
 *                  h = tanh(W3 tanh(W2 tanh(W1 x + b1) + b2) + b3), W1, W2 (n+1) x (n+1),
 *                  W3 n x (n+1); p = (W1, b1, W2, b2, W3, b3, f_a, T) row-major, per series
 *                  (P = 2 (n+1)^2 + 2 (n+1) + n (n+1) + n + 2); block solver
 *
 * The block solver (models above marked so) keeps one n x n block per wavefront,
 * one row per lane, one workgroup of 8 wavefronts per series (Section 3 for
 * blocks too large for one lane): TVI_F64, per-series parameters, backward
 * Euler, zero or extrapolated start, chunk <= 1024.  tvi_options.steps_per_lane
 * is its segment length T: each segment composes T steps serially (Thomas's
 * algorithm) and ceil(log2(chunk / T)) PCR levels join the segments; T = chunk
 * (or 0) is Thomas's algorithm, T = 1 pure PCR (lanes is ignored).  Its
 * forward pass needs tvi_options.workspace of tvi_forward_workspace_bytes()
 * bytes; its adjoint reads the stored trajectory (no recomputation) and needs
 * the workspace of tvi_adjoint_workspace_bytes().
 */
#ifndef TVI_H
#define TVI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TVI_LINEAR = 0,
    TVI_VANDERPOL = 1,
    TVI_ROBERTSON = 2,
    TVI_MLP = 3,
    TVI_CHABOCHE = 4,
    TVI_NEURON = 5,
    TVI_MDS = 6,
    TVI_FNODE = 7
} tvi_model_kind;

typedef enum { TVI_F32 = 0, TVI_F64 = 1 } tvi_dtype;

typedef enum {
    /* per series, written to status[] on the device */
    TVI_OK = 0,
    TVI_NOT_CONVERGED = 1, /* max_newton corrections at the shortest chunk allowed */
    TVI_SINGULAR = 2,      /* a diagonal block had a zero or non-finite pivot       */
    TVI_NONFINITE = 3,     /* a residual became NaN or infinite                     */
    /* returned by the host entry points */
    TVI_EINVAL = -1,
    TVI_EHIP = -2,
    TVI_ENOMEM = -3,
    TVI_EUNSUPPORTED = -4,
    TVI_ESCRATCH = -5      /* the workspace a call needs exceeds the static scratch of
                              tvi_solve_adjoint_noalloc (TVI_NOALLOC_SCRATCH_BYTES)  */
} tvi_status;

typedef enum {
    TVI_INIT_ZERO = 0,     /* Delta y = 0 over the chunk (Section 2.3)                        */
    TVI_INIT_EXTRAP = 1,   /* extrapolate the last step's slope over the chunk:
                              dy0_j = (t_{s+j} - t_s) h(y_s, t_s)                           */
    TVI_INIT_PREDICTOR = 2 /* the learned chunk predictor: dy0_j = base_j + p_j, base = the zero
                              start (predictor_base 0) or the extrapolated one (1), p = the
                              tvi_predictor network (n_in = n + 2: y_s, t_s, log(t_{s+1} - t_s);
                              n_out = n * predictor_steps), kept only where its chunk residual
                              is below the base's.  Analytic models: needs >= 4 lanes per series
                              and steps_per_lane * n <= 12 (TVI_EUNSUPPORTED otherwise)        */
} tvi_init;

typedef enum {
    TVI_BACKWARD_EULER = 0, /* y_k - y_{k-1} - dt_k h(y_k, t_k) = 0 (Section 2.2, Eq. backward-euler)  */
    TVI_FORWARD_EULER = 1   /* y_k - y_{k-1} - dt_k h(y_{k-1}, t_{k-1}) = 0 (Eq. forward-euler):
                               the same chunked Newton solve with identity diagonal blocks and
                               sub-diagonal blocks -(I + dt_j j(y_{j-1})), no block inverse; one
                               correction per chunk for a linear h.  Every model; not with
                               TVI_INIT_PREDICTOR (TVI_EUNSUPPORTED).  The adjoint is that of
                               the explicit map                                                */
} tvi_scheme;

typedef enum {
    TVI_JACOBIAN_ANALYTIC = 0,  /* the hand-written j = dh/dy (Section 2.2, the analytic option)          */
    TVI_JACOBIAN_FORWARD_AD = 1 /* forward-mode automatic differentiation of h (Section 2.2, the forward
                                   AD option): one evaluation of h on dual numbers seeded with the unit
                                   vectors gives j in registers.  Analytic models with TVI_F64 storage,
                                   backward Euler, zero or extrapolated start
                                   (TVI_EUNSUPPORTED otherwise)                                        */
} tvi_jacobian;

typedef struct {
    int32_t kind;          /* tvi_model_kind                                   */
    int32_t n;             /* state size                                       */
    int32_t dtype;         /* tvi_dtype of every floating-point array          */
    int32_t params_shared; /* 1: one parameter vector [P] for all series       */
    int32_t hidden;        /* MLP hidden width (ignored by the other models)   */
} tvi_model;

typedef struct {
    int32_t chunk;          /* steps solved together, >= 1 (Section 2.3)           */
    int32_t lanes;          /* lanes per series S: 1,4,8,16,32,64 (one wavefront;
                               chunk <= 512), or 128, 256 (2 or 4 wavefronts, one
                               workgroup per series, steps_per_lane 2, 4 or 8, chunk
                               <= 2048; TVI_VANDERPOL and TVI_ROBERTSON with
                               TVI_F64 storage, backward Euler, analytic Jacobian,
                               zero or extrapolated start, the forward pass and
                               the adjoint from the stored trajectory;
                               TVI_EUNSUPPORTED otherwise); 0 = choose from chunk
                               (above 512 steps: 8 steps per lane over 2 or 4
                               wavefronts)                                           */
    int32_t steps_per_lane; /* steps a lane composes serially T: 1,2,4,8; 0 = choose;
                               chunk <= lanes * steps_per_lane                       */
    int32_t max_newton;     /* Newton corrections per attempt, >= 1                   */
    double tol_a, tol_r;    /* converged iff ||R|| <= tol_a or ||R|| <= tol_r ||R0||,
                               R the chunk residual (Algorithm 1)                     */
    int32_t init;           /* tvi_init                                              */
    int32_t halving;        /* 1: retry a failed chunk at half its length, down to 1 */
    const void *predictor;  /* TVI_INIT_PREDICTOR: the predictor's parameters in the
                               inference layout written by tvi_predictor_pack (device) */
    int32_t predictor_hidden;  /* its hidden width, <= 256                          */
    int32_t predictor_steps;   /* steps it predicts, >= chunk                       */
    int32_t predictor_base;    /* 0: corrections to the zero start, 1: to the
                                  extrapolated start (TVI_INIT_EXTRAP)              */
    const int32_t *order;      /* NULL, or the launch order [B] (device): series
                                  order[i] is solved in launch slot i.  Must be a
                                  permutation of 0..B-1 (entries outside [0, B)
                                  leave their slot idle; repeated entries give
                                  undefined results; a series no entry names is
                                  not solved: its outputs are left unwritten, and
                                  a shared-parameter gradient (the neural ODE's
                                  dL/dtheta) is undefined).  See
                                  tvi_order_longest_first                          */
    int32_t scheme;            /* tvi_scheme                                        */
    int32_t jacobian;          /* tvi_jacobian: how the state Jacobian j is formed   */
    int32_t reference_residual;/* the R0 of the relative test ||R|| <= tol_r ||R0||:
                                  0: the residual of the attempt's first iterate
                                  (for the zero start, Algorithm 1's n0); 1: the
                                  residual at dy = 0 whatever the start (Algorithm
                                  1's n0 in every case: a better start may stop
                                  sooner; one more residual evaluation per attempt.
                                  Analytic models: backward Euler, extrapolated start,
                                  no AD Jacobian, not the
                                  one-step-per-lane models (TVI_EUNSUPPORTED
                                  otherwise); the neural ODE: any start          */
    void *workspace;           /* block-solver forward pass: device buffer of
                                  tvi_forward_workspace_bytes() bytes (caller-owned,
                                  contents need no initialisation); NULL otherwise */
    size_t workspace_bytes;    /* its size                                           */
    const double *g_divisor;   /* adjoint: NULL, or a device scalar that divides every
                                  entry of g: with g = y and g_divisor = the loss of
                                  tvi_loss_grad(TVI_LOSS_FROBENIUS, ..., g = NULL, loss),
                                  g = y / L is used without being formed in memory */
    const int32_t *obs_idx;    /* adjoint: NULL (g in the trajectory's layout), or the
                                  observed steps, strictly increasing step indices
                                  (device, uniform grids only): g is then
                                  [B][n_obs][n], dL/dy at step obs_idx[i] in row i,
                                  and zero at every other step (Appendix A: dL/dy
                                  enters only where the loss observes the state)    */
    int32_t n_obs;             /* its length, >= 1 when obs_idx is given            */
                               /* g_divisor and obs_idx: the neural ODE (TVI_MLP) and
                                  the block solver (state sizes above 8); g_divisor
                                  also in the stored-trajectory adjoint over several
                                  waves (Robertson and Van der Pol, TVI_F64, lanes
                                  128 or 256).  Elsewhere the adjoint returns
                                  TVI_EUNSUPPORTED when either is set              */
    int32_t max_newton_chunk;  /* corrections an attempt of more than one step may take
                                  before it is halved (0: max_newton); a single step
                                  still takes up to max_newton.  A failing long
                                  attempt then costs less; the converged result is
                                  the same fixed point (the register and wide
                                  solvers; the neural ODE and the block solver
                                  ignore it)                                       */
    double *series_sumsq;      /* forward: NULL, or [B] (device, written): each
                                  series' sum of squares of its states y_0 .. y_N as
                                  they are committed (a failed series: those before
                                  its failure), summed in a fixed order.  The
                                  Frobenius loss then needs no pass over the
                                  trajectory (tvi_loss_from_sums).  The forward
                                  pass over several waves only (lanes 128 or 256,
                                  Robertson and Van der Pol, TVI_F64);
                                  TVI_EUNSUPPORTED elsewhere                        */
} tvi_options;

/* Fills `opt` with the defaults: chunk 64, tol_a 1e-8, tol_r 1e-6 (Section 2.3),
 * max_newton 50, lanes/steps chosen from chunk, TVI_INIT_ZERO, halving on, no
 * predictor (predictor_base 1 once one is given), series in index order,
 * backward Euler, the analytic Jacobian, the first iterate's residual as the reference of the relative test. */
void tvi_default_options(tvi_options *opt);

/* tvi_order_longest_first -- the launch order that solves ragged series
 * longest first (ties by index): order[B] (device, written) from the point
 * offsets [B+1] (device).  Each series is one workgroup or lane segment and
 * the dispatcher hands out workgroups in launch order as slots free up, so
 * this is the longest-processing-time-first schedule of the batch (series are
 * independent, Section 2.1).  Results do not depend on the order.  Enqueued on
 * `stream`; O(B^2 / 1024) LDS-tiled comparisons, computed once per batch. */
tvi_status tvi_order_longest_first(const int64_t *offsets, int64_t B, int32_t *order, void *stream);

const char *tvi_status_str(int32_t status);
const char *tvi_version(void);
int32_t tvi_param_count(const tvi_model *model);

/*
 * tvi_model_eval -- the model rate h(y, t; p) and its state Jacobian
 * j = dh/dy for M independent states: the assembly of the chunk system's
 * residual and diagonal blocks (Section 2.3) as an entry point of its own.
 *
 *   states [M][n], times [M] or NULL (t = 0; every model here is autonomous),
 *   params [M][P] or shared [P] (model->params_shared; required for TVI_MLP),
 *   f [M][n] or NULL, J [M][n][n] or NULL (not both NULL).
 * Returns TVI_OK once enqueued, TVI_EINVAL / TVI_EUNSUPPORTED on bad arguments.
 */
tvi_status tvi_model_eval(const tvi_model *model, int64_t M, const void *states, const void *times,
                          const void *params, void *f, void *J, void *stream);

/*
 * tvi_pcr_solve -- batched block-bidiagonal solve (Section 3), the linear
 * kernel of the chunked Newton update (Eq. batched-update).
 *
 * For each of B independent systems of m block rows with n x n diagonal
 * blocks D[b][j] and sub-diagonal blocks -I, solves
 *   transpose = 0:  D_1 x_1 = r_1,          D_j x_j - x_{j-1} = r_j  (j = 2..m)
 *   transpose = 1:  D_m^T x_m = r_m,        D_j^T x_j - x_{j+1} = r_j (j = m-1..1)
 * by parallel cyclic reduction: every block is inverted (Gauss-Jordan with
 * partial pivoting), a lane composes T consecutive rows, and log2(S)
 * reduction levels run across the S lanes of the system.  The tiling is the
 * library's: the fewest rows per lane that hold m rows in one wave, raised
 * for 3 x 3 and larger blocks (to 2 rows per lane, 8 for float 4 x 4) while
 * at least four lanes share a system.
 *
 *   D  [B][m][n][n]   r, x  [B][m][n]     (dtype float or double, device)
 *   n in {2, 3, 4}, 1 <= m <= 512; n = 8 (the neural ODE's blocks) with
 *   TVI_F32 and 1 <= m <= 128.  Double storage computes in double, float
 *   storage in float.
 * A system with a singular block gets NaN in x.  Returns TVI_OK once enqueued,
 * TVI_EINVAL on bad sizes or null pointers, TVI_EHIP on a launch failure.
 */
tvi_status tvi_pcr_solve(int32_t dtype, int32_t n, int64_t B, int64_t m, const void *D, const void *r,
                         void *x, int32_t transpose, void *stream);

/*
 * tvi_solve_forward -- chunked backward Euler (Algorithm 1).
 *
 * Integrates every series over its grid; each chunk of opt->chunk steps is
 * solved by Newton iterations on the chunk residual (Eq. batched-backward-
 * euler) started from opt->init.  A chunk whose Newton iteration fails is
 * retried at half its length when opt->halving is set (the result -- the
 * backward-Euler trajectory -- does not depend on the chunk length); a
 * failure at length 1 stops the series: status[b] gets the code and y from
 * the failed step on is NaN.
 *
 *   y_out   [B][N+1][n] or ragged (required)
 *   ckpt    [B][ceil(N_max/chunk)+1][n] or NULL
 *   status  int32 [B] (required), iters int32 [B] total Newton corrections (or NULL)
 * N is the number of steps of the uniform grid, or, with offsets, the largest
 * N_b (it sizes the checkpoint array).  y_out may be NULL when ckpt is given.
 */
tvi_status tvi_solve_forward(const tvi_model *model, const tvi_options *opt, int64_t B, int64_t N,
                             const int64_t *offsets, const void *times, const void *y0,
                             const void *params, void *y_out, void *ckpt, int32_t *status,
                             int32_t *iters, void *stream);

/*
 * tvi_solve_adjoint -- discrete adjoint of tvi_solve_forward (Appendix A).
 *
 * With F_k = y_k - y_{k-1} - dt_k h(y_k, t_k; p) the backward-Euler map and
 * g_k = dL/dy_k, computes
 *   (I - dt_k j_k)^T lam_k = lam_{k+1} + g_k   (k = N_b..1, lam_{N_b+1} = 0),
 *   dL/dp  = sum_k dt_k (dh/dp (y_k))^T lam_k,   dL/dy0 = g_0 + lam_1,
 * with j_k = dh/dy at the converged y_k, chunk by chunk in reverse order: each
 * chunk is the transposed block-bidiagonal system of Appendix A.2, solved by
 * the same reduction run backwards.
 *
 * The states come either from the full trajectory `y` (then ckpt may be
 * NULL) or, when y is NULL, are recomputed chunk by chunk from the
 * checkpoints `ckpt` written by tvi_solve_forward with the same options;
 * recomputed states are bitwise those of the forward pass.  `workspace` of
 * tvi_adjoint_workspace_bytes() bytes (device) is needed for recomputation
 * and, for TVI_MLP, always (per-series partial gradients, summed afterwards
 * over the series in a fixed order); otherwise it may be NULL.
 *
 *   g       dL/dy [B][N+1][n] or ragged (required); [B][n_obs][n] with
 *           tvi_options.obs_idx (uniform grids; TVI_MLP and the block solver)
 *   dLdp    [B][P] for per-series parameters (TVI_LINEAR, TVI_VANDERPOL,
 *           TVI_ROBERTSON); [P] for the shared parameters of TVI_MLP
 *   dLdy0   [B][n]
 *   status  int32 [B]: SINGULAR if a transposed block could not be inverted,
 *           or the code of a failed recomputation; that series' outputs are NaN
 */
size_t tvi_adjoint_workspace_bytes(const tvi_model *model, const tvi_options *opt, int64_t B);

/* Bytes of tvi_options.workspace the forward pass of B series needs: nonzero
 * only for models solved by the block solver (per series: the chunk's inverse
 * blocks, segment maps, offsets and Newton iterate, 8 (chunk (NP^2 + 2 NP) +
 * 2 S NP^2 + ...) bytes with NP the state size padded to 8, 16, 24, 32 or 40
 * and S = ceil(chunk / steps_per_lane)).  0 for unsupported arguments. */
size_t tvi_forward_workspace_bytes(const tvi_model *model, const tvi_options *opt, int64_t B);

tvi_status tvi_solve_adjoint(const tvi_model *model, const tvi_options *opt, int64_t B, int64_t N,
                             const int64_t *offsets, const void *times, const void *params,
                             const void *y, const void *ckpt, const void *g, void *dLdp,
                             void *dLdy0, int32_t *status, void *workspace, size_t workspace_bytes,
                             void *stream);

/*
 * tvi_solve_adjoint_noalloc -- tvi_solve_adjoint for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The same computation and kernels, with the
 * workspace taken from a static device array of TVI_NOALLOC_SCRATCH_BYTES
 * bytes instead of a caller buffer; each GPU the library runs on holds its own
 * copy of that array until the process ends.  Nothing is allocated or freed.
 *
 * Arguments as tvi_solve_adjoint without the workspace.  The current device
 * (hipSetDevice) must be the one `stream` belongs to: its copy of the array is
 * used, its address looked up on the first call on that device.
 * Returns TVI_ESCRATCH, with nothing enqueued, when
 * tvi_adjoint_workspace_bytes(model, opt, B) exceeds TVI_NOALLOC_SCRATCH_BYTES
 * (recomputed states need B * chunk * n doubles, the neural ODE B * P floats),
 * TVI_EHIP when the array's address cannot be obtained, otherwise what
 * tvi_solve_adjoint returns.  The array keeps the last call's contents; every
 * byte a call reads from it was written earlier in the same call, so nothing
 * needs clearing.  Calls on one GPU share the array: calls that overlap in
 * time there (two streams, or two host threads) race and give undefined
 * results; calls in sequence on one stream are safe.
 */
#define TVI_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
tvi_status tvi_solve_adjoint_noalloc(const tvi_model *model, const tvi_options *opt, int64_t B, int64_t N,
                                     const int64_t *offsets, const void *times, const void *params,
                                     const void *y, const void *ckpt, const void *g, void *dLdp, void *dLdy0,
                                     int32_t *status, void *stream);

/*
 * tvi_loss_grad -- value and gradient g = dL/dy of the losses the benchmarks
 * integrate, over `points` states of size n (y and g [points][n], device):
 *   TVI_LOSS_FROBENIUS    L = sqrt(sum y^2) over every entry (the timing loss of
 *                         Section 5.2), g = y / L
 *   TVI_LOSS_MEAN_SQUARE  L = sum over observed points of |y|^2 / (n_observed n),
 *                         g = 2 y / (n_observed n) at observed points, 0 elsewhere;
 *                         observed: uint8 [points] (device), n_observed its count
 * The sum is reduced in a fixed order (deterministic).  loss: one double
 * (device).  g may be NULL: then only the loss is computed (for the Frobenius
 * loss the adjoint can take g = y with tvi_options.g_divisor = loss).
 * workspace: tvi_loss_workspace_bytes() bytes (device).  Enqueued on `stream`
 * without host synchronisation, so it can be captured in a graph.
 */
typedef enum { TVI_LOSS_FROBENIUS = 0, TVI_LOSS_MEAN_SQUARE = 1 } tvi_loss_kind;
size_t tvi_loss_workspace_bytes(void);
tvi_status tvi_loss_grad(int32_t kind, int32_t dtype, int64_t points, int32_t n, const void *y,
                         const uint8_t *observed, int64_t n_observed, void *g, double *loss, void *workspace,
                         size_t workspace_bytes, void *stream);

/*
 * tvi_loss_from_sums -- the Frobenius loss L = sqrt(sum_b sums[b]) of the
 * timing loss (Section 5.2) from per-series sums of squares (sums [B], device,
 * as tvi_options.series_sumsq writes them), summed in a fixed order; loss: one
 * double (device).  With it a captured step needs no pass over the trajectory
 * before the adjoint reads g = y / L (tvi_options.g_divisor = loss).  Enqueued
 * on `stream` without host synchronisation; TVI_EINVAL for B < 1 or NULL
 * pointers.
 */
tvi_status tvi_loss_from_sums(const double *sums, int64_t B, double *loss, void *stream);

/*
 * Learned chunk predictor: x -> GELU(W1 x + b1) -> GELU(W2 . + b2) -> W3 . + b3,
 * x standardised by fixed constants.  Float32.  params (device) packs
 * W1[hidden][n_in], b1[hidden], W2[hidden][hidden], b2[hidden],
 * W3[n_out][hidden], b3[n_out], then mean[n_in] and std[n_in] of the inputs:
 * tvi_predictor_param_count() floats; the first count - 2 n_in are the
 * trained network.  GELU is the exact x (1 + erf(x / sqrt 2)) / 2.
 *
 * tvi_predictor_forward      out [M][n_out] for inputs x [M][n_in].
 * tvi_predictor_train_step   one step of Adam (Kingma and Ba; beta1 0.9,
 *   beta2 0.999, eps 1e-8, bias-corrected; `step` counts from 1) on the
 *   mean squared error L = mean (out - target)^2 over a batch of M samples:
 *   writes L to loss[0] and dL/dnetwork to grad (count - 2 n_in floats),
 *   updates adam_m, adam_v (same size, zero before the first step) and the
 *   network part of params in place.  lr = 0 only evaluates L and the
 *   gradient.
 * Both need workspace of tvi_predictor_workspace_bytes(M) bytes (device).
 * tvi_predictor_pack         the inference layout the solvers read
 *   (tvi_options.predictor): the same count of floats with W1, W2, W3 stored
 *   transposed (W1^T[n_in][hidden], b1, W2^T[hidden][hidden], b2,
 *   W3^T[hidden][n_out], b3, mean, std), so that lanes computing neighbouring
 *   outputs read neighbouring weights.  packed must not alias params.
 */
typedef struct {
    int32_t n_in, hidden, n_out;
} tvi_predictor;
int64_t tvi_predictor_param_count(const tvi_predictor *p);
size_t tvi_predictor_workspace_bytes(const tvi_predictor *p, int64_t M);
tvi_status tvi_predictor_forward(const tvi_predictor *p, int64_t M, const float *x, const float *params,
                                 float *out, void *workspace, size_t workspace_bytes, void *stream);
tvi_status tvi_predictor_train_step(const tvi_predictor *p, int64_t M, const float *x, const float *target,
                                    float *params, float *grad, float *adam_m, float *adam_v, int64_t step,
                                    float lr, float *loss, void *workspace, size_t workspace_bytes,
                                    void *stream);
tvi_status tvi_predictor_pack(const tvi_predictor *p, const float *params, float *packed, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TVI_H */
