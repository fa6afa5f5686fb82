/*
 * rm.h -- C ABI of the MI355X (gfx950) long-step Richardson(m) library.
 *
 * What it computes (Wang, Liu, Cui, Shu, "Momentum-Accelerated Richardson(m) and
 * Their Multilevel Neural Solvers", arXiv 2412.08076):
 *   - the operator A of a batch of independent 2D problems: the bilinear (Q1) FEM
 *     9-point stencil of -div(C grad u) = f with C = R(theta) diag(1, eps) R(theta)^T
 *     (§2.3, eq. anisotropy-poisson), or the 5-point finite-difference Helmholtz
 *     stencil (§3.2, eq. Helmholtz-Sponge-stencil), zero Dirichlet boundary;
 *   - Richardson(m) and NAG-Richardson(m) (§2, eq. Richardson(m); Table 1) with
 *     per-instance, per-inner-step weights omega_i and momentum alpha_i (§2.2,
 *     the weight vector of the neural solver), the relative residual
 *     ||f - A u|| / ||f|| after every outer iteration (§2.3 stopping rule);
 *   - the reverse-mode derivative of a K-step unroll with respect to omega, alpha
 *     and f, used to train the weight network (§2.2, Algorithm 1, loss L2);
 *   - the weight network Meta(theta; mu) itself (§2.2-2.3): a fully connected
 *     network from (log10 eps, theta) to the m weights and the momentum.
 *
 * Conventions shared by every call
 *   - Every vector, weight array and gradient is a DEVICE pointer owned by the
 *     caller.  Host pointers are marked "host".  The library owns only its
 *     context, plans and internal scratch.
 *   - A batch of B instances is placed in instance order at the plan's offsets
 *     (back to back unless rm_plan is given offsets); instance b has n_b x n_b
 *     interior unknowns stored row-major as u[j][i] with i (the x index) fastest
 *     and y increasing with j; h = 1/(n_b + 1).  P_tot is the length of every
 *     vector (the sum of n_b^2 when packed).  Boundary values are never stored
 *     (they are zero).
 *   - Weight arrays omega[B][m], alpha[B][m] are row-major; inner step s of a
 *     solve uses index i = s mod m, so omega[b][0] is applied first (the order
 *     T_m = (I - omega_m A) ... (I - omega_1 A) of eq. Chebyshev(m)T).  The
 *     library never reorders weights.
 *   - All work is enqueued on the stream given to rm_create.  Calls return as
 *     soon as the work is enqueued, except where a call says it blocks.
 *   - Errors: a non-zero rm_status is returned, nothing is thrown.  Argument
 *     errors are detected on the host before anything is launched (RM_EINVAL).
 *     RM_EHIP means a HIP runtime call failed; rm_last_error() describes it.
 *   - A context and its plans may be used from one host thread at a time.
 */
#ifndef RM_H
#define RM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RM_OK = 0,
  RM_EINVAL = 1,       /* bad argument; nothing was launched                    */
  RM_ENOMEM = 2,       /* device allocation failed                             */
  RM_EHIP = 3,         /* a HIP runtime call failed                            */
  RM_ENOTCONV = 4,     /* an instance hit its iteration or round cap           */
  RM_EDIVERGED = 5,    /* an instance produced a non-finite or growing residual */
  RM_EUNSUPPORTED = 6  /* valid request the library does not implement         */
} rm_status;

typedef enum { RM_Q1_ANISO = 0, RM_FD5_HELMHOLTZ = 1 } rm_op;

/* Table 1 of the paper, last column.  All four run in the NAGex form
 *   u~ = u + at_i v;  v' = a_i v + omega_i B^{-1} (f - A u~);  u' = u + v'
 * with: RM_RICHARDSON a = at = 0 (alpha ignored, may be NULL); RM_NAG at = a;
 * RM_MOM at = 0; RM_NAGEX a and at independent.  alpha holds a as [B][m]; for
 * RM_NAGEX it holds [2][B][m]: a, then at. */
typedef enum { RM_RICHARDSON = 0, RM_NAG = 1, RM_MOM = 2, RM_NAGEX = 3 } rm_method;

typedef enum { RM_F32 = 0, RM_F64 = 1 } rm_dtype;

typedef enum {
  RM_UNROLL = 0,  /* exactly K inner steps from (x0, v = 0), optional checkpoints */
  RM_TO_TOL = 1   /* FP32 sweeps inside FP64 iterative refinement, until tol      */
} rm_mode;

/* One problem instance (host).  op = RM_Q1_ANISO uses eps in (0, 1] and theta;
 * op = RM_FD5_HELMHOLTZ uses kappa (constant wavenumber, no sponge layer). */
typedef struct {
  int32_t n;       /* interior nodes per direction, 1 <= n <= 16384 */
  int32_t op;      /* rm_op */
  double eps;
  double theta;
  double kappa;
} rm_instance;

typedef struct {
  int32_t mode;        /* rm_mode                                                 */
  int32_t dtype;       /* RM_UNROLL: precision of the sweeps (RM_F32 or RM_F64)   */
  int32_t m;           /* inner steps per outer iteration, 1..64                  */
  int32_t K;           /* RM_UNROLL: inner steps, a multiple of m                 */
  int32_t ckpt_every;  /* RM_UNROLL: checkpoint spacing (divides K), 0 = none     */
  int32_t max_outer;   /* RM_TO_TOL: outer iterations per refinement round, cap   */
  int32_t max_rounds;  /* RM_TO_TOL: refinement rounds, cap                       */
  int32_t check_every; /* RM_TO_TOL + RM_FLAG_GRAPH: iterations between polls >= 1 */
  int32_t flags;       /* RM_FLAG_* bits                                          */
  int32_t hist_len;    /* RM_TO_TOL: rows of hist (outer iterations recorded)     */
  double tol;          /* RM_TO_TOL: target ||b - A x|| / ||b|| (FP64)            */
  double tol_inner;    /* RM_TO_TOL: inner relative residual that ends a round    */
  double relax;        /* RM_FLAG_SSOR: relaxation factor a, 0 < a < 2           */
} rm_solve_opts;

/* RM_FLAG_GRAPH: RM_TO_TOL captures one outer iteration of the inner solve (its
 * sweep launches, the residual reduction and the convergence bookkeeping) in a
 * HIP graph and replays it instead of launching the kernels one by one.  Results
 * are identical either way; on ROCm 7.2 / MI355X replay measured 1-20 % slower
 * than direct launches for this loop, so it is off by default. */
#define RM_FLAG_GRAPH 1
/* RM_FLAG_JACOBI: weighted-Jacobi preconditioning (§2.1, eq. momentum-m-Binv with
 * B^{-1} = D^{-1}, D the constant diagonal of the instance's operator): every
 * omega_i is multiplied by 1/D; a relaxation factor is the caller's scaling of
 * omega.  Accepted by rm_solve (both modes) and rm_solve_adjoint (which then
 * returns the gradient with respect to the unscaled omega).  RM_EINVAL if an
 * instance has a zero diagonal. */
#define RM_FLAG_JACOBI 2
/* RM_FLAG_SSOR: SSOR preconditioning (§2.1, the SSOR entry of the stationary
 * preconditioners), B^{-1} = a (2 - a) (D - aU)^{-1} D (D - aL)^{-1} with A = D - L - U
 * and a = opts->relax.  L and U follow the four-colour ordering colour(i, j) =
 * (i mod 2) + 2 (j mod 2) on 0-based interior indices (the paper does not state an
 * ordering; this one leaves no two points of a colour coupled, so each triangular
 * solve is four parallel passes).  Every step is then one launch (no temporal
 * blocking).  Accepted wherever RM_FLAG_JACOBI is; the two exclude each other;
 * RM_EINVAL unless 0 < relax < 2. */
#define RM_FLAG_SSOR 4

/* Per-instance results of RM_TO_TOL (host arrays, any may be NULL; length B unless
 * stated).  history has max_rounds + 1 rows of B: row j holds
 * rho_j = ||b - A x_j|| / ||b|| (FP64) of the refinement round j (row 0: the initial
 * guess), the quantity the stopping rule of §2.3 tests; rows an instance did not reach
 * hold -1. */
typedef struct {
  int32_t* outer_iters;  /* outer iterations summed over all rounds          */
  int32_t* rounds;       /* refinement rounds used                           */
  double* relres;        /* final ||b - A x|| / ||b|| computed in FP64       */
  int32_t* status;       /* RM_OK, RM_ENOTCONV or RM_EDIVERGED per instance  */
  double* history;       /* [max_rounds + 1][B] rho_j per round, see above   */
} rm_report;

typedef struct rm_ctx rm_ctx;
typedef struct rm_plan_s rm_plan_t;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the handle.
 * rm_destroy waits for the stream; plans built on the context should be freed
 * first, and a plan that outlives it accepts only rm_plan_free. */
rm_status rm_create(rm_ctx** out, int32_t device, void* hip_stream);
rm_status rm_destroy(rm_ctx* ctx);

/* Build a plan for a batch (host array inst[B]).  Computes the stencil
 * coefficients of every instance in FP64 (§2.3 / §3.2), the offsets and the tile
 * tables, and uploads them.  Rejects n < 1, n > 16384, eps outside (0, 1],
 * non-finite parameters, unknown op.
 * offsets (host int64 [B + 1], copied; NULL = packed back to back from 0): instance b
 * occupies elements [offsets[b], offsets[b] + n_b^2) of every vector, and P_tot =
 * offsets[B] is the length of every vector.  Needs offsets[0] >= 0 and
 * offsets[b + 1] - offsets[b] >= n_b^2 (RM_EINVAL otherwise).  Elements outside the
 * instances (gaps) are never read; the library may overwrite the gaps of its output
 * vectors (x, ckpt, gradients) with unspecified values. */
rm_status rm_plan(rm_ctx* ctx, int32_t B, const rm_instance* inst, const int64_t* offsets, rm_plan_t** out);
rm_status rm_plan_free(rm_plan_t* plan);

/* Host queries: number of instances, P_tot, and the offsets
 * (host array off[B + 1], off[B] = P_tot). */
int32_t rm_plan_batch(const rm_plan_t* plan);
int64_t rm_plan_points(const rm_plan_t* plan);
rm_status rm_plan_offsets(const rm_plan_t* plan, int64_t* off);
/* Host copy of the five stencil coefficients per instance (host coef[B][5]:
 * centre, (+-1,0), (0,+-1), (1,1)/(-1,-1), (-1,1)/(1,-1)) and of the
 * Gershgorin bound |centre| + sum |off-diagonal| (host gersh[B]). */
rm_status rm_plan_coefficients(const rm_plan_t* plan, double* coef, double* gersh);

/* Kernel configuration of the FP32 sweeps.  Instances are grouped by size n;
 * every size class runs a temporal-blocked kernel that advances up to T inner
 * steps per launch on extended tiles of cw x 8R points (cw a multiple of 8),
 * using 8 cw threads per workgroup.  Tile edges on the domain boundary need no
 * halo; interior edges overlap by T + 1 points, so an instance that fits in one
 * tile is computed without redundancy.  Kernel variant `shape` fixes R and the
 * largest cw: 0: R = 8, cw <= 64; 1: R = 16, cw <= 64; 2: R = 8, cw <= 128;
 * 3: R = 13, cw <= 64; 4: R = 16, cw <= 128; 5: R = 12, cw <= 96;
 * 6: R = 13, cw <= 104; 7: R = 32, cw <= 64; 8: R = 32, cw <= 96 (a 256-row tile
 * covers n <= 256 without a vertical halo).  Shape 9 is the row-streaming kernel
 * (n <= 1024, T <= 8): one workgroup of 64 ceil(n / 64) threads holds whole rows and
 * pipelines the T steps down a window of cw rows (cw >= n: the whole height, no
 * halo; otherwise windows overlap by T + 1 rows).  rm_plan picks a configuration
 * per class from a cost model; rm_tune measures.  All shapes reproduce one launch
 * per inner step bit for bit.
 * rm_plan_set_kernel: set (shape, T, cw) for the class of size n (n <= 0: all
 * classes; cw <= 0: the width the cost model prefers; 1 <= T <= 64); shape = -1
 * switches the whole plan to one launch per inner step.  It also resets the
 * class's tail configuration (below).  RM_EINVAL if the halo or width does not
 * fit the variant or no instance has size n. */
rm_status rm_plan_set_kernel(rm_plan_t* plan, int32_t n, int32_t shape, int32_t T, int32_t cw);
rm_status rm_plan_get_kernel(const rm_plan_t* plan, int32_t n, int32_t* shape, int32_t* T,
                             int32_t* cw);

/* Tail configuration of a size class: the kernel the refined RM_TO_TOL solve uses
 * once the fraction of instances still active drops below the switch point.  A
 * row-streaming launch costs about the same for one active instance as for all of
 * them, a tiled launch costs in proportion, so after rm_plan_set_kernel the tail is
 * the main configuration, or the cost model's best tiled variant when the main one
 * is row-streaming.  Same arguments and errors as rm_plan_set_kernel (shape >= 0).
 * Each size class switches on its own, from the count of its instances still active.
 * rm_plan_set_tail_switch: fraction of a class's instances still active below which
 * its tail runs, for every class (frac <= 1; 0: never; 1: always; < 0, the default:
 * per class, the ratio rm_tune measured between the main configuration's launch with
 * one instance active and the tail's with all active, or 0.35 before tuning).  Results
 * do not depend on the switch: every configuration computes the same iterates. */
rm_status rm_plan_set_tail_kernel(rm_plan_t* plan, int32_t n, int32_t shape, int32_t T, int32_t cw);
rm_status rm_plan_get_tail_kernel(const rm_plan_t* plan, int32_t n, int32_t* shape, int32_t* T,
                                  int32_t* cw);
rm_status rm_plan_set_tail_switch(rm_plan_t* plan, double frac);

/* Mixed-size launch (the batch of instances of different sizes of Algorithm 1 and
 * §2.3, advanced together).  on != 0: every size class whose main configuration is
 * the row pipeline with 8 steps per launch (rm_plan_set_kernel shape 9, T = 8) is
 * advanced, in that configuration, by one launch per chunk of steps shared by all
 * such classes: 1024-thread workgroups, each holding 1024 / (64 ceil(n / 64)) row
 * windows of equal height of one class.  Classes with another main configuration,
 * classes in their tail configuration and classes from the 65th on keep launches of
 * their own.  on = 0 (the default): one launch per class.  Iterates, residuals and
 * reports are bit for bit the same either way.  rm_plan_get_mixed returns the
 * setting.  RM_EINVAL for a null plan or pointer. */
rm_status rm_plan_set_mixed(rm_plan_t* plan, int32_t on);
rm_status rm_plan_get_mixed(const rm_plan_t* plan, int32_t* on);

/* Autotuner: for every size class, time each valid (shape, T, cw) on this plan's
 * data (16 inner steps of `method` with the given device weights and right-hand
 * side, best of 3) and keep the fastest as the main configuration and the fastest
 * tiled one as the tail; when the main one is row-streaming, also time it with one
 * instance active (the switch point).  cache_path (host string, may be NULL)
 * names a JSON file of choices keyed by "<gfx arch> n=<n> B=<class size>
 * m=<m> method=<method>", each [shape, T, cw, us, tail shape, tail T, tail cw,
 * tail us, one-active us] (entries of only the first four keep the model's
 * tail): classes found there are not timed again, new results are written back.  *us_per_step (may be NULL) receives the summed per-step
 * time of the chosen configurations in microseconds.  Blocks. */
rm_status rm_tune(rm_ctx* ctx, rm_plan_t* plan, int32_t method, int32_t m, const float* omega,
                  const float* alpha, const float* b, const char* cache_path, double* us_per_step);

/* y = A x for every instance (§2.3, §3.2).  x, y: device [P_tot] of `dtype`,
 * must not overlap. */
rm_status rm_apply_A(rm_ctx* ctx, const rm_plan_t* plan, int32_t dtype, const void* x, void* y);

/* r = b - A x and, per instance, ||r||^2 and ||b||^2 accumulated in FP64, and the
 * squared relative residual ||r||^2 / ||b||^2 (the per-instance loss of §2.2,
 * eq. loss-fun-relative-res, squared).
 * b, x: device [P_tot] of `dtype`; r: device [P_tot] of `dtype` or NULL (not
 * stored); r2, b2: device double [B] or NULL; rel2: device float [B] or NULL. */
rm_status rm_residual(rm_ctx* ctx, const rm_plan_t* plan, int32_t dtype, const void* b,
                      const void* x, void* r, double* r2, double* b2, float* rel2);

/* rm_residual without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results (bit for bit) and asynchrony as rm_residual;
 * the plan must already exist (rm_plan allocates its tables).  Its per-tile partial
 * sums go to a file-scope device array of RM_NOALLOC_MAX_TILES * 2 doubles (1 MiB)
 * that each GPU the library runs on holds until the process ends; its address is
 * looked up once per device by rm_create.  A plan has one tile per 64 x 32 block of
 * every instance (ceil(n / 64) * ceil(n / 32) for instance n) plus padding to a
 * multiple of 8: a plan with more than RM_NOALLOC_MAX_TILES tiles gives RM_EINVAL
 * before anything is launched.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's partials: calls that overlap on one GPU (other streams,
 * other contexts, other host threads) race and must be serialised by the caller. */
#define RM_NOALLOC_MAX_TILES 65536
rm_status rm_residual_noalloc(rm_ctx* ctx, const rm_plan_t* plan, int32_t dtype, const void* b,
                              const void* x, void* r, double* r2, double* b2, float* rel2);

/* Batched Richardson(m) / NAG-Richardson(m) (Table 1, last column; §2.3 evaluation).
 *
 * RM_UNROLL (asynchronous): K inner steps from u = x (in), v = 0, in opts->dtype.
 *   b, x: device [P_tot] of opts->dtype; x is overwritten with u_K.
 *   ckpt: device [K / ckpt_every][2][P_tot] of opts->dtype or NULL; slot c
 *         receives (u, v) before step c * ckpt_every (slot 0 = (x0, 0)).
 *   hist: device double [K / m][B] or NULL; receives ||b - A u||^2 after every
 *         outer iteration (squared, not divided by ||b||^2).
 *   rep is ignored.
 * RM_TO_TOL (blocks until every instance is done; runs on a stream of the
 *   context's own that first waits for the work already enqueued on the
 *   context's stream): FP64 iterative refinement
 *   around FP32 inner solves A d = fl32(b - A x) started from d = 0, v = 0, each
 *   run in whole outer iterations until its relative residual is <= tol_inner
 *   or max_outer is reached; x += d in FP64; stop when ||b - A x|| / ||b|| <= tol.
 *   b, x: device double [P_tot]; x holds the initial guess and receives the
 *   result.  ckpt must be NULL.  hist: device double [opts->hist_len][B] or
 *   NULL; row k receives ||r_j - A d||^2 of the inner solve after the instance's
 *   k-th outer iteration counted over all rounds from 0 (r_j the round's FP32
 *   right-hand side, so hist / ||b||^2 follows ||b - A x||^2 / ||b||^2 through
 *   the rounds), -1 in rows it did not reach; later iterations are not
 *   recorded.  rep (host) receives per-instance counts, final FP64 relative
 *   residuals, status and the per-round history; the call returns the worst
 *   per-instance status.  After an error other than RM_ENOTCONV / RM_EDIVERGED
 *   the call still waits for what it had queued.  The host learns how many instances are still
 *   active from a word the GPU writes into pinned memory after every outer
 *   iteration; it reads each iteration's word while the next iteration is
 *   already queued (without RM_FLAG_GRAPH), or synchronises every check_every
 *   replays (with it).
 * omega: device float [B][m]; alpha: device float [B][m] ([2][B][m] for RM_NAGEX;
 * ignored, may be NULL, for RM_RICHARDSON). */
rm_status rm_solve(rm_ctx* ctx, const rm_plan_t* plan, int32_t method, const rm_solve_opts* opts,
                   const float* omega, const float* alpha, const void* b, void* x, void* ckpt,
                   double* hist, rm_report* rep);

/* Reverse mode through the K-step FP32 unroll that rm_solve(RM_UNROLL) performed
 * with the same plan, method, opts, omega, alpha, b and its checkpoints ckpt
 * (opts->ckpt_every > 0 required).  Forward states are recomputed one
 * checkpoint segment at a time; A is symmetric, so the backward sweep applies
 * the same stencil.  When every size class runs the row-streaming kernel the
 * reverse steps run up to three per launch in its row pipeline, else one per
 * launch; both give the same d_b and loss bit for bit and the same weight
 * gradients up to the order of their FP64 sums.
 *   g_uK:  device float [P_tot], the seed dJ/du_K; or NULL for the loss mode
 *          J = sum_b g_loss[b] * ||b - A u_K||^2 / ||b||^2.
 *   g_loss: device float [B] (loss mode only; NULL = all ones).
 *   d_omega: device float [B][m]; d_alpha: device float [B][m] ([2][B][m] for
 *          RM_NAGEX: momentum then look-ahead factor; zeros for RM_RICHARDSON),
 *          overwritten with dJ/domega, dJ/dalpha.
 *   d_b: device float [P_tot] or NULL, overwritten with dJ/db.
 *   loss: device float [B] or NULL (loss mode: ||b - A u_K||^2 / ||b||^2).
 * Asynchronous.  Dot products are accumulated per tile in FP64 and summed in a
 * fixed order, so repeated calls give bitwise identical results. */
rm_status rm_solve_adjoint(rm_ctx* ctx, const rm_plan_t* plan, int32_t method,
                           const rm_solve_opts* opts, const float* omega, const float* alpha,
                           const float* b, const void* ckpt, const float* g_uK,
                           const float* g_loss, float* d_omega, float* d_alpha, float* d_b,
                           float* loss);

/* Two-grid cycle of the Helmholtz multilevel variant (§3: the smoothing
 * iteration eq. dl-him-b with a Table-1 scheme as smoother, then the spectral
 * correction eq. dl-him-h on a coarse grid).  One cycle from u_k:
 *   m inner steps of `method` from (u_k, v = 0) with omega_1 .. omega_m -> u_h;
 *   u_{k+1} = u_h + P S (symbol * (S R (b - A u_h) S)) S,
 * R full weighting onto the coarse grid (coarse point (I, J) on fine point
 * (2I+1, 2J+1), nc = (n - 1) / 2 per direction), P bilinear interpolation
 * (P = 4 R^T), S the orthonormal DST-I of the coarse grid (S = S^T = S^-1, the
 * eigenvector basis of every constant-coefficient Dirichlet operator there).
 * Every instance needs n + 1 a power of two, 8 <= n + 1 <= 1024; otherwise
 * RM_EUNSUPPORTED.
 * Coarse fields are packed like fine ones: instance b at coff[b], nc x nc, row
 * = y.  rm_plan_coarse_points returns their total Pc (-1 if the plan does not
 * qualify); rm_plan_coarse_offsets fills host coff[B].
 * symbol: device float [Pc], instance b's block [q][p] multiplies the sine
 *   coefficient of mode sin(p pi x) sin(q pi y) (p, q = 1..nc, stored at
 *   [q-1][p-1]).
 * rm_twogrid_solve (asynchronous): K = opts->K cycles in FP32 (opts->mode
 *   RM_UNROLL, opts->dtype RM_F32, opts->m smoothing steps per cycle,
 *   RM_FLAG_JACOBI honoured) from u = x.  b, x: device float [P_tot]; x is
 *   overwritten with u_K.  ckpt: device float [K][P_tot] or NULL, receives u_k
 *   at the start of every cycle (the adjoint needs it).  hist: device double
 *   [K][B] or NULL, receives ||b - A u_{k+1}||^2 after every cycle.
 * omega, alpha: as for rm_solve. */
int64_t rm_plan_coarse_points(const rm_plan_t* plan);
rm_status rm_plan_coarse_offsets(const rm_plan_t* plan, int64_t* coff);
rm_status rm_twogrid_solve(rm_ctx* ctx, const rm_plan_t* plan, int32_t method,
                           const rm_solve_opts* opts, const float* omega, const float* alpha,
                           const float* symbol, const float* b, float* x, float* ckpt,
                           double* hist);
/* Reverse mode through the K cycles rm_twogrid_solve performed (from any start
 * x; the start is ckpt slot 0), with the same plan, method, opts, omega, alpha,
 * symbol and b, and its ckpt (required).  Smoothing states are recomputed per cycle.  g_uK, g_loss,
 * d_omega, d_alpha, d_b, loss: as for rm_solve_adjoint.  d_symbol: device float
 * [Pc], overwritten with dJ/dsymbol.  Asynchronous; repeated calls give bitwise
 * identical results. */
rm_status rm_twogrid_adjoint(rm_ctx* ctx, const rm_plan_t* plan, int32_t method,
                             const rm_solve_opts* opts, const float* omega, const float* alpha,
                             const float* symbol, const float* b, const float* ckpt,
                             const float* g_uK, const float* g_loss, float* d_omega,
                             float* d_alpha, float* d_symbol, float* d_b, float* loss);

/* Symbol network of the two-grid cycle (§3: the meta network that produces the diagonal
 * Lambda~ of the spectral correction, eq. dl-him-h, there an FNO whose architecture the
 * text does not give; §3.2 learns the smoother weight in log form, and the exponential
 * below does the same for the symbol).  The one built here: per coarse mode (p, q) of instance
 * b (nc = (n - 1)/2, h = 1/(n + 1)), with lam the fine-grid eigenvalue
 * (4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2)) - kappa^2,
 *   features  (lam h^2 / 8, p / (nc + 1), q / (nc + 1)),
 *   z = conv3(tanh(conv2(tanh(conv1(features))))),  3 x 3 cross-correlations with zero
 *       padding, 3 -> 16 -> 16 -> 1 channels,
 *   symbol = lam / (lam^2 + 1) * exp(z)   (a log-form correction of the regularised
 *            inverse eigenvalue; layout as the symbol of rm_twogrid_solve).
 * params: device float [rm_symbolnet_param_count() = 2913], layout
 *   W1[16][3][3][3], b1[16], W2[16][16][3][3], b2[16], W3[1][16][3][3], b3[1].
 * Every instance must be Helmholtz and qualify for the two-grid cycle (RM_EINVAL /
 * RM_EUNSUPPORTED otherwise).  rm_symbolnet_forward: symbol (device float [Pc]) for every
 * instance.  rm_symbolnet_backward: d_params (device float [2913], overwritten) = the
 * gradient of sum(d_symbol * symbol) with respect to params, summed over the batch in a
 * fixed order (repeated calls give identical bits); d_symbol: device float [Pc], e.g. the
 * d_symbol of rm_twogrid_adjoint.  Both asynchronous. */
int32_t rm_symbolnet_param_count(void);
rm_status rm_symbolnet_forward(rm_ctx* ctx, const rm_plan_t* plan, const float* params, float* symbol);
rm_status rm_symbolnet_backward(rm_ctx* ctx, const rm_plan_t* plan, const float* params, const float* d_symbol,
                                float* d_params);

/* Restarted flexible GMRES with a neural solver as the preconditioner (§3.2: FGMRES,
 * restart 20, preconditioned by a multilevel neural solver).  Every instance runs its
 * own FGMRES in FP64 (basis, Hessenberg, Givens rotations); the preconditioner maps
 * v to the FP32 result z of `inner` applied to A z = fl32(v) from z = 0:
 *   inner == NULL:            z = fl32(v) (plain restarted GMRES);
 *   symbol == NULL:           inner->K inner steps of `method` (inner->m weights,
 *                             RM_FLAG_JACOBI / RM_FLAG_SSOR honoured);
 *   symbol != NULL:           inner->K two-grid cycles (see rm_twogrid_solve).
 * inner->mode must be RM_UNROLL, inner->dtype RM_F32.  Because the preconditioner is an
 * iteration, its action may vary between steps; FGMRES keeps the directions z_j.
 * Instance b stops when ||b - A x|| / ||b|| <= tol (tested on the FP64 residual at each
 * restart, estimated by the rotations in between) or after max_iter Arnoldi steps.
 * b, x: device double [P_tot]; x is the initial guess and receives the result.
 * rep (host, may be NULL): Arnoldi steps (outer_iters), cycles (rounds), the last true
 * relative residual and RM_OK / RM_ENOTCONV / RM_EDIVERGED per instance (history is not
 * written).  Blocks; the call returns the worst per-instance status. */
typedef struct {
  int32_t restart;   /* Krylov dimension per cycle, 1..64 */
  int32_t max_iter;  /* Arnoldi steps per instance        */
  double tol;        /* relative residual target          */
} rm_fgmres_opts;
rm_status rm_fgmres(rm_ctx* ctx, const rm_plan_t* plan, const rm_fgmres_opts* fo, int32_t method,
                    const rm_solve_opts* inner, const float* omega, const float* alpha,
                    const float* symbol, const double* b, double* x, rm_report* rep);

/* Meta network (§2.2-2.3).  params: device float [5457 for m = 16; in general
 * 64*2 + 64 + 64*64 + 64 + (m+1)*64 + (m+1)], layout
 *   W1[64][2], b1[64], W2[64][64], b2[64], W3[m+1][64], b3[m+1]  (out x in).
 * Input of instance b is (log10 eps_b, theta_b) taken from the plan (Q1
 * instances; Helmholtz instances use (0, kappa)).  Forward:
 *   z = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3,
 *   omega[b][i] = exp(z_i) / G_b (G_b the Gershgorin bound), alpha[b][i] = 1/(1+exp(-z_m)).
 * omega, alpha: device float [B][m] outputs. */
rm_status rm_meta_forward(rm_ctx* ctx, const rm_plan_t* plan, int32_t m, const float* params,
                          float* omega, float* alpha);
/* Gradient of sum_b <d_omega_b, omega_b> + <d_alpha_b, alpha_b> with respect to
 * params, summed over the batch in a fixed order.  d_params: device float
 * [n_params], overwritten. */
rm_status rm_meta_backward(rm_ctx* ctx, const rm_plan_t* plan, int32_t m, const float* params,
                           const float* d_omega, const float* d_alpha, float* d_params);

/* Number of meta-network parameters for a given m. */
int32_t rm_meta_param_count(int32_t m);

const char* rm_status_string(rm_status s);
/* Text of the last error recorded on this thread (argument or HIP error). */
const char* rm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RM_H */
