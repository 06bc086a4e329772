/*
 * blob_rd: linear solves of the minimally-resolved reactive blob model
 * (Bhalla, Griffith, Patankar, Donev, arXiv:1306.3159) on one AMD Instinct
 * MI355X (gfx950).
 *
 * Problem (all on a 3-D periodic, cell-centred grid, cell k centred at
 * (k + 1/2) h, arrays laid out [z][y][x] with x fastest):
 *   L          the standard 7-point Laplacian (Sec. III.A);
 *   J          local averaging, (J c)_i = sum_k phi_w(q_i - r_k) c_k, with the
 *              tensor-product Peskin kernel phi_w, w = 4 or 3 (Sec. III.A,
 *              eq. tensor_product);
 *   S          spreading, S = h^-3 J^T (Sec. III.A);
 *   kappa      per-blob reaction rates (eq. c_t_blob).
 *
 * Conventions for every entry point:
 *   - Grid vectors (f, c) are caller-owned DEVICE pointers to nx*ny*nz
 *     doubles, contiguous, [z][y][x].
 *   - Blob vectors (q, kappa, lambda) are caller-owned DEVICE pointers:
 *     q is [N][3] doubles (x, y, z, physical units, any real value: wrapped
 *     periodically), kappa and lambda are [N] doubles.
 *   - The library allocates no device memory: all scratch lives in the
 *     caller's workspace (blob_rd_workspace_bytes). The handle owns only a
 *     small host structure.
 *   - Work is enqueued on the caller's HIP stream (NULL = legacy default
 *     stream). Solves return once convergence is known: they synchronise the
 *     stream to read convergence scalars; outputs are complete on return.
 *   - Return codes: 0 success; BLOB_RD_ENOTCONV (1) iteration limit reached,
 *     best iterate written and stats filled; negative values are hard
 *     errors (nothing meaningful written). No exception crosses the ABI;
 *     blob_rd_last_error() describes the most recent failure on the calling
 *     thread.
 */
#ifndef BLOB_RD_H
#define BLOB_RD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BLOB_RD_OK 0
#define BLOB_RD_ENOTCONV 1
#define BLOB_RD_EINVAL (-1)
#define BLOB_RD_ENOMEM (-2)   /* workspace too small */
#define BLOB_RD_EDEVICE (-3)  /* HIP runtime error */
#define BLOB_RD_ESINGULAR (-4)
#define BLOB_RD_ENUMERIC (-5) /* NaN/Inf detected or Krylov breakdown */

#define BLOB_RD_FP64 0   /* FP64 V-cycles */
#define BLOB_RD_MIXED 1  /* FP32 V-cycles under FP64 Krylov, residuals and refinement */

#define BLOB_RD_PRECOND_NONE 0
#define BLOB_RD_PRECOND_DIAGONAL 1 /* scalar gamma^-1 of eq. Schur_diagonal */
#define BLOB_RD_PRECOND_LEARNED 2  /* sparse pairwise network preconditioner */

/* Absorbing solves of a handle (blob_rd_params.saddle_solver). The block
 * solvers reserve the flexible-GMRES basis (restart = gmres_restart) in the
 * handle's workspace, see blob_rd_solve_absorbing_fgmres. */
#define BLOB_RD_SOLVER_SCHUR 0         /* Schur-complement GMRES with inner multigrid-CG solves */
#define BLOB_RD_SOLVER_BLOCK 1         /* block FGMRES, approximate-Schur preconditioner (m = 5, n = 1) */
#define BLOB_RD_SOLVER_BLOCK_LEARNED 2 /* the same with the learned inner preconditioning */

/* Domain of a handle (blob_rd_params.boundary).
 * PERIODIC: the periodic cell of Sec. III (every operation of this header).
 * DIRICHLET: a box whose faces hold c = boundary_value (the single-blob tests of
 * Sec. IV.C, eq. c_r_approx). On the cell-centred grid the face value is the
 * mean of a boundary cell and its ghost, so the 7-point Laplacian takes the
 * ghost 2 c_b - c. Solves work on u = c - c_b: the operator becomes
 * alpha I - D L_0 (ghost -u, invertible for every alpha >= 0, no null space),
 * the reactive right side f - alpha c_b - c_b S kappa and the absorbing
 * constraint J u = -c_b; c is returned with c_b added back. Every blob must lie
 * at least 3h inside each face (its kernel support then stays off the boundary
 * cells and J 1 = 1), else blob_rd_create returns EINVAL. Supported: the
 * reactive solve and step, the absorbing solve and step with saddle_solver
 * BLOCK or BLOCK_LEARNED (the learned part is never used in a box: its network
 * models the periodic cell), blob_rd_solve_absorbing_fgmres and the operator
 * calls (blob_rd_apply applies the homogeneous operator alpha I - D L_0 [+ S kappa J],
 * blob_rd_vcycle its V-cycle, blob_rd_time_kernel the box forms of its kernels).
 * EINVAL: absorbing solves with saddle_solver SCHUR, blob_rd_precond_build,
 * blob_rd_autotune; batched calls run box handles on their own streams, never in
 * the lock-step launches. */
#define BLOB_RD_BOUNDARY_PERIODIC 0
#define BLOB_RD_BOUNDARY_DIRICHLET 1

typedef struct blob_rd* blob_rd_t;

typedef struct {
    int32_t nx, ny, nz;      /* grid cells per axis; each >= 8; coarsening must reach <= 512 cells */
    double h;                /* grid spacing (> 0) */
    double D;                /* diffusion coefficient chi (> 0) */
    int32_t kernel_w;        /* 4 (Peskin four-point) or 3 (three-point) */
    int64_t n_blobs;         /* N >= 0 */
    const double* q;         /* device [N][3] positions */
    const double* kappa;     /* device [N] rates, or NULL (all zero) */
    int32_t precision;       /* BLOB_RD_FP64 | BLOB_RD_MIXED */
    int32_t schur_precond;   /* BLOB_RD_PRECOND_* (absorbing solves) */
    double rtol;             /* target relative residual (unweighted 2-norm), e.g. 1e-8 */
    int32_t max_iter;        /* outer iteration cap (CG or Schur GMRES), 0 = default */
    int32_t gmres_restart;   /* 0 = default 30 */
    int32_t inner_max_iter;  /* cap per inner Poisson solve, 0 = default */
    void* workspace;         /* device memory owned by the caller */
    size_t workspace_bytes;
    void* stream;            /* hipStream_t, NULL = default stream */
    int32_t saddle_solver;   /* BLOB_RD_SOLVER_*: how blob_rd_solve_absorbing solves (default Schur GMRES) */
    int32_t boundary;        /* BLOB_RD_BOUNDARY_*: periodic cell (default) or a box with fixed faces */
    double boundary_value;   /* c on the faces of a Dirichlet box (c_inf); ignored when periodic */
} blob_rd_params;

typedef struct {
    int32_t outer_iters;       /* CG iterations (reactive/step) or Schur GMRES iterations */
    int32_t inner_iters_total; /* inner CG iterations summed over Schur matvecs */
    int32_t vcycles;           /* multigrid V-cycles applied (the paper's cost proxy) */
    int32_t fallback;          /* 1 if the learned preconditioner was replaced by the plain one */
    int32_t refinements;       /* outer refinement passes (true FP64 residual checks that restarted) */
    double rel_resid;          /* true FP64 relative residual of the returned solution */
    double seconds;            /* wall time of the call */
    double alg_bytes;          /* algorithmic HBM bytes of the grid kernels launched */
} blob_rd_stats;

/* Bytes of device workspace needed for these parameters (0 on invalid parameters). */
size_t blob_rd_workspace_bytes(const blob_rd_params* p);

/* Validate parameters, place blobs on the grid (wrap, kernel weights, tile
 * binning: one pass of kernels on the stream), build the multigrid hierarchy
 * and the dense coarsest-grid (pseudo-)inverse. q and kappa are copied into
 * the workspace, so the caller may free them afterwards. The workspace must
 * stay valid until blob_rd_destroy. Errors: EINVAL (dims < 8, a level that
 * cannot coarsen to <= 512 cells, kernel_w not 3/4, h or D not positive,
 * N < 0, an unknown boundary, a non-finite boundary_value, a blob closer than
 * 3h to a face of a Dirichlet box), ENOMEM (workspace too small), EDEVICE. */
int blob_rd_create(const blob_rd_params* p, blob_rd_t* out);

/* Release the host handle (the caller frees the workspace). NULL is accepted. */
int blob_rd_destroy(blob_rd_t h);

/* Reactive system (eqs. unsteady_system, steady_state):
 *   (alpha I - D L + S kappa J) c = f,   alpha >= 0.
 * c: on entry the initial guess, on exit the solution. Multigrid-
 * preconditioned CG (Sec. III.E, eq. Pinv_Poisson); for alpha = 0 the
 * constant mode is corrected exactly. ESINGULAR if alpha = 0 and
 * sum(kappa) = 0. */
int blob_rd_solve_reactive(blob_rd_t h, double alpha, const double* f, double* c,
                           blob_rd_stats* stats);

/* Absorbing (diffusion-limited) saddle point (eq. saddle_point with
 * zeta = 1, xi = 1/dV_f):
 *   (alpha I - D L) c + S lambda = f,   J c = 0.
 * Schur-complement GMRES(restart) on J (alpha I - D L)^+ S (eqs. c_exact,
 * r_schur) with inner multigrid-preconditioned CG solves; for alpha = 0
 * the periodic null space is handled as in Appendix A (sum(lambda) =
 * h^3 sum(f), mean-zero fluctuation, mean concentration recovered from the
 * constraint). c (grid) and lambda (N) are outputs. EINVAL if N = 0.
 * With saddle_solver = BLOB_RD_SOLVER_BLOCK(_LEARNED) the handle solves the
 * same system by the paper's block FGMRES instead (as
 * blob_rd_solve_absorbing_fgmres, with its basis in the handle's workspace). */
int blob_rd_solve_absorbing(blob_rd_t h, double alpha, const double* f, double* c,
                            double* lambda, blob_rd_stats* stats);

/* One backward-Euler step (eq. c_np1) of dc/dt = D L c - S kappa J c + f:
 *   (I/dt - D L + S kappa J) c^{n+1} = c^n/dt + f.
 * c: c^n on entry, c^{n+1} on exit (warm-started from c^n). */
int blob_rd_step(blob_rd_t h, double dt, const double* f, double* c, blob_rd_stats* stats);

/* One backward-Euler step of a diffusion-limited (absorbing) suspension:
 * eq. c_np1 without the reaction term, with the blob sinks fixed by the
 * constraint of eq. saddle_point at finite dt (Sec. III.C, A = I/dt - D L
 * invertible, no null space):
 *   (I/dt - D L) c^{n+1} + S lambda = c^n/dt + f,   J c^{n+1} = 0.
 * Solved like blob_rd_solve_absorbing with alpha = 1/dt (Schur GMRES on
 * J A^{-1} S, eqs. c_exact and r_schur). c: c^n on entry, c^{n+1} on exit.
 * lambda: N sink strengths, written on exit; with warm != 0 its entry values
 * (say the previous step's multipliers) are GMRES's initial guess, with
 * warm = 0 they are ignored and GMRES starts from zero. On a handle with
 * saddle_solver = BLOB_RD_SOLVER_BLOCK(_LEARNED) the step is solved by the
 * block FGMRES started from (c^n, lambda or zero). stats->rel_resid is
 * measured against g = c^n/dt + f. Errors: EINVAL (null pointer, dt not
 * positive and finite, N = 0), ENOTCONV, ENUMERIC, EDEVICE. */
int blob_rd_step_absorbing(blob_rd_t h, double dt, const double* f, double* c, double* lambda, int warm,
                           blob_rd_stats* stats);

/* Message for the last failure on the calling thread (never NULL). */
const char* blob_rd_last_error(blob_rd_t h);

/* ---- Operator-level entry points (same handle, same stream rules) ---- */

/* lambda_out[i] = (J c)_i (Sec. III.A local averaging). */
int blob_rd_interp(blob_rd_t h, const double* c, double* out);

/* out = S lambda (Sec. III.A spreading, S = h^-3 J^T); overwrites out. */
int blob_rd_spread(blob_rd_t h, const double* lambda, double* out);

/* y = (alpha I - D L + S kappa J) x (with_blobs = 1) or (alpha I - D L) x (0). */
int blob_rd_apply(blob_rd_t h, double alpha, int with_blobs, const double* x, double* y);

/* z = one multigrid V(2,2) cycle for alpha I - D L applied to r from a zero
 * initial guess, in the handle's precision (Sec. III.E, eq. Helmholtz). No
 * mean projection is applied. */
int blob_rd_vcycle(blob_rd_t h, double alpha, const double* r, double* z);

/* ---- The paper's own saddle-point solver ----
 *
 * Sec. III.E (diffusion-limited case) and the appendix on preconditioning the
 * saddle-point solver: a Krylov method on the whole block system
 *   [alpha I - D L, S; J, 0] [c; lambda] = [f; 0]
 * (eq. saddle_point with zeta = 1), preconditioned by an approximate solve of
 * the same system through the Schur complement M = J A^{-1} S (eqs. c_exact,
 * r_schur). One preconditioner application on [vg; vf]:
 *   1. c* = n multigrid cycles on A c = vg - lbar S 1 (zero initial guess);
 *   2. lam~ from J c* - vf: the diagonal variant scales it by D/gamma
 *      (eq. Schur_diagonal, gamma = 1/(4 pi a0)); the approximate-Schur
 *      variant runs m GMRES iterations (modified Gram-Schmidt, zero guess) on
 *      (J A1^{-1} S) lam~ = J c* - vf, A1^{-1} one multigrid cycle (eq.
 *      approx_Schur); the learned variant runs the same iterations on
 *      (J A1^{-1} S P W P) y = J c* - vf and takes lam~ = P W P y, W the
 *      learned sparse approximation of the inverse Schur complement (below);
 *   3. c = c* + n cycles of the stationary iteration on A c = vg - lbar S 1 -
 *      S lam~, started at c*;
 *   4.-5. for alpha = 0 only (A singular on the periodic grid): lbar =
 *      h^3 sum(vg) / N, the blob mean projected out of J c* - vf, of every
 *      inner product and of lam~, c shifted by the blob mean of vf - J c, and
 *      lambda = lam~ + lbar; for alpha > 0 lbar = 0 and these steps are skipped.
 * The multigrid cycles are the handle's V(2,2) cycles in its precision. The
 * outer solver is flexible GMRES (right preconditioned, the preconditioned
 * directions kept, restarted, modified Gram-Schmidt) on the concatenated
 * [grid; blob] vectors with unweighted 2-norms, from a zero initial guess; it
 * stops when the true FP64 residual |b - K x| recomputed at a restart is
 * <= rtol |b|. */
#define BLOB_RD_SADDLE_DIAGONAL 0     /* lam~ = (D/gamma)(J c* - vf) */
#define BLOB_RD_SADDLE_APPROX_SCHUR 1 /* m inner GMRES iterations, one cycle per product (right-
                                         preconditioned by B of a coarse level built for alpha) */
#define BLOB_RD_SADDLE_LEARNED 2      /* approximate-Schur variant whose inner GMRES is right-
                                         preconditioned by the handle's learned W (alpha = 0; otherwise,
                                         or without a built W, the plain variant, stats->fallback = 1),
                                         or by the two-level B around W when a Fourier coarse level is
                                         built for alpha (blob_rd_coarse_build) */

typedef struct {
    int32_t precond; /* BLOB_RD_SADDLE_* */
    int32_t m;       /* inner GMRES iterations of the approximate-Schur variant; 0 = 5; <= gmres_restart */
    int32_t n;       /* multigrid cycles per approximate Poisson solve; 0 = 1; <= 64 */
    int32_t restart; /* FGMRES restart length; 0 = 30; <= 1024 */
    int32_t maxit;   /* total FGMRES iterations; 0 = 1000 */
    double rtol;     /* relative residual target; 0 = the handle's rtol */
    double diag;     /* D/gamma of the diagonal variant; 0 = 4 pi a0 D with a0 = 1.255 h for the
                        four-point kernel, 0.885 h for the three-point one (Sec. IV.A) */
} blob_rd_saddle_opts;

/* Device bytes of the caller's FGMRES workspace for this handle and restart
 * length (0 = 30): 2 restart + 1 long vectors of ncell + N doubles, the
 * Hessenberg matrix and rotations. 0 if h is NULL or restart > 1024. */
size_t blob_rd_fgmres_workspace_bytes(blob_rd_t h, int restart);

/* Solve the absorbing saddle point with the solver above (opts NULL = the
 * approximate-Schur variant with m = 5, n = 1, restart 30). c (grid) and
 * lambda (N) are outputs. workspace: device memory, 256-byte aligned, at least
 * blob_rd_fgmres_workspace_bytes(h, restart) bytes, caller-owned; its contents
 * are overwritten. Grid scratch comes from the handle's workspace. stats:
 * outer_iters = FGMRES iterations, inner_iters_total = inner GMRES iterations,
 * vcycles = multigrid cycles (the paper's cost measure), refinements = restarts,
 * rel_resid = the true FP64 relative residual. Errors: EINVAL (null pointer,
 * N = 0, alpha < 0, bad options, misaligned workspace), ENOMEM (workspace too
 * small), ENOTCONV (maxit reached, or two restarts in a row that cut the true
 * residual by less than 1 %: rtol below its rounding floor), ENUMERIC, EDEVICE. */
int blob_rd_solve_absorbing_fgmres(blob_rd_t h, double alpha, const blob_rd_saddle_opts* opts, const double* f,
                                   double* c, double* lambda, void* workspace, size_t workspace_bytes,
                                   blob_rd_stats* stats);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc and the like):
 * blob_rd_solve_absorbing_fgmres with the flexible-GMRES basis in a device
 * array of the library instead of a caller workspace. The array holds
 * BLOB_RD_NOALLOC_BYTES (256 MiB) on each GPU the library runs on, in each
 * process, from the load of the library's device code until the process ends;
 * its address is taken once per device by blob_rd_create. Same arguments and
 * results as blob_rd_solve_absorbing_fgmres otherwise; the call allocates and
 * frees nothing. Limit: blob_rd_fgmres_workspace_bytes(h, restart) <=
 * BLOB_RD_NOALLOC_BYTES (for instance 64^3 cells with restart 30), else ENOMEM
 * before any work. The array is shared by every call on that GPU: calls from
 * one process are serialised by a lock, and each call synchronises the handle's
 * stream before returning, so its contents (the last call's basis) never carry
 * over; overlapping use from outside these calls would race. EINVAL also when
 * alpha would evict a cached coarse inverse whose captured CG graphs it would
 * have to free (solve with one of the handle's last four alphas). */
#define BLOB_RD_NOALLOC_BYTES (256u << 20)
int blob_rd_solve_absorbing_fgmres_noalloc(blob_rd_t h, double alpha, const blob_rd_saddle_opts* opts,
                                           const double* f, double* c, double* lambda, blob_rd_stats* stats);

/* One application of the preconditioner above: [zg; zl] ~ K^{-1} [vg; vf]
 * (grid vectors of ncell doubles, blob vectors of N doubles, device pointers;
 * vg, vf are not modified and must not alias zg, zl). Synchronises the
 * handle's stream. Errors: EINVAL (null pointer, N = 0, alpha < 0, bad
 * options), EDEVICE. */
int blob_rd_saddle_precond(blob_rd_t h, double alpha, const blob_rd_saddle_opts* opts, const double* vg,
                           const double* vf, double* zg, double* zl);

/* ---- Learned Schur preconditioner ----
 *
 * The paper preconditions the Schur complement M = J A^+ S with the diagonal
 * M^{-1} ~ chi gamma^{-1} I, gamma ~ (4 pi a)^{-1} (Sec. III.E, eq.
 * Schur_diagonal). The learned preconditioner keeps that diagonal (a0 =
 * 1.255 h, the averaged reactive radius of Sec. IV.A) and adds a symmetric
 * pairwise correction for blob pairs closer than r_c = 12 h:
 *   W_ij = D h [delta_ij 4 pi a0/h + (g(i,j) + g(j,i))/2],
 * g a 12 -> 64 -> 64 -> 1 SiLU network of pair features
 *   [d/r_c (3), |d|/r_c, frac(q_i/h - 1/2) (3), frac(q_j/h - 1/2) (3), nu_i/4, nu_j/4]
 * (d the minimum-image separation, nu_i the number of other blobs within
 * r_c/2 of blob i: the pair's surroundings), bfloat16 weights with float32
 * accumulation. GMRES applies z = P W P r as a right preconditioner on
 * steady (alpha = 0) absorbing solves when schur_precond = LEARNED.
 * Training minimises (1/S) sum_s |P W y_s - x_s|^2/|x_s|^2 over sample pairs
 * (x_s, y_s = P M P x_s) from blob_rd_schur_apply, with Adam.
 *
 * Parameters are one float32 vector of BLOB_RD_NET_PARAMS values:
 * [W1 (64 x 12, row = output unit) | b1 (64) | W2 (64 x 64) | b2 (64) | w3 (64) | b3]. */
#define BLOB_RD_NET_PARAMS 5057

typedef struct blob_rd_net* blob_rd_net_t;

/* Device bytes a network object needs (weights, Adam moments, gradient, per-wave partials). */
size_t blob_rd_net_workspace_bytes(void);
/* Network object on caller-owned device memory; parameters start at zero. */
int blob_rd_net_create(void* workspace, size_t bytes, void* stream, blob_rd_net_t* out);
int blob_rd_net_destroy(blob_rd_net_t net);
/* Copy parameters from a device float32 vector; resets the Adam moments, the step count and the gradient. */
int blob_rd_net_set_params(blob_rd_net_t net, const float* params);
int blob_rd_net_get_params(blob_rd_net_t net, float* params);  /* device float32 [BLOB_RD_NET_PARAMS] */
int blob_rd_net_zero_grad(blob_rd_net_t net);
int blob_rd_net_get_grad(blob_rd_net_t net, float* grad);      /* device float32 [BLOB_RD_NET_PARAMS] */
/* One Adam step (Kingma and Ba 2015, beta1 0.9, beta2 0.999, eps 1e-8) with the accumulated gradient. */
int blob_rd_net_adam_step(blob_rd_net_t net, float lr);

/* Build the pair list of the handle's blobs and evaluate W with the current
 * network into caller-owned device memory `buf`. With buf == NULL only the
 * required size is returned in *needed (this counts the pairs on the GPU).
 * The buffer must stay valid while the handle uses the preconditioner.
 * Non-finite entries mark the preconditioner unusable: solves then run
 * without it and report stats.fallback = 1. */
int blob_rd_precond_build(blob_rd_t h, blob_rd_net_t net, void* buf, size_t bytes, size_t* needed);
/* z = P W P r (N-vectors, device). */
int blob_rd_precond_apply(blob_rd_t h, const double* r, double* z);
/* ---- The handle's own network ----
 *
 * A periodic handle with at least one blob created with schur_precond =
 * BLOB_RD_PRECOND_LEARNED or saddle_solver = BLOB_RD_SOLVER_BLOCK_LEARNED owns
 * a network (its parameters, Adam moments and gradient) and room for W in its
 * workspace (blob_rd_workspace_bytes counts both: about 20 MB for the network
 * plus 20 B per pair for up to BLOB_RD_LEARNED_ROW_CAP pairs per blob on
 * average). Its network starts untrained (zero parameters: W is the
 * diagonal above), and blob_rd_create builds that W (ENOMEM there when the
 * blobs have more pairs than the room). The three calls below act on that network and keep the
 * handle's W built from it; other handles return EINVAL. blob_rd_precond_build
 * with another network still replaces W (in the caller's buffer). */
#define BLOB_RD_LEARNED_ROW_CAP 256

/* The network's inference weights as one host byte blob, little endian:
 * W1 bfloat16 [64][12] | b1 float32 [64] | W2 bfloat16 [64][64] | b2 float32 [64] |
 * w3 bfloat16 [64] | b3 float32, packed without padding (10372 bytes). */
#define BLOB_RD_PRECOND_BLOB_BYTES 10372

/* Set the handle's network from a weight blob (host memory, bytes =
 * BLOB_RD_PRECOND_BLOB_BYTES; the weights become the float32 masters exactly),
 * reset its Adam state and build W (pair list of the handle's blobs, network
 * evaluated on the GPU). Non-finite weights give a W that solves never use
 * (stats.fallback = 1). Errors: EINVAL (null pointer, wrong size, a handle
 * without its own network), ENOMEM (more pairs than the reserved room), EDEVICE. */
int blob_rd_precond_set_weights(blob_rd_t h, const void* bf16_blob, size_t bytes);
/* Copy the handle's network out as a weight blob (host memory), its float32
 * masters rounded to bfloat16 (nearest, ties to even) where the blob holds bf16. */
int blob_rd_precond_get_weights(blob_rd_t h, void* bf16_blob, size_t bytes);

/* Sample pairs of one training step for one handle: rows x_s and y_s = P M P x_s
 * (M the handle's Schur complement, say from blob_rd_schur_apply), device
 * [n_samples][N] doubles, 1 <= n_samples <= 64 and 2 n_samples N + 64 <= cells. */
typedef struct {
    int32_t n_samples;
    const double* x;
    const double* y;
} blob_rd_train_batch;

/* One training step of the handle's network on the loss above: the loss and its
 * gradient over the batch (W built from the current weights), one Adam step
 * with learning rate lr (as blob_rd_net_adam_step), then W rebuilt from the new
 * weights. batch_desc points to a blob_rd_train_batch; *loss (host, may be NULL)
 * receives the loss before the step. Errors: EINVAL (null pointer, lr not
 * positive, bad batch, a handle without its own network), ENOMEM, EDEVICE. */
int blob_rd_precond_train_step(blob_rd_t h, const void* batch_desc, float lr, float* loss);

/* ---- Fourier coarse level of the Schur preconditioner ----
 *
 * The diagonal of eq. Schur_diagonal (Sec. III.E) and the learned W are local;
 * the long-wave modes of M = J (alpha I - D L)^+ S, whose eigenvalues grow
 * like (N/V)/(alpha + D |k|^2), are left to GMRES. The coarse level adds the
 * span of the lowest Fourier modes of the blob set,
 *   Z = [cos(k.q_i) - mean, sin(k.q_i) - mean],  k = 2 pi (m_x/L_x, m_y/L_y, m_z/L_z),
 * over the integer wave vectors 0 < |m|^2 <= m2max (one of each +-m pair;
 * m2max = 1, 2, 3, 6, 12, 16 give K = 6, 18, 26, 80, 178, 256 columns), and the Schur
 * GMRES of blob_rd_solve_absorbing and blob_rd_step_absorbing then applies
 * the balancing two-level preconditioner (Mandel 1993)
 *   B = Q + (I - Q M) W (I - M Q),   Q = Z E^{-1} Z^T,  E = Z^T M Z,
 * with W = P W_learned P when the handle uses the learned preconditioner at
 * alpha = 0 and otherwise the diagonal 4 pi a0 D I of eq. Schur_diagonal (a0 as
 * in blob_rd_saddle_opts.diag; P (4 pi a0 D) P at alpha = 0). B solves the coarse
 * modes exactly and keeps residuals orthogonal to them. This extends the
 * paper's Schur preconditioner; the paper has no coarse level.
 *
 * The block solver's learned variant (blob_rd_solve_absorbing_fgmres with
 * BLOB_RD_SADDLE_LEARNED) right-preconditions its inner GMRES on the one-cycle
 * Schur system with the same B (W = P W_learned P) instead of W alone; its
 * approximate-Schur variant (BLOB_RD_SADDLE_APPROX_SCHUR, and the block
 * handles' time steps) with B around the diagonal W, where it has no inner
 * preconditioner otherwise, when the level is built for the solve's alpha; the
 * diagonal variant never uses the level.
 *
 * Building costs K Schur products (inner multigrid-CG solves to inner_rtol)
 * and holds for the alpha given: solves at another alpha ignore it. */
#define BLOB_RD_COARSE_MAX_COLS 256

/* Device bytes blob_rd_coarse_build needs for m2max (about 32 K N bytes); 0 on
 * a bad argument (null handle, no blobs, m2max outside [1, 16]). */
size_t blob_rd_coarse_bytes(blob_rd_t h, int32_t m2max);
/* Build the coarse level for alpha into caller-owned device memory buf (at
 * least blob_rd_coarse_bytes; it must stay valid until blob_rd_coarse_clear,
 * a rebuild or blob_rd_destroy). inner_rtol = 0 means 1e-6. *ncols (host, may
 * be NULL) receives K. Synchronises the handle's stream. Errors: EINVAL (null
 * pointer, no blobs, a box handle, a handle in a batch, alpha < 0, inner_rtol
 * outside (0, 1), m2max outside [1, 16], K above N - 1 at
 * alpha = 0 or N otherwise), ENOMEM (buffer too small), ENUMERIC (E not
 * positive definite: the level stays unbuilt), EDEVICE. */
int blob_rd_coarse_build(blob_rd_t h, double alpha, int32_t m2max, double inner_rtol, void* buf, size_t bytes,
                         int32_t* ncols);
/* Drop the coarse level (the buffer is the caller's again). */
int blob_rd_coarse_clear(blob_rd_t h);
/* z = B r with the built coarse level (N-vectors, device, r != z), W as the solve
 * at the level's alpha would use it. EINVAL if nothing is built. */
int blob_rd_coarse_apply(blob_rd_t h, const double* r, double* z);

/* Copy the CSR of W (rows ascending, columns ascending) to device buffers; any may be NULL. */
int blob_rd_precond_csr(blob_rd_t h, int64_t* nnz, int32_t* rowptr, int32_t* col, double* val);
/* Loss over S sample pairs (X, Y device [S][N], rows x_s and y_s) and its
 * gradient, added into the network's gradient (computed with the network
 * the preconditioner was built from). *loss (host) receives the loss. */
int blob_rd_precond_loss_grad(blob_rd_t h, blob_rd_net_t net, const double* X, const double* Y, int32_t S,
                              double* loss);
/* y = P J (alpha I - D L)^+ S P x (P projects out the mean for alpha = 0;
 * identity otherwise): one Schur-complement product with an inner
 * multigrid-CG solve to relative tolerance inner_rtol (eq. r_schur). */
int blob_rd_schur_apply(blob_rd_t h, double alpha, const double* x, double* y, double inner_rtol);
/* y = P J A_n^{-1} S P x with A_n^{-1} n multigrid cycles from a zero guess in
 * the handle's precision (1 <= cycles <= 64): the Schur operator of eq.
 * approx_Schur that the inner GMRES of the paper's approximate-Schur
 * preconditioner applies (the learned W can be trained against it). */
int blob_rd_schur_apply_cycles(blob_rd_t h, double alpha, const double* x, double* y, int cycles);

/* ---- Batches of independent suspensions ----
 *
 * Solve n independent instances (each its own handle, created with its own
 * stream) concurrently: `threads` host workers take instances largest-first
 * and drive their solves, so the kernels and graph replays of different
 * instances overlap on the GPU. kind[i] = 0 reactive (c[i] initial guess in,
 * solution out; lambda[i] ignored), 1 absorbing (c[i], lambda[i] out). The
 * results are bitwise those of solving each instance alone. Returns the
 * first hard error, else BLOB_RD_ENOTCONV if any instance missed its
 * tolerance, else 0; stats (may be NULL) receives one entry per instance. */
int blob_rd_solve_streams(blob_rd_t* h, int32_t n, const int32_t* kind, double alpha, const double* const* f,
                          double* const* c, double* const* lambda, int32_t threads, blob_rd_stats* stats);

/* Lock-step batched form of the same. The CG iterations of the member
 * instances run as one sequence of batched launches (one launch per step,
 * e.g. one Gauss-Seidel half-sweep of one level, over a work list of every
 * member's work-group slices; a fixed grid strides over the list), captured
 * once as a HIP graph and replayed in rounds of two iterations on `stream`.
 * A member takes part in a round while it is in a CG run and drops out when
 * its done flag is set (a run may use one iteration past its limit). Each
 * instance's own solver logic (Schur GMRES, set-up, final solves) runs on a
 * host thread per instance and its handle's stream. Members: grids of at
 * most lockstep_max_cells cells (<= 0: no limit) whose finest levels are
 * launched per level and vectorizable (x edge divisible by 16 for FP32, 8 for
 * FP64) above a coarse tail, in the first member's precision; the other
 * instances run their whole solves on their own streams meanwhile, at most
 * `threads` at a time (0: all). Absorbing members whose handles solve by the
 * block FGMRES (saddle_solver BLOCK or BLOCK_LEARNED) hand the executor their
 * multigrid V-cycles instead: a second captured graph runs one V-cycle of every
 * member waiting for one (level-0 right side and first red sweep written by the
 * member on its own stream, ordered by an event), in rounds that start when
 * every such member still solving is waiting or 300 us after the first request
 * (environment BLOB_RD_VROUND_WAIT_US). The results are bitwise those of
 * solving each instance alone. workspace: caller-owned device memory of
 * blob_rd_batch_workspace_bytes(n) bytes (descriptors and work lists). */
size_t blob_rd_batch_workspace_bytes(int32_t n);
int blob_rd_solve_batched(blob_rd_t* h, int32_t n, const int32_t* kind, double alpha, const double* const* f,
                          double* const* c, double* const* lambda, int64_t lockstep_max_cells, int32_t threads,
                          void* workspace, size_t workspace_bytes, void* stream, blob_rd_stats* stats);

/* A batch handle: n_inst instances, each created from p[i] exactly as by
 * blob_rd_create (own workspace, stream, precision, solver), with the solve
 * kind[i] (0 reactive, 1 absorbing) that blob_rd_solve_batch runs on it. The
 * executor's descriptor tables live in member 0's workspace, which must hold
 * blob_rd_workspace_bytes(&p[0]) + blob_rd_batch_workspace_bytes(n_inst)
 * bytes (the tables take the tail). The executor runs on a stream of its own
 * (created here, default priority). A separate handle type keeps batch and
 * single-instance calls apart. Errors: EINVAL (bad kind, an absorbing
 * instance without blobs, any member's create error), ENOMEM, EDEVICE. */
typedef struct blob_rd_batch* blob_rd_batch_t;
int blob_rd_create_batch(const blob_rd_params* p, int32_t n_inst, const int32_t* kind, blob_rd_batch_t* out);
/* Destroys the members too. NULL is accepted. */
int blob_rd_destroy_batch(blob_rd_batch_t b);
/* Member i (owned by the batch: tune it, solve it alone, never destroy it), NULL if out of range. */
blob_rd_t blob_rd_batch_member(blob_rd_batch_t b, int32_t i);
/* Executor settings of blob_rd_solve_batch (lockstep_max_cells and threads as in
 * blob_rd_solve_batched); defaults 64^3 cells and 8 threads. */
int blob_rd_batch_set_executor(blob_rd_batch_t b, int64_t lockstep_max_cells, int32_t threads);
/* Steady solves (alpha = 0) of every member by the lock-step executor of
 * blob_rd_solve_batched: f[i], c[i] grid vectors of member i (c[i] the initial
 * guess of a reactive member), lambda[i] the multipliers of an absorbing member
 * (ignored for reactive ones; lambda may be NULL when no member is absorbing).
 * stats (may be NULL) receives one entry per member. Returns the first hard
 * error, else ENOTCONV if a member missed its tolerance, else 0. */
int blob_rd_solve_batch(blob_rd_batch_t b, const double* const* f, double* const* c, double* const* lambda,
                        blob_rd_stats* stats);

/* ---- Measurement ---- */

#define BLOB_RD_KERNEL_GS 0        /* one Gauss-Seidel half-sweep on the finest level */
#define BLOB_RD_KERNEL_STENCIL 1   /* FP64 operator apply y = alpha x - D L x (+ CG partial dots) */
#define BLOB_RD_KERNEL_RESTRICT 2  /* finest residual + full-weighting restriction */
#define BLOB_RD_KERNEL_PROLONG 3   /* trilinear prolongation + correction onto the finest level */
#define BLOB_RD_KERNEL_VCYCLE 4    /* one whole V-cycle (all levels) */
#define BLOB_RD_KERNEL_STENCIL_PLAIN 6 /* FP64 operator apply without the CG dots, the block solver's form */
#define BLOB_RD_KERNEL_STREAM 5    /* probe: out = a + b over three arrays of the finest half-level's size in the
                                      V-cycle precision, in the half-sweep's launch shape: the streaming ceiling of
                                      a launch that moves the half-sweep's bytes */
#define BLOB_RD_KERNEL_COLD 256    /* OR-ed flag: evict the last-level cache before each timed launch */

/* Launch one kernel of the solve path `reps` times back to back on the
 * handle's stream, bracketed by HIP events, on the handle's own workspace
 * buffers (their contents are overwritten). BLOB_RD_KERNEL_COLD asks for HBM
 * rather than last-level-cache bandwidth: the Gauss-Seidel and stencil
 * kernels then run back to back over independent buffer sets carved from the
 * handle's eight FP64 grid vectors (64 bytes per cell in all, more than the
 * 256 MB Infinity Cache from 160^3 cells), so each launch finds its data
 * evicted; the other kernels are each timed alone after >= 512 MB have been
 * streamed through the cache. avg_ms receives the mean time per launch and
 * bytes the algorithmic HBM bytes one launch must move (each input read once,
 * each output written once). On a Dirichlet-box handle the box forms of the
 * kernels are timed (same byte counts). */
int blob_rd_time_kernel(blob_rd_t h, int kernel, int reps, double* avg_ms, double* bytes);

/* ---- Launch-shape autotuning ----
 *
 * The multigrid kernels launched per level (Gauss-Seidel half-sweep,
 * residual, restriction, prolongation; the single-work-group coarse tail is
 * not tuned) take their work-group size from a per-handle table,
 * BLOB_RD_TUNE_KINDS entries per level, level-major, finest level first.
 * Every entry is one of 64, 128, 256, 512; the default is 256. The choice
 * changes timing only: each kernel updates every cell independently of how
 * cells are grouped, so solves are bitwise identical for any table. */
#define BLOB_RD_TUNE_KINDS 4

/* Number of levels with per-level launches for this handle's precision
 * (the table then has 4 * that many entries). */
int blob_rd_tune_levels(blob_rd_t h);

/* Copy the table out (n_entries >= 4 * levels) or replace it (every entry
 * validated, else BLOB_RD_EINVAL and nothing changes). Replacing it drops
 * the handle's captured graphs, which are captured again on next use. */
int blob_rd_get_tuning(blob_rd_t h, int32_t* table, int32_t n_entries);
int blob_rd_set_tuning(blob_rd_t h, const int32_t* table, int32_t n_entries);

/* Time every candidate work-group size of every tuned kernel on every
 * level (reps back-to-back launches each, HIP events on the handle's
 * stream, on the handle's workspace, whose contents are overwritten) and
 * keep the fastest; the default size stays unless another is at least 3%
 * faster. cache_path (NULL: the environment variable BLOB_RD_TUNE_CACHE,
 * if set; NULL and unset: no cache) names a JSON object file mapping
 * "<gfx arch>|<f32|f64>|<nx>x<ny>x<nz>|<gs|resid|restrict|prolong>" to a
 * work-group size, keyed by the level's own dimensions so that handles of
 * different sizes share entries. Levels whose four entries are all found
 * there are not timed; the newly timed ones are merged into the file
 * (written to a temporary file, then renamed). *timed (may be NULL)
 * receives the number of levels timed. Synchronises the handle's stream. */
int blob_rd_autotune(blob_rd_t h, int32_t reps, const char* cache_path, int32_t* timed);

#ifdef __cplusplus
}
#endif

#endif /* BLOB_RD_H */
