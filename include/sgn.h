/*
 * libsgn -- the hot path of a Fourier-spectral / GMRES solver of the 2D
 * Serre-Green-Naghdi (SGN) equations on one MI355X (gfx950) GPU, after
 * Gavrilyuk & Klein, "Numerical study of the Serre-Green-Naghdi equations in
 * 2D" (arXiv 2306.09731).
 *
 * The method (paper, Sections 2.2 and 3):
 *   state       depth h > 0 and the generalized velocity v = grad(phi)
 *   elliptic    L_h[sigma] = 3 sigma / h^3 - div(grad sigma / h) = -div v   (eq. (sigmav))
 *   evolution   h_t = -div(h v) + Laplacian(sigma)                           (eq. (1))
 *               v_t = -grad(|v|^2/2 - |grad sigma|^2/(2 h^2) + g h - 9/2 sigma^2/h^4)  (eq. (2), gradient form)
 *   space       Fourier collocation on the torus of periods 2 pi Lx x 2 pi Ly;
 *               derivatives are multiplications by i k
 *   solver      GMRES on M^-1 L sigma = M^-1 b, left preconditioner
 *               M = 3 + kx^2 + ky^2 (L at h = 1), warm-started from the last sigma
 *   time        classical explicit RK4; optional Krasny filter (zero DFT
 *               coefficients with modulus below a threshold)
 *   invariants  mass, momentum and energy (Section 2.3)
 *
 * Conventions shared by every call
 *   - Fields are DEVICE pointers owned by the caller: contiguous, row-major
 *     [ny][nx] (x contiguous), 256-byte aligned, of double in SGN_FP64 mode
 *     and of float in SGN_FP32_MIXED mode (hence void* in the signatures).
 *     Grid points are x_j = -pi Lx + j * 2 pi Lx / nx (same in y).
 *   - Wavenumbers are k = m / L, m in [-n/2, n/2), with the Nyquist mode of
 *     every derivative set to zero; the preconditioner uses the same k, with
 *     M = 3 / h_inf^3 + (kx^2 + ky^2) / h_inf (= 3 + k^2 for h_inf = 1).
 *   - The library never allocates device memory itself: all scratch lives in
 *     the caller's workspace (sgn_workspace_bytes).  It allocates a few bytes
 *     of pinned host memory for status read-back; sgn_rk4_step_graph also
 *     creates a stream, two events and up to two executable graphs per
 *     context (HIP runtime objects, released by sgn_destroy).
 *   - All work is ordered on the stream given to sgn_init.  The GMRES loop
 *     reads a status word back once per batch of speculative iterations, so
 *     the solving calls synchronise that stream before they return.
 *   - A context is not thread-safe; use one per stream.
 *   - Argument checks happen on the host before any launch.
 */
#ifndef SGN_H
#define SGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  SGN_OK = 0,
  SGN_ERR_INVALID_ARG = 1,   /* null or misaligned pointer, bad size, tol <= 0, ... */
  SGN_ERR_UNSUPPORTED = 2,   /* nx or ny not a power of two in [8, 4096], restart > 64 */
  SGN_ERR_HIP = 3,           /* HIP runtime error; see sgn_last_error */
  SGN_ERR_NOT_CONVERGED = 4, /* GMRES hit gmres_max_iters; outputs hold the last iterate */
  SGN_ERR_CAVITATION = 5,    /* min h <= 0 (the method assumes h > 0, Section 1) */
  SGN_ERR_NONFINITE = 6      /* NaN or Inf in the state */
};

/* Working precision (sgn_config.precision). */
enum {
  SGN_FP64 = 0,       /* everything in FP64 */
  SGN_FP32_MIXED = 1  /* fields, spectra, the Krylov basis, every FFT, the operator, the fluxes and the
                         RK4 combine in FP32; inner products and norms accumulated in FP64, and the
                         GMRES projections, Hessenberg matrix, Givens rotations and invariants in
                         FP64.  The GMRES tolerance is raised to at least 1e-6 (the attainable residual
                         of an FP32 operator); results agree with FP64 to about 1e-6 per call. */
};

/* Initial guess of the sigma solve in each RK4 stage (sgn_config.guess). */
enum {
  SGN_GUESS_PREVIOUS = 0,        /* the sigma of the previous RHS evaluation (Section 3) */
  SGN_GUESS_STAGE_INCREMENT = 1  /* that sigma plus the increment the same stage had over its
                                    predecessor in the previous step: sigma_i(n) ~ sigma_{i-1}(n)
                                    + [sigma_i(n-1) - sigma_{i-1}(n-1)].  The increments start at
                                    zero in each sgn_rk4_step call, so its first step is the same
                                    as SGN_GUESS_PREVIOUS; 4 extra fields of workspace. */
};

/* Problem and solver parameters.  Defaults in brackets (sgn_config_default). */
typedef struct sgn_config {
  int32_t nx, ny;          /* grid, powers of two in [8, 4096] */
  double Lx, Ly;           /* periods are 2 pi Lx, 2 pi Ly; box [-pi L, pi L) */
  double g;                /* gravity [1] (the paper sets g = h_inf = 1, Section 4) */
  double h_inf;            /* depth at infinity [1] */
  int32_t precision;       /* SGN_FP64 [default] or SGN_FP32_MIXED */
  int32_t gmres_restart;   /* restart length m [20], 1..64 */
  double gmres_tol;        /* stop when ||M^-1 (b - L s)|| <= tol ||M^-1 b|| [1e-10] */
  int32_t gmres_max_iters; /* total Arnoldi steps per solve [10 * restart] */
  int32_t batch;           /* ensemble members of one context [1], 1..SGN_MAX_MEMBERS (see below) */
  double krasny;           /* Krasny threshold on |DFT| / (nx ny) [0 = off; the paper uses 1e-12] */
  double invariants_tol;   /* GMRES tolerance of the sigma solve in sgn_invariants [1e-13] */
  int32_t dealias;         /* [0] 1: after every RK4 step also zero the modes with 3 |m_x| > nx or
                              3 |m_y| > ny (Orszag's two-thirds rule).  Not part of the paper's
                              scheme, which filters with the Krasny threshold only; it suppresses
                              the grid-scale aliasing growth that long runs of transversally
                              perturbed solitons develop with the Krasny filter alone. */
  int32_t guess;           /* SGN_GUESS_PREVIOUS [default] or SGN_GUESS_STAGE_INCREMENT; only the
                              starting iterate of GMRES depends on it, not the tolerance met */
} sgn_config;

/* Ensembles in one launch.  A context with batch = B > 1 holds B independent
 * members of the same configuration (grid, box, g, h_inf, precision, GMRES
 * parameters, filter, guess) and runs every kernel of a call once for all of
 * them (member index = blockIdx.z).  Its fields are B consecutive fields,
 * [B][ny][nx]; its workspace is B member workspaces; each member has its own
 * GMRES state, so members converge, restart and stop independently (a member
 * that has converged skips the launches of the others' further iterations).
 * The info / out arguments of sgn_elliptic_solve, sgn_rhs, sgn_rk4_step and
 * sgn_invariants then point to arrays of B entries, one per member; the
 * status returned is the first error of any member (NOT_CONVERGED if any
 * member did not converge).  Each member's results are bitwise those of a
 * context with batch = 1 on that member's fields.  Not available with
 * batch > 1: the captured step, the learned guess, the refined solve, the
 * autotuner and the host-thread ensemble calls (SGN_ERR_UNSUPPORTED). */
#define SGN_MAX_MEMBERS 64

typedef struct sgn_ctx sgn_ctx;

typedef struct sgn_solve_info {
  int32_t iters;            /* Arnoldi steps over all cycles */
  int32_t restarts;         /* completed cycles that did not converge */
  int32_t converged;        /* 1 if the stopping test was met */
  int32_t pad;
  double rel_resid_precond; /* ||M^-1 (b - L s)|| / ||M^-1 b|| at exit (GMRES estimate) */
  double rel_resid_true;    /* ||b - L s|| / ||b|| (computed by sgn_elliptic_solve only, else -1) */
} sgn_solve_info;

typedef struct sgn_step_info {
  int64_t total_iters;         /* Arnoldi steps over all solves */
  int32_t max_iters_per_solve;
  int32_t solves;              /* 4 per RK4 step */
  double min_h;                /* min h after the last step */
  int32_t any_unconverged;
  int32_t pad;
} sgn_step_info;

typedef struct sgn_invariants_out {
  double mass;          /* integral of (h - h_inf)                      (Section 2.3) */
  double px, py;        /* integral of h u, u = v - grad(sigma)/h        (Section 2.3) */
  double energy;        /* integral of h|u|^2/2 + 3 sigma^2/(2 h^3) + g (h - h_inf)^2 / 2 (Section 2.3) */
  double min_h, max_h;  /* extrema of h on the grid (Section 4.2 monitors the max) */
  double curl_l2;       /* L2 norm of d_x v_y - d_y v_x (zero for potential flows, Section 2.1) */
  double spectral_tail; /* largest |DFT(h)| / (nx ny) with |m_x| > nx/4 or |m_y| > ny/4 (Section 3) */
} sgn_invariants_out;

/* Fill *cfg with the defaults for an nx x ny grid on periods 2 pi Lx x 2 pi Ly. */
void sgn_config_default(sgn_config* cfg, int32_t nx, int32_t ny, double Lx, double Ly);

/* Bytes of device workspace sgn_init needs for cfg, or 0 if cfg is invalid.
 * Holds the twiddle tables, the Krylov basis ((restart + 1) fields), the
 * spectral scratch, the RK4 registers and the reduction scratch. */
size_t sgn_workspace_bytes(const sgn_config* cfg);

/* Validate cfg, lay out the caller's device workspace (ws, ws_bytes >=
 * sgn_workspace_bytes(cfg), 256-byte aligned), upload the twiddle tables
 * and the GMRES state, and return a context in *out.  hip_stream is a
 * hipStream_t (NULL = the default stream).  The workspace must outlive the
 * context.  Errors: SGN_ERR_INVALID_ARG, SGN_ERR_UNSUPPORTED, SGN_ERR_HIP. */
int sgn_init(const sgn_config* cfg, void* ws, size_t ws_bytes, void* hip_stream, sgn_ctx** out);

/* Free the host side of the context (the workspace stays the caller's). */
int sgn_destroy(sgn_ctx* ctx);

/* Solve L_h sigma = b (eq. (sigmav) with a given right-hand side) by
 * restarted left-preconditioned GMRES.  h, b: device fields; sigma: device
 * field, in = initial guess, out = solution.  info may be NULL.  Returns
 * SGN_ERR_NOT_CONVERGED (sigma = last iterate) if gmres_max_iters is hit. */
int sgn_elliptic_solve(sgn_ctx* ctx, const void* h, const void* b, void* sigma, sgn_solve_info* info);

typedef struct sgn_refine_info {
  int32_t rounds;            /* FP32 correction solves performed */
  int32_t inner_iters;       /* their GMRES iterations, summed */
  double rel_resid_first;    /* ||b - L sigma|| / ||b|| of the starting sigma (FP64) */
  double rel_resid_true;     /* the same for the returned sigma */
} sgn_refine_info;

/* Mixed-precision iterative refinement of the elliptic solve (the published
 * method of Wilkinson and Moler applied to eq. (sigmav) with a given b):
 * repeat r = b - L sigma (FP64, ctx64), stop when ||r|| <= tol ||b||,
 * solve L d = r in the mixed-precision mode (ctx32: FP32 transforms and
 * operator, FP64 reductions, its own tolerance of at least 1e-6, d from 0),
 * sigma += d (FP64).  ctx64 (SGN_FP64) and ctx32 (SGN_FP32_MIXED) describe
 * the same grid, box, g and h_inf on the current device.  h, b: FP64 device
 * fields; sigma: FP64 device field, in = initial guess, out = refined
 * solution.  Uses the checkpoint fields of ctx64's workspace as scratch;
 * synchronises both contexts' streams.  Returns SGN_ERR_NOT_CONVERGED after
 * max_rounds corrections without reaching tol (sigma = the last iterate),
 * SGN_ERR_INVALID_ARG / SGN_ERR_UNSUPPORTED for mismatched contexts. */
int sgn_elliptic_solve_refined(sgn_ctx* ctx64, sgn_ctx* ctx32, const double* h, const double* b, double* sigma,
                               double tol, int32_t max_rounds, sgn_refine_info* info);

typedef struct sgn_refined_step_info {
  int64_t inner_iters;          /* FP32 GMRES iterations of the correction solves, summed */
  int64_t rounds;               /* correction solves, summed over the stage solves */
  int32_t solves;               /* 4 per RK4 step */
  int32_t max_rounds_per_solve;
  double max_rel_resid;         /* largest ||b - L sigma|| / ||b|| returned by a stage solve (FP64) */
  double min_h;                 /* min h after the last step */
} sgn_refined_step_info;

/* nsteps RK4 steps of sgn_rk4_step in FP64 (ctx64) whose stage solves are
 * mixed-precision iterative refinements (sgn_elliptic_solve_refined, ctx32
 * for the FP32 corrections): each stage forms b = -div v in FP64, refines
 * sigma from the previous stage's until ||b - L sigma|| <= tol ||b|| in the
 * FP64 residual (at most max_rounds corrections), and computes the fluxes,
 * the Bernoulli function, the RK4 combine and the per-step filter in FP64.
 * So the GMRES iterations run in FP32 while sigma and the state carry FP64
 * accuracy: the precision form's FP64 residual refinement inside the RK4
 * step.  h, vx, vy, sigma: FP64 device fields of ctx64's grid (in place;
 * sigma in = first warm start, out = last stage's sigma).  Contexts as for
 * sgn_elliptic_solve_refined, batch = 1.  Uses ctx64's Krylov-basis and
 * checkpoint fields as scratch; synchronises both streams.  Returns
 * SGN_ERR_NOT_CONVERGED (after finishing the steps) if a stage solve did not
 * reach tol in max_rounds corrections.  info may be NULL. */
int sgn_rk4_step_refined(sgn_ctx* ctx64, sgn_ctx* ctx32, double* h, double* vx, double* vy, double* sigma,
                         double dt, int32_t nsteps, double tol, int32_t max_rounds, sgn_refined_step_info* info);

/* One evaluation of the right-hand side of the (h, v) system (Section 3):
 *   b = -div v;  sigma = GMRES(L_h, b; x0 = sigma);
 *   dh = -div(h v - grad sigma);  dv = -grad B,
 *   B = |v|^2/2 - |grad sigma|^2/(2 h^2) + g h - 9/2 sigma^2/h^4.
 * sigma is in/out (warm start in, solution out).  dh, dvx, dvy: outputs. */
int sgn_rhs(sgn_ctx* ctx, const void* h, const void* vx, const void* vy, void* sigma, void* dh, void* dvx,
            void* dvy, sgn_solve_info* info);

/* nsteps classical RK4 steps of size dt, in place on (h, vx, vy) (Section 3).
 * sigma is in/out: the warm start of the first solve, and on return the sigma
 * of the last RHS evaluation; each solve starts from the previous one's
 * sigma.  With cfg.krasny > 0 the Krasny filter is applied to h, vx, vy
 * after every step.  info may be NULL. */
int sgn_rk4_step(sgn_ctx* ctx, void* h, void* vx, void* vy, void* sigma, double dt, int32_t nsteps,
                 sgn_step_info* info);

/* The same RK4 steps with each step replayed as one captured HIP graph, so
 * that a step costs no host round trips.  In a graph the solve of RK stage s
 * is a single GMRES cycle of budget[s] Arnoldi steps, each kernel predicated
 * on the device status and the device's iteration cap set to budget[s], so the
 * solve stops at convergence exactly as in sgn_rk4_step; a device counter
 * records any solve that reaches its budget unconverged.  Budgets: iter_budget
 * for every stage (1 <= iter_budget <= gmres_restart), or with iter_budget <= 0
 * automatic: per stage, the most iterations that stage needed in the
 * host-driven steps of the context so far (the first two steps of the first
 * call run host-driven to measure them), plus SGN_GRAPH_MARGIN (environment at
 * sgn_init, 0..4, default 0).  The steps run in chunks of 16 replays: each
 * chunk starts from a checkpoint of (h, vx, vy) and of the solver state carried
 * between steps (workspace), and ends with one status read; a chunk in which a
 * solve reached its budget is restored and redone host-driven, and automatic
 * budgets grow to what the redone steps needed.  Solves that need restarts
 * keep the rest of the call host-driven.  Results are bitwise those of
 * sgn_rk4_step with the same arguments.  The graphs are captured on a stream
 * private to the context, ordered after the work on the context's stream and
 * before work enqueued there later, and are cached per (h, vx, vy, dt,
 * budgets, launch shapes).  Kernel timing (sgn_kernel_timing) counts
 * host-driven launches only.  *replayed (may be NULL): the number of steps run
 * as graph replays (0 if the call ran host-driven).  Errors: as sgn_rk4_step;
 * SGN_ERR_INVALID_ARG for iter_budget > gmres_restart. */
int sgn_rk4_step_graph(sgn_ctx* ctx, void* h, void* vx, void* vy, void* sigma, double dt, int32_t nsteps,
                       int32_t iter_budget, sgn_step_info* info, int32_t* replayed);

/* Conserved quantities of Section 2.3 for the state (h, vx, vy): sigma is
 * first solved to cfg.invariants_tol from the guess in sigma (in/out), then
 * mass, momentum, energy, min/max h, ||curl v|| and the spectral tail of h are
 * reduced in FP64 and written to the host struct *out. */
int sgn_invariants(sgn_ctx* ctx, const void* h, const void* vx, const void* vy, void* sigma,
                   sgn_invariants_out* out);

/* Ensembles: nsteps RK4 steps of n independent contexts at once.  Context i
 * is ctxs[i] (own grid, precision, workspace and stream; the contexts must be
 * distinct) with its fields h[i], vx[i], vy[i], sigma[i] and step dt[i]; each
 * is advanced exactly as by sgn_rk4_step, on a host thread of its own, so that
 * the GPU runs the other contexts' kernels while one context's thread waits
 * for its GMRES status.  Give the contexts different streams for their work to
 * overlap.  A context may hold several members (cfg.batch > 1): its fields are
 * then [batch][ny][nx] and its infos the batch consecutive entries that follow
 * those of ctxs[0..i-1].  infos: NULL or (sum of the contexts' batch) entries.
 * Every context is run; the first non-OK status is returned. */
int sgn_rk4_step_ensemble(int32_t n, sgn_ctx* const* ctxs, void* const* h, void* const* vx, void* const* vy,
                          void* const* sigma, const double* dt, int32_t nsteps, sgn_step_info* infos);

/* The same, each context's steps run by sgn_rk4_step_graph (automatic
 * iteration budget) on its thread: no host round trip per solve, so the
 * contexts' kernels interleave more densely.  Results are bitwise those of
 * sgn_rk4_step_ensemble.  A context with a learned guess attached, or with
 * several members, is refused (SGN_ERR_UNSUPPORTED), as by
 * sgn_rk4_step_graph. */
int sgn_rk4_step_ensemble_graph(int32_t n, sgn_ctx* const* ctxs, void* const* h, void* const* vx, void* const* vy,
                                void* const* sigma, const double* dt, int32_t nsteps, sgn_step_info* infos);

/* Autotuner of the launch schedule: times a few GMRES solves of a synthetic
 * smooth problem with each Arnoldi schedule this grid supports (four kernels
 * with one transform chain per block; four kernels with two chains; the
 * three-kernel step), then, for the fastest, the column tile widths (the
 * widest tiles that keep 128, 256, 512 or 1024 blocks) and rows per row block
 * (64, 128 or 256 threads) that give a launch shape not yet timed, and, for
 * an ensemble context on the three-kernel step with 512 or 1024 points per
 * row, the radix of the members' two-chain row transforms (4 or 8 values per
 * thread); keeps the fastest for the context and caches the choice per (nx,
 * ny, precision, restart, members, device) for the process.  All choices compute the same
 * quantities (reductions may sum in another order).  Uses the context's RK4
 * stage buffers (their contents are overwritten) and its stream;
 * synchronises.  *chosen (may be NULL): the schedule, 0, 1 or 2 in the order
 * above. */
int sgn_autotune(sgn_ctx* ctx, int32_t* chosen);

/* The context's launch choices: out[0] the Arnoldi schedule (as above),
 * out[1] the column-tile block target, out[2] the row-block thread target,
 * out[3], out[4] row pairs per block of the single-chain and three-chain row
 * kernels, out[5], out[6] columns per tile of the single-chain and two-chain
 * column kernels (0: no such kernel at this size), out[7] the values per
 * thread of the members' two-chain row kernel (0: the default radix).
 * out: 8 host int32. */
int sgn_launch_shape(const sgn_ctx* ctx, int32_t* out);

/* ---- Learned initial guess (a network of the project, not of the paper) ----
 * The paper starts every GMRES solve from the previous sigma (Section 3).  The
 * learned guess corrects that warm start: with r0 = b - L sigma_prev (eq. (3))
 * the exact correction is L^-1 r0, and a network of SGN_CNN_LAYERS 3x3
 * periodic convolutions (32 channels, ReLU between layers, BF16 weights and
 * activations, FP32 accumulation on the matrix cores) predicts L^-1 r0 / |r0|
 * from the three channels r0 / |r0|, M^-1 r0 / |r0| and h - h_inf (|r0| the
 * RMS).  Fields here are FP32 device arrays; in3 is [H][W][3] (channels last),
 * targets and outputs are [H][W].  H and W are powers of two, W >= 32.
 * Parameters (host FP32, SGN_CNN_PARAMS values): per layer l the weights
 * w[tap][cout][cin] (9 x 32 x 32, tap = 3 ky + kx reading the input at
 * (y + ky - 1, x + kx - 1) modulo the grid), then the 32 biases; the unused
 * input channels (3..31) of layer 0 and output channels (1..31) of the last
 * layer are ignored and get zero gradient. */
#define SGN_CNN_LAYERS 6
#define SGN_CNN_PARAMS (SGN_CNN_LAYERS * (9 * 32 * 32 + 32))
typedef struct sgn_cnn sgn_cnn;

/* Workspace bytes for an H x W network context (weights, Adam moments,
 * activations, gradient buffers); 0 if H, W are unsupported. */
size_t sgn_cnn_workspace_bytes(int32_t H, int32_t W);
/* Lay out the caller's 256-byte aligned device workspace; weights start at
 * zero.  Work is ordered on hip_stream.  SGN_ERR_UNSUPPORTED for bad sizes. */
int sgn_cnn_init(int32_t H, int32_t W, void* ws, size_t ws_bytes, void* hip_stream, sgn_cnn** out);
int sgn_cnn_destroy(sgn_cnn* net);
/* Copy SGN_CNN_PARAMS host floats in (and reset the Adam state) or out; both synchronise. */
int sgn_cnn_set_params(sgn_cnn* net, const float* params);
int sgn_cnn_get_params(sgn_cnn* net, float* params);
/* out = network(in3), output channel 0 before rounding (stream-ordered). */
int sgn_cnn_forward(sgn_cnn* net, const float* in3, float* out);
/* Mean squared error of network(in3) against target and its gradients in all
 * parameters (grads: host, SGN_CNN_PARAMS floats, may be NULL; loss may be
 * NULL); synchronises when either is requested. */
int sgn_cnn_gradients(sgn_cnn* net, const float* in3, const float* target, float* grads, double* loss);
/* One training step: gradients as above, then Adam (Kingma & Ba, Algorithm 1;
 * beta1 0.9, beta2 0.999, eps 1e-8, step size lr) on the FP32 master weights. */
int sgn_cnn_train_step(sgn_cnn* net, const float* in3, const float* target, float lr, double* loss);
const char* sgn_cnn_last_error(const sgn_cnn* net);

/* Attach a network to a solver context (its grid: H = cfg.ny, W = cfg.nx), or
 * NULL to detach.  With a network, every solve of sgn_rk4_step starts from
 * sigma_prev + |r0| net(r0 / |r0|, M^-1 r0 / |r0|, h - h_inf) instead of the
 * warm start sigma_prev; GMRES then runs, unchanged, to the same tolerance
 * from the corrected guess.  record (device FP32, capacity slots of 4 H W floats, or
 * NULL): every solve of sgn_rk4_step writes one training sample into slot
 * (count mod capacity): the network input [H][W][3] of the warm start, then
 * the target (sigma - sigma_prev) / |r0| [H][W] with sigma the converged
 * solution.  Needs cfg.guess = SGN_GUESS_PREVIOUS (SGN_ERR_UNSUPPORTED
 * otherwise); the captured step (sgn_rk4_step_graph) refuses contexts with a
 * network or recorder attached.  Resets the recorded count. */
int sgn_learned_guess_attach(sgn_ctx* ctx, sgn_cnn* net, float* record, int32_t capacity);

/* Which RK stages' solves the attached network corrects: bit s of stage_mask
 * (s = 0..3) for stage s; the other stages start from the plain warm start
 * (the recorder, if attached, still records every solve).  Default 0xF (every
 * stage); 0x1 runs the network once per RK4 step.  Errors: SGN_ERR_INVALID_ARG
 * for a mask outside 0..15. */
int sgn_learned_guess_stages(sgn_ctx* ctx, int32_t stage_mask);

typedef struct sgn_fgmres_info {
  int32_t fgmres_iters;       /* flexible GMRES iterations (network applications) */
  int32_t fgmres_cycles;      /* restart cycles */
  int32_t gmres_iters;        /* iterations of the plain GMRES judge that follows */
  int32_t converged;          /* the judge's verdict at cfg.gmres_tol */
  double fgmres_rel_resid;    /* ||b - L sigma|| / ||b|| when the flexible solve stopped (its estimate) */
  double rel_resid_true;      /* ||b - L sigma|| / ||b|| of the returned sigma */
} sgn_fgmres_info;

/* The learned preconditioner: flexible GMRES (Saad's FGMRES, restart
 * gmres_restart / 2, at most 15) on L_h sigma = b (eq. (sigmav) with a given
 * b), right-preconditioned by the network: z_j = s net(v_j / s, M^-1 v_j / s,
 * h - h_inf) with s the RMS of v_j, the map the learned guess was trained as
 * (an approximation of L^-1 applied to a residual).  Arnoldi with two passes
 * of classical Gram-Schmidt on FP64 physical fields; the basis V and the
 * preconditioned directions Z share the Krylov fields of the workspace.  It
 * stops when its residual estimate reaches cfg.gmres_tol ||b||, after
 * max_iters network applications, or when a direction adds nothing (a
 * network output of zero); then plain GMRES (sgn_elliptic_solve, left
 * preconditioned by M) runs from the result to cfg.gmres_tol: the fallback
 * and the judge of the error.  net: attached to no other context, grid H =
 * cfg.ny, W = cfg.nx.  sigma: in = initial guess, out = solution.  FP64
 * contexts with batch = 1 only (SGN_ERR_UNSUPPORTED otherwise); synchronises
 * the stream.  Returns what the judge returns. */
int sgn_elliptic_solve_fgmres(sgn_ctx* ctx, sgn_cnn* net, const void* h, const void* b, void* sigma,
                              int32_t max_iters, sgn_fgmres_info* info);
/* Samples recorded since the last attach. */
int sgn_learned_guess_recorded(sgn_ctx* ctx, int64_t* count);

/* Building blocks of the hot path, exposed for testing.
 * sgn_derivative: out = d f / dx (axis 0) or d f / dy (axis 1) (Section 3: i k).
 * sgn_apply_operator: out = L_h s (eq. (3)), or M^-1 L_h s if precondition != 0.
 * sgn_apply_precond: out = M^-1 r (Section 3).
 * sgn_krasny_filter: the per-step spectral filter of f in place: Krasny threshold
 *   cfg.krasny (Section 3; 0 = none) and, if cfg.dealias, the two-thirds rule.
 * All fields are device pointers; out may not alias an input. */
int sgn_derivative(sgn_ctx* ctx, int32_t axis, const void* f, void* out);
int sgn_apply_operator(sgn_ctx* ctx, const void* h, const void* s, void* out, int32_t precondition);
int sgn_apply_precond(sgn_ctx* ctx, const void* r, void* out);
int sgn_krasny_filter(sgn_ctx* ctx, void* f);

/* For callers that cannot allocate device memory or create a context at call
 * time (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): sgn_apply_operator without a context or workspace.
 * out = L_h s, or M^-1 L_h s if precondition != 0, for the grid, box, h_inf
 * and precision of *cfg (the other fields must be valid but are unused;
 * batch must be 1).  h, s, out: device fields of cfg->nx x cfg->ny points as
 * for sgn_apply_operator (double, or float in SGN_FP32_MIXED), out not
 * aliasing h or s.  The work is enqueued on hip_stream (NULL: the null
 * stream) and the call returns without synchronising; launch errors are
 * reported.  Scratch: a fixed device array of the library, 256 KiB of
 * twiddle tables plus four fields of SGN_NOALLOC_MAX_POINTS doubles
 * (32.25 MiB per GPU, held from the first call on that GPU until the process
 * ends); the call allocates nothing.  Grids of more than
 * SGN_NOALLOC_MAX_POINTS points are refused with SGN_ERR_UNSUPPORTED before
 * any GPU work, with the reason in sgn_last_error(NULL).  Calls on one GPU
 * share its scratch: calls that overlap on one GPU (concurrent streams or
 * host threads) race and must be serialised by the caller.  Results match
 * sgn_apply_operator to rounding (its twiddle tables are computed on the
 * device instead of the host). */
#define SGN_NOALLOC_MAX_POINTS (1 << 20)
int sgn_apply_operator_noalloc(const sgn_config* cfg, const void* h, const void* s, void* out,
                               int32_t precondition, void* hip_stream);

/* Measurement support.  While timing is enabled for a kernel class, every
 * p-th launch of that class is bracketed by HIP events recorded on the
 * context stream, so its device time can be read without a profiler.
 * sgn_kernel_timing(ctx, kind, p) with p >= 1 clears the totals and starts
 * timing kind (one class at a time); (ctx, kind, 0) stops it.
 * sgn_kernel_time synchronises the stream and returns the number of launches
 * of the class while timing was on and their total duration in milliseconds:
 * the sum over the launches with events, times launches / launches with
 * events (p = 1: the measured sum).  Errors: SGN_ERR_INVALID_ARG for an
 * unknown kind or p < 0, SGN_ERR_HIP. */
enum {
  SGN_KERNEL_ROW_MATVEC = 0,     /* x part of the elliptic operator (Arnoldi step) */
  SGN_KERNEL_COL_BASIS = 1,      /* projection of the new vector + inverse y transforms */
  SGN_KERNEL_COL_PRECOND_DOT = 2,/* y part of the operator, M^-1, new basis vector, projections */
  SGN_KERNEL_GS_UPDATE = 3,      /* Gram-Schmidt update, norms, Givens */
  SGN_KERNEL_ROW_FLUX = 4,       /* x part of the fluxes + RK4 combine of v_x */
  SGN_KERNEL_COL_FLUX = 5,       /* y part of the fluxes + RK4 combine of h, v_y */
  SGN_KERNEL_COUNT = 6
};
int sgn_kernel_timing(sgn_ctx* ctx, int32_t kind, int32_t enable);
/* algo_bytes (may be NULL): algorithmic bytes (fields read and written once
 * each, FP64) of the timed launches that did work, i.e. excluding Arnoldi
 * steps the device skipped after convergence; counted for the Arnoldi
 * classes of the default (three-kernel) Arnoldi step. */
int sgn_kernel_time(sgn_ctx* ctx, int32_t kind, int64_t* launches, double* total_ms, double* algo_bytes);

/* Human-readable name of a status code, and the last error of a context
 * (ctx = NULL: of this thread's last failed call that takes no context). */
const char* sgn_status_string(int status);
const char* sgn_last_error(const sgn_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SGN_H */
