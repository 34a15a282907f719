/*
 * pfch.h - C ABI of libpfch, a gfx950 (MI355X) implementation of the
 * preconditioned Nesterov accelerated gradient descent (PAGD) solve inside
 * each fully implicit second-order step of the phase field crystal (PFC) and
 * functionalized Cahn-Hilliard (FCH) equations with periodic Fourier
 * collocation (Park, Salgado & Wise, arXiv 2204.07247).
 *
 * Conventions
 *  - All floating point is IEEE float64.  Fields are C-order real arrays
 *    [Ny][Nx] (2D) or [Nz][Ny][Nx] (3D) with x fastest; n[0] = Nx,
 *    n[1] = Ny, n[2] = Nz.
 *  - Field pointers passed to pfch_set_state, pfch_get_state and pfch_solve
 *    are DEVICE pointers to contiguous arrays of Nx*Ny doubles owned by the
 *    caller.  The library never keeps a caller pointer after a call returns.
 *  - All device work is ordered on the HIP stream given to pfch_create.
 *    Calls that report statistics synchronise that stream before returning.
 *  - Functions return PFCH_OK (0) or a negative error code; argument errors
 *    are detected on the host before any device work is queued.
 *  - One context per stream; calls on one context are not thread-safe.
 */
#ifndef PFCH_H
#define PFCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PFCH_VERSION 1

enum {
  PFCH_OK = 0,
  PFCH_E_INVAL = -1,       /* invalid argument or descriptor */
  PFCH_E_NOMEM = -2,       /* device or host allocation failed */
  PFCH_E_HIP = -3,         /* a HIP runtime call failed */
  PFCH_E_NOCONV = -4,      /* PAGD reached max_iter without ||d||_inf < tol */
  PFCH_E_NONFINITE = -5,   /* ||d||_inf became Inf or NaN */
  PFCH_E_PRECOND = -6,     /* averaged-Newton symbol not positive on some mode */
  PFCH_E_UNSUPPORTED = -7, /* valid but not supported (grid size, ndim) */
  PFCH_E_INTERNAL = -8,    /* internal inconsistency: a solve's stop record was not
                              final when read; no result is reported or accepted */
  PFCH_E_SCRATCH = -9      /* the grid needs more than the static scratch of
                              pfch_rhs_noalloc holds */
};

enum { PFCH_PFC = 0, PFCH_FCH = 1 };  /* model */
enum { PFCH_BDF2 = 0, PFCH_MP = 1, PFCH_LBDF2 = 2, PFCH_LMP = 3 };  /* time scheme */

/*
 * One simulation instance.  Model (Sec. 2 of the paper):
 *   PFC: E = int u^4/4 + (1-eps) u^2/2 - |grad u|^2 + (Delta u)^2/2
 *   FCH: E = int (eps^2 Delta u - F'(u))^2/2 - (eps^2 eta1 |grad u|^2/2 + eta2 F(u)),
 *        F(z) = (z+1)^2 ((z-1)^2/2 + (2/3) tau (z-2)) / 2
 * with d_t u = M Delta mu, M = mobility.  eta1 and eta2 are the
 * coefficients as they stand in the energy (e.g. 1.45 eps and 2 eps).
 * Scheme (Sec. 3.1): PFCH_BDF2 (variable-step BDF2, backward Euler on the
 * first step) or PFCH_MP (implicit midpoint), each solved by PAGD; or the
 * linear IMEX schemes PFCH_LBDF2 / PFCH_LMP (eq. eqn:FCH-semidis-simplicit
 * with the paper's splitting of the chemical potential: PFC
 * L = (1 + Delta)^2; FCH L = eps^4 Delta^2 - kappa2 Delta + kappa0,
 * kappa0 = 1 - 2 tau^2 + eta2, kappa2 = 1), one linear k-space solve per
 * step; for these s, eta, tol, theta_l and max_iter are not used, guess
 * must be 0 and the statistics report one iteration.
 * Solver (Alg. 2): step size s, friction sweep eta[0..n_eta-1] (one entry:
 * constant friction; n_eta = 0: no momentum, the preconditioned gradient
 * descent of Alg. 1), stop when ||d_i||_inf < tol, at most max_iter
 * iterations.  theta_l weights the
 * beta_0/beta_2/beta_4 part of the averaged-Newton preconditioner
 * (Sec. 3.4.1); 1.0 is the operator as printed.
 * guess: 0 = extrapolated initial guess u^n + rho (u^n - u^{n-1}) (Alg. 2
 * input x_0, extrapolation as in Sec. 3.1); 1 = learned guess when a network
 * is attached with pfch_set_fno (otherwise extrapolated).  reserved must be 0.
 * Grids: ndim = 2 with Nx, Ny powers of two in [8, 2048] or 192; ndim = 3
 * (PFC only) with Nx as in 2D and Ny, Nz in
 * {8, 16, 32, 64, 128, 192, 256}.  Other valid descriptors give
 * PFCH_E_UNSUPPORTED.
 */
typedef struct pfch_instance_desc {
  double len[3]; /* periods per axis, x first */
  double eps, eta1, eta2, tau, mobility;
  double s, tol, theta_l;
  double eta[8];
  int32_t model, scheme, ndim, n_eta, max_iter, guess;
  int32_t n[3]; /* points per axis, x first; n[2] ignored for ndim = 2 */
  int32_t reserved;
} pfch_instance_desc;

/* Per-instance result of one step or solve. */
typedef struct pfch_stats {
  double dnorm_inf; /* ||d||_inf of the last iteration (Alg. 2's stopping test) */
  double beta[4];   /* beta_-2, beta_0, beta_2, beta_4 used for this step */
  double mass;      /* mean of the accepted solution (NaN if not computed) */
  double rnorm_inf; /* ||r||_inf, r = -G'(x) of eq. obj:G' at the returned
                       solution x (the residual of the step problem, without
                       the preconditioner); NaN unless statistics detail 2 was
                       set and the solve converged; NaN for the IMEX schemes */
  double gain;      /* gain g of the learned correction fitted for this
                       step's guess (used if at least 0.98, else the
                       correction is left out; see pfch_set_fno); NaN unless
                       guess is 1 */
  int32_t iters;    /* PAGD iterations */
  int32_t fft_pairs;/* 2D transform pairs of real fields used (setup + iterations) */
  int32_t status;   /* PFCH_OK or the error of this instance */
  int32_t guess;    /* initial guess used: 0 extrapolated, 1 learned,
                       2 learned guess failed, step solved again from the
                       extrapolated guess */
} pfch_stats;

typedef struct pfch_ctx pfch_ctx; /* opaque; owned by the library */

/* Host-only check of a descriptor; needs no GPU.  Returns PFCH_OK,
 * PFCH_E_INVAL or PFCH_E_UNSUPPORTED. */
int pfch_validate_desc(const pfch_instance_desc* desc);

/* Create a context holding n_inst instances that advance together in each
 * pfch_step.  Each instance is one discrete problem of Sec. 3.2 (periodic
 * Fourier collocation of the model on its grid) stepped by the scheme of
 * Sec. 3.1 with the solver of Alg. 2; descs is a host array of n_inst
 * descriptors, copied.  `hip_stream` is a hipStream_t (NULL = default
 * stream).  All workspaces, transform tables and launch graphs are
 * allocated here and owned by the context; *out is NULL on error.  Errors:
 * PFCH_E_INVAL / PFCH_E_UNSUPPORTED for a descriptor pfch_validate_desc
 * rejects, PFCH_E_NOMEM, PFCH_E_HIP.  The initial state of every instance is
 * undefined until pfch_set_state. */
int pfch_create(const pfch_instance_desc* descs, int32_t n_inst, void* hip_stream,
                pfch_ctx** out);

/* Set the step history of instance `inst`: the data a multistep scheme
 * needs to take its next step (Sec. 3.1; the inputs u^n, u^{n-1} and the
 * previous step size of Alg. 3).  u^n (and u^{n-1}, or NULL when there is no
 * history yet, so that the next BDF2 step is backward Euler) are device
 * arrays of Nx*Ny(*Nz) doubles, copied; t, dt_prev (the step that produced
 * u^n, > 0, ignored when u_nm1 is NULL) and the step index n are host
 * values.  Discards a queued set-up and sets the gain of a learned
 * correction to 1.  PFCH_E_INVAL for a bad instance index or null u_n. */
int pfch_set_state(pfch_ctx* ctx, int32_t inst, const double* u_n, const double* u_nm1,
                   double t, double dt_prev, int32_t step_index);

/* Copy the step history of instance `inst` (u^n, u^{n-1}, t, the last step
 * size and the step index; Sec. 3.1 and Alg. 3) out to caller-owned device
 * arrays and host scalars; any pointer may be NULL.  u_nm1 is left untouched
 * when the instance has no history.  PFCH_E_INVAL for a bad instance
 * index. */
int pfch_get_state(pfch_ctx* ctx, int32_t inst, double* u_n, double* u_nm1, double* t,
                   double* dt_prev, int32_t* step_index);

/* Advance every instance by one step of size dt[i] (host array of n_inst).
 * Each step: coefficients (eq. obj:BDF2 / obj:MP), initial guess
 * u^n + rho (u^n - u^{n-1}) with rho = dt/dt_prev (u^n on the first step),
 * averaged-Newton constants at the guess, PAGD to ||d||_inf < tol.  An
 * instance whose solve fails keeps its state (the step is transactional per
 * instance); the return value is the first failing instance's code.
 * `st` is a host array of n_inst or NULL.  After a step whose sizes equal
 * the previous call's, the next step's set-up (with its learned guesses) is
 * already queued on the context's stream when this returns; a following
 * pfch_step with the same sizes uses it, any other call on the context that
 * changes its state discards it.  Results do not depend on this. */
int pfch_step(pfch_ctx* ctx, const double* dt, pfch_stats* st);

/* Solve one step problem of instance `inst` with caller-given coefficients
 * (a, b, c) of a u + b u^n + c u^{n-1} = M Delta mu(u_breve)
 * (eq. eqn:FCH-fulldis-implicit); u_breve follows the instance's scheme.
 * `x` holds the initial guess on entry and the solution on return (the last
 * iterate on PFCH_E_NOCONV).  u_nm1 may be NULL when c == 0.  The instance's
 * own state is not changed. */
int pfch_solve(pfch_ctx* ctx, int32_t inst, double a, double b, double c, const double* u_n,
               const double* u_nm1, double* x, pfch_stats* st);

/*
 * Adaptive time stepping (Sec. 3.1.2, Alg. 3), 2D grids and 3D PFC.
 *
 * One call is one pass of the loop body of Alg. 3 for every instance: a
 * tentative solve with step size res[i].dt_try, an error estimate ERR, the
 * decision, and the next tentative size.
 *   AM3 (eq. fml:AM3-high-sol, fml:AM3-err), rho = dt~/dt_n (0 on the first
 *   step, where the R(u^{n-1}) term drops):
 *     u^ = u^n + dt~/6 [(3+2rho)/(1+rho) R(u~) + (3+rho) R(u^n)
 *                       - rho^2/(1+rho) R(u^{n-1})],
 *     ERR = ||u~ - u^||_2 / ||u^||_2,  R(v) = M Delta mu(v).
 *   midAB2 (eq. fml:midAB2-high-sol, fml:midAB2-err): u^ is the quadratic
 *     through u^n, u^{n-1}, u^{n-2} at t_n + dt~ and
 *     ERR = ||u~ - u^|| / ||u^|| / (1 - 1/(24 R_n)),
 *     R_n = 1/24 + (1 + dt_n/dt~)(1 + 2 dt_n/dt~ + dt_{n-1}/dt~)/8;
 *     used once three solutions exist, AM3 before that.
 *   Accept when ERR <= tol or dt~ <= dt_min: u^{n+1} = u~, t += dt~.
 *   Next size (eqs. fml:time-step, fml:time-step-med):
 *     dt_try = max(dt_min, min(0.9 (tol/ERR)^(1/3) dt~, dt_max)),
 *   also after a rejection.  A tentative solve that fails counts as
 *   ERR = +inf (rejected, next size dt_min).
 * estimator: PFCH_EST_AUTO = midAB2 for PFCH_MP, AM3 otherwise.
 * The history the estimators need (u^{n-2}, R(u^n), R(u^{n-1}), dt_{n-1})
 * is kept by the context across pfch_step_adaptive calls; pfch_set_state
 * and pfch_step restart it from u^n, u^{n-1}.  Norm sums are taken in a
 * fixed order, so results do not depend on batching.
 * res: host array of n_inst; dt_try is read (> 0) and written.  Returns
 * PFCH_OK, or the solve's error code when an instance's solve failed at
 * dt~ <= dt_min (that instance cannot advance).
 */
enum { PFCH_EST_AUTO = 0, PFCH_EST_AM3 = 1, PFCH_EST_MIDAB2 = 2 };

typedef struct pfch_adapt_desc {
  double tol;     /* stepping tolerance TOL > 0 */
  double dt_min;  /* 0 < dt_min <= dt_max */
  double dt_max;
  int32_t estimator;
  int32_t reserved; /* must be 0 */
} pfch_adapt_desc;

typedef struct pfch_adapt_result {
  double dt_try;    /* in: tentative step size; out: the next one */
  double dt;        /* out: size of this attempt */
  double err;       /* out: ERR (+inf if the solve failed) */
  int32_t accepted; /* out: 1 = history advanced */
  int32_t estimator;/* out: PFCH_EST_AM3 or PFCH_EST_MIDAB2, as used */
  pfch_stats solve; /* out: the tentative solve */
} pfch_adapt_result;

int pfch_step_adaptive(pfch_ctx* ctx, const pfch_adapt_desc* a, pfch_adapt_result* res);

/* R(v) = M Delta mu(v) (the right-hand side of the PDE, Sec. 2) of instance
 * `inst`'s model on its grid, v and out device arrays of Nx*Ny (3D:
 * Nx*Ny*Nz) doubles (may not alias).  Uses the instance's transform
 * workspace; its state is not changed. */
int pfch_rhs(pfch_ctx* ctx, int32_t inst, const double* v, double* out);

/* Allocation-free variant of pfch_rhs, for callers that cannot allocate or
 * synchronise (code under HIP graph capture, tight serving loops).  Same
 * arguments and result, bitwise, as pfch_rhs; it allocates nothing, makes
 * no runtime look-up and does not synchronise: the result is ready in
 * stream order on the context's stream.  Its spectral workspace is a static
 * device array of 32 MiB (plus 256 bytes for the source and destination
 * pointers) that each device holds until the process ends; grids needing
 * more (PFC: 2 fields, FCH: 3 fields of Ny*Nx/2 complex doubles, e.g. FCH
 * beyond 1024 x 1024 points) give PFCH_E_SCRATCH.  Unlike pfch_rhs it
 * leaves the context's workspaces untouched (a queued set-up is kept).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (on different streams, or from different contexts) race, and
 * the caller must order them.  2D only (PFCH_E_UNSUPPORTED for 3D);
 * PFCH_E_INVAL for a bad instance, null or aliasing v and out. */
int pfch_rhs_noalloc(pfch_ctx* ctx, int32_t inst, const double* v, double* out);

/* Statistics detail of pfch_step, pfch_step_adaptive and pfch_solve when
 * st != NULL: 0 = iterations, status and ||d||_inf only (read from the
 * convergence records, no extra synchronisation); 1 (default) = also beta
 * and the mass of the accepted solution (one extra reduction and
 * synchronisation per step); 2 = also ||r||_inf of each converged solution
 * (one more evaluation of the residual per instance: the set-up and one
 * iteration of the solver's kernels with the identity in place of the
 * preconditioner, and one synchronisation per instance). */
int pfch_set_stats_detail(pfch_ctx* ctx, int32_t detail);

/* Kernel timing for measurement.  Solves `reps` times the step of size dt
 * from instance 0's current state (as pfch_step would, launching the same
 * iteration kernels in the same order, without accepting the result), with a
 * HIP start/stop event pair attached to every iteration-kernel launch
 * (hipExtLaunchKernel).  out[k] = average microseconds of the k-th iteration
 * kernel over the launches that did an iteration's work: 2D {column, row,
 * 0, 0}; 3D {y forward, z, y inverse, row}.  Then solves it `reps` times
 * more with one event before the first launch and one after the last
 * iteration in which every instance worked: out[4] = microseconds per
 * iteration of that chain of launches (no per-launch events; the gaps
 * between launches included).  The instance's state (u^n, u^{n-1}, t, step
 * index) is not changed; its iteration workspaces are. */
int pfch_time_kernels(pfch_ctx* ctx, double dt, int32_t reps, double out[5]);

/* The same timing for the grouped launches of every instance of `inst`'s
 * group (instances of one model, scheme and grid share each iteration-kernel
 * launch in pfch_step): the grouped launch as the solve runs it, an event
 * pair on each launch; averages over the iterations in which every member
 * still worked.  The members' states are not changed; their iteration
 * workspaces are. */
int pfch_time_group(pfch_ctx* ctx, int32_t inst, double dt, int32_t reps, double out[5]);

/* Kernel timing with HIP events: sets up one step of instance 0 (as
 * pfch_step would), then launches each iteration kernel `reps` times back
 * to back on the context's stream (every launch doing an iteration's full
 * work) with one event pair around each batch.  out as for
 * pfch_time_kernels.  Back-to-back launches of one kernel find the caches
 * warm from its previous launch, unlike the solve.  The instance's state is
 * not changed; its iteration workspaces are. */
int pfch_time_kernels_events(pfch_ctx* ctx, double dt, int32_t reps, double out[4]);

/* Launch geometry of instance `inst` for reporting: {row grid, row block,
 * row LDS bytes, column grid, column block, column LDS bytes}. */
int pfch_get_launch_config(pfch_ctx* ctx, int32_t inst, int64_t out[6]);

/*
 * Learned initial guess: a Fourier neural operator (FNO) in float32.
 *
 * The network maps (u^n, u^{n-1}) to a correction of the extrapolated guess:
 *   input  x[0] = (u^n - mu)/su,  x[1] = (u^n - u^{n-1})/sd
 *   guess  x_0 = u^n + rho (u^n - u^{n-1}) + g so * Pi_0 y
 * where Pi_0 removes the mean (the PAGD solve keeps the mean of its initial
 * guess, so the mass stays that of the extrapolation), norm = {mu, su, sd,
 * so}, and g is the instance's gain on the correction: 1 after
 * pfch_set_state or pfch_set_fno; after each pfch_step that took the learned
 * guess and accepted the solution x it reached, the least-squares gain of
 * that step's correction c = so Pi_0 y against x - (u^n + rho (u^n -
 * u^{n-1})), clamped to [0, 1], is the next guess's g (steps of
 * pfch_step_adaptive leave g as it is); a fitted gain below 0.98 (the
 * correction over-predicts the solutions) is applied as 0, the correction
 * left out.  pfch_stats.gain reports the fitted gain.  Gate: when a
 * pfch_step fitted a gain below 0.98, or when its learned guess was
 * replaced (guess 2), the instance takes the extrapolated guess, with no
 * network call, for the next 16 << min(f, 3) accepted fixed-size steps
 * (f: probes in a row that closed the gate again); then two probe steps
 * use the network again (the first with gain 0, the second with the gain
 * fitted to the first, which reopens or closes the gate).  pfch_set_state
 * and pfch_set_fno open the gate.  PAGD still iterates to
 * ||d||_inf < tol from this guess, so the
 * solution differs from the extrapolated-guess solution only within that
 * tolerance; a guess from which the solve fails is replaced by the
 * extrapolated one.
 *
 * Network: lift 2 -> W channels, L spectral layers
 *   z = K v + W_l^T v + b_l,  v <- gelu(z) (no gelu after the last layer),
 * K keeping kx in [0, M) and, on y (and z in 3D), k in {0..M-1} U
 * {N-M..N-1} of the real transform with complex per-mode channel mixing,
 * then projection W -> 1.
 * Flat float32 parameter vector, in order: P[2][W], pb[W], per layer
 * R[W][W][modes][re, im] with modes [2M][M] (2D: ky, kx) or [2M][2M][M]
 * (3D: kz, ky, kx; index ki >= M on a full axis holds k = N - 2M + ki),
 * Wl[W][W], bl[W]; then Q[W], qb.  All fields are [B][C][Ny][Nx] (2D) or
 * [B][C][Nz][Ny][Nx] (3D) float32, x fastest.  One network object is used by
 * one stream at a time (its activations live in the object).  The learned
 * guess only changes PAGD's starting point; the paper's own guess is the
 * extrapolation.
 */
typedef struct pfch_fno pfch_fno; /* opaque; owned by the library */

/* Number of parameters of a 2D / 3D network, or PFCH_E_INVAL for invalid
 * sizes (W in [1, 64], M in [1, 64], L in [1, 16]). */
int64_t pfch_fno_num_params(int32_t width, int32_t modes, int32_t layers);
int64_t pfch_fno_num_params_3d(int32_t width, int32_t modes, int32_t layers);

/* Create a network of width W <= 64, M modes (2M <= Ny, M <= Nx/2), L
 * layers, for Ny x Nx fields and batches of at most max_batch samples.
 * Parameters start at zero (see pfch_fno_init_params).  The network lives
 * on `hip_stream` (NULL: the default stream).  PFCH_E_INVAL for invalid
 * sizes, PFCH_E_UNSUPPORTED when a product would exceed the launch limits
 * (B W > 65535, 2M^2 > 65535), PFCH_E_NOMEM / PFCH_E_HIP on
 * allocation or copy failure; *out is NULL on error. */
int pfch_fno_create(int32_t width, int32_t modes, int32_t layers, int32_t ny, int32_t nx,
                    int32_t max_batch, void* hip_stream, pfch_fno** out);

/* The same for Nz x Ny x Nx fields (2M <= Nz as well; limits B W Nz
 * <= 65535, 4M^3 <= 65535).  Every other pfch_fno_* call
 * takes either kind; a 3D network attaches to 3D instances only. */
int pfch_fno_create_3d(int32_t width, int32_t modes, int32_t layers, int32_t nz, int32_t ny,
                       int32_t nx, int32_t max_batch, void* hip_stream, pfch_fno** out);

/* Deterministic pseudo-random initial parameters (scaled uniform). */
int pfch_fno_init_params(pfch_fno* f, uint64_t seed);

/* Copy the n parameters from / to a device float32 array. */
int pfch_fno_set_params(pfch_fno* f, const float* theta, int64_t n);
int pfch_fno_get_params(pfch_fno* f, float* theta, int64_t n);

/* y[batch][grid] = network(x[batch][2][grid]); device arrays. */
int pfch_fno_forward(pfch_fno* f, const float* x, float* y, int32_t batch);

/* Mean squared error of the network on (x, t[batch][grid]) and its
 * gradient with respect to the parameters, kept for pfch_fno_adam_step and
 * copied to `grad` (device, n floats) when it is not NULL.  `loss` (host) is
 * written when not NULL, which synchronises the stream. */
int pfch_fno_grad(pfch_fno* f, const float* x, const float* t, int32_t batch, float* grad,
                  double* loss);

/* One Adam update with the last gradient; `step` counts from 1 (moments are
 * cleared at step 1). */
int pfch_fno_adam_step(pfch_fno* f, float lr, float beta1, float beta2, float eps, int32_t step);

/* Network input x[2][grid] (and, when u_np1 and t are not NULL, the
 * training target t = (u^{n+1} - u^n - rho (u^n - u^{n-1}))/so) of one
 * sample from float64 device fields. */
int pfch_fno_prepare(pfch_fno* f, const double* u_nm1, const double* u_n, const double* u_np1,
                     double rho, const double norm[4], float* x, float* t);

/* The same sample prepared from float64 fields on a finer Ny x Nx grid (2D,
 * Ny, Nx at least the network's and even): inputs and target are formed on
 * the fine grid and then resampled to the network's grid by keeping the
 * modes |k| < N/2 of the network's grid on each axis (its Nyquist mode
 * dropped) and sampling that band-limited field at the network's points.
 * Buffers for the fine grid are kept by the network (made on first use). */
int pfch_fno_prepare_resampled(pfch_fno* f, int32_t ny, int32_t nx, const double* u_nm1, const double* u_n,
                               const double* u_np1, double rho, const double norm[4], float* x, float* t);

void pfch_fno_destroy(pfch_fno* f);

/* Attach network `f` (NULL detaches) to instance `inst`: its steps then use
 * the learned guess when the instance's desc.guess is 1 and it has a
 * history.  The network's grid equals the instance's, or (2D) is coarser
 * on both axes, both even: the network then runs on its own grid, its
 * inputs resampled down as in pfch_fno_prepare_resampled and its output
 * interpolated back with the same band (modes |k| < Nc/2 of the network's
 * grid, zero beyond), so the learned correction holds those modes only.
 * norm = {mu, su, sd, so}, su, sd, so > 0; the gain of the correction is
 * set to 1 and its gate opened.  The network is not owned; it must outlive
 * its use and must not be used on another stream while the context steps.
 * PFCH_E_INVAL for a grid that fits neither case; PFCH_E_UNSUPPORTED for an
 * instance with an odd number of grid points (no supported grid has one). */
int pfch_set_fno(pfch_ctx* ctx, int32_t inst, pfch_fno* f, const double norm[4]);

/* Transform plans and launch geometry of the iteration kernels of instance
 * `inst`'s group (all instances of one model, scheme and grid share them),
 * as chosen by the autotuner at pfch_create, which times the candidates on
 * the device and keeps the choice for the process (set PFCH_AUTOTUNE=0 in
 * the environment to keep the defaults).  With PFCH_TUNE_FILE naming a text
 * file, a valid choice recorded there for the group's (model, scheme, Nx,
 * Ny, Nz) is used without timing and new choices are appended, so that
 * separate processes run the same kernels.  out[37]:
 *   0 row plan alternative (-1 = default), 1 row pairs per block,
 *   2 column plan alternative (2D), 3 columns per block (2D),
 *   4 y-pass plan alternative (3D), 5 y-pass columns per block (3D),
 *   6 z-pass plan alternative (3D), 7 z-pass ky per block (3D),
 *   8..11 numbers of row, column, y and z alternatives,
 *   12..19 row radices, 20..27 column (2D) or y-pass (3D) radices,
 *   28..35 z-pass radices (unused passes have radix 1),
 *   36 reserved (0).
 * Every launch has one block per row-pair block and per column block of
 * each instance it covers, so an instance's arithmetic does not depend on
 * how many instances share the launch. */
int pfch_get_plan(pfch_ctx* ctx, int32_t inst, int32_t out[37]);

/* Override that choice: choice = out[0..7] of pfch_get_plan plus choice[8],
 * reserved, which must be 0; entries that do not apply to the grid's
 * dimension are ignored.  Each is validated against the kernels' limits
 * (PFCH_E_INVAL otherwise).  Results of different plans agree to
 * rounding. */
int pfch_set_plan(pfch_ctx* ctx, int32_t inst, const int32_t choice[9]);

/* The host's decision on a solve's stop record, exported so that it can be
 * checked without a GPU.  stop_iter is -1 while the solve runs, j when
 * ||d_j||_inf decided the stop (Alg. 2: the solve returns x_{j+1} after j+1
 * iterations), max_iter at the iteration cap; flags bit 0 = the
 * averaged-Newton symbol was not positive (Sec. 3.4.1); norm_bits =
 * ||d_j||_inf as IEEE bits.  Returns PFCH_E_PRECOND, PFCH_E_NOCONV,
 * PFCH_E_NONFINITE, PFCH_OK, or PFCH_E_INTERNAL for a record still marked
 * running (never reported as a result); *iters and *dnorm_inf (host) get
 * the iteration count and the norm.  PFCH_E_INVAL for null outputs or
 * max_iter < 1.  Needs no GPU. */
int pfch_stop_status(int32_t stop_iter, int32_t flags, uint64_t norm_bits, int32_t max_iter,
                     int32_t* iters, double* dnorm_inf);

void pfch_destroy(pfch_ctx* ctx);
const char* pfch_strerror(int code);
int pfch_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PFCH_H */
