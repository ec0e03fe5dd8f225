/*
 * sps.h — C ABI of the MI355X spectral IMEX timestep and discrete-adjoint library.
 *
 * The library advances an initial-value problem written as
 *     M dX/dt + L X = F(X)                     (paper, Supplementary: Initial value problems)
 * with a sparse ultraspherical/tau discretization (paper: Sparse spectral methods),
 * an IMEX scheme (ARS(2,2,2) or ARS(4,4,3) Runge-Kutta, SBDF2-4 multistep), and computes gradients by
 * the adjoint-state method (paper: equ:adjoint and equ:efficient_gradient): a forward
 * sweep with checkpoints, a reverse sweep through transposed solves that reuse the LU
 * factors (paper, Methods: Linear system solves) and vector-Jacobian products of F
 * through adjoint transforms (paper, Methods: Spectral transforms).
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers (allocated by the caller, e.g. torch tensors)
 *    unless stated otherwise; the caller keeps ownership.  Complex numbers are stored as
 *    (re, im) pairs of doubles.
 *  - State layout: X[k][s], k = 0..K-1 Fourier wavenumbers (half spectrum, Nyquist dropped),
 *    s = 0..S-1 slots of one wavenumber block; complex.  For the 2D Rayleigh-Benard problem
 *    S = 4N + 7: u[0:N], w[N:2N], b[2N:3N], p[3N:4N] (Chebyshev-T coefficients), then
 *    tau_u1, tau_w1, tau_b1, tau_u2, tau_w2, tau_b2, tau_p.  For 1D Kuramoto-Sivashinsky
 *    S = 1.  sps_state_size() returns K*S*2 doubles.
 *  - Cotangents (Xbar, dJdX) use the same layout and the real inner product
 *    <a, b> = sum Re(conj(a) b) of the real parameterization.
 *  - Calls are asynchronous on the stream given to sps_build_problem; results are valid
 *    after sps_sync() or a synchronization of that stream.  Argument errors are returned
 *    at once; device-detected errors (zero pivot, non-finite state) set a sticky flag
 *    that the next sps_sync() reports.  No C++ exception crosses this interface.
 *  - A handle is used from one host thread at a time.
 */
#ifndef SPS_H
#define SPS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sps_problem sps_problem;

enum sps_status {
  SPS_OK = 0,
  SPS_E_ARG = -1,          /* invalid argument or unsupported size */
  SPS_E_NOMEM = -2,        /* device allocation failed */
  SPS_E_HIP = -3,          /* HIP runtime error */
  SPS_E_SINGULAR = -4,     /* zero pivot in the LU factorization */
  SPS_E_NONFINITE = -5,    /* a state became NaN or infinite */
  SPS_E_STATE = -6,        /* call out of order (e.g. adjoint without a recorded forward run) */
  SPS_E_UNSUPPORTED = -7,
  SPS_E_NOCONV = -8,       /* an eigenvalue iteration did not converge (reported by sps_sync) */
  SPS_E_IO = -9            /* the checkpoint file could not be created, written or read */
};

enum sps_equation { SPS_RBC2D = 1, SPS_KS1D = 2, SPS_SH2D = 3, SPS_COUETTE3D = 4 };
enum sps_scheme { SPS_RK222 = 1, SPS_SBDF2 = 2, SPS_SBDF3 = 3, SPS_SBDF4 = 4, SPS_RK443 = 5 };

typedef struct {
  int equation;          /* sps_equation */
  int scheme;            /* sps_scheme; RBC: SPS_RK222 or SPS_RK443, KS any of them */
  int nx;                /* Fourier grid points at scale 1 (K = nx/2 stored wavenumbers) */
  int nz;                /* Chebyshev modes N (RBC), ignored for KS */
  double lx;             /* Fourier period */
  double param0;         /* RBC: Rayleigh number Ra */
  double param1;         /* RBC: Prandtl number Pr */
  double dealias;        /* padding factor of the collocation grid (1.5) */
  double dt;             /* timestep */
  int checkpoint_every;  /* steps between stored checkpoints in the forward sweep */
  int max_steps;         /* largest nsteps accepted by sps_step / sps_gradient */
} sps_desc;

/* The caller's device allocator (for example a framework's caching allocator), used for every
 * device allocation of the problems and networks built after the call: alloc_fn(bytes, ctx)
 * returns a device pointer (NULL: the build fails with SPS_E_NOMEM), free_fn(ptr, ctx) returns
 * it.  A handle allocates at build time (and on the first use of a feature that needs more
 * memory: a second factor set, checkpoint slots, the parameter gradient's records), never per
 * step; it frees its blocks in sps_destroy, after the device has finished the work that used
 * them, through the functions that allocated them.  alloc_fn = free_fn = NULL returns to
 * hipMalloc / hipFree.  Process-wide; set it while no other thread builds a problem.  SPS_E_ARG
 * if only one function is given. */
int sps_set_allocator(void *(*alloc_fn)(size_t bytes, void *ctx), void (*free_fn)(void *ptr, void *ctx), void *ctx);

/* Build a problem: assembles the banded operators and transform tables on the host,
 * allocates device workspace and the checkpoint store (paper, Supplementary: Initial
 * value problems; checkpointing).  hip_stream may be NULL (the null stream).
 * Returns SPS_E_ARG for unsupported sizes.  *out owns all device memory it allocates. */
int sps_build_problem(const sps_desc *desc, void *hip_stream, sps_problem **out);

/* A batch of `batch` independent instances of the 2D problem of desc (equation SPS_RBC2D, RK222 or RK443)
 * that differ in their Rayleigh number: ra (host array of batch values, copied; NULL: desc's
 * param0 for every instance), Prandtl number, sizes and step from desc.  Every instance has its
 * own LU factors (L depends on Ra through nu and kappa), and every stage launch of the sweeps
 * covers all instances (the per-wavenumber kernels run batch x K systems, the grid-row kernels
 * batch x Ngz rows).  Layouts: states and cotangents hold the instances in order (batch blocks of
 * the single-problem layout, sps_state_size() = batch K S 2 doubles); grid arrays of
 * sps_initial_state[_adjoint] hold batch (nx x nz) grids; sps_cost's and sps_gradient's J have
 * one value per instance, and the gradient is that of their sum.  sps_step, sps_adjoint_step,
 * sps_gradient (uniform checkpoints, graph mode included; no dJdtheta), sps_cost,
 * sps_initial_state[_adjoint], sps_factor, sps_set_dt, sps_set_graph and the timers work as for
 * one problem; the other entry points return SPS_E_UNSUPPORTED for a batch. */
int sps_build_rbc_batch(const sps_desc *desc, int batch, const double *ra, void *hip_stream, sps_problem **out);

/* Batched 2D Swift-Hohenberg problems u_t = r u - (1 + Laplacian)^2 u - u^3 on [0, lx)^2,
 * periodic (IVP form of the Supplementary, "Initial value problems": M = 1,
 * L = -r + (1 - |k|^2)^2, F = -u^3 with the cube on a grid padded by 2), SBDF2 with an SBDF1
 * first step, one independent instance per entry of n (N_i x N_i modes, N_i even, 8..512,
 * factors 2 and 3 only) and r (host arrays of length batch, copied).  Every forward sweep,
 * cost seed and reverse sweep of the whole batch runs as one cooperative persistent launch;
 * at build time the library times a few steps of each tile configuration (columns per
 * column tile and row pairs per row tile, per size class, and the block count) and keeps
 * the fastest.
 * Layouts: a state holds, per instance in order, X[m][iy] (m < N/2 the k_x index, iy < N the
 * k_y index in FFT order, iy = N/2 unused and zero), complex as (re, im); grid arrays hold
 * per instance u[y][x] (N x N).  sps_gradient's J output and sps_cost's J have one value per
 * instance: J_i = 1/2 mean of u_i(T)^2 over the N_i x N_i grid; the gradient is of the sum.
 * sps_initial_state maps grid fields to states (the N x N discrete Fourier transform / N^2,
 * kept modes); sps_solve applies (1.5/dt + L)^-1.  max_steps bounds nsteps; the library
 * keeps every state of the last forward sweep. */
int sps_build_sh_batch(int batch, const int *n, const double *r, double lx, double dt, int max_steps,
                       void *hip_stream, sps_problem **out);

/* The tile configuration the build-time tuning chose for a batched Swift-Hohenberg problem:
 * col_tile[4] and row_tile[4] for the size classes N <= 64, <= 96, <= 128, larger; the
 * persistent block count and threads per block; the measured time of one forward step of
 * the batch (ms). */
int sps_sh_tuning(const sps_problem *P, int *col_tile, int *row_tile, int *blocks, int *threads, double *step_ms);

/* 3D plane Couette flow, Fourier (x, period lx) x Chebyshev (y in [-1, 1]) x Fourier (z, period lz):
 * the perturbation u = (u, v, w) of the laminar flow U = y between walls moving with -1, +1,
 * u_t + (u.grad) u + U u_x + v U' e_x + grad p - (1/re) Laplacian u = 0, div u = 0, u = 0 at the
 * walls, in the IVP form of the Supplementary, "Initial value problems" (Stokes part implicit,
 * products and base-flow terms explicit on the 3/2 padded grid), RK222 with checkpoints every
 * checkpoint_every steps and the discrete adjoint of the sweep (equ:adjoint).  Modes: x index
 * m < nx/2, z index n < nz in FFT order (the z Nyquist n = nz/2 unforced), mode k = m nz + n;
 * nx, nz even with 3/2 nx and 3/2 nz factoring into 2 and 3; ny even in [8, 128].
 * State layout per mode (S = 4 ny + 7 complex slots): u_par, v, u_perp, p (ny Chebyshev
 * coefficients each, T_n(y)), then the tau slots (par, v, perp first-order, then second-order,
 * then tau_p).  u_par = (kx u + kz w)/kh and u_perp = (-kz u + kx w)/kh in the frame of the wave
 * vector (kh = |(kx, kz)|; at kh = 0, u_par = u and u_perp = w); tau values are those of the
 * problem scaled to unit wall distance, twice the ones of the unscaled equations.
 * sps_cost gives J = 1/2 int |u|^2 dV (mode 0 by its real part, z Nyquist modes excluded) and
 * dJ/dX; sps_gradient, sps_step and sps_adjoint_step work as for the 2D problem;
 * sps_eval_F, sps_eval_F_vjp and sps_solve act in the scaled frame (time unit t/2);
 * sps_initial_state[_adjoint] return SPS_E_UNSUPPORTED (states are given as coefficients). */
int sps_build_couette(int nx, int ny, int nz, double lx, double lz, double re, double dt, int checkpoint_every,
                      int max_steps, void *hip_stream, sps_problem **out);

/* Plane Couette states (or cotangents) between the physical layout and the library's.
 * Physical layout per mode (S = 4 ny + 7 complex slots): u, v, w, p (ny Chebyshev coefficients
 * each), then the taus of the unscaled equations: first-order tau of u, v, w, second-order tau
 * of u, v, w, tau_p.  Library layout: the one described for sps_build_couette (u_par, v, u_perp
 * and the taus in the frame of the mode's wave vector, taus twice the unscaled ones).  to_library
 * != 0 maps physical -> library, else library -> physical.  cotangent != 0 treats the arrays as
 * cotangents (gradients) of states: the rotation is orthogonal, so velocities rotate alike, and
 * the tau slots scale by the inverse factor.  in and out are device arrays of sps_state_size()
 * doubles and must not overlap.  Asynchronous on the problem's stream.  SPS_E_UNSUPPORTED for
 * other problems. */
int sps_couette_frame(sps_problem *P, const double *in, double *out, int to_library, int cotangent);

/* Batched 2D Kolmogorov flow in vorticity form on [0, 2 pi)^2, periodic:
 * omega_t + u . grad omega = nu Laplacian omega - drag omega - 4 cos 4y (+ closure),
 * u = (d_y psi, -d_x psi), psi = omega / |k|^2, nu = 1/re, drag >= 0 a linear friction.  IVP
 * form of the Supplementary, "Initial value problems": M = 1, L = nu |k|^2 + drag,
 * F = -u . grad omega + f (+ closure) with the advection on the 3/2
 * padded grid; SBDF2 with an SBDF1 first step (equ:imex) and its discrete adjoint
 * (equ:IMEX_adjoint).  batch independent instances of N x N modes (N a multiple of 4 with
 * factors 2 and 3 only, 8..1024).  closure != 0 adds the closure network (sps_cnn_*) evaluated
 * on the N x N vorticity grid to F (N a multiple of 32); its parameters start at zero.
 * keep_history != 0 keeps every state of the last forward run (max_steps + 1 states), which
 * the reverse sweep, sps_kolmo_rollout's gradients, sps_adjoint_step and sps_eval_F_vjp need;
 * keep_history == 0 keeps three states, for long forward runs of any length.
 * Layout: as the Swift-Hohenberg problems, per instance X[m][iy] (m < N/2, iy in FFT order,
 * iy = N/2 unused and zero), complex (re, im); the grid values of a state are
 * omega(x, y) = Re sum w_m X[m][iy] e^{i (m x + k_y y)}, w_0 = 1, w_m = 2.
 * sps_step, sps_adjoint_step, sps_eval_F and sps_eval_F_vjp work as for every problem;
 * sps_cost, sps_gradient, sps_solve and sps_initial_state* return SPS_E_UNSUPPORTED. */
int sps_build_kolmo(int batch, int n, double re, double drag, double dt, int max_steps, int closure,
                    int keep_history, void *hip_stream, sps_problem **out);

/* Copy the closure parameters (FP64 device vector of sps_cnn_nparam() values, order as for
 * sps_cnn_set_params) into the problem.  SPS_E_ARG without the closure. */
int sps_kolmo_set_params(sps_problem *P, const double *theta);

/* Forward run of nsteps steps from X0 (device state, read only); XN (nullable) receives the
 * last state.  snap (nullable): every `every` steps the state truncated to the nc x nc modes
 * of a coarse grid (|k_x|, |k_y| < nc/2, coarse Nyquist row zero) is written in the coarse
 * state layout, snapshot s (steps (s+1) every) at snap + s * batch * nc * nc (doubles); the
 * caller sizes it for nsteps / every snapshots.  Without keep_history nsteps is unbounded. */
int sps_kolmo_forward(sps_problem *P, const double *X0, int nsteps, double *XN, double *snap, int every, int nc);

/* Rollout loss and its gradients through the discrete adjoint (equ:efficient_gradient):
 * J[b] = (1/nsteps) sum_{k=1..nsteps} mean over the N x N grid of (omega_k - target_k)^2 with
 * targets[k-1] the k-th target state (device, nsteps * state size doubles, state layout);
 * the cotangent of every intermediate state enters the reverse sweep.  XN, J (batch values),
 * dJdX0 (state layout) and dJdtheta (sps_cnn_nparam() values, the SUM over instances of
 * dJ[b]/dtheta, overwritten) are nullable; the gradients need keep_history and nsteps <=
 * max_steps, dJdtheta the closure. */
int sps_kolmo_rollout(sps_problem *P, const double *X0, const double *targets, int nsteps, double *XN, double *J,
                      double *dJdX0, double *dJdtheta);

/* theta_bar += (dF/dtheta)^T Fbar at state X (closure parameters' cotangent of one explicit-
 * term evaluation, summed over instances).  Needs the closure and keep_history. */
int sps_kolmo_param_vjp(sps_problem *P, const double *X, const double *Fbar, double *theta_bar);

/* One Adam update of the closure parameters theta (device, sps_cnn_nparam() values, updated in
 * place and then loaded as the problem's parameters) with gradient grad and moment vectors m1,
 * m2 (device, same length, updated in place; start at zero), learning rate lr, step count
 * t >= 1, beta1 = 0.9, beta2 = 0.999, eps = 1e-8.  Not part of the paper's method: the
 * optimiser of the closure's training. */
int sps_kolmo_adam(sps_problem *P, double *theta, const double *grad, double *m1, double *m2, double lr, int t);

/* Number of doubles in one state vector (K * S * 2). */
long long sps_state_size(const sps_problem *P);

/* LU-factor the implicit matrices of the scheme for every wavenumber (paper, Methods:
 * Linear system solves; factors are reused until dt changes).  Idempotent. */
int sps_factor(sps_problem *P);

/* Forward sweep: advance X (in/out, state layout) by nsteps steps of the IMEX scheme
 * (paper, equ:imex and the IMEX Runge-Kutta stage equations), storing a checkpoint
 * every checkpoint_every steps so that sps_adjoint_step can reverse this run.
 * 1 <= nsteps <= max_steps.  Factors automatically if needed. */
int sps_step(sps_problem *P, double *X, int nsteps);

/* Reverse sweep over the run recorded by the last sps_step (paper, equ:IMEX_adjoint
 * and the RK adjoint equations): on entry Xbar holds the cotangent of the final state,
 * on exit the cotangent of the initial state.  Segments between checkpoints are
 * recomputed.  nsteps must equal the recorded run length, else SPS_E_STATE. */
int sps_adjoint_step(sps_problem *P, double *Xbar, int nsteps);

/* Cost functional and its gradient at a state (paper, equ:efficient_gradient seed):
 * RBC: J = 1/2 int int (u^2 + w^2) dz dx; KS: J = 1/2 (1/L) int u^2 dx.
 * J_out: device pointer to one double; dJdX: cotangent in state layout. */
int sps_cost(sps_problem *P, const double *X, double *J_out, double *dJdX);

/* Full gradient (paper: equ:adjoint and equ:efficient_gradient): X0 -> forward nsteps with
 * checkpoints -> the final-time cotangent -> reverse sweep -> dJ/dX0.
 *  dJdXN (nullable, input): the cotangent of the final state from an upstream vector-Jacobian
 *        product (Supplementary, Initial value problems: the final-time condition of the adjoint
 *        comes from the cost's VJP, which may belong to a larger computation); the reverse sweep
 *        starts there.  NULL: the built-in cost of the problem (sps_cost) and its gradient.
 *  XN (nullable, output): the final state.
 *  dJdX0 (output, required): the gradient with respect to the initial state, state layout.  It
 *        may be the same array as dJdXN (read first, then overwritten).
 *  dJdtheta (nullable, output): the gradient with respect to the problem's parameters (the
 *        efficient-gradient identity: minus the sum over steps and stages of the stage adjoints
 *        against the parameter derivative of each stage's residual).  The 2D problem: two
 *        doubles, dJ/dRa and dJ/dPr (L depends on them through nu = (Ra/Pr)^(-1/2) and
 *        kappa = (Ra Pr)^(-1/2); M and F do not), with the uniform checkpoint schedule (the
 *        recorded segments also keep each step's stage states: 2 states per step of a segment,
 *        allocated on the first such call).  Other problems and schedules return
 *        SPS_E_UNSUPPORTED when it is not NULL.
 *  J_out (nullable, output, one double): the built-in cost; must be NULL when dJdXN is given
 *        (SPS_E_ARG). */
int sps_gradient(sps_problem *P, const double *X0, int nsteps, const double *dJdXN, double *XN, double *dJdX0,
                 double *dJdtheta, double *J_out);

/* Initial state from scale-1 grid values (paper, Methods: Spectral transforms, forward
 * transform f_hat = T f).  RBC: grid is b0[x][z], nx * nz doubles; the state gets b and
 * zero u, w, p, taus.  KS: grid is u0[x], nx doubles. */
int sps_initial_state(sps_problem *P, const double *grid, double *X);

/* Adjoint of sps_initial_state (T^H applied to the cotangent): gradient with respect to
 * the scale-1 grid values. */
int sps_initial_state_adjoint(sps_problem *P, const double *Xbar, double *grid_bar);

/* Components of one step, exposed for verification of single rows of the path. */
/* F(X) in state layout (rows are equation slots). */
int sps_eval_F(sps_problem *P, const double *X, double *F);
/* (dF/dX)^H Fbar at X. */
int sps_eval_F_vjp(sps_problem *P, const double *X, const double *Fbar, double *Xbar);
/* sps_eval_F for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same result, bit for bit, with
 * the intermediates (x-spectral z-grid fields and nonlinear terms, 9 * K * Ngz complex values,
 * Ngz = 3 nz / 2) in the library's static scratch of 2 MiB per GPU instead of the problem's
 * workspace.  The call allocates nothing (no hipMalloc, no events): it launches three kernels on
 * the problem's stream.  The scratch is looked up once per device (the device current when the
 * problem was built) on the first call and held until the process ends; every call on a GPU
 * shares it, so calls that overlap on one GPU (several streams or host threads) race and must be
 * serialized by the caller.  SPS_E_ARG when the problem needs more than the 2 MiB (nx = 256,
 * nz = 64 needs 1.77 MB; nx = 324, nz = 64 is refused); SPS_E_UNSUPPORTED for problems other
 * than SPS_RBC2D. */
int sps_eval_F_noalloc(sps_problem *P, const double *X, double *F);
/* Solve A x = r (adjoint = 0) or A^H x = r (adjoint = 1) with the current factors of the
 * scheme's implicit matrix (RK222: M + dt*gamma*L; RK443: M + dt/2 L; SBDF-k: a_0 M + L with the
 * steady a_0 = 3/2, 11/6, 25/12 over dt for k = 2, 3, 4). */
int sps_solve(sps_problem *P, const double *R, double *X, int adjoint);

/* Eigenvalue problem of the 2D problem's operator (Supplementary, "Eigenvalue problems"):
 * linear stability of the conduction state b0 = 1 - z, u = 0, i.e. (lambda M + L_s) X = 0 per
 * wavenumber with L_s the IVP's L plus the linearized advection of b0 (-S10 w in the b rows),
 * lambda the growth rate.  For every wavenumber k of the problem at once: the eigenvalue
 * nearest the real shift sigma by inverse iteration with A = sigma M + L_s (one blocked
 * almost-banded LU per call, `iters` iterations), the adjoint eigenvector
 * ((conj(lambda) M^H + L_s^H) Y = 0) by the same number of iterations through the transposed
 * solves of the same factors, and the eigenvalue sensitivities of equ:eigenvalue_sens,
 * d lambda/dp = -<Y, dL/dp X> / <Y, M X> for p = Ra (at fixed Pr) and p = k.  Device arrays:
 * lam[K] complex; X and Y [K][S] complex in the state layout, unit Euclidean norm per
 * wavenumber; dlam[K][2] complex (d/dRa, d/dk).  Convergence is linear in
 * |lambda - sigma| / |lambda_2 - sigma|; the caller picks sigma and iters.  The stability bands
 * and a third factor set are built on the first call.  SPS_E_UNSUPPORTED for other problems. */
int sps_stability(sps_problem *P, double sigma, int iters, double *lam, double *X, double *Y, double *dlam);

/* Eigenvector sensitivities (Supplementary, "Eigenvalue problems", equ:eigenvector_sens with
 * dM/dp = 0): for p = Ra (at fixed Pr) and p = k, per wavenumber, the solution z of
 * (lambda M + L_s) z = -(dlambda/dp M + dL/dp) X with <X, z> = 0 (unique, the right-hand side
 * being orthogonal to Y).  lam, X, Y, dlam: the outputs of sps_stability with the same sigma
 * (device arrays, read only).  z is found through one blocked LU of sigma M + L_s by `iters`
 * iterations z <- P (sigma M + L_s)^-1 (r - (lambda - sigma) M z), P the spectral projector
 * I - X (Y^H M .)/(Y^H M X), then z's component along X is removed; each iteration contracts
 * the error by |lambda - sigma| / min_j |lambda_j - sigma| (the other eigenvalues lambda_j of the
 * wavenumber), so a shift near the eigenvalue converges in a few iterations.  dX: device
 * array [2][K][S] complex (p-major: dX/dRa of every wavenumber, then dX/dk).  The 2D problem;
 * SPS_E_UNSUPPORTED otherwise. */
int sps_stability_vector_sens(sps_problem *P, double sigma, int iters, const double *lam, const double *X,
                              const double *Y, const double *dlam, double *dX);

/* Several eigenvalues nearest the real shift sigma per wavenumber of the same stability problem
 * (Supplementary, "Eigenvalue problems": shift-invert about a target with a Krylov eigensolver):
 * m Arnoldi steps on B = (sigma M + L_s)^-1 M through one blocked LU of sigma M + L_s, each
 * new vector orthogonalized by classical Gram-Schmidt applied twice, then the eigenpairs
 * (nu, y) of the m x m Hessenberg matrix by shifted QR steps on the device, and
 * lambda = sigma - 1/nu.  2 <= m <= min(64, 3 nz), 1 <= nev <= m.  Device arrays:
 *   v0   (nullable) [K][S] complex start vectors in the state layout (any norm); NULL uses a
 *        fixed start vector;
 *   lam  [K][nev] complex: the nev eigenvalues with the largest |nu| (nearest sigma), in
 *        that order;
 *   X    (nullable) [K][nev][S] complex Ritz vectors V_m y, unit Euclidean norm;
 *   res  (nullable) [K][nev] doubles: the residuals |h_{m+1,m}| |e_m^T y| (|y| = 1) of the
 *        pairs of B; a pair has converged when res is small against |nu|;
 *   H    (nullable) [K][m+1][m] complex: the Arnoldi matrix, row-major.
 * The 2D problem; SPS_E_UNSUPPORTED otherwise.  A QR iteration that does not converge in
 * 30 m steps sets a flag that the next sps_sync() reports as SPS_E_NOCONV. */
int sps_stability_arnoldi(sps_problem *P, double sigma, int m, int nev, const double *v0, double *lam, double *X,
                          double *res, double *H);

/* Linear stability of plane Poiseuille flow, the paper's neutral-curve example (Results,
 * "Parametric sensitivity and numerical continuation"; Supplementary, "Eigenvalue problems"):
 * flow between walls y = 0 and y = 2 with base flow U = y (2 - y), two-dimensional perturbations
 * (u, v, p) ~ exp(i alpha x + lambda t), (lambda M + L(alpha, Re)) X = 0 with the growth rate
 * Re(lambda), discretized as the 2D problem (Chebyshev-T unknowns, C2 momentum and C1 continuity
 * rows, lifted taus; state slots u[0:nz], v[nz:2nz], p[2nz:3nz], tau_u1, tau_v1, tau_u2, tau_v2,
 * tau_p, S = 3 nz + 5).  The handle holds the operator parts and factor storage for up to
 * max_systems systems solved at once; 8 <= nz <= 256.  Only sps_poiseuille_solve, sps_sync,
 * sps_state_size and sps_destroy apply to it. */
int sps_build_poiseuille(int nz, int max_systems, void *hip_stream, sps_problem **out);
/* nsys independent systems at once (one thread block each).  params: HOST array [nsys][5] of
 * (alpha, Re, sigma_re, sigma_im, ds), copied (ds: the continuation step of mode 3).  For each system: the complex banded LU of
 * sigma M + L with partial pivoting, `iters` inverse iterations for the eigenvalue nearest the
 * shift sigma and its right eigenvector, and (through the same factors, the conjugate-transposed
 * solves) the left eigenvector Y, ((conj(lambda) M^H + L^H) Y = 0), then the sensitivities of
 * equ:eigenvalue_sens, d lambda/dp = -<Y, dL/dp X> / <Y, M X>, for p = Re and p = alpha.
 * mode 0: that eigenpair; mode 1: Newton's method on the growth rate in Re at fixed alpha
 * (Re <- Re - Re(lambda) / Re(d lambda/dRe), the next shift at the new eigenvalue) until
 * |Re(lambda)| <= tol or maxit eigenvalue solves; mode 2: the same in alpha at fixed Re; mode 3: one
 * step of the continuation along the neutral curve from a point on it (Results, "Parametric
 * sensitivity and numerical continuation"): the point moves by ds along the tangent of the curve
 * in (alpha, ln Re) (the gradient (d/dalpha, Re d/dRe) of the growth rate turned by a right angle,
 * so that the unstable side stays on the same hand), then minimum-norm Newton steps in
 * (alpha, ln Re) along the gradient bring it back onto the curve (turning points included).  Device
 * outputs: lam[nsys] complex; dlam[nsys][2] complex (d/dRe, d/dalpha); info[nsys][3] doubles
 * (alpha, Re at the end, eigenvalue solves used); X, Y (nullable) [nsys][S] complex in the state
 * layout, unit Euclidean norm.  A Newton run that ends above tol sets a flag that the next
 * sps_sync() reports as SPS_E_NOCONV, a zero pivot SPS_E_SINGULAR.  Returns after the launch has
 * read params (the call synchronizes the problem's stream). */
int sps_poiseuille_solve(sps_problem *P, int nsys, const double *params, int iters, int mode, double tol,
                         int maxit, double *lam, double *dlam, double *info, double *X, double *Y);

/* A new constant step dt > 0 for the following runs (a step-size change between segments of a
 * run, as an adaptive step controller makes it; equ:imex: the implicit matrices depend on dt).
 * The 2D problem and plane Couette refactor every wavenumber's M + dt gamma L at once (one
 * blocked LU per wavenumber on the problem's stream); KS takes the new dt in its SBDF rows
 * (unless variable steps are set) or RK stage coefficients.  Drops the recorded forward run and
 * captured graphs: the reverse sweep of a segment runs with that segment's step, so a gradient
 * through a run with step changes reverses the segments one by one, each after sps_set_dt of
 * its own step and a recomputation of its forward sweep.  sps_solve then uses the new matrix.
 * The batched Swift-Hohenberg and Kolmogorov problems take it in their SBDF2 coefficients (their
 * implicit operators are diagonal).  SPS_E_ARG for dt <= 0 or not finite. */
int sps_set_dt(sps_problem *P, double dt);

/* Variable time steps of the multistep schemes (equ:imex: the coefficients of step n depend on
 * the step sizes, lower order while the history is short).  dts: HOST array of n step sizes
 * (dts[i] = t_{i+1} - t_i, positive), copied; later sps_step / sps_gradient runs of at most n
 * steps take step i + 1 with dts[i], and sps_adjoint_step reverses them with the same rows.
 * Step n's row is the SBDF-k of the problem's scheme on the non-uniform nodes t_n .. t_{n-q},
 * q = min(n, k): a_j the derivative at t_n of the Lagrange basis polynomial of node t_{n-j}
 * (backward difference of M dX/dt), c_i the value at t_n of the basis polynomial of t_{n-i}
 * on t_{n-1} .. t_{n-q} (extrapolation of F); equal steps give the constant-step rows.
 * With the RK schemes step i + 1 uses dts[i] in its stage coefficients; KS's implicit matrices
 * are diagonal, so nothing is refactored.  The 2D problem, its batches and plane Couette (RK222 or
 * RK443) factor M + dts[i] H_ii L once per distinct step (at most 16 in one call; the factor sets
 * are kept for later calls, 64 distinct steps over a problem's life) and step i + 1 of a run, its
 * recomputation and its reverse step use that step's set and stage coefficients, so one
 * recorded run and its gradient span the step changes (any checkpoint schedule, graph mode
 * included); runs longer than n steps are refused (SPS_E_ARG).
 * dts = NULL or n = 0 returns to the constant step of the descriptor (sps_solve always uses
 * it).  Drops the recorded forward run and captured graphs.  SPS_E_UNSUPPORTED for the batched
 * Swift-Hohenberg and Kolmogorov problems. */
int sps_set_timesteps(sps_problem *P, const double *dts, int n);

/* Checkpointing of the Runge-Kutta sweeps (Supplementary, "Initial value problems": the reverse
 * sweep needs every forward state, kept through a checkpoint schedule that trades storage for
 * recomputation).  scheme SPS_CKPT_UNIFORM (the default): a stored state every
 * checkpoint_every steps and the stage data of one segment, segments recomputed on a second
 * stream while the adjoint of the next one runs.  scheme SPS_CKPT_BINOMIAL: `slots` >= 1 stored
 * states (slot 0 holds X_0) placed by the binomial schedule of sps_checkpoint_schedule, which
 * needs the fewest forward recomputations for that storage; sps_step runs its forward sweep,
 * sps_adjoint_step and sps_gradient its reverse sweep, all on the problem's stream.  scheme
 * SPS_CKPT_TWO_LEVEL: the state at the start of every segment of checkpoint_every steps is
 * stored in pinned host memory by the forward sweep; the reverse sweep brings the segments
 * back from the last and reverses each with the binomial schedule of its length on `slots`
 * device states (sps_gradient then runs eagerly, also in graph mode).  Gradients are the same
 * as with the default schedule.  Device memory: `slots` states (K S complex values each);
 * host memory (two levels): ceil(max_steps / checkpoint_every) states, or the outer slot count
 * of sps_set_outer_slots when smaller; held until sps_destroy.  With SPS_CKPT_BINOMIAL the reverse
 * sweep reuses the snapshot slots, so a recorded run is reversed once (a second
 * sps_adjoint_step returns SPS_E_STATE).  Drops recorded graphs and the recorded forward run
 * (sps_adjoint_step needs a new sps_step).  The 2D and plane Couette problems;
 * SPS_E_UNSUPPORTED otherwise. */
enum sps_checkpointing { SPS_CKPT_UNIFORM = 0, SPS_CKPT_BINOMIAL = 1, SPS_CKPT_TWO_LEVEL = 2 };
int sps_set_checkpointing(sps_problem *P, int scheme, int slots);

/* Disk level of the SPS_CKPT_TWO_LEVEL schedule (Supplementary, "Initial value problems": stored
 * states on slower, larger storage when a run outgrows device and host memory).  path != NULL:
 * the state at the start of every segment goes to this file (created or truncated, owner-only
 * permissions, removed when the problem is destroyed or another path is set) instead of pinned
 * host memory, staged through two pinned buffers of one state each: the forward sweep writes
 * segment g's start once its device-to-host copy is done, while later segments run; the reverse
 * sweep reads segment g's start while segment g+1 is reversed.  The host thread waits on
 * those copies, so sps_step and sps_gradient return after the sweep's last file access.
 * path = NULL returns to pinned host memory.  Drops the recorded forward run.  File errors
 * return SPS_E_IO.  The 2D problem and plane Couette; SPS_E_UNSUPPORTED otherwise. */
int sps_set_checkpoint_file(sps_problem *P, const char *path);

/* Number of outer-level states (pinned host memory, or the checkpoint file) of the
 * SPS_CKPT_TWO_LEVEL schedule.  0 (the default): one per segment of checkpoint_every steps.
 * 1 <= slots < the number of segments of a run: nested binomial checkpointing (Supplementary,
 * "Initial value problems": multi-level schedules that trade storage on each level for
 * recomputation) - the segment starts are placed on the outer slots by the binomial schedule
 * over segments (slot 0 holds X_0; segments are recomputed from earlier stored starts), and
 * each segment is reversed with the binomial schedule of its length on the device slots.  With
 * a file the outer accesses are synchronous (each waits for its copy).  Gradients are
 * bit-identical to the other schedules.  As with SPS_CKPT_BINOMIAL, the reverse sweep reuses
 * the stored states, so a recorded run is reversed once (a second sps_adjoint_step returns
 * SPS_E_STATE).  Drops the recorded forward run.  The 2D problem and
 * plane Couette; SPS_E_UNSUPPORTED otherwise. */
int sps_set_outer_slots(sps_problem *P, int slots);

/* Costs of the outer level of the nested schedule (Supplementary, "Initial value problems":
 * multi-level schedules on slower storage, whose reads and writes cost time; the paper's runs
 * use the H-revolve schedule for RAM and disk): write_cost and read_cost are the times of
 * storing and loading one outer state, in units of one forward step.  Both >= 0: the segment
 * starts are placed on the outer slots by the schedule of least total cost (forward steps of the
 * segments recomputed, outer writes and reads; every split of the binomial recursion searched,
 * segments of checkpoint_every steps) instead of the fewest forward steps; each segment is
 * still reversed with the binomial schedule of its length on the device slots.  Negative (the
 * default): the binomial placement.  Gradients are bit-identical either way.  SPS_E_ARG when
 * only one of the two is negative; SPS_E_UNSUPPORTED as sps_set_outer_slots. */
int sps_set_outer_costs(sps_problem *P, double write_cost, double read_cost);

/* The binomial schedule for nsteps steps and `slots` stored states (host arrays; no problem
 * or device needed): phase 0 the forward sweep, phase 1 the reverse sweep.  Writes *count
 * actions as (op, a, b) triples into actions (capacity: actions it can hold); op 1 = advance
 * the working state from step a to step b, 2 = store the working state (step b) in slot a,
 * 3 = load slot a (the state of step b) into the working state, 4 = run step a forward
 * recording its stage data and then its adjoint.  The reverse sweep's op-4 actions visit
 * steps nsteps-1 .. 0 in order.  SPS_E_ARG (with *count set) when capacity is too small. */
int sps_checkpoint_schedule(int nsteps, int slots, int phase, int *actions, int capacity, int *count);

/* The schedule of least cost for the same problem when a forward step costs adv, storing a
 * state wr and loading one rd (all >= 0; the outer level of sps_set_outer_costs, whose units are
 * segments): the snapshot positions minimize adv x (forward steps of the reverse sweep)
 * + wr x (states stored, X_0 included) + rd x (states loaded) over every split of the binomial
 * recursion, which for wr = rd = 0 gives the fewest forward steps.  Same action format and
 * errors as sps_checkpoint_schedule (SPS_E_ARG also for a negative or non-finite cost, and when
 * nsteps^2 min(slots, nsteps) exceeds 2e10, the search's work); *cost (nullable) gets the
 * schedule's total cost. */
int sps_checkpoint_schedule_costs(int nsteps, int slots, double adv, double wr, double rd, int phase,
                                  int *actions, int capacity, int *count, double *cost);

/* Linear boundary value problem of the 2D problem's operator (Supplementary, "Linear boundary
 * value problems"): L X = M f + c, the steady state of the IVP without its explicit term,
 * driven by body forces and a heat source f, with the IVP's boundary data c (no-slip walls,
 * b(0) = 1 and b(1) = 0 for the horizontal mean, the pressure gauge).  f and X are device
 * arrays in the state layout; only the u, w, b coefficient blocks of f are read (T_n(2z-1)
 * coefficients of the forcing of each equation), its p and tau slots are ignored.  X is the
 * full solution (velocity, buoyancy, pressure, taus): an admissible initial state for
 * sps_step / sps_gradient, so that an IVP cost can be differentiated through the LBVP.
 * L is LU-factored per wavenumber on the first call (the blocked almost-banded factors of the
 * IVP, a second set held by the problem until sps_destroy) and reused by every later call and
 * by sps_lbvp_adjoint.  A zero pivot sets the sticky device flag (sps_sync returns
 * SPS_E_SINGULAR).  SPS_E_UNSUPPORTED for problems other than SPS_RBC2D. */
int sps_lbvp_solve(sps_problem *P, const double *f, double *X);

/* Adjoint of sps_lbvp_solve: the adjoint state equation L^H Y = Xbar through the same
 * factors, then the VJP of the right-hand side, fbar = M^H Y (u, w, b blocks; zero p and tau
 * slots).  Xbar is the cotangent of X (for example dJ/dX_0 from sps_adjoint_step); fbar is the
 * gradient with respect to the forcing coefficients in the real inner product of the state
 * layout.  Device arrays; asynchronous like every call. */
int sps_lbvp_adjoint(sps_problem *P, const double *Xbar, double *fbar);

/* Kernel timing of one kernel class inside the library (HIP events stamped by each launch's
 * dispatch on the problem's stream; launches on the auxiliary stream and inside graph capture
 * are not timed).  kind: 0 = per-wavenumber forward stage kernel (transforms in z, RHS
 * assembly, banded solve), 1 = per-wavenumber adjoint stage kernel (transposed solve, adjoint
 * transforms), 2 = grid-row forward kernel (x transforms and products), 3 = grid-row adjoint
 * kernel (their VJP); the 2D problem takes all four, other problems kind 0 where they have a
 * timer.  One kind is followed at a time.  sps_timer_read returns launches and total
 * milliseconds since sps_timer_enable and resets the counters. */
int sps_timer_enable(sps_problem *P, int kind, int on);
int sps_timer_read(sps_problem *P, long long *launches, double *total_ms);

/* Graph mode for sps_gradient (a step sequence captured once and replayed as one HIP graph;
 * the paper's method is unchanged, only how the launches reach the GPU).  With on != 0 the
 * first sps_gradient call for a given (X0, nsteps, XN, dJdX0, J) tuple records its whole
 * launch sequence (forward sweep, checkpoint copies, cost seed, and the reverse sweep on
 * both of the problem's streams) into a graph, on a private capture stream, and launches it
 * on the problem's stream; later calls with the same tuple replay it.  Results are identical
 * to eager launches.  The graphs hold kernel and device-to-device copy nodes only (no
 * memsets) and keep the pointers of their tuple: the arrays must stay allocated while graph
 * mode is on.  on = 0 (the default) launches eagerly and frees the recorded graphs.  The
 * kernel timer is not fed by replays.  SPS_E_UNSUPPORTED for problems without graph mode. */
int sps_set_graph(sps_problem *P, int on);

/* Closure network on its own (the explicit-term closure of the Kolmogorov problem; not part
 * of the paper's method): three periodic 3x3 convolutions 1 -> 32 -> 32 -> 1 with GELU, bf16
 * weights and activations, FP32 accumulation (MFMA for the 32 -> 32 layer).  Images are FP64
 * device arrays [batch][H][W] (W a multiple of 32); parameters one FP64 device vector of
 * sps_cnn_nparam() values in the order w1 (32x1x3x3), b1, w2 (32x32x3x3), b2, w3 (1x32x3x3), b3,
 * w[o][c][dy+1][dx+1] multiplying the input at (y+dy, x+dx), periodic.  sps_cnn_vjp writes the
 * input cotangent and ADDS the parameter cotangent to theta_bar (nullable).  Calls run on the
 * handle's stream. */
typedef struct sps_cnn sps_cnn;
int sps_cnn_build(int batch, int H, int W, void *hip_stream, sps_cnn **out);
int sps_cnn_nparam(void);
int sps_cnn_set_params(sps_cnn *C, const double *theta);
int sps_cnn_forward(sps_cnn *C, const double *x, double *y);
int sps_cnn_vjp(sps_cnn *C, const double *x, const double *ybar, double *xbar, double *theta_bar);
void sps_cnn_destroy(sps_cnn *C);

/* Wait for the problem's stream; report a deferred device error. */
int sps_sync(sps_problem *P);

/* Message of the last error on this thread (static storage). */
const char *sps_last_error(void);

/* Release everything the handle owns. */
void sps_destroy(sps_problem *P);

#ifdef __cplusplus
}
#endif

#endif /* SPS_H */
