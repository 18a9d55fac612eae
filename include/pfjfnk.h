/*
 * pfjfnk.h -- C ABI of the MI355X (gfx950) matrix-free JFNK hot path for the
 * implicit phase-field method of Ghosh, Newman & Francois, "Tusas: a fully
 * implicit parallel approach for coupled phase-field equations".
 *
 * Problem (paper Sec. 2): nodal Q1 finite elements on a structured box mesh
 * [-L0,L0] x [-L1,L1] (x [-L2,L2]) with n[k] elements and n[k]+1 nodes per
 * axis, two fields per node (phi, u), the weighted (theta) method in time
 * (Sec. 2.1.2, Eqs. dpf, dtemp, theta; theta = 1 is backward Euler).  The
 * residual of the step from U^n (and U^(n-1)) to U is F(U; U^n) + E(U^n, U^(n-1))
 * with the part that depends on U
 *
 *   F1_i = (a^2 (phi - phi^n)/dt, psi_i)
 *          + theta [ (J(grad phi), grad psi_i) - (phi - phi^3 - lambda (1 - phi^2)^2 u, psi_i) ]
 *   F2_i = ((u - u^n)/dt - theta (phi - phi^n)/(2 dt), psi_i) + theta (D grad u, grad psi_i)
 *
 * and the part fixed by the previous states (zero when theta = 1)
 *
 *   E_i = (1 - theta) [ the spatial terms of F at U^n ]
 *         - (1 - theta) ((phi^n - phi^(n-1))/(2 dt), psi_i)  on the u rows,
 *
 * with the fourfold anisotropy a(g) = 1 - 3 eps4 + 4 eps4 sum g_k^4/(|g|^2 +
 * delta2)^2 (Eq. gs), J(g) = d/dg (a^2 |g|^2 / 2) (the variational form of the
 * anisotropic terms of Eq. pf2), the lambda coupling of Eq. lambda, the thermal
 * equation of Eq. temp1 with the latent rate of Eq. theta, and 3 Gauss points
 * per axis (Secs. 4.1, 4.2).  The mobility factor a^2 of the time term is taken
 * at the new state.
 *
 * Vector layout: every state, residual and direction vector is a DEVICE array
 * of 2 * n_nodes doubles, interleaved node-major: V[2*node + 0] = phi part,
 * V[2*node + 1] = u part, node = i + (n0+1) * (j + (n1+1) * k).  All such
 * arrays are owned by the caller (e.g. torch tensors), must be contiguous and
 * 16-byte aligned, and may not alias each other unless a function says so.
 *
 * Streams: every call enqueues its work on the caller's hipStream_t passed as
 * void* (NULL = default stream).  Calls marked [async] return after enqueue;
 * calls marked [sync] synchronise the stream because the host takes
 * decisions on device results (norms, Krylov coefficients).
 *
 * Errors: every function returns PF_OK (0) or a negative PF_ERR_* code;
 * pf_last_error() returns a thread-local description of the last failure.
 * Invalid arguments are detected on the host before anything is launched.
 *
 * Thread safety: a pf_problem handle is not thread-safe; use one per thread.
 */
#ifndef PFJFNK_H
#define PFJFNK_H

#ifdef __cplusplus
extern "C" {
#endif

#define PF_OK 0
#define PF_ERR_INVALID_ARG (-1)   /* null pointer, bad size, unsupported option */
#define PF_ERR_HIP (-2)           /* a HIP runtime call failed                   */
#define PF_ERR_NONFINITE (-3)     /* a residual norm became NaN or Inf           */
#define PF_ERR_NOT_CONVERGED (-4) /* Newton hit max_newton before Eq. tolerance  */
#define PF_ERR_LINEAR (-5)        /* FGMRES did not reach its tolerance          */
#define PF_ERR_LINESEARCH (-6)    /* no Lambda satisfied Eq. glob                */
#define PF_ERR_OOM (-7)           /* device allocation failed                    */

#define PF_JV_FD 0       /* (F(U + eps v) - F(U))/eps, Eq. JFmatvec           */
#define PF_JV_ANALYTIC 1 /* exact tangent of the residual                     */

#define PF_PC_NONE 0   /* M = I                                               */
#define PF_PC_JACOBI 1 /* M = diag of the blocks of Eq. pre                   */
#define PF_PC_GMG 2    /* one geometric V-cycle per block of Eq. pre          */

#define PF_FP64 0
#define PF_FP32 1

#define PF_MAX_LOG 64

/* Model and mesh.  dim = 2 or 3; n[k] >= 1 elements per axis (n[2] ignored
 * in 2-D); half_width[k] > 0.  dt > 0, D > 0, delta2 > 0 (regularises the
 * anisotropy where grad phi = 0, where Eq. gs is undefined; 1e-8 is the
 * default reading: a(g) is then smooth at the scale of the gradient
 * perturbations of FD products and of the FP32 preconditioner (about 1e-8),
 * which keeps Newton convergent at exactly symmetric states, and moves a on
 * the interface by about eps4 delta2/|grad phi|^2 ~ 1e-9.  Values near the
 * size of those perturbations, such as 1e-16, can stall Newton's line search
 * there); theta in
 * (0, 1]: the time weight of Eq. dpf (1 backward Euler, 1/2 the trapezoidal
 * or Crank-Nicolson rule).  order: Lagrange element order, 1 (bilinear /
 * trilinear; 0 is read as 1) or 2 (biquadratic, 2-D, free-growth model only):
 * order-2 meshes have 2 n[k] + 1 nodes per axis. */
typedef struct {
  int dim;
  int n[3];
  double half_width[3];
  double dt;
  double eps4;
  double lambda;
  double D;
  double delta2;
  double theta;
  int order;
} pf_params;

/* Newton-Krylov options (Sec. 2.2).  The forcing term follows Eqs. force1 to
 * forcing: eta_0 = eta0, eta_l = min(eta_max, max(gamma (|F_l|/|F_{l-1}|)^omega,
 * gamma eta_{l-1}^omega, eta_min)).  gmres_m is the restart length (<= the
 * value given to pf_create), gmres_maxit the total FGMRES iteration cap per
 * linear solve. */
typedef struct {
  double tau_r;
  double tau_a;
  int max_newton;
  int max_backtracks;
  int gmres_m;
  int gmres_maxit;
  double eta0;
  double eta_min;
  double eta_max;
  double gamma;
  double omega;
  int jv_mode;      /* PF_JV_FD or PF_JV_ANALYTIC */
  int pc;           /* PF_PC_NONE, PF_PC_JACOBI or PF_PC_GMG */
  int pc_precision; /* PF_FP64 or PF_FP32 (GMG only) */
} pf_solver_opts;

/* Statistics of one pf_newton_step / pf_linear_solve / pf_adjoint_step call.
 * t_total_ms is the host wall-clock time of the call's own work: a [sync]
 * call first drains the stream of what the caller queued before it, then
 * starts its clock. */
typedef struct {
  int status;
  int newton_its;
  int gmres_its_total;
  int backtracks;
  double f0;
  double f_final;
  int gmres_its[PF_MAX_LOG];
  double fnorm[PF_MAX_LOG + 1];
  double t_total_ms;
} pf_solver_stats;

typedef struct pf_problem pf_problem;

/* Fill opts with the paper's nonlinear-solver values (Sec. 4.1: eta0 = 0.1,
 * eta_min = 1e-6, eta_max = 0.01, omega = 1.5, gamma = 0.9, tau_a = 0) with
 * tau_r = 1e-10, FGMRES(30), at most 300 iterations per solve, 8 backtracks,
 * 30 Newton iterations, FD Jv, FP64 GMG.  Host only. */
void pf_default_opts(pf_solver_opts* opts);

/* Create a problem: validates params, allocates every device workspace the
 * other calls need (FGMRES basis for restart length gmres_m_max, multigrid
 * hierarchy, reduction buffers) on the current HIP device.  *out receives the
 * handle.  Returns PF_ERR_INVALID_ARG or PF_ERR_OOM on failure. */
int pf_create(const pf_params* params, int gmres_m_max, pf_problem** out);

/* Free the handle and its workspaces (synchronises the device). */
int pf_destroy(pf_problem* pb);

/* Replace the scalar model parameters (dt, eps4, lambda, D, delta2, theta) of an
 * existing handle; mesh fields of params must match the handle.  Host only. */
int pf_set_params(pf_problem* pb, const pf_params* params);

/* Number of nodes and of unknowns (2 * nodes) of the handle's mesh. */
long long pf_num_nodes(const pf_problem* pb);

/* [async] F = F(U; Uprev) - rhs, the part of the step residual above that
 * depends on U (Sec. 2.1.2, Eqs. dpf, dtemp; the whole residual when
 * theta = 1), less an optional load vector rhs (e.g. the volume and boundary
 * integrals of a manufactured solution; NULL for none).  The subtraction is one
 * rounding of the exact difference.  U, Uprev, rhs, F: device, 2*n_nodes
 * doubles.  F must not alias U, Uprev or rhs. */
int pf_residual(pf_problem* pb, const double* U, const double* Uprev, const double* rhs, double* F,
                void* stream);

/* [async] pf_residual without a handle and without any device allocation,
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  F =
 * F(U; Uprev) for the thermal model of params (order-1 elements, 2-D or 3-D),
 * bit for bit equal to pf_residual on a handle of the same params.  The
 * kernels' scratch (3-D: tile-face partial sums, 2-D: element vectors) is a
 * fixed array of 64 MiB inside the library, one copy per device, held from the
 * first call on that device until the process ends; its device address is
 * looked up on that first call.  Meshes whose scratch exceeds it -- beyond
 * 2727 tiles of 16^3 elements in 3-D (128^3 and 192^3 fit, 256^3 does not),
 * or 2^20 elements in 2-D (1024^2 fits) -- are rejected with
 * PF_ERR_INVALID_ARG before anything is launched.  All calls on one device share that array: calls that overlap in
 * time on one device (other streams or threads) race and must not be issued.
 * The array holds the last call's partial sums; nothing in it needs clearing.
 * U, Uprev, F: device, 2*n_nodes doubles; F must not alias U or Uprev. */
int pf_residual_noalloc(const pf_params* params, const double* U, const double* Uprev, double* F,
                        void* stream);

/* [async] E = E(Uprev, Uprev2), the part of the step residual fixed by the two
 * previous states (Eqs. dpf, dtemp and the lagged half of the rate of Eq.
 * theta); all zeros when theta = 1.  Uprev = U^n, Uprev2 = U^(n-1), E: device,
 * 2*n_nodes doubles; E must not alias the inputs. */
int pf_theta_explicit(pf_problem* pb, const double* Uprev, const double* Uprev2, double* E,
                      void* stream);

/* [async] Jacobian-vector product Jv = F'(U) v (Sec. 2.2).
 * mode PF_JV_FD: Jv = (F(U + eps v) - F0)/eps (Eq. JFmatvec) with
 *   eps = sqrt(2^-52) (1 + |U|_2)/|v|_2 computed on the device; F0 must be
 *   F(U; Uprev) (computed internally when F0 is NULL).
 * mode PF_JV_ANALYTIC: the exact tangent of the residual; F0 is ignored.
 * v == 0 gives Jv = 0.  Jv must not alias the inputs. */
int pf_jvp(pf_problem* pb, const double* U, const double* Uprev, const double* v,
           const double* F0, int mode, double* Jv, void* stream);

/* [async] Vector-Jacobian product of F(U; Uprev) (E held fixed) for the
 * cotangent w:
 *   gU     = (dF/dU)^T w         (may be NULL)
 *   gUprev = (dF/dUprev)^T w     (may be NULL)
 *   gparams[0] = w . dF/d eps4, gparams[1] = w . dF/d lambda  (device, 2
 *   doubles; may be NULL).  Reductions are deterministic.  With gU NULL a 3-D
 *   call runs a lighter kernel that forms gUprev and gparams only (no
 *   Hessian-vector product of the anisotropic flux); its results equal those
 *   of a call with gU to rounding.  With gU alone (gUprev and gparams NULL)
 *   the call runs the kernel of the transposed Krylov operator. */
int pf_vjp(pf_problem* pb, const double* U, const double* Uprev, const double* w,
           double* gU, double* gUprev, double* gparams, void* stream);

/* [async] Build the preconditioner of Eq. pre at the state U: the blocks
 * M11 = (1/dt)(c psi_j, psi_i) + theta (c grad psi_j, grad psi_i) with c the
 * cell mean of a(grad phi)^2 (Eqs. m11, pref2 with k = 1) and
 * M22 = (1/dt)(psi_j, psi_i) + theta D (grad psi_j, grad psi_i) (Eqs. m22,
 * preconc2).  kind: PF_PC_NONE, PF_PC_JACOBI, PF_PC_GMG; precision PF_FP64 or
 * PF_FP32 (the GMG V-cycle's arithmetic; Jacobi is always FP64).  The first
 * GMG set-up of a precision allocates its level hierarchy (about 1.2 x 5
 * vectors of the grid in that precision, plus the cell coefficients and the
 * diagonal) and may return PF_ERR_OOM.  The environment variable
 * PF_GMG_TILE_GROUPS (a positive integer, read at that allocation) sets the
 * workgroup target of the tiled 3-D smoothers' z-march (default 4096); it
 * changes the work split, not the result. */
int pf_precond_setup(pf_problem* pb, const double* U, int kind, int precision, void* stream);

/* [async] z = M^-1 r with the preconditioner of the last pf_precond_setup
 * (Jacobi: diagonal scaling; GMG: one V-cycle per block).  M^-1 is linear and
 * symmetric.  z must not alias r.  On meshes of at most 2^20 unknowns the
 * V-cycle is captured once as a HIP graph (on a stream the handle owns) and
 * replayed between copies into and out of two handle-owned vectors, allocated
 * on the first such apply (PF_ERR_OOM if they do not fit); the result is the
 * same bit for bit.  The environment variable PF_GMG_GRAPH=0, read by
 * pf_create, keeps eager launches. */
int pf_precond_apply(pf_problem* pb, const double* r, double* z, void* stream);

/* [sync] Solve F'(U) x = b (transpose = 0) or F'(U)^T x = b (transpose = 1)
 * by right-preconditioned FGMRES with the preconditioner already set up, to
 * |b - A x| <= rtol |b| starting from x = 0.  The transposed solve uses the
 * VJP as its operator (opts->jv_mode is then ignored).  Returns PF_ERR_LINEAR
 * when opts->gmres_maxit iterations do not reach rtol (x holds the last
 * iterate). */
int pf_linear_solve(pf_problem* pb, const double* U, const double* Uprev, const double* b,
                    double* x, int transpose, double rtol, const pf_solver_opts* opts,
                    pf_solver_stats* stats, void* stream);

/* [sync] Newton-Krylov (Sec. 2.2) for F(U; Uprev) = 0 (one backward-Euler
 * step when theta = 1) starting from U_inout, with the forcing term, the
 * backtracking of Eq. glob (Lambda halved up to max_backtracks times), the
 * termination test of Eq. tolerance and the preconditioner rebuilt at every
 * Newton iterate.  On success U_inout holds the solution.  On failure it holds
 * the last accepted iterate and the code says why. */
int pf_newton_step(pf_problem* pb, const double* Uprev, double* U_inout,
                   const pf_solver_opts* opts, pf_solver_stats* stats, void* stream);

/* [sync] One theta-method step: as pf_newton_step for
 * F(U; Uprev) + E(Uprev, Uprev2) = 0, with E built internally (see
 * pf_theta_explicit; the handle keeps one extra 2*n_nodes workspace for it,
 * allocated on first use when theta < 1).  With theta = 1 it is
 * pf_newton_step and Uprev2 is not read. */
int pf_newton_step_theta(pf_problem* pb, const double* Uprev2, const double* Uprev,
                         double* U_inout, const pf_solver_opts* opts, pf_solver_stats* stats,
                         void* stream);

/* [sync] steps theta-method steps (backward Euler when theta = 1) from
 * states[0]: states is a device array of (steps + 1) * 2 * n_nodes doubles
 * holding U^0 on entry; on return states[k] = U^k (the checkpoints of the
 * adjoint).  Each step starts Newton from the previous state; the first step
 * takes U^(-1) = U^0.  stats (optional) receives the last step's statistics
 * with gmres_its_total and newton_its summed over steps. */
int pf_evolve(pf_problem* pb, double* states, int steps, const pf_solver_opts* opts,
              pf_solver_stats* stats, void* stream);

/* [sync] One step of the discrete adjoint of backward-Euler stepping, for the
 * step U = U^k from Uprev = U^{k-1}:  solve F'(U)^T lam = mu by FGMRES with
 * the preconditioner rebuilt at U, then
 *   mu_prev = -(dF/dUprev)^T lam       (device, 2*n_nodes; may be NULL)
 *   gparams[0..1] -= (lam . dF/d eps4, lam . dF/d lambda)   (device, 2 doubles)
 * lam (device, 2*n_nodes) receives the multiplier.  rtol = opts->tau_r.
 * Requires theta = 1 (PF_ERR_INVALID_ARG otherwise). */
int pf_adjoint_step(pf_problem* pb, const double* U, const double* Uprev, const double* mu,
                    double* lam, double* mu_prev, double* gparams, const pf_solver_opts* opts,
                    pf_solver_stats* stats, void* stream);

/* [sync] Adjoint solve of Sec. 2.2's Jacobian: F'(U)^T lam = rhs (E held
 * fixed, any theta) by right-preconditioned FGMRES with the transposed
 * residual-family kernel as operator and the preconditioner of Eq. pre
 * (symmetric, so it serves the transposed system unchanged) set up at U with
 * opts->pc and opts->pc_precision, to |rhs - F'(U)^T lam| <= opts->tau_r |rhs|
 * from lam = 0.  U, Uprev, rhs, lam: device, 2*n_nodes doubles; lam must not
 * alias the inputs.  PF_ERR_LINEAR when opts->gmres_maxit iterations do not
 * reach the tolerance (lam holds the last iterate). */
int pf_adjoint_solve(pf_problem* pb, const double* U, const double* Uprev, const double* rhs,
                     double* lam, const pf_solver_opts* opts, pf_solver_stats* stats, void* stream);

/* [async] Misfit of the phase field against a target:
 *   L = 1/2 sum_i m_i (phi_i - phi*_i)^2 with the lumped nodal mass
 *   m_i = integral of psi_i;  *L_dev (device double) receives L and dLdU
 *   (device, 2*n_nodes) the gradient (zero u part).  phi_target: device,
 *   n_nodes doubles. */
int pf_misfit(pf_problem* pb, const double* U, const double* phi_target, double* L_dev,
              double* dLdU, void* stream);

/* [async] Deterministic dot product *out_dev = x . y over 2*n_nodes entries
 * (device result).  Exposed for tests of the reduction kernels. */
int pf_dot(pf_problem* pb, const double* x, const double* y, double* out_dev, void* stream);

/* ------------------------------------------------------------------------
 * Alloy model: directional solidification of a dilute binary alloy (Sec. 4.3,
 * Eqs. pf2, lambda, directional, conc2, jat, with the weight theta of Eq.
 * theta).  u is the non-dimensional solute field, cu = 1 + (1 - k) u, and the
 * part of the step residual that depends on the new state U is
 *
 *   F1_i = (cu a^2 (phi - phi^n)/dt, psi_i) + theta (J(grad phi), grad psi_i)
 *          - theta (phi - phi^3 - lambda (1 - phi^2)^2 (u + G4(x, t)), psi_i)
 *   F2_i = ((1 + k)/2 (u - u^n)/dt, psi_i) + theta (D (1 - phi)/2 grad u, grad psi_i)
 *          + (cu phihat grad phi / (2 sqrt(2) |grad phi|), grad psi_i) - (phihat cu / 2, psi_i)
 *
 * with phihat = theta (phi - phi^n)/dt + (1 - theta)(phi^n - phi^(n-1))/dt
 * (Eq. theta), the frozen temperature G4(x, t) = (x - x_iso - v_pull t)/l_T
 * (Eq. directional, x = mesh coordinate along axis 0) and |grad phi| taken as
 * sqrt(|grad phi|^2 + delta2).  The part fixed by U^n is
 *   E = (1 - theta) [ (J(grad phi^n), grad psi) - (G3(phi^n)(u^n + G4(x, t^n)), psi) ;
 *                     (D (1 - phi^n)/2 grad u^n, grad psi) ].
 * The anisotropy, dt, theta, lambda, D, delta2 come from pf_params.  The
 * preconditioner keeps the block form of Eq. pre with the phi block
 * (1/dt) M_c + theta K_c (c = cell mean of cu a^2, the mobility factor of the
 * time term) and the u block
 * (1+k)/(2 dt) M + theta D K (the one-sided mobility taken as its liquid
 * value).  A handle switched to this model accepts only the pf_alloy_* calls
 * below, pf_precond_setup/apply, pf_misfit and pf_dot; no VJP or adjoint.
 * ------------------------------------------------------------------------ */
typedef struct {
  double k;      /* partition coefficient, 0 < k <= 1 */
  double l_T;    /* thermal length in units of W0, > 0 (+inf: no gradient) */
  double x_iso;  /* isotherm position at t = 0 (mesh coordinate along axis 0) */
  double v_pull; /* pulling speed in units of W0/tau0 */
} pf_alloy_params;

/* Switch the handle to the alloy model (host; allocates the history field
 * and, in 3-D, the element buffer of the two-pass element kernels:
 * 16 * 8 bytes per element).  PF_ERR_INVALID_ARG on bad parameters,
 * PF_ERR_OOM when the buffers do not fit. */
int pf_set_alloy(pf_problem* pb, const pf_alloy_params* alloy);

/* [async] F = implicit part of the alloy step at time t (= t^{n+1}) from
 * Uprev = U^n and Uprev2 = U^(n-1).  All vectors: device, 2*n_nodes doubles. */
int pf_alloy_residual(pf_problem* pb, const double* U, const double* Uprev, const double* Uprev2,
                      double t, double* F, void* stream);

/* [async] E = part of the alloy step fixed by Uprev = U^n at time t_prev = t^n. */
int pf_alloy_explicit(pf_problem* pb, const double* Uprev, double t_prev, double* E, void* stream);

/* [async] Jv of the implicit part (modes as pf_jvp: PF_JV_FD with F0 the
 * implicit part at U, or NULL; PF_JV_ANALYTIC exact, by forward-mode
 * differentiation of the pointwise terms). */
int pf_alloy_jvp(pf_problem* pb, const double* U, const double* Uprev, const double* Uprev2,
                 double t, const double* v, const double* F0, int mode, double* Jv, void* stream);

/* [sync] One alloy step from t_prev: Newton-Krylov as pf_newton_step on
 * F(U) + E = 0 starting from U_inout (usually a copy of Uprev). */
int pf_alloy_step(pf_problem* pb, const double* Uprev2, const double* Uprev, double t_prev,
                  double* U_inout, const pf_solver_opts* opts, pf_solver_stats* stats, void* stream);

/* [sync] steps alloy steps from states[0] at time t0 (layout as pf_evolve;
 * the first step takes U^(-1) = U^0). */
int pf_alloy_evolve(pf_problem* pb, double* states, int steps, double t0,
                    const pf_solver_opts* opts, pf_solver_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Free-growth model: a pure melt with phi in [0, 1] (1 solid) and temperature
 * T (Sec. 4.1, Eqs. pf1, g1, gs, temp1, with the weight theta of Eq. theta),
 * on order-1 or order-2 elements.  The part of the step residual that depends
 * on the new state U = (phi, T) is
 *
 *   F1_i = (a^2 (phi - phi^n)/dt, psi_i) + theta beta Gamma (J(grad phi), grad psi_i)
 *          + theta (G2(phi, T), psi_i)
 *   F3_i = ((T - T^n)/dt, psi_i) + theta alpha (grad T, grad psi_i) - (Lcp phihat, psi_i)
 *   G2   = beta Gamma phi (1 - phi)(1 - 2 phi)/W^2 - 5 beta (Tm - T) phi^2 (1 - phi)^2 / W
 *
 * with a, J of the thermal model (eps4, delta2 from pf_params), phihat of Eq.
 * theta, and E = (1 - theta) times the spatial terms at U^n.  The second
 * field of every vector is T.  The preconditioner is Eq. pre with the blocks
 * of Eqs. m11 and m22: (1/dt) M_c + theta beta Gamma K_c (c = cell mean of
 * a^2) and (1/dt) M + theta alpha K; on order-2 meshes it is the order-1
 * operator on the grid of order-2 nodes (each element split into 2^dim
 * cells), a spectrally equivalent stand-in.  pf_params.D and lambda are not
 * used by this model.  A handle switched to it accepts only the pf_fg_* calls,
 * pf_precond_setup/apply, pf_dot.
 * ------------------------------------------------------------------------ */
typedef struct {
  double beta;   /* kinetic coefficient */
  double Gamma;  /* 1/beta in the paper's table; > 0 */
  double W;      /* interface width, > 0 */
  double alpha;  /* thermal diffusivity, > 0 */
  double Lcp;    /* latent heat over heat capacity */
  double Tm;     /* melting temperature */
} pf_freegrowth_params;

/* Switch the handle to the free-growth model (host; allocates the history
 * field and the element buffer, 16 (order 1, 2-D), 16 (order 1, 3-D: 8
 * corners) or 18 (order 2) doubles per element).  PF_ERR_INVALID_ARG,
 * PF_ERR_OOM. */
int pf_set_freegrowth(pf_problem* pb, const pf_freegrowth_params* fg);

/* [async] F = implicit part from Uprev = U^n and Uprev2 = U^(n-1). */
int pf_fg_residual(pf_problem* pb, const double* U, const double* Uprev, const double* Uprev2,
                   double* F, void* stream);

/* [async] E = part of the step fixed by Uprev = U^n. */
int pf_fg_explicit(pf_problem* pb, const double* Uprev, double* E, void* stream);

/* [async] Jv of the implicit part (modes as pf_jvp; the analytic product is
 * forward-mode differentiation of the pointwise terms on dual numbers). */
int pf_fg_jvp(pf_problem* pb, const double* U, const double* Uprev, const double* Uprev2,
              const double* v, const double* F0, int mode, double* Jv, void* stream);

/* [sync] One theta step (Newton-Krylov on F + E = 0 from U_inout). */
int pf_fg_step(pf_problem* pb, const double* Uprev2, const double* Uprev, double* U_inout,
               const pf_solver_opts* opts, pf_solver_stats* stats, void* stream);

/* [sync] steps theta steps from states[0] (layout as pf_evolve; the first
 * step takes U^(-1) = U^0). */
int pf_fg_evolve(pf_problem* pb, double* states, int steps, const pf_solver_opts* opts,
                 pf_solver_stats* stats, void* stream);

/* Thread-local message describing the last error ("" if none). */
const char* pf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PFJFNK_H */
