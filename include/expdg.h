/*
 * expdg.h -- C ABI of the MI355X (gfx950) exponential-DG library.
 *
 * The library evaluates the hot path of the exponential DG method of Kang &
 * Bui-Thanh ("A scalable exponential-DG approach for nonlinear conservation
 * laws: with application to Burger and Euler equations"):
 *
 *   q_t + div F(q) = 0 on a uniform periodic mesh (Section 2.2, eq. pde),
 *   DG semi-discretization dq/dt = R(q) = L q + N(q) with LGL collocation and
 *   Lax-Friedrichs / Rusanov numerical fluxes (Section 2.2,
 *   eq. EXPO-SemiDiscretizedForm_ode; Sections 3.1 and 3.2), and viscous
 *   Burgers u_t + (u^2/2)_x = kappa u_xx + s (Section 3.1, eqs.
 *   gov-burgers1d-gradu and Burger) with central or LDG diffusion fluxes
 *   (Appendix A), the entropy flux, and zero Dirichlet ends,
 *   phi-function combinations sum_k tau^k phi_k(tau L) b_k by Krylov
 *   projection of the augmented matrix (Section 2.3,
 *   eq. linear_combination_of_phifunctions), and
 *   the exponential steppers EPI2 and EXPRB32 (footnotes of Section 5.1),
 *   EXPRB42 (footnote of Section 5.2) and Tokman's EPI3 (cited in Section 1).
 *
 * Every compute step runs in HIP kernels on the device.  All entry points are
 * plain C: pointers and sizes, no C++ or framework types.
 *
 * Nodal layout of every state vector (device memory):
 *     idx = (c * K + e) * Np + n,   c = variable, e = (ez * ny + ey) * nx + ex,
 *     n = (k * (p + 1) + j) * (p + 1) + i  (i along x, j along y, k along z),
 * Burgers: one variable u.  Euler 2D: (rho, rho u, rho v, rho E).  Euler 3D:
 * (rho, rho u, rho v, rho w, rho E) (the system of Section 3.2 with three
 * velocity components; the extruded problem of Section 5.2).
 * Np = (p + 1)^dim; K = nx * ny * nz; ndof = nvar * K * Np.
 *
 * Precision: in EXPDG_FP64 every buffer is double.  In EXPDG_FP32_BULK the
 * operator buffers of expdg_rhs / expdg_jvp / expdg_phi_krylov are float and
 * the Krylov basis is stored in float, while inner products, norms, the
 * Hessenberg matrix, its exponential and the controller stay in double, and
 * expdg_step keeps its state q in double.  The operators compute in double in
 * both modes and round only what they store; expdg_step / expdg_integrate
 * form every residual, the frozen fields of the linear operator and the stage
 * differences from the double states (a float copy of the state would put
 * its rounding into each residual as high-frequency noise), so FP32_BULK
 * steps take the FP64 Krylov iteration counts at the same tolerance.
 *
 * Ownership: the caller owns every state, input and output buffer; the mesh
 * owns its geometry tables and the Krylov workspace, allocated once by
 * expdg_mesh_create (sized by m_max) and released by expdg_mesh_destroy.  No
 * entry point allocates device memory after creation.
 *
 * Streams: hip_stream is a hipStream_t passed as void* (NULL = the null
 * stream).  expdg_rhs and expdg_jvp are asynchronous on that stream.
 * expdg_phi_krylov and expdg_step return after the work has completed, so
 * their statistics are valid on return.
 *
 * Errors: every entry point returns EXPDG_OK (0) or a negative status and
 * never throws.  Arguments are validated before anything is launched; on
 * EXPDG_EINVAL outputs are untouched.  On EXPDG_ENOCONV / EXPDG_ENONFINITE
 * the output is undefined and the mesh stays usable.  expdg_last_error()
 * returns a thread-local description of the last failure.  A mesh handle may
 * be used by one host thread at a time.
 */
#ifndef EXPDG_H
#define EXPDG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { EXPDG_BURGERS1D = 1, EXPDG_EULER2D = 2, EXPDG_EULER3D = 3 };
enum { EXPDG_FP64 = 0, EXPDG_FP32_BULK = 1 };
enum { EXPDG_EPI2 = 2, EXPDG_EPI3 = 3, EXPDG_EXPRB32 = 32, EXPDG_EXPRB42 = 42 };
enum { EXPDG_FLUX_LF = 0, EXPDG_FLUX_EF = 1, EXPDG_FLUX_EF_LOCAL = 2 };
enum { EXPDG_BC_PERIODIC = 0, EXPDG_BC_DIRICHLET = 1, EXPDG_BC_WALL_Y = 2 };
enum {
    EXPDG_OK = 0,
    EXPDG_EINVAL = -1,     /* invalid argument */
    EXPDG_ENOMEM = -2,     /* device allocation failed */
    EXPDG_EDEVICE = -3,    /* HIP runtime error */
    EXPDG_ENOCONV = -4,    /* Krylov substep fell below its floor */
    EXPDG_ENONFINITE = -5  /* non-finite norm, Hessenberg entry or state */
};

/* Mesh description.  Uniform mesh: nx intervals on [x0, x1] (Burgers,
 * ny = 1), nx x ny periodic quadrilaterals on [x0, x1] x [y0, y1] (Euler 2D),
 * or nx x ny x nz periodic hexahedra on [x0, x1] x [y0, y1] x [z0, z1]
 * (Euler 3D; nz, z0, z1 are read only there).  p is the LGL degree (1..6).  m_max bounds the Krylov basis (1..64).  gamma
 * is used by Euler only.
 *
 * Burgers options (Section 3.1; all zero = inviscid, periodic,
 * Lax-Friedrichs; Euler requires them zero, except bc below):
 *   kappa  viscosity >= 0.  With kappa > 0 the flux is u^2/2 - kappa q with
 *          the auxiliary q = u_x of eq. gov-burgers1d-gradu, and all of the
 *          diffusion belongs to the linear operator L (eq. BurgerL);
 *   flux   EXPDG_FLUX_LF, EXPDG_FLUX_EF or EXPDG_FLUX_EF_LOCAL: the
 *          numerical flux (u^2/2)* of the residual; EF is (1/3)({{u^2/2}} +
 *          {{u}}^2) + (sigma/h)[[u]] with h the half-width h_e/2 of an
 *          element; EF_LOCAL takes sigma = kappa/100 + h max|u^+-| at each
 *          face (the steep-gradient example of Section 5.1; sigma is then
 *          not read).  The linear flux (u~ u)* is always Lax-Friedrichs;
 *   beta   diffusion fluxes u** = {{u}} - beta [[u]], q** = {{q}} + beta [[q]]
 *          with [[v]] = v_left - v_right: 0 central (Section 3.1), 1/2 LDG
 *          (Appendix A); |beta| <= 1/2;
 *   bc     EXPDG_BC_PERIODIC, or EXPDG_BC_DIRICHLET: u = 0 at x0 and x1, taken
 *          as in the footnote at the start of Section 6 (exterior state 0 in
 *          the convective fluxes, u** = 0, q** = q^-);
 *   has_source  nonzero: the mesh holds a source vector s added to R (not to
 *          L), set by expdg_mesh_set_source (zero until then).
 *
 * Euler 2D boundaries (bc): EXPDG_BC_PERIODIC, or EXPDG_BC_WALL_Y: periodic in
 * x, no-slip walls at y0 and y1 (the Kelvin-Helmholtz problem of Section 5.3).
 * At a wall face node the exterior state is the mirror M q = (rho, -rho u,
 * -rho v, rho E) in the Rusanov flux of R, and M v at the mirrored reference
 * state in L; with entropy viscosity the gradient takes (v + M v)/2 on the
 * wall and the diffusive flux through it is the interior one for the momenta
 * and zero for density and energy; the face jump of u S . n is 2 |v S| and a
 * wall vertex averages its two elements.
 *
 * Entropy viscosity (Euler 2D only; Section 3.2, "Artificial viscosity"):
 *   ev_ce, ev_cmax  the constants c_E and c_max (both >= 0; the paper takes 1
 *          and 0.1).  With ev_ce > 0 the mesh holds a nodal viscosity nu
 *          (bulk precision, zero at creation) and both operators gain the
 *          linear diffusion div(nu grad v) of each conserved variable, with
 *          central fluxes: F^EV = nu grad q in R, nu grad v in L.  Every step
 *          (expdg_step, expdg_integrate) first sets nu from q^n and q^{n-1}
 *          (q^n again when it has no history) as expdg_entropy_viscosity does;
 *          expdg_rhs, expdg_jvp and expdg_phi_krylov use nu as it stands. */
typedef struct {
    int equation;   /* EXPDG_BURGERS1D, EXPDG_EULER2D or EXPDG_EULER3D */
    int nx, ny;
    int p;
    int precision;  /* EXPDG_FP64 or EXPDG_FP32_BULK */
    int device;     /* HIP device ordinal */
    double x0, x1, y0, y1;
    double gamma;
    int m_max;
    double kappa;
    int flux;
    double sigma;
    double beta;
    int bc;
    int has_source;
    int nz;
    double z0, z1;
    double ev_ce, ev_cmax;
} expdg_mesh_desc;

typedef struct expdg_mesh expdg_mesh; /* opaque, library-owned */

/* Sizes of a created mesh. */
typedef struct {
    size_t ndof;       /* nvar * K * Np */
    int nvar, K, Np;
    int elem_bytes;    /* 8 (FP64) or 4 (FP32_BULK) for operator buffers */
    double hx, hy;     /* element sizes */
    double dx_min;     /* smallest LGL node spacing in physical units */
    double hz;         /* element size along z (3D; 1 otherwise) */
} expdg_mesh_info;

/* One accepted Krylov substep: basis size m, substep length dtau, last != 0
 * when it completes its phi evaluation. */
typedef struct {
    int m;
    int last;
    double dtau;
} expdg_substep;

/* Krylov controller options (Section 2.3; the paper runs an adaptive Krylov
 * method with unreported parameters, so the controller is fixed here):
 * error checked at m_min and every check_every iterations after it; tol is
 * relative to nu = ||b_0|| + sum_k tau^k ||b_k|| / k!.  If n_forced > 0 the
 * substeps in forced[] are replayed with no error checks (m_max is then
 * ignored except as the workspace bound). */
typedef struct {
    double tol;
    int m_min, m_max, check_every;
    const expdg_substep *forced;
    int n_forced;
    int iop;  /* 0: full orthogonalization (classical Gram-Schmidt applied
                 twice); L in 1..64: incomplete orthogonalization, each new
                 vector against the L most recent basis vectors only (one
                 pass, explicit norm), the IOP option of KIOPS (Section 2.3).
                 Served solves take it from their request. */
    int adapt;  /* 0: the fixed controller above.  1: cost-based choice of the
                   Krylov size and the substep (after KIOPS, Section 2.3): the
                   error is checked only at the target size m of a substep, as
                   omega = err tau / (tol nu dtau) (accepted when <= 1); after
                   each check, keeping m with dtau scaled by
                   clamp((0.8/omega)^(1/q), 0.2, 5) (0.9 at most after a
                   rejection) and keeping dtau (capped to R) with m moved by
                   ln(omega'/0.8)/ln(kappa), omega' = omega (min(dtau, R) /
                   dtau)^q (within [m_min, min(m_max, 4m/3)]) are priced at
                   ceil(R/dtau') substeps of m'^2 + 9m' state-vector passes
                   each (m'(2L + 7) with a window of L), R the interval left,
                   and the cheaper one is taken (omega rounded up to a power of
                   10^(1/4), q and kappa to two significant digits).  q (the order of omega in
                   dtau) starts at m and
                   kappa (the gain of one more vector) at 2, and both are
                   re-estimated from two checks of the same substep.  A
                   rejection either re-checks the same basis with the shorter
                   substep or extends the Arnoldi process. */
    int m_init; /* adapt = 1: first target size (0: m_min) */
} expdg_krylov_opts;

/* Statistics, accumulated over the call (zero them before the call).  If
 * log != NULL accepted substeps are appended while log_len < log_cap
 * (log_len counts all of them). */
typedef struct {
    int substeps, rejects, krylov_iters, jvps, breakdown, phi_calls, rhs_calls;
    double err_est;
    expdg_substep *log;
    int log_cap, log_len;
    int checks;  /* small exponentials evaluated (error checks) */
    int m_next;  /* adapt = 1: the Krylov size chosen for a next substep */
} expdg_krylov_stats;

/* ---- mesh -------------------------------------------------------------- */

/* Create a mesh on desc->device: builds the LGL tables (Section 4 opening:
 * LGL quadrature), allocates the Krylov workspace.  *out receives the
 * handle.  EXPDG_EINVAL for an invalid description, EXPDG_ENOMEM if the
 * workspace does not fit. */
int expdg_mesh_create(const expdg_mesh_desc *desc, expdg_mesh **out);
int expdg_mesh_destroy(expdg_mesh *m);
/* Device bytes expdg_mesh_create would allocate for desc (0 if invalid). */
size_t expdg_workspace_bytes(const expdg_mesh_desc *desc);
int expdg_mesh_get_info(const expdg_mesh *m, expdg_mesh_info *info);
/* Physical node coordinates, host arrays of K*Np doubles (y, z may be NULL;
 * coordinates a mesh does not have are written as 0). */
int expdg_mesh_nodes(const expdg_mesh *m, double *x, double *y, double *z);
/* Copies the source term of a mesh created with has_source: s is a device
 * array of ndof doubles (the nodal values of the source of Section 5.1's
 * manufactured solutions), stored in the mesh in its bulk precision.
 * Asynchronous on hip_stream; s may be reused once the stream has passed the
 * copy.  EXPDG_EINVAL without has_source or with s == NULL. */
int expdg_mesh_set_source(expdg_mesh *m, const double *s, void *hip_stream);
/* Entropy viscosity of the state q after q_prev, one step dt apart (Section
 * 3.2, "Artificial viscosity", with the entropy residual of its footnote):
 * S = rho/(gamma-1) log(p / rho^gamma), Res = (S(q) - S(q_prev))/dt +
 * (div(u S)(q) + div(u S)(q_prev))/2 from each element's own derivative;
 * per element, with h = sqrt(hx^2 + hy^2)/p (twice the circumradius over the
 * degree), nu_E = c_E h^2 max(max |Res|, max |[[u S . n]]| / h) over its nodes
 * and faces, nu_max = c_max h max(|u . e_d| + a), nu_e = min(nu_max, nu_E);
 * each vertex averages its four elements and nu at a node is the bilinear
 * interpolant of its element's vertex values.  q, q_prev: device arrays of
 * ndof doubles (conserved variables, rho > 0, p > 0); the result becomes the
 * mesh's nu and, if nu != NULL, is also written to nu (device, K*Np doubles,
 * one per node).  Asynchronous on hip_stream.  EXPDG_EINVAL unless the mesh
 * was created with ev_ce > 0, for dt <= 0 or NULL q / q_prev. */
int expdg_entropy_viscosity(expdg_mesh *m, const double *q, const double *q_prev, double dt,
                            double *nu, void *hip_stream);
/* Sets the mesh's nodal viscosity to nu (device, K*Np doubles; stored in the
 * bulk precision), for operators outside a step.  Asynchronous on
 * hip_stream.  EXPDG_EINVAL unless the mesh was created with ev_ce > 0. */
int expdg_mesh_set_viscosity(expdg_mesh *m, const double *nu, void *hip_stream);
/* The library's LGL reference element: nodes, weights, and the
 * differentiation matrix D[i*(p+1)+j] = l_j'(xi_i); host arrays. */
int expdg_lgl(int p, double *xi, double *w, double *D);

/* ---- operators (Section 2.2; Sections 3.1 and 3.2) ---------------------- */

/* r = R(q): full DG residual with Lax-Friedrichs / Rusanov flux, lambda =
 * max(|u^-|, |u^+|) (Burgers) or max(|u.n| + a) over the two traces
 * (Euler).  q, r: device buffers of ndof bulk-type elements. */
int expdg_rhs(expdg_mesh *m, const void *q, void *r, void *hip_stream);

/* w = L(qref) v: the DG operator of the linear flux F_L = A(qref) v (eq.
 * linearflux; Burgers F_L = u~ v, Euler the flux Jacobian of Section 3.2),
 * with the numerical flux dissipation frozen at qref.  Device buffers of
 * ndof bulk-type elements; v and w must not alias. */
int expdg_jvp(expdg_mesh *m, const void *qref, const void *v, void *w, void *hip_stream);

/* Allocation-free linear operator, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): w = L(qref) v exactly as expdg_jvp computes it on a mesh
 * created from *desc (bitwise the same result), without a mesh handle.  The
 * frozen fields of the Euler operators (velocities, enthalpy and face wave
 * speeds of qref) are kept in a static device array of
 * EXPDG_NOALLOC_SCRATCH_MIB MiB that every GPU the library runs on holds until
 * the process ends; meshes whose frozen fields need more are rejected with
 * EXPDG_EINVAL (in FP64 about 0.85 * ndof * 8 bytes at p = 4: up to roughly
 * 9.8 million DOF).  The description is validated as for expdg_mesh_create
 * (m_max is not used); entropy viscosity (ev_ce > 0) needs a mesh and is
 * rejected.  The call allocates nothing: no hipMalloc, no hipFree, no events
 * or streams.  Asynchronous on hip_stream.  All calls on one GPU share its
 * scratch array, so calls that overlap on one GPU (other streams, other host
 * threads) race; the array keeps the last call's contents, and nothing in it
 * needs to start at zero (each call writes the fields before reading them). */
enum { EXPDG_NOALLOC_SCRATCH_MIB = 64 };
int expdg_jvp_noalloc(const expdg_mesh_desc *desc, const void *qref, const void *v, void *w,
                      void *hip_stream);

/* Largest wave speed max(|u|) or max(|u.n| + a) over the nodes of q
 * (device, FP64 state) into *cmax (host); synchronous.  Used for the CFL
 * time step dt = Cr dx_min / c (Courant number of Section 5). */
int expdg_max_speed(expdg_mesh *m, const double *q, double *cmax, void *hip_stream);

/* ---- phi combinations (Section 2.3) ------------------------------------- */

/* w = sum_{k=0}^{p} tau^k phi_k(tau L(qref)) b_k, 0 <= p <= 3, by adaptive
 * Arnoldi (classical Gram-Schmidt, two passes, FP64 inner products) on the
 * augmented matrix [[L, W], [0, J]].  b is a host array of p+1 device
 * pointers (NULL entries are zero vectors); qref, b[k] and w are bulk-type
 * device buffers of ndof elements.  Returns after completion. */
int expdg_phi_krylov(expdg_mesh *m, const void *qref, double tau, int p,
                     const void *const *b, void *w, const expdg_krylov_opts *o,
                     expdg_krylov_stats *s, void *hip_stream);

/* ---- time step (footnotes of Section 5.1; EPI3 after Tokman) ------------ */

/* One step of size dt of scheme EXPDG_EPI2, EXPDG_EPI3, EXPDG_EXPRB32 or
 * EXPDG_EXPRB42 on the FP64 device state q (in/out).  EPI3 uses q_prev: when have_prev != 0
 * it holds q^{n-1} on entry; when have_prev == 0 the step is an EPI2 step.
 * With entropy viscosity (ev_ce > 0) every scheme uses it too: the step's
 * viscosity comes from q and, when q_prev != NULL and have_prev != 0, from
 * q_prev as q^{n-1} (otherwise from q alone).  If q_prev != NULL it receives
 * q^n on return (for every scheme).  Returns after completion. */
int expdg_step(expdg_mesh *m, int scheme, double dt, double *q, double *q_prev, int have_prev,
               const expdg_krylov_opts *o, expdg_krylov_stats *s, void *hip_stream);

/* nsteps >= 1 steps of size dt, the same as nsteps calls of expdg_step (the
 * first with have_prev as given, every later one with the history the step
 * before left in q_prev, which must then be non-NULL for EPI3), with bitwise
 * the same results, but the host waits for the device only once, at the end.
 * A forced substep schedule in o applies to every step.  The statistics
 * accumulate over the steps.  On an error the call returns at once with the
 * state as the failing step left it. */
int expdg_integrate(expdg_mesh *m, int scheme, double dt, int nsteps, double *q, double *q_prev,
                    int have_prev, const expdg_krylov_opts *o, expdg_krylov_stats *s,
                    void *hip_stream);

/* Exponential of a small dense matrix on the device with the same kernel the
 * Krylov controller uses for the projected Hessenberg matrix (diagonal Pade
 * (6,6) with scaling and squaring, Section 2.3).  A and E are row-major
 * n x n FP64 device buffers, 1 <= n <= 65; asynchronous on hip_stream.  E
 * is NaN if the Pade denominator is singular. */
int expdg_small_expm(int n, const double *A, double *E, void *hip_stream);

/* ---- live kernel timing ------------------------------------------------ */

/* Kernel classes that can be timed with HIP events recorded around each
 * launch on the launching stream. */
enum {
    EXPDG_K_RESIDUAL = 0,       /* DG residual R(q) */
    EXPDG_K_LINEAR = 1,         /* DG linear operator L(q~) v (+ augmented block) */
    EXPDG_K_GS_DOTS = 2,        /* Arnoldi dot pass after the 1D operator (the 2D operator carries it) */
    EXPDG_K_SMALLEXPM = 3,      /* exponential of the projected Hessenberg matrix */
    EXPDG_K_COMBINE = 4,        /* Krylov combine z = beta V F e_1 */
    EXPDG_K_GS_UPDATE = 5,      /* Arnoldi update sweep: second pass of the previous vector,
                                   first pass of the new one */
    EXPDG_K_GS_NORM = 6,        /* norm of a substep's start vector */
    EXPDG_K_GS_FINISH = 7,      /* fixed-order sums of the block partials (step finish) */
    EXPDG_K_EV_VISC = 8,        /* entropy viscosity: element viscosity and its nodal
                                   reconstruction (two launches per evaluation) */
    EXPDG_K_GS_FOLD = 9,        /* fold of long partial rows before the finish (operators of
                                   more than 1024 blocks) */
    EXPDG_K_NCLASSES = 10
};

/* Accumulated timing of one kernel class: launches, summed event-measured
 * duration, and summed algorithmic bytes (each input vector element read
 * once, each output element written once). */
typedef struct {
    long long launches;
    double total_ms;
    double bytes;
} expdg_kernel_profile;

/* Enable (enable != 0) or disable timing of kernel_class on mesh m; either
 * call resets its counters.  Timing adds two event records per launch of that
 * class only. */
int expdg_profile_enable(expdg_mesh *m, int kernel_class, int enable);
/* Read the counters of kernel_class (waits for the recorded events). */
int expdg_profile_read(expdg_mesh *m, int kernel_class, expdg_kernel_profile *out);

/* ------------------------------------------------------------------------
 * Solve server: many independent solves share the device.
 *
 * A pattern on top of the method (the paper runs one solve at a time).  Each
 * submitted request is a whole time integration: nsteps steps of EPI2 or EPI3
 * (FP64) from the initial state q0 on its own mesh, with the adaptive Krylov
 * controller of expdg_step.  Requests are admitted in arrival order while
 * their device memory (expdg_request_bytes) fits the HBM budget given at
 * creation and fewer than max_active solves run; an admitted solve keeps its
 * state and Krylov workspace resident until it ends.  The server advances all
 * running solves together in ticks (expdg_server_tick): in one tick every
 * solve that is ready takes one Arnoldi step, and the same step of all of
 * them runs as grouped launches -- one linear-operator launch per (equation,
 * degree) and one launch per Gram-Schmidt pass over all solves -- while the
 * small Hessenberg exponentials of all solves that check their Krylov error in
 * that tick run as one batched launch on a second stream.  A solve gives the
 * same bits as expdg_step on its own mesh with the same options, whatever
 * else runs beside it.
 *
 * Threading: a server handle is used by one host thread at a time.  All host
 * buffers passed in are copied before the call returns.
 * ------------------------------------------------------------------------ */
typedef struct expdg_server expdg_server; /* opaque, library-owned */

typedef struct {
    expdg_mesh_desc mesh; /* precision must be EXPDG_FP64; device is ignored
                             (the server's device is used); no source term,
                             not 3D; entropy viscosity (ev_ce > 0) and walls as
                             for expdg_step, the viscosity of each step from
                             q^n and q^{n-1} (q^n on the first) for EPI2 and
                             EPI3 alike */
    int scheme;           /* EXPDG_EPI2 or EXPDG_EPI3 (first step EPI2) */
    int nsteps;           /* >= 1 */
    double dt;            /* > 0: the step; <= 0: cfl * dx_min / max wave speed of q0 */
    double cfl;           /* used when dt <= 0 (must then be > 0) */
    double tol;           /* Krylov options as in expdg_krylov_opts (no forced schedule) */
    int m_min, m_max, check_every;
    int iop;              /* 0: full orthogonalization; L in 1..64: incomplete (as in
                             expdg_krylov_opts.iop) */
    int adapt;            /* 0 or 1, as in expdg_krylov_opts.adapt */
} expdg_request;

enum {
    EXPDG_REQ_QUEUED = 0,    /* waiting for admission */
    EXPDG_REQ_ACTIVE = 1,    /* admitted, running */
    EXPDG_REQ_DONE = 2,      /* finished; the state can be fetched */
    EXPDG_REQ_FAILED = 3     /* stopped with an error (info.error) */
};

typedef struct {
    int state;               /* EXPDG_REQ_* */
    int error;               /* status of a failed solve, else EXPDG_OK */
    int steps_done;
    double dt;               /* the step used (after the cfl rule) */
    expdg_krylov_stats stats; /* accumulated over all steps; log is NULL */
    double t_submit, t_admit, t_done; /* seconds on the server clock (-1: not yet) */
    size_t bytes;            /* device memory the solve holds while running */
} expdg_request_info;

typedef struct {
    long long ticks;             /* ticks that launched work */
    long long grouped_launches;  /* grouped operator + Gram-Schmidt launches */
    long long batched_checks;    /* batched small-exponential launches */
    long long arnoldi_items;     /* Arnoldi steps run inside grouped launches */
    long long check_items;       /* checks run inside batched launches */
    int active, queued, done;
    size_t arena_bytes, arena_used, arena_peak;
} expdg_server_stats;

/* Device memory one request holds while running (workspace + states);
 * 0 if the request is invalid. */
size_t expdg_request_bytes(const expdg_request *r);
/* hbm_budget: bytes of device memory the server reserves at creation and
 * admits solves into; max_active: most solves running at once (1..4096). */
int expdg_server_create(int device, size_t hbm_budget, int max_active, expdg_server **out);
/* Waits for the device, releases everything (running solves are dropped). */
int expdg_server_destroy(expdg_server *s);
/* Queues a request with its initial state q0 (host, ndof doubles, copied).
 * EINVAL if it is invalid or can never fit the budget; *id identifies it. */
int expdg_server_submit(expdg_server *s, const expdg_request *r, const double *q0, long long *id);
/* Admits what fits, advances every ready solve and launches the tick's grouped
 * work.  block != 0: while fewer than 90 % of the running solves are ready and
 * earlier ticks are still on the device, first wait for the oldest of them
 * (so a tick carries most solves instead of running thin batches ahead of the
 * device), and if no solve is ready, wait until one is.  Returns the number of
 * solves that finished in this call in *finished (may be NULL). */
int expdg_server_tick(expdg_server *s, int block, int *finished);
/* Ids of solves finished (DONE or FAILED) since the last call, at most cap;
 * returns the count written (or a negative status). */
int expdg_server_finished(expdg_server *s, long long *ids, int cap);
int expdg_server_poll(expdg_server *s, long long id, expdg_request_info *info);
/* Copies the final state of a DONE solve to q_out (host, ndof doubles) and
 * releases the solve. */
int expdg_server_fetch(expdg_server *s, long long id, double *q_out);
/* Drops a request in any state (a running solve stops; its memory returns
 * to the budget once the device is done with it). */
int expdg_server_cancel(expdg_server *s, long long id);
/* Counters; memory of ended solves the device is done with is reclaimed first. */
int expdg_server_get_stats(expdg_server *s, expdg_server_stats *out);
/* Waits until the device has finished everything launched so far and
 * reclaims the memory of ended solves. */
int expdg_server_sync(expdg_server *s);
/* Seconds since the server was created (the clock of the info timestamps). */
double expdg_server_clock(const expdg_server *s);

/* Thread-local description of the last error (never NULL). */
const char *expdg_last_error(void);
/* ABI version: major * 10000 + minor * 100 + patch. */
int expdg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EXPDG_H */
