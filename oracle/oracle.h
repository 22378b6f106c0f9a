/*
 * oracle.h -- plain FP64 CPU oracle for the exponential-DG hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library,
 * its Python binding, the server) may include, link or call this code.  Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark use
 * it.  It shares no source with the GPU path.
 *
 * What it computes (Kang & Bui-Thanh, "A scalable exponential-DG approach for
 * nonlinear conservation laws"):
 *   - LGL reference element (LGL quadrature, Section 4 opening remarks)
 *   - nodal DG residual R(q) of q_t + div F(q) = 0 with Lax-Friedrichs /
 *     Rusanov numerical flux (Sections 3.1-3.2, Burgers LF flux and Euler
 *     system with the flux Jacobian A(q) of Section 3.2)
 *   - the linear operator L(q~) v of the flux-Jacobian split (eq. linearflux,
 *     eq. split-goveq-continuous), numerical flux dissipation frozen at q~
 *   - phi-function linear combinations sum_k tau^k phi_k(tau A) b_k
 *     (eq. linear_combination_of_phifunctions) by Krylov projection of the
 *     augmented matrix (Section 2.3), and densely for small systems
 *   - viscous Burgers (Section 3.1, eqs. gov-burgers1d, Burger): auxiliary
 *     q = u_x with central or LDG (Appendix A) diffusion fluxes, the entropy
 *     flux (EF) or Lax-Friedrichs for (u^2/2)*, zero Dirichlet ends as in the
 *     footnote at the start of Section 6, and a nodal source term
 *   - entropy viscosity for 2D Euler (Section 3.2, "Artificial viscosity"):
 *     entropy residual, element viscosity, vertex-averaged bilinear
 *     smoothing, and the linear diffusion div(nu grad q) with central fluxes
 *   - the exponential steppers EPI2, EXPRB32 (footnotes in Section 5.1),
 *     EXPRB42 (footnote in Section 5.2) and EPI3 (Tokman's two-step scheme,
 *     cited in Section 1)
 *
 * Layout of every nodal vector: idx = (c*K + e)*Np + n, c = variable,
 * e = (ez*ny + ey)*nx + ex, n = (k*(p+1) + j)*(p+1) + i with i along x.
 * Burgers has one variable; Euler 2D (rho, rho u, rho v, rho E); Euler 3D
 * (rho, rho u, rho v, rho w, rho E).
 *
 * Return codes: 0 on success, negative on invalid input or failure.
 */
#ifndef EXPDG_ORACLE_H
#define EXPDG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BURGERS1D = 1, ORC_EULER2D = 2, ORC_EULER3D = 3 };
enum { ORC_EPI2 = 2, ORC_EPI3 = 3, ORC_EXPRB32 = 32, ORC_EXPRB42 = 42 };
/* Burgers (u^2/2)*: Lax-Friedrichs, the entropy flux with the constant
 * sigma, or the entropy flux with sigma = kappa/100 + h max|u^+-| at each face
 * (the steep-gradient example of Section 5.1). */
enum { ORC_FLUX_LF = 0, ORC_FLUX_EF = 1, ORC_FLUX_EF_LOCAL = 2 };
/* ORC_BC_DIRICHLET: Burgers, u = 0 at x0, x1.  ORC_BC_WALL_Y: Euler 2D,
 * no-slip walls at y0 and y1 (periodic in x), as in Section 5.3. */
enum { ORC_BC_PERIODIC = 0, ORC_BC_DIRICHLET = 1, ORC_BC_WALL_Y = 2 };

/* The fields after gamma describe viscous Burgers (Section 3.1); zero-filled
 * they give the inviscid periodic Lax-Friedrichs problem.  Euler requires
 * kappa = 0, flux LF, periodic and no source. */
typedef struct {
    int equation;      /* ORC_BURGERS1D or ORC_EULER2D */
    int nx, ny;        /* elements per direction; ny must be 1 for Burgers */
    int p;             /* polynomial degree, 1..15 */
    double x0, x1, y0, y1;
    double gamma;      /* ratio of specific heats (Euler only) */
    double kappa;      /* viscosity, >= 0 */
    int flux;          /* ORC_FLUX_LF, ORC_FLUX_EF or ORC_FLUX_EF_LOCAL */
    double sigma;      /* EF jump coefficient: the flux adds (sigma/h)[[u]], h = h_e/2 */
    double beta;       /* diffusion fluxes: 0 central, 1/2 LDG (Appendix A) */
    int bc;            /* ORC_BC_PERIODIC, ORC_BC_DIRICHLET or ORC_BC_WALL_Y */
    const double *source; /* NULL or a nodal source added to R (not to L) */
    int nz;            /* elements along z (Euler 3D; 0 or 1 otherwise) */
    double z0, z1;
    /* Entropy viscosity (Euler 2D, Section 3.2 "Artificial viscosity"):
     * ev_ce > 0 enables it; the steppers then compute the nodal viscosity of
     * each step from q^n and q^{n-1} (orc_entropy_viscosity) and add the
     * linear diffusion div(nu grad q) to R and L; outside a step, nu (NULL =
     * none) is the nodal viscosity the operators use. */
    double ev_ce, ev_cmax;
    const double *nu;
} orc_mesh;

/* One accepted Krylov substep: basis size m, substep length dtau, and
 * last != 0 when it completes the phi evaluation it belongs to. */
typedef struct {
    int m;
    int last;
    double dtau;
} orc_substep;

typedef struct {
    double tol;        /* relative tolerance, scaled by nu */
    int m_min, m_max;  /* first check at m_min; Arnoldi never exceeds m_max */
    int check_every;   /* check the error every this many iterations */
    const orc_substep *forced; /* if n_forced > 0: replay this schedule */
    int n_forced;
    int iop;           /* 0: full orthogonalization (two passes); L > 0: one
                          pass against the L most recent vectors (KIOPS' IOP) */
    int adapt;         /* 0: the fixed controller; 1: the cost-based choice of
                          the Krylov size and the substep (after KIOPS) */
    int m_init;        /* adapt = 1: first target size (0: m_min) */
} orc_kopts;

typedef struct {
    int substeps, rejects, krylov_iters, jvps, breakdown, phi_calls, rhs_calls;
    double err_est;
    orc_substep *log;  /* optional: accepted substeps are appended here */
    int log_cap, log_len;
    int checks;        /* small exponentials evaluated */
    int m_next;        /* adapt = 1: the size chosen for a next substep */
} orc_kstats;

/* LGL nodes xi (ascending), weights w, differentiation matrix
 * D[i*(p+1)+j] = l_j'(xi_i). */
int orc_lgl(int p, double *xi, double *w, double *D);

int orc_ndof(const orc_mesh *m);
int orc_nodes(const orc_mesh *m, double *x, double *y, double *z);
/* Diagonal mass entries per nodal value (LGL quadrature weight times the
 * element Jacobian), one per node of one variable: K*Np entries. */
int orc_mass(const orc_mesh *m, double *mass);

/* R(q): full nonlinear DG residual. */
int orc_rhs(const orc_mesh *m, const double *q, double *r);
/* L(qref) v: DG operator of the linear flux A(qref) v with dissipation
 * frozen at qref. */
int orc_jvp(const orc_mesh *m, const double *qref, const double *v, double *w);
/* Auxiliary variable q(u) of the viscous Burgers problem (eq.
 * gov-burgers1d-gradu); Burgers only. */
int orc_gradient(const orc_mesh *m, const double *u, double *q);
/* Nodal entropy viscosity of q (with q_prev the previous step's state and dt
 * the step; Euler 2D): the entropy residual, the element viscosity
 * min(nu_max, nu_E) and its vertex-averaged bilinear reconstruction.  K*Np
 * values, one per node of one variable. */
int orc_entropy_viscosity(const orc_mesh *m, const double *q, const double *q_prev, double dt,
                          double *nu);
/* The diffusion operator div(nu grad v) alone (central fluxes), with the
 * mesh's nodal nu (Euler 2D). */
int orc_ev_diffusion(const orc_mesh *m, const double *v, double *out);
/* Complex-step derivative Im R_frozen(qref + i h v) / h with the flux
 * dissipation evaluated at qref (used to pin orc_jvp). */
int orc_jvp_complex_step(const orc_mesh *m, const double *qref, const double *v,
                         double h, double *w);
/* Dense matrix of L(qref), column-major n x n (n = orc_ndof). */
int orc_assemble_jvp(const orc_mesh *m, const double *qref, double *Lmat);
/* Largest wave speed over the nodes and the LGL minimum node spacing. */
int orc_max_speed(const orc_mesh *m, const double *q, double *cmax, double *dxmin);

/* Dense exponential, row-major n x n, Pade(6,6) with scaling and squaring. */
int orc_expm(int n, const double *A, double *E);
/* Dense phi combination sum_{k=0}^p tau^k phi_k(tau A) b_k through the
 * exponential of the augmented matrix; A row-major n x n, b[k] has n entries
 * (NULL means zero). */
int orc_phi_dense(int n, const double *A, double tau, int p,
                  const double *const *b, double *out);

/* m Arnoldi steps on a dense A (row-major) from b, with the orthogonalization
 * of the phi evaluations (iop as in orc_kopts): V (m+1) x n row-major (vector
 * i at V + i n), H (m+1) x m row-major.  Fails on a breakdown. */
int orc_arnoldi_dense(int n, const double *A, const double *b, int m, int iop, double *V,
                      double *H);
/* Adaptive Krylov phi combination with a dense operator (row-major A). */
int orc_phi_krylov_dense(int n, const double *A, double tau, int p,
                         const double *const *b, double *out,
                         const orc_kopts *o, orc_kstats *s);
/* Adaptive Krylov phi combination with the DG operator L(qref). */
int orc_phi_krylov_dg(const orc_mesh *m, const double *qref, double tau, int p,
                      const double *const *b, double *out,
                      const orc_kopts *o, orc_kstats *s);

/* One exponential step; q in/out.  q_prev (EPI3 only, may be NULL on the
 * first step) holds q^{n-1} on entry and q^n on return. */
int orc_step(const orc_mesh *m, int scheme, double dt, double *q, double *q_prev,
             int have_prev, const orc_kopts *o, orc_kstats *s);

/* Classical fourth-order Runge-Kutta steps of dq/dt = R(q) (test reference). */
int orc_rk4(const orc_mesh *m, double dt, int nsteps, double *q);

/* Threads the OpenMP element loops use (1 when built without OpenMP). */
int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
