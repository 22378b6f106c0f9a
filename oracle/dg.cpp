// Oracle (test infrastructure only): nodal DG operators R(q) and L(q~)v.
//
// Equations (paper Section 3):
//   Burgers, inviscid part:  u_t + (u^2/2)_x = 0, linear flux F_L = u~ u
//     (Section 3.1 with kappa = 0).
//   Euler 2D and 3D: q = (rho, rho u, rho E) with u of 2 or 3 components,
//     F = (rho u, rho u (x) u + p I, rho u H), p = (gamma-1)(rho E - rho |u|^2/2)
//     (Section 3.2, written for any dimension), linear flux F_L = A(q~) q with
//     the normal flux Jacobian A(n) printed there.  The 3D problem is the
//     extruded one of Section 5.2 (periodic in all directions).
//
// Semi-discretization (eq. EXPO-SemiDiscretizedForm_ode): per element,
//   (q_t, v)_K = -(div F, v)_K - <(F* - F) . n, v>_dK
// with LGL collocation and a diagonal LGL mass matrix, i.e. the strong form
//   R_i = -sum_dir (2/h_dir) (D_dir F_dir)_i
//         - sum_faces (2/h_dir) (1/w_end) (F* . n - F . n)_i
// on the face nodes.  Numerical flux: Lax-Friedrichs / Rusanov,
//   F* . n^- = {{F}} . n^- + lambda/2 [[q]] . n^-
//            = (F(q^-) + F(q^+))/2 . n^- + lambda/2 (q^- - q^+),
// (Burgers LF flux, Section 3.1; Lax-Friedrichs for Euler, Section 5.2
// opening) with lambda the larger of the two one-sided wave speeds at the
// face node: |u| for Burgers, |u . n| + a for Euler.
//
// L(q~) v is the same operator with F replaced by F_L(v) = A(q~) v and the
// dissipation lambda evaluated at q~ (the linear numerical flux (u~ u)* and
// (A~ q)* of Sections 3.1 and 3.2).
//
// Viscous Burgers (Section 3.1, eqs. gov-burgers1d-gradu, BurgerL, BurgerN):
// the flux is u^2/2 - kappa q with the auxiliary q = u_x, so
//   R(u) = R_conv(u) + kappa Diff(u) + s,   L(u~) v = L_conv(u~; v) + kappa Diff(v),
// where Diff is linear (the same in R and L, as the split puts all of the
// diffusion into L).  In strong form with the LGL lift:
//   q_i      = (2/h) sum_l D_il u_l + (2/h)(1/w_end) n (u** - u^-)   (end nodes)
//   Diff_i   = (2/h) sum_l D_il q_l + (2/h)(1/w_end) n (q** - q^-)
// with, on a face between a left element L and a right element R and the
// jump [[v]] = v_L - v_R (the paper's jump, a vector along x in 1D):
//   u** = {{u}} - beta [[u]],   q** = {{q}} + beta [[q]]
// (beta = 0: the central fluxes of Section 3.1; beta = 1/2: the LDG fluxes of
// Appendix A, i.e. u** = u_R and q** = q_L).  The nonlinear flux (u^2/2)* is
// Lax-Friedrichs or the entropy flux
//   (u^2/2)* . n^- = n^- (u^-^2 + u^- u^+ + u^+^2)/6 + (sigma/h)(u^- - u^+),
// i.e. (1/3)({{u^2/2}} + {{u}}^2) + (sigma/h)[[u]] of Section 3.1, with h read
// as the half-width h_e/2 of the element (the Jacobian of the map from
// [-1, 1]); the linear flux (u~ u)* stays Lax-Friedrichs with
// lambda = max|u~^+-|.  For the steep-gradient example of Section 5.1 the
// penalty is set per face, sigma = kappa/100 + h max|u^+-| with the same h,
// so sigma/h = kappa/(100 h) + max|u^+-|.
//
// Boundaries: periodic, or (Burgers) zero Dirichlet at both ends following
// the footnote at the start of Section 6: the exterior state is u^+ = 0 for
// (u~ u)* and (u^2/2)*, u** = 0 and q** = q^-.
//
// Euler 2D with no-slip walls at y0 and y1 (Section 5.3, periodic in x): at a
// wall face node the exterior state is the mirror q^+ = M q^-, M = diag(1, -1,
// -1, 1) (both momentum components reversed, so the mean velocity on the wall
// is zero), in the Rusanov flux of R; the linear flux takes v^+ = M v^- at the
// mirrored reference state M q~^- (lambda is the same on both sides).  The
// entropy-viscosity diffusion mirrors too: the gradient takes
// v** = (v^- + M v^-)/2 (zero momentum on the wall, density and energy
// unchanged), and the normal diffusive flux of the mirror is -M (nu g)^-, so
// (nu g)** = (I - M)(nu g)^-/2: the interior value for the momenta (as the
// Dirichlet end above) and zero for density and energy (no diffusive flux
// through the wall).
#include "oracle.h"

#include <cmath>
#include <complex>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

struct Geo {
    int eq, nx, ny, nz, p, n1, Np, K, nvar, dim;
    double hx, hy, hz, gamma, x0, y0, z0;
    double kappa, sigma, beta;
    int flux, bc;
    const double *src;
    double ev_ce, ev_cmax;
    const double *nu;
    std::vector<double> xi, w, D;
};

bool make_geo(const orc_mesh *m, Geo *g) {
    if (!m) return false;
    if (m->equation != ORC_BURGERS1D && m->equation != ORC_EULER2D &&
        m->equation != ORC_EULER3D)
        return false;
    const int nz = (m->nz > 0) ? m->nz : 1;
    if (m->p < 1 || m->p > 15 || m->nx < 1 || m->ny < 1) return false;
    if (m->equation == ORC_BURGERS1D && m->ny != 1) return false;
    if (m->equation != ORC_EULER3D && nz != 1) return false;
    if (!(m->x1 > m->x0)) return false;
    if (m->equation != ORC_BURGERS1D && (!(m->y1 > m->y0) || !(m->gamma > 1.0))) return false;
    if (m->equation == ORC_EULER3D && !(m->z1 > m->z0)) return false;
    if (!(m->kappa >= 0.0) || !(m->sigma >= 0.0) || !(std::fabs(m->beta) <= 0.5)) return false;
    if (m->flux != ORC_FLUX_LF && m->flux != ORC_FLUX_EF && m->flux != ORC_FLUX_EF_LOCAL)
        return false;
    if (m->bc != ORC_BC_PERIODIC && m->bc != ORC_BC_DIRICHLET && m->bc != ORC_BC_WALL_Y)
        return false;
    if (m->equation == ORC_BURGERS1D && m->bc == ORC_BC_WALL_Y) return false;
    if (m->equation != ORC_BURGERS1D &&
        (m->kappa != 0.0 || m->flux != ORC_FLUX_LF || m->bc == ORC_BC_DIRICHLET || m->source))
        return false;
    if (m->equation == ORC_EULER3D && m->bc != ORC_BC_PERIODIC) return false;
    if (!(m->ev_ce >= 0.0) || !(m->ev_cmax >= 0.0)) return false;
    if (m->equation != ORC_EULER2D && (m->ev_ce > 0.0 || m->nu)) return false;
    g->eq = m->equation;
    g->nx = m->nx;
    g->ny = m->ny;
    g->nz = nz;
    g->p = m->p;
    g->n1 = m->p + 1;
    g->dim = (m->equation == ORC_BURGERS1D) ? 1 : (m->equation == ORC_EULER2D ? 2 : 3);
    g->Np = (g->dim == 1) ? g->n1 : (g->dim == 2 ? g->n1 * g->n1 : g->n1 * g->n1 * g->n1);
    g->K = m->nx * m->ny * nz;
    g->nvar = (m->equation == ORC_BURGERS1D) ? 1 : g->dim + 2;
    g->hx = (m->x1 - m->x0) / m->nx;
    g->hy = (g->dim >= 2) ? (m->y1 - m->y0) / m->ny : 1.0;
    g->hz = (g->dim == 3) ? (m->z1 - m->z0) / nz : 1.0;
    g->x0 = m->x0;
    g->y0 = m->y0;
    g->z0 = m->z0;
    g->gamma = m->gamma;
    g->kappa = m->kappa;
    g->sigma = m->sigma;
    g->beta = m->beta;
    g->flux = m->flux;
    g->bc = m->bc;
    g->src = m->source;
    g->ev_ce = m->ev_ce;
    g->ev_cmax = m->ev_cmax;
    g->nu = m->nu;
    g->xi.resize(g->n1);
    g->w.resize(g->n1);
    g->D.resize(g->n1 * g->n1);
    return orc_lgl(g->p, g->xi.data(), g->w.data(), g->D.data()) == 0;
}

// Neighbour of element e = (ez ny + ey) nx + ex across its face in direction
// dir (0 = x, 1 = y, 2 = z) on side s (-1 = lower, +1 = upper); -1 at a
// Dirichlet end or a wall.
int neighbour(const Geo &g, int e, int dir, int s) {
    int ex = e % g.nx, ey = (e / g.nx) % g.ny, ez = e / (g.nx * g.ny);
    if (g.bc == ORC_BC_DIRICHLET && dir == 0 && (ex + s < 0 || ex + s >= g.nx)) return -1;
    if (g.bc == ORC_BC_WALL_Y && dir == 1 && (ey + s < 0 || ey + s >= g.ny)) return -1;
    if (dir == 0)
        ex = (ex + s + g.nx) % g.nx;
    else if (dir == 1)
        ey = (ey + s + g.ny) % g.ny;
    else
        ez = (ez + s + g.nz) % g.nz;
    return (ez * g.ny + ey) * g.nx + ex;
}

// Node index of (i, j, k) (i along x, j along y, k along z).
inline int node(const Geo &g, int i, int j, int k = 0) {
    return (g.dim == 1) ? i : (g.dim == 2 ? j * g.n1 + i : (k * g.n1 + j) * g.n1 + i);
}

template <class T>
void load(const Geo &g, const T *q, int e, int n, T *out) {
    for (int c = 0; c < g.nvar; ++c) out[c] = q[((size_t)c * g.K + e) * g.Np + n];
}

// The wall mirror M q: both momentum components reversed (Euler 2D).
template <class T>
void mirror(const T *q, T *out) {
    out[0] = q[0];
    out[1] = -q[1];
    out[2] = -q[2];
    out[3] = q[3];
}

// ---- physics -------------------------------------------------------------

// Physical flux F_dir(q).
template <class T>
void flux(const Geo &g, const T *q, int dir, T *f) {
    if (g.eq == ORC_BURGERS1D) {
        f[0] = 0.5 * q[0] * q[0];
        return;
    }
    const double gm = g.gamma;
    const int d = g.dim, iE = d + 1;
    T rho = q[0];
    T u[3] = {T(0.0), T(0.0), T(0.0)};
    for (int a = 0; a < d; ++a) u[a] = q[1 + a] / rho;
    T mu = q[1] * u[0];
    for (int a = 1; a < d; ++a) mu += q[1 + a] * u[a];
    T p = (gm - 1.0) * (q[iE] - 0.5 * mu);
    T un = u[dir];
    f[0] = rho * un;
    for (int a = 0; a < d; ++a) f[1 + a] = q[1 + a] * un + ((dir == a) ? p : T(0.0));
    f[iE] = (q[iE] + p) * un;
}

// Linear flux A_dir(qt) v: the paper's normal flux Jacobian with n = e_dir,
//   A(n) = [ 0,                 n^T,                               0        ]
//          [ phi n - u u_n,     u (x) n - (g-1) n (x) u + u_n I,   (g-1) n  ]
//          [ (phi - H) u_n,     H n^T - (g-1) u^T u_n,             g u_n    ]
// with phi = (g-1)/2 |u|^2 and u_n = n . u.  Burgers: A(u~) v = u~ v.
template <class T>
void lin_flux(const Geo &g, const double *qt, const T *v, int dir, T *f) {
    if (g.eq == ORC_BURGERS1D) {
        f[0] = qt[0] * v[0];
        return;
    }
    const double gm = g.gamma, gt = g.gamma - 1.0;
    const int d = g.dim, iE = d + 1;
    const double rho = qt[0];
    double u[3] = {0.0, 0.0, 0.0}, n[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) u[a] = qt[1 + a] / rho;
    double uu = u[0] * u[0];
    for (int a = 1; a < d; ++a) uu += u[a] * u[a];
    const double p = gt * (qt[iE] - 0.5 * rho * uu);
    const double H = (qt[iE] + p) / rho;
    const double phi = 0.5 * gt * uu;
    n[dir] = 1.0;
    double un = n[0] * u[0];
    for (int a = 1; a < d; ++a) un += n[a] * u[a];
    T f0 = n[0] * v[1];
    for (int a = 1; a < d; ++a) f0 += n[a] * v[1 + a];
    f[0] = f0;
    for (int a = 0; a < d; ++a) {
        T acc = (phi * n[a] - u[a] * un) * v[0];
        for (int b = 0; b < d; ++b) {
            double Mab = u[a] * n[b] - gt * n[a] * u[b] + ((a == b) ? un : 0.0);
            acc += Mab * v[1 + b];
        }
        acc += gt * n[a] * v[iE];
        f[1 + a] = acc;
    }
    T fe = (phi - H) * un * v[0];
    for (int a = 0; a < d; ++a) fe += (H * n[a] - gt * u[a] * un) * v[1 + a];
    fe += gm * un * v[iE];
    f[iE] = fe;
}

// One-sided wave speed for the Lax-Friedrichs dissipation.
double wave_speed(const Geo &g, const double *q, int dir) {
    if (g.eq == ORC_BURGERS1D) return std::fabs(q[0]);
    const int d = g.dim, iE = d + 1;
    const double rho = q[0];
    double u[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < d; ++k) u[k] = q[1 + k] / rho;
    double uu = u[0] * u[0];
    for (int k = 1; k < d; ++k) uu += u[k] * u[k];
    const double p = (g.gamma - 1.0) * (q[iE] - 0.5 * rho * uu);
    const double a = std::sqrt(g.gamma * p / rho);
    return std::fabs(u[dir]) + a;
}

// ---- generic DG operator ------------------------------------------------
//
// out = DG operator applied to the field u with
//   node_flux(e, n, dir, f): flux at a node (volume and face traces),
//   lam_ref: real state whose traces give the LF wave speed lambda.
//   entropy: the nonlinear Burgers face flux is EF instead of LF.
// wall_flux(e, n, dir, fp, up): exterior flux and field at a wall face node.
template <class T, class FluxAt, class WallAt>
void dg_apply(const Geo &g, const T *u, const double *lam_ref, FluxAt node_flux, WallAt wall_flux,
              T *out, bool entropy = false) {
    const int n1 = g.n1, Np = g.Np, nv = g.nvar;
    const double h[3] = {g.hx, g.hy, g.hz};
#pragma omp parallel for schedule(static)
    for (int e = 0; e < g.K; ++e) {
        // fluxes at all nodes of this element, per direction
        std::vector<T> F((size_t)g.dim * Np * nv);
        for (int dir = 0; dir < g.dim; ++dir)
            for (int n = 0; n < Np; ++n) node_flux(e, n, dir, &F[((size_t)dir * Np + n) * nv]);
        for (int kk = 0; kk < (g.dim == 3 ? n1 : 1); ++kk)
        for (int jj = 0; jj < (g.dim >= 2 ? n1 : 1); ++jj) {
            for (int i = 0; i < n1; ++i) {
                const int n = node(g, i, jj, kk);
                const int crd[3] = {i, jj, kk};
                // the node with its coordinate along dir replaced by l
                auto along = [&](int dir, int l) {
                    return node(g, dir == 0 ? l : i, dir == 1 ? l : jj, dir == 2 ? l : kk);
                };
                T res[5];
                for (int c = 0; c < nv; ++c) res[c] = T(0.0);
                // volume: -(2/h_dir) sum_l D_{il} F_dir at the nodes of the line
                for (int dir = 0; dir < g.dim; ++dir) {
                    const int a = crd[dir];  // coordinate index along dir
                    for (int l = 0; l < n1; ++l) {
                        const int nl = along(dir, l);
                        const double Dal = g.D[a * n1 + l];
                        for (int c = 0; c < nv; ++c)
                            res[c] -= (2.0 / h[dir]) * Dal * F[((size_t)dir * Np + nl) * nv + c];
                    }
                }
                // faces: -(2/h_dir)(1/w_end) (F* . n - F(u^-) . n)
                for (int dir = 0; dir < g.dim; ++dir) {
                    const int a = crd[dir];
                    for (int s = -1; s <= 1; s += 2) {
                        if ((s == -1 && a != 0) || (s == 1 && a != g.p)) continue;
                        const int en = neighbour(g, e, dir, s);
                        // mirror node on the neighbour: coordinate along dir flips end
                        const int am = g.p - a;
                        const int nn = along(dir, am);
                        T fm[5], fp[5], um[5], up[5];
                        for (int c = 0; c < nv; ++c) fm[c] = F[((size_t)dir * Np + n) * nv + c];
                        load(g, u, e, n, um);
                        double qm[5], qp[5];
                        load(g, lam_ref, e, n, qm);
                        if (en >= 0) {
                            node_flux(en, nn, dir, fp);
                            load(g, u, en, nn, up);
                            load(g, lam_ref, en, nn, qp);
                        } else if (g.bc == ORC_BC_WALL_Y) {  // wall: the mirror state
                            wall_flux(e, n, dir, fp, up);
                            mirror(qm, qp);
                        } else {  // Dirichlet end (Burgers): exterior state 0, flux 0
                            fp[0] = T(0.0);
                            up[0] = T(0.0);
                            qp[0] = 0.0;
                        }
                        const double lam =
                            std::fmax(wave_speed(g, qm, dir), wave_speed(g, qp, dir));
                        const double sn = (double)s;  // n^- . e_dir
                        for (int c = 0; c < nv; ++c) {
                            T fstar_n = 0.5 * sn * (fm[c] + fp[c]) + 0.5 * lam * (um[c] - up[c]);
                            if (entropy) {
                                // sigma / h with h the half-width; the face-dependent
                                // sigma = kappa/100 + h max|u^+-| gives
                                // sigma / h = kappa / (100 h) + max|u^+-| (lam here)
                                const double pen = (g.flux == ORC_FLUX_EF_LOCAL)
                                                       ? 2.0 * g.kappa / (100.0 * g.hx) + lam
                                                       : 2.0 * g.sigma / g.hx;
                                fstar_n = sn * (um[0] * um[0] + um[0] * up[0] + up[0] * up[0]) /
                                              6.0 +
                                          pen * (um[0] - up[0]);
                            }
                            T f_n = sn * fm[c];
                            res[c] -= (2.0 / h[dir]) / g.w[a] * (fstar_n - f_n);
                        }
                    }
                }
                for (int c = 0; c < nv; ++c) out[((size_t)c * g.K + e) * Np + n] = res[c];
            }
        }
    }
}

// ---- viscous Burgers: auxiliary gradient and diffusion --------------------

// Face values of the element e at its end on side s (-1 left, +1 right):
// the left and right elements of that face (-1 beyond a Dirichlet end).
inline void face_sides(const Geo &g, int e, int s, int *eL, int *eR) {
    const int en = neighbour(g, e, 0, s);
    *eL = (s < 0) ? en : e;
    *eR = (s < 0) ? e : en;
}

// q(u) of eq. gov-burgers1d-gradu (strong form, see the header).
template <class T>
void aux_gradient(const Geo &g, const T *u, T *q) {
    const int n1 = g.n1, p = g.p;
    const double rh = 2.0 / g.hx;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < g.K; ++e) {
        for (int i = 0; i < n1; ++i) {
            T acc = T(0.0);
            for (int l = 0; l < n1; ++l) acc += rh * g.D[i * n1 + l] * u[(size_t)e * n1 + l];
            for (int s = -1; s <= 1; s += 2) {
                if ((s == -1 && i != 0) || (s == 1 && i != p)) continue;
                int eL, eR;
                face_sides(g, e, s, &eL, &eR);
                T ustar = T(0.0);  // Dirichlet end: u** = 0
                if (eL >= 0 && eR >= 0) {
                    const T uL = u[(size_t)eL * n1 + p], uR = u[(size_t)eR * n1];
                    ustar = 0.5 * (uL + uR) - g.beta * (uL - uR);
                }
                acc += rh / g.w[i] * (double)s * (ustar - u[(size_t)e * n1 + i]);
            }
            q[(size_t)e * n1 + i] = acc;
        }
    }
}

// out += kappa Diff(u), the diffusion part of eq. BurgerL (see the header).
template <class T>
void add_diffusion(const Geo &g, const T *u, T *out) {
    if (g.kappa == 0.0) return;
    const int n1 = g.n1, p = g.p;
    const double rh = 2.0 / g.hx;
    std::vector<T> q((size_t)g.K * n1);
    aux_gradient(g, u, q.data());
#pragma omp parallel for schedule(static)
    for (int e = 0; e < g.K; ++e) {
        for (int i = 0; i < n1; ++i) {
            T acc = T(0.0);
            for (int l = 0; l < n1; ++l) acc += rh * g.D[i * n1 + l] * q[(size_t)e * n1 + l];
            for (int s = -1; s <= 1; s += 2) {
                if ((s == -1 && i != 0) || (s == 1 && i != p)) continue;
                int eL, eR;
                face_sides(g, e, s, &eL, &eR);
                const T qm = q[(size_t)e * n1 + i];
                T qstar = qm;  // Dirichlet end: q** = q^-
                if (eL >= 0 && eR >= 0) {
                    const T qL = q[(size_t)eL * n1 + p], qR = q[(size_t)eR * n1];
                    qstar = 0.5 * (qL + qR) + g.beta * (qL - qR);
                }
                acc += rh / g.w[i] * (double)s * (qstar - qm);
            }
            out[(size_t)e * n1 + i] += g.kappa * acc;
        }
    }
}

// ---- entropy viscosity (Euler 2D) ------------------------------------------
//
// The linear diffusion div(nu grad v) of each conserved variable with the
// nodal viscosity nu (Section 3.2, "Artificial viscosity": F^EV = nu grad q,
// treated like the Burgers diffusion with central fluxes): per direction d
//   g_d = (2/h_d) D_d v + (2/h_d)(1/w_end) n_d ({{v}} - v^-)          (faces along d)
//   out += (2/h_d) D_d (nu g_d) + (2/h_d)(1/w_end) n_d ({{nu g_d}} - (nu g_d)^-).
template <class T>
void ev_diffusion(const Geo &g, const T *v, T *out) {
    if (!g.nu) return;
    const int n1 = g.n1, Np = g.Np, p = g.p;
    const double h[2] = {g.hx, g.hy};
    const size_t plane = (size_t)g.K * Np;
    std::vector<T> G(2 * plane);
    auto along = [&](int i, int j, int d, int l) { return d == 0 ? j * n1 + l : l * n1 + i; };
    for (int c = 0; c < 4; ++c) {
        const T *vc = v + c * plane;
#pragma omp parallel for schedule(static)
        for (int e = 0; e < g.K; ++e)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    const int n = j * n1 + i, crd[2] = {i, j};
                    for (int d = 0; d < 2; ++d) {
                        const int a = crd[d];
                        T acc = T(0.0);
                        for (int l = 0; l < n1; ++l)
                            acc += (2.0 / h[d]) * g.D[a * n1 + l] * vc[(size_t)e * Np + along(i, j, d, l)];
                        for (int s = -1; s <= 1; s += 2) {
                            if ((s == -1 && a != 0) || (s == 1 && a != p)) continue;
                            const int en = neighbour(g, e, d, s);
                            const int nn = along(i, j, d, p - a);
                            const T vm = vc[(size_t)e * Np + n];
                            // wall: the mirror's component (momentum reversed)
                            const T vp = en >= 0 ? vc[(size_t)en * Np + nn]
                                                 : ((c == 1 || c == 2) ? -vm : vm);
                            acc += (2.0 / h[d]) / g.w[a] * (double)s * (0.5 * (vm + vp) - vm);
                        }
                        G[d * plane + (size_t)e * Np + n] = acc;
                    }
                }
#pragma omp parallel for schedule(static)
        for (int e = 0; e < g.K; ++e)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    const int n = j * n1 + i, crd[2] = {i, j};
                    T acc = T(0.0);
                    for (int d = 0; d < 2; ++d) {
                        const int a = crd[d];
                        for (int l = 0; l < n1; ++l) {
                            const size_t at = (size_t)e * Np + along(i, j, d, l);
                            acc += (2.0 / h[d]) * g.D[a * n1 + l] * (g.nu[at] * G[d * plane + at]);
                        }
                        for (int s = -1; s <= 1; s += 2) {
                            if ((s == -1 && a != 0) || (s == 1 && a != p)) continue;
                            const int en = neighbour(g, e, d, s);
                            if (en < 0) {
                                // wall: (nu g)** = 0 for density and energy, (nu g)^- for
                                // the momenta (no face term)
                                if (c == 0 || c == 3) {
                                    const size_t am = (size_t)e * Np + n;
                                    const T fm = g.nu[am] * G[d * plane + am];
                                    acc += (2.0 / h[d]) / g.w[a] * (double)s * (0.0 - fm);
                                }
                                continue;
                            }
                            const size_t am = (size_t)e * Np + n;
                            const size_t ap = (size_t)en * Np + along(i, j, d, p - a);
                            const T fm = g.nu[am] * G[d * plane + am];
                            const T fp = g.nu[ap] * G[d * plane + ap];
                            acc += (2.0 / h[d]) / g.w[a] * (double)s * (0.5 * (fm + fp) - fm);
                        }
                    }
                    out[c * plane + (size_t)e * Np + n] += acc;
                }
    }
}

template <class T>
void residual_frozen(const Geo &g, const T *q, const double *lam_ref, T *r) {
    auto fl = [&](int e, int n, int dir, T *f) {
        T qn[5];
        load(g, q, e, n, qn);
        flux(g, qn, dir, f);
    };
    auto wall = [&](int e, int n, int dir, T *f, T *up) {
        T qn[5];
        load(g, q, e, n, qn);
        mirror(qn, up);
        flux(g, up, dir, f);
    };
    dg_apply(g, q, lam_ref, fl, wall, r, g.eq == ORC_BURGERS1D && g.flux != ORC_FLUX_LF);
    if (g.eq == ORC_BURGERS1D) add_diffusion(g, q, r);
    if (g.eq == ORC_EULER2D) ev_diffusion(g, q, r);
}

void linear_op(const Geo &g, const double *qt, const double *v, double *w) {
    auto fl = [&](int e, int n, int dir, double *f) {
        double qn[5], vn[5];
        load(g, qt, e, n, qn);
        load(g, v, e, n, vn);
        lin_flux(g, qn, vn, dir, f);
    };
    auto wall = [&](int e, int n, int dir, double *f, double *up) {
        double qn[5], qm[5], vn[5];
        load(g, qt, e, n, qn);
        load(g, v, e, n, vn);
        mirror(qn, qm);
        mirror(vn, up);
        lin_flux(g, qm, up, dir, f);
    };
    dg_apply(g, v, qt, fl, wall, w);
    if (g.eq == ORC_BURGERS1D) add_diffusion(g, v, w);
    if (g.eq == ORC_EULER2D) ev_diffusion(g, v, w);
}

}  // namespace

extern "C" {

int orc_ndof(const orc_mesh *m) {
    Geo g;
    if (!make_geo(m, &g)) return -1;
    return g.nvar * g.K * g.Np;
}

int orc_nodes(const orc_mesh *m, double *x, double *y, double *z) {
    Geo g;
    if (!make_geo(m, &g) || !x) return -1;
    for (int e = 0; e < g.K; ++e) {
        const int ex = e % g.nx, ey = (e / g.nx) % g.ny, ez = e / (g.nx * g.ny);
        for (int kk = 0; kk < (g.dim == 3 ? g.n1 : 1); ++kk)
        for (int jj = 0; jj < (g.dim >= 2 ? g.n1 : 1); ++jj)
            for (int i = 0; i < g.n1; ++i) {
                const size_t at = (size_t)e * g.Np + node(g, i, jj, kk);
                x[at] = g.x0 + ex * g.hx + 0.5 * (g.xi[i] + 1.0) * g.hx;
                if (y) y[at] = (g.dim >= 2) ? g.y0 + ey * g.hy + 0.5 * (g.xi[jj] + 1.0) * g.hy : 0.0;
                if (z) z[at] = (g.dim == 3) ? g.z0 + ez * g.hz + 0.5 * (g.xi[kk] + 1.0) * g.hz : 0.0;
            }
    }
    return 0;
}

int orc_mass(const orc_mesh *m, double *mass) {
    Geo g;
    if (!make_geo(m, &g) || !mass) return -1;
    for (int e = 0; e < g.K; ++e)
        for (int kk = 0; kk < (g.dim == 3 ? g.n1 : 1); ++kk)
        for (int jj = 0; jj < (g.dim >= 2 ? g.n1 : 1); ++jj)
            for (int i = 0; i < g.n1; ++i) {
                double v = 0.5 * g.hx * g.w[i];
                if (g.dim >= 2) v *= 0.5 * g.hy * g.w[jj];
                if (g.dim == 3) v *= 0.5 * g.hz * g.w[kk];
                mass[(size_t)e * g.Np + node(g, i, jj, kk)] = v;
            }
    return 0;
}

int orc_rhs(const orc_mesh *m, const double *q, double *r) {
    Geo g;
    if (!make_geo(m, &g) || !q || !r) return -1;
    residual_frozen<double>(g, q, q, r);
    if (g.src) {
        const size_t n = (size_t)g.nvar * g.K * g.Np;
        for (size_t i = 0; i < n; ++i) r[i] += g.src[i];
    }
    return 0;
}

int orc_ev_diffusion(const orc_mesh *m, const double *v, double *out) {
    Geo g;
    if (!make_geo(m, &g) || g.eq != ORC_EULER2D || !v || !out) return -1;
    const size_t n = (size_t)g.nvar * g.K * g.Np;
    for (size_t i = 0; i < n; ++i) out[i] = 0.0;
    ev_diffusion<double>(g, v, out);
    return 0;
}

// Entropy viscosity (Section 3.2, "Artificial viscosity", with the entropy
// residual of its footnote): with S = rho/(g-1) log(p/rho^g) and the entropy
// flux u S,
//   Res = (S(q) - S(q_prev))/dt + (div(u S)(q) + div(u S)(q_prev))/2
// at the nodes (element-local derivative); per element, with h = 2r/k (r the
// radius of the element's circumscribed circle, k = p) = sqrt(hx^2+hy^2)/p,
//   nu_E = c_E h^2 max(max|Res|, max|[[u S . n]]| / h),
//   nu_max = c_max h max(|u . e_d| + a),  nu_e = min(nu_max, nu_E);
// the vertex values average the four elements around each vertex, and nu at
// a node is their bilinear interpolant on its element.
int orc_entropy_viscosity(const orc_mesh *m, const double *q, const double *q_prev, double dt,
                          double *nu) {
    Geo g;
    if (!make_geo(m, &g) || g.eq != ORC_EULER2D || !q || !q_prev || !nu || !(dt > 0.0))
        return -1;
    const int n1 = g.n1, Np = g.Np, p = g.p;
    const size_t plane = (size_t)g.K * Np;
    const double gm = g.gamma, h[2] = {g.hx, g.hy};
    // S and the entropy flux at every node of q and q_prev
    std::vector<double> S(2 * plane), F(4 * plane);  // F[(st*2 + d) * plane + i]
    for (int st = 0; st < 2; ++st) {
        const double *qq = st == 0 ? q : q_prev;
        for (size_t i = 0; i < plane; ++i) {
            const double rho = qq[i], u = qq[plane + i] / rho, v = qq[2 * plane + i] / rho;
            const double pr = (gm - 1.0) * (qq[3 * plane + i] - 0.5 * rho * (u * u + v * v));
            const double Sv = rho / (gm - 1.0) * std::log(pr / std::pow(rho, gm));
            S[st * plane + i] = Sv;
            F[(st * 2 + 0) * plane + i] = u * Sv;
            F[(st * 2 + 1) * plane + i] = v * Sv;
        }
    }
    const double he = std::sqrt(g.hx * g.hx + g.hy * g.hy) / p;
    std::vector<double> nue(g.K);
    for (int e = 0; e < g.K; ++e) {
        double rmax = 0.0, jmax = 0.0, lam = 0.0;
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                const int n = j * n1 + i, crd[2] = {i, j};
                const size_t at = (size_t)e * Np + n;
                double div[2] = {0.0, 0.0};
                for (int st = 0; st < 2; ++st)
                    for (int d = 0; d < 2; ++d)
                        for (int l = 0; l < n1; ++l) {
                            const int nl = d == 0 ? j * n1 + l : l * n1 + i;
                            div[st] += (2.0 / h[d]) * g.D[crd[d] * n1 + l] *
                                       F[(st * 2 + d) * plane + (size_t)e * Np + nl];
                        }
                const double res = (S[at] - S[plane + at]) / dt + 0.5 * (div[0] + div[1]);
                rmax = std::fmax(rmax, std::fabs(res));
                double qn[4];
                load(g, q, e, n, qn);
                for (int d = 0; d < 2; ++d) {
                    lam = std::fmax(lam, wave_speed(g, qn, d));
                    const int a = crd[d];
                    for (int s = -1; s <= 1; s += 2) {
                        if ((s == -1 && a != 0) || (s == 1 && a != p)) continue;
                        const int en = neighbour(g, e, d, s);
                        const int nn = d == 0 ? j * n1 + (p - a) : (p - a) * n1 + i;
                        // a wall's mirror state carries -v S: the jump is 2 v S
                        const double fp = en >= 0 ? F[d * plane + (size_t)en * Np + nn]
                                                  : -F[d * plane + at];
                        const double jump = F[d * plane + at] - fp;
                        jmax = std::fmax(jmax, std::fabs(jump));
                    }
                }
            }
        const double nu_e = g.ev_ce * he * he * std::fmax(rmax, jmax / he);
        const double nu_max = g.ev_cmax * he * lam;
        nue[e] = std::fmin(nu_max, nu_e);
    }
    // vertex (vx, vy) is the lower-left corner of element (vx, vy); with walls
    // there is one more row of vertices (y1), and a wall vertex averages the
    // two elements it belongs to
    const bool walls = g.bc == ORC_BC_WALL_Y;
    const int nvy = walls ? g.ny + 1 : g.ny;
    std::vector<double> vert((size_t)nvy * g.nx);
    for (int vy = 0; vy < nvy; ++vy)
        for (int vx = 0; vx < g.nx; ++vx) {
            const int xm = (vx + g.nx - 1) % g.nx;
            if (walls && (vy == 0 || vy == g.ny)) {
                const int ey = vy == 0 ? 0 : g.ny - 1;
                vert[(size_t)vy * g.nx + vx] =
                    0.5 * (nue[ey * g.nx + vx] + nue[ey * g.nx + xm]);
                continue;
            }
            const int ym = (vy + g.ny - 1) % g.ny;
            vert[(size_t)vy * g.nx + vx] = 0.25 * ((nue[vy * g.nx + vx] + nue[vy * g.nx + xm]) +
                                                   (nue[ym * g.nx + vx] + nue[ym * g.nx + xm]));
        }
    for (int e = 0; e < g.K; ++e) {
        const int ex = e % g.nx, ey = e / g.nx;
        const int xp = (ex + 1) % g.nx, yp = walls ? ey + 1 : (ey + 1) % g.ny;
        const double v00 = vert[ey * g.nx + ex], v10 = vert[ey * g.nx + xp];
        const double v01 = vert[yp * g.nx + ex], v11 = vert[yp * g.nx + xp];
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                const double r = 0.5 * (g.xi[i] + 1.0), t = 0.5 * (g.xi[j] + 1.0);
                nu[(size_t)e * Np + j * n1 + i] =
                    (1.0 - r) * (1.0 - t) * v00 + r * (1.0 - t) * v10 + (1.0 - r) * t * v01 +
                    r * t * v11;
            }
    }
    return 0;
}

int orc_gradient(const orc_mesh *m, const double *u, double *q) {
    Geo g;
    if (!make_geo(m, &g) || g.eq != ORC_BURGERS1D || !u || !q) return -1;
    aux_gradient<double>(g, u, q);
    return 0;
}

int orc_jvp(const orc_mesh *m, const double *qref, const double *v, double *w) {
    Geo g;
    if (!make_geo(m, &g) || !qref || !v || !w) return -1;
    linear_op(g, qref, v, w);
    return 0;
}

int orc_jvp_complex_step(const orc_mesh *m, const double *qref, const double *v, double h,
                         double *w) {
    Geo g;
    if (!make_geo(m, &g) || !qref || !v || !w || !(h > 0)) return -1;
    const size_t n = (size_t)g.nvar * g.K * g.Np;
    std::vector<cplx> qc(n), rc(n);
    for (size_t i = 0; i < n; ++i) qc[i] = cplx(qref[i], h * v[i]);
    residual_frozen<cplx>(g, qc.data(), qref, rc.data());
    for (size_t i = 0; i < n; ++i) w[i] = rc[i].imag() / h;
    return 0;
}

int orc_assemble_jvp(const orc_mesh *m, const double *qref, double *Lmat) {
    Geo g;
    if (!make_geo(m, &g) || !qref || !Lmat) return -1;
    const size_t n = (size_t)g.nvar * g.K * g.Np;
    std::vector<double> e(n, 0.0);
    for (size_t j = 0; j < n; ++j) {
        e[j] = 1.0;
        linear_op(g, qref, e.data(), Lmat + j * n);
        e[j] = 0.0;
    }
    return 0;
}

int orc_max_speed(const orc_mesh *m, const double *q, double *cmax, double *dxmin) {
    Geo g;
    if (!make_geo(m, &g) || !q) return -1;
    double c = 0.0;
    for (int e = 0; e < g.K; ++e)
        for (int n = 0; n < g.Np; ++n) {
            double qn[5];
            load(g, q, e, n, qn);
            for (int dir = 0; dir < g.dim; ++dir) c = std::fmax(c, wave_speed(g, qn, dir));
        }
    double dmin = 1e300;
    for (int i = 0; i < g.p; ++i) dmin = std::fmin(dmin, g.xi[i + 1] - g.xi[i]);
    double h = g.hx;
    if (g.dim >= 2) h = std::fmin(h, g.hy);
    if (g.dim == 3) h = std::fmin(h, g.hz);
    if (cmax) *cmax = c;
    if (dxmin) *dxmin = 0.5 * h * dmin;
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

}  // extern "C"
