// Oracle (test infrastructure only): exponential time steppers built on the
// phi-function combination, with L^n = L(q^n) (flux Jacobian at q^n) and
// R^n = R(q^n).
//
//   EPI2 (footnote in Section 5.1):   q^{n+1} = q^n + dt phi_1(dt L^n) R^n.
//   EXPRB32 (footnote in Section 5.1):
//       q2      = q^n + dt phi_1(dt L^n) R^n
//       q^{n+1} = q^n + dt phi_1(dt L^n) R^n + 2 dt phi_3(dt L^n) D,
//       D = N(q2) - N(q^n) = R(q2) - R^n - L^n (q2 - q^n).
//     As a phi combination: q^{n+1} = q2 + sum_k dt^k phi_k b_k with
//     b_3 = 2 D / dt^2 and b_0 = b_1 = b_2 = 0.
//   EXPRB42 (the fourth-order two-stage scheme, footnote of the comparison of
//     exponential integrators in Section 5.2):
//       q2      = q^n + (3/4) dt phi_1((3/4) dt L^n) R^n
//       q^{n+1} = q^n + dt phi_1(dt L^n) R^n + (32/9) dt phi_3(dt L^n) D,
//       D = N(q2) - N(q^n) = R(q2) - R^n - L^n (q2 - q^n),
//     i.e. a combination with tau = 3 dt / 4, b_1 = R^n, then one with
//     tau = dt, b_1 = R^n, b_3 = (32/9) D / dt^2 (b_0 = b_2 = 0).
//   EPI3 (Tokman's two-step scheme, cited in Section 1; the paper names it
//     but does not print it):
//       q^{n+1} = q^n + dt phi_1(dt L^n) R^n + (2/3) dt phi_2(dt L^n) r,
//       r = R(q^{n-1}) - R^n - L^n (q^{n-1} - q^n),
//     i.e. one combination with b_1 = R^n and b_2 = (2/3) r / dt.  The first
//     step, which has no q^{n-1}, is an EPI2 step.
//   RK4: the classical four-stage Runge-Kutta method (test reference only).
// With entropy viscosity (Euler 2D) each step first computes its nodal
// viscosity from q^n and q^{n-1} and keeps it for all its operators.
#include "oracle.h"

#include <cmath>
#include <functional>
#include <vector>

int orc_phi_krylov_op(size_t n, const std::function<void(const double *, double *)> &A,
                      double tau, int p, const double *const *b, double *out, const orc_kopts *o,
                      orc_kstats *st, int *fpos);

extern "C" int orc_step(const orc_mesh *m, int scheme, double dt, double *q, double *q_prev,
                        int have_prev, const orc_kopts *o, orc_kstats *s) {
    const int ni = orc_ndof(m);
    if (ni < 1 || !q || !(dt > 0.0) || !o) return -1;
    if (scheme != ORC_EPI2 && scheme != ORC_EPI3 && scheme != ORC_EXPRB32 &&
        scheme != ORC_EXPRB42)
        return -1;
    const size_t n = (size_t)ni;
    // entropy viscosity: this step's nodal viscosity from q^n and q^{n-1}
    // (q^n itself on a first step); every operator of the step uses it
    orc_mesh mev = *m;
    std::vector<double> nuv;
    if (m->ev_ce > 0.0) {
        nuv.resize(n / 4);
        const int rc0 = orc_entropy_viscosity(m, q, (q_prev && have_prev) ? q_prev : q, dt,
                                              nuv.data());
        if (rc0) return rc0;
        mev.nu = nuv.data();
        m = &mev;
    }
    std::vector<double> qn(q, q + n), Rn(n), w(n);
    std::function<void(const double *, double *)> Ln = [&](const double *x, double *y) {
        orc_jvp(m, qn.data(), x, y);
    };
    int fpos = 0;
    int rc = orc_rhs(m, qn.data(), Rn.data());
    if (s) s->rhs_calls += 1;
    if (rc) return rc;
    std::vector<double> qnew(n);

    if (scheme == ORC_EPI2 || (scheme == ORC_EPI3 && !(q_prev && have_prev))) {
        const double *b[2] = {nullptr, Rn.data()};
        rc = orc_phi_krylov_op(n, Ln, dt, 1, b, w.data(), o, s, &fpos);
        if (rc) return rc;
        for (size_t i = 0; i < n; ++i) qnew[i] = qn[i] + w[i];
    } else if (scheme == ORC_EPI3) {
        std::vector<double> Rp(n), d(n), Ld(n), b2(n);
        rc = orc_rhs(m, q_prev, Rp.data());
        if (rc) return rc;
        for (size_t i = 0; i < n; ++i) d[i] = q_prev[i] - qn[i];
        Ln(d.data(), Ld.data());
        if (s) {
            s->rhs_calls += 1;
            s->jvps += 1;
        }
        for (size_t i = 0; i < n; ++i) b2[i] = (2.0 / 3.0) * (Rp[i] - Rn[i] - Ld[i]) / dt;
        const double *b[3] = {nullptr, Rn.data(), b2.data()};
        rc = orc_phi_krylov_op(n, Ln, dt, 2, b, w.data(), o, s, &fpos);
        if (rc) return rc;
        for (size_t i = 0; i < n; ++i) qnew[i] = qn[i] + w[i];
    } else if (scheme == ORC_EXPRB42) {
        const double *b1[2] = {nullptr, Rn.data()};
        rc = orc_phi_krylov_op(n, Ln, 0.75 * dt, 1, b1, w.data(), o, s, &fpos);
        if (rc) return rc;
        std::vector<double> q2(n), R2(n), d(n), Ld(n), b3(n), w2(n);
        for (size_t i = 0; i < n; ++i) q2[i] = qn[i] + w[i];
        rc = orc_rhs(m, q2.data(), R2.data());
        if (rc) return rc;
        for (size_t i = 0; i < n; ++i) d[i] = q2[i] - qn[i];
        Ln(d.data(), Ld.data());
        if (s) {
            s->rhs_calls += 1;
            s->jvps += 1;
        }
        for (size_t i = 0; i < n; ++i) b3[i] = (32.0 / 9.0) * (R2[i] - Rn[i] - Ld[i]) / (dt * dt);
        const double *b[4] = {nullptr, Rn.data(), nullptr, b3.data()};
        rc = orc_phi_krylov_op(n, Ln, dt, 3, b, w2.data(), o, s, &fpos);
        if (rc) return rc;
        for (size_t i = 0; i < n; ++i) qnew[i] = qn[i] + w2[i];
    } else {  // EXPRB32
        const double *b1[2] = {nullptr, Rn.data()};
        rc = orc_phi_krylov_op(n, Ln, dt, 1, b1, w.data(), o, s, &fpos);
        if (rc) return rc;
        std::vector<double> q2(n), R2(n), d(n), Ld(n), b3(n), w2(n);
        for (size_t i = 0; i < n; ++i) q2[i] = qn[i] + w[i];
        rc = orc_rhs(m, q2.data(), R2.data());
        if (rc) return rc;
        for (size_t i = 0; i < n; ++i) d[i] = q2[i] - qn[i];
        Ln(d.data(), Ld.data());
        if (s) {
            s->rhs_calls += 1;
            s->jvps += 1;
        }
        for (size_t i = 0; i < n; ++i) b3[i] = 2.0 * (R2[i] - Rn[i] - Ld[i]) / (dt * dt);
        const double *b[4] = {nullptr, nullptr, nullptr, b3.data()};
        rc = orc_phi_krylov_op(n, Ln, dt, 3, b, w2.data(), o, s, &fpos);
        if (rc) return rc;
        for (size_t i = 0; i < n; ++i) qnew[i] = q2[i] + w2[i];
    }
    for (size_t i = 0; i < n; ++i) {
        if (!std::isfinite(qnew[i])) return -5;
    }
    if (q_prev)
        for (size_t i = 0; i < n; ++i) q_prev[i] = qn[i];
    for (size_t i = 0; i < n; ++i) q[i] = qnew[i];
    return 0;
}

extern "C" int orc_rk4(const orc_mesh *m, double dt, int nsteps, double *q) {
    const int ni = orc_ndof(m);
    if (ni < 1 || !q || nsteps < 0) return -1;
    const size_t n = (size_t)ni;
    std::vector<double> k1(n), k2(n), k3(n), k4(n), t(n);
    for (int s = 0; s < nsteps; ++s) {
        orc_rhs(m, q, k1.data());
        for (size_t i = 0; i < n; ++i) t[i] = q[i] + 0.5 * dt * k1[i];
        orc_rhs(m, t.data(), k2.data());
        for (size_t i = 0; i < n; ++i) t[i] = q[i] + 0.5 * dt * k2[i];
        orc_rhs(m, t.data(), k3.data());
        for (size_t i = 0; i < n; ++i) t[i] = q[i] + dt * k3[i];
        orc_rhs(m, t.data(), k4.data());
        for (size_t i = 0; i < n; ++i)
            q[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    return 0;
}
