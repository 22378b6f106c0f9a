// Oracle (test infrastructure only): adaptive Krylov evaluation of
//   w = sum_{k=0}^p tau^k phi_k(tau A) b_k
// (eq. linear_combination_of_phifunctions) by Arnoldi projection of the
// augmented matrix (Section 2.3).  The paper runs KIOPS with parameters it
// does not report; this is the fixed, written-out controller both the oracle
// and the GPU library follow:
//
//  1. Scaling.  eta = 2^-round(log2 max_{k>=1} ||b_k||) (1 if all zero).  The
//     augmented operator is
//        Aug [x; y] = [A x + eta sum_{k=1}^p y_k b_{p+1-k}; y_2, ..., y_p, 0]
//     and the start vector z = [b_0; 0, ..., 0, 1/eta]; the top n entries of
//     exp(tau Aug) z are w (similarity by diag(I, I/eta)).
//  2. Tolerance.  nu = ||b_0|| + sum_k tau^k ||b_k|| / k!, tol_abs = tol nu;
//     a substep of length dtau is accepted when err <= tol_abs dtau / tau.
//  3. Substeps.  beta = ||z||, Arnoldi with classical Gram-Schmidt applied
//     twice from v_1 = z / beta over the n + p entries (Euclidean product).
//     At j = m_min and every check_every iterations after it (and at m_max)
//     F = expm(dtau Hhat_j), Hhat_j = [[H_j, 0], [h_{j+1,j} e_j^T, 0]],
//     err = beta |F_{j+1,1}|.  Happy breakdown (h_{j+1,j} <= 1e-12 ||H||_F)
//     is exact: the substep takes the whole remaining interval.  If m_max is
//     reached without passing, dtau shrinks on the same basis,
//        dtau <- RND2(dtau max(0.2, 0.9 (tol_abs dtau/tau / err)^(1/m_max))),
//     until it passes.  Accept: z <- beta V_j F_{1:j,1}; the next dtau is
//        min(remaining, RND2(dtau clamp(0.9 (tol_abs dtau/tau/err)^(1/j), 1, 5))).
//     RND2 rounds up to two significant decimal digits.
//  4. The top n entries of z are the result.
// A forced schedule (list of (m, dtau, last)) replays given substeps with no
// error checks.
//
// Cost-based adaptivity (adapt = 1, after KIOPS, which the paper cites for its
// phi evaluations in Section 2.3; the paper gives no parameters, so these are
// the written rules both the oracle and the GPU library follow).  The error is
// checked only at the target size m of the substep, as
//    omega = err tau / (tol_abs dtau)       (accept when omega <= 1),
// and after every check two candidates for going on are priced:
//    A: keep m, dtau_A = RND2(dtau clamp((0.8/omega)^(1/q), 0.2, 5)),
//    B: keep dtau (capped to R), m_B = ceil(m + ln(omega_B/0.8)/ln kappa)
//       clamped to [m_min, min(m_max, ceil(4m/3))], omega_B =
//       omega (min(dtau, R)/dtau)^q,
// each at ceil(R/dtau') substeps of cost C(m') = m'^2 + 9m' (full
// orthogonalization; m'(2L + 7) with a window of L), R the interval still to
// cover; the cheaper one is taken (A on a tie).  omega and omega_B are rounded up
// to a power of 10^(1/4), q and kappa to two significant digits (RND2), before
// they are used, so both implementations take the same decisions (a tiny error
// estimate has few correct digits).  q, the order of omega in dtau,
// is m (the Expokit estimate) until two checks of one substep share m and
// differ in dtau, then max(1, ln(omega/omega')/ln(dtau/dtau')); kappa, the factor one more
// Krylov vector gains, is 2 until two checks share dtau and differ in m, then
// max(1.1, (omega'/omega)^(1/(m - m'))).  A rejected check retries with A on
// the same basis (dtau_A then at most RND2(0.9 dtau)) or extends the same
// Arnoldi process to m_B; at m_max only A is possible.  An accepted substep
// hands the chosen candidate to the next one (dtau capped to what remains).
// The first substep starts at m = m_init (m_min if 0) and dtau = tau; a happy
// breakdown is exact and takes the whole remaining interval as above.
//
// Incomplete orthogonalization (iop = L > 0, the IOP option of KIOPS cited in
// Section 2.3): each new vector is orthogonalized, with one classical
// Gram-Schmidt pass, against the L most recent basis vectors only (the one it
// was computed from included), then normalised by its explicit norm.  H is
// then banded (h_{i,j} = 0 for i < j + 1 - L) and V is orthonormal only
// within windows of L consecutive vectors; everything else is unchanged.
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>

namespace {

using Op = std::function<void(const double *x, double *y)>;  // y = A x

// Dot product in fixed chunks, summed in chunk order: the result does not
// depend on the number of threads.
double dot(const double *a, const double *b, size_t n) {
    const size_t chunk = 4096;
    const size_t nc = (n + chunk - 1) / chunk;
    std::vector<double> part(nc, 0.0);
#pragma omp parallel for schedule(static)
    for (long long c = 0; c < (long long)nc; ++c) {
        double acc = 0.0;
        const size_t lo = (size_t)c * chunk, hi = std::min(n, lo + chunk);
        for (size_t i = lo; i < hi; ++i) acc += a[i] * b[i];
        part[c] = acc;
    }
    double s = 0.0;
    for (size_t c = 0; c < nc; ++c) s += part[c];
    return s;
}

double norm2(const double *a, size_t n) { return std::sqrt(dot(a, a, n)); }

// Rounds up to a power of 10^(1/4) (quarter decades): error ratios are used
// on this grid, which is coarse next to the accuracy of a tiny error estimate.
double q4(double x) {
    if (!(x > 0.0)) return x;
    return std::pow(10.0, std::ceil(4.0 * std::log10(x)) / 4.0);
}

double rnd2(double x) {
    if (!(x > 0.0)) return x;
    const double s = std::pow(10.0, std::floor(std::log10(x)) - 1.0);
    return std::ceil(x / s) * s;
}

void log_substep(orc_kstats *st, int m, int last, double dtau) {
    if (!st) return;
    st->substeps += 1;
    if (st->log && st->log_len < st->log_cap) {
        st->log[st->log_len].m = m;
        st->log[st->log_len].last = last;
        st->log[st->log_len].dtau = dtau;
    }
    st->log_len += 1;
}

// F = expm(dtau Hhat_j), (j+1) x (j+1), from the Hessenberg H stored with
// leading dimension ldh (H[r * ldh + c]).
int small_expm(const std::vector<double> &H, int ldh, int j, double dtau, std::vector<double> &F) {
    const int nh = j + 1;
    std::vector<double> X((size_t)nh * nh, 0.0);
    for (int r = 0; r <= j; ++r)
        for (int c = 0; c < j; ++c) X[(size_t)r * nh + c] = dtau * H[(size_t)r * ldh + c];
    F.assign((size_t)nh * nh, 0.0);
    return orc_expm(nh, X.data(), F.data());
}

// Orthogonalizes w against the basis vectors V[0..j-1] by classical
// Gram-Schmidt -- two passes over all of them (iop = 0), or one pass over the
// last iop of them -- and adds the coefficients to column j-1 of H.
void orthogonalize(const std::vector<double> &V, size_t na, std::vector<double> &H, int ldh,
                   int j, int iop, double *w) {
    const int i_lo = (iop > 0) ? std::max(0, j - iop) : 0;
    for (int pass = 0; pass < (iop > 0 ? 1 : 2); ++pass) {
        std::vector<double> h(j, 0.0);
        for (int i = i_lo; i < j; ++i) h[i] = dot(&V[(size_t)i * na], w, na);
        for (int i = i_lo; i < j; ++i) {
            const double *vi = &V[(size_t)i * na];
            for (size_t r = 0; r < na; ++r) w[r] -= h[i] * vi[r];
            H[(size_t)i * ldh + (j - 1)] += h[i];
        }
    }
}

// Cost of one substep of Krylov size m (in state-vector passes): the operator
// and the two Gram-Schmidt sweeps of each Arnoldi step, m^2 + 9m with full
// orthogonalization, m (2L + 7) with a window of L.
double substep_cost(int m, int iop) {
    return iop > 0 ? (double)m * (2.0 * iop + 7.0) : (double)m * m + 9.0 * m;
}

// The two candidates after a check at (m, dtau) with error ratio omega: A
// keeps m and takes dtau_a, B keeps dtau and takes m_b; *take_a when A is the
// cheaper way to cover rem.  rejected: dtau_a < dtau is enforced.
struct CostChoice {
    double dtau_a;
    int m_b;
    bool take_a;
};
CostChoice cost_choice(int m, double dtau, double omega, double q, double kappa, double rem,
                       bool rejected, const orc_kopts *o) {
    const double gam = 0.8;
    const double om = std::max(omega, 1e-300);
    CostChoice c;
    double fa = std::pow(gam / om, 1.0 / q);
    fa = std::min(rejected ? 0.9 : 5.0, std::max(0.2, fa));
    c.dtau_a = rnd2(dtau * fa);
    // B takes min(dtau, rem): its error ratio scales by (that / dtau)^q
    const double dtb = (rem > 0.0) ? std::min(dtau, rem) : dtau;
    const double om_b = q4(std::max(om * std::pow(dtb / dtau, q), 1e-300));
    const int hi = std::min(o->m_max, (4 * m + 2) / 3);
    const double mb = std::ceil(m + std::log(om_b / gam) / std::log(kappa));
    c.m_b = (int)std::min((double)hi, std::max((double)o->m_min, mb));
    if (!(rem > 0.0)) {
        c.take_a = true;  // nothing left to cover
        return c;
    }
    const double ca = std::ceil(rem / std::min(c.dtau_a, rem)) * substep_cost(m, o->iop);
    const double cb = std::ceil(rem / dtb) * substep_cost(c.m_b, o->iop);
    c.take_a = ca <= cb || (rejected && c.m_b <= m);
    return c;
}

}  // namespace

extern "C" int orc_arnoldi_dense(int n, const double *A, const double *b, int m, int iop,
                                 double *Vout, double *Hout) {
    if (n < 1 || m < 1 || iop < 0 || !A || !b || !Vout || !Hout) return -1;
    const size_t na = (size_t)n;
    std::vector<double> V((size_t)(m + 1) * na, 0.0), H((size_t)(m + 1) * m, 0.0), w(na);
    const double beta = norm2(b, na);
    if (!(beta > 0.0)) return -1;
    for (size_t r = 0; r < na; ++r) V[r] = b[r] / beta;
    for (int j = 1; j <= m; ++j) {
        const double *vj = &V[(size_t)(j - 1) * na];
        for (int r = 0; r < n; ++r) {
            double acc = 0.0;
            for (int c = 0; c < n; ++c) acc += A[(size_t)r * n + c] * vj[c];
            w[r] = acc;
        }
        orthogonalize(V, na, H, m, j, iop, w.data());
        const double hn = norm2(w.data(), na);
        if (!(hn > 0.0)) return -1;
        H[(size_t)j * m + (j - 1)] = hn;
        for (size_t r = 0; r < na; ++r) V[(size_t)j * na + r] = w[r] / hn;
    }
    std::copy(V.begin(), V.end(), Vout);
    std::copy(H.begin(), H.end(), Hout);
    return 0;
}

// Shared by the dense and DG entry points and by the steppers.  *fpos is the
// cursor into the forced schedule (advanced by the substeps replayed).
int orc_phi_krylov_op(size_t n, const Op &A, double tau, int p, const double *const *b,
                      double *out, const orc_kopts *o, orc_kstats *st, int *fpos) {
    if (!o || !out || p < 0 || p > 8 || !(tau >= 0.0)) return -1;
    if (!(o->tol > 0.0) || o->m_min < 1 || o->m_max < o->m_min || o->m_max > 256 ||
        o->check_every < 1 || o->iop < 0)
        return -1;
    const bool forced = o->forced && o->n_forced > 0;
    const size_t na = n + (size_t)p;
    auto bk = [&](int k) -> const double * { return b ? b[k] : nullptr; };
    if (st) st->phi_calls += 1;

    // 1. scaling and 2. tolerance
    double bmax = 0.0;
    std::vector<double> bnorm(p + 1, 0.0);
    for (int k = 0; k <= p; ++k)
        if (bk(k)) bnorm[k] = norm2(bk(k), n);
    for (int k = 1; k <= p; ++k) bmax = std::max(bmax, bnorm[k]);
    const double eta = (bmax > 0.0) ? std::ldexp(1.0, -(int)std::lround(std::log2(bmax))) : 1.0;
    double nu = bnorm[0], tk = 1.0, fact = 1.0;
    for (int k = 1; k <= p; ++k) {
        tk *= tau;
        fact *= k;
        nu += tk * bnorm[k] / fact;
    }
    if (!std::isfinite(nu)) return -5;
    if (nu == 0.0 || tau == 0.0) {
        for (size_t i = 0; i < n; ++i) out[i] = bk(0) ? bk(0)[i] : 0.0;
        return 0;
    }
    const double tol_abs = o->tol * nu;

    auto aug = [&](const double *x, double *y) {
        A(x, y);
        for (int k = 1; k <= p; ++k) {
            const double *bb = bk(p + 1 - k);
            if (!bb) continue;
            const double yk = eta * x[n + k - 1];
            for (size_t i = 0; i < n; ++i) y[i] += yk * bb[i];
        }
        for (int k = 0; k + 1 < p; ++k) y[n + k] = x[n + k + 1];
        if (p > 0) y[n + p - 1] = 0.0;
    };

    std::vector<double> z(na, 0.0);
    if (bk(0))
        for (size_t i = 0; i < n; ++i) z[i] = bk(0)[i];
    if (p > 0) z[n + p - 1] = 1.0 / eta;

    int mmax = o->m_max;
    if (forced)
        for (int k = *fpos; k < o->n_forced; ++k) mmax = std::max(mmax, o->forced[k].m);
    if (mmax > 256) return -1;
    const int ldh = mmax;
    std::vector<double> V((size_t)(mmax + 1) * na), H((size_t)(mmax + 1) * mmax), w(na), F;

    auto expm_at = [&](int j, double dt) {
        if (st) st->checks += 1;
        return small_expm(H, ldh, j, dt, F);
    };

    // one Arnoldi step: v_{j} from v_{j-1} (1-based j); 1 on a happy breakdown
    auto arnoldi_step = [&](int j) -> int {
        const double *vj = &V[(size_t)(j - 1) * na];
        aug(vj, w.data());
        if (st) {
            st->krylov_iters += 1;
            st->jvps += 1;
        }
        orthogonalize(V, na, H, ldh, j, o->iop, w.data());
        const double hn = norm2(w.data(), na);
        if (!std::isfinite(hn)) return -5;
        H[(size_t)j * ldh + (j - 1)] = hn;
        double hf = 0.0;
        for (int r = 0; r <= j; ++r)
            for (int c = 0; c < j; ++c) hf += H[(size_t)r * ldh + c] * H[(size_t)r * ldh + c];
        hf = std::sqrt(hf);
        if (hn <= 1e-12 * hf) {
            H[(size_t)j * ldh + (j - 1)] = 0.0;
            if (st) st->breakdown += 1;
            return 1;
        }
        for (size_t r = 0; r < na; ++r) V[(size_t)j * na + r] = w[r] / hn;
        return 0;
    };

    // z <- beta V_j F_{1:j,1}
    auto combine = [&](int j_acc, double beta) {
        const int nh = j_acc + 1;
        std::fill(z.begin(), z.end(), 0.0);
        for (int i = 0; i < j_acc; ++i) {
            const double c = beta * F[(size_t)i * nh + 0];
            const double *vi = &V[(size_t)i * na];
            for (size_t r = 0; r < na; ++r) z[r] += c * vi[r];
        }
    };

    if (o->adapt == 1 && !forced) {
        // cost-based choice of the Krylov size and the substep
        int m = std::min(o->m_max, std::max(o->m_min, o->m_init > 0 ? o->m_init : o->m_min));
        double t_done = 0.0, dtau = tau;
        while (true) {
            const double rem0 = tau - t_done;
            bool last = !(dtau < rem0);
            if (last) dtau = rem0;
            const double beta = norm2(z.data(), na);
            if (!std::isfinite(beta)) return -5;
            if (beta == 0.0) {
                for (size_t i = 0; i < n; ++i) out[i] = 0.0;
                return 0;
            }
            for (size_t i = 0; i < na; ++i) V[i] = z[i] / beta;
            std::fill(H.begin(), H.end(), 0.0);
            int j = 0, j_acc = 0;
            double err = 0.0;
            double q = m, kappa = 2.0;
            double om_p = 0.0, dt_p = 0.0;
            int m_p = -1;
            CostChoice next{};
            while (true) {
                bool brk = false;
                while (j < m) {
                    const int rc = arnoldi_step(j + 1);
                    if (rc < 0) return rc;
                    ++j;
                    if (rc == 1) {
                        brk = true;
                        break;
                    }
                }
                if (brk) {
                    // happy breakdown: exact, the whole remaining interval
                    dtau = rem0;
                    last = true;
                    if (expm_at(j, dtau)) return -5;
                    err = 0.0;
                    j_acc = j;
                    next = CostChoice{dtau, m, true};
                    break;
                }
                if (expm_at(m, dtau)) return -5;
                err = beta * std::fabs(F[(size_t)m * (m + 1) + 0]);
                if (!std::isfinite(err)) return -5;
                // omega rounded up to a quarter decade, q and kappa to two
                // significant digits, so that decisions do not turn on the
                // last bits of err
                const double om = q4(err * tau / (tol_abs * dtau));
                if (m_p == m && dt_p != dtau && om_p > 0.0 && om > 0.0)
                    q = rnd2(std::max(1.0, std::log(om / om_p) / std::log(dtau / dt_p)));
                if (m_p >= 0 && m_p != m && dt_p == dtau && om > 0.0 && om_p > 0.0)
                    kappa = rnd2(std::max(1.1, std::pow(om_p / om, 1.0 / (m - m_p))));
                const bool ok = om <= 1.0;
                const double rem = ok ? rem0 - dtau : rem0;
                next = cost_choice(m, dtau, om, q, kappa, rem, !ok, o);
                if (ok) {
                    j_acc = m;
                    break;
                }
                if (st) st->rejects += 1;
                om_p = om;
                dt_p = dtau;
                m_p = m;
                if (next.take_a) {
                    dtau = next.dtau_a;  // same basis, shorter substep
                    last = false;
                    if (!(dtau > 1e-12 * tau)) return -4;
                } else {
                    m = next.m_b;  // extend the Arnoldi process
                }
            }
            combine(j_acc, beta);
            t_done += dtau;
            log_substep(st, j_acc, last ? 1 : 0, dtau);
            if (st) st->err_est = err;
            const double rem = tau - t_done;
            if (last || !(rem > 1e-15 * tau)) {
                if (!last && st && st->log && st->log_len >= 1 && st->log_len <= st->log_cap)
                    st->log[st->log_len - 1].last = 1;
                if (st) st->m_next = next.take_a ? m : next.m_b;
                break;
            }
            if (next.take_a)
                dtau = next.dtau_a;
            else
                m = next.m_b;
        }
        for (size_t i = 0; i < n; ++i) out[i] = z[i];
        return 0;
    }

    double t_done = 0.0, dtau = tau;
    bool reaches_end = true;  // the current dtau covers the rest of [0, tau]
    while (true) {
        int m_target = o->m_max;
        double dt_sub = dtau;
        bool sub_last = reaches_end;
        if (forced) {
            if (*fpos >= o->n_forced) return -1;
            m_target = o->forced[*fpos].m;
            dt_sub = o->forced[*fpos].dtau;
            sub_last = o->forced[*fpos].last != 0;
            if (m_target < 1 || m_target > mmax || !(dt_sub > 0.0)) return -1;
        }
        const double beta = norm2(z.data(), na);
        if (!std::isfinite(beta)) return -5;
        if (beta == 0.0) {
            for (size_t i = 0; i < n; ++i) out[i] = 0.0;
            return 0;
        }
        for (size_t i = 0; i < na; ++i) V[i] = z[i] / beta;
        std::fill(H.begin(), H.end(), 0.0);

        int j_acc = 0;
        double err = 0.0;
        for (int j = 1; j <= m_target; ++j) {
            const double *vj = &V[(size_t)(j - 1) * na];
            aug(vj, w.data());
            if (st) {
                st->krylov_iters += 1;
                st->jvps += 1;
            }
            orthogonalize(V, na, H, ldh, j, o->iop, w.data());
            const double hn = norm2(w.data(), na);
            if (!std::isfinite(hn)) return -5;
            H[(size_t)j * ldh + (j - 1)] = hn;
            double hf = 0.0;
            for (int r = 0; r <= j; ++r)
                for (int c = 0; c < j; ++c) hf += H[(size_t)r * ldh + c] * H[(size_t)r * ldh + c];
            hf = std::sqrt(hf);
            const bool brk = hn <= 1e-12 * hf;
            if (brk) {
                H[(size_t)j * ldh + (j - 1)] = 0.0;
                if (st) st->breakdown += 1;
            } else {
                for (size_t r = 0; r < na; ++r) V[(size_t)j * na + r] = w[r] / hn;
            }

            if (forced) {
                if (brk || j == m_target) {
                    if (expm_at(j, dt_sub)) return -5;
                    j_acc = j;
                    break;
                }
                continue;
            }
            const bool check =
                brk || j == o->m_max || (j >= o->m_min && (j - o->m_min) % o->check_every == 0);
            if (!check) continue;
            if (brk) {
                dt_sub = tau - t_done;
                sub_last = true;
                if (expm_at(j, dt_sub)) return -5;
                err = 0.0;
                j_acc = j;
                break;
            }
            if (expm_at(j, dt_sub)) return -5;
            err = beta * std::fabs(F[(size_t)j * (j + 1) + 0]);
            if (err <= tol_abs * dt_sub / tau) {
                j_acc = j;
                break;
            }
            if (j == o->m_max) {
                // shrink the substep on the same basis until it passes
                while (err > tol_abs * dt_sub / tau) {
                    const double ratio = tol_abs * dt_sub / tau / err;
                    const double fac = std::max(0.2, 0.9 * std::pow(ratio, 1.0 / o->m_max));
                    dt_sub = rnd2(dt_sub * fac);
                    sub_last = false;
                    if (st) st->rejects += 1;
                    if (!(dt_sub > 1e-12 * tau)) return -4;
                    if (expm_at(j, dt_sub)) return -5;
                    err = beta * std::fabs(F[(size_t)j * (j + 1) + 0]);
                }
                j_acc = j;
                break;
            }
        }
        if (j_acc == 0) return -1;

        // accept: z <- beta V_j F_{1:j,1}
        const int nh = j_acc + 1;
        std::fill(z.begin(), z.end(), 0.0);
        for (int i = 0; i < j_acc; ++i) {
            const double c = beta * F[(size_t)i * nh + 0];
            const double *vi = &V[(size_t)i * na];
            for (size_t r = 0; r < na; ++r) z[r] += c * vi[r];
        }
        t_done += dt_sub;
        log_substep(st, j_acc, sub_last ? 1 : 0, dt_sub);
        if (st) st->err_est = err;
        if (forced) *fpos += 1;
        if (sub_last) break;
        const double rem = tau - t_done;
        if (!(rem > 1e-15 * tau)) {
            // the accepted substeps already cover [0, tau]: the last one ends
            // the evaluation, and the log says so (a replay stops there too)
            if (st && st->log && st->log_len >= 1 && st->log_len <= st->log_cap)
                st->log[st->log_len - 1].last = 1;
            break;
        }
        if (forced) continue;

        const double ratio = (err > 0.0) ? tol_abs * dt_sub / tau / err : 0.0;
        double fac = (err > 0.0) ? 0.9 * std::pow(ratio, 1.0 / j_acc) : 5.0;
        fac = std::min(5.0, std::max(1.0, fac));
        const double cand = rnd2(dt_sub * fac);
        if (cand >= rem) {
            dtau = rem;
            reaches_end = true;
        } else {
            dtau = cand;
            reaches_end = false;
        }
    }
    for (size_t i = 0; i < n; ++i) out[i] = z[i];
    return 0;
}

extern "C" int orc_phi_krylov_dense(int n, const double *A, double tau, int p,
                                    const double *const *b, double *out, const orc_kopts *o,
                                    orc_kstats *s) {
    if (n < 1 || !A) return -1;
    Op op = [&](const double *x, double *y) {
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += A[(size_t)i * n + j] * x[j];
            y[i] = acc;
        }
    };
    int pos = 0;
    return orc_phi_krylov_op((size_t)n, op, tau, p, b, out, o, s, &pos);
}

extern "C" int orc_phi_krylov_dg(const orc_mesh *m, const double *qref, double tau, int p,
                                 const double *const *b, double *out, const orc_kopts *o,
                                 orc_kstats *s) {
    const int n = orc_ndof(m);
    if (n < 1 || !qref) return -1;
    Op op = [&](const double *x, double *y) { orc_jvp(m, qref, x, y); };
    int pos = 0;
    return orc_phi_krylov_op((size_t)n, op, tau, p, b, out, o, s, &pos);
}
