// The adaptive Krylov controller and the exponential steppers, written once as
// coroutines over an executor.
//
// The controller (Section 2.3: Krylov projection of the augmented matrix whose
// exponential yields the phi combination; the paper leaves the adaptivity
// parameters unreported, so the rules below are a fixed written specification
// that the test oracle follows too) makes every decision on the host from a
// few scalars per check; all state-sized arithmetic is launched on the
// executor's stream.  The executor decides when the Arnoldi steps and the
// small exponentials run:
//   * the stand-alone entry points launch each operation at once and wait in
//     place (no coroutine ever suspends);
//   * the solve server collects the same Arnoldi step of many solves into
//     grouped launches and all pending checks into one batched launch per
//     tick, suspending each solve until its results are there.
// Both make the same decisions from the same numbers, so a solve gives the
// same bits alone, in the server, or among other solves.
//
// An executor X provides
//   hipStream_t stream();
//   awaitable<int> iterate(m, a, k, naug_nz, const CheckReq *chk, Check *c, bool iop):
//       the Arnoldi step k (linear operator on u_{k-1}, dot pass over the a.nv
//       vectors from a.basis, finish, update sweep; it finishes dimension
//       k - 1) and, if chk, the check of dimension k - 1 behind it; iop: the
//       incomplete orthogonalization's finish and update (window in a.basis);
//   awaitable<int> check(m, req, Check *c): a check on the current basis;
//   awaitable<int> wait_check(m, c): the check's header is in the pinned mirror;
//   int after_check(m, c): the stream waits for the check's coefficients;
//   awaitable<int> readback(m): device-to-host copies enqueued so far are done;
//   awaitable<int> finish(m): the end of one library call;
//   static constexpr int kLookahead: how many Arnoldi steps a check's decision
//       may lag behind the step that launched it (1 .. kCheckSlots - 2).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "runtime.h"
#include "task.h"

namespace expdg {

// A check asked for: dimension j, substep dtau, result slot (0 or 1).
struct CheckReq {
    int j;
    double dtau;
    int slot;
};

// A check enqueued (tick: the server's batch that runs it).
struct Check {
    int j = 0;
    int slot = 0;
    long long tick = 0;
};

struct CheckResult {
    double err;
    int singular, brk, nonfinite;
};

// The header of a check as the small-exponential kernel wrote it into the
// pinned mirror.  The Krylov flags are read while the next (speculative)
// Arnoldi step may already run, so a breakdown or a non-finite norm counts for
// this check only if it happened at a dimension <= j.
inline CheckResult read_check(const expdg_mesh *m, const Check &c) {
    const volatile double *pv = m->pin + kPinSlots + c.slot * 8;
    CheckResult r;
    r.err = pv[kSlotErr];
    r.singular = pv[kSlotSingular] != 0.0;
    const int brk = (int)pv[kSlotBreak];
    const int nf = (int)pv[kSlotNonfinite];
    r.brk = (brk > 0 && brk <= c.j) ? brk : 0;
    r.nonfinite = (nf > 0 && nf <= c.j) ? 1 : 0;
    return r;
}

// Scalars of one phi evaluation shared by its loop and its decisions.
template <typename T, typename X>
struct PhiRun {
    X &x;
    expdg_mesh *m;
    const expdg_krylov_opts *o;
    expdg_krylov_stats *st;
    double tau = 0.0, tol_abs = 0.0;
    double t_done = 0.0, dt_sub = 0.0, err = 0.0;
    bool sub_last = true;
    int j_acc = 0, nchecks = 0;
    Check acc;

    PhiRun(X &x_, expdg_mesh *m_, const expdg_krylov_opts *o_, expdg_krylov_stats *st_)
        : x(x_), m(m_), o(o_), st(st_) {}

    CheckReq req(int j, double dtau) {
        if (st) st->checks += 1;
        return CheckReq{j, dtau, (nchecks++) % kCheckSlots};
    }

    // Decision on check c: accept (possibly after shrinking the substep on the
    // same basis at m_max), take a happy breakdown, or go on (done = false).
    Task<int> decide(Check c, bool *done) {
        *done = false;
        CO_TRY(co_await x.wait_check(m, c));
        const CheckResult r = read_check(m, c);
        if (r.nonfinite) co_return fail(EXPDG_ENONFINITE, "non-finite Krylov norm");
        if (r.brk > 0) {
            // happy breakdown: the space is invariant, take the whole remaining interval
            dt_sub = tau - t_done;
            sub_last = true;
            Check bc;
            CO_TRY(co_await x.check(m, req(r.brk, dt_sub), &bc));
            CO_TRY(co_await x.wait_check(m, bc));
            const CheckResult br = read_check(m, bc);
            if (br.singular) co_return fail(EXPDG_ENONFINITE, "singular Pade denominator");
            if (st) st->breakdown += 1;
            err = 0.0;
            j_acc = r.brk;
            acc = bc;
            *done = true;
            co_return EXPDG_OK;
        }
        if (r.singular) co_return fail(EXPDG_ENONFINITE, "singular Pade denominator");
        if (!std::isfinite(r.err)) co_return fail(EXPDG_ENONFINITE, "non-finite error estimate");
        if (r.err <= tol_abs * dt_sub / tau) {
            err = r.err;
            j_acc = c.j;
            acc = c;
            *done = true;
            co_return EXPDG_OK;
        }
        if (c.j == o->m_max) {
            // shrink on the same basis until it passes
            double e = r.err;
            Check sc = c;
            while (e > tol_abs * dt_sub / tau) {
                const double ratio = tol_abs * dt_sub / tau / e;
                const double fac = std::max(0.2, 0.9 * std::pow(ratio, 1.0 / o->m_max));
                dt_sub = round2(dt_sub * fac);
                sub_last = false;
                if (st) st->rejects += 1;
                if (!(dt_sub > 1e-12 * tau))
                    co_return fail(EXPDG_ENOCONV, "Krylov substep below its floor");
                CO_TRY(co_await x.check(m, req(c.j, dt_sub), &sc));
                CO_TRY(co_await x.wait_check(m, sc));
                const CheckResult sr = read_check(m, sc);
                if (sr.singular || !std::isfinite(sr.err))
                    co_return fail(EXPDG_ENONFINITE, "non-finite error estimate");
                e = sr.err;
            }
            err = e;
            j_acc = c.j;
            acc = sc;
            *done = true;
        }
        co_return EXPDG_OK;
    }
};

// Error ratios of the cost-based adaptivity are used rounded up to a power of
// 10^(1/4) (a tiny error estimate has few correct digits; the oracle rounds
// the same way).
inline double quarter_decade(double x) {
    if (!(x > 0.0)) return x;
    return std::pow(10.0, std::ceil(4.0 * std::log10(x)) / 4.0);
}

// Cost-based adaptivity (expdg_krylov_opts.adapt = 1): state-vector passes of
// one substep of Krylov size m (the operator and the two Gram-Schmidt sweeps
// of each Arnoldi step).
inline double adapt_substep_cost(int m, int iop) {
    return iop > 0 ? (double)m * (2.0 * iop + 7.0) : (double)m * m + 9.0 * m;
}

// The two ways to go on after a check at size m and substep dtau with error
// ratio omega (q, kappa: the current order estimates; rem: the interval still
// to cover): A keeps m and takes dtau_a, B keeps dtau and takes m_b.
struct AdaptChoice {
    double dtau_a;
    int m_b;
    bool take_a;
};
inline AdaptChoice adapt_choice(int m, double dtau, double omega, double q, double kappa,
                                double rem, bool rejected, const expdg_krylov_opts *o) {
    constexpr double kSafety = 0.8;
    const double om = std::max(omega, 1e-300);
    AdaptChoice c;
    const double f = std::min(rejected ? 0.9 : 5.0,
                              std::max(0.2, std::pow(kSafety / om, 1.0 / q)));
    c.dtau_a = round2(dtau * f);
    // B takes min(dtau, rem): its error ratio scales by (that / dtau)^q
    const double dtb = (rem > 0.0) ? std::min(dtau, rem) : dtau;
    const double om_b = quarter_decade(std::max(om * std::pow(dtb / dtau, q), 1e-300));
    const int hi = std::min(o->m_max, (4 * m + 2) / 3);
    const double mb = std::ceil(m + std::log(om_b / kSafety) / std::log(kappa));
    c.m_b = (int)std::min((double)hi, std::max((double)o->m_min, mb));
    if (!(rem > 0.0)) {
        c.take_a = true;
        return c;
    }
    const double cost_a = std::ceil(rem / std::min(c.dtau_a, rem)) * adapt_substep_cost(m, o->iop);
    const double cost_b = std::ceil(rem / dtb) * adapt_substep_cost(c.m_b, o->iop);
    c.take_a = cost_a <= cost_b || (rejected && c.m_b <= m);
    return c;
}

// Awaits a sub-task, reporting a frame allocation failure as ENOMEM.
#define CO_AWAIT_TASK(task_expr)                                                   \
    do {                                                                           \
        auto t_ = (task_expr);                                                     \
        if (!t_.valid()) co_return ::expdg::fail(EXPDG_ENOMEM, "coroutine frame"); \
        CO_TRY(co_await t_);                                                       \
    } while (0)

// w = sum_{k=0}^{p} tau^k phi_k(tau L~) b_k by the augmented Krylov method
// (Section 2.3), with L~ the linear operator frozen at qref.  b[k] == nullptr
// is a zero vector.  *fpos walks a forced substep schedule.  lin_ready: the
// frozen fields of qref are already in the workspace.  nested: called inside a
// step, whose own end waits for the device, so this evaluation ends without
// waiting (a speculative check may still run on a side stream; it only
// writes its own result slot, and a later check that reuses the slot queues
// behind it on the same side stream).
template <typename T, typename X>
Task<int> phi_co(X &x, expdg_mesh *m, const T *qref, double tau, int p, const T *const *b, T *out,
                 const expdg_krylov_opts *o, expdg_krylov_stats *st, int *fpos, bool lin_ready,
                 bool nested) {
    hipStream_t s = x.stream();
    const size_t n = m->n, L = n + (size_t)p;
    const size_t stride = m->stride;
    T *V = (T *)m->V;
    KrylovDev &kd = m->kd;
    const bool forced = o->n_forced > 0;
    const bool iop = o->iop > 0;
    const int lookahead = X::kLookahead + (iop ? 1 : 0);  // at most kCheckSlots - 2
    const RowPartition rp = row_partition(L);
    if (st) st->phi_calls += 1;

    // 1. scaling and 2. tolerance: norms of b_0..b_p
    const T *bx[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k <= p; ++k) bx[k] = b ? b[k] : nullptr;
    // (written straight into the mapped pinned mirror)
    CO_HIPTRY(launch_norms<T>(bx, p + 1, n, kd.part, m->pin_dev + kPinNorms, s));
    CO_TRY(co_await x.readback(m));
    double bn[4] = {0, 0, 0, 0};
    for (int k = 0; k <= p; ++k) bn[k] = bx[k] ? m->pin[kPinNorms + k] : 0.0;
    double bmax = 0.0;
    for (int k = 1; k <= p; ++k) bmax = std::max(bmax, bn[k]);
    const double eta = (bmax > 0.0) ? std::ldexp(1.0, -(int)std::lround(std::log2(bmax))) : 1.0;
    double nu = bn[0], tk = 1.0, fact = 1.0;
    for (int k = 1; k <= p; ++k) {
        tk *= tau;
        fact *= k;
        nu += tk * bn[k] / fact;
    }
    if (!std::isfinite(nu)) co_return fail(EXPDG_ENONFINITE, "non-finite input norm");
    if (nu == 0.0 || tau == 0.0) {
        if (bx[0])
            CO_HIPTRY(launch_copy(bx[0], out, n, s));
        else
            CO_HIPTRY(launch_fill<T>(out, 0.0, n, s));
        if (!nested) CO_TRY(co_await x.finish(m));
        co_return EXPDG_OK;
    }
    PhiRun<T, X> R(x, m, o, st);
    R.tau = tau;
    R.tol_abs = o->tol * nu;

    // z = [b_0; 0, ..., 0, 1/eta] lives in V_0; flags cleared
    CO_HIPTRY(launch_phi_init<T>(V, bx[0], n, p, 1.0 / eta, kd.flags, s));

    if (!lin_ready) CO_HIPTRY(prepare_lin<T>(m, qref, s));
    OpArgs<T> a = op_args<T>(m);
    a.q = qref;
    a.lin = (const T *)m->lin;
    a.eta = eta;
    // the dot pass of each Arnoldi step runs inside the 2D/3D linear operator (a
    // Burgers tile has too little work to carry it: separate pass there)
    const bool fuse_dots = m->d.equation != EXPDG_BURGERS1D;
    a.basis = V;
    a.bstride = stride;
    a.dpart = kd.part;
    a.dnb = dg_blocks(m->d.equation, m->d.p, m->K);
    a.dots = fuse_dots ? 1 : 0;
    a.vscale = nullptr;  // the operator acts on the stored, unscaled vector
    a.naug = p;
    int naug_nz = 0;
    for (int k = 1; k <= p; ++k) {
        a.aug[k - 1] = bx[p + 1 - k];
        naug_nz += bx[p + 1 - k] ? 1 : 0;
    }
    const double eb = (double)sizeof(T);

    if (o->adapt == 1 && !forced) {
        // cost-based choice of the Krylov size and the substep: the error is
        // checked at the target size mt only; a rejection re-checks the same
        // basis with a shorter substep or extends the Arnoldi process
        int mt = std::min(o->m_max, std::max(o->m_min, o->m_init > 0 ? o->m_init : o->m_min));
        double dtau = tau;
        while (true) {
            const double rem0 = tau - R.t_done;
            R.sub_last = !(dtau < rem0);
            R.dt_sub = R.sub_last ? rem0 : dtau;
            CO_TRY(prof_begin(m, EXPDG_K_GS_NORM));
            CO_HIPTRY(launch_gs_norm<T>(V, L, rp, kd.part, s));
            CO_TRY(prof_end(m, EXPDG_K_GS_NORM, (double)L * eb));
            CO_TRY(prof_begin(m, EXPDG_K_GS_FINISH));
            CO_HIPTRY(launch_gs_finish_norm(kd.part, rp, kd.H, kd.S, kd.flags, kd.res, s));
            CO_TRY(prof_end(m, EXPDG_K_GS_FINISH, 8.0 * rp.nrb));
            int k = 0;  // Arnoldi steps of this substep (step k finishes dimension k - 1)
            double q = mt, kappa = 2.0, om_p = 0.0, dt_p = 0.0;
            int m_p = -1;
            AdaptChoice next{};
            Check pend;
            bool have_pend = false;
            R.j_acc = 0;
            while (true) {
                while (k < mt + 1) {
                    ++k;
                    const int D = k - 1;
                    a.v = V + (size_t)(k - 1) * stride;
                    a.out = V + (size_t)k * stride;
                    a.vtail = a.v + n;
                    a.otail = a.out + n;
                    const int k0 = iop ? std::max(0, k - o->iop) : 0;
                    a.basis = V + (size_t)k0 * stride;
                    a.nv = k - 1 - k0;
                    const bool is_check = D == mt;
                    CheckReq cr{};
                    if (is_check) cr = R.req(D, R.dt_sub);
                    Check cur;
                    CO_TRY(co_await x.iterate(m, a, k, naug_nz, is_check ? &cr : nullptr, &cur,
                                              iop));
                    if (st) {
                        st->krylov_iters += 1;
                        st->jvps += 1;
                    }
                    if (is_check) {
                        pend = cur;
                        have_pend = true;
                    }
                }
                if (!have_pend) {
                    // the basis already reaches mt (after a shorter substep): check it
                    CO_TRY(co_await x.check(m, R.req(mt, R.dt_sub), &pend));
                }
                have_pend = false;
                CO_TRY(co_await x.wait_check(m, pend));
                const CheckResult r = read_check(m, pend);
                if (r.nonfinite) co_return fail(EXPDG_ENONFINITE, "non-finite Krylov norm");
                if (r.brk > 0) {
                    // happy breakdown: exact, the whole remaining interval
                    R.dt_sub = rem0;
                    R.sub_last = true;
                    Check bc;
                    CO_TRY(co_await x.check(m, R.req(r.brk, R.dt_sub), &bc));
                    CO_TRY(co_await x.wait_check(m, bc));
                    const CheckResult br = read_check(m, bc);
                    if (br.singular) co_return fail(EXPDG_ENONFINITE, "singular Pade denominator");
                    if (st) st->breakdown += 1;
                    R.err = 0.0;
                    R.j_acc = r.brk;
                    R.acc = bc;
                    next = AdaptChoice{R.dt_sub, mt, true};
                    break;
                }
                if (r.singular) co_return fail(EXPDG_ENONFINITE, "singular Pade denominator");
                if (!std::isfinite(r.err)) co_return fail(EXPDG_ENONFINITE, "non-finite error estimate");
                // omega rounded up to a quarter decade, q and kappa to two
                // significant digits (the oracle does the same), so decisions
                // do not turn on the last bits of err
                const double om = quarter_decade(r.err * tau / (R.tol_abs * R.dt_sub));
                if (m_p == mt && dt_p != R.dt_sub && om_p > 0.0 && om > 0.0)
                    q = round2(std::max(1.0, std::log(om / om_p) / std::log(R.dt_sub / dt_p)));
                if (m_p >= 0 && m_p != mt && dt_p == R.dt_sub && om > 0.0 && om_p > 0.0)
                    kappa = round2(std::max(1.1, std::pow(om_p / om, 1.0 / (mt - m_p))));
                const bool ok = om <= 1.0;
                next = adapt_choice(mt, R.dt_sub, om, q, kappa, ok ? rem0 - R.dt_sub : rem0, !ok,
                                    o);
                if (ok) {
                    R.err = r.err;
                    R.j_acc = mt;
                    R.acc = pend;
                    break;
                }
                if (st) st->rejects += 1;
                om_p = om;
                dt_p = R.dt_sub;
                m_p = mt;
                if (next.take_a) {
                    R.dt_sub = next.dtau_a;  // same basis, shorter substep
                    R.sub_last = false;
                    if (!(R.dt_sub > 1e-12 * tau))
                        co_return fail(EXPDG_ENOCONV, "Krylov substep below its floor");
                } else {
                    mt = next.m_b;  // extend the Arnoldi process
                }
            }
            CO_TRY(x.after_check(m, R.acc));
            CO_TRY(prof_begin(m, EXPDG_K_COMBINE));
            CO_HIPTRY(launch_combine<T>(V, stride, R.j_acc,
                                        m->slots + R.acc.slot * kSlotSize + kSlotCoef, V, L, s));
            CO_TRY(prof_end(m, EXPDG_K_COMBINE, (double)(R.j_acc + 1) * L * eb));
            R.t_done += R.dt_sub;
            log_sub(st, R.j_acc, R.sub_last ? 1 : 0, R.dt_sub);
            if (st) st->err_est = R.err;
            const double rem = tau - R.t_done;
            if (R.sub_last || !(rem > 1e-15 * tau)) {
                if (!R.sub_last && st && st->log && st->log_len >= 1 && st->log_len <= st->log_cap)
                    st->log[st->log_len - 1].last = 1;
                if (st) st->m_next = next.take_a ? mt : next.m_b;
                break;
            }
            if (next.take_a)
                dtau = next.dtau_a;
            else {
                mt = next.m_b;
                dtau = R.dt_sub;
            }
        }
        CO_HIPTRY(launch_copy(V, out, n, s));
        if (!nested) CO_TRY(co_await x.finish(m));
        co_return EXPDG_OK;
    }

    double dtau = tau;
    bool reaches_end = true;
    while (true) {
        int m_target = o->m_max;
        R.dt_sub = dtau;
        R.sub_last = reaches_end;
        if (forced) {
            if (*fpos >= o->n_forced) co_return fail(EXPDG_EINVAL, "forced schedule exhausted");
            m_target = o->forced[*fpos].m;
            R.dt_sub = o->forced[*fpos].dtau;
            R.sub_last = o->forced[*fpos].last != 0;
        }
        // beta = ||z||, S[0] = 1/beta, flags cleared
        CO_TRY(prof_begin(m, EXPDG_K_GS_NORM));
        CO_HIPTRY(launch_gs_norm<T>(V, L, rp, kd.part, s));
        CO_TRY(prof_end(m, EXPDG_K_GS_NORM, (double)L * eb));
        CO_TRY(prof_begin(m, EXPDG_K_GS_FINISH));
        CO_HIPTRY(launch_gs_finish_norm(kd.part, rp, kd.H, kd.S, kd.flags, kd.res, s));
        CO_TRY(prof_end(m, EXPDG_K_GS_FINISH, 8.0 * rp.nrb));

        R.j_acc = 0;
        R.err = 0.0;
        Check pend[kCheckSlots];  // checks launched and not yet decided, oldest first
        int np = 0;
        // Arnoldi step k finishes dimension D = k - 1 (its basis vectors and
        // Hessenberg columns), so dimension m_target needs step m_target + 1.
        for (int k = 1; k <= m_target + 1; ++k) {
            const int D = k - 1;
            T *vin = V + (size_t)(k - 1) * stride;
            T *w = V + (size_t)k * stride;
            a.v = vin;
            a.out = w;
            a.vtail = vin + n;
            a.otail = w + n;
            // full orthogonalization: the dot pass runs over u_0..u_{k-2};
            // incomplete (window of L): over the last min(k-1, L-1) of them
            const int k0 = iop ? std::max(0, k - o->iop) : 0;
            a.basis = V + (size_t)k0 * stride;
            a.nv = k - 1 - k0;
            const bool is_check = !forced && D >= 1 &&
                                  (D == o->m_max ||
                                   (D >= o->m_min && (D - o->m_min) % o->check_every == 0));
            CheckReq cr{};
            if (is_check) cr = R.req(D, R.dt_sub);
            Check cur;
            CO_TRY(co_await x.iterate(m, a, k, naug_nz, is_check ? &cr : nullptr, &cur, iop));
            if (st) {
                st->krylov_iters += 1;
                st->jvps += 1;
            }
            if (forced) continue;
            // decide the checks at least kLookahead steps old (all of them at
            // the last step): the device works on the newer steps meanwhile.
            // The short steps of incomplete orthogonalization take one step
            // more, so that a check (longer than such a step) is done by then.
            if (is_check) pend[np++] = cur;
            bool done = false;
            while (np > 0 && (D == m_target || pend[0].j <= D - lookahead)) {
                const Check c = pend[0];
                for (int q = 1; q < np; ++q) pend[q - 1] = pend[q];
                --np;
                CO_AWAIT_TASK(R.decide(c, &done));
                if (done) break;
            }
            if (done) break;
        }
        if (forced) {
            Check fc;
            CO_TRY(co_await x.check(m, R.req(m_target, R.dt_sub), &fc));
            R.acc = fc;
            R.j_acc = m_target;
            R.err = 0.0;
        }
        if (R.j_acc == 0) co_return fail(EXPDG_ENOCONV, "Krylov controller made no decision");

        // accept: z <- beta V_j F_{1:j,1} (once the check's coefficients are written)
        CO_TRY(x.after_check(m, R.acc));
        CO_TRY(prof_begin(m, EXPDG_K_COMBINE));
        CO_HIPTRY(launch_combine<T>(V, stride, R.j_acc,
                                    m->slots + R.acc.slot * kSlotSize + kSlotCoef, V, L, s));
        CO_TRY(prof_end(m, EXPDG_K_COMBINE, (double)(R.j_acc + 1) * L * eb));
        R.t_done += R.dt_sub;
        log_sub(st, R.j_acc, R.sub_last ? 1 : 0, R.dt_sub);
        if (st) st->err_est = R.err;
        if (forced) *fpos += 1;
        if (R.sub_last) break;
        const double rem = tau - R.t_done;
        if (!(rem > 1e-15 * tau)) {
            // the accepted substeps already cover [0, tau]: the last one ends
            // the evaluation, and the log says so (a replay stops there too)
            if (st && st->log && st->log_len >= 1 && st->log_len <= st->log_cap)
                st->log[st->log_len - 1].last = 1;
            break;
        }
        if (forced) continue;

        const double ratio = (R.err > 0.0) ? R.tol_abs * R.dt_sub / tau / R.err : 0.0;
        double fac = (R.err > 0.0) ? 0.9 * std::pow(ratio, 1.0 / R.j_acc) : 5.0;
        fac = std::min(5.0, std::max(1.0, fac));
        const double cand = round2(R.dt_sub * fac);
        if (cand >= rem) {
            dtau = rem;
            reaches_end = true;
        } else {
            dtau = cand;
            reaches_end = false;
        }
    }
    CO_HIPTRY(launch_copy(V, out, n, s));
    if (forced) {
        // a forced run reads no check back: surface non-finite values here
        CO_HIPTRY(hipMemcpyAsync(m->pin + kPinNorms, kd.flags, 8, hipMemcpyDeviceToHost, s));
        CO_TRY(co_await x.readback(m));
        int fl[2];
        std::memcpy(fl, m->pin + kPinNorms, 8);
        if (fl[1]) co_return fail(EXPDG_ENONFINITE, "non-finite Krylov norm");
    }
    if (!nested) CO_TRY(co_await x.finish(m));
    co_return EXPDG_OK;
}

// One step of EPI2, EPI3 (Tokman's three-stage form; the first step, without
// history, is EPI2) or EXPRB32 (the schemes of Section 5.1), on the FP64 state
// q (and its history q_prev for EPI3).  In FP32_BULK the residuals, the frozen
// fields and the stage differences are formed from the FP64 states (rounding
// the state first would put its rounding noise into every residual, and the
// Krylov process would spend iterations resolving it); only the Krylov
// vectors, the b vectors and the linear operator's reference state (Burgers)
// are FP32.
template <typename T, typename X>
Task<int> step_co(X &x, expdg_mesh *m, int scheme, double dt, double *q, double *q_prev,
                  int have_prev, const expdg_krylov_opts *o, expdg_krylov_stats *st,
                  bool nested = false) {
    hipStream_t s = x.stream();
    const size_t n = m->n;
    constexpr bool bulk = !std::is_same<T, double>::value;
    T *Rn = (T *)m->vec[0], *Rp = (T *)m->vec[1], *d = (T *)m->vec[2], *Ld = (T *)m->vec[3],
      *w = (T *)m->vec[4], *w2 = (T *)m->vec[5];
    // operator view of the FP64 state q^n
    auto view = [&](double *src, T **dst) -> hipError_t {
        if constexpr (!bulk) {
            *dst = (T *)src;
            return hipSuccess;
        } else {
            *dst = (T *)m->bq;
            return launch_convert(src, (float *)*dst, n, s);
        }
    };
    T *qb = nullptr;
    // residual of an FP64 state (FP32 storage: read in FP64, stored in FP32)
    auto residual = [&](const double *state, T *out) -> int {
        if constexpr (bulk)
            return apply_op<T>(m, false, qb, nullptr, out, s, state);
        else
            return apply_op<T>(m, false, (const T *)state, nullptr, out, s);
    };
    int fpos = 0;
    // entropy viscosity of the step from q^n and q^{n-1} (q^n without history)
    if (m->nu)
        CO_TRY(entropy_viscosity<T>(m, q, (q_prev && have_prev) ? q_prev : q, dt, s));
    CO_HIPTRY(view(q, &qb));
    // every linear operator of the step is frozen at q^n
    CO_HIPTRY(prepare_lin<T>(m, (const double *)q, s));
    CO_TRY(residual(q, Rn));
    if (st) st->rhs_calls += 1;

    if (scheme == EXPDG_EPI2 || (scheme == EXPDG_EPI3 && !(q_prev && have_prev))) {
        const T *b[2] = {nullptr, Rn};
        CO_AWAIT_TASK((phi_co<T, X>(x, m, qb, dt, 1, b, w, o, st, &fpos, true, true)));
        CO_HIPTRY(launch_step_update<T>(q, q_prev, w, n, s));
    } else if (scheme == EXPDG_EPI3) {
        CO_TRY(residual(q_prev, Rp));
        CO_HIPTRY((launch_lincomb<T, double>(d, 1.0, q_prev, -1.0, q, 0.0, nullptr, n, s)));
        CO_TRY(apply_op<T>(m, true, qb, d, Ld, s));
        if (st) {
            st->rhs_calls += 1;
            st->jvps += 1;
        }
        const double c = 2.0 / (3.0 * dt);
        CO_HIPTRY((launch_lincomb<T, T>(d, c, Rp, -c, Rn, -c, Ld, n, s)));  // b_2 into d
        const T *b[3] = {nullptr, Rn, d};
        CO_AWAIT_TASK((phi_co<T, X>(x, m, qb, dt, 2, b, w, o, st, &fpos, true, true)));
        CO_HIPTRY(launch_step_update<T>(q, q_prev, w, n, s));
    } else if (scheme == EXPDG_EXPRB42) {
        // q2 = q^n + (3/4) dt phi_1((3/4) dt L) R^n; q^{n+1} = q^n + dt phi_1(dt L) R^n
        // + dt^3 phi_3(dt L) b_3 with b_3 = (32/9) D / dt^2, D = R(q2) - R^n - L (q2 - q^n)
        const T *b1[2] = {nullptr, Rn};
        CO_AWAIT_TASK((phi_co<T, X>(x, m, qb, 0.75 * dt, 1, b1, w, o, st, &fpos, true, true)));
        CO_HIPTRY(launch_add_mixed<T>(m->q2, q, w, n, s));  // q2 = q^n + w1
        CO_TRY(residual(m->q2, Rp));                       // R(q2)
        CO_HIPTRY((launch_lincomb<T, double>(d, 1.0, m->q2, -1.0, q, 0.0, nullptr, n, s)));
        CO_TRY(apply_op<T>(m, true, qb, d, Ld, s));
        if (st) {
            st->rhs_calls += 1;
            st->jvps += 1;
        }
        const double c = (32.0 / 9.0) / (dt * dt);
        CO_HIPTRY((launch_lincomb<T, T>(d, c, Rp, -c, Rn, -c, Ld, n, s)));  // b_3 into d
        const T *b[4] = {nullptr, Rn, nullptr, d};
        CO_AWAIT_TASK((phi_co<T, X>(x, m, qb, dt, 3, b, w2, o, st, &fpos, true, true)));
        if (q_prev) CO_HIPTRY(launch_copy(q, q_prev, n, s));
        CO_HIPTRY(launch_add_to<T>(q, w2, n, s));
    } else {  // EXPRB32
        const T *b1[2] = {nullptr, Rn};
        CO_AWAIT_TASK((phi_co<T, X>(x, m, qb, dt, 1, b1, w, o, st, &fpos, true, true)));
        CO_HIPTRY(launch_add_mixed<T>(m->q2, q, w, n, s));  // q2 = q^n + w1
        CO_TRY(residual(m->q2, Rp));                       // R(q2)
        CO_HIPTRY((launch_lincomb<T, double>(d, 1.0, m->q2, -1.0, q, 0.0, nullptr, n, s)));
        CO_TRY(apply_op<T>(m, true, qb, d, Ld, s));
        if (st) {
            st->rhs_calls += 1;
            st->jvps += 1;
        }
        const double c = 2.0 / (dt * dt);
        CO_HIPTRY((launch_lincomb<T, T>(d, c, Rp, -c, Rn, -c, Ld, n, s)));  // b_3 into d
        const T *b[4] = {nullptr, nullptr, nullptr, d};
        CO_AWAIT_TASK((phi_co<T, X>(x, m, qb, dt, 3, b, w2, o, st, &fpos, true, true)));
        if (q_prev) CO_HIPTRY(launch_copy(q, q_prev, n, s));
        CO_HIPTRY(launch_add_mixed<T>(q, m->q2, w2, n, s));
    }
    if (!nested) CO_TRY(co_await x.finish(m));
    co_return EXPDG_OK;
}

// nsteps steps of step_co; the end of the whole run is the only wait for the
// device.  Steps after the first have history when q_prev holds it.
template <typename T, typename X>
Task<int> integrate_co(X &x, expdg_mesh *m, int scheme, double dt, int nsteps, double *q,
                       double *q_prev, int have_prev, const expdg_krylov_opts *o,
                       expdg_krylov_stats *st) {
    for (int k = 0; k < nsteps; ++k) {
        const int hp = (k == 0) ? have_prev : (q_prev != nullptr ? 1 : 0);
        CO_AWAIT_TASK((step_co<T, X>(x, m, scheme, dt, q, q_prev, hp, o, st, true)));
    }
    CO_TRY(co_await x.finish(m));
    co_return EXPDG_OK;
}

}  // namespace expdg
