// C ABI of the MI355X exponential-DG library: validation, mesh and workspace,
// the adaptive Krylov controller, and the exponential steppers.  Every
// arithmetic step on state-sized data runs in the HIP kernels of
// dg_kernels.hip and krylov_kernels.hip; the host only makes the scalar
// controller decisions (Section 2.3: adaptive Krylov evaluation of the phi
// combination; the paper leaves the controller parameters unreported, so the
// controller below is a fixed written specification shared with the test
// oracle).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"

using namespace expdg;

// ---------------------------------------------------------------------------
// errors
namespace {

thread_local char g_err[512] = "no error";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIPTRY(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(EXPDG_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));        \
    } while (0)

#define TRY(call)                    \
    do {                             \
        int rc_ = (call);            \
        if (rc_ != EXPDG_OK) return rc_; \
    } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Two significant decimal digits, rounded up (step-size quantisation of the
// controller, so that oracle and device take the same decisions).
double round2(double x) {
    if (!(x > 0.0)) return x;
    const double s = std::pow(10.0, std::floor(std::log10(x)) - 1.0);
    return std::ceil(x / s) * s;
}

}  // namespace

namespace expdg {
LaunchEvents &next_launch_events() {
    thread_local LaunchEvents e;
    return e;
}
}  // namespace expdg

// ---------------------------------------------------------------------------
// LGL reference element (library construction).
//
// Nodes are the zeros of g(x) = P_{p-1}(x) - x P_p(x) = (1 - x^2) P_p'(x) / p
// (endpoints and the extrema of P_p), found by Newton's method; weights
// w_i = 2 / (p (p+1) P_p(x_i)^2); differentiation matrix in the closed
// Legendre form D_ij = P_p(x_i) / (P_p(x_j)(x_i - x_j)) (i != j),
// D_00 = -p(p+1)/4, D_pp = p(p+1)/4, other diagonal entries 0.
namespace expdg {

static void legendre_pd(int p, double x, double *P, double *dP, double *Pm1, double *dPm1) {
    // P_k and P_k' with P'_{k+1} = x P'_k + (k+1) P_k
    double a = 1.0, da = 0.0;  // P_0
    double b = x, db = 1.0;    // P_1
    if (p == 1) {
        *P = b, *dP = db, *Pm1 = a, *dPm1 = da;
        return;
    }
    for (int k = 1; k < p; ++k) {
        const double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
        const double dc = x * db + (k + 1.0) * b;
        a = b, da = db;
        b = c, db = dc;
    }
    *P = b, *dP = db, *Pm1 = a, *dPm1 = da;
}

int lgl_tables(int p, double *xi, double *w, double *D) {
    if (p < 1 || p > kMaxP) return EXPDG_EINVAL;
    const int n1 = p + 1;
    const double pi = std::acos(-1.0);
    for (int i = 0; i <= p; ++i) {
        if (i == 0) {
            xi[i] = -1.0;
            continue;
        }
        if (i == p) {
            xi[i] = 1.0;
            continue;
        }
        double x = -std::cos(pi * i / p);
        for (int it = 0; it < 200; ++it) {
            double P, dP, Pm, dPm;
            legendre_pd(p, x, &P, &dP, &Pm, &dPm);
            const double g = Pm - x * P;
            const double dg = dPm - P - x * dP;
            const double step = g / dg;
            x -= step;
            if (std::fabs(step) <= 1e-17 * (1.0 + std::fabs(x))) break;
        }
        xi[i] = x;
    }
    std::vector<double> Pv(n1);
    for (int i = 0; i <= p; ++i) {
        double P, dP, Pm, dPm;
        legendre_pd(p, xi[i], &P, &dP, &Pm, &dPm);
        Pv[i] = P;
        w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
    for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= p; ++j) {
            double d = 0.0;
            if (i != j)
                d = Pv[i] / (Pv[j] * (xi[i] - xi[j]));
            else if (i == 0)
                d = -p * (p + 1.0) / 4.0;
            else if (i == p)
                d = p * (p + 1.0) / 4.0;
            D[i * n1 + j] = d;
        }
    return EXPDG_OK;
}

}  // namespace expdg

// ---------------------------------------------------------------------------
// mesh

struct expdg_mesh {
    expdg_mesh_desc d;
    int nvar, n1, Np, K, dim;
    size_t n;       // ndof
    size_t stride;  // elements between Krylov vectors (>= n + kMaxAug)
    int ebytes;     // bytes per bulk element
    double hx, hy, dxmin;
    double xi[kMaxP + 1], w[kMaxP + 1], D[(kMaxP + 1) * (kMaxP + 1)];

    void *V = nullptr;           // (m_max+1) x stride bulk
    void *vec[6] = {};           // bulk work vectors (stride each)
    void *bq[3] = {};            // bulk copies of FP64 states (FP32_BULK only)
    double *q2 = nullptr;        // FP64 stage state (EXPRB32)
    KrylovDev kd{};
    double *slots = nullptr;     // 2 x kSlotSize
    double *dnorm = nullptr;     // 8
    double *spart = nullptr;     // 1024 (wave-speed partials)
    double *pin = nullptr;       // pinned host mirror
    hipEvent_t ev[2] = {nullptr, nullptr};   // check results ready (side stream)
    hipEvent_t evH[2] = {nullptr, nullptr};  // Hessenberg column ready (main stream)
    hipStream_t side = nullptr;              // small exponentials run here
    size_t bytes = 0;
    std::vector<void *> allocs;

    // live timing of one or more kernel classes
    struct Prof {
        bool on = false;
        std::vector<hipEvent_t> ev;  // start/stop pairs
        std::vector<double> bytes;   // algorithmic bytes per recorded launch
        int used = 0;
        long long launches = 0;
        double ms = 0.0, total_bytes = 0.0;
    } prof[EXPDG_K_NCLASSES];
};

namespace {

constexpr int kPinSlots = 0;    // 2 x 8 doubles: err, s, singular, flags...
constexpr int kPinNorms = 16;   // 8 doubles
constexpr int kPinSpeed = 32;   // 1024 doubles
constexpr int kPinSize = 32 + 1024;

bool desc_ok(const expdg_mesh_desc *d, std::string *why) {
    if (!d) return *why = "desc is NULL", false;
    if (d->equation != EXPDG_BURGERS1D && d->equation != EXPDG_EULER2D)
        return *why = "equation must be EXPDG_BURGERS1D or EXPDG_EULER2D", false;
    if (d->p < 1 || d->p > kMaxP) return *why = "p must be in 1..6", false;
    if (d->nx < 1 || d->ny < 1) return *why = "nx and ny must be >= 1", false;
    if (d->equation == EXPDG_BURGERS1D && d->ny != 1) return *why = "Burgers needs ny == 1", false;
    if ((long long)d->nx * d->ny > (1LL << 26)) return *why = "too many elements", false;
    if (d->precision != EXPDG_FP64 && d->precision != EXPDG_FP32_BULK)
        return *why = "precision must be EXPDG_FP64 or EXPDG_FP32_BULK", false;
    if (!(d->x1 > d->x0) || !std::isfinite(d->x0) || !std::isfinite(d->x1))
        return *why = "need x1 > x0", false;
    if (d->equation == EXPDG_EULER2D) {
        if (!(d->y1 > d->y0) || !std::isfinite(d->y0) || !std::isfinite(d->y1))
            return *why = "need y1 > y0", false;
        if (!(d->gamma > 1.0) || !std::isfinite(d->gamma)) return *why = "need gamma > 1", false;
    }
    if (d->m_max < 1 || d->m_max > kMaxM) return *why = "m_max must be in 1..64", false;
    if (d->device < 0) return *why = "device must be >= 0", false;
    return true;
}

struct Sizes {
    size_t n, stride, total;
    int ebytes;
};

Sizes sizes_of(const expdg_mesh_desc *d) {
    Sizes s{};
    const int n1 = d->p + 1;
    const int Np = (d->equation == EXPDG_BURGERS1D) ? n1 : n1 * n1;
    const int nvar = (d->equation == EXPDG_BURGERS1D) ? 1 : 4;
    s.n = (size_t)nvar * d->nx * d->ny * Np;
    s.stride = (s.n + kMaxAug + 63) / 64 * 64;
    s.ebytes = (d->precision == EXPDG_FP64) ? 8 : 4;
    size_t t = 0;
    t += (size_t)(d->m_max + 1) * s.stride * s.ebytes;                      // V
    t += 6 * s.stride * s.ebytes;                                          // work vectors
    if (d->precision == EXPDG_FP32_BULK) t += 3 * s.stride * s.ebytes;     // bulk state copies
    t += s.stride * 8;                                                     // q2
    t += (size_t)(kMaxM + 1) * kMaxM * 8 + 3 * (kMaxM + 1) * 8 + 64;       // H, S, coefs
    t += (size_t)kRedBlocks * (kMaxM + 1) * 8 + 64 * 8 + 16;               // part, res, flags
    t += 2 * kSlotSize * 8 + 8 * 8 + 1024 * 8;                             // slots, norms, speed
    s.total = t;
    return s;
}

template <typename P>
int dalloc(expdg_mesh *m, P **ptr, size_t bytes) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(EXPDG_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    m->allocs.push_back(p);
    m->bytes += bytes;
    *ptr = (P *)p;
    return EXPDG_OK;
}

void release(expdg_mesh *m) {
    for (void *p : m->allocs) (void)hipFree(p);
    m->allocs.clear();
    if (m->pin) (void)hipHostFree(m->pin);
    for (auto &e : m->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : m->evH)
        if (e) (void)hipEventDestroy(e);
    if (m->side) (void)hipStreamDestroy(m->side);
    for (auto &P : m->prof)
        for (auto &e : P.ev) (void)hipEventDestroy(e);
}

constexpr int kProfPairs = 1024;

// Fold the recorded launches of class c into its counters.
int prof_flush(expdg_mesh *m, int c) {
    auto &P = m->prof[c];
    for (int k = 0; k < P.used; ++k) {
        HIPTRY(hipEventSynchronize(P.ev[2 * k + 1]));
        float ms = 0.0f;
        HIPTRY(hipEventElapsedTime(&ms, P.ev[2 * k], P.ev[2 * k + 1]));
        P.ms += ms;
        P.launches += 1;
        P.total_bytes += P.bytes[k];
    }
    P.used = 0;
    return EXPDG_OK;
}

// The next kernel launch records the event pair as part of its own dispatch
// (hipExtLaunchKernelGGL), so the interval is the kernel's execution.
int prof_begin(expdg_mesh *m, int c, hipStream_t s) {
    (void)s;
    auto &P = m->prof[c];
    if (!P.on) return EXPDG_OK;
    if (P.used == kProfPairs) TRY(prof_flush(m, c));
    next_launch_events() = LaunchEvents{P.ev[2 * P.used], P.ev[2 * P.used + 1]};
    return EXPDG_OK;
}

int prof_end(expdg_mesh *m, int c, hipStream_t s, double bytes) {
    (void)s;
    auto &P = m->prof[c];
    if (!P.on) return EXPDG_OK;
    next_launch_events() = LaunchEvents{};
    P.bytes[P.used] = bytes;
    P.used += 1;
    return EXPDG_OK;
}

template <typename T>
OpArgs<T> op_args(const expdg_mesh *m) {
    OpArgs<T> a{};
    a.K = m->K;
    a.nx = m->d.nx;
    a.ny = m->d.ny;
    a.rhx = (T)(2.0 / m->hx);
    a.rhy = (T)(2.0 / m->hy);
    a.lift = (T)(1.0 / m->w[0]);
    a.gamma = (T)m->d.gamma;
    for (int k = 0; k < m->n1 * m->n1; ++k) a.D[k] = (T)m->D[k];
    a.eta = 1.0;
    return a;
}

}  // namespace

extern "C" size_t expdg_workspace_bytes(const expdg_mesh_desc *d) {
    std::string why;
    if (!desc_ok(d, &why)) return 0;
    return sizes_of(d).total;
}

extern "C" int expdg_mesh_create(const expdg_mesh_desc *d, expdg_mesh **out) {
    std::string why;
    if (!out) return fail(EXPDG_EINVAL, "out is NULL");
    if (!desc_ok(d, &why)) return fail(EXPDG_EINVAL, "invalid mesh description: %s", why.c_str());
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(EXPDG_EDEVICE, "no HIP device available");
    if (d->device >= ndev) return fail(EXPDG_EINVAL, "device %d out of range", d->device);
    DeviceGuard g(d->device);
    if (!g.ok) return fail(EXPDG_EDEVICE, "hipSetDevice(%d) failed", d->device);

    expdg_mesh *m = new (std::nothrow) expdg_mesh();
    if (!m) return fail(EXPDG_ENOMEM, "host allocation failed");
    m->d = *d;
    m->dim = (d->equation == EXPDG_BURGERS1D) ? 1 : 2;
    m->n1 = d->p + 1;
    m->Np = (m->dim == 1) ? m->n1 : m->n1 * m->n1;
    m->K = d->nx * d->ny;
    m->nvar = (m->dim == 1) ? 1 : 4;
    const Sizes sz = sizes_of(d);
    m->n = sz.n;
    m->stride = sz.stride;
    m->ebytes = sz.ebytes;
    m->hx = (d->x1 - d->x0) / d->nx;
    m->hy = (m->dim == 2) ? (d->y1 - d->y0) / d->ny : 1.0;
    lgl_tables(d->p, m->xi, m->w, m->D);
    double dmin = 2.0;
    for (int i = 0; i < d->p; ++i) dmin = std::min(dmin, m->xi[i + 1] - m->xi[i]);
    m->dxmin = 0.5 * ((m->dim == 2) ? std::min(m->hx, m->hy) : m->hx) * dmin;

    int rc = EXPDG_OK;
    const size_t vb = m->stride * m->ebytes;
    auto chk = [&](int r) {
        if (rc == EXPDG_OK && r != EXPDG_OK) rc = r;
    };
    chk(dalloc(m, &m->V, (size_t)(d->m_max + 1) * vb));
    for (auto &v : m->vec) chk(dalloc(m, &v, vb));
    if (d->precision == EXPDG_FP32_BULK)
        for (auto &v : m->bq) chk(dalloc(m, &v, vb));
    chk(dalloc(m, &m->q2, m->stride * 8));
    chk(dalloc(m, &m->kd.H, (size_t)(kMaxM + 1) * kMaxM * 8));
    chk(dalloc(m, &m->kd.S, (size_t)(kMaxM + 1) * 8));
    chk(dalloc(m, &m->kd.coefA, (size_t)(kMaxM + 1) * 8));
    chk(dalloc(m, &m->kd.coefB, (size_t)(kMaxM + 1) * 8));
    chk(dalloc(m, &m->kd.part, (size_t)kRedBlocks * (kMaxM + 1) * 8));
    chk(dalloc(m, &m->kd.res, 64 * 8));
    chk(dalloc(m, &m->kd.flags, 16));
    chk(dalloc(m, &m->slots, 2 * kSlotSize * 8));
    chk(dalloc(m, &m->dnorm, 8 * 8));
    chk(dalloc(m, &m->spart, 1024 * 8));
    if (rc == EXPDG_OK && hipHostMalloc((void **)&m->pin, kPinSize * 8) != hipSuccess) {
        m->pin = nullptr;
        rc = fail(EXPDG_ENOMEM, "pinned host allocation failed");
    }
    for (auto &e : m->ev)
        if (rc == EXPDG_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            rc = fail(EXPDG_EDEVICE, "hipEventCreate failed");
    for (auto &e : m->evH)
        if (rc == EXPDG_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            rc = fail(EXPDG_EDEVICE, "hipEventCreate failed");
    // default-priority side stream for the small exponentials
    if (rc == EXPDG_OK && hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking) != hipSuccess)
        rc = fail(EXPDG_EDEVICE, "hipStreamCreate failed");
    if (rc == EXPDG_OK) {
        // zero the whole Krylov block once (padding stays zero)
        if (hipMemset(m->V, 0, (size_t)(d->m_max + 1) * vb) != hipSuccess ||
            hipMemset(m->kd.flags, 0, 16) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            rc = fail(EXPDG_EDEVICE, "workspace initialisation failed");
    }
    if (rc != EXPDG_OK) {
        release(m);
        delete m;
        return rc;
    }
    *out = m;
    return EXPDG_OK;
}

extern "C" int expdg_mesh_destroy(expdg_mesh *m) {
    if (!m) return fail(EXPDG_EINVAL, "mesh is NULL");
    DeviceGuard g(m->d.device);
    (void)hipDeviceSynchronize();
    release(m);
    delete m;
    return EXPDG_OK;
}

extern "C" int expdg_mesh_get_info(const expdg_mesh *m, expdg_mesh_info *info) {
    if (!m || !info) return fail(EXPDG_EINVAL, "NULL argument");
    info->ndof = m->n;
    info->nvar = m->nvar;
    info->K = m->K;
    info->Np = m->Np;
    info->elem_bytes = m->ebytes;
    info->hx = m->hx;
    info->hy = m->hy;
    info->dx_min = m->dxmin;
    return EXPDG_OK;
}

extern "C" int expdg_mesh_nodes(const expdg_mesh *m, double *x, double *y) {
    if (!m || !x) return fail(EXPDG_EINVAL, "NULL argument");
    for (int e = 0; e < m->K; ++e) {
        const int ex = e % m->d.nx, ey = e / m->d.nx;
        for (int nn = 0; nn < m->Np; ++nn) {
            const int i = nn % m->n1, j = nn / m->n1;
            x[(size_t)e * m->Np + nn] = m->d.x0 + ex * m->hx + 0.5 * (m->xi[i] + 1.0) * m->hx;
            if (y)
                y[(size_t)e * m->Np + nn] =
                    (m->dim == 2) ? m->d.y0 + ey * m->hy + 0.5 * (m->xi[j] + 1.0) * m->hy : 0.0;
        }
    }
    return EXPDG_OK;
}

extern "C" int expdg_lgl(int p, double *xi, double *w, double *D) {
    if (!xi || !w || !D) return fail(EXPDG_EINVAL, "NULL argument");
    if (p < 1 || p > kMaxP) return fail(EXPDG_EINVAL, "p must be in 1..6");
    return lgl_tables(p, xi, w, D);
}

// ---------------------------------------------------------------------------
// operators

namespace {

template <typename T>
int apply_op(expdg_mesh *m, bool jvp, const T *q, const T *v, T *out, hipStream_t s) {
    OpArgs<T> a = op_args<T>(m);
    a.q = q;
    a.v = v;
    a.out = out;
    const int cls = jvp ? EXPDG_K_LINEAR : EXPDG_K_RESIDUAL;
    TRY(prof_begin(m, cls, s));
    HIPTRY(launch_dg_op(m->d.equation, m->d.p, jvp, a, s));
    TRY(prof_end(m, cls, s, (double)(jvp ? 3 : 2) * m->n * m->ebytes));
    return EXPDG_OK;
}

}  // namespace

extern "C" int expdg_rhs(expdg_mesh *m, const void *q, void *r, void *stream) {
    if (!m || !q || !r) return fail(EXPDG_EINVAL, "NULL argument");
    if (q == r) return fail(EXPDG_EINVAL, "q and r must not alias");
    DeviceGuard g(m->d.device);
    hipStream_t s = (hipStream_t)stream;
    if (m->d.precision == EXPDG_FP64)
        return apply_op<double>(m, false, (const double *)q, nullptr, (double *)r, s);
    return apply_op<float>(m, false, (const float *)q, nullptr, (float *)r, s);
}

extern "C" int expdg_jvp(expdg_mesh *m, const void *qref, const void *v, void *w, void *stream) {
    if (!m || !qref || !v || !w) return fail(EXPDG_EINVAL, "NULL argument");
    if (v == w || qref == w) return fail(EXPDG_EINVAL, "output must not alias an input");
    DeviceGuard g(m->d.device);
    hipStream_t s = (hipStream_t)stream;
    if (m->d.precision == EXPDG_FP64)
        return apply_op<double>(m, true, (const double *)qref, (const double *)v, (double *)w, s);
    return apply_op<float>(m, true, (const float *)qref, (const float *)v, (float *)w, s);
}

extern "C" int expdg_max_speed(expdg_mesh *m, const double *q, double *cmax, void *stream) {
    if (!m || !q || !cmax) return fail(EXPDG_EINVAL, "NULL argument");
    DeviceGuard g(m->d.device);
    hipStream_t s = (hipStream_t)stream;
    const size_t npts = (size_t)m->K * m->Np;
    const int nblk = max_speed_blocks(npts);
    HIPTRY(launch_max_speed(m->d.equation, q, npts, m->d.gamma, m->spart, nblk, s));
    HIPTRY(hipMemcpyAsync(m->pin + kPinSpeed, m->spart, nblk * 8, hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    double c = 0.0;
    for (int b = 0; b < nblk; ++b) c = std::max(c, m->pin[kPinSpeed + b]);
    if (!std::isfinite(c)) return fail(EXPDG_ENONFINITE, "non-finite wave speed");
    *cmax = c;
    return EXPDG_OK;
}

// ---------------------------------------------------------------------------
// phi combinations

namespace {

int check_opts(const expdg_mesh *m, const expdg_krylov_opts *o) {
    if (!o) return fail(EXPDG_EINVAL, "options are NULL");
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(EXPDG_EINVAL, "tol must be > 0");
    if (o->n_forced < 0 || (o->n_forced > 0 && !o->forced))
        return fail(EXPDG_EINVAL, "invalid forced schedule");
    if (o->n_forced > 0) {
        for (int k = 0; k < o->n_forced; ++k)
            if (o->forced[k].m < 1 || o->forced[k].m > m->d.m_max || !(o->forced[k].dtau > 0.0))
                return fail(EXPDG_EINVAL, "forced substep %d out of range", k);
        return EXPDG_OK;
    }
    if (o->m_min < 1 || o->m_max < o->m_min || o->m_max > m->d.m_max)
        return fail(EXPDG_EINVAL, "need 1 <= m_min <= m_max <= mesh m_max (%d)", m->d.m_max);
    if (o->check_every < 1) return fail(EXPDG_EINVAL, "check_every must be >= 1");
    return EXPDG_OK;
}

void log_sub(expdg_krylov_stats *st, int mm, int last, double dtau) {
    if (!st) return;
    st->substeps += 1;
    if (st->log && st->log_len < st->log_cap) {
        st->log[st->log_len].m = mm;
        st->log[st->log_len].last = last;
        st->log[st->log_len].dtau = dtau;
    }
    st->log_len += 1;
}

// A check (small exponential + error) enqueued but not yet read.
struct Check {
    int j = 0;       // Krylov dimension
    int slot = 0;    // device / pinned slot
};

template <typename T>
int phi_impl(expdg_mesh *m, const T *qref, double tau, int p, const T *const *b, T *out,
             const expdg_krylov_opts *o, expdg_krylov_stats *st, int *fpos, hipStream_t s) {
    const size_t n = m->n, L = n + (size_t)p;
    const size_t stride = m->stride;
    T *V = (T *)m->V;
    KrylovDev &kd = m->kd;
    const bool forced = o->n_forced > 0;
    const RowPartition rp = row_partition(L);
    if (st) st->phi_calls += 1;

    // 1. scaling and 2. tolerance: norms of b_0..b_p
    const T *bx[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k <= p; ++k) bx[k] = b ? b[k] : nullptr;
    HIPTRY(launch_norms<T>(bx, p + 1, n, kd.part, m->dnorm, s));
    HIPTRY(hipMemcpyAsync(m->pin + kPinNorms, m->dnorm, (p + 1) * 8, hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
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
    if (!std::isfinite(nu)) return fail(EXPDG_ENONFINITE, "non-finite input norm");
    if (nu == 0.0 || tau == 0.0) {
        if (bx[0])
            HIPTRY(launch_copy(bx[0], out, n, s));
        else
            HIPTRY(launch_fill<T>(out, 0.0, n, s));
        HIPTRY(hipStreamSynchronize(s));
        return EXPDG_OK;
    }
    const double tol_abs = o->tol * nu;

    // z = [b_0; 0, ..., 0, 1/eta] lives in V_0
    if (bx[0])
        HIPTRY(launch_copy(bx[0], V, n, s));
    else
        HIPTRY(launch_fill<T>(V, 0.0, n, s));
    if (p > 0) HIPTRY(launch_set_tail<T>(V + n, p, 1.0 / eta, s));
    HIPTRY(launch_fill<int>(kd.flags, 0.0, 4, s));

    OpArgs<T> a = op_args<T>(m);
    a.q = qref;
    a.eta = eta;
    a.naug = p;
    int naug_nz = 0;
    for (int k = 1; k <= p; ++k) {
        a.aug[k - 1] = bx[p + 1 - k];
        naug_nz += bx[p + 1 - k] ? 1 : 0;
    }
    const double eb = (double)sizeof(T);

    int nchecks = 0;
    // enqueue the small exponential for dimension j and substep dtau
    // The small exponential of check j runs on the side stream once the
    // Hessenberg column j-1 is complete on the main stream, overlapping the
    // next Arnoldi iteration; its result is read back one iteration later.
    hipStream_t side = m->side;
    auto enqueue_check = [&](int j, double dtau, Check *c) -> int {
        c->j = j;
        c->slot = (nchecks++) & 1;
        double *slot = m->slots + c->slot * kSlotSize;
        HIPTRY(hipEventRecord(m->evH[c->slot], s));
        HIPTRY(hipStreamWaitEvent(side, m->evH[c->slot], 0));
        TRY(prof_begin(m, EXPDG_K_SMALLEXPM, side));
        HIPTRY(launch_hess_expm(kd.H, j, dtau, kd.S, kd.res, slot, side));
        TRY(prof_end(m, EXPDG_K_SMALLEXPM, side, 0.0));
        HIPTRY(hipMemcpyAsync(m->pin + kPinSlots + c->slot * 8, slot, 4 * 8,
                              hipMemcpyDeviceToHost, side));
        HIPTRY(hipMemcpyAsync((char *)(m->pin + kPinSlots + c->slot * 8 + 4), kd.flags, 2 * 4,
                              hipMemcpyDeviceToHost, side));
        HIPTRY(hipEventRecord(m->ev[c->slot], side));
        return EXPDG_OK;
    };
    struct CheckResult {
        double err;
        int singular, brk, nonfinite;
    };
    auto read_check = [&](const Check &c, CheckResult *r) -> int {
        HIPTRY(hipEventSynchronize(m->ev[c.slot]));
        const double *pv = m->pin + kPinSlots + c.slot * 8;
        r->err = pv[kSlotErr];
        r->singular = pv[2] != 0.0;
        int fl[2];
        std::memcpy(fl, pv + 4, 8);
        r->brk = fl[0];
        r->nonfinite = fl[1];
        return EXPDG_OK;
    };

    double t_done = 0.0, dtau = tau;
    bool reaches_end = true;
    while (true) {
        int m_target = o->m_max;
        double dt_sub = dtau;
        bool sub_last = reaches_end;
        if (forced) {
            if (*fpos >= o->n_forced) return fail(EXPDG_EINVAL, "forced schedule exhausted");
            m_target = o->forced[*fpos].m;
            dt_sub = o->forced[*fpos].dtau;
            sub_last = o->forced[*fpos].last != 0;
        }
        // beta = ||z||, S[0] = 1/beta
        TRY(prof_begin(m, EXPDG_K_GS_UPDATE_NORM, s));
        HIPTRY(launch_gs_update_norm<T>(V, stride, 0, nullptr, V, L, rp, kd.part, kd.H, kd.S, -1,
                                        kd.flags, kd.res, s));
        TRY(prof_end(m, EXPDG_K_GS_UPDATE_NORM, s, (double)L * eb));
        TRY(prof_begin(m, EXPDG_K_GS_FINISH, s));
        HIPTRY(launch_gs_finish_norm(kd.part, rp, kd.H, kd.S, -1, kd.flags, kd.res, s));
        TRY(prof_end(m, EXPDG_K_GS_FINISH, s, 8.0 * rp.nrb));
        HIPTRY(launch_fill<double>(kd.H, 0.0, (size_t)(kMaxM + 1) * kMaxM, s));

        int j_acc = 0;
        double err = 0.0;
        Check pending, acc_check;
        bool have_pending = false;
        for (int j = 1; j <= m_target; ++j) {
            const int col = j - 1;
            T *vin = V + (size_t)(j - 1) * stride;
            T *w = V + (size_t)j * stride;
            // w = S[j-1] * Aug(u_{j-1})
            a.v = vin;
            a.out = w;
            a.vtail = vin + n;
            a.otail = w + n;
            a.vscale = kd.S + (j - 1);
            TRY(prof_begin(m, EXPDG_K_LINEAR, s));
            HIPTRY(launch_dg_op(m->d.equation, m->d.p, true, a, s));
            TRY(prof_end(m, EXPDG_K_LINEAR, s, (double)(3 + naug_nz) * n * eb));
            // classical Gram-Schmidt, two passes, then the norm
            const double fin_bytes = 8.0 * rp.nrb * j;
            TRY(prof_begin(m, EXPDG_K_GS_DOTS, s));
            HIPTRY(launch_gs_dots<T>(V, stride, j, w, L, rp, kd.part, kd.S, kd.H, col, 0, kd.coefA,
                                     s));
            TRY(prof_end(m, EXPDG_K_GS_DOTS, s, (double)(j + 1) * L * eb));
            TRY(prof_begin(m, EXPDG_K_GS_FINISH, s));
            HIPTRY(launch_gs_finish_dots(kd.part, j, rp, kd.S, kd.H, col, 0, kd.coefA, s));
            TRY(prof_end(m, EXPDG_K_GS_FINISH, s, fin_bytes));
            // (j > 32: a plain update then a dot pass, 2j + 3 vectors of traffic)
            TRY(prof_begin(m, EXPDG_K_GS_UPDATE_DOTS, s));
            HIPTRY(launch_gs_update_dots<T>(V, stride, j, kd.coefA, w, L, rp, kd.part, kd.S, kd.H,
                                            col, kd.coefB, s));
            TRY(prof_end(m, EXPDG_K_GS_UPDATE_DOTS, s,
                         (double)(j <= 32 ? j + 2 : 2 * j + 3) * L * eb));
            TRY(prof_begin(m, EXPDG_K_GS_FINISH, s));
            HIPTRY(launch_gs_finish_dots(kd.part, j, rp, kd.S, kd.H, col, 1, kd.coefB, s));
            TRY(prof_end(m, EXPDG_K_GS_FINISH, s, fin_bytes));
            TRY(prof_begin(m, EXPDG_K_GS_UPDATE_NORM, s));
            HIPTRY(launch_gs_update_norm<T>(V, stride, j, kd.coefB, w, L, rp, kd.part, kd.H, kd.S,
                                            col, kd.flags, kd.res, s));
            TRY(prof_end(m, EXPDG_K_GS_UPDATE_NORM, s, (double)(j + 2) * L * eb));
            TRY(prof_begin(m, EXPDG_K_GS_FINISH, s));
            HIPTRY(launch_gs_finish_norm(kd.part, rp, kd.H, kd.S, col, kd.flags, kd.res, s));
            TRY(prof_end(m, EXPDG_K_GS_FINISH, s, 8.0 * rp.nrb));
            if (st) {
                st->krylov_iters += 1;
                st->jvps += 1;
            }
            if (forced) continue;

            const bool is_check =
                j == o->m_max || (j >= o->m_min && (j - o->m_min) % o->check_every == 0);
            Check cur;
            if (is_check) TRY(enqueue_check(j, dt_sub, &cur));
            // look one check behind: the device works on iteration j meanwhile
            auto decide = [&](const Check &c, bool *done) -> int {
                CheckResult r;
                TRY(read_check(c, &r));
                *done = false;
                if (r.nonfinite) return fail(EXPDG_ENONFINITE, "non-finite Krylov norm");
                if (r.brk > 0) {
                    // happy breakdown: exact, take the whole remaining interval
                    dt_sub = tau - t_done;
                    sub_last = true;
                    Check bc;
                    TRY(enqueue_check(r.brk, dt_sub, &bc));
                    CheckResult br;
                    TRY(read_check(bc, &br));
                    if (br.singular) return fail(EXPDG_ENONFINITE, "singular Pade denominator");
                    if (st) st->breakdown += 1;
                    err = 0.0;
                    j_acc = r.brk;
                    acc_check = bc;
                    *done = true;
                    return EXPDG_OK;
                }
                if (r.singular) return fail(EXPDG_ENONFINITE, "singular Pade denominator");
                if (!std::isfinite(r.err)) return fail(EXPDG_ENONFINITE, "non-finite error estimate");
                if (r.err <= tol_abs * dt_sub / tau) {
                    err = r.err;
                    j_acc = c.j;
                    acc_check = c;
                    *done = true;
                    return EXPDG_OK;
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
                            return fail(EXPDG_ENOCONV, "Krylov substep below its floor");
                        TRY(enqueue_check(c.j, dt_sub, &sc));
                        CheckResult sr;
                        TRY(read_check(sc, &sr));
                        if (sr.singular || !std::isfinite(sr.err))
                            return fail(EXPDG_ENONFINITE, "non-finite error estimate");
                        e = sr.err;
                    }
                    err = e;
                    j_acc = c.j;
                    acc_check = sc;
                    *done = true;
                }
                return EXPDG_OK;
            };
            bool done = false;
            if (have_pending) {
                TRY(decide(pending, &done));
                have_pending = false;
                if (done) break;
            }
            if (is_check) {
                pending = cur;
                have_pending = true;
            }
            if (j == m_target && have_pending) {
                TRY(decide(pending, &done));
                have_pending = false;
                if (done) break;
            }
        }
        if (forced) {
            Check fc;
            TRY(enqueue_check(m_target, dt_sub, &fc));
            acc_check = fc;
            j_acc = m_target;
            err = 0.0;
        }
        if (j_acc == 0) return fail(EXPDG_ENOCONV, "Krylov controller made no decision");

        // accept: z <- beta V_j F_{1:j,1} (after the check's side-stream work)
        HIPTRY(hipStreamWaitEvent(s, m->ev[acc_check.slot], 0));
        TRY(prof_begin(m, EXPDG_K_COMBINE, s));
        HIPTRY(launch_combine<T>(V, stride, j_acc, m->slots + acc_check.slot * kSlotSize + kSlotCoef,
                                 V, L, s));
        TRY(prof_end(m, EXPDG_K_COMBINE, s, (double)(j_acc + 1) * L * eb));
        t_done += dt_sub;
        log_sub(st, j_acc, sub_last ? 1 : 0, dt_sub);
        if (st) st->err_est = err;
        if (forced) *fpos += 1;
        if (sub_last) break;
        if (forced) continue;

        const double ratio = (err > 0.0) ? tol_abs * dt_sub / tau / err : 0.0;
        double fac = (err > 0.0) ? 0.9 * std::pow(ratio, 1.0 / j_acc) : 5.0;
        fac = std::min(5.0, std::max(1.0, fac));
        const double cand = round2(dt_sub * fac);
        const double rem = tau - t_done;
        if (!(rem > 1e-15 * tau)) break;
        if (cand >= rem) {
            dtau = rem;
            reaches_end = true;
        } else {
            dtau = cand;
            reaches_end = false;
        }
    }
    HIPTRY(launch_copy(V, out, n, s));
    HIPTRY(hipStreamSynchronize(side));  // no speculative check left running
    if (forced) {
        // a forced run reads nothing back: surface non-finite values here
        HIPTRY(hipMemcpyAsync(m->pin + kPinSlots, kd.flags, 8, hipMemcpyDeviceToHost, s));
    }
    HIPTRY(hipStreamSynchronize(s));
    if (forced) {
        int fl[2];
        std::memcpy(fl, m->pin + kPinSlots, 8);
        if (fl[1]) return fail(EXPDG_ENONFINITE, "non-finite Krylov norm");
    }
    return EXPDG_OK;
}

}  // namespace

extern "C" int expdg_phi_krylov(expdg_mesh *m, const void *qref, double tau, int p,
                                const void *const *b, void *w, const expdg_krylov_opts *o,
                                expdg_krylov_stats *s, void *stream) {
    if (!m || !qref || !w) return fail(EXPDG_EINVAL, "NULL argument");
    if (p < 0 || p > kMaxAug) return fail(EXPDG_EINVAL, "p must be in 0..3");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(EXPDG_EINVAL, "tau must be >= 0");
    TRY(check_opts(m, o));
    if (b)
        for (int k = 0; k <= p; ++k)
            if (b[k] == w) return fail(EXPDG_EINVAL, "w must not alias b[%d]", k);
    DeviceGuard g(m->d.device);
    int fpos = 0;
    hipStream_t st = (hipStream_t)stream;
    if (m->d.precision == EXPDG_FP64)
        return phi_impl<double>(m, (const double *)qref, tau, p, (const double *const *)b,
                                (double *)w, o, s, &fpos, st);
    return phi_impl<float>(m, (const float *)qref, tau, p, (const float *const *)b, (float *)w, o,
                           s, &fpos, st);
}

// ---------------------------------------------------------------------------
// steppers (EPI2, EXPRB32: footnotes of Section 5.1; EPI3 after Tokman)

namespace {

template <typename T>
int step_impl(expdg_mesh *m, int scheme, double dt, double *q, double *q_prev, int have_prev,
              const expdg_krylov_opts *o, expdg_krylov_stats *st, hipStream_t s) {
    const size_t n = m->n;
    const bool bulk = !std::is_same<T, double>::value;
    T *Rn = (T *)m->vec[0], *Rp = (T *)m->vec[1], *d = (T *)m->vec[2], *Ld = (T *)m->vec[3],
      *w = (T *)m->vec[4], *w2 = (T *)m->vec[5];
    // operator views of the FP64 states
    auto view = [&](double *x, int k) -> T * {
        if (!bulk) return (T *)x;
        T *y = (T *)m->bq[k];
        (void)launch_convert(x, (float *)y, n, s);  // errors surface via hipGetLastError
        return y;
    };
    int fpos = 0;
    T *qb = view(q, 0);
    HIPTRY(hipGetLastError());
    TRY(apply_op<T>(m, false, qb, nullptr, Rn, s));
    if (st) st->rhs_calls += 1;

    if (scheme == EXPDG_EPI2 || (scheme == EXPDG_EPI3 && !(q_prev && have_prev))) {
        const T *b[2] = {nullptr, Rn};
        TRY(phi_impl<T>(m, qb, dt, 1, b, w, o, st, &fpos, s));
        if (q_prev) HIPTRY(launch_copy(q, q_prev, n, s));
        HIPTRY(launch_add_to<T>(q, w, n, s));
    } else if (scheme == EXPDG_EPI3) {
        T *qpb = view(q_prev, 1);
        HIPTRY(hipGetLastError());
        TRY(apply_op<T>(m, false, qpb, nullptr, Rp, s));
        HIPTRY((launch_lincomb<T, T>(d, 1.0, qpb, -1.0, qb, 0.0, nullptr, n, s)));
        TRY(apply_op<T>(m, true, qb, d, Ld, s));
        if (st) {
            st->rhs_calls += 1;
            st->jvps += 1;
        }
        const double c = 2.0 / (3.0 * dt);
        HIPTRY((launch_lincomb<T, T>(d, c, Rp, -c, Rn, -c, Ld, n, s)));  // b_2 into d
        const T *b[3] = {nullptr, Rn, d};
        TRY(phi_impl<T>(m, qb, dt, 2, b, w, o, st, &fpos, s));
        HIPTRY(launch_copy(q, q_prev, n, s));
        HIPTRY(launch_add_to<T>(q, w, n, s));
    } else {  // EXPRB32
        const T *b1[2] = {nullptr, Rn};
        TRY(phi_impl<T>(m, qb, dt, 1, b1, w, o, st, &fpos, s));
        HIPTRY(launch_add_mixed<T>(m->q2, q, w, n, s));  // q2 = q^n + w1
        T *q2b = view(m->q2, 2);
        HIPTRY(hipGetLastError());
        TRY(apply_op<T>(m, false, q2b, nullptr, Rp, s));  // R(q2)
        HIPTRY((launch_lincomb<T, T>(d, 1.0, q2b, -1.0, qb, 0.0, nullptr, n, s)));
        TRY(apply_op<T>(m, true, qb, d, Ld, s));
        if (st) {
            st->rhs_calls += 1;
            st->jvps += 1;
        }
        const double c = 2.0 / (dt * dt);
        HIPTRY((launch_lincomb<T, T>(d, c, Rp, -c, Rn, -c, Ld, n, s)));  // b_3 into d
        const T *b[4] = {nullptr, nullptr, nullptr, d};
        TRY(phi_impl<T>(m, qb, dt, 3, b, w2, o, st, &fpos, s));
        if (q_prev) HIPTRY(launch_copy(q, q_prev, n, s));
        HIPTRY(launch_add_mixed<T>(q, m->q2, w2, n, s));
    }
    HIPTRY(hipStreamSynchronize(s));
    return EXPDG_OK;
}

}  // namespace

extern "C" int expdg_step(expdg_mesh *m, int scheme, double dt, double *q, double *q_prev,
                          int have_prev, const expdg_krylov_opts *o, expdg_krylov_stats *s,
                          void *stream) {
    if (!m || !q) return fail(EXPDG_EINVAL, "NULL argument");
    if (scheme != EXPDG_EPI2 && scheme != EXPDG_EPI3 && scheme != EXPDG_EXPRB32)
        return fail(EXPDG_EINVAL, "unknown scheme %d", scheme);
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(EXPDG_EINVAL, "dt must be > 0");
    if (scheme == EXPDG_EPI3 && have_prev && !q_prev)
        return fail(EXPDG_EINVAL, "EPI3 with have_prev needs q_prev");
    if (q_prev == q) return fail(EXPDG_EINVAL, "q_prev must not alias q");
    TRY(check_opts(m, o));
    DeviceGuard g(m->d.device);
    hipStream_t st = (hipStream_t)stream;
    if (m->d.precision == EXPDG_FP64)
        return step_impl<double>(m, scheme, dt, q, q_prev, have_prev, o, s, st);
    return step_impl<float>(m, scheme, dt, q, q_prev, have_prev, o, s, st);
}

// ---------------------------------------------------------------------------

extern "C" int expdg_small_expm(int n, const double *A, double *E, void *stream) {
    if (!A || !E || n < 1 || n > kMaxM + 1) return fail(EXPDG_EINVAL, "need 1 <= n <= 65");
    HIPTRY(launch_dense_expm(A, n, E, (hipStream_t)stream));
    return EXPDG_OK;
}

extern "C" int expdg_profile_enable(expdg_mesh *m, int c, int enable) {
    if (!m || c < 0 || c >= EXPDG_K_NCLASSES) return fail(EXPDG_EINVAL, "bad kernel class");
    DeviceGuard g(m->d.device);
    auto &P = m->prof[c];
    if (P.used) TRY(prof_flush(m, c));
    if (enable && P.ev.empty()) {
        P.ev.resize(2 * kProfPairs, nullptr);
        P.bytes.resize(kProfPairs, 0.0);
        for (auto &e : P.ev) HIPTRY(hipEventCreate(&e));
    }
    P.on = enable != 0;
    P.launches = 0;
    P.ms = 0.0;
    P.total_bytes = 0.0;
    return EXPDG_OK;
}

extern "C" int expdg_profile_read(expdg_mesh *m, int c, expdg_kernel_profile *out) {
    if (!m || !out || c < 0 || c >= EXPDG_K_NCLASSES) return fail(EXPDG_EINVAL, "bad argument");
    DeviceGuard g(m->d.device);
    TRY(prof_flush(m, c));
    out->launches = m->prof[c].launches;
    out->total_ms = m->prof[c].ms;
    out->bytes = m->prof[c].total_bytes;
    return EXPDG_OK;
}

extern "C" const char *expdg_last_error(void) { return g_err; }

extern "C" int expdg_version(void) { return 100; }
