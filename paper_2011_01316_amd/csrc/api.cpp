// C ABI of the MI355X exponential-DG library: validation, mesh and workspace,
// the stand-alone operator, phi and step entry points, and live kernel timing.
// Every arithmetic step on state-sized data runs in the HIP kernels of
// dg_kernels.hip and krylov_kernels.hip; the host only makes the scalar
// controller decisions (controller.h).  The solve server is in serve.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "controller.h"
#include "runtime.h"

using namespace expdg;

// ---------------------------------------------------------------------------
// errors, shared helpers
namespace expdg {

namespace {
thread_local char g_err[512] = "no error";
}

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

double round2(double x) {
    if (!(x > 0.0)) return x;
    const double s = std::pow(10.0, std::floor(std::log10(x)) - 1.0);
    return std::ceil(x / s) * s;
}

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
    double Pv[kMaxP + 1];
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

namespace expdg {

bool desc_ok(const expdg_mesh_desc *d, const char **why) {
    if (!d) return *why = "desc is NULL", false;
    if (d->equation != EXPDG_BURGERS1D && d->equation != EXPDG_EULER2D &&
        d->equation != EXPDG_EULER3D)
        return *why = "equation must be EXPDG_BURGERS1D, EXPDG_EULER2D or EXPDG_EULER3D", false;
    if (d->equation == EXPDG_EULER3D) {
        if (d->nz < 1) return *why = "Euler 3D needs nz >= 1", false;
        if (!(d->z1 > d->z0) || !std::isfinite(d->z0) || !std::isfinite(d->z1))
            return *why = "need z1 > z0", false;
    } else if (d->nz > 1) {
        return *why = "nz > 1 needs EXPDG_EULER3D", false;
    }
    if (d->p < 1 || d->p > kMaxP) return *why = "p must be in 1..6", false;
    if (d->nx < 1 || d->ny < 1) return *why = "nx and ny must be >= 1", false;
    if (d->equation == EXPDG_BURGERS1D && d->ny != 1) return *why = "Burgers needs ny == 1", false;
    const long long nzz = (d->equation == EXPDG_EULER3D) ? d->nz : 1;
    if ((long long)d->nx * d->ny * nzz > (1LL << 26)) return *why = "too many elements", false;
    {
        // the kernels address one variable plane with 32-bit byte offsets
        const long long n1 = d->p + 1;
        const long long np = (d->equation == EXPDG_BURGERS1D) ? n1
                             : (d->equation == EXPDG_EULER2D) ? n1 * n1 : n1 * n1 * n1;
        if ((long long)d->nx * d->ny * nzz * np > (1LL << 29) - 1)
            return *why = "too many nodes (at most 2^29 - 1 per variable)", false;
    }
    if (d->precision != EXPDG_FP64 && d->precision != EXPDG_FP32_BULK)
        return *why = "precision must be EXPDG_FP64 or EXPDG_FP32_BULK", false;
    if (!(d->x1 > d->x0) || !std::isfinite(d->x0) || !std::isfinite(d->x1))
        return *why = "need x1 > x0", false;
    if (d->equation != EXPDG_BURGERS1D) {
        if (!(d->y1 > d->y0) || !std::isfinite(d->y0) || !std::isfinite(d->y1))
            return *why = "need y1 > y0", false;
        if (!(d->gamma > 1.0) || !std::isfinite(d->gamma)) return *why = "need gamma > 1", false;
    }
    if (d->m_max < 1 || d->m_max > kMaxM) return *why = "m_max must be in 1..64", false;
    if (d->device < 0) return *why = "device must be >= 0", false;
    if (!(d->kappa >= 0.0) || !std::isfinite(d->kappa)) return *why = "need kappa >= 0", false;
    if (!(d->sigma >= 0.0) || !std::isfinite(d->sigma)) return *why = "need sigma >= 0", false;
    if (!(std::fabs(d->beta) <= 0.5)) return *why = "need |beta| <= 1/2", false;
    if (d->flux != EXPDG_FLUX_LF && d->flux != EXPDG_FLUX_EF && d->flux != EXPDG_FLUX_EF_LOCAL)
        return *why = "flux must be EXPDG_FLUX_LF, EXPDG_FLUX_EF or EXPDG_FLUX_EF_LOCAL", false;
    if (d->bc != EXPDG_BC_PERIODIC && d->bc != EXPDG_BC_DIRICHLET && d->bc != EXPDG_BC_WALL_Y)
        return *why = "bc must be EXPDG_BC_PERIODIC, EXPDG_BC_DIRICHLET or EXPDG_BC_WALL_Y", false;
    if (d->bc == EXPDG_BC_WALL_Y && d->equation != EXPDG_EULER2D)
        return *why = "EXPDG_BC_WALL_Y needs EXPDG_EULER2D", false;
    if (d->equation != EXPDG_BURGERS1D &&
        (d->kappa != 0.0 || d->flux != EXPDG_FLUX_LF || d->sigma != 0.0 || d->beta != 0.0 ||
         d->bc == EXPDG_BC_DIRICHLET || d->has_source))
        return *why = "Euler takes no Burgers options (kappa, flux, sigma, beta, Dirichlet, source)",
               false;
    if (!(d->ev_ce >= 0.0) || !std::isfinite(d->ev_ce) || !(d->ev_cmax >= 0.0) ||
        !std::isfinite(d->ev_cmax))
        return *why = "need ev_ce >= 0 and ev_cmax >= 0", false;
    if (d->ev_ce > 0.0 && d->equation != EXPDG_EULER2D)
        return *why = "entropy viscosity needs EXPDG_EULER2D", false;
    return true;
}

namespace {

// Lays the device buffers of a mesh out in one block (256-byte aligned);
// assigns the pointers if base is given and returns the block size.
size_t layout(expdg_mesh *m, const expdg_mesh_desc *d, size_t stride, int eb, char *base) {
    size_t off = 0;
    auto take = [&](auto *&ptr, size_t bytes) {
        using P = std::remove_reference_t<decltype(ptr)>;
        off = (off + 255) / 256 * 256;
        if (base) ptr = (P)(base + off);
        off += bytes;
    };
    const size_t vb = stride * eb;
    // m_max + 2 vectors: the step that finishes dimension m_max also writes the next one
    take(m->V, (size_t)(d->m_max + 2) * vb);
    for (auto &v : m->vec) take(v, vb);
    if (d->precision == EXPDG_FP32_BULK) take(m->bq, vb);
    take(m->q2, stride * 8);
    if (d->has_source) take(m->src, vb);
    // elements of the mesh (nz counts in 3D only)
    const int K = d->nx * d->ny * (d->equation == EXPDG_EULER3D ? d->nz : 1);
    const size_t nlin = lin_elems(d->equation, d->p, K);
    if (nlin) take(m->lin, nlin * eb);
    if (d->ev_ce > 0.0) {
        const size_t pts = (size_t)K * (d->p + 1) * (d->p + 1);
        take(m->nu, pts * eb);
        take(m->nue, (size_t)K * 8);
    }
    take(m->kd.H, (size_t)(kMaxM + 1) * kLDH * 8);
    take(m->kd.S, (size_t)(kMaxM + 1) * 8);
    take(m->kd.coefA, (size_t)(kMaxM + 1) * 8);
    take(m->kd.coefB, (size_t)(kMaxM + 3) * 8);
    // block partials: row-partitioned passes (<= kRedBlocks) and the dot pass
    // fused into the linear operator (one partial per operator block)
    const size_t npart = std::max<size_t>(kRedBlocks, dg_blocks(d->equation, d->p, K));
    take(m->kd.part, npart * kPartRows * 8);
    take(m->kd.fold, (size_t)std::max(1, fold_chunks((int)npart)) * kPartRows * 8);
    take(m->kd.res, 64 * 8);
    take(m->kd.flags, 16);
    take(m->slots, (size_t)kCheckSlots * kSlotSize * 8);
    take(m->dnorm, 8 * 8);
    take(m->spart, 1024 * 8);
    return (off + 255) / 256 * 256;
}

}  // namespace

Sizes sizes_of(const expdg_mesh_desc *d) {
    Sizes s{};
    const int n1 = d->p + 1;
    const int dim = (d->equation == EXPDG_BURGERS1D) ? 1 : (d->equation == EXPDG_EULER2D ? 2 : 3);
    const int Np = (dim == 1) ? n1 : (dim == 2 ? n1 * n1 : n1 * n1 * n1);
    const int nvar = (dim == 1) ? 1 : dim + 2;
    const size_t K = (size_t)d->nx * d->ny * (dim == 3 ? d->nz : 1);
    s.n = (size_t)nvar * K * Np;
    s.stride = (s.n + kMaxAug + 63) / 64 * 64;
    s.ebytes = (d->precision == EXPDG_FP64) ? 8 : 4;
    expdg_mesh probe;
    s.total = layout(&probe, d, s.stride, s.ebytes, nullptr);
    return s;
}

void mesh_setup(expdg_mesh *m, const expdg_mesh_desc *d) {
    m->d = *d;
    m->dim = (d->equation == EXPDG_BURGERS1D) ? 1 : (d->equation == EXPDG_EULER2D ? 2 : 3);
    m->n1 = d->p + 1;
    m->Np = (m->dim == 1) ? m->n1 : (m->dim == 2 ? m->n1 * m->n1 : m->n1 * m->n1 * m->n1);
    m->K = d->nx * d->ny * (m->dim == 3 ? d->nz : 1);
    m->nvar = (m->dim == 1) ? 1 : m->dim + 2;
    const Sizes sz = sizes_of(d);
    m->n = sz.n;
    m->stride = sz.stride;
    m->ebytes = sz.ebytes;
    m->bytes = sz.total;
    m->hx = (d->x1 - d->x0) / d->nx;
    m->hy = (m->dim >= 2) ? (d->y1 - d->y0) / d->ny : 1.0;
    m->hz = (m->dim == 3) ? (d->z1 - d->z0) / d->nz : 1.0;
    lgl_tables(d->p, m->xi, m->w, m->D);
    double dmin = 2.0;
    for (int i = 0; i < d->p; ++i) dmin = std::min(dmin, m->xi[i + 1] - m->xi[i]);
    double hmin = m->hx;
    if (m->dim >= 2) hmin = std::min(hmin, m->hy);
    if (m->dim == 3) hmin = std::min(hmin, m->hz);
    m->dxmin = 0.5 * hmin * dmin;
}

void mesh_carve(expdg_mesh *m, void *block) {
    m->block = block;
    layout(m, &m->d, m->stride, m->ebytes, (char *)block);
}

// ---- live timing ----

namespace {

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

}  // namespace

// The next kernel launch records the event pair as part of its own dispatch
// (hipExtLaunchKernelGGL), so the interval is the kernel's execution.
int prof_begin(expdg_mesh *m, int c) {
    auto &P = m->prof[c];
    if (!P.on) return EXPDG_OK;
    if (P.used == kProfPairs) TRY(prof_flush(m, c));
    next_launch_events() = LaunchEvents{P.ev[2 * P.used], P.ev[2 * P.used + 1]};
    return EXPDG_OK;
}

int prof_end(expdg_mesh *m, int c, double bytes) {
    auto &P = m->prof[c];
    if (!P.on) return EXPDG_OK;
    next_launch_events() = LaunchEvents{};
    P.bytes[P.used] = bytes;
    P.used += 1;
    return EXPDG_OK;
}

}  // namespace expdg

namespace {

void release(expdg_mesh *m) {
    if (m->owns_block && m->block) (void)hipFree(m->block);
    m->block = nullptr;
    if (m->owns_pin && m->pin) (void)hipHostFree(m->pin);
    m->pin = nullptr;
    for (auto &e : m->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : m->evH)
        if (e) (void)hipEventDestroy(e);
    for (auto &st : m->side)
        if (st) (void)hipStreamDestroy(st);
    for (auto &P : m->prof)
        for (auto &e : P.ev) (void)hipEventDestroy(e);
}

}  // namespace

extern "C" size_t expdg_workspace_bytes(const expdg_mesh_desc *d) {
    const char *why = "";
    if (!desc_ok(d, &why)) return 0;
    return sizes_of(d).total;
}

extern "C" int expdg_mesh_create(const expdg_mesh_desc *d, expdg_mesh **out) {
    const char *why = "";
    if (!out) return fail(EXPDG_EINVAL, "out is NULL");
    if (!desc_ok(d, &why)) return fail(EXPDG_EINVAL, "invalid mesh description: %s", why);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(EXPDG_EDEVICE, "no HIP device available");
    if (d->device >= ndev) return fail(EXPDG_EINVAL, "device %d out of range", d->device);
    DeviceGuard g(d->device);
    if (!g.ok) return fail(EXPDG_EDEVICE, "hipSetDevice(%d) failed", d->device);

    expdg_mesh *m = new (std::nothrow) expdg_mesh();
    if (!m) return fail(EXPDG_ENOMEM, "host allocation failed");
    mesh_setup(m, d);

    int rc = EXPDG_OK;
    void *block = nullptr;
    if (hipMalloc(&block, m->bytes) != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(EXPDG_ENOMEM, "hipMalloc of %zu bytes failed", m->bytes);
    } else {
        m->owns_block = true;
        mesh_carve(m, block);
    }
    // pinned mirror, also written by the check kernels through its device address
    if (rc == EXPDG_OK) {
        if (hipHostMalloc((void **)&m->pin, kPinSize * 8,
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            m->pin = nullptr;
            rc = fail(EXPDG_ENOMEM, "pinned host allocation failed");
        } else {
            m->owns_pin = true;
            if (hipHostGetDevicePointer((void **)&m->pin_dev, m->pin, 0) != hipSuccess)
                rc = fail(EXPDG_EDEVICE, "hipHostGetDevicePointer failed");
        }
    }
    for (auto &e : m->ev)
        if (rc == EXPDG_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            rc = fail(EXPDG_EDEVICE, "hipEventCreate failed");
    for (auto &e : m->evH)
        if (rc == EXPDG_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            rc = fail(EXPDG_EDEVICE, "hipEventCreate failed");
    // two default-priority side streams for the small exponentials: checks
    // alternate between them by slot parity, so two run at once (a slot's
    // next user queues behind its previous one on the same stream)
    for (auto &st : m->side)
        if (rc == EXPDG_OK && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            rc = fail(EXPDG_EDEVICE, "hipStreamCreate failed");
    if (rc == EXPDG_OK) {
        // zero the whole workspace once (vector padding stays zero)
        if (hipMemset(m->block, 0, m->bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
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
    info->hz = m->hz;
    info->dx_min = m->dxmin;
    return EXPDG_OK;
}

extern "C" int expdg_mesh_nodes(const expdg_mesh *m, double *x, double *y, double *z) {
    if (!m || !x) return fail(EXPDG_EINVAL, "NULL argument");
    const int n1 = m->n1;
    for (int e = 0; e < m->K; ++e) {
        const int ex = e % m->d.nx, ey = (e / m->d.nx) % m->d.ny, ez = e / (m->d.nx * m->d.ny);
        for (int nn = 0; nn < m->Np; ++nn) {
            const int i = nn % n1, j = (nn / n1) % n1, k = nn / (n1 * n1);
            const size_t at = (size_t)e * m->Np + nn;
            x[at] = m->d.x0 + ex * m->hx + 0.5 * (m->xi[i] + 1.0) * m->hx;
            if (y)
                y[at] = (m->dim >= 2) ? m->d.y0 + ey * m->hy + 0.5 * (m->xi[j] + 1.0) * m->hy : 0.0;
            if (z)
                z[at] = (m->dim == 3) ? m->d.z0 + ez * m->hz + 0.5 * (m->xi[k] + 1.0) * m->hz : 0.0;
        }
    }
    return EXPDG_OK;
}

extern "C" int expdg_mesh_set_source(expdg_mesh *m, const double *src, void *stream) {
    if (!m || !src) return fail(EXPDG_EINVAL, "NULL argument");
    if (!m->src) return fail(EXPDG_EINVAL, "the mesh was created without has_source");
    DeviceGuard g(m->d.device);
    hipStream_t s = (hipStream_t)stream;
    if (m->d.precision == EXPDG_FP64)
        HIPTRY(launch_copy(src, (double *)m->src, m->n, s));
    else
        HIPTRY(launch_convert(src, (float *)m->src, m->n, s));
    return EXPDG_OK;
}

extern "C" int expdg_mesh_set_viscosity(expdg_mesh *m, const double *nu, void *stream) {
    if (!m || !nu) return fail(EXPDG_EINVAL, "NULL argument");
    if (!m->nu) return fail(EXPDG_EINVAL, "the mesh was created without entropy viscosity");
    DeviceGuard g(m->d.device);
    hipStream_t s = (hipStream_t)stream;
    const size_t pts = (size_t)m->K * m->Np;
    if (m->d.precision == EXPDG_FP64)
        HIPTRY(launch_copy(nu, (double *)m->nu, pts, s));
    else
        HIPTRY(launch_convert(nu, (float *)m->nu, pts, s));
    return EXPDG_OK;
}

extern "C" int expdg_entropy_viscosity(expdg_mesh *m, const double *q, const double *q_prev,
                                       double dt, double *nu, void *stream) {
    if (!m || !q || !q_prev) return fail(EXPDG_EINVAL, "NULL argument");
    if (!m->nu) return fail(EXPDG_EINVAL, "the mesh was created without entropy viscosity");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(EXPDG_EINVAL, "dt must be > 0");
    DeviceGuard g(m->d.device);
    hipStream_t s = (hipStream_t)stream;
    const size_t pts = (size_t)m->K * m->Np;
    if (m->d.precision == EXPDG_FP64) {
        TRY(entropy_viscosity<double>(m, q, q_prev, dt, s));
        if (nu) HIPTRY(launch_copy((const double *)m->nu, nu, pts, s));
    } else {
        TRY(entropy_viscosity<float>(m, q, q_prev, dt, s));
        if (nu) HIPTRY(launch_convert((const float *)m->nu, nu, pts, s));
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
    if (m->d.precision == EXPDG_FP64) {
        HIPTRY(prepare_lin<double>(m, (const double *)qref, s));
        return apply_op<double>(m, true, (const double *)qref, (const double *)v, (double *)w, s);
    }
    HIPTRY(prepare_lin<float>(m, (const float *)qref, s));
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
// Allocation-free linear operator.  The only device memory the linear operator
// needs beyond its inputs and output is the frozen-field buffer of the 2D and
// 3D Euler operators; expdg_jvp_noalloc keeps it in a file-scope device array
// (one copy per GPU, resident until the process ends) instead of a mesh
// workspace, so it needs no mesh handle and allocates nothing.

namespace {

constexpr size_t kScratchBytes = (size_t)EXPDG_NOALLOC_SCRATCH_MIB << 20;
constexpr int kScratchDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};

// Device address of the current device's copy of scratch, looked up once per
// device (with that device current) and kept.  The array's host-side name is
// only a stand-in: kernels get this address.
int scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(EXPDG_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s",
                        device, hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return EXPDG_OK;
}

}  // namespace

extern "C" int expdg_jvp_noalloc(const expdg_mesh_desc *d, const void *qref, const void *v,
                                 void *w, void *stream) {
    const char *why = "";
    if (!desc_ok(d, &why)) return fail(EXPDG_EINVAL, "invalid mesh description: %s", why);
    if (d->ev_ce > 0.0)
        return fail(EXPDG_EINVAL, "entropy viscosity needs a mesh (it holds nu): use expdg_jvp");
    if (!qref || !v || !w) return fail(EXPDG_EINVAL, "NULL argument");
    if (v == w || qref == w) return fail(EXPDG_EINVAL, "output must not alias an input");
    if (d->device >= kScratchDevices) return fail(EXPDG_EINVAL, "device %d out of range", d->device);
    expdg_mesh m;  // host-side description only: no device block, events or streams
    mesh_setup(&m, d);
    const size_t need = lin_elems(d->equation, d->p, m.K) * (size_t)m.ebytes;
    if (need > kScratchBytes)
        return fail(EXPDG_EINVAL,
                    "the frozen fields of this mesh take %zu bytes, more than the %zu bytes of "
                    "static scratch of expdg_jvp_noalloc",
                    need, kScratchBytes);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(EXPDG_EDEVICE, "no HIP device available");
    if (d->device >= ndev) return fail(EXPDG_EINVAL, "device %d out of range", d->device);
    DeviceGuard g(d->device);
    if (!g.ok) return fail(EXPDG_EDEVICE, "hipSetDevice(%d) failed", d->device);
    void *scr = nullptr;
    TRY(scratch_address(d->device, &scr));
    m.lin = need ? scr : nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (d->precision == EXPDG_FP64) {
        HIPTRY(prepare_lin<double>(&m, (const double *)qref, s));
        return apply_op<double>(&m, true, (const double *)qref, (const double *)v, (double *)w, s);
    }
    HIPTRY(prepare_lin<float>(&m, (const float *)qref, s));
    return apply_op<float>(&m, true, (const float *)qref, (const float *)v, (float *)w, s);
}

// ---------------------------------------------------------------------------
// phi combinations and steps: the controller driven by the immediate executor

namespace expdg {

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
    if (o->iop < 0 || o->iop > kMaxM) return fail(EXPDG_EINVAL, "iop must be in 0..64");
    if (o->adapt != 0 && o->adapt != 1) return fail(EXPDG_EINVAL, "adapt must be 0 or 1");
    if (o->m_init < 0 || o->m_init > o->m_max)
        return fail(EXPDG_EINVAL, "m_init must be in 0..m_max");
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

}  // namespace expdg

namespace {

// Launches everything at once on stream s; a check's small exponential runs on
// one of the mesh's two side streams behind the Hessenberg column it needs,
// overlapping the next Arnoldi steps (and the previous check), and is read
// back one step later.
template <typename T>
struct DirectExec {
    // a check is decided one Arnoldi step after the one that launched it (a
    // deeper lookahead measured slower: the host, not the check, sets the pace)
    static constexpr int kLookahead = 1;
    hipStream_t s;

    hipStream_t stream() const { return s; }

    // A check in two parts: mark_check records, on the main stream, the point
    // after which H and S hold what the check reads; submit_check queues the
    // small exponential behind that point on a side stream.  Main-stream
    // work enqueued in between does not wait for the side-stream calls.
    int mark_check(expdg_mesh *m, const CheckReq &r, Check *c) {
        c->j = r.j;
        c->slot = r.slot;
        HIPTRY(hipEventRecord(m->evH[c->slot], s));
        return EXPDG_OK;
    }
    int submit_check(expdg_mesh *m, const CheckReq &r, const Check &c) {
        hipStream_t side = m->side[c.slot & 1];
        HIPTRY(hipStreamWaitEvent(side, m->evH[c.slot], 0));
        const KrylovDev &kd = m->kd;
        ExpmItem it{kd.H,
                    kd.S,
                    kd.res,
                    kd.flags,
                    m->slots + c.slot * kSlotSize,
                    m->pin_dev + kPinSlots + c.slot * 8,
                    r.dtau,
                    r.j};
        TRY(prof_begin(m, EXPDG_K_SMALLEXPM));
        HIPTRY(launch_hess_expm(it, side));
        TRY(prof_end(m, EXPDG_K_SMALLEXPM, 0.0));
        HIPTRY(hipEventRecord(m->ev[c.slot], side));
        return EXPDG_OK;
    }
    int enqueue_check(expdg_mesh *m, const CheckReq &r, Check *c) {
        TRY(mark_check(m, r, c));
        return submit_check(m, r, *c);
    }

    // Arnoldi step k: the operator on x = u_{k-1} (and, in 2D, the dot pass
    // in its epilogue), the dot pass (1D), the finish, the update sweep.
    int iterate_now(expdg_mesh *m, const OpArgs<T> &a, int k, int naug_nz, const CheckReq *cr,
                    Check *c, bool iop) {
        const size_t n = m->n, L = n + (size_t)a.naug, stride = m->stride;
        const RowPartition rp = row_partition(L);
        const KrylovDev &kd = m->kd;
        T *V = (T *)m->V;
        T *x = V + (size_t)(k - 1) * stride, *w = a.out;
        const T *basis = a.basis;
        const int nv = a.nv;  // vectors the dot pass and the update read
        const double eb = (double)sizeof(T);
        const bool fused = a.dots != 0;
        TRY(prof_begin(m, EXPDG_K_LINEAR));
        HIPTRY(launch_dg_op(m->d.equation, m->d.p, true, a, s));
        TRY(prof_end(m, EXPDG_K_LINEAR,
                     op_bytes(m, true) + (double)(naug_nz + (fused ? nv : 0)) * n * eb));
        if (!fused) {
            TRY(prof_begin(m, EXPDG_K_GS_DOTS));
            HIPTRY(launch_gs_dots2<T>(basis, stride, nv, x, w, L, rp, kd.part, s));
            TRY(prof_end(m, EXPDG_K_GS_DOTS, (double)(nv + 2) * L * eb));
        }
        int nrb = fused ? a.dnb : rp.nrb;
        const double *part = kd.part;
        const int rows = 2 * nv + 2;
        if (fold_chunks(nrb) > 0) {
            // long partial rows (one per block of a large operator launch)
            TRY(prof_begin(m, EXPDG_K_GS_FOLD));
            HIPTRY(launch_fold(kd.part, nrb, rows, kd.fold, s));
            TRY(prof_end(m, EXPDG_K_GS_FOLD, 8.0 * rows * (nrb + fold_chunks(nrb))));
            part = kd.fold;
            nrb = fold_chunks(nrb);
        }
        TRY(prof_begin(m, EXPDG_K_GS_FINISH));
        if (iop)
            HIPTRY(launch_iop_finish(part, nrb, k, k - 1 - nv, nv, kd.S, kd.H, kd.coefA, kd.coefB,
                                     kd.flags, s));
        else
            HIPTRY(launch_dcgs_finish(part, nrb, k, kd.S, kd.H, kd.coefA, kd.coefB, kd.flags, s));
        TRY(prof_end(m, EXPDG_K_GS_FINISH, 8.0 * nrb * rows));
        // the check needs H and S only: it starts while the update sweep runs
        if (cr) TRY(mark_check(m, *cr, c));
        TRY(prof_begin(m, EXPDG_K_GS_UPDATE));
        // incomplete orthogonalization leaves x as it is (only its scale is new)
        // with the dot pass in the operator's epilogue, the sweep runs against
        // the operator's order (kUpdateLanesPerPlane; the 3D operator walks
        // its columns through every z layer, which eight lanes per plane only
        // approximate, and its vectors are too large for the cache to matter);
        // after the separate 1D dot pass, which walks the rows upwards, one
        // lane walked downwards
        const int lanes = fused ? kUpdateLanesPerPlane * m->nvar : 1;
        HIPTRY(launch_dcgs_update<T>(basis, stride, nv, kd.coefA, kd.coefB, x, w, L, rp, s,
                                     !iop, lanes));
        TRY(prof_end(m, EXPDG_K_GS_UPDATE,
                     (double)(nv + ((nv > 0 && !iop) ? 4 : 3)) * L * eb));
        if (cr) TRY(submit_check(m, *cr, *c));
        return EXPDG_OK;
    }

    Ready iterate(expdg_mesh *m, const OpArgs<T> &a, int k, int naug_nz, const CheckReq *cr,
                  Check *c, bool iop) {
        return Ready{iterate_now(m, a, k, naug_nz, cr, c, iop)};
    }
    Ready check(expdg_mesh *m, const CheckReq &r, Check *c) { return Ready{enqueue_check(m, r, c)}; }
    Ready wait_check(expdg_mesh *m, const Check &c) { return Ready{sync_event(m->ev[c.slot])}; }
    int after_check(expdg_mesh *m, const Check &c) {
        HIPTRY(hipStreamWaitEvent(s, m->ev[c.slot], 0));
        return EXPDG_OK;
    }
    Ready readback(expdg_mesh *) { return Ready{sync_stream(s)}; }
    Ready finish(expdg_mesh *m) {
        // no speculative check left running on a side stream
        int rc = sync_stream(m->side[0]);
        if (rc == EXPDG_OK) rc = sync_stream(m->side[1]);
        if (rc == EXPDG_OK) rc = sync_stream(s);
        return Ready{rc};
    }

    static int sync_event(hipEvent_t e) {
        HIPTRY(hipEventSynchronize(e));
        return EXPDG_OK;
    }
    static int sync_stream(hipStream_t st) {
        HIPTRY(hipStreamSynchronize(st));
        return EXPDG_OK;
    }
};

// Runs a controller task to completion (the immediate executor never suspends).
int run_now(Task<int> t) {
    if (!t.valid()) return fail(EXPDG_ENOMEM, "coroutine frame allocation failed");
    t.start();
    if (!t.done()) return fail(EXPDG_EDEVICE, "controller suspended under the immediate executor");
    return t.result();
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
    if (m->d.precision == EXPDG_FP64) {
        DirectExec<double> x{st};
        return run_now(phi_co<double>(x, m, (const double *)qref, tau, p, (const double *const *)b,
                                      (double *)w, o, s, &fpos, false, false));
    }
    DirectExec<float> x{st};
    return run_now(phi_co<float>(x, m, (const float *)qref, tau, p, (const float *const *)b,
                                 (float *)w, o, s, &fpos, false, false));
}

extern "C" int expdg_step(expdg_mesh *m, int scheme, double dt, double *q, double *q_prev,
                          int have_prev, const expdg_krylov_opts *o, expdg_krylov_stats *s,
                          void *stream) {
    if (!m || !q) return fail(EXPDG_EINVAL, "NULL argument");
    if (scheme != EXPDG_EPI2 && scheme != EXPDG_EPI3 && scheme != EXPDG_EXPRB32 &&
        scheme != EXPDG_EXPRB42)
        return fail(EXPDG_EINVAL, "unknown scheme %d", scheme);
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(EXPDG_EINVAL, "dt must be > 0");
    if (scheme == EXPDG_EPI3 && have_prev && !q_prev)
        return fail(EXPDG_EINVAL, "EPI3 with have_prev needs q_prev");
    if (q_prev == q) return fail(EXPDG_EINVAL, "q_prev must not alias q");
    TRY(check_opts(m, o));
    DeviceGuard g(m->d.device);
    hipStream_t st = (hipStream_t)stream;
    if (m->d.precision == EXPDG_FP64) {
        DirectExec<double> x{st};
        return run_now(step_co<double>(x, m, scheme, dt, q, q_prev, have_prev, o, s));
    }
    DirectExec<float> x{st};
    return run_now(step_co<float>(x, m, scheme, dt, q, q_prev, have_prev, o, s));
}

extern "C" int expdg_integrate(expdg_mesh *m, int scheme, double dt, int nsteps, double *q,
                               double *q_prev, int have_prev, const expdg_krylov_opts *o,
                               expdg_krylov_stats *s, void *stream) {
    if (!m || !q) return fail(EXPDG_EINVAL, "NULL argument");
    if (nsteps < 1) return fail(EXPDG_EINVAL, "nsteps must be >= 1");
    if (scheme != EXPDG_EPI2 && scheme != EXPDG_EPI3 && scheme != EXPDG_EXPRB32 &&
        scheme != EXPDG_EXPRB42)
        return fail(EXPDG_EINVAL, "unknown scheme %d", scheme);
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(EXPDG_EINVAL, "dt must be > 0");
    if (scheme == EXPDG_EPI3 && (have_prev || nsteps > 1) && !q_prev)
        return fail(EXPDG_EINVAL, "EPI3 over several steps needs q_prev");
    if (q_prev == q) return fail(EXPDG_EINVAL, "q_prev must not alias q");
    TRY(check_opts(m, o));
    DeviceGuard g(m->d.device);
    hipStream_t st = (hipStream_t)stream;
    if (m->d.precision == EXPDG_FP64) {
        DirectExec<double> x{st};
        return run_now(
            integrate_co<double>(x, m, scheme, dt, nsteps, q, q_prev, have_prev, o, s));
    }
    DirectExec<float> x{st};
    return run_now(integrate_co<float>(x, m, scheme, dt, nsteps, q, q_prev, have_prev, o, s));
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

extern "C" int expdg_version(void) { return 200; }
