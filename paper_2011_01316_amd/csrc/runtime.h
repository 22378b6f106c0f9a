// Host runtime of the library (not part of the C ABI): the mesh / workspace
// object, error reporting, live kernel timing, and the small helpers shared by
// the stand-alone entry points and the solve server.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <vector>

#include "internal.h"

// Mesh, reference element, and the Krylov workspace of one solve.  All device
// buffers are carved out of one contiguous block (owned by the mesh for the
// stand-alone entry points, by the server's HBM arena for served solves).
struct expdg_mesh {
    expdg_mesh_desc d;
    int nvar, n1, Np, K, dim;
    size_t n;       // ndof
    size_t stride;  // elements between Krylov vectors (>= n + kMaxAug)
    int ebytes;     // bytes per bulk element
    double hx, hy, hz, dxmin;
    double xi[expdg::kMaxP + 1], w[expdg::kMaxP + 1];
    double D[(expdg::kMaxP + 1) * (expdg::kMaxP + 1)];

    void *block = nullptr;       // the device block (owned iff owns_block)
    bool owns_block = false;
    void *V = nullptr;           // (m_max+1) x stride bulk
    void *vec[6] = {};           // bulk work vectors (stride each)
    void *bq = nullptr;          // bulk copy of the FP64 state q^n (FP32_BULK only)
    double *q2 = nullptr;        // FP64 stage state (EXPRB32)
    void *src = nullptr;         // source term of the residual (bulk type; has_source only)
    void *lin = nullptr;         // frozen fields of the 2D linear operator (bulk type)
    void *nu = nullptr;          // entropy viscosity at the nodes (bulk type; ev_ce > 0 only)
    double *nue = nullptr;       // element viscosities (K)
    expdg::KrylovDev kd{};
    double *slots = nullptr;     // kCheckSlots x kSlotSize
    double *dnorm = nullptr;     // 8
    double *spart = nullptr;     // 1024 (wave-speed partials)
    double *pin = nullptr;       // pinned, device-mapped host mirror (kPinSize doubles)
    double *pin_dev = nullptr;   // the device's address of pin
    bool owns_pin = false;
    hipEvent_t ev[expdg::kCheckSlots] = {};   // check results ready (side stream)
    hipEvent_t evH[expdg::kCheckSlots] = {};  // Hessenberg column ready (main stream)
    hipStream_t side[2] = {};                // small exponentials run here (slot parity)
    size_t bytes = 0;

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

namespace expdg {

// pinned mirror layout (doubles)
constexpr int kPinSlots = 0;                      // kCheckSlots x 8: check slot headers
constexpr int kPinNorms = kPinSlots + kCheckSlots * 8;  // 8 input norms
constexpr int kPinSpeed = kPinNorms + 8;             // 1024 wave-speed partials (stand-alone only)
constexpr int kPinServed = kPinSpeed;                // doubles a served solve needs
constexpr int kPinSize = kPinSpeed + 1024;

// Records the message (thread-local, read by expdg_last_error) and returns code.
int fail(int code, const char *fmt, ...);

#define HIPTRY(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::expdg::fail(EXPDG_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define TRY(call)                        \
    do {                                 \
        int rc_ = (call);                \
        if (rc_ != EXPDG_OK) return rc_; \
    } while (0)

#define CO_HIPTRY(call)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            co_return ::expdg::fail(EXPDG_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define CO_TRY(expr)                        \
    do {                                    \
        int rc_ = (expr);                   \
        if (rc_ != EXPDG_OK) co_return rc_; \
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
double round2(double x);

// Description checks and workspace size of a mesh.
bool desc_ok(const expdg_mesh_desc *d, const char **why);
struct Sizes {
    size_t n, stride, total;
    int ebytes;
};
Sizes sizes_of(const expdg_mesh_desc *d);
// Host tables and sizes of a mesh (no device work).
void mesh_setup(expdg_mesh *m, const expdg_mesh_desc *d);
// Points every device buffer into block (sizes_of(d).total bytes, 256-aligned).
void mesh_carve(expdg_mesh *m, void *block);

// Live timing of kernel class c around the next launch (declared above).

template <typename T>
OpArgs<T> op_args(const expdg_mesh *m) {
    OpArgs<T> a{};
    a.K = m->K;
    a.nx = m->d.nx;
    a.ny = m->d.ny;
    a.rhx = 2.0 / m->hx;
    a.rhy = 2.0 / m->hy;
    a.rhz = 2.0 / m->hz;
    a.lift = 1.0 / m->w[0];
    a.gamma = m->d.gamma;
    for (int k = 0; k < m->n1 * m->n1; ++k) a.D[k] = m->D[k];
    a.eta = 1.0;
    a.kappa = m->d.kappa;
    // entropy flux penalty sigma / (h/2): constant, or kappa/100 + (h/2) max|u^+-|
    // per face (the kernel adds max|u^+-| to 2 kappa / (100 h))
    a.ef_local = m->d.flux == EXPDG_FLUX_EF_LOCAL;
    a.ef_pen = a.ef_local ? 2.0 * m->d.kappa / (100.0 * m->hx) : 2.0 * m->d.sigma / m->hx;
    a.beta = m->d.beta;
    a.ef = m->d.flux != EXPDG_FLUX_LF;
    a.dirichlet = m->d.bc == EXPDG_BC_DIRICHLET;
    a.src = (const T *)m->src;
    a.nu = (const T *)m->nu;
    a.ywall = m->d.equation == EXPDG_EULER2D && m->d.bc == EXPDG_BC_WALL_Y;
    return a;
}

// Entropy viscosity parameters of the mesh for a step dt.
inline EvParams ev_params(const expdg_mesh *m, double dt) {
    EvParams ep{};
    ep.K = m->K;
    ep.nx = m->d.nx;
    ep.ny = m->d.ny;
    ep.p = m->d.p;
    ep.ywall = m->d.bc == EXPDG_BC_WALL_Y;
    ep.rhx = 2.0 / m->hx;
    ep.rhy = 2.0 / m->hy;
    ep.lift = 1.0 / m->w[0];
    ep.gamma = m->d.gamma;
    ep.dt = dt;
    ep.ce = m->d.ev_ce;
    ep.cmax = m->d.ev_cmax;
    ep.he = std::sqrt(m->hx * m->hx + m->hy * m->hy) / m->d.p;
    for (int k = 0; k < m->n1; ++k) ep.xi[k] = m->xi[k];
    for (int k = 0; k < m->n1 * m->n1; ++k) ep.D[k] = m->D[k];
    return ep;
}

int prof_begin(expdg_mesh *m, int c);
int prof_end(expdg_mesh *m, int c, double bytes);

// The mesh's nodal viscosity from the FP64 states q and q_prev (ev_ce > 0).
// Algorithmic bytes: both states and the element viscosities (element
// kernel); the element viscosities and the nodal output (reconstruction).
template <typename T>
int entropy_viscosity(expdg_mesh *m, const double *q, const double *q_prev, double dt,
                      hipStream_t s) {
    const EvParams ep = ev_params(m, dt);
    const double pts = (double)m->K * m->Np;
    TRY(prof_begin(m, EXPDG_K_EV_VISC));
    HIPTRY(launch_ev_element(ep, q, q_prev, m->nue, s));
    TRY(prof_end(m, EXPDG_K_EV_VISC, 2.0 * m->n * 8.0 + m->K * 8.0));
    TRY(prof_begin(m, EXPDG_K_EV_VISC));
    HIPTRY(launch_ev_smooth<T>(ep, m->nue, (T *)m->nu, s));
    TRY(prof_end(m, EXPDG_K_EV_VISC, m->K * 8.0 + pts * sizeof(T)));
    return EXPDG_OK;
}

// Frozen fields of the linear operator at the reference state q (into m->lin);
// q may be the FP64 state of an FP32-bulk mesh.
template <typename T, typename Q>
hipError_t prepare_lin(expdg_mesh *m, const Q *q, hipStream_t s) {
    return launch_lin_prepare<Q, T>(m->d.equation, m->d.p, q, (T *)m->lin, m->K, m->d.nx,
                                    m->d.ny, m->d.gamma, s);
}

// Algorithmic bytes of one residual (jvp = false) or linear-operator
// application: the input state and the output (residual); the input vector,
// the output and either the frozen fields (2D) or the reference state (1D)
// (linear operator).  Augmented blocks and fused dots are added by the caller.
inline double op_bytes(const expdg_mesh *m, bool jvp) {
    const double n = (double)m->n, eb = (double)m->ebytes;
    // entropy viscosity: the nodal viscosity
    const double ev = m->nu ? (double)m->K * m->Np * eb : 0.0;
    if (!jvp) return 2.0 * n * eb + ev;
    const double lin = (double)lin_elems(m->d.equation, m->d.p, m->K);
    return (lin > 0.0 ? 2.0 * n + lin : 3.0 * n) * eb + ev;
}


// Residual (jvp = false) or linear operator of the mesh on stream s; the
// linear operator needs the frozen fields of q prepared (prepare_lin).  q64
// (FP32 storage, residual only): the state in FP64, read instead of q.
template <typename T>
int apply_op(expdg_mesh *m, bool jvp, const T *q, const T *v, T *out, hipStream_t s,
             const double *q64 = nullptr) {
    OpArgs<T> a = op_args<T>(m);
    a.q = q;
    a.q64 = q64;
    a.v = v;
    a.out = out;
    a.lin = (const T *)m->lin;
    const int cls = jvp ? EXPDG_K_LINEAR : EXPDG_K_RESIDUAL;
    TRY(prof_begin(m, cls));
    HIPTRY(launch_dg_op(m->d.equation, m->d.p, jvp, a, s));
    TRY(prof_end(m, cls, op_bytes(m, jvp)));
    return EXPDG_OK;
}

// Validation of Krylov options against a mesh.
int check_opts(const expdg_mesh *m, const expdg_krylov_opts *o);
// Appends one accepted substep to the statistics.
void log_sub(expdg_krylov_stats *st, int mm, int last, double dtau);

}  // namespace expdg
