// Fused nodal DG operator kernels for gfx950: residual R(q) and the linear
// operator L(q~) v of the flux-Jacobian split, plus elementwise helpers.
//
// Operator (Section 2.2, eq. EXPO-SemiDiscretizedForm_ode, in strong form on
// LGL nodes with the diagonal LGL mass matrix):
//   out_i = -sum_dir (2/h_dir) sum_l D_il F_dir,l
//           - sum_faces (2/h_dir)(1/w_0) [ s (F^+ - F^-)/2 + lambda (u^- - u^+)/2 ]
// on face nodes, s = +-1 the outward normal along dir.  The residual uses the
// physical flux F(q) and the Lax-Friedrichs / Rusanov speed lambda(q); the
// linear operator uses F_L = A(q~) v with lambda(q~) (Sections 3.1-3.2).
//
// Work mapping: one thread per LGL node, floor(256/Np) whole elements per
// 256-thread block, so a block reads each variable plane as one contiguous
// run.  The per-node fluxes go through LDS for the tensor-product derivative
// (a (p+1)-point contraction per direction: too small for MFMA tiles, it is
// bandwidth-bound).  Face traces of the neighbour are gathered from global
// memory; the block -> tile map gives each XCD a contiguous range of
// elements so y-neighbours (nx elements away) are usually resident in that
// XCD's L2.
#include <type_traits>

#include "internal.h"
#include "reduce.h"

namespace expdg {
namespace {

// Hardware dispatches block b to XCD b % 8.  Give XCD x the contiguous tile
// range it would own under a block partition of the tiles.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    const int q = G >> 3, r = G & 7;
    const int x = b & 7, k = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// ---- Euler physics --------------------------------------------------------
// The operators compute in FP64 for both storage types: the FP32-bulk mode
// loads FP32 vectors, computes in FP64 and rounds only what it stores, so the
// linear operator stays linear up to the storage rounding of its output.
// (With FP32 arithmetic the rounding inside the flux evaluations made the
// Krylov process take 20-35% more iterations than FP64 at the same tolerance;
// FP32 storage alone does not.)
// Reciprocal and square root of the flux and wave-speed evaluations: the
// hardware approximation refined by Newton steps (within an ulp or two of the
// rounded result).  The IEEE-exact FP64 division and square root expand to
// sequences several times longer, and the residual, which evaluates the full
// flux and the Rusanov speeds at every face node, is bound by them.
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double root(double y) {
    const double r = __builtin_amdgcn_rsq(y);  // about 1/sqrt(y)
    const double h = 0.5 * r;
    double s = y * r;
    s = fma(h, fma(-s, s, y), s);
    return fma(h, fma(-s, s, y), s);
}

// Physical fluxes F_x, F_y of q = (rho, m, n, E), m = rho u, n = rho v.
template <typename T>
__device__ __forceinline__ void euler_flux(const T *q, T gm1, T *fx, T *fy) {
    const T ir = recip(q[0]);
    const T u = q[1] * ir, v = q[2] * ir;
    const T p = gm1 * (q[3] - T(0.5) * (q[1] * u + q[2] * v));
    fx[0] = q[1];
    fx[1] = q[1] * u + p;
    fx[2] = q[2] * u;
    fx[3] = (q[3] + p) * u;
    fy[0] = q[2];
    fy[1] = q[1] * v;
    fy[2] = q[2] * v + p;
    fy[3] = (q[3] + p) * v;
}

// Directional derivatives dF_x(q)[d], dF_y(q)[d], written through the
// pressure perturbation dp = (g-1)(|u|^2/2 drho - u dm - v dn + dE); equal to
// the flux Jacobian of Section 3.2 applied to d.
template <typename T>
__device__ __forceinline__ void euler_jac(const T *q, const T *d, T gm1, T *fx, T *fy) {
    const T ir = recip(q[0]);
    const T u = q[1] * ir, v = q[2] * ir;
    const T p = gm1 * (q[3] - T(0.5) * (q[1] * u + q[2] * v));
    const T H = (q[3] + p) * ir;
    const T dp = gm1 * (T(0.5) * (u * u + v * v) * d[0] - u * d[1] - v * d[2] + d[3]);
    fx[0] = d[1];
    fx[1] = T(2) * u * d[1] - u * u * d[0] + dp;
    fx[2] = u * d[2] + v * d[1] - u * v * d[0];
    fx[3] = u * (d[3] + dp) + H * (d[1] - u * d[0]);
    fy[0] = d[2];
    fy[1] = v * d[1] + u * d[2] - u * v * d[0];
    fy[2] = T(2) * v * d[2] - v * v * d[0] + dp;
    fy[3] = v * (d[3] + dp) + H * (d[2] - v * d[0]);
}

// One direction only (for the neighbour trace).
template <typename T, int DIR>
__device__ __forceinline__ void euler_flux_dir(const T *q, T gm1, T *f) {
    const T ir = recip(q[0]);
    const T u = q[1] * ir, v = q[2] * ir;
    const T p = gm1 * (q[3] - T(0.5) * (q[1] * u + q[2] * v));
    const T un = DIR == 0 ? u : v;
    f[0] = q[1 + DIR];
    f[1] = q[1] * un + (DIR == 0 ? p : T(0));
    f[2] = q[2] * un + (DIR == 1 ? p : T(0));
    f[3] = (q[3] + p) * un;
}

template <typename T, int DIR>
__device__ __forceinline__ void euler_jac_dir(const T *q, const T *d, T gm1, T *f) {
    const T ir = recip(q[0]);
    const T u = q[1] * ir, v = q[2] * ir;
    const T p = gm1 * (q[3] - T(0.5) * (q[1] * u + q[2] * v));
    const T H = (q[3] + p) * ir;
    const T dp = gm1 * (T(0.5) * (u * u + v * v) * d[0] - u * d[1] - v * d[2] + d[3]);
    if (DIR == 0) {
        f[0] = d[1];
        f[1] = T(2) * u * d[1] - u * u * d[0] + dp;
        f[2] = u * d[2] + v * d[1] - u * v * d[0];
        f[3] = u * (d[3] + dp) + H * (d[1] - u * d[0]);
    } else {
        f[0] = d[2];
        f[1] = v * d[1] + u * d[2] - u * v * d[0];
        f[2] = T(2) * v * d[2] - v * v * d[0] + dp;
        f[3] = v * (d[3] + dp) + H * (d[2] - v * d[0]);
    }
}

// |u . e_dir| + a, a = sqrt(gamma p / rho).
template <typename T, int DIR>
__device__ __forceinline__ T euler_speed(const T *q, T gamma) {
    const T ir = recip(q[0]);
    const T u = q[1] * ir, v = q[2] * ir;
    const T p = (gamma - T(1)) * (q[3] - T(0.5) * (q[1] * u + q[2] * v));
    return fabs(DIR == 0 ? u : v) + root(gamma * p * ir);
}

// The same directional derivatives from the frozen fields w = (u, v, H) of
// the reference state (linear operator; no division or square root), with
// alpha = dm - u drho, beta = dn - v drho:
//   dp = (g-1)(dE - u alpha - v beta - |u|^2/2 drho),
//   dF_x = (dm, u (dm + alpha) + dp, u dn + v alpha, u (dE + dp) + H alpha),
//   dF_y = (dn, u dn + v alpha, v (dn + beta) + dp, v (dE + dp) + H beta).
template <typename T>
__device__ __forceinline__ void euler_jac_lin(const T *w, const T *d, T gm1, T *fx, T *fy) {
    const T u = w[0], v = w[1], H = w[2];
    const T al = fma(-u, d[0], d[1]), be = fma(-v, d[0], d[2]);
    const T k = T(0.5) * fma(u, u, v * v);
    const T dp = gm1 * fma(-k, d[0], fma(-v, be, fma(-u, al, d[3])));
    const T ep = d[3] + dp;
    const T cross = fma(u, d[2], v * al);
    fx[0] = d[1];
    fx[1] = fma(u, d[1] + al, dp);
    fx[2] = cross;
    fx[3] = fma(u, ep, H * al);
    fy[0] = d[2];
    fy[1] = cross;
    fy[2] = fma(v, d[2] + be, dp);
    fy[3] = fma(v, ep, H * be);
}

template <typename T, int DIR>
__device__ __forceinline__ void euler_jac_lin_dir(const T *w, const T *d, T gm1, T *f) {
    T fx[4], fy[4];
    euler_jac_lin(w, d, gm1, fx, fy);
#pragma unroll
    for (int c = 0; c < 4; ++c) f[c] = DIR == 0 ? fx[c] : fy[c];
}

// Wall mirror of a state or direction (both momenta reversed).
template <typename T>
__device__ __forceinline__ void wall_mirror(const T *q, T *out) {
    out[0] = q[0];
    out[1] = -q[1];
    out[2] = -q[2];
    out[3] = q[3];
}

// |v| + a at a wall from the frozen fields (u, v, H) of the reference state:
// a^2 = (g-1)(H - |u|^2/2) = gamma p / rho (the mirror has the same speed).
template <typename T>
__device__ __forceinline__ T wall_speed_lin(const T *z, T gm1) {
    return fabs(z[1]) + root(gm1 * (z[2] - T(0.5) * (z[0] * z[0] + z[1] * z[1])));
}

// Load of base[off] through a 32-bit byte offset from a block-uniform base
// (one addressing instruction instead of 64-bit index arithmetic); callers
// keep every plane below 2^32 bytes.
template <typename T>
__device__ __forceinline__ T ld32(const T *base, unsigned off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                        (unsigned)(off * (unsigned)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st32(T *base, unsigned off, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (unsigned)(off * (unsigned)sizeof(T))) =
        v;
}

// Frozen fields of the linear operator at the reference state q~ (computed
// once per reference state): planes u, v, H, then the Rusanov speed of every
// x face, lamx[e (p+1) + j] = max(|u|+a) over the face between element e and
// its x+ neighbour at node row j, and of every y face, lamy[e (p+1) + i].
template <int P, typename Q, typename S>
__global__ __launch_bounds__(256) void euler_lin_prepare(const Q *q, S *lin, int K, int nx, int ny,
                                                         double gamma) {
    using T = double;  // arithmetic; S is the storage type
    constexpr int N1 = P + 1, NP = N1 * N1;
    const size_t plane = (size_t)K * NP;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= plane) return;
    const int e = (int)(t / NP), n = (int)(t - (size_t)e * NP);
    const int i = n % N1, j = n / N1;
    T qq[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) qq[c] = q[c * plane + t];
    const T ir = recip(qq[0]);
    const T u = qq[1] * ir, v = qq[2] * ir;
    const T p = (gamma - T(1)) * (qq[3] - T(0.5) * (qq[1] * u + qq[2] * v));
    lin[t] = (S)u;
    lin[plane + t] = (S)v;
    lin[2 * plane + t] = (S)((qq[3] + p) * ir);
    S *lamx = lin + 3 * plane, *lamy = lamx + (size_t)K * N1;
    const int ex = e % nx, ey = e / nx;
    if (i == P) {
        const int en = ey * nx + (ex + 1 == nx ? 0 : ex + 1);
        const size_t nidx = (size_t)en * NP + j * N1;
        T qn[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) qn[c] = q[c * plane + nidx];
        lamx[(size_t)e * N1 + j] = (S)fmax(euler_speed<T, 0>(qq, gamma), euler_speed<T, 0>(qn, gamma));
    }
    if (j == P) {
        const int en = (ey + 1 == ny ? 0 : ey + 1) * nx + ex;
        const size_t nidx = (size_t)en * NP + i;
        T qn[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) qn[c] = q[c * plane + nidx];
        lamy[(size_t)e * N1 + i] = (S)fmax(euler_speed<T, 1>(qq, gamma), euler_speed<T, 1>(qn, gamma));
    }
}

// Dot pass of an Arnoldi step from the tile just produced: over the tile's
// nodes, u_i^T w and u_i^T x for i < nv (x = the input, w = the output, both as
// stored), then x^T x and x^T w; tile 0 adds the augmented entries.  Row r of
// the partials goes to dpart[r * dnb + tile], rows as in launch_gs_dots2.
// CH basis vectors per chunk (2 CH FP64 accumulators per thread): the 2D and
// 3D operators take 8, which keeps the 3D operator at four waves per SIMD
// instead of three and the FP32-bulk 2D operator at five instead of four.
template <typename T, int NV, int NW = 4, int CH = 16, int HV = 1>
__device__ __forceinline__ void op_dots2(const OpArgs<T> &a, bool active, unsigned idx,
                                         size_t plane, const double *xv, const double *wv,
                                         int tile, bool first) {
    static_assert(NW == 4 || NW == 6, "blocks of 256 or 384 threads");
    static_assert(CH == 16 || CH == 8, "chunks of 16 or 8 vectors");
    static_assert(HV == 1 || (HV == 2 && NW == 4), "two halves of 256 threads");
    // HV = 2: the block is two halves of NW waves over the same nodes (thread
    // t and t + 256 hold node t); half h takes chunks h, h + 2, ...  A row's
    // partial is still one half's NW waves in the same order, so the result
    // equals that of one half taking every chunk.
    __shared__ double sw[HV][NW][32];
    __shared__ double s2[NW][2];
    // fixed-order sum over the block's waves
    auto wsum = [](double v0, double v1, double v2, double v3, double v4, double v5) {
        const double s4 = (v0 + v1) + (v2 + v3);
        return NW == 4 ? s4 : s4 + (v4 + v5);
    };
    const int h = HV == 2 ? (int)(threadIdx.x >> 8) : 0;
    const int tid = HV == 2 ? (int)(threadIdx.x & 255) : (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const size_t ntot = NV * plane;
    const int nv = a.nv;
    const bool tail = first && tid == 0 && a.naug > 0;
    const double sc = a.vscale ? *a.vscale : 1.0;
    const int nch = (nv + CH - 1) / CH, iters = (nch + HV - 1) / HV;
    for (int it = 0; it < iters; ++it) {
        const int i0 = (it * HV + h) * CH;
        const bool run = i0 < nv;  // this half has a chunk in this round
        double acc[2 * CH];
#pragma unroll
        for (int k = 0; k < 2 * CH; ++k) acc[k] = 0.0;
        if (active && run) {
            // loads in groups of KG vectors, all issued before their products
            // (vector index clamped, the extra sums dropped), so a group's
            // loads are in flight together
            constexpr int KG = (NV >= 4) ? 4 : CH;
#pragma unroll
            for (int k0 = 0; k0 < CH; k0 += KG) {
                T u[KG][NV];
#pragma unroll
                for (int kk = 0; kk < KG; ++kk) {
                    const T *Vi = a.basis + (size_t)min(i0 + k0 + kk, nv - 1) * a.bstride;
#pragma unroll
                    for (int c = 0; c < NV; ++c) u[kk][c] = ld32(Vi + c * plane, idx);
                }
#pragma unroll
                for (int kk = 0; kk < KG; ++kk) {
                    double sw_ = 0.0, sx_ = 0.0;
#pragma unroll
                    for (int c = 0; c < NV; ++c) {
                        sw_ += (double)u[kk][c] * (double)wv[c];
                        sx_ += (double)u[kk][c] * (double)xv[c];
                    }
                    const bool in = i0 + k0 + kk < nv;
                    acc[k0 + kk] = in ? sw_ : 0.0;
                    acc[CH + k0 + kk] = in ? sx_ : 0.0;
                }
            }
        }
        if (tail && run) {
            for (int t = 0; t < a.naug; ++t) {
                const T wt = (t + 1 < a.naug) ? (T)(sc * (double)a.vtail[t + 1]) : T(0);
                const T xt = a.vtail[t];
#pragma unroll
                for (int k = 0; k < CH; ++k)
                    if (i0 + k < nv) {
                        const double u = (double)a.basis[(size_t)(i0 + k) * a.bstride + ntot + t];
                        acc[k] += u * (double)wt;
                        acc[CH + k] += u * (double)xt;
                    }
            }
        }
        if constexpr (CH == 16) {
            const double v = transpose_reduce32(acc);
            if ((lane & 1) == 0) sw[h][wave][lane >> 1] = v;
        } else {
            const double v = transpose_reduce16(acc);
            if ((lane & 3) == 0) sw[h][wave][lane >> 2] = v;
        }
        __syncthreads();
        if (run && tid < 2 * CH && i0 + (tid % CH) < nv) {
            const int row = (tid < CH) ? i0 + tid : nv + i0 + (tid - CH);
            a.dpart[(size_t)row * a.dnb + tile] =
                wsum(sw[h][0][tid], sw[h][1][tid], sw[h][2][tid], sw[h][3][tid],
                     sw[h][NW > 4 ? 4 : 0][tid], sw[h][NW > 5 ? 5 : 0][tid]);
        }
        __syncthreads();
    }
    // x^T x and x^T w: the first half (both halves hold the same sums)
    double xx = 0.0, xw = 0.0;
    if (active) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            xx += (double)xv[c] * (double)xv[c];
            xw += (double)xv[c] * (double)wv[c];
        }
    }
    if (tail) {
        for (int t = 0; t < a.naug; ++t) {
            const T wt = (t + 1 < a.naug) ? (T)(sc * (double)a.vtail[t + 1]) : T(0);
            const T xt = a.vtail[t];
            xx += (double)xt * (double)xt;
            xw += (double)xt * (double)wt;
        }
    }
    xx = wave_sum(xx);
    xw = wave_sum(xw);
    if (lane == 0 && h == 0) {
        s2[wave][0] = xx;
        s2[wave][1] = xw;
    }
    __syncthreads();
    if (h == 0 && tid < 2)
        a.dpart[(size_t)(2 * nv + tid) * a.dnb + tile] =
            wsum(s2[0][tid], s2[1][tid], s2[2][tid], s2[3][tid], s2[NW > 4 ? 4 : 0][tid],
                 s2[NW > 5 ? 5 : 0][tid]);
}

// ---- Euler 2D operator ------------------------------------------------------
// One tile (floor(256/Np) elements) of the operator; first marks the item's
// first block, which also writes the augmented entries of the output.  The
// linear operator reads the frozen fields of euler_lin_prepare (a.lin), the
// residual the state itself.  Face and augmented terms need no LDS and are
// added before the barrier; -(2/h) D is staged in LDS for the derivative.
// Node offsets are 32-bit within one variable plane.
template <int P, typename S, bool JVP, bool EV = false, typename Q = S, int HV = 1>
__device__ __forceinline__ void euler_op_body(const OpArgs<S> &a, int tile, bool first) {
    using T = double;  // arithmetic; S is the storage type
    static_assert(!JVP || std::is_same<Q, S>::value, "the linear operator reads stored vectors");
    constexpr int N1 = P + 1, NP = N1 * N1, EPB = 256 / NP, NT = EPB * NP;
    __shared__ T sF[8][NT];
    __shared__ T sDx[N1 * N1], sDy[N1 * N1];
    static_assert(HV == 1 || (JVP && !EV), "two halves: the linear operator's dot pass");
    // HV = 2: 512 threads, the second half joins for the dot pass only
    const bool lead = HV == 1 || threadIdx.x < 256;
    const int tid = HV == 2 ? (int)(threadIdx.x & 255) : (int)threadIdx.x;
    const int le = tid / NP;
    const int n = tid - le * NP;
    const int i = n % N1, j = n / N1;
    const int e = tile * EPB + le;
    const bool node = (tid < NT) && (e < a.K);
    const bool active = lead && node;
    const size_t plane = (size_t)a.K * NP;
    const unsigned idx = (unsigned)e * NP + n;
    const T gm1 = a.gamma - T(1);
    if (lead && tid < N1 * N1) {
        sDx[tid] = -a.rhx * a.D[tid];
        sDy[tid] = -a.rhy * a.D[tid];
    }
    // block-uniform plane pointers; the residual reads the state as stored,
    // or its FP64 copy (Q = double with FP32 storage)
    const Q *qin = (const Q *)(std::is_same<Q, S>::value ? (const void *)a.q : (const void *)a.q64);
    const Q *src[4], *vin[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        // lin: u, v, H planes (the fourth unused)
        src[c] = (JVP ? (const Q *)(const void *)a.lin : qin) + c * plane;
        vin[c] = JVP ? (const Q *)(const void *)a.v + c * plane : src[c];
    }

    T sc = T(1);
    if (a.vscale) sc = (T)(*a.vscale);
    // augmented entries of the output: (y_2, ..., y_p, 0), scaled
    if (a.naug > 0 && first && lead && tid == 0) {
        for (int k = 0; k < a.naug; ++k)
            a.otail[k] = (k + 1 < a.naug) ? (S)(sc * (T)a.vtail[k + 1]) : S(0);
    }

    const int ex = e % a.nx, ey = e / a.nx;
    const S *lamx = a.lin + 3 * plane, *lamy = lamx + (size_t)a.K * N1;
    T q[4], u[4], fx[4], fy[4];
    if (active) {
        if (JVP) {
#pragma unroll
            for (int c = 0; c < 3; ++c) q[c] = ld32(src[c], idx);
#pragma unroll
            for (int c = 0; c < 4; ++c) u[c] = ld32(vin[c], idx);
            euler_jac_lin(q, u, gm1, fx, fy);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) q[c] = u[c] = ld32(src[c], idx);
            euler_flux(q, gm1, fx, fy);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) q[c] = u[c] = fx[c] = fy[c] = T(0);
    }
    T res[4] = {T(0), T(0), T(0), T(0)};
    if constexpr (EV) {
        // Entropy viscosity: the flux becomes F - nu g, g the central gradient
        // of the differentiated field v (u here), g_d = (2/h_d) D_d v +
        // (2/h_d)(1/w_0) n_d ({{v}} - v^-) on the faces along d.  g at the
        // node comes from the element's v staged in LDS; g at the neighbour's
        // matching face node from that neighbour's row of nodes along the
        // normal and the shared face's mean.
        __shared__ T sV[4][NT];
        if (lead && tid < NT) {
#pragma unroll
            for (int c = 0; c < 4; ++c) sV[c][tid] = u[c];
        }
        const bool onx = active && (i == 0 || i == P), ony = active && (j == 0 || j == P);
        const int sx = (i == P) ? 1 : -1, sy = (j == P) ? 1 : -1;
        int exn = ex + sx, eyn = ey + sy;
        exn = exn < 0 ? a.nx - 1 : (exn >= a.nx ? 0 : exn);
        eyn = eyn < 0 ? a.ny - 1 : (eyn >= a.ny ? 0 : eyn);
        const int enx = ey * a.nx + exn, eny = eyn * a.nx + ex;
        const unsigned nix = (unsigned)enx * NP + j * N1 + (P - i);
        const unsigned niy = (unsigned)eny * NP + (P - j) * N1 + i;
        T unx[4], fnx[4], uny[4], fny[4], lx = T(0), ly = T(0);
        if (onx) {
            T qn[4];
            if (JVP) {
#pragma unroll
                for (int c = 0; c < 3; ++c) qn[c] = ld32(src[c], nix);
#pragma unroll
                for (int c = 0; c < 4; ++c) unx[c] = ld32(vin[c], nix);
                euler_jac_lin_dir<T, 0>(qn, unx, gm1, fnx);
                lx = ld32(lamx, (unsigned)(sx > 0 ? e : enx) * N1 + j);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) qn[c] = unx[c] = ld32(src[c], nix);
                euler_flux_dir<T, 0>(qn, gm1, fnx);
                lx = fmax(euler_speed<T, 0>(q, a.gamma), euler_speed<T, 0>(qn, a.gamma));
            }
        }
        const bool wy = ony && a.ywall && ((sy < 0 && ey == 0) || (sy > 0 && ey == a.ny - 1));
        if (ony) {
            T qn[4];
            if (wy) {
                // no-slip wall: the mirror state
                if (JVP) {
                    qn[0] = -q[0];
                    qn[1] = -q[1];
                    qn[2] = q[2];
                    wall_mirror(u, uny);
                    euler_jac_lin_dir<T, 1>(qn, uny, gm1, fny);
                    ly = wall_speed_lin(q, gm1);
                } else {
                    wall_mirror(q, qn);
                    wall_mirror(q, uny);
                    euler_flux_dir<T, 1>(qn, gm1, fny);
                    ly = euler_speed<T, 1>(q, a.gamma);
                }
            } else if (JVP) {
#pragma unroll
                for (int c = 0; c < 3; ++c) qn[c] = ld32(src[c], niy);
#pragma unroll
                for (int c = 0; c < 4; ++c) uny[c] = ld32(vin[c], niy);
                euler_jac_lin_dir<T, 1>(qn, uny, gm1, fny);
                ly = ld32(lamy, (unsigned)(sy > 0 ? e : eny) * N1 + i);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) qn[c] = uny[c] = ld32(src[c], niy);
                euler_flux_dir<T, 1>(qn, gm1, fny);
                ly = fmax(euler_speed<T, 1>(q, a.gamma), euler_speed<T, 1>(qn, a.gamma));
            }
        }
        __syncthreads();
        if (active) {
            const int base = le * NP;
            const T nuv = ld32(a.nu, idx);
            T gx[4] = {T(0), T(0), T(0), T(0)}, gy[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int l = 0; l < N1; ++l) {
                const T dx = sDx[i * N1 + l], dy = sDy[j * N1 + l];  // -(2/h) D
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    gx[c] = fma(-dx, sV[c][base + j * N1 + l], gx[c]);
                    gy[c] = fma(-dy, sV[c][base + l * N1 + i], gy[c]);
                }
            }
            if (onx) {
                const T cf = a.rhx * a.lift * T(sx);
#pragma unroll
                for (int c = 0; c < 4; ++c) gx[c] += cf * (T(0.5) * (u[c] + unx[c]) - u[c]);
                // the neighbour's node: index P - i along x, outward normal -sx
                const T nun = ld32(a.nu, nix);
                const unsigned row = (unsigned)enx * NP + j * N1;
                const int an = P - i;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    T g = T(0);
#pragma unroll
                    for (int l = 0; l < N1; ++l) g = fma(-sDx[an * N1 + l], ld32(vin[c], row + l), g);
                    g -= cf * (T(0.5) * (unx[c] + u[c]) - unx[c]);
                    fnx[c] -= nun * g;
                }
            }
            if (wy) {
                // wall: v** = (v + M v)/2; the mirror's diffusive flux is
                // -M (nu g), so the face flux is the interior one for the
                // momenta and zero for density and energy
                const T cf = a.rhy * a.lift * T(sy);
#pragma unroll
                for (int c = 0; c < 4; ++c) gy[c] += cf * (T(0.5) * (u[c] + uny[c]) - u[c]);
                fny[0] += nuv * gy[0];
                fny[1] -= nuv * gy[1];
                fny[2] -= nuv * gy[2];
                fny[3] += nuv * gy[3];
            } else if (ony) {
                const T cf = a.rhy * a.lift * T(sy);
#pragma unroll
                for (int c = 0; c < 4; ++c) gy[c] += cf * (T(0.5) * (u[c] + uny[c]) - u[c]);
                const T nun = ld32(a.nu, niy);
                const unsigned col = (unsigned)eny * NP + i;
                const int an = P - j;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    T g = T(0);
#pragma unroll
                    for (int l = 0; l < N1; ++l)
                        g = fma(-sDy[an * N1 + l], ld32(vin[c], col + l * N1), g);
                    g -= cf * (T(0.5) * (uny[c] + u[c]) - uny[c]);
                    fny[c] -= nun * g;
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                fx[c] -= nuv * gx[c];
                fy[c] -= nuv * gy[c];
            }
        }
        if (lead && tid < NT) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                sF[c][tid] = fx[c];
                sF[4 + c][tid] = fy[c];
            }
        }
        // res -= (2/h)(1/w_0) [ s (F_n - F)/2 + lam (u - u_n)/2 ]
        if (onx) {
            const T cf = a.rhx * a.lift;
            const T ca = cf * T(0.5) * T(sx), cb = cf * T(0.5) * lx;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                res[c] = fma(-cb, u[c] - unx[c], fma(-ca, fnx[c] - fx[c], res[c]));
        }
        if (ony) {
            const T cf = a.rhy * a.lift;
            const T ca = cf * T(0.5) * T(sy), cb = cf * T(0.5) * ly;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                res[c] = fma(-cb, u[c] - uny[c], fma(-ca, fny[c] - fy[c], res[c]));
        }
    } else {
        if (lead && tid < NT) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                sF[c][tid] = fx[c];
                sF[4 + c][tid] = fy[c];
            }
        }

        if (active && (i == 0 || i == P)) {
            const int s = (i == P) ? 1 : -1;
            int exn = ex + s;
            exn = exn < 0 ? a.nx - 1 : (exn >= a.nx ? 0 : exn);
            const int en = ey * a.nx + exn;
            const unsigned nidx = (unsigned)en * NP + j * N1 + (P - i);
            T qn[4], un[4], fn[4], lam;
            if (JVP) {
#pragma unroll
                for (int c = 0; c < 3; ++c) qn[c] = ld32(src[c], nidx);
#pragma unroll
                for (int c = 0; c < 4; ++c) un[c] = ld32(vin[c], nidx);
                euler_jac_lin_dir<T, 0>(qn, un, gm1, fn);
                lam = ld32(lamx, (unsigned)(s > 0 ? e : en) * N1 + j);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) qn[c] = un[c] = ld32(src[c], nidx);
                euler_flux_dir<T, 0>(qn, gm1, fn);
                lam = fmax(euler_speed<T, 0>(q, a.gamma), euler_speed<T, 0>(qn, a.gamma));
            }
            // res -= (2/h)(1/w_0) [ s (F_n - F)/2 + lam (u - u_n)/2 ]
            const T cf = a.rhx * a.lift;
            const T ca = cf * T(0.5) * T(s), cb = cf * T(0.5) * lam;
#pragma unroll
            for (int c = 0; c < 4; ++c) res[c] = fma(-cb, u[c] - un[c], fma(-ca, fn[c] - fx[c], res[c]));
        }
        if (active && (j == 0 || j == P)) {
            const int s = (j == P) ? 1 : -1;
            int eyn = ey + s;
            eyn = eyn < 0 ? a.ny - 1 : (eyn >= a.ny ? 0 : eyn);
            const int en = eyn * a.nx + ex;
            const unsigned nidx = (unsigned)en * NP + (P - j) * N1 + i;
            const bool wall = a.ywall && ((s < 0 && ey == 0) || (s > 0 && ey == a.ny - 1));
            T qn[4], un[4], fn[4], lam;
            if (wall) {
                // no-slip wall: the mirror state
                if (JVP) {
                    qn[0] = -q[0];
                    qn[1] = -q[1];
                    qn[2] = q[2];
                    wall_mirror(u, un);
                    euler_jac_lin_dir<T, 1>(qn, un, gm1, fn);
                    lam = wall_speed_lin(q, gm1);
                } else {
                    wall_mirror(q, qn);
                    wall_mirror(q, un);
                    euler_flux_dir<T, 1>(qn, gm1, fn);
                    lam = euler_speed<T, 1>(q, a.gamma);
                }
            } else if (JVP) {
#pragma unroll
                for (int c = 0; c < 3; ++c) qn[c] = ld32(src[c], nidx);
#pragma unroll
                for (int c = 0; c < 4; ++c) un[c] = ld32(vin[c], nidx);
                euler_jac_lin_dir<T, 1>(qn, un, gm1, fn);
                lam = ld32(lamy, (unsigned)(s > 0 ? e : en) * N1 + i);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) qn[c] = un[c] = ld32(src[c], nidx);
                euler_flux_dir<T, 1>(qn, gm1, fn);
                lam = fmax(euler_speed<T, 1>(q, a.gamma), euler_speed<T, 1>(qn, a.gamma));
            }
            const T cf = a.rhy * a.lift;
            const T ca = cf * T(0.5) * T(s), cb = cf * T(0.5) * lam;
#pragma unroll
            for (int c = 0; c < 4; ++c) res[c] = fma(-cb, u[c] - un[c], fma(-ca, fn[c] - fy[c], res[c]));
        }
    }
    // augmented block: + eta sum_k y_k b_{p+1-k}
    if (active) {
        for (int k = 0; k < a.naug; ++k) {
            const S *b = a.aug[k];
            if (!b) continue;
            const T yk = (T)a.eta * a.vtail[k];
#pragma unroll
            for (int c = 0; c < 4; ++c) res[c] = fma(yk, ld32(b + c * plane, idx), res[c]);
        }
    }
    __syncthreads();

    T wv[4];
    if (active) {
        const int base = le * NP;
#pragma unroll
        for (int l = 0; l < N1; ++l) {
            const T dx = sDx[i * N1 + l];
            const T dy = sDy[j * N1 + l];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                res[c] = fma(dy, sF[4 + c][base + l * N1 + i], fma(dx, sF[c][base + j * N1 + l], res[c]));
        }
        S *out[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) out[c] = a.out + c * plane;
        // the dot pass sees the output as stored
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const S ws = (S)(sc * res[c]);
            wv[c] = (T)ws;
            st32(out[c], idx, ws);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) wv[c] = T(0);
    }
    if constexpr (HV == 2) {
        // the second half takes the node's input and output from the first
        __shared__ double sXW[8][256];
        if (lead) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                sXW[c][tid] = u[c];
                sXW[4 + c][tid] = wv[c];
            }
        }
        __syncthreads();
        if (!lead) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                u[c] = sXW[c][tid];
                wv[c] = sXW[4 + c][tid];
            }
        }
        op_dots2<S, 4, 4, 8, 2>(a, node, idx, plane, u, wv, tile, first);
    } else if (JVP && a.dots) {
        op_dots2<S, 4, 4, 8>(a, active, idx, plane, u, wv, tile, first);
    }
}

// ---- entropy viscosity (2D Euler) ---------------------------------------------
// Section 3.2, "Artificial viscosity": S = rho/(g-1) log(p / rho^g), entropy
// flux u S; Res = (S(q) - S(q_prev))/dt + (div(uS)(q) + div(uS)(q_prev))/2 at
// the nodes (element-local derivative); per element nu_E = c_E h^2 max(max|Res|,
// max|[[uS . n]]| / h), nu_max = c_max h max(|u . e_d| + a), nu_e = min of the
// two (h = sqrt(hx^2 + hy^2)/p); the nodal nu is the bilinear interpolant of
// the vertex averages of nu_e.

__device__ __forceinline__ void ev_entropy(const double *q, double gamma, double *S, double *fx,
                                           double *fy) {
    const double rho = q[0], u = q[1] / rho, v = q[2] / rho;
    const double pr = (gamma - 1.0) * (q[3] - 0.5 * rho * (u * u + v * v));
    *S = rho / (gamma - 1.0) * log(pr / pow(rho, gamma));
    *fx = u * *S;
    *fy = v * *S;
}

template <int P>
__global__ __launch_bounds__(256) void ev_element_kernel(EvParams ep, const double *q,
                                                         const double *qp, double *nue) {
    constexpr int N1 = P + 1, NP = N1 * N1, EPB = 256 / NP, NT = EPB * NP;
    __shared__ double sF[4][NT];   // uS_x(q), uS_y(q), uS_x(q_prev), uS_y(q_prev)
    __shared__ double sR[3][NT];   // |Res|, face jumps, wave speed
    const int tid = threadIdx.x;
    const int le = tid / NP, n = tid - le * NP;
    const int i = n % N1, j = n / N1;
    const int e = blockIdx.x * EPB + le;
    const bool active = (tid < NT) && (e < ep.K);
    const size_t plane = (size_t)ep.K * NP;
    const size_t idx = (size_t)e * NP + n;
    double qq[4], qo[4], S = 0.0, So = 0.0, fx = 0.0, fy = 0.0, fxo = 0.0, fyo = 0.0;
    if (active) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            qq[c] = q[c * plane + idx];
            qo[c] = qp[c * plane + idx];
        }
        ev_entropy(qq, ep.gamma, &S, &fx, &fy);
        ev_entropy(qo, ep.gamma, &So, &fxo, &fyo);
    }
    if (tid < NT) {
        sF[0][tid] = fx;
        sF[1][tid] = fy;
        sF[2][tid] = fxo;
        sF[3][tid] = fyo;
    }
    __syncthreads();
    double ares = 0.0, jmax = 0.0, lam = 0.0;
    if (active) {
        const int base = le * NP;
        double div[2] = {0.0, 0.0};
#pragma unroll
        for (int st = 0; st < 2; ++st) {
#pragma unroll
            for (int l = 0; l < N1; ++l)
                div[st] += ep.rhx * ep.D[i * N1 + l] * sF[2 * st][base + j * N1 + l];
#pragma unroll
            for (int l = 0; l < N1; ++l)
                div[st] += ep.rhy * ep.D[j * N1 + l] * sF[2 * st + 1][base + l * N1 + i];
        }
        ares = fabs((S - So) / ep.dt + 0.5 * (div[0] + div[1]));
        const double u = qq[1] / qq[0], v = qq[2] / qq[0];
        const double pr = (ep.gamma - 1.0) * (qq[3] - 0.5 * qq[0] * (u * u + v * v));
        const double a = sqrt(ep.gamma * pr / qq[0]);
        lam = fmax(fabs(u) + a, fabs(v) + a);
        const int ex = e % ep.nx, ey = e / ep.nx;
        if (i == 0 || i == P) {
            const int s = (i == P) ? 1 : -1;
            const int exn = (ex + s + ep.nx) % ep.nx;
            const size_t nidx = (size_t)(ey * ep.nx + exn) * NP + j * N1 + (P - i);
            double qn[4], Sn, fxn, fyn;
#pragma unroll
            for (int c = 0; c < 4; ++c) qn[c] = q[c * plane + nidx];
            ev_entropy(qn, ep.gamma, &Sn, &fxn, &fyn);
            jmax = fmax(jmax, fabs(fx - fxn));
        }
        if (j == 0 || j == P) {
            const int s = (j == P) ? 1 : -1;
            if (ep.ywall && ((s < 0 && ey == 0) || (s > 0 && ey == ep.ny - 1))) {
                // wall: the mirror carries -v S
                jmax = fmax(jmax, fabs(fy - (-fy)));
            } else {
                const int eyn = (ey + s + ep.ny) % ep.ny;
                const size_t nidx = (size_t)(eyn * ep.nx + ex) * NP + (P - j) * N1 + i;
                double qn[4], Sn, fxn, fyn;
#pragma unroll
                for (int c = 0; c < 4; ++c) qn[c] = q[c * plane + nidx];
                ev_entropy(qn, ep.gamma, &Sn, &fxn, &fyn);
                jmax = fmax(jmax, fabs(fy - fyn));
            }
        }
    }
    if (tid < NT) {
        sR[0][tid] = ares;
        sR[1][tid] = jmax;
        sR[2][tid] = lam;
    }
    __syncthreads();
    if (active && n == 0) {
        const int base = le * NP;
        double rm = 0.0, jm = 0.0, lm = 0.0;
        for (int k = 0; k < NP; ++k) {
            rm = fmax(rm, sR[0][base + k]);
            jm = fmax(jm, sR[1][base + k]);
            lm = fmax(lm, sR[2][base + k]);
        }
        const double nu_e = ep.ce * ep.he * ep.he * fmax(rm, jm / ep.he);
        const double nu_max = ep.cmax * ep.he * lm;
        nue[e] = fmin(nu_max, nu_e);
    }
}

template <int P, typename T>
__global__ __launch_bounds__(256) void ev_smooth_kernel(EvParams ep, const double *nue, T *nu) {
    constexpr int N1 = P + 1, NP = N1 * N1;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)ep.K * NP) return;
    const int e = (int)(t / NP), n = (int)(t - (size_t)e * NP);
    const int i = n % N1, j = n / N1;
    const int nx = ep.nx, ny = ep.ny;
    const int ex = e % nx, ey = e / nx;
    // vertex (vx, vy) is the lower-left corner of element (vx, vy); with walls
    // the vertices on y0 and y1 average the two elements they belong to
    const bool walls = ep.ywall != 0;
    auto vert = [&](int vx, int vy) {
        const int xm = (vx + nx - 1) % nx;
        if (walls && (vy == 0 || vy == ny)) {
            const int ew = vy == 0 ? 0 : ny - 1;
            return 0.5 * (nue[ew * nx + vx] + nue[ew * nx + xm]);
        }
        const int ym = (vy + ny - 1) % ny;
        return 0.25 * ((nue[vy * nx + vx] + nue[vy * nx + xm]) +
                       (nue[ym * nx + vx] + nue[ym * nx + xm]));
    };
    const int xp = (ex + 1) % nx, yp = walls ? ey + 1 : (ey + 1) % ny;
    const double v00 = vert(ex, ey), v10 = vert(xp, ey), v01 = vert(ex, yp), v11 = vert(xp, yp);
    const double r = 0.5 * (ep.xi[i] + 1.0), s = 0.5 * (ep.xi[j] + 1.0);
    nu[t] = (T)((1.0 - r) * (1.0 - s) * v00 + r * (1.0 - s) * v10 + (1.0 - r) * s * v01 +
                r * s * v11);
}

// ---- Euler 3D operator ------------------------------------------------------
// q = (rho, m, n, l, E) with (m, n, l) = rho (u, v, w); the system of
// Section 3.2 written for three velocity components (the extruded problem of
// Section 5.2).  Frozen fields of the linear operator: planes u, v, w, H, then
// the Rusanov speed of every x, y and z face node (N1^2 per element each).

// Physical flux along DIR.
template <typename T, int DIR>
__device__ __forceinline__ void euler3_flux_dir(const T *q, T gm1, T *f) {
    const T ir = recip(q[0]);
    const T u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
    const T p = gm1 * (q[4] - T(0.5) * (q[1] * u + q[2] * v + q[3] * w));
    const T un = DIR == 0 ? u : (DIR == 1 ? v : w);
    f[0] = q[1 + DIR];
    f[1] = q[1] * un + (DIR == 0 ? p : T(0));
    f[2] = q[2] * un + (DIR == 1 ? p : T(0));
    f[3] = q[3] * un + (DIR == 2 ? p : T(0));
    f[4] = (q[4] + p) * un;
}

template <typename T, int DIR>
__device__ __forceinline__ T euler3_speed(const T *q, T gamma) {
    const T ir = recip(q[0]);
    const T u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
    const T p = (gamma - T(1)) * (q[4] - T(0.5) * (q[1] * u + q[2] * v + q[3] * w));
    return fabs(DIR == 0 ? u : (DIR == 1 ? v : w)) + root(gamma * p * ir);
}

// Directional derivative of the flux along DIR from the frozen fields
// z = (u, v, w, H): with al = dm - u drho, be = dn - v drho, ga = dl - w drho,
// dp = (g-1)(dE - u al - v be - w ga - |u|^2/2 drho),
//   dF_x = (dm, u (dm + al) + dp, u dn + v al, u dl + w al, u (dE + dp) + H al),
//   dF_y = (dn, u dn + v al, v (dn + be) + dp, v dl + w be, v (dE + dp) + H be),
//   dF_z = (dl, u dl + w al, v dl + w be, w (dl + ga) + dp, w (dE + dp) + H ga).
template <typename T, int DIR>
__device__ __forceinline__ void euler3_jac_lin_dir(const T *z, const T *d, T gm1, T *f) {
    const T u = z[0], v = z[1], w = z[2], H = z[3];
    const T al = fma(-u, d[0], d[1]), be = fma(-v, d[0], d[2]), ga = fma(-w, d[0], d[3]);
    const T k = T(0.5) * fma(u, u, fma(v, v, w * w));
    const T dp = gm1 * fma(-k, d[0], fma(-w, ga, fma(-v, be, fma(-u, al, d[4]))));
    const T ep = d[4] + dp;
    if (DIR == 0) {
        f[0] = d[1];
        f[1] = fma(u, d[1] + al, dp);
        f[2] = fma(u, d[2], v * al);
        f[3] = fma(u, d[3], w * al);
        f[4] = fma(u, ep, H * al);
    } else if (DIR == 1) {
        f[0] = d[2];
        f[1] = fma(u, d[2], v * al);
        f[2] = fma(v, d[2] + be, dp);
        f[3] = fma(v, d[3], w * be);
        f[4] = fma(v, ep, H * be);
    } else {
        f[0] = d[3];
        f[1] = fma(u, d[3], w * al);
        f[2] = fma(v, d[3], w * be);
        f[3] = fma(w, d[3] + ga, dp);
        f[4] = fma(w, ep, H * ga);
    }
}

template <int P, typename Q, typename St>
__global__ __launch_bounds__(256) void euler3_lin_prepare(const Q *q, St *lin, int K, int nx,
                                                          int ny, int nz, double gamma) {
    using T = double;  // arithmetic; St is the storage type
    constexpr int N1 = P + 1, NP = N1 * N1 * N1, NF = N1 * N1;
    const size_t plane = (size_t)K * NP;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= plane) return;
    const int e = (int)(t / NP), n = (int)(t - (size_t)e * NP);
    const int i = n % N1, j = (n / N1) % N1, k = n / NF;
    T qq[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) qq[c] = q[c * plane + t];
    const T ir = recip(qq[0]);
    const T u = qq[1] * ir, v = qq[2] * ir, w = qq[3] * ir;
    const T p = (gamma - T(1)) * (qq[4] - T(0.5) * (qq[1] * u + qq[2] * v + qq[3] * w));
    lin[t] = (St)u;
    lin[plane + t] = (St)v;
    lin[2 * plane + t] = (St)w;
    lin[3 * plane + t] = (St)((qq[4] + p) * ir);
    St *lamx = lin + 4 * plane, *lamy = lamx + (size_t)K * NF, *lamz = lamy + (size_t)K * NF;
    const int ex = e % nx, ey = (e / nx) % ny, ez = e / (nx * ny);
    T qn[5];
    if (i == P) {
        const int en = (ez * ny + ey) * nx + (ex + 1 == nx ? 0 : ex + 1);
        const size_t nidx = (size_t)en * NP + (k * N1 + j) * N1;
#pragma unroll
        for (int c = 0; c < 5; ++c) qn[c] = q[c * plane + nidx];
        lamx[(size_t)e * NF + k * N1 + j] = (St)fmax(euler3_speed<T, 0>(qq, gamma), euler3_speed<T, 0>(qn, gamma));
    }
    if (j == P) {
        const int en = (ez * ny + (ey + 1 == ny ? 0 : ey + 1)) * nx + ex;
        const size_t nidx = (size_t)en * NP + (k * N1) * N1 + i;
#pragma unroll
        for (int c = 0; c < 5; ++c) qn[c] = q[c * plane + nidx];
        lamy[(size_t)e * NF + k * N1 + i] = (St)fmax(euler3_speed<T, 1>(qq, gamma), euler3_speed<T, 1>(qn, gamma));
    }
    if (k == P) {
        const int en = ((ez + 1 == nz ? 0 : ez + 1) * ny + ey) * nx + ex;
        const size_t nidx = (size_t)en * NP + j * N1 + i;
#pragma unroll
        for (int c = 0; c < 5; ++c) qn[c] = q[c * plane + nidx];
        lamz[(size_t)e * NF + j * N1 + i] = (St)fmax(euler3_speed<T, 2>(qq, gamma), euler3_speed<T, 2>(qn, gamma));
    }
}

// Block size of the 3D operator: 256 threads (floor(256/Np) elements) up to
// p = 5, one element per 384-thread block at p = 6 (343 nodes).
template <int P>
struct E3Shape {
    static constexpr int N1 = P + 1, NP = N1 * N1 * N1;
    static constexpr int BS = NP > 256 ? 384 : 256;
    static constexpr int EPB = BS / NP, NT = EPB * NP, NW = BS / 64;
};

// Face term of the node on the DIR face on side s: the neighbour's trace, its
// flux and lambda; res -= (2/h)(1/w_0) [ s (F_n - F)/2 + lam (u - u_n)/2 ].
template <int P, typename St, bool JVP, int DIR, typename Q>
__device__ __forceinline__ void euler3_face(const OpArgs<St> &a, const Q *const *src,
                                            const Q *const *vin, const St *lamd, int e, int en,
                                            unsigned nidx, int fidx, int s, double rh,
                                            const double *q, const double *u, const double *fd,
                                            double gm1, double *res) {
    using T = double;
    T qn[5], un[5], fn[5], lam;
    if (JVP) {
#pragma unroll
        for (int c = 0; c < 4; ++c) qn[c] = ld32(src[c], nidx);
#pragma unroll
        for (int c = 0; c < 5; ++c) un[c] = ld32(vin[c], nidx);
        euler3_jac_lin_dir<T, DIR>(qn, un, gm1, fn);
        constexpr int NF = (P + 1) * (P + 1);
        lam = ld32(lamd, (unsigned)(s > 0 ? e : en) * NF + fidx);
    } else {
#pragma unroll
        for (int c = 0; c < 5; ++c) qn[c] = un[c] = ld32(src[c], nidx);
        euler3_flux_dir<T, DIR>(qn, gm1, fn);
        lam = fmax(euler3_speed<T, DIR>(q, a.gamma), euler3_speed<T, DIR>(qn, a.gamma));
    }
    const T cf = rh * a.lift;
    const T ca = cf * T(0.5) * T(s), cb = cf * T(0.5) * lam;
#pragma unroll
    for (int c = 0; c < 5; ++c) res[c] = fma(-cb, u[c] - un[c], fma(-ca, fn[c] - fd[c], res[c]));
}

template <int P, typename St, bool JVP, typename Q = St>
__device__ __forceinline__ void euler3_op_body(const OpArgs<St> &a, int tile, bool first) {
    using T = double;  // arithmetic; St is the storage type
    static_assert(!JVP || std::is_same<Q, St>::value, "the linear operator reads stored vectors");
    using S = E3Shape<P>;
    constexpr int N1 = S::N1, NP = S::NP, NF = N1 * N1, EPB = S::EPB, NT = S::NT;
    __shared__ T sF[15][NT];
    __shared__ T sDx[N1 * N1], sDy[N1 * N1], sDz[N1 * N1];
    const int tid = threadIdx.x;
    const int le = tid / NP;
    const int n = tid - le * NP;
    const int i = n % N1, j = (n / N1) % N1, k = n / NF;
    // the linear operator's tiles run through the elements column by column (z
    // fastest): an element's z neighbours are the tiles next to it and its x
    // neighbours nz tiles away, so their face traces are read while they are
    // still in the XCD's L2 (measured on the 80x80x8 p = 6 run: the operator
    // 5.07 -> 4.98 ms and the update sweep after it 4.43 -> 4.21 ms, which
    // reads what the operator just wrote).  The residual keeps the plain
    // order (the column order made it read 1.45x its bytes instead of 1.26x).
    const int nxy = a.nx * a.ny, nz = a.K / nxy;
    const int el = tile * EPB + le;
    const int e = JVP ? (el % nz) * nxy + el / nz : el;
    const bool active = (tid < NT) && (el < a.K);
    const size_t plane = (size_t)a.K * NP;
    const unsigned idx = (unsigned)e * NP + n;
    const T gm1 = a.gamma - T(1);
    if (tid < N1 * N1) {
        sDx[tid] = -a.rhx * a.D[tid];
        sDy[tid] = -a.rhy * a.D[tid];
        sDz[tid] = -a.rhz * a.D[tid];
    }
    // the residual reads the state as stored, or its FP64 copy (Q = double)
    const Q *qin =
        (const Q *)(std::is_same<Q, St>::value ? (const void *)a.q : (const void *)a.q64);
    const Q *src[5], *vin[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        // lin: u, v, w, H planes (the fifth unused)
        src[c] = (JVP ? (const Q *)(const void *)a.lin : qin) + c * plane;
        vin[c] = JVP ? (const Q *)(const void *)a.v + c * plane : src[c];
    }
    T sc = T(1);
    if (a.vscale) sc = (T)(*a.vscale);
    if (a.naug > 0 && first && tid == 0) {
        for (int kk = 0; kk < a.naug; ++kk)
            a.otail[kk] = (kk + 1 < a.naug) ? (St)(sc * (T)a.vtail[kk + 1]) : St(0);
    }
    const int ex = e % a.nx, ey = (e / a.nx) % a.ny, ez = e / nxy;
    const St *lamx = a.lin + 4 * plane, *lamy = lamx + (size_t)a.K * NF,
             *lamz = lamy + (size_t)a.K * NF;
    T q[5], u[5], fx[5], fy[5], fz[5];
    if (active) {
        if (JVP) {
#pragma unroll
            for (int c = 0; c < 4; ++c) q[c] = ld32(src[c], idx);
            q[4] = T(0);
#pragma unroll
            for (int c = 0; c < 5; ++c) u[c] = ld32(vin[c], idx);
            euler3_jac_lin_dir<T, 0>(q, u, gm1, fx);
            euler3_jac_lin_dir<T, 1>(q, u, gm1, fy);
            euler3_jac_lin_dir<T, 2>(q, u, gm1, fz);
        } else {
#pragma unroll
            for (int c = 0; c < 5; ++c) q[c] = u[c] = ld32(src[c], idx);
            euler3_flux_dir<T, 0>(q, gm1, fx);
            euler3_flux_dir<T, 1>(q, gm1, fy);
            euler3_flux_dir<T, 2>(q, gm1, fz);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 5; ++c) q[c] = u[c] = fx[c] = fy[c] = fz[c] = T(0);
    }
    if (tid < NT) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            sF[c][tid] = fx[c];
            sF[5 + c][tid] = fy[c];
            sF[10 + c][tid] = fz[c];
        }
    }

    T res[5] = {T(0), T(0), T(0), T(0), T(0)};
    if (active && (i == 0 || i == P)) {
        const int s = (i == P) ? 1 : -1;
        int exn = ex + s;
        exn = exn < 0 ? a.nx - 1 : (exn >= a.nx ? 0 : exn);
        const int en = ez * nxy + ey * a.nx + exn;
        const unsigned nidx = (unsigned)en * NP + (k * N1 + j) * N1 + (P - i);
        euler3_face<P, St, JVP, 0, Q>(a, src, vin, lamx, e, en, nidx, k * N1 + j, s, a.rhx, q, u, fx,
                                  gm1, res);
    }
    if (active && (j == 0 || j == P)) {
        const int s = (j == P) ? 1 : -1;
        int eyn = ey + s;
        eyn = eyn < 0 ? a.ny - 1 : (eyn >= a.ny ? 0 : eyn);
        const int en = ez * nxy + eyn * a.nx + ex;
        const unsigned nidx = (unsigned)en * NP + (k * N1 + (P - j)) * N1 + i;
        euler3_face<P, St, JVP, 1, Q>(a, src, vin, lamy, e, en, nidx, k * N1 + i, s, a.rhy, q, u, fy,
                                  gm1, res);
    }
    if (active && (k == 0 || k == P)) {
        const int s = (k == P) ? 1 : -1;
        int ezn = ez + s;
        ezn = ezn < 0 ? nz - 1 : (ezn >= nz ? 0 : ezn);
        const int en = ezn * nxy + ey * a.nx + ex;
        const unsigned nidx = (unsigned)en * NP + ((P - k) * N1 + j) * N1 + i;
        euler3_face<P, St, JVP, 2, Q>(a, src, vin, lamz, e, en, nidx, j * N1 + i, s, a.rhz, q, u, fz,
                                  gm1, res);
    }
    if (active) {
        for (int kk = 0; kk < a.naug; ++kk) {
            const St *b = a.aug[kk];
            if (!b) continue;
            const T yk = (T)a.eta * a.vtail[kk];
#pragma unroll
            for (int c = 0; c < 5; ++c) res[c] = fma(yk, ld32(b + c * plane, idx), res[c]);
        }
    }
    __syncthreads();

    T wv[5];
    if (active) {
        const int base = le * NP;
#pragma unroll
        for (int l = 0; l < N1; ++l) {
            const T dx = sDx[i * N1 + l], dy = sDy[j * N1 + l], dz = sDz[k * N1 + l];
            const int nxl = base + (k * N1 + j) * N1 + l;
            const int nyl = base + (k * N1 + l) * N1 + i;
            const int nzl = base + (l * N1 + j) * N1 + i;
#pragma unroll
            for (int c = 0; c < 5; ++c)
                res[c] = fma(dz, sF[10 + c][nzl],
                             fma(dy, sF[5 + c][nyl], fma(dx, sF[c][nxl], res[c])));
        }
        // the dot pass sees the output as stored
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const St ws = (St)(sc * res[c]);
            wv[c] = (T)ws;
            st32(a.out + c * plane, idx, ws);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 5; ++c) wv[c] = T(0);
    }
    if (JVP && a.dots) op_dots2<St, 5, S::NW, 8>(a, active, idx, plane, u, wv, tile, first);
}

template <int P, typename T, bool JVP>
__global__ __launch_bounds__(E3Shape<P>::BS) void euler3_op(OpArgs<T> a) {
    euler3_op_body<P, T, JVP>(a, xcd_tile(blockIdx.x, gridDim.x), blockIdx.x == 0);
}

// Residual of the FP64 state a.q64 with T storage (FP32-bulk steps).
template <int P, typename T>
__global__ __launch_bounds__(E3Shape<P>::BS) void euler3_op_r64(OpArgs<T> a) {
    euler3_op_body<P, T, false, double>(a, xcd_tile(blockIdx.x, gridDim.x), blockIdx.x == 0);
}

// ---- Burgers 1D operator ----------------------------------------------------
// One thread per LGL node, EPB whole elements per block.  Residual of
// u_t + (u^2/2 - kappa q)_x = s and linear operator of the flux u~ v - kappa q(v)
// (Section 3.1, eqs. gov-burgers1d-gradu, BurgerL, BurgerN), strong form with
// the LGL lift 1/w_0 at the end nodes:
//   convective face flux: Lax-Friedrichs with lambda = max(|u~^-|, |u~^+|), or
//     (residual, ef) the entropy flux n (u^-^2 + u^- u^+ + u^+^2)/6 +
//     pen (u^- - u^+), pen = ef_pen, or ef_pen + max(|u^-|, |u^+|) with
//     ef_local (the face-dependent penalty of Section 5.1's steep gradient);
//   VISC (kappa > 0): the auxiliary q of the differentiated field z (u for the
//     residual, v for the linear operator) is formed in LDS for the block's
//     elements and the two adjacent face nodes of the neighbouring elements:
//     q = (2/h) D z + (2/h)(1/w_0) n (z** - z^-) at the end nodes, with
//     z** = {{z}} - beta [[z]] ([[z]] = z_left - z_right); the flux then gets
//     -kappa q, and the face term kappa (2/h)(1/w_0) n (q** - q^-) with
//     q** = {{q}} + beta [[q]];
//   dirichlet: beyond both ends z^+ = 0 for the convective fluxes, z** = 0 and
//     q** = q^- (no diffusive face term).
template <int P, typename S, bool JVP, bool VISC, typename Q = S>
__device__ __forceinline__ void burgers_op_body(const OpArgs<S> &a, int tile, bool first) {
    using T = double;  // arithmetic; S is the storage type
    static_assert(!JVP || std::is_same<Q, S>::value, "the linear operator reads stored vectors");
    // the state as stored, or (residual, Q = double) its FP64 copy
    const Q *qs = (const Q *)(std::is_same<Q, S>::value ? (const void *)a.q : (const void *)a.q64);
    const Q *vs = (const Q *)(const void *)a.v;
    constexpr int N1 = P + 1, EPB = 256 / N1, NT = EPB * N1;
    // VISC: slots 0 and nact + 1 hold the neighbouring elements (halo)
    constexpr int NS = VISC ? (EPB + 2) * N1 : 1;
    __shared__ T sF[NT];
    __shared__ T sZ[NS];
    __shared__ T sQ[NS];
    const int tid = threadIdx.x;
    const int le = tid / N1;
    const int i = tid - le * N1;
    const int e0 = tile * EPB;
    const int e = e0 + le;
    const bool active = (tid < NT) && (e < a.K);
    const size_t idx = (size_t)e * N1 + i;
    const bool dir = a.dirichlet != 0;

    T sc = T(1);
    if (a.vscale) sc = (T)(*a.vscale);
    if (a.naug > 0 && first && tid == 0) {
        for (int k = 0; k < a.naug; ++k)
            a.otail[k] = (k + 1 < a.naug) ? (S)(sc * (T)a.vtail[k + 1]) : S(0);
    }

    T qv = T(0), uv = T(0), f = T(0);
    // end nodes: the neighbour's trace across the face (zero beyond a
    // Dirichlet end), loaded together with the node's own values
    const bool face = active && (i == 0 || i == P);
    const int s = (i == P) ? 1 : -1;
    bool bnd = false;
    T qn = T(0), un = T(0);
    if (active) {
        qv = qs[idx];
        uv = JVP ? vs[idx] : qv;
        f = JVP ? qv * uv : T(0.5) * qv * qv;
    }
    if (face) {
        int en = e + s;
        bnd = dir && (en < 0 || en >= a.K);
        en = en < 0 ? a.K - 1 : (en >= a.K ? 0 : en);
        const size_t nidx = (size_t)en * N1 + (P - i);
        qn = bnd ? T(0) : qs[nidx];
        un = JVP ? (bnd ? T(0) : vs[nidx]) : qn;
    }
    const int nact = min(EPB, a.K - e0);  // elements of this block
    // neighbours of the block: -1 beyond a Dirichlet end
    int eLh = e0 - 1, eRh = e0 + nact;
    if (eLh < 0) eLh = dir ? -1 : a.K - 1;
    if (eRh >= a.K) eRh = dir ? -1 : 0;
    const Q *zsrc = JVP ? vs : qs;
    T qgrad = T(0);
    if constexpr (VISC) {
        if (active) sZ[(le + 1) * N1 + i] = uv;
        if (tid < N1) sZ[tid] = (eLh >= 0) ? zsrc[(size_t)eLh * N1 + tid] : T(0);
        if (tid >= N1 && tid < 2 * N1)
            sZ[(nact + 1) * N1 + (tid - N1)] =
                (eRh >= 0) ? zsrc[(size_t)eRh * N1 + (tid - N1)] : T(0);
        __syncthreads();
        const T rl = a.rhx * a.lift;
        if (active) {
            const T *z = sZ + (le + 1) * N1;
            T g = T(0);
#pragma unroll
            for (int l = 0; l < N1; ++l) g += a.D[i * N1 + l] * z[l];
            g *= a.rhx;
            if (i == 0) {  // face with the left neighbour
                const bool bnd = dir && e == 0;
                const T zl = sZ[le * N1 + P], zr = z[0];
                const T zs = bnd ? T(0) : T(0.5) * (zl + zr) - a.beta * (zl - zr);
                g -= rl * (zs - zr);
                if (le == 0 && !bnd) {  // q of the left neighbour at this face
                    const T *zh = sZ;
                    T gh = T(0);
#pragma unroll
                    for (int l = 0; l < N1; ++l) gh += a.D[P * N1 + l] * zh[l];
                    sQ[P] = a.rhx * gh + rl * (zs - zl);
                }
            }
            if (i == P) {  // face with the right neighbour
                const bool bnd = dir && e == a.K - 1;
                const T zl = z[P], zr = sZ[(le + 2) * N1];
                const T zs = bnd ? T(0) : T(0.5) * (zl + zr) - a.beta * (zl - zr);
                g += rl * (zs - zl);
                if (le == nact - 1 && !bnd) {  // q of the right neighbour at this face
                    const T *zh = sZ + (nact + 1) * N1;
                    T gh = T(0);
#pragma unroll
                    for (int l = 0; l < N1; ++l) gh += a.D[l] * zh[l];
                    sQ[(nact + 1) * N1] = a.rhx * gh - rl * (zs - zr);
                }
            }
            qgrad = g;
            sQ[(le + 1) * N1 + i] = g;
            f -= a.kappa * g;
        }
    }
    if (tid < NT) sF[tid] = f;
    __syncthreads();

    T res = T(0);
    const int base = le * N1;
    if (active) {
#pragma unroll
        for (int l = 0; l < N1; ++l) res -= a.rhx * a.D[i * N1 + l] * sF[base + l];
    }
    if (face) {
        const T fn = JVP ? qn * un : T(0.5) * qn * qn;
        const T fc = JVP ? qv * uv : T(0.5) * qv * qv;
        if (!JVP && a.ef) {
            const T pen = a.ef_local ? a.ef_pen + fmax(fabs(qv), fabs(qn)) : a.ef_pen;
            const T fs = T(s) * (qv * qv + qv * qn + qn * qn) * T(1.0 / 6.0) + pen * (qv - qn);
            res -= a.rhx * a.lift * (fs - T(s) * fc);
        } else {
            const T lam = fmax(fabs(qv), fabs(qn));
            res -= a.rhx * a.lift * (T(0.5) * T(s) * (fn - fc) + T(0.5) * lam * (uv - un));
        }
        if constexpr (VISC) {
            if (!bnd) {
                // q of the two sides of this face, left and right
                const T qL = (s < 0) ? sQ[le * N1 + P] : qgrad;
                const T qR = (s < 0) ? qgrad : sQ[(le + 2) * N1];
                const T qs = T(0.5) * (qL + qR) + a.beta * (qL - qR);
                res += a.kappa * a.rhx * a.lift * T(s) * (qs - qgrad);
            }
        }
    }
    T wv = T(0);
    if (active) {
        if (!JVP && a.src) res += a.src[idx];
        for (int k = 0; k < a.naug; ++k) {
            const S *b = a.aug[k];
            if (!b) continue;
            res += (T)a.eta * (T)a.vtail[k] * (T)b[idx];
        }
        // the dot pass sees the output as stored
        const S ws = (S)(sc * res);
        wv = (T)ws;
        a.out[idx] = ws;
    }
    if (JVP && a.dots)
        op_dots2<S, 1>(a, active, (unsigned)idx, (size_t)a.K * N1, &uv, &wv, tile, first);
}

template <int P, typename T, bool JVP, bool EV>
__global__ __launch_bounds__(256) void euler_op(OpArgs<T> a) {
    euler_op_body<P, T, JVP, EV>(a, xcd_tile(blockIdx.x, gridDim.x), blockIdx.x == 0);
}

// Residual of the FP64 state a.q64 with T storage (FP32-bulk steps).
template <int P, typename T, bool EV>
__global__ __launch_bounds__(256) void euler_op_r64(OpArgs<T> a) {
    euler_op_body<P, T, false, EV, double>(a, xcd_tile(blockIdx.x, gridDim.x), blockIdx.x == 0);
}

// The linear operator with its dot pass over 512 threads: the second half
// takes half of the basis chunks (grids of a few blocks per CU, where one
// block's chain of chunks sets the launch time).
template <int P, typename T>
__global__ __launch_bounds__(512) void euler_op_halves(OpArgs<T> a) {
    euler_op_body<P, T, true, false, T, 2>(a, xcd_tile(blockIdx.x, gridDim.x), blockIdx.x == 0);
}

template <int P, typename T, bool JVP, bool VISC>
__global__ __launch_bounds__(256) void burgers_op(OpArgs<T> a) {
    burgers_op_body<P, T, JVP, VISC>(a, xcd_tile(blockIdx.x, gridDim.x), blockIdx.x == 0);
}

// Residual of the FP64 state a.q64 with T storage (FP32-bulk steps).
template <int P, typename T, bool VISC>
__global__ __launch_bounds__(256) void burgers_op_r64(OpArgs<T> a) {
    burgers_op_body<P, T, false, VISC, double>(a, xcd_tile(blockIdx.x, gridDim.x),
                                               blockIdx.x == 0);
}

template <int P, typename T, bool JVP, bool EV>
__global__ __launch_bounds__(256) void euler_op_group(const OpArgs<T> *items, const int *bstart,
                                                      int n) {
    const int it = group_item(bstart, n, blockIdx.x);
    const int local = blockIdx.x - bstart[it], G = bstart[it + 1] - bstart[it];
    euler_op_body<P, T, JVP, EV>(items[it], xcd_tile(local, G), local == 0);
}

template <int P, typename T, bool JVP, bool VISC>
__global__ __launch_bounds__(256) void burgers_op_group(const OpArgs<T> *items, const int *bstart,
                                                        int n) {
    const int it = group_item(bstart, n, blockIdx.x);
    const int local = blockIdx.x - bstart[it], G = bstart[it + 1] - bstart[it];
    burgers_op_body<P, T, JVP, VISC>(items[it], xcd_tile(local, G), local == 0);
}

template <int P, typename T, bool VISC>
hipError_t launch_burgers_group(bool jvp, const OpArgs<T> *items, const int *bstart, int n,
                                int total, hipStream_t s) {
    if (jvp)
        return launch_kernel(burgers_op_group<P, T, true, VISC>, dim3(total), dim3(256), 0, s,
                             items, bstart, n);
    return launch_kernel(burgers_op_group<P, T, false, VISC>, dim3(total), dim3(256), 0, s, items,
                         bstart, n);
}

template <int P, typename T>
hipError_t launch_group_p(int equation, bool jvp, bool visc, const OpArgs<T> *items,
                          const int *bstart, int n, int total, hipStream_t s) {
    if (equation == EXPDG_EULER3D) return hipErrorInvalidValue;  // not served
    if (equation == EXPDG_EULER2D) {
        // visc: the items carry an entropy viscosity
        if (visc) {
            if (jvp)
                return launch_kernel(euler_op_group<P, T, true, true>, dim3(total), dim3(256), 0,
                                     s, items, bstart, n);
            return launch_kernel(euler_op_group<P, T, false, true>, dim3(total), dim3(256), 0, s,
                                 items, bstart, n);
        }
        if (jvp)
            return launch_kernel(euler_op_group<P, T, true, false>, dim3(total), dim3(256), 0, s,
                                 items, bstart, n);
        return launch_kernel(euler_op_group<P, T, false, false>, dim3(total), dim3(256), 0, s,
                             items, bstart, n);
    }
    if (visc) return launch_burgers_group<P, T, true>(jvp, items, bstart, n, total, s);
    return launch_burgers_group<P, T, false>(jvp, items, bstart, n, total, s);
}

template <int P, typename T>
hipError_t launch_p(int equation, bool jvp, const OpArgs<T> &a, hipStream_t s) {
    if constexpr (!std::is_same<T, double>::value) {
        // FP32 storage: the residual of an FP64 state (a.q64) reads it directly
        if (!jvp && a.q64) {
            if (equation == EXPDG_EULER3D) {
                using S = E3Shape<P>;
                const int grid = (a.K + S::EPB - 1) / S::EPB;
                return launch_kernel(euler3_op_r64<P, T>, dim3(grid), dim3(S::BS), 0, s, a);
            }
            if (equation == EXPDG_EULER2D) {
                constexpr int EPB = 256 / ((P + 1) * (P + 1));
                const int grid = (a.K + EPB - 1) / EPB;
                if (a.nu)
                    return launch_kernel(euler_op_r64<P, T, true>, dim3(grid), dim3(256), 0, s, a);
                return launch_kernel(euler_op_r64<P, T, false>, dim3(grid), dim3(256), 0, s, a);
            }
            constexpr int EPB = 256 / (P + 1);
            const int grid = (a.K + EPB - 1) / EPB;
            if (a.kappa != 0.0)
                return launch_kernel(burgers_op_r64<P, T, true>, dim3(grid), dim3(256), 0, s, a);
            return launch_kernel(burgers_op_r64<P, T, false>, dim3(grid), dim3(256), 0, s, a);
        }
    }
    if (equation == EXPDG_EULER3D) {
        using S = E3Shape<P>;
        const int grid = (a.K + S::EPB - 1) / S::EPB;
        if (jvp) return launch_kernel(euler3_op<P, T, true>, dim3(grid), dim3(S::BS), 0, s, a);
        return launch_kernel(euler3_op<P, T, false>, dim3(grid), dim3(S::BS), 0, s, a);
    }
    if (equation == EXPDG_EULER2D) {
        constexpr int EPB = 256 / ((P + 1) * (P + 1));
        const int grid = (a.K + EPB - 1) / EPB;
        if (a.nu) {
            if (jvp)
                return launch_kernel(euler_op<P, T, true, true>, dim3(grid), dim3(256), 0, s, a);
            return launch_kernel(euler_op<P, T, false, true>, dim3(grid), dim3(256), 0, s, a);
        }
        if (jvp && a.dots && grid <= kHalvesBlocks)
            return launch_kernel(euler_op_halves<P, T>, dim3(grid), dim3(512), 0, s, a);
        if (jvp) return launch_kernel(euler_op<P, T, true, false>, dim3(grid), dim3(256), 0, s, a);
        return launch_kernel(euler_op<P, T, false, false>, dim3(grid), dim3(256), 0, s, a);
    }
    constexpr int EPB = 256 / (P + 1);
    const int grid = (a.K + EPB - 1) / EPB;
    if (a.kappa != 0.0) {
        if (jvp)
            return launch_kernel(burgers_op<P, T, true, true>, dim3(grid), dim3(256), 0, s, a);
        return launch_kernel(burgers_op<P, T, false, true>, dim3(grid), dim3(256), 0, s, a);
    }
    if (jvp) return launch_kernel(burgers_op<P, T, true, false>, dim3(grid), dim3(256), 0, s, a);
    return launch_kernel(burgers_op<P, T, false, false>, dim3(grid), dim3(256), 0, s, a);
}

template <typename T>
hipError_t launch_any(int equation, int p, bool jvp, const OpArgs<T> &a, hipStream_t s) {
    switch (p) {
        case 1: return launch_p<1, T>(equation, jvp, a, s);
        case 2: return launch_p<2, T>(equation, jvp, a, s);
        case 3: return launch_p<3, T>(equation, jvp, a, s);
        case 4: return launch_p<4, T>(equation, jvp, a, s);
        case 5: return launch_p<5, T>(equation, jvp, a, s);
        case 6: return launch_p<6, T>(equation, jvp, a, s);
        default: return hipErrorInvalidValue;
    }
}

// ---- wave speed -------------------------------------------------------------
__global__ __launch_bounds__(256) void max_speed_kernel(int equation, const double *q,
                                                        size_t npts, double gamma,
                                                        double *part) {
    __shared__ double sm[256];
    double mx = 0.0;
    for (size_t r = (size_t)blockIdx.x * 256 + threadIdx.x; r < npts;
         r += (size_t)gridDim.x * 256) {
        if (equation == EXPDG_BURGERS1D) {
            mx = fmax(mx, fabs(q[r]));
        } else if (equation == EXPDG_EULER3D) {
            const double qq[5] = {q[r], q[npts + r], q[2 * npts + r], q[3 * npts + r],
                                  q[4 * npts + r]};
            mx = fmax(mx, fmax(euler3_speed<double, 0>(qq, gamma),
                               fmax(euler3_speed<double, 1>(qq, gamma),
                                    euler3_speed<double, 2>(qq, gamma))));
        } else {
            const double qq[4] = {q[r], q[npts + r], q[2 * npts + r], q[3 * npts + r]};
            mx = fmax(mx, fmax(euler_speed<double, 0>(qq, gamma), euler_speed<double, 1>(qq, gamma)));
        }
    }
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// ---- elementwise ------------------------------------------------------------
template <typename TO, typename TI>
__global__ __launch_bounds__(256) void convert_kernel(const TI *x, TO *y, size_t n) {
    for (size_t r = (size_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (size_t)gridDim.x * 256)
        y[r] = (TO)x[r];
}

template <typename TO, typename TX>
__global__ __launch_bounds__(256) void lincomb_kernel(TO *out, double a, const TX *x, double b,
                                                      const TX *y, double c, const TX *z,
                                                      size_t n) {
    for (size_t r = (size_t)blockIdx.x * 256 + threadIdx.x; r < n;
         r += (size_t)gridDim.x * 256) {
        double acc = a * (double)x[r];
        if (y) acc += b * (double)y[r];
        if (z) acc += c * (double)z[r];
        out[r] = (TO)acc;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void add_to_kernel(double *q, const T *w, size_t n) {
    for (size_t r = (size_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (size_t)gridDim.x * 256)
        q[r] += (double)w[r];
}

// out = x + y (FP64 out and x, y of the bulk type)
template <typename T>
__global__ __launch_bounds__(256) void add_mixed_kernel(double *out, const double *x, const T *y,
                                                        size_t n) {
    for (size_t r = (size_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (size_t)gridDim.x * 256)
        out[r] = x[r] + (double)y[r];
}

template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(T *x, T val, size_t n) {
    for (size_t r = (size_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (size_t)gridDim.x * 256)
        x[r] = val;
}

// x[0..p) = (0, ..., 0, last)
template <typename T>
__global__ void set_tail_kernel(T *x, int p, double last) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        for (int k = 0; k < p; ++k) x[k] = (k == p - 1) ? (T)last : T(0);
}

// Start vector of a phi evaluation: z[0..n) = b0 (or 0), z[n..n+p) =
// (0, ..., 0, last); the Krylov flags (4 ints) cleared.
template <typename T>
__global__ __launch_bounds__(256) void phi_init_kernel(T *z, const T *b0, size_t n, int p,
                                                       double last, int *flags) {
    for (size_t r = (size_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (size_t)gridDim.x * 256)
        z[r] = b0 ? b0[r] : T(0);
    if (blockIdx.x == 0 && threadIdx.x < 4) flags[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int k = 0; k < p; ++k) z[n + k] = (k == p - 1) ? (T)last : T(0);
}

// End of a step: q_prev = q (if given), then q += w.
template <typename T>
__global__ __launch_bounds__(256) void step_update_kernel(double *q, double *q_prev, const T *w,
                                                          size_t n) {
    for (size_t r = (size_t)blockIdx.x * 256 + threadIdx.x; r < n;
         r += (size_t)gridDim.x * 256) {
        const double x = q[r];
        if (q_prev) q_prev[r] = x;
        q[r] = x + (double)w[r];
    }
}

int grid_for(size_t n) {
    size_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_ev_element(const EvParams &ep, const double *q, const double *q_prev,
                             double *nue, hipStream_t s) {
    const int np = (ep.p + 1) * (ep.p + 1), epb = 256 / np;
    const dim3 grid((unsigned)((ep.K + epb - 1) / epb));
    switch (ep.p) {
        case 1: return launch_kernel(ev_element_kernel<1>, grid, dim3(256), 0, s, ep, q, q_prev, nue);
        case 2: return launch_kernel(ev_element_kernel<2>, grid, dim3(256), 0, s, ep, q, q_prev, nue);
        case 3: return launch_kernel(ev_element_kernel<3>, grid, dim3(256), 0, s, ep, q, q_prev, nue);
        case 4: return launch_kernel(ev_element_kernel<4>, grid, dim3(256), 0, s, ep, q, q_prev, nue);
        case 5: return launch_kernel(ev_element_kernel<5>, grid, dim3(256), 0, s, ep, q, q_prev, nue);
        case 6: return launch_kernel(ev_element_kernel<6>, grid, dim3(256), 0, s, ep, q, q_prev, nue);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_ev_smooth(const EvParams &ep, const double *nue, T *nu, hipStream_t s) {
    const size_t npts = (size_t)ep.K * (ep.p + 1) * (ep.p + 1);
    const dim3 grid((unsigned)((npts + 255) / 256));
    switch (ep.p) {
        case 1: return launch_kernel(ev_smooth_kernel<1, T>, grid, dim3(256), 0, s, ep, nue, nu);
        case 2: return launch_kernel(ev_smooth_kernel<2, T>, grid, dim3(256), 0, s, ep, nue, nu);
        case 3: return launch_kernel(ev_smooth_kernel<3, T>, grid, dim3(256), 0, s, ep, nue, nu);
        case 4: return launch_kernel(ev_smooth_kernel<4, T>, grid, dim3(256), 0, s, ep, nue, nu);
        case 5: return launch_kernel(ev_smooth_kernel<5, T>, grid, dim3(256), 0, s, ep, nue, nu);
        case 6: return launch_kernel(ev_smooth_kernel<6, T>, grid, dim3(256), 0, s, ep, nue, nu);
        default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_ev_smooth<double>(const EvParams &, const double *, double *,
                                             hipStream_t);
template hipError_t launch_ev_smooth<float>(const EvParams &, const double *, float *,
                                            hipStream_t);

template <typename Q, typename T>
hipError_t launch_lin_prepare(int equation, int p, const Q *q, T *lin, int K, int nx, int ny,
                              double gamma, hipStream_t s) {
    if (equation == EXPDG_EULER3D) {
        const size_t npts = (size_t)K * (p + 1) * (p + 1) * (p + 1);
        const dim3 grid((unsigned)((npts + 255) / 256));
        const int nz = K / (nx * ny);
        switch (p) {
            case 1: return launch_kernel(euler3_lin_prepare<1, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, nz, gamma);
            case 2: return launch_kernel(euler3_lin_prepare<2, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, nz, gamma);
            case 3: return launch_kernel(euler3_lin_prepare<3, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, nz, gamma);
            case 4: return launch_kernel(euler3_lin_prepare<4, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, nz, gamma);
            case 5: return launch_kernel(euler3_lin_prepare<5, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, nz, gamma);
            case 6: return launch_kernel(euler3_lin_prepare<6, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, nz, gamma);
            default: return hipErrorInvalidValue;
        }
    }
    if (equation != EXPDG_EULER2D) return hipSuccess;  // Burgers reads the state itself
    const size_t npts = (size_t)K * (p + 1) * (p + 1);
    const dim3 grid((unsigned)((npts + 255) / 256));
    switch (p) {
        case 1: return launch_kernel(euler_lin_prepare<1, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, gamma);
        case 2: return launch_kernel(euler_lin_prepare<2, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, gamma);
        case 3: return launch_kernel(euler_lin_prepare<3, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, gamma);
        case 4: return launch_kernel(euler_lin_prepare<4, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, gamma);
        case 5: return launch_kernel(euler_lin_prepare<5, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, gamma);
        case 6: return launch_kernel(euler_lin_prepare<6, Q, T>, grid, dim3(256), 0, s, q, lin, K, nx, ny, gamma);
        default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_lin_prepare<double, double>(int, int, const double *, double *, int,
                                                       int, int, double, hipStream_t);
template hipError_t launch_lin_prepare<float, float>(int, int, const float *, float *, int, int,
                                                     int, double, hipStream_t);
template hipError_t launch_lin_prepare<double, float>(int, int, const double *, float *, int, int,
                                                      int, double, hipStream_t);

size_t lin_elems(int equation, int p, int K) {
    const size_t n1 = (size_t)p + 1;
    if (equation == EXPDG_EULER3D) return (size_t)K * (4 * n1 * n1 * n1 + 3 * n1 * n1);
    if (equation != EXPDG_EULER2D) return 0;
    return (size_t)K * (3 * n1 * n1 + 2 * n1);
}

int dg_block_threads(int equation, int p) {
    return (equation == EXPDG_EULER3D && (p + 1) * (p + 1) * (p + 1) > 256) ? 384 : 256;
}

int dg_blocks(int equation, int p, int K) {
    const int n1 = p + 1;
    const int np = (equation == EXPDG_EULER3D) ? n1 * n1 * n1
                   : (equation == EXPDG_EULER2D) ? n1 * n1 : n1;
    const int epb = dg_block_threads(equation, p) / np;
    return (K + epb - 1) / epb;
}

hipError_t launch_dg_op_group(int equation, int p, bool jvp, bool visc,
                              const OpArgs<double> *items, const int *bstart, int n, int total,
                              hipStream_t s) {
    if (visc && equation == EXPDG_EULER3D) return hipErrorInvalidValue;
    switch (p) {
        case 1: return launch_group_p<1, double>(equation, jvp, visc, items, bstart, n, total, s);
        case 2: return launch_group_p<2, double>(equation, jvp, visc, items, bstart, n, total, s);
        case 3: return launch_group_p<3, double>(equation, jvp, visc, items, bstart, n, total, s);
        case 4: return launch_group_p<4, double>(equation, jvp, visc, items, bstart, n, total, s);
        case 5: return launch_group_p<5, double>(equation, jvp, visc, items, bstart, n, total, s);
        case 6: return launch_group_p<6, double>(equation, jvp, visc, items, bstart, n, total, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dg_op(int equation, int p, bool jvp, const OpArgs<double> &a, hipStream_t s) {
    return launch_any<double>(equation, p, jvp, a, s);
}
hipError_t launch_dg_op(int equation, int p, bool jvp, const OpArgs<float> &a, hipStream_t s) {
    return launch_any<float>(equation, p, jvp, a, s);
}

int max_speed_blocks(size_t npts) {
    size_t g = (npts + 255) / 256;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_max_speed(int equation, const double *q, size_t npts, double gamma, double *part,
                            int nblk, hipStream_t s) {
    max_speed_kernel<<<nblk, 256, 0, s>>>(equation, q, npts, gamma, part);
    return hipGetLastError();
}

hipError_t launch_convert(const double *x, float *y, size_t n, hipStream_t s) {
    convert_kernel<float, double><<<grid_for(n), 256, 0, s>>>(x, y, n);
    return hipGetLastError();
}
hipError_t launch_convert(const float *x, double *y, size_t n, hipStream_t s) {
    convert_kernel<double, float><<<grid_for(n), 256, 0, s>>>(x, y, n);
    return hipGetLastError();
}
hipError_t launch_copy(const double *x, double *y, size_t n, hipStream_t s) {
    convert_kernel<double, double><<<grid_for(n), 256, 0, s>>>(x, y, n);
    return hipGetLastError();
}
hipError_t launch_copy(const float *x, float *y, size_t n, hipStream_t s) {
    convert_kernel<float, float><<<grid_for(n), 256, 0, s>>>(x, y, n);
    return hipGetLastError();
}

template <typename TO, typename TX>
hipError_t launch_lincomb(TO *out, double a, const TX *x, double b, const TX *y, double c,
                          const TX *z, size_t n, hipStream_t s) {
    lincomb_kernel<TO, TX><<<grid_for(n), 256, 0, s>>>(out, a, x, b, y, c, z, n);
    return hipGetLastError();
}
template hipError_t launch_lincomb<double, double>(double *, double, const double *, double,
                                                   const double *, double, const double *,
                                                   size_t, hipStream_t);
template hipError_t launch_lincomb<float, float>(float *, double, const float *, double,
                                                 const float *, double, const float *, size_t,
                                                 hipStream_t);
template hipError_t launch_lincomb<float, double>(float *, double, const double *, double,
                                                  const double *, double, const double *,
                                                  size_t, hipStream_t);

template <typename T>
hipError_t launch_add_to(double *q, const T *w, size_t n, hipStream_t s) {
    add_to_kernel<T><<<grid_for(n), 256, 0, s>>>(q, w, n);
    return hipGetLastError();
}
template hipError_t launch_add_to<double>(double *, const double *, size_t, hipStream_t);
template hipError_t launch_add_to<float>(double *, const float *, size_t, hipStream_t);

template <typename T>
hipError_t launch_add_mixed(double *out, const double *x, const T *y, size_t n, hipStream_t s) {
    add_mixed_kernel<T><<<grid_for(n), 256, 0, s>>>(out, x, y, n);
    return hipGetLastError();
}
template hipError_t launch_add_mixed<double>(double *, const double *, const double *, size_t,
                                             hipStream_t);
template hipError_t launch_add_mixed<float>(double *, const double *, const float *, size_t,
                                            hipStream_t);

template <typename T>
hipError_t launch_fill(T *x, double val, size_t n, hipStream_t s) {
    fill_kernel<T><<<grid_for(n), 256, 0, s>>>(x, (T)val, n);
    return hipGetLastError();
}
template hipError_t launch_fill<double>(double *, double, size_t, hipStream_t);
template hipError_t launch_fill<float>(float *, double, size_t, hipStream_t);
template hipError_t launch_fill<int>(int *, double, size_t, hipStream_t);

template <typename T>
hipError_t launch_set_tail(T *x, int p, double last, hipStream_t s) {
    set_tail_kernel<T><<<1, 64, 0, s>>>(x, p, last);
    return hipGetLastError();
}
template hipError_t launch_set_tail<double>(double *, int, double, hipStream_t);
template hipError_t launch_set_tail<float>(float *, int, double, hipStream_t);

template <typename T>
hipError_t launch_phi_init(T *z, const T *b0, size_t n, int p, double last, int *flags,
                           hipStream_t s) {
    phi_init_kernel<T><<<grid_for(n), 256, 0, s>>>(z, b0, n, p, last, flags);
    return hipGetLastError();
}
template hipError_t launch_phi_init<double>(double *, const double *, size_t, int, double, int *,
                                            hipStream_t);
template hipError_t launch_phi_init<float>(float *, const float *, size_t, int, double, int *,
                                           hipStream_t);

template <typename T>
hipError_t launch_step_update(double *q, double *q_prev, const T *w, size_t n, hipStream_t s) {
    step_update_kernel<T><<<grid_for(n), 256, 0, s>>>(q, q_prev, w, n);
    return hipGetLastError();
}
template hipError_t launch_step_update<double>(double *, double *, const double *, size_t,
                                               hipStream_t);
template hipError_t launch_step_update<float>(double *, double *, const float *, size_t,
                                              hipStream_t);

}  // namespace expdg
