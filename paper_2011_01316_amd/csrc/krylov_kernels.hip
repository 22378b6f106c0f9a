// Arnoldi / Krylov kernels for gfx950 (Section 2.3: Krylov projection of the
// augmented matrix).  The orthogonalisation is classical Gram-Schmidt applied
// twice, with the second pass of each vector delayed into the next Arnoldi
// step so that one dot pass and one update sweep serve both passes.
//
// Basis storage: V holds unnormalised vectors u_i (bulk type, float or
// double) with FP64 scales S[i] so that v_i = S[i] u_i; no separate
// normalisation pass is needed.  Inner products and norms are accumulated in
// FP64 over a fixed row partition; the block partials are summed in a fixed
// order by a small finishing kernel, so results are identical run to run.
// (Two alternatives measured slower on MI355X: letting the last block of each
// launch finish needs a device-scope release fence in every block, which
// writes back the XCD's L2 each time; letting every block of the consuming
// kernel re-derive the sums makes each block wait on partials that other XCDs
// wrote.)
//
// Arnoldi step k (the operator was applied to x = u_{k-1}, which has had its
// first pass only; w = A x):
//   dot pass     u_i^T w, u_i^T x (i < k-1), x^T x, x^T w: block partials
//                from the 2D linear operator's epilogue, or gs_dots2 (2D grid:
//                row blocks x 16-vector chunks) after the 1D operator
//   dcgs_finish  second pass of x (a = V^T x, beta = sqrt(x^T x - |a|^2) by
//                Pythagoras): column k-2 of H and H[k-1][k-2] final; the
//                Arnoldi relation A V = V H turns w = A x into
//                A v_{k-1} = (w - V_k t) / beta, t = H a, whose first pass g
//                (column k-1 of H) follows from the same dots; breakdown test
//   dcgs_update  x -= V a and w <- (w - V_k t) / beta - V_k g in one sweep
// Block sums use a transpose reduction: 32 accumulators of a wave are summed
// with 32 cross-lane exchanges instead of 6 per accumulator.
//
// The small (j+1) x (j+1) exponential of the projected Hessenberg matrix runs
// in one 256-thread workgroup with four FP64 matrices in LDS (gfx950 gives a
// workgroup up to 160 KB): diagonal Pade (6,6) with scaling and squaring.  Its
// rational form D^-1 N is evaluated with matrix products only (the scaled
// denominator is within 0.2805 of the identity, so a product of five Neumann
// factors reaches FP64 accuracy), which keeps every step parallel over the
// workgroup instead of a sequential elimination.
#include "internal.h"
#include "reduce.h"

namespace expdg {
namespace {

constexpr int LDH = kLDH;   // leading dimension of H
constexpr int CH = 16;      // basis vectors per chunk of the dot kernel

// 16-byte vector access: 2 doubles or 4 floats per lane per load.
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    static constexpr int N = 2;
    using type = double2;
};
template <>
struct Vec16<float> {
    static constexpr int N = 4;
    using type = float4;
};

template <typename T>
__device__ __forceinline__ void ld16(const T *p, double *out) {
    using VT = typename Vec16<T>::type;
    const VT v = *reinterpret_cast<const VT *>(p);
    const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
    for (int k = 0; k < Vec16<T>::N; ++k) out[k] = (double)e[k];
}

// Stores the values rounded to T and returns the rounded values in x.
template <typename T>
__device__ __forceinline__ void st16(T *p, double *x) {
    using VT = typename Vec16<T>::type;
    VT v;
    T *e = reinterpret_cast<T *>(&v);
#pragma unroll
    for (int k = 0; k < Vec16<T>::N; ++k) {
        e[k] = (T)x[k];
        x[k] = (double)e[k];
    }
    *reinterpret_cast<VT *>(p) = v;
}

// ---- start vector of a substep ----------------------------------------------
// Block partials of ||z||^2.
template <typename T>
__device__ __forceinline__ void gs_norm_body(const T *__restrict__ z, size_t L, size_t rpb,
                                             double *__restrict__ part, int rb) {
    __shared__ double sw[4];
    const int tid = threadIdx.x;
    const size_t r0 = (size_t)rb * rpb;
    const size_t r1 = (r0 + rpb < L) ? r0 + rpb : L;
    double acc = 0.0;
    constexpr int N = Vec16<T>::N;
    const size_t nsw = (r1 - r0) / (256 * N);
    for (size_t k = 0; k < nsw; ++k) {
        const size_t r = r0 + (k * 256 + tid) * N;
        double x[N];
        ld16(z + r, x);
#pragma unroll
        for (int e = 0; e < N; ++e) acc += x[e] * x[e];
    }
    for (size_t r = r0 + nsw * 256 * N + tid; r < r1; r += 256) {
        const double x = (double)z[r];
        acc += x * x;
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) sw[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) part[rb] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

template <typename T>
__global__ __launch_bounds__(256) void gs_norm_kernel(const T *__restrict__ z, size_t L,
                                                      size_t rpb, double *__restrict__ part) {
    gs_norm_body<T>(z, L, rpb, part, blockIdx.x);
}

struct NormFinish {
    double *H;
    double *S;
    int *flags;     // [0] first breakdown dimension, [1] first non-finite one
    double *res;    // res[0] = beta
};

// beta = ||z|| from the partials in a fixed order; S[0] = 1/beta, the flags
// reset, and the Hessenberg matrix cleared for the new substep.
__device__ __forceinline__ void finish_norm_body(const double *part, int nrb, const NormFinish &f) {
    __shared__ double sw[4];
    const int tid = threadIdx.x;
    double a = 0.0;
    for (int b = tid; b < nrb; b += 256) a += part[b];
    a = wave_sum(a);
    if ((tid & 63) == 0) sw[tid >> 6] = a;
    __syncthreads();
    const double hn = sqrt((sw[0] + sw[1]) + (sw[2] + sw[3]));
    if (tid == 0) {
        f.res[0] = hn;
        f.S[0] = (hn > 0.0) ? 1.0 / hn : 0.0;
        f.flags[0] = 0;
        f.flags[1] = isfinite(hn) ? 0 : 1;
    }
    for (int e = tid; e < (kMaxM + 1) * LDH; e += 256) f.H[e] = 0.0;
}

__global__ __launch_bounds__(256) void finish_norm_kernel(const double *part, int nrb,
                                                          NormFinish f) {
    finish_norm_body(part, nrb, f);
}

// ---- one Arnoldi step: dot pass, finish, update sweep -----------------------
// Block partials of step k (nv = k - 1 finished vectors), for the block's rows
// and the chunk of CH basis vectors i0 = chunk * CH: rows i0 + i (u^T w) and
// nv + i0 + i (u^T x); chunk 0 also gives rows 2 nv (x^T x) and 2 nv + 1 (x^T w).
template <typename T>
__device__ __forceinline__ void gs_dots2_body(const T *__restrict__ V, size_t stride, int nv,
                                              const T *__restrict__ x, const T *__restrict__ w,
                                              size_t L, size_t rpb, int nrb,
                                              double *__restrict__ part, int rb, int chunk) {
    __shared__ double sw[4][2 * CH];
    __shared__ double s2[4][2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i0 = chunk * CH;
    const int nloc = max(0, min(CH, nv - i0));
    const bool own = chunk == 0;  // this block also sums x^T x and x^T w
    const size_t r0 = (size_t)rb * rpb;
    const size_t r1 = (r0 + rpb < L) ? r0 + rpb : L;
    double acc[2 * CH];
#pragma unroll
    for (int i = 0; i < 2 * CH; ++i) acc[i] = 0.0;
    double axx = 0.0, axw = 0.0;
    const T *Vc = V + (size_t)i0 * stride;
    constexpr int N = Vec16<T>::N;
    const size_t nsw = (r1 - r0) / (256 * N);
    for (size_t k = 0; k < nsw; ++k) {
        const size_t r = r0 + (k * 256 + tid) * N;
        double xv[N], wv[N];
        ld16(x + r, xv);
        ld16(w + r, wv);
        if (nloc > 0) {
            // unconditional loads (vector index clamped, extra products
            // dropped), so the chunk's loads are in flight together
            double vv[CH][N];
#pragma unroll
            for (int i = 0; i < CH; ++i) ld16(Vc + (size_t)min(i, nloc - 1) * stride + r, vv[i]);
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const bool in = i < nloc;
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    acc[i] += in ? vv[i][e] * wv[e] : 0.0;
                    acc[CH + i] += in ? vv[i][e] * xv[e] : 0.0;
                }
            }
        }
        if (own) {
#pragma unroll
            for (int e = 0; e < N; ++e) {
                axx += xv[e] * xv[e];
                axw += xv[e] * wv[e];
            }
        }
    }
    for (size_t r = r0 + nsw * 256 * N + tid; r < r1; r += 256) {
        const double xs = (double)x[r], ws = (double)w[r];
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (i < nloc) {
                const double u = (double)Vc[(size_t)i * stride + r];
                acc[i] += u * ws;
                acc[CH + i] += u * xs;
            }
        if (own) {
            axx += xs * xs;
            axw += xs * ws;
        }
    }
    const double v = transpose_reduce32(acc);
    if ((lane & 1) == 0) sw[wave][lane >> 1] = v;
    axx = wave_sum(axx);
    axw = wave_sum(axw);
    if (lane == 0) {
        s2[wave][0] = axx;
        s2[wave][1] = axw;
    }
    __syncthreads();
    if (tid < 2 * CH && (tid % CH) < nloc) {
        const int row = (tid < CH) ? i0 + tid : nv + i0 + (tid - CH);
        part[(size_t)row * nrb + rb] = (sw[0][tid] + sw[1][tid]) + (sw[2][tid] + sw[3][tid]);
    }
    if (own && tid < 2)
        part[(size_t)(2 * nv + tid) * nrb + rb] = (s2[0][tid] + s2[1][tid]) + (s2[2][tid] + s2[3][tid]);
}

template <typename T>
__global__ __launch_bounds__(256) void gs_dots2_kernel(const T *__restrict__ V, size_t stride,
                                                       int nv, const T *__restrict__ x,
                                                       const T *__restrict__ w, size_t L,
                                                       size_t rpb, int nrb,
                                                       double *__restrict__ part) {
    gs_dots2_body<T>(V, stride, nv, x, w, L, rpb, nrb, part, blockIdx.x, blockIdx.y);
}

// Finish of step k (one block of kFin2Threads threads); see launch_dcgs_finish.
// The finished part of H is copied to LDS once, so the norm, t = H a and the
// first pass read no global memory written within the launch; every sum runs
// in a fixed order, so results are identical run to run.
constexpr int kFin2Threads = 1024;

// sv[r] = sum_b part[r * nrb + b] for r < rows: each row gets tpr consecutive
// lanes of one wave (tpr the largest power of two <= 64 with rows tpr <=
// kFin2Threads); lane j sums b = j, j + tpr, ... in ascending order, then the
// row's lanes are summed by butterfly.  All rows are summed at once.
__device__ __forceinline__ void fin_row_sums(const double *part, int rows, int nrb, double *sv) {
    const int tid = threadIdx.x;
    int lg = 6;
    while (lg > 0 && (rows << lg) > kFin2Threads) --lg;
    const int tpr = 1 << lg;
    const int r = tid >> lg, j = tid & (tpr - 1);
    double s = 0.0;
    if (r < rows) {
        // batches of UB loads in flight together (index clamped, extra
        // values dropped), added in the same ascending order
        constexpr int UB = 16;
        const double *pr = part + (size_t)r * nrb;
        for (int b0 = j; b0 < nrb; b0 += UB * tpr) {
            double v[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) v[u] = pr[min(b0 + u * tpr, nrb - 1)];
#pragma unroll
            for (int u = 0; u < UB; ++u) s += (b0 + u * tpr < nrb) ? v[u] : 0.0;
        }
    }
    for (int off = tpr >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (j == 0 && r < rows) sv[r] = s;
}

// Fold of long partial rows (see kFoldAbove): block (c, r) of 256 threads
// sums chunk c of row r; thread t adds its four partials c kFoldChunk + t +
// 256 u in ascending u, then the wave butterfly, then the four wave sums as
// (w0 + w1) + (w2 + w3).  The order is fixed, so results repeat bitwise.
__device__ __forceinline__ void fold_body(const double *part, int nrb, double *out, int nc,
                                          int r, int c) {
    static_assert(kFoldChunk == 4 * 256, "four partials per thread");
    __shared__ double sw[4];
    const int tid = threadIdx.x;
    const double *pr = part + (size_t)r * nrb;
    const int b0 = c * kFoldChunk + tid;
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = pr[min(b0 + u * 256, nrb - 1)];
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) s += (b0 + u * 256 < nrb) ? v[u] : 0.0;
    s = wave_sum(s);
    if ((tid & 63) == 0) sw[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) out[(size_t)r * nc + c] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

__global__ __launch_bounds__(256) void fold_kernel(const double *part, int nrb, double *out,
                                                   int nc) {
    fold_body(part, nrb, out, nc, blockIdx.y, blockIdx.x);
}

struct DcgsFinish {
    double *S, *H;
    int k;
    double *coefA, *coefB;
    int *flags;
};

__device__ __forceinline__ void dcgs_finish_body(const double *part, int nrb,
                                                 const DcgsFinish &f) {
    constexpr int NW = kFin2Threads / 64;
    __shared__ double sH[(kMaxM + 1) * LDH];
    __shared__ double sv[kPartRows];
    __shared__ double sa[kMaxM + 1], st[kMaxM + 1], se[kMaxM + 1];
    __shared__ double sw[NW];
    __shared__ double saa, sab, sbeta;
    const int k = f.k, nv = k - 1, col = k - 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *H = f.H, *S = f.S;
    // the scales, rows 0..k-1 and columns 0..k-2 of H (loads unconditional,
    // indices clamped into range, so a wave's loads are in flight together),
    // and the row sums of the block partials
    const double Si = (tid < nv) ? S[tid] : 0.0;
    {
        constexpr int QH = (kMaxM + 1 + NW - 1) / NW;
        const int cc = min(lane, max(col, 0));
        double hv[QH];
#pragma unroll
        for (int q = 0; q < QH; ++q) hv[q] = H[(size_t)min(wave + q * NW, kMaxM) * LDH + cc];
#pragma unroll
        for (int q = 0; q < QH; ++q)
            if (wave + q * NW < k && lane <= col) sH[(wave + q * NW) * LDH + lane] = hv[q];
    }
    fin_row_sums(part, 2 * nv + 2, nrb, sv);
    __syncthreads();
    // a_i = v_i^T x and b_i = v_i^T w; nv <= kMaxM, so all of them in wave 0
    double ai = 0.0, bi = 0.0;
    if (tid < nv) {
        ai = Si * sv[nv + tid];
        bi = Si * sv[tid];
        sa[tid] = ai;
    }
    if (wave == 0) {
        const double aa = wave_sum(ai * ai), ab = wave_sum(ai * bi);
        if (lane == 0) {
            saa = aa;
            sab = ab;
        }
    }
    __syncthreads();
    const double gam = sv[2 * nv], del = sv[2 * nv + 1];
    if (k == 1) {
        // x = u_0 is the finished start vector
        if (tid == 0) sbeta = 1.0 / S[0];
        __syncthreads();
    } else {
        // second pass of x: ||x - V a||^2 = x^T x - |a|^2 (Pythagoras); the
        // finished column k-2 is the first pass plus a
        const double q2 = gam - saa;
        const double beta = (q2 < 0.0) ? 0.0 : sqrt(q2);  // NaN stays NaN
        if (tid <= col) sH[tid * LDH + col] += sa[tid];
        if (tid == 0) sH[(k - 1) * LDH + col] = beta;
        __syncthreads();
        // ||H_{0:k, 0:k-1}||_F with the finished column and the new subdiagonal
        double acc = 0.0;
        for (int r = wave; r < k; r += NW)
            for (int c = lane; c <= col; c += 64) {
                const double h = (r <= c + 1) ? sH[r * LDH + c] : 0.0;
                acc += h * h;
            }
        acc = wave_sum(acc);
        if (lane == 0) sw[wave] = acc;
        __syncthreads();
        if (tid <= col) H[(size_t)tid * LDH + col] = sH[tid * LDH + col];
        if (tid == 0) {
            double s = 0.0;
            for (int q = 0; q < NW; ++q) s += sw[q];
            const double hf = sqrt(s);
            if ((!isfinite(beta) || !isfinite(hf)) && f.flags[1] == 0) f.flags[1] = k - 1;
            const bool brk = beta <= 1e-12 * hf;
            if (brk) {
                H[(size_t)(k - 1) * LDH + col] = 0.0;
                S[k - 1] = 0.0;
                if (f.flags[0] == 0) f.flags[0] = k - 1;
            } else {
                H[(size_t)(k - 1) * LDH + col] = beta;
                S[k - 1] = 1.0 / beta;
            }
            sH[(k - 1) * LDH + col] = brk ? 0.0 : beta;
            sbeta = brk ? 1.0 : beta;  // after a breakdown the step only has to stay finite
        }
        __syncthreads();
    }
    const double bet = sbeta;
    // t = H_{0:k, 0:k-1} a (A V_{k-1} a expressed in the basis V_k): one wave per row
    for (int r = wave; r < k; r += NW) {
        double t = 0.0;
        for (int c = max(r - 1, 0) + lane; c <= col; c += 64) t += sH[r * LDH + c] * sa[c];
        t = wave_sum(t);
        if (lane == 0) st[r] = t;
    }
    __syncthreads();
    // first pass of A v_{k-1} = (w - V_k t) / beta; e = t / beta + g
    if (tid < k) {
        double g;
        if (tid < nv)
            g = (bi - st[tid]) / bet;
        else
            g = ((del - sab) / bet - st[tid]) / bet;
        H[(size_t)tid * LDH + (k - 1)] = g;
        se[tid] = st[tid] / bet + g;
    }
    __syncthreads();
    const double ek = se[k - 1];
    if (tid < nv) {
        f.coefA[tid] = Si * sa[tid];
        f.coefB[tid] = Si * (se[tid] - sa[tid] * ek / bet);
    }
    if (tid == 0) {
        f.coefB[kScalW] = 1.0 / bet;
        f.coefB[kScalX] = ek / bet;
    }
}

__global__ __launch_bounds__(kFin2Threads) void dcgs_finish_kernel(const double *part, int nrb,
                                                                   DcgsFinish f) {
    dcgs_finish_body(part, nrb, f);
}

// Update sweep of step k: x -= sum_i cA_i u_i (nv > 0) and
// w <- cB[kScalW] w - cB[kScalX] x_old - sum_i cB_i u_i, reading each u_i once.
template <typename T>
__device__ __forceinline__ void dcgs_update_body(const T *__restrict__ V, size_t stride, int nv,
                                                 const double *cA, const double *cB,
                                                 T *__restrict__ x, T *__restrict__ w, size_t r0,
                                                 size_t r1, bool wx) {
    __shared__ double sA[kMaxM], sB[kMaxM], sWX[2];
    const int tid = threadIdx.x;
    if (tid < nv) {
        sA[tid] = cA[tid];
        sB[tid] = cB[tid];
    }
    if (tid == 0) {
        sWX[0] = cB[kScalW];
        sWX[1] = cB[kScalX];
    }
    __syncthreads();
    const double cw = sWX[0], cx = sWX[1];
    constexpr int N = Vec16<T>::N;
    const size_t nsw = (r1 - r0) / (256 * N);
    for (size_t k = 0; k < nsw; ++k) {
        const size_t r = r0 + (k * 256 + tid) * N;
        double xv[N], wv[N], xn[N], wn[N];
        ld16(x + r, xv);
        ld16(w + r, wv);
#pragma unroll
        for (int e = 0; e < N; ++e) {
            xn[e] = xv[e];
            wn[e] = cw * wv[e] - cx * xv[e];
        }
        // batches of UB vectors loaded together (index clamped, coefficient 0
        // past the end), applied in ascending order
        constexpr int UB = 8;
        for (int i0 = 0; i0 < nv; i0 += UB) {
            double vv[UB][N];
#pragma unroll
            for (int u = 0; u < UB; ++u) ld16(V + (size_t)min(i0 + u, nv - 1) * stride + r, vv[u]);
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const bool in = i0 + u < nv;
                const double ca = in ? sA[min(i0 + u, nv - 1)] : 0.0;
                const double cb = in ? sB[min(i0 + u, nv - 1)] : 0.0;
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    xn[e] -= ca * vv[u][e];
                    wn[e] -= cb * vv[u][e];
                }
            }
        }
        if (wx) st16(x + r, xn);
        st16(w + r, wn);
    }
    for (size_t r = r0 + nsw * 256 * N + tid; r < r1; r += 256) {
        const double xs = (double)x[r];
        double xn = xs, wn = cw * (double)w[r] - cx * xs;
        for (int i = 0; i < nv; ++i) {
            const double u = (double)V[(size_t)i * stride + r];
            xn -= sA[i] * u;
            wn -= sB[i] * u;
        }
        if (wx) x[r] = (T)xn;
        w[r] = (T)wn;
    }
}

// Lane l of nl over L rows starts at row (l L / nl) rounded down to a multiple
// of 1024; the last lane ends at L.
__device__ __host__ __forceinline__ size_t lane_start(int l, int nl, size_t L) {
    return l >= nl ? L : ((size_t)l * L / (size_t)nl) / 1024 * 1024;
}

// Block b takes lane l = b % nl and in it the chunk that is (b / nl)-th from
// the lane's end: chunks of rpb rows, the lane's last chunk taking the rest
// of the lane.  Lane starts and rpb are multiples of 1024, so every chunk
// starts on a whole sweep.
template <typename T>
__global__ __launch_bounds__(256) void dcgs_update_kernel(const T *__restrict__ V, size_t stride,
                                                          int nv, const double *cA,
                                                          const double *cB, T *__restrict__ x,
                                                          T *__restrict__ w, size_t L,
                                                          size_t rpb, int nl, int wx) {
    const int l = (int)(blockIdx.x % (unsigned)nl), back = (int)(blockIdx.x / (unsigned)nl);
    const size_t s0 = lane_start(l, nl, L), len = lane_start(l + 1, nl, L) - s0;
    const size_t nch = (len / rpb > 0) ? len / rpb : 1;
    if ((size_t)back >= nch) return;
    const size_t j = nch - 1 - (size_t)back;
    const size_t r0 = s0 + j * rpb, r1 = (j == nch - 1) ? s0 + len : r0 + rpb;
    dcgs_update_body<T>(V, stride, nv, cA, cB, x, w, r0, r1, wx != 0);
}

// Finish of step k with incomplete orthogonalization (window of L vectors):
// see launch_iop_finish.
struct IopFinish {
    double *S, *H;
    int k, k0, nw;
    double *coefA, *coefB;
    int *flags;
};

__device__ __forceinline__ void iop_finish_body(const double *part, int nrb, const IopFinish &f) {
    constexpr int NW = kFin2Threads / 64;
    __shared__ double sv[kPartRows];
    __shared__ double sw[NW];
    __shared__ double sbeta;
    const int k = f.k, nw = f.nw, k0 = f.k0, col = k - 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *H = f.H, *S = f.S;
    fin_row_sums(part, 2 * nw + 2, nrb, sv);
    __syncthreads();
    const double gam = sv[2 * nw], del = sv[2 * nw + 1];
    if (k == 1) {
        // x = u_0 is the start vector, its norm already known
        if (tid == 0) sbeta = 1.0 / S[0];
        __syncthreads();
    } else {
        // the explicit norm of the stored u_{k-1} finishes column k-2
        const double beta = sqrt(gam);
        double acc = 0.0;
        for (int r = wave; r < k; r += NW)
            for (int c = lane; c <= col; c += 64) {
                const double h = (r == k - 1 && c == col) ? beta
                                 : (r <= c + 1)           ? H[(size_t)r * LDH + c]
                                                          : 0.0;
                acc += h * h;
            }
        acc = wave_sum(acc);
        if (lane == 0) sw[wave] = acc;
        __syncthreads();
        if (tid == 0) {
            double s2 = 0.0;
            for (int q = 0; q < NW; ++q) s2 += sw[q];
            const double hf = sqrt(s2);
            if ((!isfinite(beta) || !isfinite(hf)) && f.flags[1] == 0) f.flags[1] = k - 1;
            const bool brk = beta <= 1e-12 * hf;
            if (brk) {
                H[(size_t)(k - 1) * LDH + col] = 0.0;
                S[k - 1] = 0.0;
                if (f.flags[0] == 0) f.flags[0] = k - 1;
            } else {
                H[(size_t)(k - 1) * LDH + col] = beta;
                S[k - 1] = 1.0 / beta;
            }
            sbeta = brk ? 1.0 : beta;  // after a breakdown the step only has to stay finite
        }
        __syncthreads();
    }
    const double bet = sbeta;
    // column k-1: h_i = v_i^T A v_{k-1} = S_i (u_i^T w) / beta over the window,
    // and the diagonal x^T w / beta^2; u_k = w / beta - sum_i h_i v_i - h_d x / beta
    if (tid < nw) {
        const double Sg = S[k0 + tid];
        const double h = Sg * sv[tid] / bet;
        H[(size_t)(k0 + tid) * LDH + (k - 1)] = h;
        f.coefA[tid] = 0.0;
        f.coefB[tid] = Sg * h;
    }
    if (tid == 0) {
        const double hd = del / (bet * bet);
        H[(size_t)(k - 1) * LDH + (k - 1)] = hd;
        f.coefB[kScalW] = 1.0 / bet;
        f.coefB[kScalX] = hd / bet;
    }
}

__global__ __launch_bounds__(kFin2Threads) void iop_finish_kernel(const double *part, int nrb,
                                                                  IopFinish f) {
    iop_finish_body(part, nrb, f);
}

template <typename T>
struct NormArgs {
    const T *x[4];
};

template <typename T>
__global__ __launch_bounds__(256) void norms_kernel(NormArgs<T> a, int nx, size_t n, size_t rpb,
                                                    double *part) {
    __shared__ double sred[4][4];
    const int tid = threadIdx.x;
    const size_t r0 = (size_t)blockIdx.x * rpb;
    const size_t r1 = (r0 + rpb < n) ? r0 + rpb : n;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t r = r0 + tid; r < r1; r += 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nx && a.x[k]) {
                const double v = (double)a.x[k][r];
                acc[k] += v * v;
            }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double s = wave_sum(acc[k]);
        if ((tid & 63) == 0) sred[k][tid >> 6] = s;
    }
    __syncthreads();
    if (tid < 4)
        part[(size_t)tid * gridDim.x + blockIdx.x] =
            (sred[tid][0] + sred[tid][1]) + (sred[tid][2] + sred[tid][3]);
}

__global__ __launch_bounds__(256) void norms_finish_kernel(const double *part, int nblk,
                                                           double *out) {
    __shared__ double sw[4];
    const int tid = threadIdx.x;
    double a = 0.0;
    for (int b = tid; b < nblk; b += 256) a += part[(size_t)blockIdx.x * nblk + b];
    a = wave_sum(a);
    if ((tid & 63) == 0) sw[tid >> 6] = a;
    __syncthreads();
    if (tid == 0) out[blockIdx.x] = sqrt((sw[0] + sw[1]) + (sw[2] + sw[3]));
}

// ---- small dense exponential in LDS -----------------------------------------
constexpr int NMAX = kMaxM + 1;
constexpr int LDA = NMAX;  // LDS row stride (doubles)

// C = A * B, or C += A * B with ACC (n x n in LDS, row stride LDA; C may alias
// A or B: every operand is read before the first store).  The 256 threads
// form a 16 x 16 grid; thread (ty, tx) owns rows ty + 16 a and columns
// tx + 16 b (a, b < TILE), so a wave reads 16 consecutive B columns and
// broadcasts A.  The operands of four consecutive k are loaded together before
// their products are added, so LDS latency is paid once per four k; each entry
// is still summed over k in ascending order.
template <int TILE, bool ACC>
__device__ __forceinline__ void mm_tile(const double *A, const double *B, double *C, int n) {
    n = __builtin_amdgcn_readfirstlane(n);  // uniform: scalar loop control
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    double acc[TILE][TILE];
    int ra[TILE], cb[TILE];
#pragma unroll
    for (int a = 0; a < TILE; ++a) {
        ra[a] = min(ty + 16 * a, n - 1) * LDA;
        cb[a] = min(tx + 16 * a, n - 1);
#pragma unroll
        for (int b = 0; b < TILE; ++b) acc[a][b] = 0.0;
    }
    constexpr int U = 4;
    int q = 0;
    for (; q + U <= n; q += U) {
        double av[U][TILE], bv[U][TILE];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int a = 0; a < TILE; ++a) av[u][a] = A[ra[a] + q + u];
#pragma unroll
            for (int b = 0; b < TILE; ++b) bv[u][b] = B[(q + u) * LDA + cb[b]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int a = 0; a < TILE; ++a)
#pragma unroll
                for (int b = 0; b < TILE; ++b) acc[a][b] += av[u][a] * bv[u][b];
    }
    for (; q < n; ++q) {
        double av[TILE], bv[TILE];
#pragma unroll
        for (int a = 0; a < TILE; ++a) av[a] = A[ra[a] + q];
#pragma unroll
        for (int b = 0; b < TILE; ++b) bv[b] = B[q * LDA + cb[b]];
#pragma unroll
        for (int a = 0; a < TILE; ++a)
#pragma unroll
            for (int b = 0; b < TILE; ++b) acc[a][b] += av[a] * bv[b];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < TILE; ++a)
#pragma unroll
        for (int b = 0; b < TILE; ++b) {
            const int r = ty + 16 * a, c = tx + 16 * b;
            if (r < n && c < n) C[r * LDA + c] = ACC ? C[r * LDA + c] + acc[a][b] : acc[a][b];
        }
    __syncthreads();
}

template <bool ACC = false>
__device__ __forceinline__ void matmul(const double *A, const double *B, double *C, int n) {
    n = __builtin_amdgcn_readfirstlane(n);
    if (n <= 16)
        mm_tile<1, ACC>(A, B, C, n);
    else if (n <= 32)
        mm_tile<2, ACC>(A, B, C, n);
    else if (n <= 48)
        mm_tile<3, ACC>(A, B, C, n);
    else if (n <= 64)
        mm_tile<4, ACC>(A, B, C, n);
    else
        mm_tile<5, ACC>(A, B, C, n);
}

// Diagonal Pade (6,6) approximant of exp(X), X (n x n) in sX, after scaling X
// by 2^-s with s from its infinity norm.  The numerator and denominator are
// formed from their even and odd parts, E = c0 I + c2 X^2 + c4 X^4 + c6 X^6
// and O = X (c1 I + c3 X^2 + c5 X^4), as N = E + O (sN) and D = E - O (sD):
// four products instead of six.  Returns s.
__device__ __forceinline__ int expm_pade(double *sX, double *sP, double *sN, double *sD, int n) {
    n = __builtin_amdgcn_readfirstlane(n);  // the same in every lane: scalar control flow
    __shared__ double swm[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // infinity norm
    double rs = 0.0;
    if (tid < n)
        for (int c = 0; c < n; ++c) rs += fabs(sX[tid * LDA + c]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off, 64));
    if (lane == 0) swm[wave] = rs;
    __syncthreads();
    const double nrm = fmax(fmax(swm[0], swm[1]), fmax(swm[2], swm[3]));
    int s = 0;
    if (nrm > 0.5) s = max(0, (int)ceil(log2(nrm / 0.5)));
    const double scale = ldexp(1.0, -s);
    for (int r = wave; r < n; r += 4)
        for (int c = lane; c < n; c += 64) sX[r * LDA + c] *= scale;
    __syncthreads();
    // Pade coefficients c_k = c_{k-1} (q - k + 1) / (k (2q - k + 1)), q = 6
    double cf[7];
    cf[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= 6; ++k) cf[k] = cf[k - 1] * (6 - k + 1) / (double)(k * (12 - k + 1));
    matmul(sX, sX, sP, n);  // X^2
    matmul(sP, sP, sN, n);  // X^4
    matmul(sN, sP, sD, n);  // X^6
    for (int r = wave; r < n; r += 4)
        for (int c = lane; c < n; c += 64) {
            const double id = (r == c) ? 1.0 : 0.0;
            const double x2 = sP[r * LDA + c], x4 = sN[r * LDA + c], x6 = sD[r * LDA + c];
            sD[r * LDA + c] = cf[0] * id + cf[2] * x2 + cf[4] * x4 + cf[6] * x6;  // even part
            sN[r * LDA + c] = cf[1] * id + cf[3] * x2 + cf[5] * x4;                // odd / X
        }
    __syncthreads();
    matmul(sX, sN, sP, n);  // odd part
    for (int r = wave; r < n; r += 4)
        for (int c = lane; c < n; c += 64) {
            const double ev = sD[r * LDA + c], od = sP[r * LDA + c];
            sN[r * LDA + c] = ev + od;
            sD[r * LDA + c] = ev - od;
        }
    __syncthreads();
    return s;
}

// R = D^-1 N into sN, with matrix products only.  After the scaling,
// ||X||_inf <= 1/2, so F = I - D = -sum_{k>=1} (-1)^k c_k X^k has
// ||F||_inf <= sum_{k>=1} c_k 2^-k < 0.2805 and
//   D^-1 = (I + F)(I + F^2)(I + F^4)(I + F^8)(I + F^16) + F^32 D^-1,
// where the last term is below 0.2805^32 / (1 - 0.2805) < 3e-18 relative, under
// the FP64 rounding of the products.  The factors are applied to N one after
// the other (R <- R + F^(2^m) R) while F is squared, nine products in all and
// no sequential elimination.  sD holds F, and sX (free after the Pade step)
// takes every other power of it.
__device__ __forceinline__ void expm_solve(double *sX, double *sD, double *sN, int n) {
    n = __builtin_amdgcn_readfirstlane(n);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int r = wave; r < n; r += 4)
        for (int c = lane; c < n; c += 64) {
            const double id = (r == c) ? 1.0 : 0.0;
            sD[r * LDA + c] = id - sD[r * LDA + c];
        }
    __syncthreads();
    double *f = sD, *g = sX;
    for (int m = 0; m < 5; ++m) {
        matmul<true>(f, sN, sN, n);  // R += F^(2^m) R
        if (m < 4) {
            matmul(f, f, g, n);
            double *t = f;
            f = g;
            g = t;
        }
    }
}

// s squarings of R (in sN), alternating between sN and sP; returns the buffer
// that holds the result.  With col0 only the first column of the result is
// formed: the last squaring becomes a product with one column.
__device__ __forceinline__ double *expm_square(double *sN, double *sP, int n, int s, bool col0) {
    n = __builtin_amdgcn_readfirstlane(n);
    s = __builtin_amdgcn_readfirstlane(s);
    col0 = __builtin_amdgcn_readfirstlane((int)col0) != 0;
    const int tid = threadIdx.x;
    double *cur = sN, *nxt = sP;
    const int full = col0 ? s - 1 : s;
    for (int k = 0; k < full; ++k) {
        matmul(cur, cur, nxt, n);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (col0 && s > 0) {
        double acc = 0.0;
        if (tid < n)
            for (int q = 0; q < n; ++q) acc += cur[tid * LDA + q] * cur[q * LDA];
        if (tid < n) nxt[tid * LDA] = acc;
        __syncthreads();
        cur = nxt;
    }
    return cur;
}

// E = expm(X) for X (n x n) in sX (overwritten): Pade (6,6), the solve for its
// rational form, squarings.  Returns the buffer (sN or sP) that holds E (only
// its first column with col0); *s = number of squarings.
__device__ __forceinline__ double *lds_expm(double *sX, double *sP, double *sN, double *sD, int n,
                                            bool col0, int *s) {
    *s = expm_pade(sX, sP, sN, sD, n);
    expm_solve(sX, sD, sN, n);
    return expm_square(sN, sP, n, *s, col0);
}

// Small exponential of one check; writes the slot (error, the singular flag,
// which stays 0 because the scaled Pade denominator is always invertible, the
// Krylov flags as of this launch, squarings, combine coefficients) and the
// first kSummary header values to the item's host-mapped report, if any.
__device__ __forceinline__ void hess_expm_body(const ExpmItem &c) {
    extern __shared__ double smem[];
    double *sX = smem, *sP = sX + NMAX * LDA, *sN = sP + NMAX * LDA, *sD = sN + NMAX * LDA;
    const int j = c.j;
    const double dtau = c.dtau;
    const double *H = c.H;
    double *slot = c.slot;
    const int n = j + 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = wave; r < n; r += 4)
        for (int col = lane; col < n; col += 64)
            sX[r * LDA + col] = (col < j) ? dtau * H[(size_t)r * LDH + col] : 0.0;
    __syncthreads();
    int s = 0;
    const double *E = lds_expm(sX, sP, sN, sD, n, true, &s);
    __syncthreads();
    const double beta = c.res[0];
    if (threadIdx.x == 0) {
        const double hdr[kSlotHeader] = {beta * fabs(E[j * LDA + 0]), 0.0, (double)c.flags[0],
                                         (double)c.flags[1], (double)s};
        for (int k = 0; k < kSlotHeader; ++k) slot[k] = hdr[k];
        if (c.report)
            for (int k = 0; k < kSummary; ++k) c.report[k] = hdr[k];
    }
    for (int i = threadIdx.x; i < j; i += 256) slot[kSlotCoef + i] = beta * E[i * LDA + 0] * c.S[i];
}

__global__ __launch_bounds__(256) void hess_expm_kernel(ExpmItem c) { hess_expm_body(c); }

// One workgroup per check.
__global__ __launch_bounds__(256) void hess_expm_group(const ExpmItem *items) {
    hess_expm_body(items[blockIdx.x]);
}

__global__ __launch_bounds__(256) void dense_expm_kernel(const double *A, int n, double *E) {
    extern __shared__ double smem[];
    double *sX = smem, *sP = sX + NMAX * LDA, *sN = sP + NMAX * LDA, *sD = sN + NMAX * LDA;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = wave; r < n; r += 4)
        for (int c = lane; c < n; c += 64) sX[r * LDA + c] = A[(size_t)r * n + c];
    __syncthreads();
    int s = 0;
    const double *R = lds_expm(sX, sP, sN, sD, n, false, &s);
    __syncthreads();
    for (int r = wave; r < n; r += 4)
        for (int c = lane; c < n; c += 64) E[(size_t)r * n + c] = R[r * LDA + c];
}

template <typename T>
__global__ __launch_bounds__(256) void combine_kernel(const T *V, size_t stride, int m,
                                                      const double *ccoef, T *z, size_t L) {
    __shared__ double sc[kMaxM];
    if ((int)threadIdx.x < m) sc[threadIdx.x] = ccoef[threadIdx.x];
    __syncthreads();
    constexpr int N = Vec16<T>::N;
    const size_t Lv = L / N * N;  // rows covered by full 16-byte vectors
    for (size_t r = ((size_t)blockIdx.x * 256 + threadIdx.x) * N; r < Lv;
         r += (size_t)gridDim.x * 256 * N) {
        double acc[N];
#pragma unroll
        for (int e = 0; e < N; ++e) acc[e] = 0.0;
        // batches of UB basis rows loaded together (index clamped,
        // coefficient 0 past the end), summed in ascending order
        constexpr int UB = 8;
        for (int i0 = 0; i0 < m; i0 += UB) {
            double vv[UB][N];
#pragma unroll
            for (int u = 0; u < UB; ++u) ld16(V + (size_t)min(i0 + u, m - 1) * stride + r, vv[u]);
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const double c = (i0 + u < m) ? sc[min(i0 + u, m - 1)] : 0.0;
#pragma unroll
                for (int e = 0; e < N; ++e) acc[e] += c * vv[u][e];
            }
        }
        st16(z + r, acc);
    }
    if (blockIdx.x == 0)
        for (size_t r = Lv + threadIdx.x; r < L; r += 256) {
            double acc = 0.0;
            for (int i = 0; i < m; ++i) acc += sc[i] * (double)V[(size_t)i * stride + r];
            z[r] = (T)acc;
        }
}

// ---- grouped launches: one launch serves the same Arnoldi step of many
// independent solves.  Item it owns blocks [bstart[it], bstart[it+1]); an item
// with no blocks in a launch is skipped.  Each item computes exactly what its
// own single launch computes (same row partition, same block partials).
__global__ __launch_bounds__(256) void gs_dots2_group(const GsItem *items, const int *bstart,
                                                      int n) {
    const int it = group_item(bstart, n, blockIdx.x);
    const GsItem &g = items[it];
    const int local = blockIdx.x - bstart[it];
    gs_dots2_body<double>(g.V + (size_t)g.k0 * g.stride, g.stride, g.nv, g.x, g.w, g.L, g.rpb,
                          g.nrb, g.part, local % g.nrb, local / g.nrb);
}

// Fold of the items with nfold > 0: item it owns (2 nv + 2) nfold blocks,
// block (r, c) of the item folding chunk c of row r as fold_kernel does.
__global__ __launch_bounds__(256) void fold_group(const GsItem *items, const int *bstart, int n) {
    const int it = group_item(bstart, n, blockIdx.x);
    const GsItem &g = items[it];
    const int local = blockIdx.x - bstart[it];
    fold_body(g.part, g.nrb1, g.fold, g.nfold, local / g.nfold, local % g.nfold);
}

// One workgroup per item; nrb1 partials per row from the linear operator's
// blocks (nfold per row once folded), or (nrb1 = 0) nrb from the separate dot
// pass.
__global__ __launch_bounds__(kFin2Threads) void dcgs_finish_group(const GsItem *items) {
    const GsItem &g = items[blockIdx.x];
    const int nrb = g.nfold > 0 ? g.nfold : (g.nrb1 > 0 ? g.nrb1 : g.nrb);
    const double *part = g.nfold > 0 ? g.fold : g.part;
    if (g.iop)
        iop_finish_body(part, nrb, IopFinish{g.S, g.H, g.k, g.k0, g.nv, g.coefA, g.coefB, g.flags});
    else
        dcgs_finish_body(part, nrb, DcgsFinish{g.S, g.H, g.k, g.coefA, g.coefB, g.flags});
}

__global__ __launch_bounds__(256) void dcgs_update_group(const GsItem *items, const int *bstart,
                                                         int n) {
    const int it = group_item(bstart, n, blockIdx.x);
    const GsItem &g = items[it];
    // incomplete orthogonalization leaves x as it is (only its scale is new)
    const size_t r0 = (size_t)(blockIdx.x - bstart[it]) * g.rpb;
    const size_t r1 = (r0 + g.rpb < g.L) ? r0 + g.rpb : g.L;
    dcgs_update_body<double>(g.V + (size_t)g.k0 * g.stride, g.stride, g.nv, g.coefA, g.coefB,
                             g.x, g.w, r0, r1, g.k > 1 && !g.iop);
}

constexpr size_t kExpmLds = (size_t)4 * NMAX * LDA * sizeof(double);

// Allow the dynamic LDS of the exponential kernels (above the 64 KB default
// of older targets); the attribute call is harmless where it is not needed.
void allow_expm_lds() {
    (void)hipFuncSetAttribute((const void *)hess_expm_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kExpmLds);
    (void)hipFuncSetAttribute((const void *)hess_expm_group,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kExpmLds);
    (void)hipFuncSetAttribute((const void *)dense_expm_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kExpmLds);
    (void)hipGetLastError();
}

}  // namespace

RowPartition row_partition(size_t L) {
    RowPartition p;
    size_t nrb = (L + 255) / 256;
    if (nrb > (size_t)kRedBlocks) nrb = kRedBlocks;
    if (nrb < 1) nrb = 1;
    size_t rpb = (L + nrb - 1) / nrb;
    rpb = (rpb + 1023) / 1024 * 1024;  // whole 16-byte sweeps for double and float
    p.rpb = rpb;
    p.nrb = (int)((L + rpb - 1) / rpb);
    if (p.nrb < 1) p.nrb = 1;
    return p;
}

template <typename T>
hipError_t launch_gs_dots2(const T *V, size_t stride, int nv, const T *x, const T *w, size_t L,
                           const RowPartition &rp, double *part, hipStream_t s) {
    if (nv < 0 || nv > kMaxM) return hipErrorInvalidValue;
    const dim3 grid(rp.nrb, nv > 0 ? (nv + CH - 1) / CH : 1);
    return launch_kernel(gs_dots2_kernel<T>, grid, dim3(256), 0, s, V, stride, nv, x, w, L,
                         rp.rpb, rp.nrb, part);
}

hipError_t launch_fold(const double *part, int nrb, int rows, double *out, hipStream_t s) {
    const int nc = fold_chunks(nrb);
    if (nc < 1 || rows < 1 || rows > kPartRows) return hipErrorInvalidValue;
    return launch_kernel(fold_kernel, dim3(nc, rows), dim3(256), 0, s, part, nrb, out, nc);
}

hipError_t launch_dcgs_finish(const double *part, int nrb, int k, double *S, double *H,
                              double *coefA, double *coefB, int *flags, hipStream_t s) {
    if (k < 1 || k > kMaxM + 1 || nrb < 1) return hipErrorInvalidValue;
    return launch_kernel(dcgs_finish_kernel, dim3(1), dim3(kFin2Threads), 0, s, part, nrb,
                         DcgsFinish{S, H, k, coefA, coefB, flags});
}

template <typename T>
hipError_t launch_dcgs_update(const T *V, size_t stride, int nv, const double *coefA,
                              const double *coefB, T *x, T *w, size_t L, const RowPartition &rp,
                              hipStream_t s, bool write_x, int lanes) {
    if (nv < 0 || nv > kMaxM || lanes < 1 || L < 1) return hipErrorInvalidValue;
    // the sweep has no partials: it may take more blocks than the reductions'
    // partition (whole 1024-row sweeps per block, the same rows in the scalar
    // tail, so the result does not depend on the split or on the order)
    const size_t rpb = std::max<size_t>(1024, (rp.rpb / kUpdateSplit + 1023) / 1024 * 1024);
    // lanes of at least 1024 rows (lane_start); the grid has as many chunks
    // per lane as the longest lane
    const int nl = (int)std::max<size_t>(1, std::min<size_t>((size_t)lanes, L / 1024));
    size_t nch = 1;
    for (int l = 0; l < nl; ++l)
        nch = std::max(nch, (lane_start(l + 1, nl, L) - lane_start(l, nl, L)) / rpb);
    const unsigned nb = (unsigned)(nch * nl);
    return launch_kernel(dcgs_update_kernel<T>, dim3(nb), dim3(256), 0, s, V, stride, nv,
                         coefA, coefB, x, w, L, rpb, nl, (write_x && nv > 0) ? 1 : 0);
}

hipError_t launch_iop_finish(const double *part, int nrb, int k, int k0, int nw, double *S,
                             double *H, double *coefA, double *coefB, int *flags, hipStream_t s) {
    if (k < 1 || k > kMaxM + 1 || nrb < 1 || nw < 0 || k0 < 0 || k0 + nw != k - 1)
        return hipErrorInvalidValue;
    return launch_kernel(iop_finish_kernel, dim3(1), dim3(kFin2Threads), 0, s, part, nrb,
                         IopFinish{S, H, k, k0, nw, coefA, coefB, flags});
}

template <typename T>
hipError_t launch_gs_norm(const T *z, size_t L, const RowPartition &rp, double *part,
                          hipStream_t s) {
    return launch_kernel(gs_norm_kernel<T>, dim3(rp.nrb), dim3(256), 0, s, z, L, rp.rpb, part);
}

hipError_t launch_gs_finish_norm(const double *part, const RowPartition &rp, double *H, double *S,
                                 int *flags, double *res, hipStream_t s) {
    return launch_kernel(finish_norm_kernel, dim3(1), dim3(256), 0, s, part, rp.nrb,
                         NormFinish{H, S, flags, res});
}

#define EXPDG_INST(T)                                                                          \
    template hipError_t launch_gs_dots2<T>(const T *, size_t, int, const T *, const T *, size_t, \
                                           const RowPartition &, double *, hipStream_t);        \
    template hipError_t launch_dcgs_update<T>(const T *, size_t, int, const double *,           \
                                              const double *, T *, T *, size_t,                 \
                                              const RowPartition &, hipStream_t, bool, int);    \
    template hipError_t launch_gs_norm<T>(const T *, size_t, const RowPartition &, double *,    \
                                          hipStream_t);
EXPDG_INST(double)
EXPDG_INST(float)
#undef EXPDG_INST

template <typename T>
hipError_t launch_norms(const T *const *x, int nx, size_t n, double *part, double *out,
                        hipStream_t s) {
    if (nx < 1 || nx > 4) return hipErrorInvalidValue;
    NormArgs<T> a;
    for (int k = 0; k < 4; ++k) a.x[k] = (k < nx) ? x[k] : nullptr;
    const RowPartition rp = row_partition(n);
    norms_kernel<T><<<rp.nrb, 256, 0, s>>>(a, nx, n, rp.rpb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    norms_finish_kernel<<<nx, 256, 0, s>>>(part, rp.nrb, out);
    return hipGetLastError();
}
template hipError_t launch_norms<double>(const double *const *, int, size_t, double *, double *,
                                         hipStream_t);
template hipError_t launch_norms<float>(const float *const *, int, size_t, double *, double *,
                                        hipStream_t);

hipError_t launch_hess_expm(const ExpmItem &c, hipStream_t s) {
    if (c.j < 1 || c.j > kMaxM) return hipErrorInvalidValue;
    static bool once = (allow_expm_lds(), true);
    (void)once;
    return launch_kernel(hess_expm_kernel, dim3(1), dim3(256), (unsigned)kExpmLds, s, c);
}

hipError_t launch_hess_expm_group(const ExpmItem *items, int n, hipStream_t s) {
    if (n < 1) return hipErrorInvalidValue;
    static bool once = (allow_expm_lds(), true);
    (void)once;
    return launch_kernel(hess_expm_group, dim3(n), dim3(256), (unsigned)kExpmLds, s, items);
}

void arnoldi_group_layout(const GsItem *items, int n, int *bstart, int *totals) {
    int t[kGroupLaunches] = {};
    for (int it = 0; it < n; ++it) {
        const GsItem &g = items[it];
        const int nv = g.nv;
        const int chunks = nv > 0 ? (nv + CH - 1) / CH : 1;
        const int blocks[kGroupLaunches] = {g.nrb1 > 0 ? 0 : g.nrb * chunks,
                                            g.nfold > 0 ? (2 * nv + 2) * g.nfold : 0, g.nrb};
        for (int k = 0; k < kGroupLaunches; ++k) {
            bstart[k * (n + 1) + it] = t[k];
            t[k] += blocks[k];
        }
    }
    for (int k = 0; k < kGroupLaunches; ++k) {
        bstart[k * (n + 1) + n] = t[k];
        totals[k] = t[k];
    }
}

hipError_t launch_arnoldi_group(const GsItem *items, const int *bstart, const int *totals, int n,
                                hipStream_t s) {
    if (n < 1) return hipErrorInvalidValue;
    const int *b[kGroupLaunches];
    for (int k = 0; k < kGroupLaunches; ++k) b[k] = bstart + (size_t)k * (n + 1);
    hipError_t e;
    // dot pass of the items whose linear operator does not carry it
    if (totals[0] > 0) {
        e = launch_kernel(gs_dots2_group, dim3(totals[0]), dim3(256), 0, s, items, b[0], n);
        if (e != hipSuccess) return e;
    }
    // fold of the long partial rows of large meshes
    if (totals[1] > 0) {
        e = launch_kernel(fold_group, dim3(totals[1]), dim3(256), 0, s, items, b[1], n);
        if (e != hipSuccess) return e;
    }
    e = launch_kernel(dcgs_finish_group, dim3(n), dim3(kFin2Threads), 0, s, items);
    if (e != hipSuccess) return e;
    return launch_kernel(dcgs_update_group, dim3(totals[2]), dim3(256), 0, s, items, b[2], n);
}

hipError_t launch_dense_expm(const double *A, int n, double *E, hipStream_t s) {
    if (n < 1 || n > NMAX) return hipErrorInvalidValue;
    static bool once = (allow_expm_lds(), true);
    (void)once;
    dense_expm_kernel<<<1, 256, kExpmLds, s>>>(A, n, E);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_combine(const T *V, size_t stride, int m, const double *ccoef, T *z, size_t L,
                          hipStream_t s) {
    if (m < 1 || m > kMaxM) return hipErrorInvalidValue;
    size_t g = (L + 255) / 256;
    if (g > 4096) g = 4096;
    return launch_kernel(combine_kernel<T>, dim3((unsigned)g), dim3(256), 0, s, V, stride, m,
                         ccoef, z, L);
}
template hipError_t launch_combine<double>(const double *, size_t, int, const double *, double *,
                                           size_t, hipStream_t);
template hipError_t launch_combine<float>(const float *, size_t, int, const double *, float *,
                                          size_t, hipStream_t);

}  // namespace expdg
