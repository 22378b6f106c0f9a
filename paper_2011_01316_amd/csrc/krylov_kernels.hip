// Arnoldi / Krylov kernels for gfx950 (Section 2.3: Krylov projection of the
// augmented matrix; classical Gram-Schmidt applied twice).
//
// Basis storage: V holds unnormalised vectors u_i (bulk type, float or
// double) with FP64 scales S[i] so that v_i = S[i] u_i; no separate
// normalisation pass is needed.  Inner products and norms are accumulated in
// FP64 with a fixed two-stage reduction (per-block partials over a fixed row
// partition, then a fixed-order tree), so results do not depend on timing and
// are identical run to run.
//
// The small (j+1) x (j+1) exponential of the projected Hessenberg matrix
// runs in one 256-thread workgroup with four FP64 matrices resident in LDS
// (gfx950 gives a workgroup up to 160 KB): diagonal Pade (6,6) with scaling
// and squaring and Gaussian elimination with partial pivoting.
#include "internal.h"

namespace expdg {
namespace {

constexpr int LDH = kMaxM;  // leading dimension of H

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Row partition shared by every row-partitioned kernel: block b owns rows
// [b*rpb, min(L, (b+1)*rpb)); rpb is a multiple of 256.
__host__ __device__ inline size_t rows_per_block(size_t L) {
    size_t rpb = (L + kRedBlocks - 1) / kRedBlocks;
    rpb = (rpb + 255) / 256 * 256;
    return rpb;
}

// mode 0: part[i*nblk + b] = sum_r V_i[r] w'[r] (i < nv)
// mode 1: part[b]          = sum_r w'[r]^2
// where w' = w - sum_i coef[i] V_i (coef may be nullptr: w' = w); if coef is
// given, w' is stored back.
template <typename T, int NVMAX, int MODE>
__global__ __launch_bounds__(256) void cgs_kernel(const T *__restrict__ V, size_t stride, int nv,
                                                  const double *__restrict__ coef,
                                                  T *__restrict__ w, size_t L, size_t rpb,
                                                  double *__restrict__ part) {
    __shared__ double scoef[NVMAX];
    __shared__ double sred[NVMAX > 0 ? NVMAX : 1][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (coef && tid < nv) scoef[tid] = coef[tid];
    __syncthreads();
    const size_t r0 = (size_t)blockIdx.x * rpb;
    const size_t r1 = (r0 + rpb < L) ? r0 + rpb : L;
    double acc[MODE == 0 ? NVMAX : 1];
#pragma unroll
    for (int i = 0; i < (MODE == 0 ? NVMAX : 1); ++i) acc[i] = 0.0;
    for (size_t r = r0 + tid; r < r1; r += 256) {
        double x = (double)w[r];
        if (coef) {
#pragma unroll
            for (int i = 0; i < NVMAX; ++i)
                if (i < nv) x -= scoef[i] * (double)V[(size_t)i * stride + r];
            w[r] = (T)x;
            x = (double)(T)x;
        }
        if (MODE == 0) {
#pragma unroll
            for (int i = 0; i < NVMAX; ++i)
                if (i < nv) acc[i] += (double)V[(size_t)i * stride + r] * x;
        } else {
            acc[0] += x * x;
        }
    }
    const int nout = (MODE == 0) ? nv : 1;
#pragma unroll
    for (int i = 0; i < (MODE == 0 ? NVMAX : 1); ++i) {
        if (i < nout) {
            const double s = wave_sum(acc[i]);
            if (lane == 0) sred[i][wave] = s;
        }
    }
    __syncthreads();
    if (tid < nout) {
        const double s = (sred[tid][0] + sred[tid][1]) + (sred[tid][2] + sred[tid][3]);
        part[(size_t)tid * gridDim.x + blockIdx.x] = s;
    }
}

// Fixed-order sum of nblk partials by one block; returns the total to all.
__device__ double block_sum_partials(const double *p, int nblk) {
    __shared__ double sw[4];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int b = tid; b < nblk; b += 256) acc += p[b];
    acc = wave_sum(acc);
    if ((tid & 63) == 0) sw[tid >> 6] = acc;
    __syncthreads();
    const double t = (sw[0] + sw[1]) + (sw[2] + sw[3]);
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(256) void dot_finish_kernel(const double *part, int nblk,
                                                         const double *S, double *H, int col,
                                                         int accumulate, double *coef) {
    const int i = blockIdx.x;
    const double t = block_sum_partials(part + (size_t)i * nblk, nblk);
    if (threadIdx.x == 0) {
        const double h = S[i] * t;
        double *hij = &H[(size_t)i * LDH + col];
        *hij = accumulate ? *hij + h : h;
        coef[i] = h * S[i];
    }
}

__global__ __launch_bounds__(256) void norm_finish_kernel(const double *part, int nblk, double *H,
                                                          double *S, int col, int *flags) {
    __shared__ double sw[4];
    const double t = block_sum_partials(part, nblk);
    const double hn = sqrt(t);
    // ||H_{0:col+2, 0:col+1}||_F including the new subdiagonal entry
    double acc = 0.0;
    const int rows = col + 2, cols = col + 1;
    for (int e = threadIdx.x; e < rows * cols; e += 256) {
        const int r = e / cols, c = e % cols;
        const double h = (r == col + 1) ? ((c == col) ? hn : 0.0) : H[(size_t)r * LDH + c];
        acc += h * h;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double hf = sqrt((sw[0] + sw[1]) + (sw[2] + sw[3]));
        if (!isfinite(hn) || !isfinite(hf)) flags[1] = 1;
        const bool brk = hn <= 1e-12 * hf;
        if (brk) {
            H[(size_t)(col + 1) * LDH + col] = 0.0;
            S[col + 1] = 0.0;
            if (flags[0] == 0) flags[0] = col + 1;
        } else {
            H[(size_t)(col + 1) * LDH + col] = hn;
            S[col + 1] = 1.0 / hn;
        }
    }
}

__global__ __launch_bounds__(256) void beta_finish_kernel(const double *part, int nblk, double *S,
                                                          double *res, int *flags) {
    const double t = block_sum_partials(part, nblk);
    if (threadIdx.x == 0) {
        const double beta = sqrt(t);
        res[0] = beta;
        S[0] = (beta > 0.0) ? 1.0 / beta : 0.0;
        flags[0] = 0;
        if (!isfinite(beta)) flags[1] = 1;
    }
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
    if (tid < 4) part[(size_t)tid * gridDim.x + blockIdx.x] =
        (sred[tid][0] + sred[tid][1]) + (sred[tid][2] + sred[tid][3]);
}

__global__ __launch_bounds__(256) void norms_finish_kernel(const double *part, int nblk,
                                                           double *out) {
    const double t = block_sum_partials(part + (size_t)blockIdx.x * nblk, nblk);
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(t);
}

// ---- small dense exponential in LDS -----------------------------------------
constexpr int NMAX = kMaxM + 1;
constexpr int LDA = NMAX;  // LDS row stride (doubles)

// C = A * B for n x n matrices in LDS (C may alias A or B): results are held
// in registers until every thread has read its operands.
__device__ void lds_matmul(const double *A, const double *B, double *C, int n) {
    constexpr int PER = (NMAX * NMAX + 255) / 256;
    double t[PER];
    const int tot = n * n;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        double acc = 0.0;
        if (e < tot) {
            const int r = e / n, c = e - (e / n) * n;
            for (int q = 0; q < n; ++q) acc += A[r * LDA + q] * B[q * LDA + c];
        }
        t[k] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        if (e < tot) {
            const int r = e / n, c = e - (e / n) * n;
            C[r * LDA + c] = t[k];
        }
    }
    __syncthreads();
}

// E = expm(X) for X (n x n) already in sX; result left in sN.  Returns the
// number of squarings; sets *singular if the Pade denominator is singular.
__device__ int lds_expm(double *sX, double *sP, double *sN, double *sD, int n, int *singular) {
    __shared__ double sred[256];
    __shared__ int spiv;
    __shared__ double sf[NMAX];
    const int tid = threadIdx.x;
    // infinity norm
    double rs = 0.0;
    if (tid < n)
        for (int c = 0; c < n; ++c) rs += fabs(sX[tid * LDA + c]);
    sred[tid] = rs;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) sred[tid] = fmax(sred[tid], sred[tid + w]);
        __syncthreads();
    }
    const double nrm = sred[0];
    __syncthreads();
    int s = 0;
    if (nrm > 0.5) s = max(0, (int)ceil(log2(nrm / 0.5)));
    const double scale = ldexp(1.0, -s);
    for (int e = tid; e < n * n; e += 256) {
        const int r = e / n, c = e % n;
        sX[r * LDA + c] *= scale;
        const double id = (r == c) ? 1.0 : 0.0;
        sP[r * LDA + c] = id;
        sN[r * LDA + c] = id;
        sD[r * LDA + c] = id;
    }
    __syncthreads();
    double cf = 1.0;
    const int q = 6;
    for (int k = 1; k <= q; ++k) {
        cf = cf * (q - k + 1) / (double)(k * (2 * q - k + 1));
        lds_matmul(sX, sP, sP, n);
        const double sg = (k % 2 == 0) ? 1.0 : -1.0;
        for (int e = tid; e < n * n; e += 256) {
            const int r = e / n, c = e % n;
            const double pv = sP[r * LDA + c];
            sN[r * LDA + c] += cf * pv;
            sD[r * LDA + c] += sg * cf * pv;
        }
        __syncthreads();
    }
    // solve D F = N (partial pivoting, first maximal row on ties)
    for (int k = 0; k < n; ++k) {
        if (tid < 64) {
            double best = -1.0;
            int bi = n;
            for (int r = k + tid; r < n; r += 64) {
                const double v = fabs(sD[r * LDA + k]);
                if (v > best) {
                    best = v;
                    bi = r;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            if (tid == 0) spiv = bi;
        }
        __syncthreads();
        const int piv = spiv;
        if (sD[piv * LDA + k] == 0.0) {
            if (tid == 0) *singular = 1;
            return s;
        }
        if (piv != k) {
            for (int c = tid; c < n; c += 256) {
                double t = sD[k * LDA + c];
                sD[k * LDA + c] = sD[piv * LDA + c];
                sD[piv * LDA + c] = t;
                t = sN[k * LDA + c];
                sN[k * LDA + c] = sN[piv * LDA + c];
                sN[piv * LDA + c] = t;
            }
            __syncthreads();
        }
        for (int r = k + 1 + tid; r < n; r += 256) sf[r] = sD[r * LDA + k] / sD[k * LDA + k];
        __syncthreads();
        const int rows = n - k - 1;
        for (int e = tid; e < rows * n; e += 256) {
            const int r = k + 1 + e / n, c = e % n;
            const double f = sf[r];
            if (c >= k) sD[r * LDA + c] -= f * sD[k * LDA + c];
            sN[r * LDA + c] -= f * sN[k * LDA + c];
        }
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        for (int c = tid; c < n; c += 256) {
            double acc = sN[k * LDA + c];
            for (int r = k + 1; r < n; ++r) acc -= sD[k * LDA + r] * sN[r * LDA + c];
            sN[k * LDA + c] = acc / sD[k * LDA + k];
        }
        __syncthreads();
    }
    for (int k = 0; k < s; ++k) lds_matmul(sN, sN, sN, n);
    return s;
}

__global__ __launch_bounds__(256) void hess_expm_kernel(const double *H, int j, double dtau,
                                                        const double *S, const double *res,
                                                        double *slot) {
    extern __shared__ double smem[];
    double *sX = smem, *sP = sX + NMAX * LDA, *sN = sP + NMAX * LDA, *sD = sN + NMAX * LDA;
    __shared__ int singular;
    const int n = j + 1;
    if (threadIdx.x == 0) singular = 0;
    for (int e = threadIdx.x; e < n * n; e += 256) {
        const int r = e / n, c = e % n;
        sX[r * LDA + c] = (c < j) ? dtau * H[(size_t)r * LDH + c] : 0.0;
    }
    __syncthreads();
    const int s = lds_expm(sX, sP, sN, sD, n, &singular);
    __syncthreads();
    const double beta = res[0];
    if (threadIdx.x == 0) {
        slot[kSlotErr] = beta * fabs(sN[j * LDA + 0]);
        slot[1] = (double)s;
        slot[2] = (double)singular;
    }
    for (int i = threadIdx.x; i < j; i += 256) slot[kSlotCoef + i] = beta * sN[i * LDA + 0] * S[i];
}

__global__ __launch_bounds__(256) void dense_expm_kernel(const double *A, int n, double *E) {
    extern __shared__ double smem[];
    double *sX = smem, *sP = sX + NMAX * LDA, *sN = sP + NMAX * LDA, *sD = sN + NMAX * LDA;
    __shared__ int singular;
    if (threadIdx.x == 0) singular = 0;
    for (int e = threadIdx.x; e < n * n; e += 256) sX[(e / n) * LDA + e % n] = A[e];
    __syncthreads();
    lds_expm(sX, sP, sN, sD, n, &singular);
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += 256)
        E[e] = singular ? __builtin_nan("") : sN[(e / n) * LDA + e % n];
}

template <typename T>
__global__ __launch_bounds__(256) void combine_kernel(const T *V, size_t stride, int m,
                                                      const double *ccoef, T *z, size_t L) {
    __shared__ double sc[kMaxM];
    if ((int)threadIdx.x < m) sc[threadIdx.x] = ccoef[threadIdx.x];
    __syncthreads();
    for (size_t r = (size_t)blockIdx.x * 256 + threadIdx.x; r < L; r += (size_t)gridDim.x * 256) {
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += sc[i] * (double)V[(size_t)i * stride + r];
        z[r] = (T)acc;
    }
}

constexpr size_t kExpmLds = (size_t)4 * NMAX * LDA * sizeof(double);

template <typename T, int NVMAX, int MODE>
hipError_t cgs_launch(const T *V, size_t stride, int nv, const double *coef, T *w, size_t L,
                      double *part, hipStream_t s) {
    const size_t rpb = rows_per_block(L);
    const int nblk = (int)((L + rpb - 1) / rpb);
    cgs_kernel<T, NVMAX, MODE><<<nblk, 256, 0, s>>>(V, stride, nv, coef, w, L, rpb, part);
    return hipGetLastError();
}

}  // namespace

int red_blocks(size_t L) {
    const size_t rpb = rows_per_block(L);
    return (int)((L + rpb - 1) / rpb);
}

template <typename T>
hipError_t launch_cgs_pass(const T *V, size_t stride, int nv, const double *coef, T *w, size_t L,
                           double *part, int mode, hipStream_t s) {
    if (nv < 0 || nv > kMaxM + 1) return hipErrorInvalidValue;
    if (mode == 1) {
        if (nv <= 8) return cgs_launch<T, 8, 1>(V, stride, nv, coef, w, L, part, s);
        if (nv <= 16) return cgs_launch<T, 16, 1>(V, stride, nv, coef, w, L, part, s);
        if (nv <= 32) return cgs_launch<T, 32, 1>(V, stride, nv, coef, w, L, part, s);
        return cgs_launch<T, kMaxM + 1, 1>(V, stride, nv, coef, w, L, part, s);
    }
    if (nv <= 8) return cgs_launch<T, 8, 0>(V, stride, nv, coef, w, L, part, s);
    if (nv <= 16) return cgs_launch<T, 16, 0>(V, stride, nv, coef, w, L, part, s);
    if (nv <= 32) return cgs_launch<T, 32, 0>(V, stride, nv, coef, w, L, part, s);
    return cgs_launch<T, kMaxM + 1, 0>(V, stride, nv, coef, w, L, part, s);
}
template hipError_t launch_cgs_pass<double>(const double *, size_t, int, const double *, double *,
                                            size_t, double *, int, hipStream_t);
template hipError_t launch_cgs_pass<float>(const float *, size_t, int, const double *, float *,
                                           size_t, double *, int, hipStream_t);

hipError_t launch_dot_finish(const double *part, int nblk, int nv, const double *S, double *H,
                             int col, int accumulate, double *coef, hipStream_t s) {
    dot_finish_kernel<<<nv, 256, 0, s>>>(part, nblk, S, H, col, accumulate, coef);
    return hipGetLastError();
}

hipError_t launch_norm_finish(const double *part, int nblk, double *H, double *S, int col,
                              int *flags, hipStream_t s) {
    norm_finish_kernel<<<1, 256, 0, s>>>(part, nblk, H, S, col, flags);
    return hipGetLastError();
}

hipError_t launch_beta_finish(const double *part, int nblk, double *S, double *res, int *flags,
                              hipStream_t s) {
    beta_finish_kernel<<<1, 256, 0, s>>>(part, nblk, S, res, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_norms(const T *const *x, int nx, size_t n, double *part, double *out,
                        hipStream_t s) {
    if (nx < 1 || nx > 4) return hipErrorInvalidValue;
    NormArgs<T> a;
    for (int k = 0; k < 4; ++k) a.x[k] = (k < nx) ? x[k] : nullptr;
    const size_t rpb = rows_per_block(n);
    const int nblk = (int)((n + rpb - 1) / rpb);
    norms_kernel<T><<<nblk, 256, 0, s>>>(a, nx, n, rpb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    norms_finish_kernel<<<nx, 256, 0, s>>>(part, nblk, out);
    return hipGetLastError();
}
template hipError_t launch_norms<double>(const double *const *, int, size_t, double *, double *,
                                         hipStream_t);
template hipError_t launch_norms<float>(const float *const *, int, size_t, double *, double *,
                                        hipStream_t);

// Allow the dynamic LDS of the exponential kernels (above the 64 KB default
// of older targets); the attribute call is harmless where it is not needed.
static void allow_expm_lds() {
    (void)hipFuncSetAttribute((const void *)hess_expm_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kExpmLds);
    (void)hipFuncSetAttribute((const void *)dense_expm_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kExpmLds);
    (void)hipGetLastError();
}

hipError_t launch_hess_expm(const double *H, int j, double dtau, const double *S,
                            const double *res_beta, double *slot, hipStream_t s) {
    if (j < 1 || j > kMaxM) return hipErrorInvalidValue;
    static bool once = (allow_expm_lds(), true);
    (void)once;
    hess_expm_kernel<<<1, 256, kExpmLds, s>>>(H, j, dtau, S, res_beta, slot);
    return hipGetLastError();
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
    combine_kernel<T><<<(int)g, 256, 0, s>>>(V, stride, m, ccoef, z, L);
    return hipGetLastError();
}
template hipError_t launch_combine<double>(const double *, size_t, int, const double *, double *,
                                           size_t, hipStream_t);
template hipError_t launch_combine<float>(const float *, size_t, int, const double *, float *,
                                          size_t, hipStream_t);

}  // namespace expdg
