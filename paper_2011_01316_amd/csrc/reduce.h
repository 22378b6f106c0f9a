// Wavefront reductions shared by the reduction kernels (gfx950, 64-wide
// waves).  Device code only.
#pragma once

#include <hip/hip_runtime.h>

namespace expdg {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One halving step of the transpose reduction: lanes with bit m set keep the
// upper half of a[0..2*HALF), the others the lower half; each adds the
// partner's copy of the half it keeps.
template <int HALF>
__device__ __forceinline__ void tr_step(double *a, int lane, int m) {
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int k = 0; k < HALF; ++k) {
        const double keep = up ? a[HALF + k] : a[k];
        const double send = up ? a[k] : a[HALF + k];
        a[k] = keep + __shfl_xor(send, m, 64);
    }
}

// Wave sums of a[0..16): lane l returns the sum of a[l >> 2].
__device__ __forceinline__ double transpose_reduce16(double *a) {
    const int lane = threadIdx.x & 63;
    tr_step<8>(a, lane, 32);
    tr_step<4>(a, lane, 16);
    tr_step<2>(a, lane, 8);
    tr_step<1>(a, lane, 4);
    double v = a[0];
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    return v;
}

// Wave sums of a[0..32): lane l returns the sum of a[l >> 1].
__device__ __forceinline__ double transpose_reduce32(double *a) {
    const int lane = threadIdx.x & 63;
    tr_step<16>(a, lane, 32);
    tr_step<8>(a, lane, 16);
    tr_step<4>(a, lane, 8);
    tr_step<2>(a, lane, 4);
    tr_step<1>(a, lane, 2);
    double v = a[0];
    v += __shfl_xor(v, 1, 64);
    return v;
}

}  // namespace expdg
