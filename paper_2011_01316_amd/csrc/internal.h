// Internal declarations of the MI355X exponential-DG library (not part of the
// C ABI).  Kernels live in dg_kernels.hip and krylov_kernels.hip; the host
// drivers in api.cpp.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/expdg.h"

namespace expdg {

constexpr int kMaxP = 6;       // largest LGL degree compiled
constexpr int kMaxM = 64;      // largest Krylov basis (Hessenberg exponential in LDS)
constexpr int kMaxAug = 3;     // largest number of phi terms beyond phi_0
constexpr int kRedBlocks = 1024;  // blocks of the row-partitioned reduction kernels
constexpr int kRedThreads = 256;

// Arguments of the fused DG operator kernels (residual or linear operator).
template <typename T>
struct OpArgs {
    const T *q;        // state (residual) or reference state (linear operator)
    const T *v;        // direction of the linear operator (nullptr for the residual)
    T *out;
    const T *aug[kMaxAug];  // aug[k-1] multiplies y_k: b_{p+1-k} (nullptr = zero)
    const T *vtail;    // the p augmented entries y of the input (nullptr if p = 0)
    T *otail;          // the p augmented entries of the output
    const double *vscale;  // device scalar multiplying the whole result (nullptr = 1)
    const T *lin;      // frozen fields of q~ for the 2D linear operator (launch_lin_prepare)
    // First Gram-Schmidt pass fused into the linear operator (nv > 0): block
    // partials dpart[i * dnb + tile] of V_i^T out over the tile's nodes (and,
    // in tile 0, the augmented entries), i < nv, V_i = basis + i * bstride.
    const T *basis;
    size_t bstride;
    int nv;
    int dnb;           // blocks of the launch (partials per vector)
    double *dpart;
    double eta;        // scaling of the augmented block
    int naug;          // p
    int K, nx, ny;
    T rhx, rhy;        // 2/hx, 2/hy
    T lift;            // 1/w_0 (= 1/w_p)
    T gamma;
    T D[(kMaxP + 1) * (kMaxP + 1)];  // D[i*(p+1)+l] = l_l'(xi_i)
};

// Start/stop events that the next kernel launch of this host thread records as
// part of its own dispatch (live kernel timing); the launch consumes them.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents &next_launch_events();

template <typename K, typename... Args>
hipError_t launch_kernel(K kernel, dim3 grid, dim3 block, unsigned shmem, hipStream_t s,
                         Args... args) {
    LaunchEvents &e = next_launch_events();
    if (e.start) {
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, e.start, e.stop, 0, args...);
        e = LaunchEvents{};
    } else {
        kernel<<<grid, block, shmem, s>>>(args...);
    }
    return hipGetLastError();
}

// Host-side LGL tables of degree p (library's own construction).
int lgl_tables(int p, double *xi, double *w, double *D);

// ---- kernel launchers (dg_kernels.hip) ----
hipError_t launch_dg_op(int equation, int p, bool jvp, const OpArgs<double> &a, hipStream_t s);
hipError_t launch_dg_op(int equation, int p, bool jvp, const OpArgs<float> &a, hipStream_t s);
// Frozen fields of the 2D linear operator at the reference state q (planes u,
// v, H, then the Rusanov speed of every x face and every y face; lin_elems
// elements).  Burgers needs none (no-op, lin_elems = 0).
template <typename T>
hipError_t launch_lin_prepare(int equation, int p, const T *q, T *lin, int K, int nx, int ny,
                              double gamma, hipStream_t s);
size_t lin_elems(int equation, int p, int K);
// Blocks one operator launch uses for K elements.
int dg_blocks(int equation, int p, int K);
// Grouped FP64 launch over n meshes of the same equation and degree: item it
// owns blocks [bstart[it], bstart[it+1]) (device arrays), total = bstart[n].
hipError_t launch_dg_op_group(int equation, int p, bool jvp, const OpArgs<double> *items,
                              const int *bstart, int n, int total, hipStream_t s);
// Per-block maxima of the wave speed (FP64 state) into part[0..nblk).
hipError_t launch_max_speed(int equation, const double *q, size_t npts, double gamma,
                            double *part, int nblk, hipStream_t s);
int max_speed_blocks(size_t npts);

// Elementwise kernels (dg_kernels.hip).  All lengths in elements.
// y = (To)x
hipError_t launch_convert(const double *x, float *y, size_t n, hipStream_t s);
hipError_t launch_convert(const float *x, double *y, size_t n, hipStream_t s);
hipError_t launch_copy(const double *x, double *y, size_t n, hipStream_t s);
hipError_t launch_copy(const float *x, float *y, size_t n, hipStream_t s);
// out = a*x + b*y + c*z (z may be nullptr)
template <typename TO, typename TX>
hipError_t launch_lincomb(TO *out, double a, const TX *x, double b, const TX *y, double c,
                          const TX *z, size_t n, hipStream_t s);
// q (double) += w (T)
template <typename T>
hipError_t launch_add_to(double *q, const T *w, size_t n, hipStream_t s);
// out (double) = x (double) + y (T)
template <typename T>
hipError_t launch_add_mixed(double *out, const double *x, const T *y, size_t n, hipStream_t s);
// x[0..n) = val
template <typename T>
hipError_t launch_fill(T *x, double val, size_t n, hipStream_t s);
// x[0..p) = (0, ..., 0, last)
template <typename T>
hipError_t launch_set_tail(T *x, int p, double last, hipStream_t s);
// Start vector of a phi evaluation: z[0..n) = b0 (nullptr: 0), z[n..n+p) =
// (0, ..., 0, last), flags[0..4) = 0.
template <typename T>
hipError_t launch_phi_init(T *z, const T *b0, size_t n, int p, double last, int *flags,
                           hipStream_t s);
// End of a step: q_prev = q (if q_prev), then q += w.
template <typename T>
hipError_t launch_step_update(double *q, double *q_prev, const T *w, size_t n, hipStream_t s);

// ---- Krylov kernels (krylov_kernels.hip) ----
struct KrylovDev {
    double *H;       // (kMaxM+1) x kMaxM Hessenberg, row-major, ld = kMaxM
    double *S;       // kMaxM+1 basis scales (v_i = S[i] * u_i)
    double *coefA;   // kMaxM+1 first-pass Gram-Schmidt coefficients h1_i S[i]
    double *coefB;   // kMaxM+1 second-pass coefficients h2_i S[i]
    double *part;    // kRedBlocks x (kMaxM+1) block partial sums
    double *res;     // res[0] = beta
    int *flags;      // [0] first breakdown iteration (0 = none), [1] non-finite
};

// Fixed row partition of a length-L vector: nrb blocks of rpb rows (rpb a
// multiple of 1024, nrb <= kRedBlocks).
struct RowPartition {
    size_t rpb;
    int nrb;
};
RowPartition row_partition(size_t L);

// Block partials of V_i^T w (i < nv) into part (the finish is a separate
// launch: launch_gs_finish_dots).
template <typename T>
hipError_t launch_gs_dots(const T *V, size_t stride, int nv, const T *w, size_t L,
                          const RowPartition &rp, double *part, const double *S, double *H,
                          int col, int accumulate, double *coef_out, hipStream_t s);
// w -= sum_i coef_in[i] V_i, then block partials of V_i^T w (rows i < nv) and
// of ||w||^2 (row nv; w must be V_nv).  nv <= 32: one fused pass; else a plain
// update then a dot pass over the nv + 1 vectors V_0..V_nv.
template <typename T>
hipError_t launch_gs_update_dots(const T *V, size_t stride, int nv, const double *coef_in, T *w,
                                 size_t L, const RowPartition &rp, double *part, const double *S,
                                 double *H, int col, double *coef_out, hipStream_t s);
// w -= sum_i coef[i] V_i (if coef), then block partials of ||w||^2.
template <typename T>
hipError_t launch_gs_update_norm(const T *V, size_t stride, int nv, const double *coef, T *w,
                                 size_t L, const RowPartition &rp, double *part, double *H,
                                 double *S, int col, int *flags, double *res, hipStream_t s);
// Fixed-order finish of a dot pass: h_i = S[i] sum_b part[i][b]; H[i][col] set
// (accumulate = 0) or incremented; coef_out[i] = h_i S[i].
hipError_t launch_gs_finish_dots(const double *part, int nv, const RowPartition &rp,
                                 const double *S, double *H, int col, int accumulate,
                                 double *coef_out, hipStream_t s);
// w -= sum_i coef[i] V_i, no reduction.
template <typename T>
hipError_t launch_gs_update(const T *V, size_t stride, int nv, const double *coef, T *w, size_t L,
                            const RowPartition &rp, hipStream_t s);
// Fixed-order finish of the second pass with the norm (one block): h2_i from
// rows i < nv, H[i][col] += h2_i, coef_out[i] = h2_i S[i]; hn^2 = row nv -
// sum h2_i^2 (Pythagoras: the norm of w - V h2 for an orthonormal basis), then
// H[col+1][col], S[col+1] and the flags as in launch_gs_finish_norm.
hipError_t launch_gs_finish_pass2(const double *part, int nv, const RowPartition &rp, double *S,
                                  double *H, int col, double *coef_out, int *flags,
                                  hipStream_t s);
// Fixed-order finish of a norm pass: hn = sqrt(sum_b part[b]).  col >= 0:
// H[col+1][col] = hn, breakdown test against ||H||_F (flags[0] = col+1 the
// first time, S[col+1] = 0), else S[col+1] = 1/hn; flags[1] = col+1 the first
// time a norm is non-finite.  col < 0 (start vector of a substep): res[0] =
// beta = hn, S[0] = 1/beta, flags[0] = 0, flags[1] = 1 if beta is
// non-finite, else 0, and the Hessenberg matrix is cleared.
hipError_t launch_gs_finish_norm(const double *part, const RowPartition &rp, double *H, double *S,
                                 int col, int *flags, double *res, hipStream_t s);
// Norms of up to 4 vectors of length n (block partials, then finish):
// out[k] = ||x_k||_2 (device doubles).
template <typename T>
hipError_t launch_norms(const T *const *x, int nx, size_t n, double *part, double *out,
                        hipStream_t s);
// One small-exponential check: F = expm(dtau * Hhat_j) (size j+1) of the
// Hessenberg matrix H (j columns), err = beta |F[j][0]|, combine coefficients
// ccoef[i] = beta F[i][0] S[i] (i < j).  Results go to slot (layout below).
struct ExpmItem {
    const double *H;
    const double *S;
    const double *res;   // res[0] = beta
    const int *flags;    // Krylov flags, copied into the slot header
    double *slot;
    double *report;      // host-mapped copy of the first kSummary header values (or nullptr)
    double dtau;
    int j;
};
hipError_t launch_hess_expm(const ExpmItem &c, hipStream_t s);
// n checks (device array), one workgroup each.
hipError_t launch_hess_expm_group(const ExpmItem *items, int n, hipStream_t s);

// One Arnoldi step (FP64) of one solve inside a grouped launch: the CGS2
// passes and the norm of w = u_nv against the basis u_0..u_{nv-1}.
struct GsItem {
    const double *V;
    double *w;
    size_t stride, L, rpb;
    int nrb, nv, col;    // col = nv - 1
    int nrb1;            // partials per vector of a first pass fused into the linear
                         // operator (its blocks), or 0: a separate dot pass
    double *part, *S, *H, *coefA, *coefB, *res;
    int *flags;
};
// Block ranges of a grouped Arnoldi step: first dots (items whose linear
// operator does not carry them), first finish, fused update+dots+norm
// (nv <= 32), plain update (nv > 32), dots with w itself after it (nv > 32),
// final update.  (The second finish runs one block per item.)
constexpr int kGroupLaunches = 6;
// Host: block ranges bstart[k*(n+1) + it] of launch k and the totals.
void arnoldi_group_layout(const GsItem *items, int n, int *bstart, int *totals);
// Device copies of items and bstart; totals from arnoldi_group_layout.
hipError_t launch_arnoldi_group(const GsItem *items, const int *bstart, const int *totals, int n,
                                hipStream_t s);
// z = sum_{i<m} ccoef[i] * V_i (row-local; z may alias V_0).
template <typename T>
hipError_t launch_combine(const T *V, size_t stride, int m, const double *ccoef, T *z, size_t L,
                          hipStream_t s);
// Dense expm on the device for testing the small-exponential kernel: A and E
// are n x n row-major device buffers (n <= kMaxM + 1).
hipError_t launch_dense_expm(const double *A, int n, double *E, hipStream_t s);

// Slot layout written by the small-exponential kernels (doubles).
constexpr int kSlotErr = 0;        // beta |F[j][0]|
constexpr int kSlotSingular = 1;   // 1: singular Pade denominator
constexpr int kSlotBreak = 2;      // Krylov flags[0]: first breakdown iteration (0 = none)
constexpr int kSlotNonfinite = 3;  // Krylov flags[1]: a non-finite norm was seen
constexpr int kSlotSquarings = 4;
constexpr int kSlotHeader = 5;
constexpr int kSummary = 4;        // header values a check reports to the host
constexpr int kSlotCoef = 8;       // kMaxM combine coefficients
constexpr int kSlotSize = kSlotCoef + kMaxM + 8;
constexpr int kCheckSlots = 4;     // result slots of the checks in flight (one solve)

// Grouped launches: block b belongs to the largest item it with
// bstart[it] <= b (items with no blocks are skipped).
__device__ __forceinline__ int group_item(const int *bstart, int n, int b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bstart[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

}  // namespace expdg
