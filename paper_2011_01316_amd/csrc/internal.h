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
#ifndef EXPDG_UPDATE_SPLIT
#define EXPDG_UPDATE_SPLIT 8
#endif
// Blocks of the update sweep per block of the reductions' row partition: the
// sweep writes no partials, and eight times the blocks keep more loads in
// flight (measured: 256x256 p = 3 109 -> 100 us, 512x512 p = 4 FP32 bulk
// 374 -> 350 us, 128x128 p = 4 34.7 -> 32.1 us; unchanged where the
// partition is already one 1024-row sweep per block).
constexpr int kUpdateSplit = EXPDG_UPDATE_SPLIT;
// Lanes of the update sweep per variable plane when the dot pass runs in the
// operator's epilogue.  The operator's blocks give XCD x (of 8) the x-th
// eighth of the elements and walk it upwards in every plane, so when it ends
// the most recently read rows of the basis are the top of each of these
// eighths; the update walks each eighth of each plane downwards, starting on
// the rows read last (the likeliest to be still in the 256 MB last-level
// cache) and ending on the bottoms, where the next operator starts.  Results
// do not depend on the order.  (The counters at the L2's memory side count
// last-level cache hits too and read the same bytes either way.)  Measured,
// same box, bitwise-equal results: 256x256 p = 3 6.62 -> 6.26 ms/step (FP64)
// and 4.24 -> 4.00 (FP32 bulk); operator + update per Arnoldi step 192x192
// p = 4 175 -> 170 us, 128x128 p = 4 72.2 -> 71.5, 64x64 p = 3 23.0 -> 22.8;
// 512x512 p = 4 1235 -> 1245 us in FP64 (the update 3 % slower: a basis
// vector is 210 MB, there is nothing to reuse) and 13.01 -> 12.96 ms/step in
// FP32 bulk; the 3D run (702 MB vectors) unchanged.
constexpr int kUpdateLanesPerPlane = 8;
constexpr int kRedThreads = 256;

// Arguments of the fused DG operator kernels (residual or linear operator).
template <typename T>
struct OpArgs {
    const T *q;        // state (residual) or reference state (linear operator)
    // FP32-bulk residual: the state in FP64, read instead of q when set (the
    // residual of the FP32-rounded state carries that rounding's
    // high-frequency noise, which the Krylov process would have to resolve)
    const double *q64;
    const T *v;        // direction of the linear operator (nullptr for the residual)
    T *out;
    const T *aug[kMaxAug];  // aug[k-1] multiplies y_k: b_{p+1-k} (nullptr = zero)
    const T *vtail;    // the p augmented entries y of the input (nullptr if p = 0)
    T *otail;          // the p augmented entries of the output
    const double *vscale;  // device scalar multiplying the whole result (nullptr = 1)
    const T *lin;      // frozen fields of q~ for the 2D linear operator (launch_lin_prepare)
    // Dot pass of an Arnoldi step fused into the linear operator (dots != 0):
    // block partials dpart[r * dnb + tile] over the tile's nodes (and, in
    // tile 0, the augmented entries) of the rows of launch_gs_dots2 with
    // x = v, w = out and u_i = basis + i * bstride, i < nv.
    const T *basis;
    size_t bstride;
    int nv;
    int dots;
    int dnb;           // blocks of the launch (partials per row)
    double *dpart;
    double eta;        // scaling of the augmented block
    int naug;          // p
    int K, nx, ny;
    // geometry and physics constants: FP64 for both storage types (the
    // operators compute in FP64 and store in T)
    double rhx, rhy, rhz;   // 2/hx, 2/hy, 2/hz
    double lift;            // 1/w_0 (= 1/w_p)
    double gamma;
    // Burgers options (Section 3.1): viscosity, entropy flux (residual only)
    // with jump coefficient sigma / (h/2), diffusion-flux switch beta
    // (0 central, 1/2 LDG), zero Dirichlet ends, and a source added to the
    // residual (nullptr = none).
    double kappa;
    double ef_pen;     // 2 sigma / hx
    double beta;
    int ef;            // nonzero: entropy flux for (u^2/2)*
    int ef_local;      // nonzero: the penalty is ef_pen + max|u^+-| at each face
    int dirichlet;     // nonzero: u = 0 beyond both ends
    const T *src;
    // Entropy viscosity (2D Euler): nodal viscosity nu, or nullptr
    const T *nu;
    // Euler 2D: nonzero for no-slip walls at y0 and y1 (exterior state at a
    // wall face node: the mirror, both momenta reversed)
    int ywall;
    double D[(kMaxP + 1) * (kMaxP + 1)];  // D[i*(p+1)+l] = l_l'(xi_i)
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
// The state may be FP64 for FP32 fields (an FP32-bulk step prepares them from
// its FP64 state).
template <typename Q, typename T>
hipError_t launch_lin_prepare(int equation, int p, const Q *q, T *lin, int K, int nx, int ny,
                              double gamma, hipStream_t s);
size_t lin_elems(int equation, int p, int K);
// Blocks one operator launch uses for K elements.
int dg_blocks(int equation, int p, int K);
// Threads per block of the operator launches (256, or 384 for the 3D p = 6 one).
int dg_block_threads(int equation, int p);
// Grouped FP64 launch over n meshes of the same equation and degree: item it
// owns blocks [bstart[it], bstart[it+1]) (device arrays), total = bstart[n].
// visc selects the viscous Burgers kernels (every item then has kappa > 0), or
// for Euler 2D the kernels with entropy viscosity (every item has nu).
hipError_t launch_dg_op_group(int equation, int p, bool jvp, bool visc,
                              const OpArgs<double> *items, const int *bstart, int n, int total,
                              hipStream_t s);
// Entropy viscosity (2D Euler): the element viscosity of q after q_prev (FP64
// states, step dt) into nue[K], then its vertex-averaged bilinear
// reconstruction at the nodes into nu (bulk type).
struct EvParams {
    int K, nx, ny, p;
    int ywall;  // no-slip walls at y0 and y1
    double rhx, rhy, lift, gamma, dt, ce, cmax, he;
    double xi[kMaxP + 1];                // LGL nodes (bilinear reconstruction)
    double D[(kMaxP + 1) * (kMaxP + 1)];  // D[i*(p+1)+l] = l_l'(xi_i)
};
hipError_t launch_ev_element(const EvParams &ep, const double *q, const double *q_prev,
                             double *nue, hipStream_t s);
template <typename T>
hipError_t launch_ev_smooth(const EvParams &ep, const double *nue, T *nu, hipStream_t s);
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
// Arnoldi by classical Gram-Schmidt applied twice, with the second pass of
// each vector delayed into the next step (one dot pass and one update sweep
// per step).  Step k applies the operator to x = u_{k-1}, a vector that has
// had its first pass only, giving w = A x; one pass of block partials gives
// u_i^T w and u_i^T x (i < k-1), x^T x and x^T w; the finish completes x
// (second pass, norm by Pythagoras: column k-2 of H and H[k-1][k-2] become
// final), rescales w to A v_{k-1} through the Arnoldi relation, and takes
// the first pass of w (column k-1 of H); one sweep then stores the finished
// x and the once-orthogonalised new vector.
constexpr int kLDH = kMaxM + 1;          // row stride of H
constexpr int kPartRows = 2 * kMaxM + 2;  // partial rows of one step: V^T w, V^T x, x^T x, x^T w
constexpr int kScalW = kMaxM + 1;        // coefB[kScalW] = 1 / beta (scale of w)
constexpr int kScalX = kMaxM + 2;        // coefB[kScalX] = e_{k-1} / beta (multiple of x)
struct KrylovDev {
    double *H;       // (kMaxM+1) x kLDH Hessenberg, row-major
    double *S;       // kMaxM+1 basis scales (v_i = S[i] * u_i)
    double *coefA;   // kMaxM+1: x -= sum_i coefA[i] u_i
    double *coefB;   // kMaxM+3: w <- coefB[kScalW] w - coefB[kScalX] x - sum_i coefB[i] u_i
    double *part;    // partials: kPartRows rows of max(kRedBlocks, operator blocks)
    double *fold;    // folded partials: kPartRows rows of fold_chunks(operator blocks)
    double *res;     // res[0] = beta
    int *flags;      // [0] first breakdown dimension (0 = none), [1] first non-finite one
};

// Fixed row partition of a length-L vector: nrb blocks of rpb rows (rpb a
// multiple of 1024, nrb <= kRedBlocks).
struct RowPartition {
    size_t rpb;
    int nrb;
};
RowPartition row_partition(size_t L);

// Block partials of step k (nv = k - 1 finished vectors u_0..u_{nv-1}):
// row i < nv: u_i^T w; row nv + i: u_i^T x; row 2 nv: x^T x; row 2 nv + 1:
// x^T w (the 1D path; the 2D linear operator writes the same rows itself).
template <typename T>
hipError_t launch_gs_dots2(const T *V, size_t stride, int nv, const T *x, const T *w, size_t L,
                           const RowPartition &rp, double *part, hipStream_t s);
// Fixed-order finish of step k from nrb partials per row (one block): with
// a_i = S[i] (u_i^T x), b_i = S[i] (u_i^T w): beta = sqrt(x^T x - |a|^2)
// (k = 1: beta = 1 / S[0], x = u_0 is already finished); H[i][k-2] += a_i,
// H[k-1][k-2] = beta, breakdown test against ||H||_F (flags[0] = k-1 the
// first time, S[k-1] = 0) else S[k-1] = 1/beta; flags[1] = k-1 the first time
// beta or ||H||_F is non-finite.  t = H_{0:k,0:k-1} a; first pass of
// A v_{k-1} = (w - V_k t) / beta: g_i = (b_i - t_i) / beta (i < k-1),
// g_{k-1} = ((x^T w - a.b) / beta - t_{k-1}) / beta, H[i][k-1] = g_i; with
// e = t / beta + g: coefA[i] = S[i] a_i, coefB[i] = S[i] (e_i - a_i e_{k-1} /
// beta), coefB[kScalW] = 1 / beta, coefB[kScalX] = e_{k-1} / beta.
hipError_t launch_dcgs_finish(const double *part, int nrb, int k, double *S, double *H,
                              double *coefA, double *coefB, int *flags, hipStream_t s);
// One sweep of step k: x -= sum_{i<nv} coefA[i] u_i (only if write_x and
// nv > 0) and w <- coefB[kScalW] w - coefB[kScalX] x_old - sum_{i<nv} coefB[i] u_i.
// The rows are cut into `lanes` contiguous lanes of nearly equal length (at
// most L / 1024 of them, each starting on a multiple of 1024 rows), each walked
// from its end to its start; see kUpdateLanesPerPlane.
template <typename T>
hipError_t launch_dcgs_update(const T *V, size_t stride, int nv, const double *coefA,
                              const double *coefB, T *x, T *w, size_t L, const RowPartition &rp,
                              hipStream_t s, bool write_x = true, int lanes = 1);
// Partial rows longer than kFoldAbove (the dot pass fused into the operator
// of a large mesh writes one partial per operator block) are first folded by a
// many-block launch: out[r * nc + c] = the fixed-order sum of chunk c
// (kFoldChunk consecutive partials) of row r, nc = fold_chunks(nrb); the
// finish then sums nc values per row instead of nrb.
constexpr int kFoldAbove = 1024;
constexpr int kFoldChunk = 1024;
inline int fold_chunks(int nrb) {
    return nrb > kFoldAbove ? (nrb + kFoldChunk - 1) / kFoldChunk : 0;
}
hipError_t launch_fold(const double *part, int nrb, int rows, double *out, hipStream_t s);
// The 2D Euler linear operator with its dot pass runs as 512-thread blocks
// (two halves splitting the basis chunks, same partials bit for bit) up to
// this many blocks: two blocks per CU or fewer leave one or two waves per
// SIMD, and a block's sequence of chunks sets the time (measured: 9-14 %
// faster at 231-410 blocks, 7-13 % slower from 640 up, where the idle
// second half costs occupancy).
#ifndef EXPDG_HALVES_BLOCKS
#define EXPDG_HALVES_BLOCKS 512
#endif
constexpr int kHalvesBlocks = EXPDG_HALVES_BLOCKS;
// Incomplete orthogonalization (window of L vectors), finish of step k: x =
// u_{k-1} (stored unnormalised), w = A x, and the nw = min(k-1, L-1) window
// vectors u_{k0}, ..., u_{k-2} (k0 = k-1-nw) with block partials in the rows
// of launch_gs_dots2 (basis = u_{k0}, nv = nw).  k > 1: beta = ||x|| (explicit
// norm), H[k-1][k-2] = beta, breakdown / non-finite tests as in
// launch_dcgs_finish, S[k-1] = 1/beta; k = 1: beta = 1/S[0].  Column k-1 of H:
// h_i = S[k0+i] (u_{k0+i}^T w) / beta on the window, h_{k-1,k-1} = x^T w /
// beta^2.  The update sweep (write_x = false) then forms u_k = w / beta -
// sum_i h_i v_{k0+i} - h_{k-1,k-1} x / beta: coefA = 0, coefB[i] = S[k0+i] h_i,
// coefB[kScalW] = 1/beta, coefB[kScalX] = h_{k-1,k-1} / beta.
hipError_t launch_iop_finish(const double *part, int nrb, int k, int k0, int nw, double *S,
                             double *H, double *coefA, double *coefB, int *flags, hipStream_t s);
// Start vector of a substep: block partials of ||z||^2 (z = V_0) ...
template <typename T>
hipError_t launch_gs_norm(const T *z, size_t L, const RowPartition &rp, double *part,
                          hipStream_t s);
// ... and their fixed-order finish: res[0] = beta = ||z||, S[0] = 1/beta,
// flags[0] = 0, flags[1] = 1 if beta is non-finite, else 0, and the Hessenberg
// matrix is cleared.
hipError_t launch_gs_finish_norm(const double *part, const RowPartition &rp, double *H, double *S,
                                 int *flags, double *res, hipStream_t s);
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

// One Arnoldi step k (FP64) of one solve inside a grouped launch.
struct GsItem {
    const double *V;     // u_0, u_1, ...: x = u_{k-1}, w = u_k
    double *x, *w;
    size_t stride, L, rpb;
    int nrb, k;
    int k0, nv;          // the vectors u_k0 .. u_{k0+nv-1} the step orthogonalizes against
    int iop;             // nonzero: incomplete orthogonalization (one pass, explicit norm)
    int nrb1;            // partials per row written by the linear operator (its blocks),
                         // or 0: a separate dot pass
    int nfold;           // fold_chunks(nrb1): > 0 when the partials are folded first
    double *part, *fold, *S, *H, *coefA, *coefB;
    int *flags;
};
// Block ranges of a grouped Arnoldi step: the dot pass (items whose linear
// operator does not carry it), the fold of long partial rows (items with
// nfold > 0) and the update sweep.  (The finish runs one block per item.)
constexpr int kGroupLaunches = 3;
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
