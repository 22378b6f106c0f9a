// Oracle (test infrastructure only): dense matrix exponential and dense
// phi-function combinations.
//
// expm: diagonal (6,6) Pade approximant with scaling and squaring, the
// textbook method of the Expokit / Higham family that the paper cites for
// the small projected exponential (Section 2.3).  Pade coefficients
//   c_0 = 1,  c_k = c_{k-1} (q - k + 1) / (k (2q - k + 1)),  q = 6,
// numerator N = sum c_k X^k, denominator D = sum (-1)^k c_k X^k, X = A/2^s
// with s = max(0, ceil(log2(||A||_inf / 0.5))), then s squarings.
//
// phi_dense: sum_{k=0}^p tau^k phi_k(tau A) b_k read off the exponential of
// the augmented matrix [[A, W], [0, J]], W = [b_p, ..., b_1], J the p x p
// upper shift, applied to [b_0; e_p] (Section 2.3, augmented-matrix
// formulation of eq. linear_combination_of_phifunctions).
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace {

using Mat = std::vector<double>;  // row-major n x n

void matmul(int n, const Mat &A, const Mat &B, Mat &C) {
    Mat T((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const double a = A[(size_t)i * n + k];
            for (int j = 0; j < n; ++j) T[(size_t)i * n + j] += a * B[(size_t)k * n + j];
        }
    C.swap(T);
}

// Solve D X = N for X (overwrites N) by Gaussian elimination with partial
// pivoting.  Returns false if D is singular.
bool solve(int n, Mat D, Mat &N) {
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(D[(size_t)i * n + k]) > std::fabs(D[(size_t)piv * n + k])) piv = i;
        if (D[(size_t)piv * n + k] == 0.0) return false;
        if (piv != k) {
            for (int j = 0; j < n; ++j) {
                std::swap(D[(size_t)k * n + j], D[(size_t)piv * n + j]);
                std::swap(N[(size_t)k * n + j], N[(size_t)piv * n + j]);
            }
        }
        for (int i = k + 1; i < n; ++i) {
            const double f = D[(size_t)i * n + k] / D[(size_t)k * n + k];
            if (f == 0.0) continue;
            for (int j = k; j < n; ++j) D[(size_t)i * n + j] -= f * D[(size_t)k * n + j];
            for (int j = 0; j < n; ++j) N[(size_t)i * n + j] -= f * N[(size_t)k * n + j];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        for (int j = 0; j < n; ++j) {
            double acc = N[(size_t)k * n + j];
            for (int i = k + 1; i < n; ++i) acc -= D[(size_t)k * n + i] * N[(size_t)i * n + j];
            N[(size_t)k * n + j] = acc / D[(size_t)k * n + k];
        }
    }
    return true;
}

}  // namespace

extern "C" int orc_expm(int n, const double *A, double *E) {
    if (n < 1 || !A || !E) return -1;
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
        double row = 0.0;
        for (int j = 0; j < n; ++j) row += std::fabs(A[(size_t)i * n + j]);
        nrm = std::fmax(nrm, row);
    }
    if (!std::isfinite(nrm)) return -5;
    int s = 0;
    if (nrm > 0.5) s = std::max(0, (int)std::ceil(std::log2(nrm / 0.5)));
    const double scale = std::ldexp(1.0, -s);
    Mat X((size_t)n * n);
    for (size_t i = 0; i < X.size(); ++i) X[i] = A[i] * scale;

    const int q = 6;
    Mat P((size_t)n * n, 0.0), N((size_t)n * n, 0.0), D((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) P[(size_t)i * n + i] = 1.0;
    double c = 1.0;
    for (size_t i = 0; i < P.size(); ++i) {
        N[i] = c * P[i];
        D[i] = c * P[i];
    }
    for (int k = 1; k <= q; ++k) {
        c = c * (q - k + 1) / (double)(k * (2 * q - k + 1));
        matmul(n, X, P, P);  // P = X^k
        const double sgn = (k % 2 == 0) ? 1.0 : -1.0;
        for (size_t i = 0; i < P.size(); ++i) {
            N[i] += c * P[i];
            D[i] += sgn * c * P[i];
        }
    }
    if (!solve(n, D, N)) return -5;
    for (int k = 0; k < s; ++k) matmul(n, N, N, N);
    for (size_t i = 0; i < N.size(); ++i) E[i] = N[i];
    return 0;
}

extern "C" int orc_phi_dense(int n, const double *A, double tau, int p, const double *const *b,
                             double *out) {
    if (n < 1 || p < 0 || !A || !out) return -1;
    const int na = n + p;
    Mat M((size_t)na * na, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) M[(size_t)i * na + j] = tau * A[(size_t)i * n + j];
    // column n + k - 1 of W holds b_{p+1-k}
    for (int k = 1; k <= p; ++k) {
        const double *bk = b ? b[p + 1 - k] : nullptr;
        if (!bk) continue;
        for (int i = 0; i < n; ++i) M[(size_t)i * na + (n + k - 1)] = tau * bk[i];
    }
    // J: (J y)_k = y_{k+1}
    for (int k = 0; k + 1 < p; ++k) M[(size_t)(n + k) * na + (n + k + 1)] = tau;
    Mat E((size_t)na * na);
    int rc = orc_expm(na, M.data(), E.data());
    if (rc) return rc;
    const double *b0 = b ? b[0] : nullptr;
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        if (b0)
            for (int j = 0; j < n; ++j) acc += E[(size_t)i * na + j] * b0[j];
        if (p > 0) acc += E[(size_t)i * na + (na - 1)];
        out[i] = acc;
    }
    return 0;
}
