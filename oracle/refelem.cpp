// Oracle (test infrastructure only): Legendre-Gauss-Lobatto reference element.
//
// The paper integrates every volume and face term with LGL quadrature
// (start of Section 4) on a nodal basis.  Nodes are the p+1 roots of
// (1 - x^2) P_p'(x); weights are 2 / (p (p+1) P_p(x_i)^2); the
// differentiation matrix is D_ij = l_j'(x_i) for the Lagrange basis l_j on
// those nodes, written with barycentric weights.  These are the textbook
// formulas; nothing here is tuned.
#include "oracle.h"

#include <cmath>
#include <vector>

namespace {

// P_p(x) and P_p'(x) by the three-term recurrence
//   (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}
// and the derivative identity P'_{k+1} = P'_{k-1} + (2k+1) P_k.
void legendre(int p, double x, double *P, double *dP) {
    double p_prev = 1.0, p_cur = x;  // P_0, P_1
    double d_prev = 0.0, d_cur = 1.0;
    if (p == 0) {
        *P = 1.0;
        *dP = 0.0;
        return;
    }
    for (int k = 1; k < p; ++k) {
        double p_next = ((2.0 * k + 1.0) * x * p_cur - k * p_prev) / (k + 1.0);
        double d_next = d_prev + (2.0 * k + 1.0) * p_cur;
        p_prev = p_cur;
        p_cur = p_next;
        d_prev = d_cur;
        d_cur = d_next;
    }
    *P = p_cur;
    *dP = d_cur;
}

}  // namespace

extern "C" int orc_lgl(int p, double *xi, double *w, double *D) {
    if (p < 1 || p > 15 || !xi || !w || !D) return -1;
    const int n = p + 1;
    // Interior nodes: roots of P_p'.  Newton's method with the second
    // derivative from Legendre's equation
    //   (1 - x^2) P'' = 2 x P' - p (p+1) P,
    // started from the Chebyshev-Gauss-Lobatto points.
    xi[0] = -1.0;
    xi[p] = 1.0;
    const double pi = std::acos(-1.0);
    for (int i = 1; i < p; ++i) {
        double x = -std::cos(pi * i / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, x, &P, &dP);
            double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
            double dx = dP / d2P;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    for (int i = 0; i < n; ++i) {
        double P, dP;
        legendre(p, xi[i], &P, &dP);
        w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
    // Barycentric weights lambda_j = 1 / prod_{k != j} (x_j - x_k).
    std::vector<double> lam(n);
    for (int j = 0; j < n; ++j) {
        double prod = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) prod *= (xi[j] - xi[k]);
        lam[j] = 1.0 / prod;
    }
    // l_j'(x_i) = (lambda_j / lambda_i) / (x_i - x_j) off the diagonal; the
    // diagonal makes every row sum to zero (derivative of a constant).
    for (int i = 0; i < n; ++i) {
        double rowsum = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d = (lam[j] / lam[i]) / (xi[i] - xi[j]);
            D[i * n + j] = d;
            rowsum += d;
        }
        D[i * n + i] = -rowsum;
    }
    return 0;
}
