// Host set-up of the fast-diagonalisation preconditioner of the spatial solves.
//
// The step matrix B = M_h + theta A_h of eq. (chp-02-03) is approximated by a
// sum of Kronecker products that fast diagonalisation inverts,
//   P = M_y (x) M_x + theta (M_y (x) K_x + K_y (x) M_x),
// with 1-D matrices: the lumped mass M = h I (the row sums of M_h are h_x h_y; for the
// bilinear variant the consistent mass h/6 tridiag(1, 4, 1), which makes P exact)
// and the 1-D fractional stiffness K = K_rho h^(1-2rho) / (2 cos(rho pi) Gamma(4-2rho)) g(|i-j|),
// g(l) = |l-2|^p - 4|l-1|^p + 6|l|^p - 4|l+1|^p + |l+2|^p, p = 3 - 2rho (the
// fourth difference of |x|^p: the Riemann-Liouville derivatives of the hat
// functions integrated against each other, as for the entries of Section 2).
// h_y K_x equals the block stiffness A_x of Section 2 with its coupling across
// y lumped onto the diagonal block (c_x (A_1 + A_2 + A_2^T)), and likewise for y.
// The caller weights K (the solver uses 0.9 K_rho; see build_fd).
// With the generalised eigenvectors K V = M V diag(lambda), V^T M V = I, of each
// direction, P^{-1} = (V_y (x) V_x) diag(1 / (1 + theta (lambda_x,i + lambda_y,j))) (V_y (x) V_x)^T.
//
// The dense symmetric eigenproblem L^{-1} K L^{-T} (M = L L^T, L bidiagonal)
// is solved by Householder reduction to tridiagonal form followed by the
// implicit QL iteration with Wilkinson-type shifts, accumulating the
// orthogonal transformations.  Host compiler only.
#include <quadmath.h>

#include <cmath>
#include <vector>

#include "mgrit_internal.h"

namespace {

// Row-major n x n helpers.
struct Mat {
    int n;
    std::vector<double> a;
    explicit Mat(int n_) : n(n_), a((size_t)n_ * n_, 0.0) {}
    double& operator()(int i, int j) { return a[(size_t)i * n + j]; }
    double operator()(int i, int j) const { return a[(size_t)i * n + j]; }
};

// Householder reduction of symmetric A to tridiagonal T = Q^T A Q.
// On return A holds Q, diag/off hold T (off[i] couples i and i+1).
void householder_tridiagonal(Mat& A, std::vector<double>& diag, std::vector<double>& off) {
    const int n = A.n;
    Mat Q(n);
    for (int i = 0; i < n; ++i) Q(i, i) = 1.0;
    std::vector<double> v(n), p(n), w(n);
    for (int k = 0; k + 2 < n; ++k) {
        double norm2 = 0.0;
        for (int i = k + 1; i < n; ++i) norm2 += A(i, k) * A(i, k);
        const double alpha = std::sqrt(norm2);
        if (alpha == 0.0) continue;
        const double x0 = A(k + 1, k);
        const double s = x0 >= 0 ? alpha : -alpha;
        // v = x + s e1 (zero above k+1)
        for (int i = 0; i < n; ++i) v[i] = 0.0;
        v[k + 1] = x0 + s;
        for (int i = k + 2; i < n; ++i) v[i] = A(i, k);
        double vv = 0.0;
        for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        // p = beta A v (trailing block rows k..n-1)
        for (int i = k; i < n; ++i) {
            double acc = 0.0;
            for (int j = k + 1; j < n; ++j) acc += A(i, j) * v[j];
            p[i] = beta * acc;
        }
        double vp = 0.0;
        for (int i = k + 1; i < n; ++i) vp += v[i] * p[i];
        const double K = 0.5 * beta * vp;
        for (int i = k; i < n; ++i) w[i] = p[i] - K * v[i];
        // A <- A - v w^T - w v^T on rows/cols k..n-1 (v[k] = 0)
        for (int i = k; i < n; ++i)
            for (int j = k; j < n; ++j) A(i, j) -= v[i] * w[j] + w[i] * v[j];
        // Q <- Q H, H = I - beta v v^T
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = k + 1; j < n; ++j) acc += Q(i, j) * v[j];
            acc *= beta;
            for (int j = k + 1; j < n; ++j) Q(i, j) -= acc * v[j];
        }
    }
    diag.assign(n, 0.0);
    off.assign(n, 0.0);
    for (int i = 0; i < n; ++i) diag[i] = A(i, i);
    for (int i = 0; i + 1 < n; ++i) off[i] = A(i + 1, i);
    A = Q;
}

// Implicit QL on the symmetric tridiagonal (diag, off); Z accumulates the rotations
// (columns of Z become eigenvectors).  The step sequence is the published implicit QL
// algorithm with Wilkinson-type shifts (Bowdler, Martin, Reinsch and Wilkinson, 1968;
// EISPACK tql2), written here from that description.  Returns false if an eigenvalue fails
// to converge.
bool tridiagonal_ql(std::vector<double>& d, std::vector<double>& e, Mat& Z) {
    const int n = (int)d.size();
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        while (true) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) return false;
            // shift from the leading 2x2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                const double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int k = 0; k < n; ++k) {
                    const double zf = Z(k, i + 1);
                    Z(k, i + 1) = s * Z(k, i) + c * zf;
                    Z(k, i) = c * Z(k, i) - s * zf;
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

}  // namespace

extern "C" double mgrit_fd_stiffness_entry(double rho, double h, double K, int l) {
    typedef __float128 q_t;
    const q_t p = 3 - 2 * (q_t)rho;
    auto g = [&](int k) -> q_t { return k == 0 ? (q_t)0 : powq((q_t)(k < 0 ? -k : k), p); };
    const q_t v = g(l - 2) - 4 * g(l - 1) + 6 * g(l) - 4 * g(l + 1) + g(l + 2);
    const q_t scale = (q_t)K * powq((q_t)h, 1 - 2 * (q_t)rho) /
                      (2 * cosq((q_t)rho * M_PIq) * tgammaq(4 - 2 * (q_t)rho));
    return (double)(scale * v);
}

namespace {

// K v = lambda M v for the dense symmetric Toeplitz 1-D stiffness K and the tridiagonal mass
// M = tridiag(m1, m0, m1): C = L^{-1} K L^{-T} with the bidiagonal Cholesky factor L of M, C = Z D Z^T,
// V = L^{-T} Z (so V^T M V = I).
int fd_eigen(double rho, int n, double h, double K, double m0, double m1, double* V, double* lambda) {
    if (n < 1) return -1;
    std::vector<double> col(n);
    for (int l = 0; l < n; ++l) col[l] = mgrit_fd_stiffness_entry(rho, h, K, l);
    // Cholesky of the tridiagonal mass: L = bidiag(dl on the diagonal, el below)
    std::vector<double> dl(n), el(n, 0.0);
    dl[0] = std::sqrt(m0);
    for (int i = 0; i + 1 < n; ++i) {
        el[i] = m1 / dl[i];
        dl[i + 1] = std::sqrt(m0 - el[i] * el[i]);
    }
    // C = L^{-1} K L^{-T}
    Mat W(n);
    for (int j = 0; j < n; ++j) {
        double prev = 0.0;
        for (int i = 0; i < n; ++i) {
            const double kij = col[i > j ? i - j : j - i];
            const double w = (kij - (i > 0 ? el[i - 1] * prev : 0.0)) / dl[i];
            W(i, j) = w;
            prev = w;
        }
    }
    Mat C(n);
    for (int i = 0; i < n; ++i) {   // row i of W is column i of W^T
        double prev = 0.0;
        for (int j = 0; j < n; ++j) {
            const double y = (W(i, j) - (j > 0 ? el[j - 1] * prev : 0.0)) / dl[j];
            C(j, i) = y;
            prev = y;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double s = 0.5 * (C(i, j) + C(j, i));
            C(i, j) = C(j, i) = s;
        }
    std::vector<double> d, e;
    householder_tridiagonal(C, d, e);     // C now holds Q
    if (!tridiagonal_ql(d, e, C)) return -2;
    // V = L^{-T} Z (back substitution, column by column), row-major V[k][i]
    for (int i = 0; i < n; ++i) {
        double next = 0.0;
        for (int k = n - 1; k >= 0; --k) {
            const double v = (C(k, i) - (k + 1 < n ? el[k] * next : 0.0)) / dl[k];
            V[(size_t)k * n + i] = v;
            next = v;
        }
        lambda[i] = d[i];
    }
    return 0;
}

}  // namespace

// lumped mass h I (the preconditioner of the P1 scheme)
extern "C" int mgrit_fd_eigen(double rho, int n, double h, double K, double* V, double* lambda) {
    return fd_eigen(rho, n, h, K, h, 0.0, V, lambda);
}

// consistent mass h/6 tridiag(1, 4, 1) (the exact inverse of the Q1 step matrix)
extern "C" int mgrit_fd_eigen_consistent(double rho, int n, double h, double K, double* V, double* lambda) {
    return fd_eigen(rho, n, h, K, 4.0 * h / 6.0, h / 6.0, V, lambda);
}
