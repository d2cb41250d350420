// Host set-up of the fractional stiffness: generating sequences of the dense
// Toeplitz factors A_1^rho, A_2^rho and the scalar in front of the block matrix
// (Section 2, the entry formulas printed after eq. (chp-02-06)).
//
// The general entries are third/fourth finite differences of l^(3-2rho) and
// l^(4-2rho); at distances of a few hundred they are ~10 orders of magnitude
// smaller than the individual terms, so FP64 evaluation loses every digit.
// Every entry is therefore evaluated in IEEE binary128 (__float128, 113-bit
// significand, libquadmath) and rounded once to FP64.
//
// Compiled by the host compiler only (no device code here).
#include <quadmath.h>

#include "mgrit_internal.h"

namespace {

typedef __float128 q_t;

q_t qpow(q_t x, q_t e) { return x == 0 ? (q_t)0 : powq(x, e); }

}  // namespace

extern "C" void mgrit_toeplitz_sequences(double rho, int n, double* t, double* u, double* w) {
    const q_t r = (q_t)rho;
    const q_t e3 = 3 - 2 * r, e4 = 4 - 2 * r;
    // A_1 (symmetric): t[l] is the entry at distance l.
    for (int l = 0; l < n; ++l) {
        q_t v;
        if (l == 0) {
            v = powq(2, 6 - 2 * r) + 16 * r - 40;
        } else if (l == 1) {
            v = 2 * powq(3, 4 - 2 * r) + (2 * r - 6) * powq(2, 5 - 2 * r) - 16 * r + 34;
        } else {
            const q_t L = l;
            v = 4 * e4 * (-qpow(L - 1, e3) + 2 * qpow(L, e3) - qpow(L + 1, e3)) - 2 * qpow(L - 2, e4) +
                4 * qpow(L - 1, e4) - 4 * qpow(L + 1, e4) + 2 * qpow(L + 2, e4);
        }
        t[l] = (double)v;
    }
    // A_2: u[l] = entry (k, k+l); diagonal and first super-diagonal share one value.
    const q_t a2_diag = 4 - powq(2, 4 - 2 * r) * r;
    for (int l = 0; l < n; ++l) {
        q_t v;
        if (l <= 1) {
            v = a2_diag;
        } else {
            const q_t L = l;
            v = e4 * (qpow(L - 2, e3) - qpow(L - 1, e3) - qpow(L, e3) + qpow(L + 1, e3)) + 2 * qpow(L - 2, e4) -
                6 * qpow(L - 1, e4) + 6 * qpow(L, e4) - 2 * qpow(L + 1, e4);
        }
        u[l] = (double)v;
    }
    // A_2: w[m] = entry (p+m, p), m >= 1; w[0] repeats the diagonal.
    w[0] = (double)a2_diag;
    for (int m = 1; m < n; ++m) {
        const q_t M = m;
        const q_t v = e4 * (qpow(M - 1, e3) - qpow(M, e3) - qpow(M + 1, e3) + qpow(M + 2, e3)) +
                      2 * qpow(M - 1, e4) - 6 * qpow(M, e4) + 6 * qpow(M + 1, e4) - 2 * qpow(M + 2, e4);
        w[m] = (double)v;
    }
}

extern "C" double mgrit_stiffness_scale(double rho, double h_par, double h_perp) {
    // h_par^(1-2rho) h_perp / (2 cos(rho pi) Gamma(5-2rho))
    const q_t r = (q_t)rho;
    const q_t v = powq((q_t)h_par, 1 - 2 * r) * (q_t)h_perp / (2 * cosq(r * M_PIq) * tgammaq(5 - 2 * r));
    return (double)v;
}
