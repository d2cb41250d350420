"""Generating sequences of the dense Toeplitz factors A_1^rho, A_2^rho.

TEST INFRASTRUCTURE ONLY.  This package is the plain FP64 CPU oracle; it is
imported by the tests, by the smoke check and by the CPU-baseline leg of the
benchmark, never by the product path.

Section 2 (entries of the Toeplitz matrices following the stiffness matrices
A_x^beta, A_y^gamma) gives closed forms for the entries of A_1 (symmetric) and
A_2 (non-symmetric).  Writing e3 = 3 - 2 rho, e4 = 4 - 2 rho:

  A_1:  diagonal      2^(6-2rho) + 16 rho - 40
        first off-diag 2*3^(4-2rho) + (2rho-6)*2^(5-2rho) - 16 rho + 34
        distance l>=2  4 e4 [-(l-1)^e3 + 2 l^e3 - (l+1)^e3]
                       - 2(l-2)^e4 + 4(l-1)^e4 - 4(l+1)^e4 + 2(l+2)^e4
  A_2:  diagonal and first super-diagonal  4 - 2^(4-2rho) rho
        super-diagonal distance l>=2
            e4 [(l-2)^e3 - (l-1)^e3 - l^e3 + (l+1)^e3]
            + 2(l-2)^e4 - 6(l-1)^e4 + 6 l^e4 - 2(l+1)^e4
        sub-diagonal distance m>=1
            e4 [(m-1)^e3 - m^e3 - (m+1)^e3 + (m+2)^e3]
            + 2(m-1)^e4 - 6 m^e4 + 6(m+1)^e4 - 2(m+2)^e4

The general formulas are finite differences of x^e3 and x^e4; evaluated in
FP64 at distances of several hundred they cancel catastrophically (the sum is
~l^(-1-2rho) while the terms are ~l^e4).  Reading taken here: evaluate every
entry with mpmath at 50 significant digits and round once to FP64.  The
sub-diagonal sequence is evaluated from its own printed formula, not from
the super-diagonal one.
"""
import mpmath
import numpy as np

_DPS = 50


def _pw(x, e):
    # 0^e = 0 for the positive exponents used here
    return mpmath.mpf(0) if x == 0 else mpmath.power(x, e)


def a1_sequence(rho, n):
    """t[l] = entry of A_1^rho at distance |i-j| = l, l = 0..n-1 (FP64)."""
    with mpmath.workdps(_DPS):
        r = mpmath.mpf(rho)
        e3, e4 = 3 - 2 * r, 4 - 2 * r
        out = []
        for l in range(n):
            if l == 0:
                v = mpmath.power(2, 6 - 2 * r) + 16 * r - 40
            elif l == 1:
                v = 2 * mpmath.power(3, 4 - 2 * r) + (2 * r - 6) * mpmath.power(2, 5 - 2 * r) - 16 * r + 34
            else:
                L = mpmath.mpf(l)
                v = (4 * e4 * (-_pw(L - 1, e3) + 2 * _pw(L, e3) - _pw(L + 1, e3))
                     - 2 * _pw(L - 2, e4) + 4 * _pw(L - 1, e4) - 4 * _pw(L + 1, e4) + 2 * _pw(L + 2, e4))
            out.append(float(v))
    return np.array(out, dtype=np.float64)


def a2_upper_sequence(rho, n):
    """u[l] = entry (k, k+l) of A_2^rho, l = 0..n-1 (FP64)."""
    with mpmath.workdps(_DPS):
        r = mpmath.mpf(rho)
        e3, e4 = 3 - 2 * r, 4 - 2 * r
        out = []
        for l in range(n):
            if l <= 1:
                v = 4 - mpmath.power(2, 4 - 2 * r) * r
            else:
                L = mpmath.mpf(l)
                v = (e4 * (_pw(L - 2, e3) - _pw(L - 1, e3) - _pw(L, e3) + _pw(L + 1, e3))
                     + 2 * _pw(L - 2, e4) - 6 * _pw(L - 1, e4) + 6 * _pw(L, e4) - 2 * _pw(L + 1, e4))
            out.append(float(v))
    return np.array(out, dtype=np.float64)


def a2_lower_sequence(rho, n):
    """w[m] = entry (p+m, p) of A_2^rho, m = 1..n-1; w[0] is unused (set to the diagonal)."""
    with mpmath.workdps(_DPS):
        r = mpmath.mpf(rho)
        e3, e4 = 3 - 2 * r, 4 - 2 * r
        out = [float(4 - mpmath.power(2, 4 - 2 * r) * r)]
        for m in range(1, n):
            M = mpmath.mpf(m)
            v = (e4 * (_pw(M - 1, e3) - _pw(M, e3) - _pw(M + 1, e3) + _pw(M + 2, e3))
                 + 2 * _pw(M - 1, e4) - 6 * _pw(M, e4) + 6 * _pw(M + 1, e4) - 2 * _pw(M + 2, e4))
            out.append(float(v))
    return np.array(out, dtype=np.float64)


def toeplitz_factors(rho, n):
    """Dense A_1^rho (n x n, symmetric) and A_2^rho (n x n) in FP64."""
    t = a1_sequence(rho, n)
    u = a2_upper_sequence(rho, n)
    w = a2_lower_sequence(rho, n)
    A1 = np.empty((n, n))
    A2 = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            A1[i, j] = t[abs(i - j)]
            A2[i, j] = u[j - i] if j >= i else w[i - j]
    return A1, A2


def stiffness_scale(rho, h_par, h_perp):
    """Scalar in front of the block matrix: h_par^(1-2rho) h_perp / (2 cos(rho pi) Gamma(5-2rho)).

    h_par is the spacing along the fractional direction, h_perp the other one.
    """
    with mpmath.workdps(_DPS):
        r = mpmath.mpf(rho)
        v = mpmath.power(mpmath.mpf(h_par), 1 - 2 * r) * mpmath.mpf(h_perp) / (
            2 * mpmath.cos(r * mpmath.pi) * mpmath.gamma(5 - 2 * r))
        return float(v)
