"""The tensor-product (Q1) variant of the space discretisation.

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; not part of the product path).

Section 2 discretises the Riesz operators with linear elements on triangles (the block matrices
M_h, A_x, A_y of eq. chp-02-03, in `fem.py`).  The variant here uses bilinear elements on the
same rectangular mesh, whose matrices are Kronecker products of 1-D linear-element matrices:

  M_h = M_y (x) M_x,    A_h = K_x M_y (x) A_x + K_y A_y (x) M_x,

with, on a uniform 1-D mesh of spacing h and n interior nodes,

  M = h/6 tridiag(1, 4, 1),
  A[i][j] = a(|i - j|),  a(l) = h^(1-2 rho) / (2 cos(rho pi) Gamma(4 - 2 rho)) g(l),
  g(l) = |l-2|^p - 4 |l-1|^p + 6 |l|^p - 4 |l+1|^p + |l+2|^p,  p = 3 - 2 rho.

The paper prints no 1-D entries; a(l) is derived here the way the 2-D entries of Section 2 are:
the Riesz derivative of order 2 rho is -1/(2 cos(rho pi)) (D_L^(2 rho) + D_R^(2 rho)), so the stiffness
form (the negative of its weak form) is a(u, v) = 1/(2 cos(rho pi)) [(D_L^rho u, D_R^rho v) + (D_R^rho u,
D_L^rho v)]; a hat function is a sum of ramps c_k (x - z_k)_+ with slope jumps (1, -2, 1)/h at its
three nodes, the fractional derivatives of ramps are powers (x - z)_+^(1-rho)/Gamma(2-rho), and the
Beta integral of two of them gives (z_l - z_k)^(3-2rho)/Gamma(4-2rho); summing over the kink pairs of
two hats at distance l h gives the fourth difference g(l).  The tests pin a(l) against a quadrature of
the Fourier form of the same bilinear form, which shares nothing with this derivation.

Unknowns are ordered x fastest as in `fem.py`; grid arrays have shape [..., n_y, n_x], and
(B (x) A) vec(V) is the array B V A^T.
"""
import math

import mpmath
import numpy as np

from . import fem

_DPS = 40


def stiffness_1d_entries(rho, n, h):
    """a(l), l = 0..n-1, evaluated with mpmath and rounded once to FP64."""
    with mpmath.workdps(_DPS):
        r = mpmath.mpf(rho)
        p = 3 - 2 * r

        def pw(k):
            return mpmath.mpf(0) if k == 0 else mpmath.power(abs(k), p)

        scale = mpmath.power(mpmath.mpf(h), 1 - 2 * r) / (2 * mpmath.cos(r * mpmath.pi) * mpmath.gamma(4 - 2 * r))
        return np.array([float(scale * (pw(l - 2) - 4 * pw(l - 1) + 6 * pw(l) - 4 * pw(l + 1) + pw(l + 2)))
                         for l in range(n)], dtype=np.float64)


def stiffness_1d(rho, n, h):
    a = stiffness_1d_entries(rho, n, h)
    idx = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])
    return a[idx]


def mass_1d(n, h):
    return (h / 6.0) * (4.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1))


class Q1Operator(fem.Operator):
    """M_h and A_h of the bilinear variant for one Problem (same interface as fem.Operator)."""

    def __init__(self, prob):
        self.prob = prob
        p = prob
        self.Ax = stiffness_1d(p.beta, p.nx, p.hx)
        self.Ay = stiffness_1d(p.gamma, p.ny, p.hy)
        self.Mx = mass_1d(p.nx, p.hx)
        self.My = mass_1d(p.ny, p.hy)

    def apply_M(self, V):
        V = np.asarray(V, dtype=np.float64)
        return self.My @ V @ self.Mx.T

    def apply_Ax(self, V):
        V = np.asarray(V, dtype=np.float64)
        return self.My @ V @ self.Ax.T

    def apply_Ay(self, V):
        V = np.asarray(V, dtype=np.float64)
        return self.Ay @ V @ self.Mx.T

    def apply_A(self, V):
        return self.prob.Kx * self.apply_Ax(V) + self.prob.Ky * self.apply_Ay(V)

    def assembled_M(self):
        return np.kron(self.My, self.Mx)

    def assembled_Ax(self):
        return np.kron(self.My, self.Ax)

    def assembled_Ay(self):
        return np.kron(self.Ay, self.Mx)

    def assembled_A(self):
        return self.prob.Kx * self.assembled_Ax() + self.prob.Ky * self.assembled_Ay()


def fourier_entry(rho, l, h):
    """Pin of a(l): the bilinear form of -d^(2 rho)/d|x|^(2 rho) has the symbol |xi|^(2 rho), so for two hats
    at distance l h, (1/pi) int_0^inf xi^(2 rho) |phi^(xi)|^2 cos(xi l h) d xi with phi^(xi) = h sinc^2(xi h/2);
    with u = xi h / 2 this is 2^(2 rho + 1) h^(1 - 2 rho) / pi * int_0^inf u^(2 rho - 4) sin^4 u cos(2 l u) du.
    The integral is taken by adaptive quadrature on [0, U]; beyond U, sin^4 u cos(2 l u) is written as a sum of
    cos(2 k u) (sin^4 u = 3/8 - cos(2u)/2 + cos(4u)/8), the k = 0 part of u^(2 rho - 4) integrated in closed form
    and each k > 0 part by the Fourier-integral rule (QAWF)."""
    import warnings

    import scipy.integrate
    warnings.filterwarnings("ignore", category=scipy.integrate.IntegrationWarning)
    e = 2 * rho - 4
    U = 40.0
    f = lambda u: u ** e * math.sin(u) ** 4 * math.cos(2 * l * u) if u > 0 else 0.0
    head = 0.0
    for a in np.arange(0.0, U, 0.5):             # panels of half a unit: a few oscillations each
        v, _ = scipy.integrate.quad(f, a, a + 0.5, limit=200, epsabs=1e-16, epsrel=1e-13)
        head += v
    coef = {}
    for k, c in ((l, 3 / 8), (l - 1, -1 / 4), (l + 1, -1 / 4), (l - 2, 1 / 16), (l + 2, 1 / 16)):
        coef[abs(k)] = coef.get(abs(k), 0.0) + c
    tail = 0.0
    for k, c in coef.items():
        if c == 0.0:
            continue
        if k == 0:
            tail += c * U ** (e + 1) / -(e + 1)
        else:
            v, _ = scipy.integrate.quad(lambda u: u ** e, U, np.inf, weight="cos", wvar=2.0 * k, limlst=100)
            tail += c * v
    return 2.0 ** (2 * rho + 1) * h ** (1 - 2 * rho) / math.pi * (head + tail)
