"""The algebra behind the FFT form of the operator, checked on the CPU against the oracle.

The GPU passes apply M_h v + theta (K_x A_x + K_y A_y) v (Section 2's block forms; the step matrix of
eq. (chp-02-03) with theta = tau / 2) as products of spectra: each Toeplitz block A_1, A_2, A_2^T of
one direction embedded in a circulant of length L >= 2n - 1, the mass stencil as 3-tap line kernels,
two real lines packed into one complex transform, the outputs at L - k taken as conjugates of those
at k, and, in the FP32 CG product, p.q summed over half the spectrum.  These tests restate each of
those identities with numpy's FFT and compare the result with the oracle's matrix-free
apply_M / apply_Ax / apply_Ay, so a wrong sign, index, conjugate or weight in the design fails here.
"""
import numpy as np
import pytest

from oracle import fem


def circulant_spectrum(T, L):
    """Spectrum of the length-L circulant whose leading n x n block is the Toeplitz matrix T."""
    n = T.shape[0]
    assert 2 * n - 1 <= L
    c = np.zeros(L)
    c[:n] = T[:, 0]
    c[L - n + 1:] = T[0, 1:][::-1]
    return np.fft.fft(c)


def tap_spectrum(taps, L):
    """Spectrum of the line kernel out[i] = sum_d taps[d] v[i + d] (d in {-1, 0, 1}) on the circle."""
    h = np.zeros(L)
    for d, w in taps.items():
        h[(-d) % L] += w
    return np.fft.fft(h)


def pad(lines, L):
    out = np.zeros(lines.shape[:-1] + (L,))
    out[..., :lines.shape[-1]] = lines
    return out


def half_spectrum_weights(L):
    """How often frequency k of a real line's spectrum stands in a sum over half the spectrum."""
    w = np.zeros(L)
    w[0] = w[L // 2] = 1.0
    w[1:L // 2] = 2.0
    return w


@pytest.fixture(scope="module")
def problem():
    # n_x = 200, n_y = 45 (both fit 512- and 1024-point transforms), beta != gamma, K_x != K_y
    return fem.Operator(fem.Problem(0.72, 0.61, 1.3, 0.8, 201, 46, a=0.0, b=1.0, c=0.0, d=2.0))


@pytest.mark.parametrize("L", [512, 1024])
def test_toeplitz_blocks_as_circulant_products(problem, L):
    rng = np.random.default_rng(11)
    for T in (problem.A1x, problem.A2x, problem.A1y, problem.A2y):
        n = T.shape[0]
        v = rng.standard_normal(n)
        got = np.fft.ifft(circulant_spectrum(T, L) * np.fft.fft(pad(v, L)))[:n]
        assert np.max(np.abs(got.imag)) <= 1e-12 * np.max(np.abs(T @ v))
        np.testing.assert_allclose(got.real, T @ v, rtol=0, atol=1e-12 * np.max(np.abs(T @ v)))


@pytest.mark.parametrize("L", [512, 1024])
def test_kernel_spectrum_symmetries(problem, L):
    """A_1 is symmetric (real spectrum); the spectrum of A_2^T is the conjugate of A_2's."""
    for A1, A2 in ((problem.A1x, problem.A2x), (problem.A1y, problem.A2y)):
        s1 = circulant_spectrum(A1, L)
        assert np.max(np.abs(s1.imag)) <= 1e-12 * np.max(np.abs(s1))
        np.testing.assert_allclose(circulant_spectrum(A2.T, L), np.conj(circulant_spectrum(A2, L)),
                                   rtol=0, atol=1e-12 * np.max(np.abs(circulant_spectrum(A2, L))))
    # the mass stencil's neighbour kernels: line j + 1 takes v(i) + v(i + 1), line j - 1 v(i) + v(i - 1)
    np.testing.assert_allclose(tap_spectrum({0: 1.0, -1: 1.0}, L), np.conj(tap_spectrum({0: 1.0, 1: 1.0}, L)),
                               rtol=0, atol=1e-13)


def test_packed_pair_unpacking():
    rng = np.random.default_rng(12)
    L = 512
    a, b = pad(rng.standard_normal((2, 300)), L)
    z = np.fft.fft(a + 1j * b)
    zc = np.conj(z[(-np.arange(L)) % L])
    np.testing.assert_allclose((z + zc) / 2, np.fft.fft(a), atol=1e-11)
    np.testing.assert_allclose((z - zc) / 2j, np.fft.fft(b), atol=1e-11)


def spectral_passes(op, V, theta, L):
    """Both passes as the GPU forms them: returns (out, x-pass spectral p.q, y-pass spectral p.q) for p = V."""
    prob = op.prob
    ny, nx = V.shape
    w = half_spectrum_weights(L)
    # x pass: lines are rows; line j couples rows j - 1, j, j + 1 (mass stencil plus K_x c_x A_x)
    sx = theta * prob.Kx * op.cx
    c1 = sx * circulant_spectrum(op.A1x, L) + op.mass_scale * tap_spectrum({-1: 1.0, 0: 6.0, 1: 1.0}, L)
    c2 = sx * circulant_spectrum(op.A2x, L) + op.mass_scale * tap_spectrum({0: 1.0, 1: 1.0}, L)
    c2t = sx * circulant_spectrum(op.A2x.T, L) + op.mass_scale * tap_spectrum({0: 1.0, -1: 1.0}, L)
    Vr = np.fft.fft(pad(V, L), axis=1)
    zero = np.zeros((1, L))
    up = np.vstack([Vr[1:], zero])            # spectrum of row j + 1 (zero past the last row)
    down = np.vstack([zero, Vr[:-1]])         # row j - 1
    Wx = c1 * Vr + c2 * up + c2t * down
    P = np.fft.ifft(Wx, axis=1)[:, :nx]
    dot_x = float(np.sum(w * np.real(np.conj(Vr) * Wx)) / L)
    # y pass: lines are columns (no mass, theta applied to its output)
    sy = prob.Ky * op.cy
    d1, d2, d2t = (sy * circulant_spectrum(T, L) for T in (op.A1y, op.A2y, op.A2y.T))
    Vc = np.fft.fft(pad(V.T, L), axis=1)
    zero = np.zeros((1, L))
    Wy = d1 * Vc + d2 * np.vstack([Vc[1:], zero]) + d2t * np.vstack([zero, Vc[:-1]])
    Y = np.fft.ifft(Wy, axis=1)[:, :ny].T
    dot_y = float(np.sum(w * np.real(np.conj(Vc) * Wy)) / L)
    return P.real + theta * Y.real, dot_x, theta * dot_y, np.max(np.abs(P.imag)) + np.max(np.abs(Y.imag))


@pytest.mark.parametrize("L", [512, 1024])
def test_operator_and_half_spectrum_dot_match_the_oracle(problem, L):
    rng = np.random.default_rng(13)
    ny, nx = problem.prob.ny, problem.prob.nx
    V = rng.standard_normal((ny, nx))
    theta = 0.37
    ref = problem.apply_M(V) + theta * problem.apply_A(V)
    out, dot_x, dot_y, imag = spectral_passes(problem, V, theta, L)
    scale = np.max(np.abs(ref))
    assert imag <= 1e-12 * scale
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12 * scale)
    # the partials of the two passes sum to p.q (p = V, q = the operator's output)
    pq = float(np.sum(V * ref))
    assert abs((dot_x + dot_y) - pq) <= 1e-12 * np.sum(np.abs(V) * np.abs(ref))
    # and each equals its own part: p.(M p + theta K_x A_x p) and theta p.(K_y A_y p)
    px = float(np.sum(V * (problem.apply_M(V) + theta * problem.prob.Kx * problem.apply_Ax(V))))
    assert abs(dot_x - px) <= 1e-12 * np.sum(np.abs(V) * np.abs(ref))


def test_half_spectrum_dot_fails_with_a_wrong_weight(problem):
    """The weights matter: counting each pair once (or the mirror half too) misses p.q by far."""
    rng = np.random.default_rng(14)
    V = rng.standard_normal((problem.prob.ny, problem.prob.nx))
    L = 512
    Vr = np.fft.fft(pad(V, L), axis=1)
    Y = np.fft.fft(pad(problem.apply_M(V), L), axis=1)
    exact = float(np.sum(V * problem.apply_M(V)))
    good = float(np.sum(half_spectrum_weights(L) * np.real(np.conj(Vr) * Y)) / L)
    once = float(np.sum((half_spectrum_weights(L) > 0) * np.real(np.conj(Vr) * Y)) / L)
    assert abs(good - exact) <= 1e-12 * abs(exact)
    assert abs(once - exact) > 1e-3 * abs(exact)
