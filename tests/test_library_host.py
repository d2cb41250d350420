"""Host-side checks of libmgrit.so that need no GPU: exports, host set-up, argument validation."""
import ctypes
import re
import subprocess

import numpy as np
import pytest

from oracle import toeplitz

HEADER = __import__("os").path.join(__import__("os").path.dirname(__file__), "..", "include", "mgrit.h")


def _lib():
    from paper_1805_06688_amd import mgrit
    return mgrit


def test_library_exports_every_declared_symbol():
    mg = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(mgrit_[a-z_]+)\s*\(", text))
    out = subprocess.run(["nm", "-D", "--defined-only", mg._LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = declared - exported
    assert not missing, missing
    assert set(mg.SYMBOLS) <= declared


@pytest.mark.parametrize("rho,n", [(0.55, 1023), (0.75, 255), (0.95, 511), (0.6, 31)])
def test_host_sequences_equal_oracle(rho, n):
    """binary128 evaluation in the library == 50-digit evaluation in the oracle, to the last bit (or one ulp)."""
    t, u, w = _lib().toeplitz_sequences(rho, n)
    ot = toeplitz.a1_sequence(rho, n)
    ou = toeplitz.a2_upper_sequence(rho, n)
    ow = toeplitz.a2_lower_sequence(rho, n)
    for a, b in ((t, ot), (u, ou), (w[1:], ow[1:])):
        ulp = np.spacing(np.abs(b))
        assert np.all(np.abs(a - b) <= ulp)
    assert w[0] == u[0]


def test_host_scale_equals_oracle():
    mg = _lib()
    for rho, hp, hq in ((0.75, 1 / 256, 1 / 256), (0.55, 0.1, 0.3), (0.95, 2.0 / 7, 1.0 / 3)):
        a = mg.stiffness_scale(rho, hp, hq)
        b = toeplitz.stiffness_scale(rho, hp, hq)
        assert abs(a - b) <= 2 * np.spacing(abs(b))


@pytest.mark.parametrize("kw,code", [
    (dict(beta=0.5), -1), (dict(gamma=1.0), -1), (dict(Kx=0.0), -1), (dict(Mx=1), -1),
    (dict(domain=(1.0, 0.0, 0.0, 1.0)), -1), (dict(m=1), -1), (dict(max_levels=1), -1),
    (dict(t=[0.0, 0.5, 0.5, 1.0]), -1), (dict(t=[0.1, 0.5, 1.0]), -1), (dict(coarse="zz"), None),
])
def test_setup_rejects_invalid_arguments(kw, code):
    mg = _lib()
    args = dict(beta=0.7, gamma=0.8, Kx=1.0, Ky=1.0, Mx=8, My=8, t=np.linspace(0, 1, 17), m=4)
    args.update(kw)
    if code is None:
        with pytest.raises(KeyError):
            mg.Solver(**args)
        return
    with pytest.raises(mg.MgritError) as ei:
        mg.Solver(**args)
    assert ei.value.code == code
