"""mgrit_apply_noalloc (the operator application that allocates nothing) against mgrit_apply.

Both run the same kernels on the same slices; the no-allocation form only takes its descriptors and the
FFT x-pass workspace from the library's fixed scratch array, so its results must equal mgrit_apply's
bit for bit, and the oracle's operator to the bound of the FP64 operator tests (1e-13 of the largest
entry).  Two calls in a row, the second with fewer slices, check that nothing left in the shared
scratch array from the first call leaks into the second.
"""
import numpy as np
import pytest

from oracle import fem
from paper_1805_06688_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mg():
    from paper_1805_06688_amd import mgrit
    return mgrit


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("opk,Mx,My", [("fft", 96, 78), ("dense", 131, 65), ("fft", 256, 256)])
def test_noalloc_apply_equals_apply(opk, Mx, My):
    mg = _mg()
    beta, gamma, Kx, Ky = 0.75, 0.85, 2.0, 1.0
    prob = fem.Problem(beta, gamma, Kx, Ky, Mx, My)
    op = fem.Operator(prob)
    with mg.Solver(beta, gamma, Kx, Ky, Mx, My, wl.uniform_grid(8), m=2, op=opk) as s:
        bytes0 = s.device_bytes()
        for call, (S, sign, use_add) in enumerate([(9, 1.0, True), (4, -1.0, False)]):
            v = wl.random_slices(31 + call, S, prob.nx, prob.ny)
            add = wl.random_slices(41 + call, S, prob.nx, prob.ny)
            theta = np.linspace(-0.5, 3.0, S) * (1 + call)
            ref_lib = s.apply(theta, dev(v), sign=sign, add=dev(add) if use_add else None)
            torch.cuda.synchronize()
            out = s.apply_noalloc(dev(theta), dev(v), sign=sign, add=dev(add) if use_add else None,
                                  out=torch.full((S * prob.nx * prob.ny,), float("nan"), dtype=torch.float64,
                                                 device="cuda"))
            torch.cuda.synchronize()
            assert torch.equal(out, ref_lib), (call, float((out - ref_lib).abs().max()))
            o = out.cpu().numpy()
            for k in range(S):
                ref = sign * (op.apply_M(v[k]) + theta[k] * op.apply_A(v[k])) + (add[k] if use_add else 0.0)
                assert np.abs(o[k] - ref).max() <= 1e-13 * np.abs(ref).max(), (call, k)
        assert s.device_bytes() == bytes0


def test_noalloc_rejects_batches_beyond_its_scratch():
    mg = _mg()
    with mg.Solver(0.6, 0.9, 1.0, 1.0, 512, 512, wl.uniform_grid(4), m=2, op="fft") as s:
        S = 33                                  # 33 slices of 511 x 511 need more than 64 MiB
        theta = torch.zeros(S, dtype=torch.float64, device="cuda")
        v = torch.zeros(S * 511 * 511, dtype=torch.float64, device="cuda")
        with pytest.raises(mg.MgritError) as e:
            s.apply_noalloc(theta, v)
        assert e.value.code == mg.EINVAL
        out = s.apply_noalloc(theta[:32], v[: 32 * 511 * 511])          # 32 fit
        torch.cuda.synchronize()
        assert not torch.any(out != 0)
