"""Serving: admission by device-memory footprint, overlapping solves, results independent of the mix."""
import numpy as np
import pytest

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


OPTS = dict(m=4, max_levels=3, coarse="opt", precond="fd-bf16", cg_rtol=1e-12, tol_abs=0.0, tol_rel=1e-10,
            max_iter=40)


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        Mx, My = int(rng.integers(24, 90)), int(rng.integers(24, 90))
        Nt = int(rng.integers(24, 80)) // 4 * 4
        beta, gamma = rng.uniform(0.55, 0.95, 2)
        t = wl.uniform_grid(Nt) if k % 2 else wl.graded_grid(Nt)
        F, psi0 = wl.random_inputs(seed * 100 + k, Nt, Mx - 1, My - 1)
        reqs.append(dict(beta=float(beta), gamma=float(gamma), Kx=1.0, Ky=1.5, Mx=Mx, My=My, t=t,
                         F=torch.from_numpy(F).cuda(), psi0=torch.from_numpy(psi0).cuda()))
    return reqs


def _alone(r):
    mg = _mg()
    with mg.Solver(r["beta"], r["gamma"], r["Kx"], r["Ky"], r["Mx"], r["My"], r["t"], **OPTS) as s:
        U, st, rc = s.solve(r["F"], r["psi0"])
        assert rc == 0
        return U.clone()


def test_footprint_covers_allocation():
    mg = _mg()
    for (M, Nt, pc) in ((40, 64, "fd-bf16"), (130, 96, "fd"), (65, 33, "none")):
        t = wl.uniform_grid(Nt)
        est = mg.footprint(0.7, 0.8, 1.0, 1.0, M, M, t, m=4, max_levels=3, coarse="opt", precond=pc)
        with mg.Solver(0.7, 0.8, 1.0, 1.0, M, M, t, m=4, max_levels=3, coarse="opt", precond=pc) as s:
            used = s.device_bytes()
        assert used <= est <= 1.3 * used + (1 << 20), (M, Nt, pc, used, est)


def test_results_identical_alone_and_in_the_mix():
    mg = _mg()
    reqs = _requests(6, 1)
    ref = [_alone(r) for r in reqs]
    with mg.Server(8 << 30, max_concurrent=4) as srv:
        handles = [srv.submit(r["F"], r["psi0"], r["beta"], r["gamma"], r["Kx"], r["Ky"], r["Mx"], r["My"], r["t"],
                              **OPTS) for r in reqs]
        out = [h.wait() for h in handles]
    starts = [info.start_s for _, info in out]
    finishes = [info.finish_s for _, info in out]
    for (U, info), R in zip(out, ref):
        assert info.rc == 0 and info.stats.converged == 1
        assert torch.equal(U.reshape(R.shape), R)              # bitwise: nothing depends on the mix
    # some solves ran at the same time
    assert any(starts[j] < finishes[i] and starts[i] < finishes[j] for i in range(6) for j in range(i + 1, 6))


def test_admission_respects_the_budget():
    """A budget that holds one solve at a time serialises them in arrival order."""
    mg = _mg()
    reqs = _requests(4, 2)
    fps = [mg.footprint(r["beta"], r["gamma"], r["Kx"], r["Ky"], r["Mx"], r["My"], r["t"], **OPTS) for r in reqs]
    budget = max(fps) + min(fps) // 2          # no two fit together
    with mg.Server(budget, max_concurrent=4) as srv:
        handles = [srv.submit(r["F"], r["psi0"], r["beta"], r["gamma"], r["Kx"], r["Ky"], r["Mx"], r["My"], r["t"],
                              **OPTS) for r in reqs]
        infos = [h.wait()[1] for h in handles]
    for a, b in zip(infos, infos[1:]):
        assert b.start_s >= a.finish_s - 1e-6
    assert all(i.rc == 0 for i in infos)


def test_oversized_request_is_rejected():
    mg = _mg()
    r = _requests(1, 3)[0]
    with mg.Server(1 << 20, max_concurrent=1) as srv:
        with pytest.raises(mg.MgritError):
            srv.submit(r["F"], r["psi0"], r["beta"], r["gamma"], r["Kx"], r["Ky"], r["Mx"], r["My"], r["t"], **OPTS)


def test_queued_same_mesh_requests_share_one_group_solve():
    """With a group limit, a worker takes the queued requests of the oldest one's mesh into one group solve
    (their sweeps share launches); requests on another mesh run on their own; every result equals its solo
    solve (FP64, no preconditioner: bit for bit)."""
    mg = _mg()
    opts = dict(OPTS, precond="none")
    Mx, My = 60, 52
    reqs = []
    for k in range(5):
        Nt = 32 + 8 * k
        t = wl.uniform_grid(Nt) if k % 2 else wl.graded_grid(Nt)
        F, psi0 = wl.random_inputs(900 + k, Nt, Mx - 1, My - 1)
        reqs.append(dict(beta=0.6 + 0.05 * k, gamma=0.9 - 0.05 * k, Kx=1.0, Ky=1.5, Mx=Mx, My=My, t=t,
                         F=torch.from_numpy(F).cuda(), psi0=torch.from_numpy(psi0).cuda()))
    other = _requests(1, 4)[0]
    reqs.insert(2, other)                      # a request on another mesh in the middle of the queue
    ref = []
    for r in reqs:
        with mg.Solver(r["beta"], r["gamma"], r["Kx"], r["Ky"], r["Mx"], r["My"], r["t"], **opts) as s:
            U, st, rc = s.solve(r["F"], r["psi0"])
            ref.append((U.clone(), st.iterations))
    blocker = _requests(1, 5)[0]
    with mg.Server(8 << 30, max_concurrent=1, group_limit=8) as srv:
        # the first request occupies the only slot while the others queue behind it
        h0 = srv.submit(blocker["F"], blocker["psi0"], blocker["beta"], blocker["gamma"], blocker["Kx"], blocker["Ky"],
                        blocker["Mx"], blocker["My"], blocker["t"], **opts)
        hs = [srv.submit(r["F"], r["psi0"], r["beta"], r["gamma"], r["Kx"], r["Ky"], r["Mx"], r["My"], r["t"], **opts)
              for r in reqs]
        out = [h.wait() for h in hs]
        h0.wait()
    sizes = [info.group_size for _, info in out]
    assert sizes == [5, 5, 1, 5, 5, 5], sizes
    for (U, info), (R, its) in zip(out, ref):
        assert info.rc == 0 and info.stats.iterations == its
        assert torch.equal(U.reshape(R.shape), R)
