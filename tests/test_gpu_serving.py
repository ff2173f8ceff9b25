"""Serving on the GPU: every result is bitwise the same alone and in the mix.

A small Poisson stream of solves of uneven size (nr 64..256, ragged tiles,
mixed diagonal modes) is served twice: one solve at a time, and with up to
three overlapping solves admitted under an HBM budget. Each request's final
factors and f-history must match bit for bit; a request with a non-finite
input (NaN in U) must not disturb the others.
"""
import numpy as np
import pytest

import synth
from gpu_cases import c64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_14973_amd as m
    m._lib.load()
    return m


def _requests(tl, n=7, poison=None):
    from paper_2412_14973_amd import serve
    rng = np.random.default_rng(77)
    dev = torch.device("cuda")
    jobs = []
    t = 0.0
    for rid in range(n):
        side = int(rng.choice([8, 12, 16]))
        mode = "half" if rid % 2 else "full"
        geom = synth.make_geometry(side, side, mode)
        d = int(rng.choice([16, 40, 64]))
        k = int(rng.integers(2, 12))
        lay = synth.uniform_layout(side * side, d, k, -1 if k >= d // 2 else k)
        prob = synth.make_problem(geom, float(rng.uniform(5, 30)), 20.0, 0.05, 95, rid)
        perm = tl.hilbert_order(geom.rec_ix, geom.rec_iy)
        U = c64(prob.U)[:, perm]
        if poison is not None and rid == poison:
            U[0, 0] = np.nan
        D = torch.from_numpy(np.ascontiguousarray(c64(prob.D)[:, perm], dtype=np.complex64)).to(dev)
        Ug = torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex64)).to(dev)
        th = torch.from_numpy(synth.init_theta(synth.theta_length(lay), 95, rid).astype(np.complex64)).to(dev)
        plan = tl.Plan.from_layout(lay, geom.ns)
        t += float(rng.exponential(1 / 200.0))
        jobs.append(serve.Job(rid=rid, arrival=t, payload=serve.SolveRequest(plan, D, Ug, th, 30)))
    return jobs


def _serve(tl, jobs, active, budget):
    from paper_2412_14973_amd import serve
    be = serve.GpuBackend(n_streams=active)
    srv = serve.Server(be, hbm_budget=budget, max_active=active)
    srv.run(jobs)
    torch.cuda.synchronize()
    return srv


def test_alone_equals_in_mix(tl):
    jobs_a = _requests(tl)
    _serve(tl, jobs_a, 1, 1 << 34)
    jobs_m = _requests(tl)
    srv = _serve(tl, jobs_m, 3, 1 << 34)
    overlaps = sum(1 for (t, ev, rid) in srv.log if ev == "admit") and max(
        sum(1 for j in jobs_m if j.admitted <= jj.admitted < j.finished) for jj in jobs_m)
    print("max overlapping solves", overlaps)
    for a, m in zip(jobs_a, jobs_m):
        assert torch.equal(a.result["theta"], m.result["theta"]), a.rid
        assert torch.equal(a.result["fhist"], m.result["fhist"]), a.rid
        fh = m.result["fhist"].cpu().numpy()
        assert np.all(np.isfinite(fh)) and fh[-1] < fh[0]


def test_budget_limits_concurrency(tl):
    jobs = _requests(tl, n=5)
    from paper_2412_14973_amd import serve
    be = serve.GpuBackend(n_streams=3)
    fps = [be.footprint(j.payload) for j in jobs]
    budget = max(fps) + min(fps) - 1        # never room for the two largest together
    srv = serve.Server(be, hbm_budget=budget, max_active=3)
    srv.run(jobs)
    torch.cuda.synchronize()
    assert srv.peak_in_use <= budget
    assert all(j.result is not None for j in jobs)


def test_nonfinite_request_isolated(tl):
    clean = _requests(tl, n=4)
    _serve(tl, clean, 1, 1 << 34)
    mixed = _requests(tl, n=4, poison=2)
    _serve(tl, mixed, 3, 1 << 34)
    for a, m in zip(clean, mixed):
        if a.rid == 2:
            assert not np.all(np.isfinite(m.result["fhist"].cpu().numpy()))
            continue
        assert torch.equal(a.result["theta"], m.result["theta"])
        assert torch.equal(a.result["fhist"], m.result["fhist"])
