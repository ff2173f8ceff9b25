"""Serving on the GPU: every result is bitwise the same alone and in the mix, and equals the oracle.

A small Poisson stream of solves of uneven size (nr 64..256, ragged tiles,
mixed diagonal modes) is served twice: one solve at a time, and with up to
three overlapping solves admitted under an HBM budget. Each request's final
factors and f-history must match bit for bit; a request with a non-finite
input (NaN in U) must not disturb the others. Then the serving workload's
shapes (nr 1024 to 4096, ragged tile 512, dense diagonal tiles, the tile
forms) with inputs made on the device at admission, served alone and four
at a time under a budget that makes admission wait for memory: bitwise the
same, and each within 1e-5 of the oracle's solve on the same inputs.
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


# ---------------------------------------------------------------------------
# the serving workload's shapes, inputs made at admission, against the oracle
# ---------------------------------------------------------------------------
# (n_side, ns_mode, tile, rank, iterations): nr 2304 with tile 512 (ragged: 4 x 512 + 256, dense forms),
# nr 1024 with dense diagonal tiles (rank 64 >= tile 128 / 2), nr 4096 / ns 2048 (tile-form line search
# and gradient), nr 1024 / ns 512 (tile forms); the large ones run fewer iterations to keep the oracle
# affordable (about 35 s for the four)
C5_SHAPES = [(48, "half", 512, 40, 20), (32, "full", 128, 64, 100), (64, "half", 256, 16, 10),
             (32, "half", 256, 12, 100)]


def _c5_jobs(tl, prec, line):
    from paper_2412_14973_amd import serve
    dev = torch.device("cuda")
    jobs, reqs = [], []
    for rid, (side, mode, d, k, iters) in enumerate(C5_SHAPES):
        r = synth.Request(rid, 0.002 * rid, side, mode, d, k, 6.0 + 7.0 * rid, iters)
        geom = synth.make_geometry(side, side, mode)
        plan = tl.Plan.from_layout(synth.request_layout(r), geom.ns)
        pd = torch.from_numpy(tl.hilbert_order(geom.rec_ix, geom.rec_iy)).to(dev)

        def inputs(r=r, pd=pd):
            D, U, th, _, _ = synth.device_problem(r, dev)
            return tl.permute_columns(D, pd), tl.permute_columns(U, pd), th
        req = serve.SolveRequest(plan, None, None, None, iters, prec, line_products=line, make_inputs=inputs,
                                 make_bytes=synth.device_generate_bytes(plan.ns, plan.nr))
        jobs.append(serve.Job(rid=rid, arrival=r.arrival, payload=req))
        reqs.append(r)
    return jobs, reqs


def test_serving_shapes_against_oracle_with_memory_bound_admission(tl):
    import oracle as O
    from paper_2412_14973_amd import serve
    prec, line = tl.FP32_3M, tl.LINE_TILE_GRAD
    alone, reqs = _c5_jobs(tl, prec, line)
    assert [tl.line_form(j.payload.plan, prec, line)[0] for j in alone] == [0, 0, 2, 2]
    assert alone[1].payload.plan.rank_diag.min() == -1 and alone[0].payload.plan.tile_size[-1] == 256
    srv1 = serve.Server(serve.GpuBackend(n_streams=1), hbm_budget=1 << 40, max_active=1)
    srv1.run(alone)
    torch.cuda.synchronize()
    mixed, _ = _c5_jobs(tl, prec, line)
    be = serve.GpuBackend(n_streams=4)
    fps = [be.footprint(j.payload) for j in mixed]
    # requests 0 and 1 arrive first and run for tens of milliseconds; request 2 arrives 2 ms after
    # request 1 and does not fit beside both: admission waits on memory (every request fits alone)
    budget = max(max(fps), fps[0] + fps[1] + fps[2] - 1)
    srv = serve.Server(be, hbm_budget=budget, max_active=4)
    srv.run(mixed)
    torch.cuda.synchronize()
    waits = [e for e in srv.log if e[1] == "wait_memory"]
    print(f"\nfootprints (GiB) {[round(f / 2 ** 30, 2) for f in fps]}, budget {budget / 2 ** 30:.2f} GiB, "
          f"peak {srv.peak_in_use / 2 ** 30:.2f} GiB, waits for memory {len(waits)}", flush=True)
    assert srv.peak_in_use <= budget and waits
    assert all(j.result is not None and not j.rejected for j in mixed)
    dev = torch.device("cuda")
    for a, m, r in zip(alone, mixed, reqs):
        assert torch.equal(a.result["theta"], m.result["theta"]), r.rid
        assert torch.equal(a.result["fhist"], m.result["fhist"]), r.rid
        # the oracle on the same inputs (made again from the request's seed), in its own Hilbert order
        D, U, th, lay, geom = synth.device_problem(r, dev)
        T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
        perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
        Do = O.permute_columns(D.cpu().numpy().astype(np.complex128), perm)
        Uo = O.permute_columns(U.cpu().numpy().astype(np.complex128), perm)
        ref = O.solve(T, Do, Uo, th.cpu().numpy().astype(np.complex128), iters=r.iters)
        thg = m.result["theta"].cpu().numpy().astype(np.complex128)
        rel_t = np.linalg.norm(thg - ref.theta) / np.linalg.norm(ref.theta)
        rel_h = np.max(np.abs(m.result["fhist"].cpu().numpy() - ref.f_hist) / ref.f_hist)
        print(f"request {r.rid} (nr {geom.nr}, ns {geom.ns}, tile {r.d}, rank {r.k}, {r.iters} iterations): "
              f"rel_theta {rel_t:.2e}, rel f_hist {rel_h:.2e}", flush=True)
        assert rel_t <= 1e-5 and rel_h <= 1e-5
