"""HIP graphs of library calls (tlrmdd_graph_begin / end / launch): a recorded solve replays the
same launches, so every replay must give the eager call's factors and f-history bit for bit.

Each recorded solve is replayed three times; between the replays the program runs its own eager
work (another solve on the same plan, torch kernels) and synchronises, and theta is restored
before each replay. Covered: one frequency of the parity workload (nr 64), the eight-frequency
batched call, a batched call with tile-form problems (whose tables the recorded call copies from
pinned host memory the graph owns) on one and two sub-batch streams, and the argument errors of
the capture calls.
"""
import ctypes

import numpy as np
import pytest

import synth
from gpu_cases import from_geometry, from_workload, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_14973_amd as m
    m._lib.load()
    return m


def _eager_noise(tl, plan, D, U, th):
    """Unrelated eager work between replays: another solve on the same plan and a torch kernel."""
    other, _ = tl.solve(plan, D, U, th * 0.5, 7)
    torch.cuda.synchronize()
    return float((other.abs() ** 2).sum().item())


def test_graph_single_solve_replays_bitwise(tl):
    case = from_workload(synth.small(), 3)
    plan, D, U, th0, _ = to_device(case, tl, torch)
    iters = 20
    th_e, fh_e = tl.solve(plan, D, U, th0, iters)
    theta = th0.clone()
    fh = torch.empty(iters + 1, dtype=torch.float64, device=D.device)
    g = tl.solve_graph(plan, D, U, theta, fh, iters)
    torch.cuda.synchronize()
    # recording ran nothing: theta is still the starting point
    assert torch.equal(theta, th0)
    for rep in range(3):
        theta.copy_(th0)
        fh.fill_(np.nan)
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(theta, th_e), rep
        assert torch.equal(fh, fh_e), rep
        _eager_noise(tl, plan, D, U, th0)


def test_graph_batched_small_workload_replays_bitwise(tl):
    wl = synth.small()
    devs = [to_device(from_workload(wl, i), tl, torch) for i in range(len(wl.freqs))]
    plans, Ds, Us, ths = [d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs], [d[3] for d in devs]
    th_e, fh_e = tl.solve_batched(plans, Ds, Us, ths, wl.iters)
    thetas = [t.clone() for t in ths]
    fhs = [torch.empty(wl.iters + 1, dtype=torch.float64, device=Ds[0].device) for _ in ths]
    g = tl.solve_batched_graph(plans, Ds, Us, thetas, fhs, wl.iters)
    for rep in range(3):
        for t, t0 in zip(thetas, ths):
            t.copy_(t0)
        g.launch()
        torch.cuda.synchronize()
        for i in range(len(ths)):
            assert torch.equal(thetas[i], th_e[i]), (rep, i)
            assert torch.equal(fhs[i], fh_e[i]), (rep, i)
        _eager_noise(tl, plans[0], Ds[0], Us[0], ths[0])


@pytest.mark.parametrize("streams", [1, 2])
def test_graph_batched_tile_forms_replay_bitwise(tl, streams):
    # 32 x 32 receivers, ns 512: four tiles of 256 and eight tiles of 128 (tile-form line search and
    # gradient, two classes) and dense diagonal tiles (dense forms); the recorded call uploads the
    # tile-form tables
    def case(seed, k_off, k_diag, tiles=(256,) * 4):
        nt = len(tiles)
        lay = synth.Layout(np.array(tiles), np.full(nt * (nt - 1) // 2, k_off), np.array(k_diag))
        return from_geometry(32, 32, "half", 14.0, lay, seed, f"tile{seed}")
    devs = [to_device(c, tl, torch) for c in (case(51, 12, [9, 14, 5, 16]), case(52, 3, [-1, 4, 5, 6]),
                                              case(53, 20, [20] * 8, tiles=(128,) * 8))]
    plans, Ds, Us, ths = [d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs], [d[3] for d in devs]
    assert [tl.line_form(p, tl.FP32_3M, tl.LINE_TILE_GRAD)[0] for p in plans] == [2, 0, 2]
    kw = dict(precision=tl.FP32_3M, line_products=tl.LINE_TILE_GRAD, streams=streams)
    iters = 12
    th_e, fh_e = tl.solve_batched(plans, Ds, Us, ths, iters, **kw)
    thetas = [t.clone() for t in ths]
    fhs = [torch.empty(iters + 1, dtype=torch.float64, device=Ds[0].device) for _ in ths]
    g = tl.solve_batched_graph(plans, Ds, Us, thetas, fhs, iters, **kw)
    for rep in range(3):
        for t, t0 in zip(thetas, ths):
            t.copy_(t0)
        g.launch()
        torch.cuda.synchronize()
        for i in range(len(ths)):
            assert torch.equal(thetas[i], th_e[i]), (rep, i)
            assert torch.equal(fhs[i], fh_e[i]), (rep, i)
        # eager batched work with its own table uploads between the replays
        tl.solve_batched(plans, Ds, Us, [t * 0.5 for t in ths], 3, **kw)
        torch.cuda.synchronize()


def test_graph_capture_argument_errors(tl):
    lib = tl._lib.load()
    h = ctypes.c_void_p()
    assert lib.tlrmdd_graph_begin(ctypes.c_void_p(0)) == tl._lib.INVALID_ARGUMENT   # null stream
    s = torch.cuda.Stream()
    sp = ctypes.c_void_p(s.cuda_stream)
    assert lib.tlrmdd_graph_end(sp, ctypes.byref(h)) == tl._lib.INVALID_ARGUMENT    # nothing open
    assert lib.tlrmdd_graph_begin(sp) == tl._lib.OK
    assert lib.tlrmdd_graph_begin(sp) == tl._lib.INVALID_ARGUMENT                   # one per thread
    assert lib.tlrmdd_graph_end(sp, ctypes.byref(h)) == tl._lib.OK                  # empty graph
    assert lib.tlrmdd_graph_launch(h, sp) == tl._lib.OK
    torch.cuda.synchronize()
    assert lib.tlrmdd_graph_destroy(h) == tl._lib.OK
    assert lib.tlrmdd_graph_launch(ctypes.c_void_p(0), sp) == tl._lib.INVALID_ARGUMENT
    # a NULL graph_out is an error that still closes the capture: a new one opens on the stream
    assert lib.tlrmdd_graph_begin(sp) == tl._lib.OK
    assert lib.tlrmdd_graph_end(sp, None) == tl._lib.INVALID_ARGUMENT
    assert lib.tlrmdd_graph_begin(sp) == tl._lib.OK
    assert lib.tlrmdd_graph_end(sp, ctypes.byref(h)) == tl._lib.OK
    assert lib.tlrmdd_graph_destroy(h) == tl._lib.OK
