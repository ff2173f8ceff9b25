"""The device entry points are stream ordered and return without waiting for the device.

A bounded spin kernel (torch.cuda._sleep) is queued on the stream first; each call must return
while that kernel is still running (the stream reports unfinished work right after the call), and
its results, once the stream is synchronised, must equal bit for bit those of the same call made
on an idle stream. Covered: forward, grad, the tile low-rank forward, single solves in the dense and
tile forms (whose tables go through the library's pinned staging buffers), batched solves mixing
the forms, ADMM, the column gather.
"""
import time

import numpy as np
import pytest

import synth
from gpu_cases import from_workload, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_14973_amd as m
    m._lib.load()
    return m


@pytest.fixture(scope="module")
def spin_cycles():
    """Cycles of torch.cuda._sleep that keep the stream busy for about 0.3 s."""
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n = 10_000_000
    a.record()
    torch.cuda._sleep(n)
    b.record()
    torch.cuda.synchronize()
    ms = max(a.elapsed_time(b), 1e-3)
    return int(min(n * 300.0 / ms, 2e10))


def returns_early(spin, fn):
    """fn() after a spin kernel: (result, stream still busy when fn returned, host seconds in fn)."""
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    torch.cuda._sleep(spin)
    t0 = time.perf_counter()
    out = fn()
    dt = time.perf_counter() - t0
    busy = not s.query()
    torch.cuda.synchronize()
    return out, busy, dt


def flat(out):
    if isinstance(out, torch.Tensor):
        return [out]
    res = []
    for o in out:
        res += flat(o) if o is not None else []
    return res


def check(spin, fn, name):
    ref = fn()
    torch.cuda.synchronize()
    got, busy, dt = returns_early(spin, fn)
    print(f"{name}: returned after {dt * 1e3:.1f} ms with the stream still busy: {busy}")
    assert busy, f"{name} waited for the device"
    for a, b in zip(flat(ref), flat(got)):
        assert torch.equal(a, b), name


@pytest.fixture(scope="module")
def problems(tl):
    wl = synth.batched()
    out = []
    for f_idx in (10, 40):   # tile 256 (tile-form line search and gradient), tile 64 (dense forms)
        case = from_workload(wl, f_idx)
        out.append(to_device(case, tl, torch))
    return out


def test_forward_grad_return_early(tl, spin_cycles, problems):
    plan, D, U, th, _ = problems[0]
    check(spin_cycles, lambda: tl.forward(plan, D, U, th, tl.FP32_3M, want_r=True)[:2], "forward")
    check(spin_cycles, lambda: tl.grad(plan, D, U, th, tl.FP32_3M), "grad")
    check(spin_cycles, lambda: tl.forward_tlr(plan, D, U, th, want_r=True), "forward_tlr")


def test_solves_return_early(tl, spin_cycles, problems):
    for k, (plan, D, U, th, _) in enumerate(problems):
        for line in (tl.LINE_DENSE, tl.LINE_TILE_GRAD):
            check(spin_cycles, lambda: tl.solve(plan, D, U, th, 3, precision=tl.FP32_3M, line_products=line),
                  f"solve[{k}, line {line}]")
    plans = [p[0] for p in problems]
    Ds, Us, ths = [p[1] for p in problems], [p[2] for p in problems], [p[3] for p in problems]
    for streams in (1, 2):
        check(spin_cycles, lambda: tl.solve_batched(plans, Ds, Us, ths, 3, precision=tl.FP32_3M, streams=streams,
                                                    line_products=tl.LINE_TILE_GRAD),
              f"solve_batched[streams {streams}]")
    check(spin_cycles, lambda: tl.admm_batched(plans, Ds, Us, ths, lams=(1.0,), outer=1, inner=2,
                                               precision=tl.FP32_3M, line_products=tl.LINE_TILE_GRAD),
          "admm_batched")


def test_permute_returns_early_and_flags_bad_entries(tl, spin_cycles, problems):
    plan, D, U, th, perm = problems[0]
    pd = torch.from_numpy(perm).cuda()
    check(spin_cycles, lambda: tl.permute_columns(D, pd), "permute_columns")
    # out-of-range entries: zero columns and the flag, no fault
    bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    pb = pd.clone()
    pb[3] = D.shape[1]
    pb[7] = -5
    out = tl.permute_columns(D, pb, bad=bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 1
    ref = D[:, pd.clamp(0, D.shape[1] - 1)]
    keep = torch.ones(D.shape[1], dtype=torch.bool, device="cuda")
    keep[3] = keep[7] = False
    assert torch.equal(out[:, keep], D[:, pb[keep]])
    assert torch.count_nonzero(out[:, ~keep]).item() == 0
    assert ref.shape == out.shape
    bad.zero_()
    tl.permute_columns(D, pd, bad=bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
