"""Kernel timing (tlrmdd_timing_begin / tlrmdd_timing_begin_kinds / tlrmdd_timing_end) on a batched
solve of the nr 64 parity workload: timing every kind and timing one kind count the same launches
and work for that kind, the other kinds read zero under the one-kind timer, and timing changes no
result (the solves under either timer equal an untimed one bit for bit)."""
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


def test_one_kind_timer_counts_what_the_full_timer_counts(tl):
    wl = synth.small()
    devs = [to_device(from_workload(wl, i), tl, torch) for i in range(len(wl.freqs))]
    plans, Ds, Us, ths = [d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs], [d[3] for d in devs]
    iters = 12
    th0, fh0 = tl.solve_batched(plans, Ds, Us, ths, iters)
    torch.cuda.synchronize()
    with tl.KernelTimer() as full:
        th1, fh1 = tl.solve_batched(plans, Ds, Us, ths, iters)
        torch.cuda.synchronize()
    with tl.KernelTimer(kinds=["gemm_line", "gram"]) as some:
        th2, fh2 = tl.solve_batched(plans, Ds, Us, ths, iters)
        torch.cuda.synchronize()
    for a, b, c in zip(th0, th1, th2):
        assert torch.equal(a, b) and torch.equal(a, c)
    for a, b, c in zip(fh0, fh1, fh2):
        assert torch.equal(a, b) and torch.equal(a, c)
    assert full.launches["gemm_line"] >= iters and full.launches["gram"] > 0
    assert full.launches["gemm_adjoint"] > 0 and full.launches["combine"] > 0
    for k in tl._lib.KIND_NAMES:
        if k in ("gemm_line", "gram"):
            assert some.launches[k] == full.launches[k], k
            assert some.flops[k] == full.flops[k] and some.bytes[k] == full.bytes[k], k
            assert some.ms[k] > 0, k
        else:
            assert some.launches[k] == 0 and some.ms[k] == 0.0, k
