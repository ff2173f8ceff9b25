"""tlrmdd_grad_noalloc (the gradient call whose scratch is the library's fixed device array) against
tlrmdd_grad with a caller workspace, called through the C ABI.

Both run the same kernels, so objective and gradient must agree bit for bit (stronger than the FP32
parity bar). Two calls in a row, the second on a smaller problem, so the second call reuses the
array the first one left behind; then the size limit: a plan whose scratch exceeds the array is
refused with TLRMDD_WORKSPACE.
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


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def grad_noalloc(tl, plan, D, U, th, precision):
    lib = tl._lib.load()
    f = torch.empty((), dtype=torch.float64, device="cuda")
    g = torch.empty_like(th)
    st = lib.tlrmdd_grad_noalloc(plan.handle, _ptr(D), _ptr(U), _ptr(th), _ptr(f), _ptr(g), precision,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, f, g


def grad_workspace(tl, plan, D, U, th, precision):
    lib = tl._lib.load()
    f = torch.empty((), dtype=torch.float64, device="cuda")
    g = torch.empty_like(th)
    ws = plan.workspace(tl._lib.OP_GRAD)
    tl._lib.check(lib.tlrmdd_grad(plan.handle, _ptr(D), _ptr(U), _ptr(th), _ptr(f), _ptr(g), precision, _ptr(ws),
                                  ws.numel(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
                  "tlrmdd_grad")
    return f, g


@pytest.mark.parametrize("precision", ["FP32", "FP32_3M", "BF16X3"])
def test_noalloc_matches_workspace_call_twice(tl, precision):
    prec = getattr(tl, precision)
    big = from_workload(synth.batched(), 12)                                    # nr = ns = 1024, tile 256
    small = from_geometry(10, 9, "full", 12.0, synth.uniform_layout(90, 32, 5, -1), 7, "ragged 90")
    for case in (big, small):
        plan, D, U, th, _ = to_device(case, tl, torch)
        st, f1, g1 = grad_noalloc(tl, plan, D, U, th, prec)
        assert st == tl._lib.OK, tl._lib.load().tlrmdd_last_error()
        f2, g2 = grad_workspace(tl, plan, D, U, th, prec)
        torch.cuda.synchronize()
        assert torch.equal(f1, f2), case.name
        assert torch.equal(g1, g2), case.name
        assert torch.isfinite(g1).all()


def test_noalloc_rejects_plans_above_the_limit(tl):
    lay = synth.uniform_layout(2048, 256, 8, 8)   # nr = ns = 2048: 160 MiB of scratch
    plan = tl.Plan.from_layout(lay, 2048)
    assert plan.workspace_bytes(tl._lib.OP_GRAD) > 64 << 20
    D = torch.zeros((2048, 2048), dtype=torch.complex64, device="cuda")
    th = torch.zeros(plan.theta_size, dtype=torch.complex64, device="cuda")
    st, _, _ = grad_noalloc(tl, plan, D, D, th, tl.FP32)
    assert st == tl._lib.WORKSPACE
    assert b"scratch" in tl._lib.load().tlrmdd_last_error()
