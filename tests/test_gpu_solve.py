"""GPU solve parity (L-BFGS / steepest descent with exact line search) vs the oracle.

Measures, after a fixed iteration count T:
  rel_f = |f(theta_gpu) - f(theta_or)| / f(theta_or), both by the oracle's FP64 forward;
  rel_X = ||C(theta_gpu) - C(theta_or)|| / ||C(theta_or)||   (gauge invariant);
  rel_theta = ||theta_gpu - theta_or|| / ||theta_or||.
The FP32 bar is 1e-5 on each.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_cases import from_geometry, from_workload, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def tl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_14973_amd as m
    m._lib.load()
    return m


def _metrics(case, th_gpu, th_or):
    f_g = O.objective(case.T, case.D, case.U, th_gpu)[0]
    f_o = O.objective(case.T, case.D, case.U, th_or)[0]
    Xg, Xo = O.assemble(case.T, th_gpu), O.assemble(case.T, th_or)
    return (abs(f_g - f_o) / f_o, np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo),
            np.linalg.norm(th_gpu - th_or) / np.linalg.norm(th_or))


def test_single_step_teacher_forced(tl):
    """One GPU iteration from the oracle's state after 10 iterations."""
    case = from_workload(synth.small(), 4)
    states = {}
    O.solve(case.T, case.D, case.U, case.theta, iters=10, record=lambda t, s: states.__setitem__(t, s))
    th10 = O.solve(case.T, case.D, case.U, case.theta, iters=10).theta
    th10 = th10.astype(np.complex64).astype(np.complex128)
    plan, D, U, _, _ = to_device(case, tl, torch)
    th = torch.from_numpy(th10.astype(np.complex64)).cuda()
    thg, fh = tl.solve(plan, D, U, th, iters=1)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, th10, iters=1)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    print(f"single step: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e}")
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL
    fh = fh.cpu().numpy()
    assert abs(fh[0] - ref.f_hist[0]) <= 1e-5 * ref.f_hist[0]
    assert abs(fh[1] - ref.f_hist[1]) <= 1e-5 * ref.f_hist[1]


@pytest.mark.parametrize("f_idx", [0, 3, 7])
def test_lbfgs_small_workload(tl, f_idx):
    wl = synth.small()
    case = from_workload(wl, f_idx)
    plan, D, U, th, _ = to_device(case, tl, torch)
    thg, fh = tl.solve(plan, D, U, th, iters=wl.iters, lbfgs_m=5)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=wl.iters, m=5)
    fh = fh.cpu().numpy()
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    rel_hist = np.abs(fh - ref.f_hist) / ref.f_hist
    print(f"f[{f_idx}] lbfgs: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e} max rel f_hist {rel_hist.max():.2e}"
          f" f0 {ref.f_hist[0]:.4e} fT {ref.f_hist[-1]:.4e}")
    assert np.all(np.diff(fh) <= 1e-6 * fh[0])
    assert rf <= FP32_TOL
    assert rx <= FP32_TOL
    assert rt <= FP32_TOL


def test_gd_small_workload(tl):
    wl = synth.small()
    case = from_workload(wl, 5)
    plan, D, U, th, _ = to_device(case, tl, torch)
    thg, fh = tl.solve(plan, D, U, th, iters=50, optimizer=tl.GD)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=50, optimizer="gd")
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    print(f"gd: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e}")
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL


def test_regularised_solve(tl):
    case = from_geometry(6, 5, "full", 17.0, synth.Layout([8, 8, 8, 6], [3, 2, 4, 1, 2, 5], [4, -1, 2, -1]),
                         1, "ragged_mixed", scale_theta=3.0)
    plan, D, U, th, _ = to_device(case, tl, torch)
    thg, fh = tl.solve(plan, D, U, th, iters=20, lam=0.1)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=20, lam=0.1)
    fh = fh.cpu().numpy()
    print("reg f_hist rel", np.max(np.abs(fh - ref.f_hist) / ref.f_hist))
    assert np.all(np.abs(fh - ref.f_hist) <= 1e-5 * ref.f_hist)


def test_batched_matches_single(tl):
    wl = synth.small()
    cases = [from_workload(wl, i) for i in range(4)]
    devs = [to_device(c, tl, torch) for c in cases]
    plans = [d[0] for d in devs]
    th_b, fh_b = tl.solve_batched(plans, [d[1] for d in devs], [d[2] for d in devs], [d[3] for d in devs],
                                  iters=20)
    singles = [tl.solve(d[0], d[1], d[2], d[3], iters=20) for d in devs]
    torch.cuda.synchronize()
    for (ts, fs), tb, fb in zip(singles, th_b, fh_b):
        assert torch.equal(ts, tb)
        assert torch.equal(fs, fb)


BF16_TOL = 5e-3


@pytest.mark.parametrize("f_idx", [1, 6])
def test_bf16x3_solve_small_workload(tl, f_idx):
    wl = synth.small()
    case = from_workload(wl, f_idx)
    plan, D, U, th, _ = to_device(case, tl, torch)
    thg, fh = tl.solve(plan, D, U, th, iters=wl.iters, precision=tl.BF16X3)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=wl.iters)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    print(f"bf16x3 f[{f_idx}]: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e}")
    assert rf <= BF16_TOL and rx <= BF16_TOL and rt <= BF16_TOL


def test_bf16x3_batched_matches_single(tl):
    wl = synth.small()
    devs = [to_device(from_workload(wl, i), tl, torch) for i in range(3)]
    th_b, fh_b = tl.solve_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs],
                                  [d[3] for d in devs], iters=10, precision=tl.BF16X3)
    singles = [tl.solve(d[0], d[1], d[2], d[3], iters=10, precision=tl.BF16X3) for d in devs]
    torch.cuda.synchronize()
    for (ts, fs), tb, fb in zip(singles, th_b, fh_b):
        assert torch.equal(ts, tb) and torch.equal(fs, fb)


@pytest.mark.parametrize("f_idx", [2, 5])
def test_fp32_3m_solve_small_workload(tl, f_idx):
    wl = synth.small()
    case = from_workload(wl, f_idx)
    plan, D, U, th, _ = to_device(case, tl, torch)
    thg, fh = tl.solve(plan, D, U, th, iters=wl.iters, precision=tl.FP32_3M)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=wl.iters)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    print(f"fp32-3m f[{f_idx}]: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e}")
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL


def test_fp32_3m_batched_matches_single(tl):
    wl = synth.small()
    devs = [to_device(from_workload(wl, i), tl, torch) for i in range(3)]
    th_b, fh_b = tl.solve_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs],
                                  [d[3] for d in devs], iters=10, precision=tl.FP32_3M)
    singles = [tl.solve(d[0], d[1], d[2], d[3], iters=10, precision=tl.FP32_3M) for d in devs]
    torch.cuda.synchronize()
    for (ts, fs), tb, fb in zip(singles, th_b, fh_b):
        assert torch.equal(ts, tb) and torch.equal(fs, fb)


@pytest.mark.parametrize("precision_name,streams", [("FP32_3M", 2), ("FP32_3M", 4), ("FP32", 3), ("BF16X3", 2)])
def test_batched_streams_match_one_stream(tl, precision_name, streams):
    """Sub-batches on their own streams give the one-stream results bit for bit (problem i in
    sub-batch i % streams; 5 problems so the sub-batches are uneven)."""
    prec = getattr(tl, precision_name)
    wl = synth.small()
    devs = [to_device(from_workload(wl, i), tl, torch) for i in range(5)]
    args = ([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs], [d[3] for d in devs])
    th1, fh1 = tl.solve_batched(*args, iters=12, precision=prec)
    thk, fhk = tl.solve_batched(*args, iters=12, precision=prec, streams=streams)
    torch.cuda.synchronize()
    for a, b, fa, fb in zip(th1, thk, fh1, fhk):
        assert torch.equal(a, b) and torch.equal(fa, fb)


def test_admm_batched_streams_match_one_stream(tl):
    wl = synth.small()
    devs = [to_device(from_workload(wl, i), tl, torch) for i in range(3)]
    args = ([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs], [d[3] for d in devs])
    kw = dict(lams=(1.0, 0.1), outer=2, inner=4, precision=tl.FP32_3M)
    th1, fh1 = tl.admm_batched(*args, **kw)
    th3, fh3 = tl.admm_batched(*args, streams=3, **kw)
    torch.cuda.synchronize()
    for a, b, fa, fb in zip(th1, th3, fh1, fh3):
        assert torch.equal(a, b) and torch.equal(fa, fb)


def test_batched_streams_invalid(tl):
    wl = synth.small()
    devs = [to_device(from_workload(wl, i), tl, torch) for i in range(2)]
    for bad in (-1, 9):
        with pytest.raises(tl.TLRMDDError) as e:
            tl.solve_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs],
                             [d[3] for d in devs], iters=2, streams=bad)
        assert e.value.status == 1
