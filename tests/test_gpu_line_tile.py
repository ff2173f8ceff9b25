"""GPU exact line search in tile form (tlrmdd_opts.line_products = TLRMDD_LINE_TILE) vs the oracle.

The line search's [a | b] = D [X1 | X2] is formed from packed factor blocks of theta and p in two
product stages instead of from the assembled X1, X2; the result is the same up to rounding, so
the solve is held to the FP32 bar against the FP64 oracle (rel_f, rel_X, rel_theta and the
f-history entry by entry). Batched calls group the problems by form; every problem's result
equals its single-problem solve bit for bit.
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


def _case(seed, k_off, k_diag, name, tiles=(256, 256)):
    """32 x 16 receivers (nr = 512), sources on every other line (ns = 256), two tiles of 256 (or
    the given tile sizes, every off-diagonal tile of rank k_off)."""
    nt = len(tiles)
    lay = synth.Layout(np.array(tiles), np.full(nt * (nt - 1) // 2, k_off), np.array(k_diag))
    return from_geometry(32, 16, "half", 12.0, lay, seed, name)


def _metrics(case, th_gpu, th_or):
    f_g = O.objective(case.T, case.D, case.U, th_gpu)[0]
    f_o = O.objective(case.T, case.D, case.U, th_or)[0]
    Xg, Xo = O.assemble(case.T, th_gpu), O.assemble(case.T, th_or)
    return (abs(f_g - f_o) / f_o, np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo),
            np.linalg.norm(th_gpu - th_or) / np.linalg.norm(th_or))


def test_line_form_query(tl):
    cases = {"eligible": _case(1, 10, [12, 20], "a"), "dense_diag": _case(1, 10, [-1, 20], "b")}
    plan = to_device(cases["eligible"], tl, torch)[0]
    assert tl.line_form(plan) == (True, 32)                       # kpad: a multiple of 32 for two tiles
    assert tl.line_form(plan, precision=tl.FP32) == (False, 0)    # tile form runs on the 3M products
    assert tl.line_form(plan, line_products=tl.LINE_DENSE) == (False, 0)
    assert tl.line_form(to_device(cases["dense_diag"], tl, torch)[0]) == (False, 0)


@pytest.mark.parametrize("seed,k_off,k_diag", [(3, 10, [12, 20]), (4, 32, [32, 7])])
def test_tile_line_search_solve_vs_oracle(tl, seed, k_off, k_diag):
    case = _case(seed, k_off, k_diag, "tile512")
    plan, D, U, th, _ = to_device(case, tl, torch)
    assert tl.line_form(plan)[0]
    iters = 20
    thg, fh = tl.solve(plan, D, U, th, iters=iters, precision=tl.FP32_3M, line_products=tl.LINE_TILE)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=iters)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    rel_h = np.max(np.abs(fh.cpu().numpy() - ref.f_hist) / ref.f_hist)
    print(f"tile line search k_off {k_off}: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e} "
          f"f_hist {rel_h:.2e}", flush=True)
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL and rel_h <= FP32_TOL


def test_tile_batched_groups_match_single(tl):
    cases = [_case(5, 10, [12, 20], "a"), _case(6, 3, [-1, 4], "dense"), _case(7, 20, [30, 9], "b"),
             _case(8, 5, [6, 7], "c")]
    devs = [to_device(c, tl, torch) for c in cases]
    kw = dict(iters=8, precision=tl.FP32_3M, line_products=tl.LINE_TILE)
    th_b, fh_b = tl.solve_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs],
                                  [d[3] for d in devs], **kw)
    singles = [tl.solve(d[0], d[1], d[2], d[3], **kw) for d in devs]
    torch.cuda.synchronize()
    for (ts, fs), tb, fb in zip(singles, th_b, fh_b):
        assert torch.equal(ts, tb) and torch.equal(fs, fb)


@pytest.mark.parametrize("streams", [1, 2, 3])
def test_tile_batched_two_classes_match_single(tl, streams):
    """Two tile classes (tile 256, kpad 32; tile 128, kpad 16) and a dense-form problem in one call,
    in an order that interleaves them: the call lists every sub-batch's problems by form; each
    problem's factors and f-history equal its single-problem solve bit for bit."""
    cases = [_case(11, 10, [12, 20], "a"), _case(12, 12, [9, 14, 5, 16], "q4a", tiles=(128,) * 4),
             _case(13, 3, [-1, 4], "dense"), _case(14, 20, [30, 9], "b"),
             _case(15, 6, [5, 6, 7, 8], "q4b", tiles=(128,) * 4)]
    devs = [to_device(c, tl, torch) for c in cases]
    forms = [tl.line_form(d[0]) for d in devs]
    assert forms == [(True, 32), (True, 16), (False, 0), (True, 32), (True, 16)]
    kw = dict(iters=6, precision=tl.FP32_3M, line_products=tl.LINE_TILE)
    th_b, fh_b = tl.solve_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs],
                                  [d[3] for d in devs], streams=streams, **kw)
    singles = [tl.solve(d[0], d[1], d[2], d[3], **kw) for d in devs]
    torch.cuda.synchronize()
    for (ts, fs), tb, fb in zip(singles, th_b, fh_b):
        assert torch.equal(ts, tb) and torch.equal(fs, fb)


def test_tile_admm_vs_oracle(tl):
    case = _case(9, 12, [10, 14], "admm")
    plan, D, U, th, _ = to_device(case, tl, torch)
    kw = dict(lams=(1.0, 0.1), outer=2, inner=6, rho=1.0)
    thg, fh = tl.admm(plan, D, U, th, precision=tl.FP32_3M, line_products=tl.LINE_TILE, **kw)
    torch.cuda.synchronize()
    ref = O.admm(case.T, case.D, case.U, case.theta, **kw)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    rel_h = np.max(np.abs(fh.cpu().numpy() - ref.f_hist) / ref.f_hist)
    print(f"tile admm: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e} f_hist {rel_h:.2e}", flush=True)
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL and rel_h <= FP32_TOL


# ---- gradient in tile form (line_products = LINE_TILE_GRAD) -------------------------------------------
# Its three products cost 3 Wg / nr of the adjoint product (Wg = nt kpad rounded up to 128), so it needs
# nr = 1024 here: 32 x 32 receivers, sources on every other line (ns = 512), four tiles of 256.

def _case_nr1024(seed, k_off, k_diag, name, tiles=(256,) * 4):
    nt = len(tiles)
    lay = synth.Layout(np.array(tiles), np.full(nt * (nt - 1) // 2, k_off), np.array(k_diag))
    return from_geometry(32, 32, "half", 12.0, lay, seed, name)


def test_tile_grad_form_query(tl):
    plan = to_device(_case_nr1024(21, 12, [9, 14, 5, 16], "g"), tl, torch)[0]
    assert tl.line_form(plan, line_products=tl.LINE_TILE_GRAD) == (2, 16)     # 3 * 128 / 1024 <= 0.6
    assert tl.line_form(plan, line_products=tl.LINE_TILE) == (1, 16)
    q8 = to_device(_case_nr1024(22, 20, [20] * 8, "q8", tiles=(128,) * 8), tl, torch)[0]
    assert tl.line_form(q8, line_products=tl.LINE_TILE_GRAD) == (2, 24)       # Wg 192: 0.5625 of the adjoint


@pytest.mark.parametrize("k_off", [6, 16])
def test_tile_grad_solve_vs_oracle(tl, k_off):
    case = _case_nr1024(23 + k_off, k_off, [4, k_off, 9, 12], f"g{k_off}")
    plan, D, U, th, _ = to_device(case, tl, torch)
    iters = 8
    thg, fh = tl.solve(plan, D, U, th, iters=iters, precision=tl.FP32_3M, line_products=tl.LINE_TILE_GRAD)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=iters)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    rel_h = np.max(np.abs(fh.cpu().numpy() - ref.f_hist) / ref.f_hist)
    print(f"tile gradient k_off {k_off}: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e} f_hist {rel_h:.2e}",
          flush=True)
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL and rel_h <= FP32_TOL


def test_tile_grad_first_gradient_vs_oracle(tl):
    """One iteration from theta0: the step is the exact line search along -g(theta0), so theta_1
    pins the tile-form gradient itself (theta_1 - theta0 = -alpha g) against the oracle's."""
    case = _case_nr1024(31, 10, [7, 10, 3, 16], "g1")
    plan, D, U, th, _ = to_device(case, tl, torch)
    thg, _ = tl.solve(plan, D, U, th, iters=1, precision=tl.FP32_3M, line_products=tl.LINE_TILE_GRAD)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=1)
    step_g = thg.cpu().numpy().astype(np.complex128) - case.theta
    step_o = ref.theta - case.theta
    rel = np.linalg.norm(step_g - step_o) / np.linalg.norm(step_o)
    print(f"tile gradient first step: rel {rel:.2e}", flush=True)
    assert rel <= FP32_TOL


@pytest.mark.parametrize("streams", [1, 2])
def test_tile_grad_batched_match_single(tl, streams):
    """Problems with the tile-form gradient in two tile classes (tile 256, kpad 16: Wg 64 in one
    64-column tile; tile 128, kpad 24: Wg 192, a full and a 64-column tile) and a dense-form problem,
    interleaved: every problem equals its single-problem solve bit for bit."""
    cases = [_case_nr1024(41, 12, [9, 14, 5, 16], "g_a"), _case_nr1024(42, 3, [-1, 4, 5, 6], "dense"),
             _case_nr1024(43, 20, [20] * 8, "q8", tiles=(128,) * 8), _case_nr1024(44, 5, [3, 4, 5, 6], "g_b")]
    devs = [to_device(c, tl, torch) for c in cases]
    kw = dict(iters=5, precision=tl.FP32_3M, line_products=tl.LINE_TILE_GRAD)
    assert [tl.line_form(d[0], line_products=tl.LINE_TILE_GRAD)[0] for d in devs] == [2, 0, 2, 2]
    th_b, fh_b = tl.solve_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs],
                                  [d[3] for d in devs], streams=streams, **kw)
    singles = [tl.solve(d[0], d[1], d[2], d[3], **kw) for d in devs]
    torch.cuda.synchronize()
    for (ts, fs), tb, fb in zip(singles, th_b, fh_b):
        assert torch.equal(ts, tb) and torch.equal(fs, fb)


def test_tile_grad_admm_vs_oracle(tl):
    case = _case_nr1024(51, 8, [6, 8, 10, 12], "gadmm")
    plan, D, U, th, _ = to_device(case, tl, torch)
    kw = dict(lams=(1.0, 0.1), outer=2, inner=4, rho=1.0)
    thg, fh = tl.admm(plan, D, U, th, precision=tl.FP32_3M, line_products=tl.LINE_TILE_GRAD, **kw)
    torch.cuda.synchronize()
    ref = O.admm(case.T, case.D, case.U, case.theta, **kw)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    rel_h = np.max(np.abs(fh.cpu().numpy() - ref.f_hist) / ref.f_hist)
    print(f"tile gradient admm: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e} f_hist {rel_h:.2e}", flush=True)
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL and rel_h <= FP32_TOL


def test_tile_grad_long_solve_with_lambda_vs_oracle(tl):
    """25 iterations (the residual is recomputed from theta at iteration 20) with the Frobenius term
    lam ||theta||^2: the tile-form gradient plus the regulariser's gradient, P_theta carried through 25
    updates."""
    case = _case_nr1024(61, 10, [8, 12, 6, 10], "glong")
    plan, D, U, th, _ = to_device(case, tl, torch)
    iters, lam = 25, 0.05
    thg, fh = tl.solve(plan, D, U, th, iters=iters, precision=tl.FP32_3M, lam=lam,
                       line_products=tl.LINE_TILE_GRAD)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=iters, lam=lam)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    rel_h = np.max(np.abs(fh.cpu().numpy() - ref.f_hist) / ref.f_hist)
    print(f"tile gradient 25 iterations, lam {lam}: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e} "
          f"f_hist {rel_h:.2e}", flush=True)
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL and rel_h <= FP32_TOL


@pytest.mark.parametrize("streams", [1, 2])
def test_tile_grad_admm_batched_match_single(tl, streams):
    cases = [_case_nr1024(71, 12, [9, 14, 5, 16], "g_a"), _case_nr1024(72, 3, [-1, 4, 5, 6], "dense"),
             _case_nr1024(73, 5, [3, 4, 5, 6], "g_b")]
    devs = [to_device(c, tl, torch) for c in cases]
    kw = dict(lams=(1.0, 0.1), outer=2, inner=3, rho=1.0, precision=tl.FP32_3M, line_products=tl.LINE_TILE_GRAD)
    th_b, fh_b = tl.admm_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs],
                                 [d[3] for d in devs], streams=streams, **kw)
    singles = [tl.admm(d[0], d[1], d[2], d[3], **kw) for d in devs]
    torch.cuda.synchronize()
    for (ts, fs), tb, fb in zip(singles, th_b, fh_b):
        assert torch.equal(ts, tb) and torch.equal(fs, fb)


def test_tile_forms_single_tile_and_ragged(tl):
    """Edge layouts: one Q Q^T tile over all receivers (nt = 1: kpad a multiple of 64) takes both tile
    forms and matches the oracle; a ragged layout (tiles 384 + 384 + 256) keeps the dense forms."""
    lay = synth.Layout(np.array([1024]), np.array([], dtype=np.int64), np.array([30]))
    case = from_geometry(32, 32, "half", 12.0, lay, 81, "one_tile")
    plan, D, U, th, _ = to_device(case, tl, torch)
    assert tl.line_form(plan, line_products=tl.LINE_TILE_GRAD) == (2, 64)   # 2.5*64/1024, 3*128/1024
    iters = 6
    thg, fh = tl.solve(plan, D, U, th, iters=iters, precision=tl.FP32_3M, line_products=tl.LINE_TILE_GRAD)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=iters)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    print(f"one tile: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e}", flush=True)
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL
    rag = synth.Layout(np.array([384, 384, 256]), np.full(3, 8), np.array([6, 6, 6]))
    plan_r = to_device(from_geometry(32, 32, "half", 12.0, rag, 82, "ragged"), tl, torch)[0]
    assert tl.line_form(plan_r, line_products=tl.LINE_TILE_GRAD) == (0, 0)


# ---- BF16 hi+lo split mode: dense products in BF16, the tile-form products on the FP32 three-product kernel
BF16_TOL = 5e-3


# In BF16 mode the tile forms must beat dense products that run about twice as fast: half the flop
# shares (both cases take both forms: Wg 64 is 0.375 of the adjoint at nr = 1024 and 0.1875 at 2048).
@pytest.mark.parametrize("shape", ["nr1024", "nr2048"])
def test_tile_forms_bf16_solve_vs_oracle(tl, shape):
    if shape == "nr1024":
        case = _case_nr1024(91, 10, [8, 12, 6, 10], "bf16")
        expect = (2, 16)
    else:
        lay = synth.Layout(np.array([256] * 8), np.full(28, 6), np.array([8, 5, 7, 8, 3, 6, 8, 4]))
        case = from_geometry(64, 32, "half", 12.0, lay, 96, "bf16_nr2048")
        expect = (2, 8)
    plan, D, U, th, _ = to_device(case, tl, torch)
    assert tl.line_form(plan, precision=tl.BF16X3, line_products=tl.LINE_TILE_GRAD) == expect
    iters = 8 if shape == "nr1024" else 4
    thg, fh = tl.solve(plan, D, U, th, iters=iters, precision=tl.BF16X3, line_products=tl.LINE_TILE_GRAD)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=iters)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    rel_h = np.max(np.abs(fh.cpu().numpy() - ref.f_hist) / ref.f_hist)
    print(f"bf16 tile forms {shape}: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e} f_hist {rel_h:.2e}",
          flush=True)
    assert rf <= BF16_TOL and rx <= BF16_TOL and rt <= BF16_TOL and rel_h <= BF16_TOL


def test_tile_forms_bf16_batched_match_single(tl):
    cases = [_case_nr1024(92, 12, [9, 14, 5, 16], "g_a"), _case_nr1024(93, 3, [-1, 4, 5, 6], "dense"),
             _case_nr1024(94, 20, [20] * 8, "q8", tiles=(128,) * 8), _case_nr1024(95, 5, [3, 4, 5, 6], "g_b")]
    devs = [to_device(c, tl, torch) for c in cases]
    kw = dict(iters=5, precision=tl.BF16X3, line_products=tl.LINE_TILE_GRAD)
    th_b, fh_b = tl.solve_batched([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs],
                                  [d[3] for d in devs], **kw)
    singles = [tl.solve(d[0], d[1], d[2], d[3], **kw) for d in devs]
    torch.cuda.synchronize()
    for (ts, fs), tb, fb in zip(singles, th_b, fh_b):
        assert torch.equal(ts, tb) and torch.equal(fs, fb)


def test_tile_grad_carried_theta_half_vs_oracle(tl):
    """nt kpad a multiple of 128 (4 tiles of 256, kpad 32): stage 1 forms only the direction half and
    the theta half is carried by P_th += step P_p, formed afresh after each residual recompute (every
    20 iterations); 25 iterations against the oracle."""
    case = _case_nr1024(101, 20, [18, 24, 30, 12], "carried")
    plan, D, U, th, _ = to_device(case, tl, torch)
    assert tl.line_form(plan, line_products=tl.LINE_TILE_GRAD) == (2, 32)
    iters = 25
    thg, fh = tl.solve(plan, D, U, th, iters=iters, precision=tl.FP32_3M, line_products=tl.LINE_TILE_GRAD)
    torch.cuda.synchronize()
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=iters)
    rf, rx, rt = _metrics(case, thg.cpu().numpy().astype(np.complex128), ref.theta)
    rel_h = np.max(np.abs(fh.cpu().numpy() - ref.f_hist) / ref.f_hist)
    print(f"carried theta half, 25 iterations: rel_f {rf:.2e} rel_X {rx:.2e} rel_theta {rt:.2e} f_hist {rel_h:.2e}",
          flush=True)
    assert rf <= FP32_TOL and rx <= FP32_TOL and rt <= FP32_TOL and rel_h <= FP32_TOL
