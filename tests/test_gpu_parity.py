"""GPU parity of the HIP library against the FP64 oracle (through the C ABI).

Tolerances follow from FP32 arithmetic: every entry of r = D X - U may carry
about sqrt(K) u (|D||X| + |U|)_entry of rounding (u = 2^-24) and the gradient
inherits the propagated bound (tests/gpu_cases.py); a factor 8 of slack
covers the constant. Objectives: relative 1e-5. Assembled X: exactly
symmetric, bit for bit.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_cases import U32, c64, from_geometry, from_workload, gradient_bound, residual_bound, to_device  # noqa: F401

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_14973_amd as m
    m._lib.load()
    return m


def _cases():
    return [
        ("small", lambda: from_workload(synth.small(), 3)),
        ("ragged_mixed", lambda: from_geometry(6, 5, "full", 17.0,
                                               synth.Layout([8, 8, 8, 6], [3, 2, 4, 1, 2, 5], [4, -1, 2, -1]),
                                               1, "ragged_mixed", scale_theta=3.0)),
        ("multi_tile", lambda: from_geometry(20, 15, "half", 23.0, synth.uniform_layout(300, 64, 12, 20),
                                             2, "multi_tile", scale_theta=2.0)),
        ("dense_diag", lambda: from_geometry(12, 11, "full", 9.0, synth.uniform_layout(132, 40, 6, -1),
                                             3, "dense_diag", scale_theta=2.0)),
        # ranks above one 64-entry gradient item and one 32-entry assembly stage; ragged 32-wide last tile
        ("high_rank", lambda: from_geometry(18, 16, "half", 27.0, synth.uniform_layout(288, 128, 70, 50),
                                            4, "high_rank")),
        # single-block tile pairs with 33-64 rank entries (two rank phases of the tile-pair gradient;
        # the second half-filled) and Q Q^T tiles past 32 rank entries
        ("two_phase", lambda: from_geometry(16, 12, "full", 31.0, synth.uniform_layout(192, 64, 45, 40),
                                            5, "two_phase")),
        # tiles of 100: every pair spans 2 x 2 blocks, the second 36 wide
        ("partial_blocks", lambda: from_geometry(20, 15, "full", 13.0, synth.uniform_layout(300, 100, 20, 30),
                                                 6, "partial_blocks", scale_theta=2.0)),
    ]


CASES = _cases()


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_forward_parity(tl, name, mk):
    case = mk()
    plan, D, U, th, perm = to_device(case, tl, torch)
    assert np.array_equal(perm, O.hilbert_order(case.ix, case.iy))
    f, r, X = tl.forward(plan, D, U, th, want_r=True, want_X=True)
    torch.cuda.synchronize()
    Xo = O.assemble(case.T, case.theta)
    fo, ro = O.objective(case.T, case.D, case.U, case.theta)
    Xg = X.cpu().numpy().astype(np.complex128)
    rg = r.cpu().numpy().astype(np.complex128)
    # X: exactly symmetric and within FP32 rounding of the oracle
    assert np.array_equal(X.cpu().numpy(), X.cpu().numpy().T)
    kmax = max([k for (_, _, k) in case.T.pairs] + [max(case.T.d)])
    tolX = 8 * np.sqrt(kmax) * U32 * (O.assemble(case.T, np.abs(case.theta).astype(complex)).real + 1e-30)
    assert np.all(np.abs(Xg - Xo) <= tolX + 8 * U32 * np.abs(Xo))
    # r element-wise against the derived FP32 bound
    bound = 8 * residual_bound(case, Xo)
    err = np.abs(rg - ro)
    assert np.all(err <= bound), f"max err/bound {np.max(err / bound)}"
    assert abs(f.item() - fo) <= 1e-5 * fo


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_gradient_parity(tl, name, mk):
    case = mk()
    plan, D, U, th, _ = to_device(case, tl, torch)
    f, g = tl.grad(plan, D, U, th)
    torch.cuda.synchronize()
    fo, go = O.gradient(case.T, case.D, case.U, case.theta)
    Xo = O.assemble(case.T, case.theta)
    ro = O.residual(case.D, Xo, case.U)
    gg = g.cpu().numpy().astype(np.complex128)
    bound = 8 * gradient_bound(case, Xo, ro) + 1e-30
    err = np.abs(gg - go)
    assert np.all(err <= bound), f"max err/bound {np.max(err / bound)}"
    assert abs(f.item() - fo) <= 1e-5 * fo


def test_forward_is_deterministic(tl):
    case = from_workload(synth.small(), 2)
    plan, D, U, th, _ = to_device(case, tl, torch)
    a = tl.grad(plan, D, U, th)
    b = tl.grad(plan, D, U, th)
    torch.cuda.synchronize()
    assert a[0].item() == b[0].item()
    assert torch.equal(a[1], b[1])


def test_zero_residual_at_true_factors(tl):
    # U built on the CPU from the complex64 factors: the GPU objective must be at FP32 rounding level
    wl = synth.small()
    geom = wl.geometry()
    prob = synth.make_problem(geom, 12.0, None, 0.0, 1, 0)
    lay = wl.layout(0)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    th = c64(wl.theta0(0, lay) * 3.0)
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    D = O.permute_columns(c64(prob.D), perm)
    U = D @ O.assemble(T, th)
    dev = torch.device("cuda")
    plan = tl.Plan.from_layout(lay, 64)
    Dg = torch.from_numpy(np.ascontiguousarray(D, dtype=np.complex64)).to(dev)
    Ug = torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex64)).to(dev)
    thg = torch.from_numpy(th.astype(np.complex64)).to(dev)
    f, g = tl.grad(plan, Dg, Ug, thg)
    torch.cuda.synchronize()
    fU = 0.5 * np.vdot(U, U).real
    assert f.item() <= 1e-10 * fU
    assert g.abs().max().item() <= 1e-4 * np.abs(O.gradient(T, D, np.zeros_like(U), th)[1]).max()


def test_invalid_arguments_raise(tl):
    case = from_workload(synth.small(), 0)
    plan, D, U, th, _ = to_device(case, tl, torch)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(tl.TLRMDDError) as e:
        tl.forward(plan, D, U, th, workspace=ws)
    assert e.value.status == 2
    with pytest.raises(tl.TLRMDDError) as e:
        tl.forward(plan, D, U, th, precision=7)
    assert e.value.status == 1


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_bf16x3_forward_and_gradient_parity(tl, name, mk):
    from gpu_cases import gradient_bound_bf16, residual_bound_bf16
    case = mk()
    plan, D, U, th, _ = to_device(case, tl, torch)
    f, r, X = tl.forward(plan, D, U, th, precision=tl.BF16X3, want_r=True, want_X=True)
    fg, g = tl.grad(plan, D, U, th, precision=tl.BF16X3)
    torch.cuda.synchronize()
    Xo = O.assemble(case.T, case.theta)
    fo, ro = O.objective(case.T, case.D, case.U, case.theta)
    _, go = O.gradient(case.T, case.D, case.U, case.theta)
    assert np.array_equal(X.cpu().numpy(), X.cpu().numpy().T)
    err = np.abs(r.cpu().numpy().astype(np.complex128) - ro)
    bound = 8 * residual_bound_bf16(case, Xo)
    print(f"{name} bf16x3: max r err/bound {np.max(err / bound):.3f}, rel f {abs(f.item() - fo) / fo:.2e}")
    assert np.all(err <= bound)
    gerr = np.abs(g.cpu().numpy().astype(np.complex128) - go)
    gb = 8 * gradient_bound_bf16(case, Xo, ro) + 1e-30
    print(f"{name} bf16x3: max g err/bound {np.max(gerr / gb):.3f}")
    assert np.all(gerr <= gb)
    assert abs(f.item() - fo) <= 5e-3 * fo and abs(fg.item() - fo) <= 5e-3 * fo


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_fp32_3m_forward_and_gradient_parity(tl, name, mk):
    """Three-real-product form: Im C = (Ar+Ai)(Br+Bi) - ArBr - AiBi adds the rounding of two sums and
    of products of magnitude up to 2|a||b|, so the FP32 bounds grow by a factor 4."""
    case = mk()
    plan, D, U, th, _ = to_device(case, tl, torch)
    f, r, _ = tl.forward(plan, D, U, th, precision=tl.FP32_3M, want_r=True)
    fg, g = tl.grad(plan, D, U, th, precision=tl.FP32_3M)
    torch.cuda.synchronize()
    Xo = O.assemble(case.T, case.theta)
    fo, ro = O.objective(case.T, case.D, case.U, case.theta)
    _, go = O.gradient(case.T, case.D, case.U, case.theta)
    err = np.abs(r.cpu().numpy().astype(np.complex128) - ro)
    bound = 4 * 8 * residual_bound(case, Xo)
    gerr = np.abs(g.cpu().numpy().astype(np.complex128) - go)
    gb = 4 * 8 * gradient_bound(case, Xo, ro) + 1e-30
    print(f"{name} fp32-3m: max r err/bound {np.max(err / bound):.3f}, max g err/bound {np.max(gerr / gb):.3f}, "
          f"rel f {abs(f.item() - fo) / fo:.2e}")
    assert np.all(err <= bound)
    assert np.all(gerr <= gb)
    assert abs(f.item() - fo) <= 1e-5 * fo and abs(fg.item() - fo) <= 1e-5 * fo


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_adjoint_solution(tl, prec):
    case = from_geometry(12, 11, "half", 14.0, synth.uniform_layout(132, 40, 6, 7), 4, "adjoint")
    plan, D, U, th, _ = to_device(case, tl, torch)
    X = tl.adjoint(plan, D, U, precision=tl.FP32 if prec == "fp32" else tl.BF16X3)
    torch.cuda.synchronize()
    ref = case.D.conj().T @ case.U
    err = np.abs(X.cpu().numpy().astype(np.complex128) - ref)
    aref = np.abs(case.D).T @ np.abs(case.U)
    unit = U32 * np.sqrt(case.D.shape[0]) if prec == "fp32" else 2.0 ** -15 + U32 * np.sqrt(case.D.shape[0])
    assert np.all(err <= 8 * unit * aref + 1e-30)


def test_benchmark_solver_closed_form(tl):
    """Preconditioned Tikhonov benchmark solver against its closed-form least-squares solution."""
    rng = np.random.default_rng(31)
    n, ns, lam = 12, 20, 0.05
    D = c64((rng.standard_normal((ns, n)) + 1j * rng.standard_normal((ns, n))) / 4)
    U = c64((rng.standard_normal((ns, n)) + 1j * rng.standard_normal((ns, n))) / 4)
    cols = []
    for q in range(n * n):
        E = np.zeros(n * n, complex)
        E[q] = 1
        E = E.reshape(n, n)
        cols.append((D @ (0.5 * (E + E.T))).ravel())
    A = np.stack(cols, axis=1)
    Aa = np.vstack([A, np.sqrt(2 * lam) * np.eye(n * n)])
    z, *_ = np.linalg.lstsq(Aa, np.concatenate([U.ravel(), np.zeros(n * n)]), rcond=None)
    Zs = z.reshape(n, n)
    Xs = 0.5 * (Zs + Zs.T)
    fstar = 0.5 * np.linalg.norm(A @ z - U.ravel()) ** 2 + lam * np.vdot(z, z).real
    dev = torch.device("cuda")
    Dg = torch.from_numpy(D.astype(np.complex64)).to(dev)
    Ug = torch.from_numpy(U.astype(np.complex64)).to(dev)
    X, fh = tl.benchmark_solve(Dg, Ug, lam, iters=150, lbfgs_m=10)
    torch.cuda.synchronize()
    assert fh[-1].item() == pytest.approx(fstar, rel=1e-5)
    assert np.allclose(X.cpu().numpy(), Xs, atol=1e-4 * np.abs(Xs).max())
