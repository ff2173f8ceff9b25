"""Pins for the oracle's tile assembly, objective and gradient.

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own formulas:
  * reciprocity: X = X^T exactly (Theory; Tile Low-rank MDD);
  * the packing order of the stacks Zbar, Lbar, Rbar against a hand-built 2x2
    and 3x3 tiling (Tile Low-rank MDD, stack definitions);
  * single-tile special cases: global Q Q^T and (Z + Z^T)/2;
  * zero residual / zero gradient at the true factors on noise-free data;
  * central finite differences and torch.autograd in complex128 (gradient
    equations DXLR);
  * gauge and Euler identities of the factorisation;
  * Hilbert equivalence f(S X_h S^T; D, U) = f(X_h; D S, U S) (eq. axb_sd).
"""
import numpy as np
import pytest

import oracle as O
import synth


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _mixed_tiling():
    # ragged tiles, mixed diagonal modes and ranks
    return O.tiling([5, 4, 3], [2, 3, 1], [2, -1, 3])


def test_packing_order_hand_built():
    T = _mixed_tiling()
    rng = np.random.default_rng(1)
    Q0 = _rand(rng, 5, 2)
    Z1 = _rand(rng, 4, 4)
    Q2 = _rand(rng, 3, 3)
    # t order: (1,0) k=2, (2,0) k=3, (2,1) k=1
    L10, L20, L21 = _rand(rng, 4, 2), _rand(rng, 3, 3), _rand(rng, 3, 1)
    R10, R20, R21 = _rand(rng, 2, 5), _rand(rng, 3, 5), _rand(rng, 1, 4)
    theta = np.concatenate([Q0.ravel(), Z1.ravel(), Q2.ravel(),
                            L10.ravel(), L20.ravel(), L21.ravel(),
                            R10.ravel(), R20.ravel(), R21.ravel()])
    assert T.size == theta.size
    X10, X20, X21 = L10 @ R10, L20 @ R20, L21 @ R21
    expect = np.block([
        [Q0 @ Q0.T, X10.T, X20.T],
        [X10, (Z1 + Z1.T) / 2, X21.T],
        [X20, X21, Q2 @ Q2.T],
    ])
    X = O.assemble(T, theta)
    assert np.allclose(X, expect, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kd", [4, -1])
def test_assembly_exactly_symmetric(kd):
    lay = synth.uniform_layout(64, 16, 4, kd)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    th = synth.init_theta(T.size, 9, 0)
    X = O.assemble(T, th)
    assert np.array_equal(X, X.T)
    X1, X2 = O.assemble_directional(T, th, synth.init_theta(T.size, 9, 1))
    assert np.array_equal(X1, X1.T) and np.array_equal(X2, X2.T)


def test_single_tile_special_cases():
    rng = np.random.default_rng(2)
    Q = _rand(rng, 7, 3)
    T = O.tiling([7], [], [3])
    assert np.allclose(O.assemble(T, Q.ravel()), Q @ Q.T, atol=1e-14)
    Z = _rand(rng, 7, 7)
    T = O.tiling([7], [], [-1])
    assert np.allclose(O.assemble(T, Z.ravel()), 0.5 * (Z + Z.T), atol=1e-14)


def test_offdiagonal_tiles_have_the_stated_rank():
    lay = synth.uniform_layout(48, 16, 3, 5)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    X = O.assemble(T, synth.init_theta(T.size, 9, 2))
    for (i, j, k) in T.pairs:
        sv = np.linalg.svd(X[T.start[i]:T.start[i] + T.d[i], T.start[j]:T.start[j] + T.d[j]],
                           compute_uv=False)
        assert np.sum(sv > 1e-12 * sv[0]) == k
    for i in range(T.n):
        sv = np.linalg.svd(X[T.start[i]:T.start[i] + 16, T.start[i]:T.start[i] + 16], compute_uv=False)
        assert np.sum(sv > 1e-12 * sv[0]) == 5


def test_zero_residual_at_true_factors():
    wl = synth.small()
    geom = wl.geometry()
    prob = synth.make_problem(geom, 12.0, None, 0.0, 1, 0)
    lay = wl.layout(0)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    th = wl.theta0(0, lay) * 3.0
    # U built by an independent route: explicit block matrix of the factors
    X = np.zeros((64, 64), complex)
    for i in range(T.n):
        B = O.diag_block(T, th, i)
        X[16 * i:16 * i + 16, 16 * i:16 * i + 16] = B @ B.T
    for t, (i, j, k) in enumerate(T.pairs):
        blk = O.L_block(T, th, t) @ O.R_block(T, th, t)
        X[16 * i:16 * i + 16, 16 * j:16 * j + 16] = blk
        X[16 * j:16 * j + 16, 16 * i:16 * i + 16] = blk.T
    U = prob.D @ X
    f, g = O.gradient(T, prob.D, U, th)
    assert f <= 1e-26 * np.vdot(U, U).real
    assert np.max(np.abs(g)) <= 1e-12 * np.max(np.abs(prob.D)) ** 2 * np.max(np.abs(th)) * 64


def _small_problem(kd=3, seed=3):
    rng = np.random.default_rng(seed)
    T = O.tiling([4, 3, 3], [2, 2, 1], [kd, -1, 2])
    D = _rand(rng, 9, T.nr) / 3
    U = _rand(rng, 9, T.nr) / 3
    th = 0.5 * _rand(rng, T.size)
    return T, D, U, th


def test_gradient_central_differences():
    T, D, U, th = _small_problem()
    f, g = O.gradient(T, D, U, th)
    idx = np.arange(T.size)
    fd = O.fd_gradient_entries(T, D, U, th, idx, h=1e-6)
    err = np.abs(fd - g)
    assert np.all(err <= 1e-6 * np.max(np.abs(g)) + 1e-9 * f)


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    T, D, U, th = _small_problem(seed=4)
    f, g = O.gradient(T, D, U, th)
    tD = torch.tensor(D)
    tU = torch.tensor(U)
    tth = torch.tensor(th, requires_grad=True)

    def blk(t, o, r, c):
        return t[o:o + r * c].reshape(r, c)

    rows = []
    pairs = {(i, j): n for n, (i, j, k) in enumerate(T.pairs)}
    for i in range(T.n):
        row = []
        for j in range(T.n):
            if i == j:
                B = blk(tth, T.off_diag[i], T.d[i], T.d[i] if T.kdiag[i] < 0 else T.kdiag[i])
                row.append(0.5 * (B + B.T) if T.kdiag[i] < 0 else B @ B.T)
            else:
                a, b = (i, j) if i > j else (j, i)
                n = pairs[(a, b)]
                k = T.pairs[n][2]
                M = blk(tth, T.off_L[n], T.d[a], k) @ blk(tth, T.off_R[n], k, T.d[b])
                row.append(M if i > j else M.T)
        rows.append(torch.cat(row, dim=1))
    X = torch.cat(rows, dim=0)
    r = tD @ X - tU
    loss = 0.5 * (r.conj() * r).real.sum()
    loss.backward()
    assert abs(loss.item() - f) <= 1e-12 * f
    # torch's complex .grad is df/dRe + i df/dIm, the convention used here
    assert np.allclose(tth.grad.numpy(), g, rtol=0, atol=1e-12 * np.max(np.abs(g)))


def test_gauge_identities():
    T, D, U, th = _small_problem(seed=5)
    _, g = O.gradient(T, D, U, th)
    rng = np.random.default_rng(6)
    for t, (i, j, k) in enumerate(T.pairs):
        A = _rand(rng, k, k)
        L, R = O.L_block(T, th, t), O.R_block(T, th, t)
        gL, gR = O.L_block(T, g, t), O.R_block(T, g, t)
        lhs = O.re_dot(gL, L @ A)
        rhs = O.re_dot(gR, A @ R)
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs) + 1)
    for i in range(T.n):
        if T.kdiag[i] < 0:
            continue
        k = T.kdiag[i]
        A = _rand(rng, k, k)
        A = A - A.T
        Q = O.diag_block(T, th, i)
        assert abs(O.re_dot(O.diag_block(T, g, i), Q @ A)) <= 1e-12 * np.linalg.norm(Q) * np.linalg.norm(g)


def test_euler_identity():
    T, D, U, th = _small_problem(seed=7)
    f, r = O.objective(T, D, U, th)
    W = D.conj().T @ r
    g = O.tile_gradient(T, th, W)
    # X_lowrank: the tiles quadratic in theta; X_dense: the linear (dense diagonal) tiles
    Xd = np.zeros((T.nr, T.nr), complex)
    for i in range(T.n):
        if T.kdiag[i] < 0:
            s = slice(T.start[i], T.start[i] + T.d[i])
            Z = O.diag_block(T, th, i)
            Xd[s, s] = 0.5 * (Z + Z.T)
    Xl = O.assemble(T, th) - Xd
    lhs = O.re_dot(g, th)
    rhs = O.re_dot(W, 2 * Xl + Xd)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_hilbert_equivalence_and_source_permutation():
    g6 = synth.make_geometry(6, 5)
    perm = O.hilbert_order(g6.rec_ix, g6.rec_iy)
    rng = np.random.default_rng(8)
    D = _rand(rng, 20, 30)
    U = _rand(rng, 20, 30)
    lay = synth.uniform_layout(30, 8, 2, 3)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    th = 0.3 * _rand(rng, T.size)
    Xh = O.assemble(T, th)
    X = O.unpermute(Xh, perm)
    f_nat = 0.5 * np.linalg.norm(D @ X - U) ** 2
    f_h, _ = O.objective(T, O.permute_columns(D, perm), O.permute_columns(U, perm), th)
    assert abs(f_nat - f_h) <= 1e-12 * f_nat
    sp = rng.permutation(20)
    f_s, _ = O.objective(T, D[sp], U[sp], th)
    f_0, _ = O.objective(T, D, U, th)
    assert abs(f_s - f_0) <= 1e-12 * f_0


def test_gradient_entries_match_full_gradient():
    """The entry-wise gradient (used for sampled checks at large sizes) equals
    the full tile gradient on every entry of a mixed layout."""
    T, D, U, th = _small_problem(seed=21)
    f, r = O.objective(T, D, U, th)
    g = O.tile_gradient(T, th, D.conj().T @ r)
    idx = np.arange(T.size)
    ge = O.gradient_entries(T, D, r, th, idx)
    assert np.allclose(ge, g, rtol=0, atol=1e-12 * np.abs(g).max())


def test_fd_entries_large_matches_plain_fd():
    T, D, U, th = _small_problem(seed=22)
    idx = np.arange(0, T.size, 3)
    a = O.fd_entries_large(T, D, U, th, idx)
    b = O.fd_gradient_entries(T, D, U, th, idx)
    assert np.allclose(a, b, rtol=1e-7, atol=1e-9)
