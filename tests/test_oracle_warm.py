"""Pins for the oracle's rank / tile-size estimate and warm start (Hyper-parameter
selection and initialization; the examples' entry-count study).

  * exactly low-rank tiles (built by the assembly from random factors) give back
    their ranks, and every count equals numpy.linalg.matrix_rank at the same
    threshold (an independent routine);
  * the entry count of the estimated layout equals the size of its packed
    theta, and is checked by hand at the true tile size;
  * the warm start reproduces an exactly low-rank X; for a general symmetric X
    each truncated tile has the Eckart-Young error sqrt(sum of the dropped sigma^2),
    and the full-rank Takagi factor gives Q Q^T = X.
"""
import numpy as np
import pytest

import oracle as O
import synth


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _low_rank_case(seed=31):
    rng = np.random.default_rng(seed)
    sizes = [8, 8, 8, 4]
    ro = [1, 3, 2, 4, 1, 2]          # (1,0) (2,0) (2,1) (3,0) (3,1) (3,2)
    rd = [2, -1, 3, 1]
    T = O.tiling(sizes, ro, rd)
    theta = _rand(rng, T.size)
    return T, O.assemble(T, theta), sizes, ro, rd


def test_exact_ranks_recovered():
    T, X, sizes, ro, rd = _low_rank_case()
    s, k_off, k_diag, v0 = O.tile_ranks(X, 8, eps=1e-9)
    assert s == sizes
    assert k_off == ro
    assert k_diag == [2, 8, 3, 1]     # the dense tile is numerically full rank
    assert v0 > 0


@pytest.mark.parametrize("d,eps", [(8, 0.01), (5, 0.05), (16, 0.001)])
def test_rank_counts_match_matrix_rank(d, eps):
    rng = np.random.default_rng(32)
    A = _rand(rng, 30, 30) * np.exp(-0.2 * np.arange(30))[None, :]
    X = A @ A.T                         # symmetric with decaying spectrum
    sizes, k_off, k_diag, v0 = O.tile_ranks(X, d, eps)
    start = np.concatenate([[0], np.cumsum(sizes)])
    t = 0
    for i in range(len(sizes)):
        for j in range(i + 1):
            blk = X[start[i]:start[i + 1], start[j]:start[j + 1]]
            k = k_diag[i] if i == j else k_off[t]
            sv = np.linalg.svd(blk, compute_uv=False)
            if not np.any(np.isclose(sv, eps * v0, rtol=1e-9)):
                assert k == np.linalg.matrix_rank(blk, tol=eps * v0)
            if i != j:
                t += 1


def test_entries_equal_theta_size_and_hand_count():
    T, X, sizes, ro, rd = _low_rank_case()
    s, k_off, k_diag, _ = O.tile_ranks(X, 8, eps=1e-9)
    rank_off, rank_diag, n = O.layout_from_ranks(s, k_off, k_diag)
    assert n == O.tiling(s, rank_off, rank_diag).size
    # by hand: off-diagonal k (d_i + d_j): 1*16 + 3*16 + 2*16 + 4*12 + 1*12 + 2*12 = 180;
    # diagonal: Q 8x2 = 16, dense 8x8 = 64, Q 8x3 = 24, Q 4x1 = 4 (rank 1 < 4/2)
    assert n == 180 + 16 + 64 + 24 + 4
    d, sizes_b, ro_b, rd_b, entries = O.choose_layout(X, [4, 8, 16], eps=1e-9)
    assert entries[1] == n and d == [4, 8, 16][int(np.argmin(entries))]


def test_warm_start_reproduces_low_rank_matrix():
    T, X, sizes, ro, rd = _low_rank_case()
    th = O.warm_start(T, X)
    Xw = O.assemble(T, th)
    assert np.allclose(Xw, X, atol=1e-10 * np.abs(X).max())


def test_warm_start_eckart_young():
    rng = np.random.default_rng(33)
    A = _rand(rng, 20, 20)
    X = A + A.T
    T = O.tiling([8, 8, 4], [3, 2, 1], [4, -1, 2])
    th = O.warm_start(T, X)
    Xw = O.assemble(T, th)
    st = T.start + [T.nr]
    for (i, j, k) in T.pairs:
        blk = X[st[i]:st[i + 1], st[j]:st[j + 1]]
        sv = np.linalg.svd(blk, compute_uv=False)
        err = np.linalg.norm(Xw[st[i]:st[i + 1], st[j]:st[j + 1]] - blk)
        assert err == pytest.approx(np.sqrt(np.sum(sv[k:] ** 2)), rel=1e-9)
    for i in range(T.n):
        blk = X[st[i]:st[i + 1], st[i]:st[i + 1]]
        err = np.linalg.norm(Xw[st[i]:st[i + 1], st[i]:st[i + 1]] - blk)
        if T.kdiag[i] < 0:
            assert err <= 1e-12 * np.abs(blk).max()
        else:
            sv = np.linalg.svd(blk, compute_uv=False)
            assert err == pytest.approx(np.sqrt(np.sum(sv[T.kdiag[i]:] ** 2)), rel=1e-9)


def test_takagi_full_rank():
    rng = np.random.default_rng(34)
    A = _rand(rng, 7, 7)
    Xs = A + A.T
    Q = O.takagi(Xs, 7)
    assert np.allclose(Q @ Q.T, Xs, atol=1e-12 * np.abs(Xs).max())


def test_hilbert_order_compresses_synthetic_green_function():
    """The examples' comparison (entry count, natural vs Hilbert ordering) on the synthetic truth."""
    geom = synth.make_geometry(16, 16, "full")
    prob = synth.make_problem(geom, 20.0, 20.0, 0.05, 96, 0)
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    Xn = prob.X_true
    Xh = Xn[np.ix_(perm, perm)]
    _, _, _, _, en = O.choose_layout(Xn, [16, 32, 64], eps=0.01)
    _, _, _, _, eh = O.choose_layout(Xh, [16, 32, 64], eps=0.01)
    assert min(eh) < min(en)
