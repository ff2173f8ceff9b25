"""The tile-form identities behind the library's factor-sized products, checked in NumPy (complex128)
against the oracle's dense definitions (CPU; no GPU code involved).

With every ordered tile pair written as a factor product X_ij = A_ij B_ij (i > j: A = L, B = R;
i < j: A = R_ji^T, B = L_ji^T; i = j: A = Q, B = Q^T):
  * line search: a = D X1 and b = D X2 column block by column block from P_i = D_:,i [A_p(i.) | A_th(i.)]
    (a_:,j = sum_i P_p(ij) B_th(ij) + P_th(ij) B_p(ij), b_:,j = sum_i P_p(ij) B_p(ij));
  * gradient: with W = D^H r, grad A_ij = D_:,i^H (r_:,j B_ij^H) and grad B_ij = (D_:,i A_ij)^H r_:,j summed
    over both orders of every pair give the gradient equations' W' R^H, L^H W', W' conj(Q);
  * residual: r_:,j = sum_i P_th(ij) B_th(ij) - U_:,j.
A wrong transpose, conjugate or pair order in the reformulation fails these comparisons.
"""
import numpy as np
import pytest

import oracle as O


def _problem(seed, tiles, k_off, k_diag, ns):
    rng = np.random.default_rng(seed)
    nt = len(tiles)
    T = O.tiling(tiles, [k_off] * (nt * (nt - 1) // 2), k_diag)
    cplx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    return T, cplx(T.size), cplx(T.size), cplx(ns, T.nr), cplx(ns, T.nr)


def _factor_pair(T, theta, i, j):
    """(A_ij, B_ij) with X_ij = A_ij B_ij."""
    if i == j:
        Q = O.diag_block(T, theta, i)
        return Q, Q.T
    if i > j:
        t = i * (i - 1) // 2 + j
        return O.L_block(T, theta, t), O.R_block(T, theta, t)
    t = j * (j - 1) // 2 + i
    return O.R_block(T, theta, t).T, O.L_block(T, theta, t).T


def _cols(T, j):
    return slice(T.start[j], T.start[j] + T.d[j])


@pytest.mark.parametrize("tiles,k_off,k_diag", [([16, 16, 16, 16], 5, [3, 6, 4, 8]),
                                                ([24, 16, 24], 7, [5, 2, 9]),
                                                ([32], 1, [11])])
def test_line_search_products_in_tile_form(tiles, k_off, k_diag):
    T, th, p, D, _ = _problem(1, tiles, k_off, k_diag, 40)
    X1, X2 = O.assemble_directional(T, th, p)
    a_ref, b_ref = D @ X1, D @ X2
    a = np.zeros_like(a_ref)
    b = np.zeros_like(b_ref)
    for j in range(T.n):
        for i in range(T.n):
            A_th, B_th = _factor_pair(T, th, i, j)
            A_p, B_p = _factor_pair(T, p, i, j)
            P_th, P_p = D[:, _cols(T, i)] @ A_th, D[:, _cols(T, i)] @ A_p   # stage 1, tile row i
            a[:, _cols(T, j)] += P_p @ B_th + P_th @ B_p                    # stage 2, tile column j
            b[:, _cols(T, j)] += P_p @ B_p
    assert np.linalg.norm(a - a_ref) <= 1e-12 * np.linalg.norm(a_ref)
    assert np.linalg.norm(b - b_ref) <= 1e-12 * np.linalg.norm(b_ref)


@pytest.mark.parametrize("tiles,k_off,k_diag", [([16, 16, 16, 16], 5, [3, 6, 4, 8]),
                                                ([24, 16, 24], 7, [5, 2, 9]),
                                                ([32], 1, [11])])
def test_gradient_in_tile_form(tiles, k_off, k_diag):
    T, th, _, D, r = _problem(2, tiles, k_off, k_diag, 40)
    g_ref = O.tile_gradient(T, th, D.conj().T @ r)
    g = np.zeros_like(g_ref)
    GA, GB = {}, {}
    for i in range(T.n):
        for j in range(T.n):
            A, B = _factor_pair(T, th, i, j)
            Di, rj = D[:, _cols(T, i)], r[:, _cols(T, j)]
            GA[i, j] = Di.conj().T @ (rj @ B.conj().T)        # W_ij B^H, without W
            GB[i, j] = (Di @ A).conj().T @ rj                  # A^H W_ij, without W
    for i in range(T.n):
        O.diag_block(T, g, i)[...] = GA[i, i] + GB[i, i].T
    for t, (i, j, _) in enumerate(T.pairs):
        O.L_block(T, g, t)[...] = GA[i, j] + GB[j, i].T      # through A_ij = L and B_ji = L^T
        O.R_block(T, g, t)[...] = GB[i, j] + GA[j, i].T      # through B_ij = R and A_ji = R^T
    assert np.linalg.norm(g - g_ref) <= 1e-12 * np.linalg.norm(g_ref)


def test_residual_in_tile_form():
    T, th, _, D, U = _problem(3, [16, 16, 16, 16], 5, [3, 6, 4, 8], 40)
    r_ref = O.residual(D, O.assemble(T, th), U)
    r = -U.copy()
    for j in range(T.n):
        for i in range(T.n):
            A, B = _factor_pair(T, th, i, j)
            r[:, _cols(T, j)] += (D[:, _cols(T, i)] @ A) @ B
    assert np.linalg.norm(r - r_ref) <= 1e-12 * np.linalg.norm(r_ref)


def test_carried_theta_half_is_exact_in_exact_arithmetic():
    """P_th(theta + s p) = P_th(theta) + s P_p(p): the factors enter A linearly."""
    T, th, p, D, _ = _problem(4, [16, 16, 16, 16], 5, [3, 6, 4, 8], 40)
    s = 0.37
    for i in range(T.n):
        for j in range(T.n):
            A_th, _ = _factor_pair(T, th, i, j)
            A_p, _ = _factor_pair(T, p, i, j)
            A_new, _ = _factor_pair(T, th + s * p, i, j)
            Di = D[:, _cols(T, i)]
            assert np.allclose(Di @ A_new, Di @ A_th + s * (Di @ A_p), rtol=1e-13, atol=1e-13)
