"""Pins for the oracle's exact line search and L-BFGS solve.

  * the step minimises the quartic phi(alpha) = f(theta + alpha p): phi' = 0
    there and no point of a dense grid is lower; phi(alpha*) equals a fresh
    objective evaluation (the assembly map is exactly quadratic);
  * brute force: on a tiny full-rank layout the tile parameterisation spans
    every symmetric X, so the solve must reach min over X = X^T of
    1/2||D X - U||^2, obtained by numpy.linalg.lstsq over the vech unknowns;
  * the regularised objective (Hyper-parameter selection, Frobenius term)
    with one dense tile against its closed-form least-squares solution;
  * the tracked objective never increases, and the tracked residual equals
    a fresh residual after many updates.
"""
import numpy as np
import pytest

import oracle as O
import synth


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_exact_step_minimises_quartic():
    rng = np.random.default_rng(10)
    T = O.tiling([4, 4, 2], [2, 2, 1], [2, -1, 1])
    D = _rand(rng, 12, T.nr)
    U = _rand(rng, 12, T.nr)
    for trial in range(5):
        th = 0.4 * _rand(rng, T.size)
        f0, g = O.gradient(T, D, U, th)
        p = -g * (0.1 + trial)
        r = O.residual(D, O.assemble(T, th), U)
        X1, X2 = O.assemble_directional(T, th, p)
        a, b = D @ X1, D @ X2
        c = O.line_coefficients(r, a, b)
        al = O.exact_step(c)
        assert al > 0
        dphi = ((c[3] * al + c[2]) * al + c[1]) * al + c[0]
        assert abs(dphi) <= 1e-9 * (abs(c[0]) + 1e-300)
        fa, _ = O.objective(T, D, U, th + al * p)
        assert abs(fa - (f0 + O.phi_increment(c, al))) <= 1e-11 * f0
        grid = np.linspace(0, 4 * al, 4001)
        vals = [O.objective(T, D, U, th + x * p)[0] for x in grid[::40]]
        assert fa <= min(vals) * (1 + 1e-12)


def test_exact_step_special_cases():
    # quadratic (b = 0): alpha = -c0/c1
    assert O.exact_step(np.array([-2.0, 4.0, 0.0, 0.0])) == pytest.approx(0.5, rel=1e-15)
    # ascent direction: no positive root
    assert O.exact_step(np.array([1.0, 1.0, 0.0, 1.0])) == 0.0
    # two minima: phi'(a) = (a-1)(a-2)(a-4) * 2 ; minima at 1 and 4, pick the lower phi
    c = 2 * np.array([-8.0, 14.0, -7.0, 1.0])
    a = O.exact_step(c)
    assert a in (pytest.approx(1.0), pytest.approx(4.0))
    assert O.phi_increment(c, a) == min(O.phi_increment(c, 1.0), O.phi_increment(c, 4.0))


def _vech_lstsq(D, U):
    """min over symmetric X of 1/2||D X - U||^2 by brute-force linear least squares."""
    n = D.shape[1]
    cols = []
    for a in range(n):
        for b in range(a, n):
            E = np.zeros((n, n), complex)
            E[a, b] = 1
            E[b, a] = 1
            cols.append((D @ E).ravel())
    A = np.stack(cols, axis=1)
    z, *_ = np.linalg.lstsq(A, U.ravel(), rcond=None)
    r = A @ z - U.ravel()
    return 0.5 * np.vdot(r, r).real


def test_solve_reaches_bruteforce_symmetric_minimum():
    rng = np.random.default_rng(11)
    D = _rand(rng, 12, 8)
    U = _rand(rng, 12, 8)
    T = O.tiling([4, 4], [4], [-1, -1])   # full-rank off-diagonal + dense diagonals
    th0 = 0.3 * _rand(rng, T.size)
    res = O.solve(T, D, U, th0, iters=400, m=8)
    fmin = _vech_lstsq(D, U)
    f_fresh, _ = O.objective(T, D, U, res.theta)
    assert f_fresh == pytest.approx(fmin, rel=1e-8)
    assert np.all(np.diff(res.f_hist) <= 1e-12 * res.f_hist[0])


def test_regularised_single_dense_tile_closed_form():
    rng = np.random.default_rng(12)
    n, ns, lam = 5, 9, 0.3
    D = _rand(rng, ns, n)
    U = _rand(rng, ns, n)
    T = O.tiling([n], [], [-1])
    # closed form: vec(D (Z+Z^T)/2) = A vec(Z); minimise 1/2||A z - u||^2 + lam ||z||^2
    cols = []
    for q in range(n * n):
        E = np.zeros(n * n, complex)
        E[q] = 1
        E = E.reshape(n, n)
        cols.append((D @ (0.5 * (E + E.T))).ravel())
    A = np.stack(cols, axis=1)
    Aa = np.vstack([A, np.sqrt(2 * lam) * np.eye(n * n)])
    ua = np.concatenate([U.ravel(), np.zeros(n * n)])
    z, *_ = np.linalg.lstsq(Aa, ua, rcond=None)
    fstar = 0.5 * np.linalg.norm(A @ z - U.ravel()) ** 2 + lam * np.vdot(z, z).real
    res = O.solve(T, D, U, np.zeros(T.size, complex), iters=200, m=10, lam=lam)
    assert res.f_hist[-1] == pytest.approx(fstar, rel=1e-9)
    assert np.allclose(res.theta, z, atol=1e-6 * np.abs(z).max())


@pytest.mark.parametrize("opt", ["lbfgs", "gd"])
def test_small_workload_monotone_and_tracked_residual(opt):
    wl = synth.small()
    geom = wl.geometry()
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    prob = wl.problem(3, geom)
    D = O.permute_columns(prob.D, perm)
    U = O.permute_columns(prob.U, perm)
    lay = wl.layout(3)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    res = O.solve(T, D, U, wl.theta0(3, lay), iters=50, optimizer=opt)
    assert np.all(np.diff(res.f_hist) <= 1e-12 * res.f_hist[0])
    assert res.f_hist[-1] < 0.5 * res.f_hist[0]
    f_fresh, _ = O.objective(T, D, U, res.theta)
    assert f_fresh == pytest.approx(res.f_hist[-1], rel=1e-9)


def test_lbfgs_beats_steepest_descent():
    wl = synth.small()
    geom = wl.geometry()
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    prob = wl.problem(5, geom)
    D = O.permute_columns(prob.D, perm)
    U = O.permute_columns(prob.U, perm)
    lay = wl.layout(5)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    a = O.solve(T, D, U, wl.theta0(5, lay), iters=50, optimizer="lbfgs")
    b = O.solve(T, D, U, wl.theta0(5, lay), iters=50, optimizer="gd")
    assert a.f_hist[-1] < b.f_hist[-1]


def test_lbfgs_two_loop_equals_dense_bfgs_inverse_update():
    """With m >= #pairs the two-loop product equals the explicit BFGS inverse
    update H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T from H0 = gamma I
    (real arithmetic on R^2n, Liu & Nocedal)."""
    rng = np.random.default_rng(13)
    n = 6
    S = [_rand(rng, n) for _ in range(3)]
    Y = [s + 0.3 * _rand(rng, n) for s in S]
    g = _rand(rng, n)
    p = O.lbfgs_direction(g, S, Y)

    def real(v):
        return np.concatenate([v.real, v.imag])
    Sr = [real(s) for s in S]
    Yr = [real(y) for y in Y]
    gamma = Sr[-1] @ Yr[-1] / (Yr[-1] @ Yr[-1])
    H = gamma * np.eye(2 * n)
    for s, y in zip(Sr, Yr):
        rho = 1.0 / (y @ s)
        V = np.eye(2 * n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    pr = -H @ real(g)
    assert np.allclose(real(p), pr, atol=1e-12 * np.abs(pr).max())
