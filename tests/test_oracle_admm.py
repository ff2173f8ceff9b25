"""Pins for the oracle's ADMM with lambda continuation (ADMM solver section,
eqs. for the X-, Z- and dual updates; hyper-parameter selection).

  * the X-update objective f + mu ||theta - c||^2 with one dense tile (a convex
    quadratic in Z) against its closed-form least-squares solution, and the
    line search along it against fresh evaluations of that objective;
  * the Z-update is the proximal point of lam ||.||^2: no random perturbation
    lowers lam ||z||^2 + rho/2 ||theta - z + u||^2, and scipy's minimiser over
    the real and imaginary parts lands on it;
  * ADMM's fixed point on the convex one-tile problem is the minimiser of
    f + lam ||theta||^2 (closed form), with z = theta and u = (2 lam / rho) z
    there; with continuation each stage ends at its own lam's minimiser.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
import synth


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _one_tile(seed, n=5, ns=9):
    rng = np.random.default_rng(seed)
    D = _rand(rng, ns, n)
    U = _rand(rng, ns, n)
    T = O.tiling([n], [], [-1])
    cols = []
    for q in range(n * n):   # vec(D (Z + Z^T)/2) = A vec(Z)
        E = np.zeros(n * n, complex)
        E[q] = 1
        E = E.reshape(n, n)
        cols.append((D @ (0.5 * (E + E.T))).ravel())
    return T, D, U, np.stack(cols, axis=1), rng


def _penalised_minimiser(A, U, mu, c):
    """argmin 1/2 ||A z - u||^2 + mu ||z - c||^2 by least squares on stacked rows."""
    n2 = A.shape[1]
    Aa = np.vstack([A, np.sqrt(2 * mu) * np.eye(n2)])
    ua = np.concatenate([U.ravel(), np.sqrt(2 * mu) * c])
    z, *_ = np.linalg.lstsq(Aa, ua, rcond=None)
    return z


def test_centered_penalty_closed_form_and_line_search():
    T, D, U, A, rng = _one_tile(21)
    mu = 0.7
    c = _rand(rng, T.size)
    zstar = _penalised_minimiser(A, U, mu, c)

    def fpen(th):
        r = A @ th - U.ravel()
        return 0.5 * np.vdot(r, r).real + mu * np.vdot(th - c, th - c).real

    checks = []

    def rec(t, st):
        th1 = st["theta"] + st["alpha"] * st["p"]
        checks.append((fpen(st["theta"]) + O.phi_increment(st["coeffs"], st["alpha"]), fpen(th1)))

    res = O.solve(T, D, U, np.zeros(T.size, complex), iters=200, m=10, lam=mu, center=c, record=rec)
    assert np.allclose(res.theta, zstar, atol=1e-7 * np.abs(zstar).max())
    assert res.f_hist[-1] == pytest.approx(fpen(zstar), rel=1e-10)
    for pred, fresh in checks[:20]:
        assert pred == pytest.approx(fresh, rel=1e-10, abs=1e-12)


def test_z_update_is_the_proximal_point():
    T, D, U, A, rng = _one_tile(22)
    lam, rho = 0.4, 1.7
    theta = _rand(rng, T.size)
    # with inner = 0 theta stays as given; the second outer step starts from a non-zero dual
    states = []
    O.admm(T, D, U, theta, lams=(lam,), outer=2, inner=0, rho=rho,
           record=lambda l, k, st: states.append(st))
    th1, u0 = states[1]["theta"], states[0]["u"]
    z = states[1]["z"]

    def h(zz):
        return lam * np.vdot(zz, zz).real + 0.5 * rho * np.vdot(th1 - zz + u0, th1 - zz + u0).real

    for _ in range(20):
        d = _rand(rng, T.size)
        assert h(z + 1e-3 * d) > h(z)
    n = T.size
    res = minimize(lambda x: h(x[:n] + 1j * x[n:]), np.zeros(2 * n), method="BFGS", options={"gtol": 1e-10})
    zs = res.x[:n] + 1j * res.x[n:]
    assert np.allclose(zs, z, atol=1e-6)
    assert not np.allclose(u0, 0)


def test_admm_fixed_point_is_regularised_minimiser():
    T, D, U, A, rng = _one_tile(23)
    lam, rho = 0.3, 1.0
    zstar = _penalised_minimiser(A, U, lam, np.zeros(T.size, complex))
    res = O.admm(T, D, U, np.zeros(T.size, complex), lams=(lam,), outer=80, inner=40, rho=rho, m=10)
    scale = np.abs(zstar).max()
    assert np.allclose(res.theta, zstar, atol=1e-6 * scale)
    assert np.allclose(res.z, res.theta, atol=1e-6 * scale)
    assert np.allclose(res.u, 2 * lam / rho * res.z, atol=1e-6 * scale)


def test_continuation_stages_end_at_their_minimisers():
    T, D, U, A, rng = _one_tile(24)
    lams = (10.0, 1.0, 0.1)
    ends = {}
    # with rho = 1 the lam = 10 stage contracts slowly (its prox shrinks by 1/21), hence 300 steps
    O.admm(T, D, U, 0.1 * _rand(rng, T.size), lams=lams, outer=300, inner=40, rho=1.0, m=10,
           record=lambda l, k, st: ends.__setitem__(l, st["theta"]))
    for lam in lams:
        zstar = _penalised_minimiser(A, U, lam, np.zeros(T.size, complex))
        assert np.allclose(ends[lam], zstar, atol=1e-8 * np.abs(zstar).max()), lam


def test_admm_on_tile_low_rank_model_lowers_misfit():
    wl = synth.small()
    geom = wl.geometry()
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    prob = wl.problem(2, geom)
    D = O.permute_columns(prob.D, perm)
    U = O.permute_columns(prob.U, perm)
    lay = wl.layout(2)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    res = O.admm(T, D, U, wl.theta0(2, lay), lams=(10.0, 1.0, 0.1), outer=3, inner=8)
    assert len(res.f_hist) == 1 + 9 and res.stage_end == [3, 6, 9]
    assert res.f_hist[-1] < 0.5 * res.f_hist[0]
    # weaker regularisation fits the data better at the end of each stage
    assert res.f_hist[9] < res.f_hist[6] < res.f_hist[3]
