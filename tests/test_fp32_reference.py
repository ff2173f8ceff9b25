"""The FP32 reference solve (tests/fp32_reference.py) is the oracle's solve when nothing is rounded,
and rounding moves it by FP32 amounts on a well-conditioned trajectory."""
import numpy as np

import oracle as O
import synth
from fp32_reference import c64, solve
from gpu_cases import from_workload


def test_without_rounding_it_is_the_oracle_solve():
    case = from_workload(synth.small(), 2)
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=30)
    th, fh = solve(case.T, case.D, case.U, case.theta, 30, refresh=0, rnd=lambda a: np.asarray(a, np.complex128))
    assert np.linalg.norm(th - ref.theta) <= 1e-12 * np.linalg.norm(ref.theta)
    assert np.allclose(fh, ref.f_hist, rtol=1e-12, atol=0)


def test_fp32_rounding_moves_a_short_solve_by_fp32_amounts():
    case = from_workload(synth.small(), 2)
    ref = O.solve(case.T, case.D, case.U, case.theta, iters=30)
    th, fh = solve(case.T, case.D, case.U, case.theta, 30, rnd=c64)
    rel = np.linalg.norm(th - ref.theta) / np.linalg.norm(ref.theta)
    assert 1e-9 < rel < 1e-5
    assert np.max(np.abs(fh - ref.f_hist) / ref.f_hist) < 1e-5
