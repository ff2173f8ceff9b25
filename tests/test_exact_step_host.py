"""The library's exact line-search step (csrc/exact_step.hpp, the same source the finalize kernel
runs on the device) compiled for the host and compared with the oracle's root selection
(ADMM solver, X-update; the step minimises the quartic phi(a) = f(theta + a p), whose derivative
phi'(a) = c0 + c1 a + c2 a^2 + c3 a^3 has the line-search sums as coefficients).

The library splits (0, inf) at the roots of phi'' into pieces where phi' is monotone and finds the
root on each by safeguarded Newton-bisection; the oracle takes the roots by numpy.roots; both keep
the positive real root with the lowest phi, ties to the smaller step. (An earlier closed-form
Cardano version returned 0 when c3 was tiny next to c2, where the roots of the depressed cubic
cancel catastrophically: the random solver-shaped cases below caught it.) Cases: random coefficients with the signs the solver produces (c0 < 0,
c1 > 0, c3 >= 0) over wide scales, two positive minima (distinct and tied), c3 = 0 with c2 != 0,
a purely linear phi', near-double and triple roots, no positive root, zero and non-finite input.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_14973_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include "exact_step.hpp"
int main() {
    double c[4];
    while (std::scanf("%la %la %la %la", &c[0], &c[1], &c[2], &c[3]) == 4)
        std::printf("%a\n", tlr::exact_step_dev(c));
    return 0;
}
"""


@pytest.fixture(scope="module")
def step_exe(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the HIP headers are missing")
    d = tmp_path_factory.mktemp("exact_step")
    src = d / "step.cpp"
    src.write_text(PROGRAM)
    exe = d / "step"
    subprocess.run(["g++", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC, str(src), "-o",
                    str(exe)], check=True)
    return str(exe)


def device_steps(exe, coeffs):
    inp = "\n".join(" ".join(float(v).hex() for v in c) for c in coeffs) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split()
    return [float.fromhex(v) for v in out]


def phi(c, a):
    return O.phi_increment(np.asarray(c, dtype=np.float64), a)


def same_choice(c, got, ref):
    """Either the same step, or (two minima at equal depth) the same phi value."""
    if got == ref == 0.0:
        return True
    if abs(got - ref) <= 1e-9 * max(1.0, abs(ref)):
        return True
    pg, pr = phi(c, got), phi(c, ref)
    return abs(pg - pr) <= 1e-12 * max(1.0, abs(pr))


def test_random_solver_shaped_coefficients(step_exe):
    rng = np.random.default_rng(14973)
    cs = []
    for _ in range(4000):
        s = 10.0 ** rng.uniform(-6, 6)
        c0 = -abs(rng.standard_normal()) * s
        c1 = abs(rng.standard_normal()) * s * 10.0 ** rng.uniform(-3, 3)
        c2 = rng.standard_normal() * s * 10.0 ** rng.uniform(-3, 3)
        c3 = abs(rng.standard_normal()) * s * 10.0 ** rng.uniform(-3, 3)
        cs.append((c0, c1, c2, c3))
    got = device_steps(step_exe, cs)
    for c, g in zip(cs, got):
        ref = O.exact_step(np.array(c))
        assert g > 0.0
        assert same_choice(c, g, ref), (c, g, ref)
        # a stationary point of phi
        d = ((c[3] * g + c[2]) * g + c[1]) * g + c[0]
        assert abs(d) <= 1e-9 * (abs(c[0]) + abs(c[1] * g) + abs(c[2] * g * g) + abs(c[3] * g ** 3))


def test_random_general_coefficients(step_exe):
    """Any signs: also cases with no positive root (step 0) and with three real roots."""
    rng = np.random.default_rng(7)
    cs = [tuple(rng.standard_normal(4) * 10.0 ** rng.uniform(-4, 4, 4)) for _ in range(4000)]
    got = device_steps(step_exe, cs)
    for c, g in zip(cs, got):
        assert same_choice(c, g, O.exact_step(np.array(c))), (c, g)


CASES = {
    # roots 1, 2, 4: minima at 1 and 4, phi(4) < phi(1)
    "two_minima_far_one_deeper": ((-8.0, 14.0, -7.0, 1.0), 4.0),
    # roots 1, 2, 3: minima at 1 and 3 with equal phi -> the smaller step
    "two_minima_tied": ((-6.0, 11.0, -6.0, 1.0), 1.0),
    # roots 1, 5, 6: minima at 1 and 6, phi(1) < phi(6)
    "two_minima_near_one_deeper": ((-30.0, 41.0, -12.0, 1.0), 1.0),
    # c3 = 0, c2 < 0: roots 1 (minimum) and 2 (maximum)
    "quadratic_concave": ((-2.0, 3.0, -1.0, 0.0), 1.0),
    # c3 = 0, c2 > 0: roots -1 and 1
    "quadratic_convex": ((-1.0, 0.0, 1.0, 0.0), 1.0),
    # c3 = c2 = 0: the exact quadratic line search a = -c0 / c1
    "linear": ((-3.0, 4.0, 0.0, 0.0), 0.75),
    # triple root at 1 (depressed cubic with P = 0)
    "triple_root": ((-1.0, 3.0, -3.0, 1.0), 1.0),
    # phi' = (a - 1)^2 (a + 1): double root at 1 is not a minimum, no positive minimum of phi;
    # the candidates are the stationary points with a > 0: only a = 1
    "double_root_inflection": ((1.0, -1.0, -1.0, 1.0), 1.0),
    # increasing phi: no positive stationary point
    "no_positive_root": ((1.0, 2.0, 1.0, 0.0), 0.0),
    "zero": ((0.0, 0.0, 0.0, 0.0), 0.0),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_special_cases(step_exe, name):
    c, expect = CASES[name]
    got = device_steps(step_exe, [c])[0]
    ref = O.exact_step(np.array(c))
    assert got == pytest.approx(expect, rel=1e-9, abs=1e-12), (name, got)
    # numpy.roots places a triple root only to about eps^(1/3) and Newton converges slowly there
    assert ref == pytest.approx(expect, rel=1e-4 if name == "triple_root" else 1e-6, abs=1e-9), (name, ref)


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_near_double_root(step_exe, eps):
    """phi' = (a + 1)(a - 1)(a - 1 - eps): a minimum at 1 + eps next to a maximum at 1 (and a minimum
    at -1 that is not a step); the cubic's discriminant is nearly zero. phi(1) - phi(1 + eps) is of
    order eps^3, below the resolution of phi once eps is small, so either point is a correct answer
    as long as its phi is the lower one to rounding; at eps = 1e-3 the minimum is resolved."""
    r = np.array([-1.0, 1.0, 1.0 + eps])
    p = np.poly(r)                      # a^3 + p1 a^2 + p2 a + p3
    c = (p[3], p[2], p[1], p[0])
    got = device_steps(step_exe, [c])[0]
    ref = O.exact_step(np.array(c))
    assert min(abs(got - 1.0), abs(got - 1.0 - eps)) <= 1e-7
    assert phi(c, got) <= phi(c, 1.0 + eps) + 1e-15
    if eps >= 1e-3:
        assert got == pytest.approx(1.0 + eps, rel=1e-9)
    assert same_choice(c, got, ref)


def test_non_finite_input_gives_zero(step_exe):
    cs = [(float("nan"), 1.0, 0.0, 1.0), (-1.0, float("inf"), 0.0, 1.0), (-1.0, 1.0, 0.0, float("-inf"))]
    assert device_steps(step_exe, cs) == [0.0, 0.0, 0.0]
