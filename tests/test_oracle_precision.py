"""Pins of oracle.predicted_objective_floor, the error scale the error table prints beside the
measured errors: the relative error of f = 1/2 ||D X - U||^2 when the product D X is rounded in a
format with unit roundoff u is expected at about 2 sqrt(nr) u || |D||X| ||_F / ||r||_F (a random
walk of nr rounding errors per entry of D X, Cauchy-Schwarz for the inner product <r, dr>).

Pinned against measured errors, not against the formula itself: f computed from products that
really are rounded - NumPy's complex64 products (FP32 with its BLAS's summation order), and the BF16
hi+lo split products emulated exactly (operands rounded to BF16 hi and lo parts, the three partial
products hi.hi + hi.lo + lo.hi summed in FP32) - must stay at or below the floor, at the nr 64
parity shape and at the nr 4096 / ns 2048 shape, for X near the data (small residual: the
demanding case) and far from it. The floor is an upper estimate, not a prediction: the measured
errors sit 10^3 to 10^4 below it (blocked BLAS sums grow slower than a random walk, and the rounding
error of r is not aligned with r, so Cauchy-Schwarz is far from tight); the pin shows that it bounds
what the products really do, which is the use the error table makes of it.
"""
import numpy as np
import pytest

import oracle as O
import synth

U32 = 2.0 ** -24
U_SPLIT = 2.0 ** -16


def bf16(x):
    """Round float32 values to BF16 (round to nearest even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16(x)
    lo = bf16(x - hi)
    return hi, lo


def split_matmul_real(A, B):
    ah, al = split(A)
    bh, bl = split(B)
    return (ah @ bh + ah @ bl + al @ bh).astype(np.float32)


def split_matmul(A, B):
    Ar, Ai = A.real.astype(np.float32), A.imag.astype(np.float32)
    Br, Bi = B.real.astype(np.float32), B.imag.astype(np.float32)
    re = split_matmul_real(Ar, Br) - split_matmul_real(Ai, Bi)
    im = split_matmul_real(Ar, Bi) + split_matmul_real(Ai, Br)
    return re.astype(np.float64) + 1j * im.astype(np.float64)


def cases(wl, f_idx):
    geom = wl.geometry()
    prob = wl.problem(f_idx, geom)
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    D = O.permute_columns(prob.D.astype(np.complex64).astype(np.complex128), perm)
    U = O.permute_columns(prob.U.astype(np.complex64).astype(np.complex128), perm)
    Xt = prob.X_true[np.ix_(perm, perm)].astype(np.complex64).astype(np.complex128)
    lay = wl.layout(f_idx)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    X0 = O.assemble(T, wl.theta0(f_idx, lay).astype(np.complex64).astype(np.complex128))
    return D, U, {"near (X_true)": Xt, "far (X of theta0)": X0.astype(np.complex64).astype(np.complex128)}


def rel_f_error(D, X, U, prod):
    r64 = D @ X - U
    f64 = 0.5 * np.vdot(r64, r64).real
    rl = prod(D, X) - U
    fl = 0.5 * np.vdot(rl, rl).real
    return abs(fl - f64) / f64, r64


@pytest.mark.parametrize("wl,f_idx", [(synth.small(), 3), (synth.large(), 10)], ids=["nr64", "nr4096"])
def test_complex64_products_stay_below_the_fp32_floor(wl, f_idx):
    D, U, Xs = cases(wl, f_idx)
    D32 = D.astype(np.complex64)
    for name, X in Xs.items():
        err, r = rel_f_error(D, X, U, lambda a, b: (D32 @ b.astype(np.complex64)).astype(np.complex128))
        floor = O.predicted_objective_floor(D, X, r, U32)
        print(f"{wl.name} {name}: measured {err:.2e}, floor {floor:.2e}")
        assert err <= floor


@pytest.mark.parametrize("wl,f_idx", [(synth.small(), 3), (synth.batched(), 20)], ids=["nr64", "nr1024"])
def test_bf16_split_products_stay_below_the_split_floor(wl, f_idx):
    D, U, Xs = cases(wl, f_idx)
    for name, X in Xs.items():
        err, r = rel_f_error(D, X, U, split_matmul)
        floor = O.predicted_objective_floor(D, X, r, U_SPLIT)
        print(f"{wl.name} {name}: measured {err:.2e}, floor {floor:.2e}")
        assert err <= floor
        # the emulation rounds as the split does: its error exceeds that of complex64 products
        err32, _ = rel_f_error(D, X, U, lambda a, b: (a.astype(np.complex64) @ b.astype(np.complex64))
                               .astype(np.complex128))
        assert err > err32


def test_split_emulation_is_the_hi_lo_definition():
    """The emulated split product equals the definition written element by element on a tiny case."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 5)).astype(np.float32)
    B = rng.standard_normal((5, 2)).astype(np.float32)
    got = split_matmul_real(A, B)
    for i in range(3):
        for j in range(2):
            acc = np.float32(0.0)
            for k in range(5):
                ah, al = split(A[i, k])
                bh, bl = split(B[k, j])
                for x, y in ((ah, bh), (ah, bl), (al, bh)):
                    acc = np.float32(acc + np.float32(x * y))
            assert abs(got[i, j] - acc) <= 4 * U32 * np.sum(np.abs(A[i]) * np.abs(B[:, j]))
    # hi + lo reproduces a float32 value to 2^-16 relative
    x = rng.standard_normal(1000).astype(np.float32)
    hi, lo = split(x)
    assert np.all(np.abs(hi.astype(np.float64) + lo - x) <= 2.0 ** -16 * np.abs(x))
