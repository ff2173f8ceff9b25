"""GPU rank / tile-size estimate and warm start (tlrmdd_tile_ranks, tlrmdd_choose_layout,
tlrmdd_warm_start) vs the oracle.

Both sides see the same complex64-rounded X. Ranks are integers and must agree exactly
(tiles with a singular value within 1e-9 of the threshold would be ambiguous and are
excluded; none occurs in these cases); v0 agrees to FP64 rounding; the warm start is
compared through the assembled tiles (singular vectors are unique only up to phase)
at FP32 output rounding.
"""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_14973_amd as m
    m._lib.load()
    return m


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _c64(X):
    return np.ascontiguousarray(X, dtype=np.complex64)


def _low_rank_X(seed=41):
    rng = np.random.default_rng(seed)
    sizes, ro, rd = [16, 16, 16, 9], [2, 5, 1, 3, 4, 2], [3, -1, 6, 2]
    T = O.tiling(sizes, ro, rd)
    return T, _c64(O.assemble(T, _rand(rng, T.size)))


def _green(nx, freq, seed=0):
    geom = synth.make_geometry(nx, nx, "full")
    prob = synth.make_problem(geom, freq, 20.0, 0.05, 97, seed)
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    return _c64(prob.X_true[np.ix_(perm, perm)])


def _margin(X, d, eps):
    """Smallest relative distance of any tile singular value from the threshold."""
    sizes = O.split_sizes(X.shape[0], d)
    st = np.concatenate([[0], np.cumsum(sizes)])
    sv = [np.linalg.svd(X[st[i]:st[i + 1], st[j]:st[j + 1]], compute_uv=False)
          for i in range(len(sizes)) for j in range(i + 1)]
    v0 = max(s[0] for s in sv)
    return min(np.min(np.abs(s - eps * v0)) for s in sv) / v0


@pytest.mark.parametrize("d,eps", [(16, 1e-4), (12, 1e-4), (32, 1e-4)])
def test_tile_ranks_low_rank(tl, d, eps):
    T, X = _low_rank_X()
    Xd = torch.from_numpy(X).cuda()
    ko, kd, v0 = tl.tile_ranks(Xd, d, eps)
    _, ko_or, kd_or, v0o = O.tile_ranks(X.astype(np.complex128), d, eps)
    assert _margin(X.astype(np.complex128), d, eps) > 1e-9
    assert list(ko) == ko_or and list(kd) == kd_or
    assert v0 == pytest.approx(v0o, rel=1e-12)
    if d == 16:
        assert list(ko) == [2, 5, 1, 3, 4, 2] and list(kd) == [3, 16, 6, 2]


@pytest.mark.parametrize("nx,freq", [(12, 8.0), (16, 25.0)])
def test_choose_layout_green_function(tl, nx, freq):
    X = _green(nx, freq)
    Xd = torch.from_numpy(X).cuda()
    cand = [16, 32, 48, 64]
    d, sizes, ro, rd, ent = tl.choose_layout(Xd, cand, eps=0.01)
    do, so, roo, rdo, ento = O.choose_layout(X.astype(np.complex128), cand, eps=0.01)
    for c in cand:
        assert _margin(X.astype(np.complex128), c, 0.01) > 1e-9
    print(f"nx {nx} f {freq}: d {d} entries {list(ent)} (dense {X.shape[0] ** 2})")
    assert d == do and list(sizes) == so and list(ro) == roo and list(rd) == rdo
    assert list(ent) == ento


def test_warm_start_matches_oracle(tl):
    X = _green(12, 15.0, seed=3)
    Xd = torch.from_numpy(X).cuda()
    d, sizes, ro, rd, _ = tl.choose_layout(Xd, [24, 36], eps=0.01)
    T = O.tiling(sizes, ro, rd)
    plan = tl.Plan(sizes, ro, rd, 144)
    th = tl.warm_start(plan, Xd).cpu().numpy().astype(np.complex128)
    tho = O.warm_start(T, X.astype(np.complex128))
    Xg, Xo = O.assemble(T, th), O.assemble(T, tho)
    rel = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    print(f"warm start d {d}: rel assembled {rel:.2e}, rel to X {np.linalg.norm(Xo - X) / np.linalg.norm(X):.2e}")
    assert rel <= 1e-6


def test_warm_start_reproduces_low_rank(tl):
    T, X = _low_rank_X(42)
    plan = tl.Plan(T.d, [k for (_, _, k) in T.pairs], T.kdiag, 64)
    th = tl.warm_start(plan, torch.from_numpy(X).cuda()).cpu().numpy().astype(np.complex128)
    Xw = O.assemble(T, th)
    assert np.linalg.norm(Xw - X) / np.linalg.norm(X) <= 1e-6


def test_rank_invalid_arguments(tl):
    X = torch.zeros(8, 8, dtype=torch.complex64, device="cuda")
    for d, eps in [(0, 0.01), (2000, 0.01), (4, -1.0)]:
        with pytest.raises(tl.TLRMDDError) as e:
            tl.tile_ranks(X, d, eps)
        assert e.value.status == 1


# tile sizes the estimate workload runs (bench --workload estimate: 64, 128, 256 at nr = ns = 1024)
@pytest.mark.parametrize("d,freq", [(128, 12.0), (256, 12.0), (128, 30.0), (256, 30.0)])
def test_tile_ranks_large_tiles(tl, d, freq):
    X = _green(32, freq, seed=5)
    assert _margin(X.astype(np.complex128), d, 0.01) > 1e-9
    ko, kd, v0 = tl.tile_ranks(torch.from_numpy(X).cuda(), d, 0.01)
    _, ko_or, kd_or, v0o = O.tile_ranks(X.astype(np.complex128), d, 0.01)
    print(f"d {d} f {freq}: ranks {list(ko)[:8]}... diagonal {list(kd)}")
    assert list(ko) == ko_or and list(kd) == kd_or
    assert v0 == pytest.approx(v0o, rel=1e-12)


@pytest.mark.parametrize("freq", [6.0, 30.0])
def test_choose_layout_estimate_candidates(tl, freq):
    X = _green(32, freq, seed=6)
    cand = [64, 128, 256]
    for c in cand:
        assert _margin(X.astype(np.complex128), c, 0.01) > 1e-9
    d, sizes, ro, rd, ent = tl.choose_layout(torch.from_numpy(X).cuda(), cand, eps=0.01)
    do, so, roo, rdo, ento = O.choose_layout(X.astype(np.complex128), cand, eps=0.01)
    print(f"f {freq}: d {d} entries {list(ent)}")
    assert d == do and list(sizes) == so and list(ro) == roo and list(rd) == rdo and list(ent) == ento


@pytest.mark.parametrize("d", [128, 256])
def test_warm_start_large_tiles(tl, d):
    X = _green(32, 18.0, seed=7)
    _, ko, kd, _ = O.tile_ranks(X.astype(np.complex128), d, 0.01)
    sizes = O.split_sizes(X.shape[0], d)
    ko = [max(1, k) for k in ko]
    kd = [-1 if k >= (s + 1) // 2 else max(1, k) for k, s in zip(kd, sizes)]
    T = O.tiling(sizes, ko, kd)
    plan = tl.Plan(sizes, ko, kd, X.shape[0])
    th = tl.warm_start(plan, torch.from_numpy(X).cuda()).cpu().numpy().astype(np.complex128)
    tho = O.warm_start(T, X.astype(np.complex128))
    Xg, Xo = O.assemble(T, th), O.assemble(T, tho)
    rel = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    print(f"warm start d {d}: rel assembled {rel:.2e}")
    assert rel <= 1e-6
