"""GPU tile low-rank product (tlrmdd_forward_tlr): r = D C(theta) - U computed as
(D A_ij) B_ij over factor pairs, without the dense X, vs the oracle's dense residual.

Error scale for this evaluation order: with per-tile factor pairs (A, B) the FP32 result
carries about (d + K) u |D| (|A||B|) + u |U| per element, and |A||B| summed over the tile
pairs is the assembly of the factor moduli, C(|theta|). The objective must match the
oracle to the matching relative bound, and the residual the dense GPU forward as well.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_cases import U32, from_geometry, from_workload, to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_14973_amd as m
    m._lib.load()
    return m


CASES = [
    ("small", lambda: from_workload(synth.small(), 3)),
    ("ragged_mixed", lambda: from_geometry(6, 5, "full", 17.0, synth.Layout([8, 8, 8, 6], [3, 2, 4, 1, 2, 5],
                                                                          [4, -1, 2, -1]), 1, "ragged_mixed",
                                           scale_theta=3.0)),
    ("multi_tile", lambda: from_geometry(20, 15, "half", 23.0, synth.uniform_layout(300, 64, 12, 20), 2,
                                         "multi_tile", scale_theta=2.0)),
    ("dense_diag", lambda: from_geometry(12, 11, "full", 9.0, synth.uniform_layout(132, 40, 6, -1), 3,
                                         "dense_diag", scale_theta=2.0)),
    ("high_rank", lambda: from_geometry(18, 16, "half", 27.0, synth.uniform_layout(288, 128, 70, 50), 4,
                                        "high_rank")),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_tlr_forward_parity(tl, name, mk):
    case = mk()
    plan, D, U, th, _ = to_device(case, tl, torch)
    f, r = tl.forward_tlr(plan, D, U, th, want_r=True)
    fd, rd, _ = tl.forward(plan, D, U, th, want_r=True)
    torch.cuda.synchronize()
    fo, ro = O.objective(case.T, case.D, case.U, case.theta)
    Xabs = O.assemble(case.T, np.abs(case.theta).astype(complex)).real
    K = max(case.T.d) + max(sum(k for (i, j, k) in case.T.pairs if i == a or j == a) + max(case.T.kdiag[a], case.T.d[a])
                            for a in range(case.T.n))
    bound = 4 * K * U32 * (np.abs(case.D) @ Xabs) + 4 * U32 * np.abs(case.U)
    rg = r.cpu().numpy().astype(np.complex128)
    err = np.abs(rg - ro)
    print(f"{name}: max err/bound {np.max(err / bound):.3f}, rel f {abs(f.item() - fo) / fo:.2e}, "
          f"rel f vs dense GPU {abs(f.item() - fd.item()) / fd.item():.2e}")
    assert np.all(err <= bound)
    assert abs(f.item() - fo) <= np.sum(np.abs(ro) * bound) + 1e-12 * fo
    assert np.allclose(rg, rd.cpu().numpy(), atol=2 * bound.max())
