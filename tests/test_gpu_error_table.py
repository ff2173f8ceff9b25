"""Mixed-precision error table at the nr 4096 shape (ns 2048, tile 256, rank 32, 100 iterations),
one frequency at 10 dB and one at 30 dB SNR, against the FP64 oracle (ADMM solver, gradient
equations DXLR and the X-update; precision policy: bulk products in FP32 or BF16 hi+lo split, FP64
for norms and step lengths).

The oracle's 100-iteration solves are stored (tests/golden/make_error_table_refs.py, which calls
only the oracle and the input generator): its f-history, f(theta_T), the predicted error floors, the
norms of theta_T and C(theta_T), and both at seeded random positions (1/16 of theta's entries, 2^18
of X's). Per precision the test solves on the GPU from the same complex64-rounded start and checks
  rel_f     = |f(theta_gpu) - f(theta_or)| / f(theta_or), f by the oracle's FP64 forward (exact);
  rel_X     = ||C(theta_gpu) - C(theta_or)|| / ||C(theta_or)||   (estimated from the stored entries);
  rel_theta = ||theta_gpu - theta_or|| / ||theta_or||             (estimated from the stored entries);
  the f-history entry by entry;
against 1e-5 (three-product FP32 with the tile-form line search and gradient: the bench's default
line) and 5e-3 (BF16 hi+lo split), printing the oracle's predicted floors beside them.
"""
import os

import numpy as np
import pytest

import oracle as O
import synth
from gpu_cases import c64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def tl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_14973_amd as m
    m._lib.load()
    return m


def sampled_rel(full_size, idx, got, ref_val, ref_norm):
    d = got.reshape(-1)[idx] - ref_val
    return float(np.sqrt(full_size / len(idx) * np.sum(np.abs(d) ** 2)) / ref_norm)


@pytest.mark.parametrize("snr", [10, 30])
def test_error_table_nr4096(tl, snr):
    ref = np.load(os.path.join(GOLDEN, f"error_table_nr4096_snr{snr}_f10.npz"))
    f_idx = int(ref["freq_index"])
    wl = synth.large(snr_db=float(snr), config_id=4)
    geom = wl.geometry()
    prob = wl.problem(f_idx, geom)
    lay = wl.layout(f_idx)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    Dn, Un, th0 = c64(prob.D), c64(prob.U), c64(wl.theta0(f_idx, lay))
    Do, Uo = O.permute_columns(Dn, perm), O.permute_columns(Un, perm)
    dev = torch.device("cuda")
    pd = torch.from_numpy(tl.hilbert_order(geom.rec_ix, geom.rec_iy)).to(dev)
    D = tl.permute_columns(torch.from_numpy(Dn.astype(np.complex64)).to(dev), pd)
    U = tl.permute_columns(torch.from_numpy(Un.astype(np.complex64)).to(dev), pd)
    th = torch.from_numpy(th0.astype(np.complex64)).to(dev)
    plan = tl.Plan.from_layout(lay, geom.ns)
    f_or, iters = float(ref["f_T"]), int(ref["iters"])
    print(f"\nSNR {snr} dB, {float(ref['freq_hz']):.2f} Hz: f_oracle {f_or:.6e}; predicted floors of rel_f: "
          f"FP32 {float(ref['floor_fp32']):.1e}, BF16 split {float(ref['floor_bf16_split']):.1e}", flush=True)
    for name, prec, tol, floor in (("fp32_3m tile forms", tl.FP32_3M, 1e-5, float(ref["floor_fp32"])),
                                   ("bf16x3", tl.BF16X3, 5e-3, float(ref["floor_bf16_split"]))):
        thT, fh = tl.solve(plan, D, U, th, iters, precision=prec, line_products=tl.LINE_TILE_GRAD)
        torch.cuda.synchronize()
        thg = thT.cpu().numpy().astype(np.complex128)
        f_g = O.objective(T, Do, Uo, thg)[0]
        rel_f = abs(f_g - f_or) / f_or
        rel_t = sampled_rel(thg.size, ref["theta_idx"], thg, ref["theta_val"], float(ref["theta_norm"]))
        Xg = O.assemble(T, thg)
        rel_x = sampled_rel(Xg.size, ref["X_idx"], Xg, ref["X_val"], float(ref["X_norm"]))
        rel_h = float(np.max(np.abs(fh.cpu().numpy() - ref["f_hist"]) / ref["f_hist"]))
        print(f"  {name}: rel_f {rel_f:.2e} (floor {floor:.1e}), rel_X {rel_x:.2e}, rel_theta {rel_t:.2e}, "
              f"rel f_hist {rel_h:.2e}, bar {tol:.0e}", flush=True)
        assert rel_f <= tol and rel_x <= tol and rel_t <= tol and rel_h <= tol
