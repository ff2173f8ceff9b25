"""Writes the oracle's reference solves of the nr 4096 mixed-precision error table.

Calls only the oracle and the seeded input generator: for every (SNR, frequency index) of the
nr 4096 / ns 2048 problem (tile 256, rank 32, 5 % noise on D, config 4 seeds), the complex64-rounded
inputs in Hilbert order are solved by oracle.solve (L-BFGS, m = 5, exact line search, complex128)
for 100 iterations from the complex64-rounded theta0, and the file keeps what the error table
compares with:
  * f_hist (the oracle's 101 objective values), f_T = oracle.objective of theta_T (a fresh forward);
  * the predicted objective floors for FP32 (u = 2^-24) and the BF16 hi+lo split (u = 2^-16),
    oracle.predicted_objective_floor of D, C(theta_T), r_T;
  * ||theta_T|| and ||C(theta_T)||_F;
  * --full: theta_T itself (rounded to complex64); otherwise (the committed test references) theta_T and X_T
    = C(theta_T) at seeded random positions (1/16 of theta's entries, 2^18 of X's; values rounded to
    complex64), from which the test estimates rel_theta and rel_X.

Usage: python tests/golden/make_error_table_refs.py --out DIR [--snrs 10,30] [--freqs 10] [--full]
The committed tests/golden/error_table_nr4096_snr{10,30}_f10.npz were written with the defaults.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

ITERS = 100
SAMPLE_SEED = 4096
THETA_SAMPLE_FRACTION = 16
X_SAMPLES = 1 << 18


def c64(a):
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def reference(snr, f_idx, full, log=print):
    wl = synth.large(snr_db=snr, config_id=4)
    geom = wl.geometry()
    prob = wl.problem(f_idx, geom)
    lay = wl.layout(f_idx)
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    D = O.permute_columns(c64(prob.D), perm)
    U = O.permute_columns(c64(prob.U), perm)
    th0 = c64(wl.theta0(f_idx, lay))
    t0 = time.perf_counter()

    def progress(t, state):
        if t % 10 == 0:
            log(f"snr {snr} f {f_idx}: oracle iteration {t}/{ITERS} ({time.perf_counter() - t0:.0f} s)")
    ref = O.solve(T, D, U, th0, iters=ITERS, record=progress)
    fT, r = O.objective(T, D, U, ref.theta)
    X = O.assemble(T, ref.theta)
    out = {
        "snr_db": snr, "freq_index": f_idx, "freq_hz": float(wl.freqs[f_idx]), "iters": ITERS,
        "f_hist": np.asarray(ref.f_hist), "f_T": fT,
        "floor_fp32": O.predicted_objective_floor(D, X, r, 2.0 ** -24),
        "floor_bf16_split": O.predicted_objective_floor(D, X, r, 2.0 ** -16),
        "theta_norm": np.linalg.norm(ref.theta), "X_norm": np.linalg.norm(X),
        "theta_size": ref.theta.size, "nr": X.shape[0], "oracle_s": time.perf_counter() - t0,
    }
    if full:
        out["theta"] = ref.theta.astype(np.complex64)   # rounded once (6e-8 relative)
    else:
        rng = np.random.default_rng(SAMPLE_SEED)
        ti = np.sort(rng.choice(ref.theta.size, ref.theta.size // THETA_SAMPLE_FRACTION, replace=False))
        xi = np.sort(rng.choice(X.size, X_SAMPLES, replace=False))
        # positions as int32, values rounded to complex64 (6e-8 relative, far below the 1e-5 bar)
        out.update(theta_idx=ti.astype(np.int32), theta_val=ref.theta[ti].astype(np.complex64),
                   X_idx=xi.astype(np.int32), X_val=X.reshape(-1)[xi].astype(np.complex64))
    return out


def path_for(out_dir, snr, f_idx):
    return os.path.join(out_dir, f"error_table_nr4096_snr{int(snr)}_f{f_idx}.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--snrs", default="10,30")
    ap.add_argument("--freqs", default="10")
    ap.add_argument("--full", action="store_true")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    for snr in [float(v) for v in args.snrs.split(",")]:
        for f_idx in [int(v) for v in args.freqs.split(",")]:
            ref = reference(snr, f_idx, args.full, log=lambda m: print(m, flush=True))
            np.savez_compressed(path_for(args.out, snr, f_idx), **ref)
            print(f"wrote {path_for(args.out, snr, f_idx)} (f_T {ref['f_T']:.6e}, {ref['oracle_s']:.0f} s)",
                  flush=True)


if __name__ == "__main__":
    main()
