#!/usr/bin/env python3
"""TLR-MDD benchmark on one MI355X.

Workload (default): the batched multi-frequency problem - 32 x 32 receiver
grid (nr = 1024, Hilbert ordered), ns = 1024 sources 40 m above, 64
frequencies from 2 to 40 Hz, rank k(f) = round(4 + 44 (f - 2)/38) with tile
256 / 128 / 64 for k <= 16 / <= 32 / larger, dense diagonal tiles when
k >= d/2, SNR 20 dB, 5 % noise on D, complex64, 100 L-BFGS iterations with
exact line search (residual recomputed every 20). One step = Hilbert column
gather of every D and U plus the full 100-iteration solve of all 64
frequencies (fused launches per phase). Complex products by default in the
three-real-product form on FP32 matrix cores (--precision fp32 for the
four-product form, bf16x3 for the BF16 hi+lo split). The line search runs
in tile form for the frequencies where that is cheaper (uniform tiles, Q Q^T
diagonals, padded rank kpad with 2.5 kpad <= 0.6 d), and so does the gradient
(its three products at most 0.6 of the adjoint product: tile 256 here);
--line-products tile keeps the dense gradient, dense the assembled X1, X2
everywhere. Every phase is one launch for all 64 frequencies except the
tile-form products: one dense launch for the frequencies that keep the dense
form, the tile-form stages per (tile size, padded rank) class.

value = grad iterations per second = 64 * 100 * steps / seconds (each grad
iteration: objective gradient, L-BFGS direction, exact line search, update).
The roofline object describes the dominant kernel (the product kind with
the most algorithmic flops: the line-search product [a | b] = D [X1 | X2]
of the frequencies whose line search stays dense),
timed with HIP events on its launch stream; achieved
counts the algorithmic 8mnk complex flops (the 3M form executes 6mnk:
executed_tflops / executed_frac).
cpu_baseline is the FP64 oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3e12, "bf16": 2.5e15}     # dense MFMA peaks of MI355X (FLOP/s)
HBM_PEAK = 8.0e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_inputs(wl, torch, tl, nfreq):
    import numpy as np
    geom = wl.geometry()
    dev = torch.device("cuda")
    Ds, Us, ths, plans = [], [], [], []
    t0 = time.time()
    for i in range(nfreq):
        prob = wl.problem(i, geom)
        lay = wl.layout(i)
        Ds.append(torch.from_numpy(prob.D.astype(np.complex64)).to(dev))
        Us.append(torch.from_numpy(prob.U.astype(np.complex64)).to(dev))
        ths.append(torch.from_numpy(wl.theta0(i, lay).astype(np.complex64)).to(dev))
        plans.append(tl.Plan.from_layout(lay, geom.ns))
        if (i + 1) % 16 == 0:
            log(f"inputs {i + 1}/{nfreq} ({time.time() - t0:.1f}s)")
    return geom, Ds, Us, ths, plans


def source_sha(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2412_14973_amd", "csrc", f), "rb").read())
    return h.hexdigest()


ADJOINT_KERNEL = {"fp32": "cgemm_f32_kernel<GM_STORE>", "fp32_3m": "cgemm3m_kernel<GM_STORE, 0>",
                  "bf16x3": "cgemm_bf16x3_kernel<GM_STORE>"}
LINE_KERNEL = {"fp32": "cgemm_f32_kernel<GM_LINE>", "fp32_3m": "cgemm3m_kernel<GM_LINE, 0>",
               "bf16x3": "cgemm_bf16x3_kernel<GM_LINE>"}
FORM_FLOPS = {"fp32": "four-product FP32, 8 m n k", "fp32_3m": "three-product FP32, 6 m n k",
              "bf16x3": "BF16 hi+lo split, 24 m n k in BF16"}


def precision_info(tl, name):
    """(library constant, dtype label, config label)."""
    return {
        "fp32": (tl.FP32, "f32", "fp32-mfma"),
        "fp32_3m": (tl.FP32_3M, "f32", "fp32-3m-mfma"),
        "bf16x3": (tl.BF16X3, "bf16x3", "bf16x3-mfma"),
    }[name]


TRAFFIC_RECORDS = {   # (precision, line-search form, product kind) -> (counter summary, kernel sources)
    ("fp32", "dense", "gemm_line"): ("cgemm_line_traffic.json", ("cgemm.hip", "gemm_common.hpp")),
    ("fp32_3m", "dense", "gemm_line"): ("cgemm3m_line_traffic.json", ("cgemm3m.hip", "gemm_common.hpp")),
    ("fp32_3m", "tile_grad", "gemm_line"): ("cgemm3m_line_traffic_tile.json", ("cgemm3m.hip", "gemm_common.hpp")),
    ("fp32_3m", "tile_grad", "gemm_adjoint"): ("cgemm3m_adjoint_traffic_tile.json",
                                               ("cgemm3m.hip", "gemm_common.hpp")),
    ("bf16x3", "dense", "gemm_line"): ("cgemm_bf16_line_traffic.json", ("cgemm_bf16.hip", "gemm_common.hpp")),
}


def measured_traffic(nfreq, workload, precision, mode, kind):
    """HBM bytes per launch (average over the launches of that product kind) from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (copy-calibrated), or None when the kernel source changed
    since the counters were taken or the configuration differs."""
    key = (precision, mode, kind)
    if key not in TRAFFIC_RECORDS:
        return None
    name, files = TRAFFIC_RECORDS[key]
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        sha = source_sha(files)
    except OSError:
        return None
    if rec.get("source_sha256") != sha or workload != rec.get("workload") or nfreq != rec.get("frequencies"):
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(wl, budget_s):
    """Time the FP64 oracle (as it stands) on a bounded sample of the workload: frequencies from the
    low, middle and high part of the band (their layouts differ: tile 256 / 128 / 64), each for up to
    the workload's iteration count, within about budget_s seconds in total."""
    import numpy as np

    import oracle as O
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = sum(int(i.get("num_threads", 0)) for i in threadpool_info()
                      if i.get("user_api") == "blas") or None
    except Exception:
        threads = None
    nf = len(wl.freqs)
    geom = wl.geometry()
    perm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
    its, secs, used = 0, 0.0, []
    picks = (nf // 6, nf // 2, (5 * nf) // 6)
    for f_idx in picks:
        left = budget_s / len(picks)   # an equal share of the budget per frequency
        prob = wl.problem(f_idx, geom)
        lay = wl.layout(f_idx)
        T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
        D = O.permute_columns(prob.D, perm)
        U = O.permute_columns(prob.U, perm)
        th = wl.theta0(f_idx, lay)
        t0 = time.perf_counter()
        O.solve(T, D, U, th, iters=2)
        per = (time.perf_counter() - t0) / 2
        n = int(max(2, min(wl.iters, left / max(per, 1e-6))))
        t0 = time.perf_counter()
        O.solve(T, D, U, th, iters=n)
        secs += time.perf_counter() - t0
        its += n
        used.append(f"index {f_idx} ({wl.freqs[f_idx]:.2f} Hz, tile {int(np.max(lay.tile_size))}) x {n} iterations")
    return {"value": its / secs, "unit": "grad-iters/s", "cores": threads or os.cpu_count(), "kind": "oracle",
            "sample": f"{len(used)} of {nf} frequencies: " + "; ".join(used) +
                      f"; L-BFGS, complex128 NumPy, {secs:.1f} s"}


def serving(tl, torch, args):
    """Poisson stream of per-frequency solves of uneven size: continuous batching
    (FIFO admission by HBM budget, up to --max-active overlapping solves) against
    the same stream solved one at a time. Inputs are generated on the device before
    the clock starts; each request's work (Hilbert column gather + 100-iteration
    solve) runs on its own stream. Results of the two runs must agree bit for bit."""
    import synth
    from paper_2412_14973_amd import serve
    prec = precision_info(tl, args.precision)[0]
    line = {"dense": tl.LINE_DENSE, "tile": tl.LINE_TILE, "tile-grad": tl.LINE_TILE_GRAD}[args.line_products]
    reqs = synth.request_stream(args.requests, iters=args.iters or 100)
    dev = torch.device("cuda")
    prepared = []
    t0 = time.time()
    for r in reqs:
        D, U, th, lay, geom = synth.device_problem(r, dev)
        perm = torch.from_numpy(tl.hilbert_order(geom.rec_ix, geom.rec_iy)).to(dev)
        plan = tl.Plan.from_layout(lay, geom.ns)
        prepared.append((r, D, U, th, perm, plan))
        form = tl.line_form(plan, prec, line)[0]
        log(f"request {r.rid}: nr {geom.nr} ns {geom.ns} d {r.d} k {r.k} form {form} ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()

    class Backend(serve.GpuBackend):
        def start(self, req):
            r, D, U, th, perm, plan = req
            sidx = self.free_streams.pop(0)
            stream = self.streams[sidx]
            stream.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(stream):
                Dh = tl.permute_columns(D, perm)
                Uh = tl.permute_columns(U, perm)
                theta, fh = tl.solve(plan, Dh, Uh, th, r.iters, precision=prec, line_products=line)
                ev = torch.cuda.Event()
                ev.record(stream)
            return {"event": ev, "stream": sidx, "theta": theta, "fhist": fh, "keep": (Dh, Uh)}

        def footprint(self, req):
            r, D, U, th, perm, plan = req
            return super().footprint(serve.SolveRequest(plan, D, U, th, r.iters, prec, line_products=line)) + \
                2 * D.numel() * 8

    out = {"metric": "TLR-MDD served solves/s, p50/p99 latency", "requests": len(reqs),
           "arrival_rate_per_s": 200.0, "iters": reqs[0].iters, "precision": args.precision,
           "line_products": args.line_products,
           "forms": [tl.line_form(p[5], prec, line)[0] for p in prepared],
           "hbm_budget_gib": args.hbm_budget_gib, "sizes": [[r.n_side ** 2, (r.n_side ** 2) // (2 if r.ns_mode == "half" else 1), r.d, r.k] for r in reqs]}
    results = {}
    for mode, active in (("one_at_a_time", 1), ("continuous", args.max_active)):
        be = Backend(n_streams=max(active, 1))
        jobs = [serve.Job(rid=p[0].rid, arrival=p[0].arrival, payload=p) for p in prepared]
        torch.cuda.synchronize()
        be.clock = serve.WallClock()
        srv = serve.Server(be, hbm_budget=int(args.hbm_budget_gib * 2 ** 30), max_active=active)
        srv.run(jobs)
        torch.cuda.synchronize()
        out[mode] = serve.summarize(jobs)
        out[mode]["max_active"] = active
        out[mode]["peak_hbm_gib"] = srv.peak_in_use / 2 ** 30
        results[mode] = {j.rid: j.result for j in jobs}
        log(f"{mode}: {out[mode]}")
    same = all(torch.equal(results["one_at_a_time"][k]["theta"], results["continuous"][k]["theta"])
               and torch.equal(results["one_at_a_time"][k]["fhist"], results["continuous"][k]["fhist"])
               for k in results["continuous"])
    out["bitwise_same_alone_and_in_mix"] = bool(same)
    out["speedup_solves_per_s"] = out["continuous"]["solves_per_s"] / out["one_at_a_time"]["solves_per_s"]
    return out


def tlr_product(tl, torch, args):
    """Dense forward (assemble X, r = D X - U on MFMA) vs the tile low-rank product (no dense X)
    on the 64 x 64-receiver problem (nr 4096, ns 2048, tile 256, rank 32): time per call, flops."""
    import numpy as np

    import synth
    wl = synth.large()
    nfreq = args.nfreq or 4
    geom, Ds, Us, ths, plans = build_inputs(wl, torch, tl, nfreq)
    dev = torch.device("cuda")
    perm = torch.from_numpy(tl.hilbert_order(geom.rec_ix, geom.rec_iy)).to(dev)
    ns, nr = geom.ns, geom.nr
    recs = []
    for i in range(nfreq):
        D = tl.permute_columns(Ds[i], perm)
        U = tl.permute_columns(Us[i], perm)
        plan, th = plans[i], ths[i]
        ws_d = plan.workspace(tl._lib.OP_FORWARD)
        ws_t = torch.empty(tl.tlr_workspace_bytes(plan), dtype=torch.uint8, device=dev)
        lay = wl.layout(i)
        d = np.asarray(lay.tile_size)
        k_pairs = sum(int(k) * (int(d[a]) + int(d[b])) for (a, b, k) in
                      [(a, b, lay.rank_off[a * (a - 1) // 2 + b]) for a in range(len(d)) for b in range(a)])
        k_diag = sum(int(d[a]) * (int(d[a]) if lay.rank_diag[a] < 0 else int(lay.rank_diag[a])) for a in range(len(d)))
        flops_tlr = 2 * 8.0 * ns * (k_pairs + k_diag)
        flops_dense = 8.0 * ns * nr * nr
        out = {}
        for name, fn in (("dense", lambda: tl.forward(plan, D, U, th, workspace=ws_d)[0]),
                         ("tlr", lambda: tl.forward_tlr(plan, D, U, th, workspace=ws_t)[0])):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(args.steps + 2):
                t0 = time.perf_counter()
                fv = fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            out[name] = {"ms": 1e3 * float(np.median(ts)), "f": float(fv.item())}
        out["dense"]["gemm_tflops_equiv"] = flops_dense / out["dense"]["ms"] / 1e9
        out["tlr"]["tflops"] = flops_tlr / out["tlr"]["ms"] / 1e9
        rec = {"freq_index": i, "flops_dense": flops_dense, "flops_tlr": flops_tlr,
               "flop_ratio": flops_tlr / flops_dense, **out,
               "speedup": out["dense"]["ms"] / out["tlr"]["ms"],
               "rel_f_diff": abs(out["tlr"]["f"] - out["dense"]["f"]) / out["dense"]["f"]}
        recs.append(rec)
        log(f"freq {i}: dense {out['dense']['ms']:.2f} ms, tlr {out['tlr']['ms']:.2f} ms "
            f"(flop ratio {rec['flop_ratio']:.3f}, speedup {rec['speedup']:.2f}, rel f diff {rec['rel_f_diff']:.1e})")
    return {"metric": "forward f = 1/2||D C(theta) - U||^2, dense vs tile low-rank product", "unit": "ms",
            "value": float(np.mean([r["tlr"]["ms"] for r in recs])), "higher_is_better": False, "n_gpus": 1,
            "data": "synthetic", "config": {"workload": wl.name, "nr": nr, "ns": ns, "frequencies": nfreq},
            "records": recs}


def estimate(tl, torch, args):
    """Rank / tile-size estimate and warm start on the 32 x 32-receiver problem (nr = ns = 1024).

    Per sampled frequency: reference solution X from the benchmark (Tikhonov, one dense tile) solve
    and from the synthetic truth; GPU per-tile FP64 SVD over tile sizes 64, 128, 256 (eps = 0.01)
    -> layout with the fewest entries; warm start of that layout; 100-iteration solves from the warm
    start and from the random start, compared by objective and by distance to the truth."""
    import numpy as np

    import synth
    wl = synth.batched()
    geom = wl.geometry()
    dev = torch.device("cuda")
    perm_np = tl.hilbert_order(geom.rec_ix, geom.rec_iy)
    perm = torch.from_numpy(perm_np).to(dev)
    nf = len(wl.freqs)
    idx = sorted(set(np.linspace(0, nf - 1, args.estimate_freqs).round().astype(int).tolist()))
    cand = [64, 128, 256]
    iters = args.iters or 100
    recs = []
    for i in idx:
        prob = wl.problem(i, geom)
        D = tl.permute_columns(torch.from_numpy(prob.D.astype(np.complex64)).to(dev), perm)
        U = tl.permute_columns(torch.from_numpy(prob.U.astype(np.complex64)).to(dev), perm)
        Xt = np.ascontiguousarray(prob.X_true[np.ix_(perm_np, perm_np)], dtype=np.complex64)
        Xt_d = torch.from_numpy(Xt).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xb, _ = tl.benchmark_solve(D, U, lam=args.bench_lambda, iters=iters)
        torch.cuda.synchronize()
        t_bench = time.perf_counter() - t0
        rec = {"freq_index": i, "freq_hz": float(wl.freqs[i]), "benchmark_solve_s": t_bench,
               "benchmark_rel_err_to_truth": float(torch.linalg.norm(Xb - Xt_d) / torch.linalg.norm(Xt_d))}
        for src, Xr in (("benchmark", Xb), ("truth", Xt_d)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            d, sizes, ro, rd, ent = tl.choose_layout(Xr, cand, eps=0.01)
            t_est = time.perf_counter() - t0
            plan = tl.Plan(sizes, ro, rd, geom.ns)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            th_w = tl.warm_start(plan, Xr)
            torch.cuda.synchronize()
            t_warm = time.perf_counter() - t0
            th_r = torch.from_numpy(synth.init_theta(plan.theta_size, wl.config_id, i).astype(np.complex64)).to(dev)
            out = {"d": d, "entries": [int(e) for e in ent], "dense_entries": int(geom.nr) ** 2,
                   "mean_rank_off": float(np.mean(ro)) if len(ro) else 0.0,
                   "dense_diagonal_tiles": int(np.sum(rd < 0)), "estimate_s": t_est, "warm_start_s": t_warm}
            for start, th0 in (("warm", th_w), ("random", th_r)):
                th, fh = tl.solve(plan, D, U, th0, iters)
                _, _, Xs = tl.forward(plan, D, U, th, want_X=True)
                out[start] = {"f0": float(fh[0].item()), "fT": float(fh[-1].item()),
                              "rel_err_to_truth": float(torch.linalg.norm(Xs - Xt_d) / torch.linalg.norm(Xt_d))}
            rec[src] = out
        recs.append(rec)
        log(f"freq {i} ({rec['freq_hz']:.1f} Hz): benchmark d {rec['benchmark']['d']} "
            f"est {rec['benchmark']['estimate_s'] * 1e3:.1f} ms warm {rec['benchmark']['warm_start_s'] * 1e3:.1f} ms; "
            f"fT warm {rec['benchmark']['warm']['fT']:.4g} vs random {rec['benchmark']['random']['fT']:.4g}")
    est = [r[s]["estimate_s"] for r in recs for s in ("benchmark", "truth")]
    return {"metric": "rank estimate (3 tile sizes) ms per frequency", "value": 1e3 * float(np.mean(est)),
            "unit": "ms", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "nr1024_ns1024_64freq_adaptive (sampled frequencies)", "candidates": cand,
                       "eps": 0.01, "iters": iters, "benchmark_lambda": args.bench_lambda},
            "records": recs}


def error_table(tl, torch, args):
    """Mixed-precision error table on the 64 x 64-receiver problem (nr 4096, ns 2048,
    tile 256, rank 32) at 10 and 30 dB: FP32 and BF16x3 solves (and the three-product FP32 solve
    with the tile-form line search and gradient) against the FP64 oracle."""
    import numpy as np

    import oracle as O
    import synth
    iters = args.iters or 100
    rows = []
    R = args.resid_refresh
    dense = tl.LINE_DENSE
    variants = [("fp32", tl.FP32, 0, dense), ("bf16x3", tl.BF16X3, 0, dense)]
    if R > 0:
        variants += [(f"fp32_refresh{R}", tl.FP32, R, dense), (f"bf16x3_refresh{R}", tl.BF16X3, R, dense),
                     (f"fp32_3m_refresh{R}", tl.FP32_3M, R, dense),
                     (f"fp32_3m_tile_forms_refresh{R}", tl.FP32_3M, R, tl.LINE_TILE_GRAD)]
    for snr in [float(v) for v in args.error_snrs.split(",")]:
        wl = synth.large(snr_db=snr, config_id=4)
        f_idx = 10
        geom = wl.geometry()
        prob = wl.problem(f_idx, geom)
        lay = wl.layout(f_idx)
        T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
        D64 = prob.D.astype(np.complex64)
        U64 = prob.U.astype(np.complex64)
        th64 = wl.theta0(f_idx, lay).astype(np.complex64)
        perm = tl.hilbert_order(geom.rec_ix, geom.rec_iy)
        dev = torch.device("cuda")
        pd = torch.from_numpy(perm).to(dev)
        D = tl.permute_columns(torch.from_numpy(D64).to(dev), pd)
        U = tl.permute_columns(torch.from_numpy(U64).to(dev), pd)
        th = torch.from_numpy(th64).to(dev)
        plan = tl.Plan.from_layout(lay, geom.ns)
        res = {}
        for name, prec, refresh, line in variants:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            thT, fh = tl.solve(plan, D, U, th, iters, precision=prec, resid_refresh=refresh, line_products=line)
            torch.cuda.synchronize()
            res[name] = (thT.cpu().numpy().astype(np.complex128), time.perf_counter() - t0)
            log(f"snr {snr}: {name} solve {res[name][1]:.2f} s")
        Do = D64.astype(np.complex128)[:, perm]
        Uo = U64.astype(np.complex128)[:, perm]
        t0 = time.perf_counter()

        def progress(t, state):
            if t % 10 == 0:
                log(f"snr {snr}: oracle iteration {t}/{iters} ({time.perf_counter() - t0:.0f} s)")
        ref = O.solve(T, Do, Uo, th64.astype(np.complex128), iters=iters, record=progress)
        t_or = time.perf_counter() - t0
        log(f"snr {snr}: oracle {t_or:.1f} s")
        fo = O.objective(T, Do, Uo, ref.theta)[0]
        Xo = O.assemble(T, ref.theta)
        for name, (thg, tg) in res.items():
            fg = O.objective(T, Do, Uo, thg)[0]
            rows.append({"snr_db": snr, "freq_hz": float(wl.freqs[f_idx]), "precision": name, "iters": iters,
                         "rel_f": abs(fg - fo) / fo,
                         "rel_X": float(np.linalg.norm(O.assemble(T, thg) - Xo) / np.linalg.norm(Xo)),
                         "rel_theta": float(np.linalg.norm(thg - ref.theta) / np.linalg.norm(ref.theta)),
                         "f_oracle": fo, "f_gpu": fg, "gpu_s": tg, "oracle_s": t_or})
    return {"error_table": rows, "workload": "nr4096_ns2048_d256_k32 (frequency index 10 of 32, 5-35 Hz)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["batched", "large", "serving", "estimate", "tlr"], default="batched")
    ap.add_argument("--estimate-freqs", type=int, default=6, help="estimate: frequencies sampled over the band")
    ap.add_argument("--bench-lambda", type=float, default=3.0, help="estimate: Tikhonov lambda of the benchmark solve")
    ap.add_argument("--requests", type=int, default=16, help="serving: requests in the Poisson stream")
    ap.add_argument("--max-active", type=int, default=4, help="serving: concurrent solves")
    ap.add_argument("--hbm-budget-gib", type=float, default=96.0, help="serving: admission budget")
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--nfreq", type=int, default=None)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp32", "bf16x3", "fp32_3m"], default="fp32_3m",
                    help="complex64 products: fp32_3m (three real FP32 products, default), fp32 (four), "
                         "bf16x3 (BF16 hi+lo split)")
    ap.add_argument("--solver", choices=["lbfgs", "admm"], default="lbfgs",
                    help="admm: lambda stages 10, 1, 0.1 x --admm-outer X-updates of --admm-inner L-BFGS iterations")
    ap.add_argument("--admm-outer", type=int, default=4)
    ap.add_argument("--admm-inner", type=int, default=8)
    ap.add_argument("--error-table", action="store_true",
                    help="per-frequency error of FP32 and BF16x3 solves against the FP64 oracle (large workload)")
    ap.add_argument("--error-snrs", default="10,30", help="error table: SNRs in dB")
    ap.add_argument("--line-products", choices=["dense", "tile", "tile-grad"], default="tile-grad",
                    help="line search products from the assembled X1, X2, or in tile form where cheaper "
                         "(tile-grad: the gradient's products too)")
    ap.add_argument("--streams", type=int, default=1,
                    help="batched solve: sub-batches on their own streams (problem i in sub-batch i %% streams)")
    ap.add_argument("--resid-refresh", type=int, default=20,
                    help="error table: also an FP32 solve that recomputes r = D C(theta) - U every this many iterations")
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help="batched workload: skip the nr 64 latency and nr 4096 throughput objects")
    ap.add_argument("--large-steps", type=int, default=2, help="timed steps of the nr 4096 object")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: frequencies are independent solves; "
              "multi-GPU sharding is not part of this build (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2412_14973_amd as tl
    import synth
    tl._lib.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    if args.error_table:
        print(json.dumps(error_table(tl, torch, args)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(serving(tl, torch, args)), flush=True)
        return
    if args.workload == "estimate":
        print(json.dumps(estimate(tl, torch, args)), flush=True)
        return
    if args.workload == "tlr":
        print(json.dumps(tlr_product(tl, torch, args)), flush=True)
        return
    prec, dtype, prec_name = precision_info(tl, args.precision)[:3]
    line_products = {"dense": tl.LINE_DENSE, "tile": tl.LINE_TILE, "tile-grad": tl.LINE_TILE_GRAD}[args.line_products]
    admm = args.solver == "admm"
    if args.workload == "batched":
        wl = synth.batched()
        nfreq = args.nfreq or len(wl.freqs)
        inputs = build_inputs(wl, torch, tl, nfreq)
    else:
        wl = synth.large()
        nfreq = args.nfreq or len(wl.freqs)
        inputs = device_inputs(wl, torch, tl, nfreq)
    run = measure_workload(tl, torch, args, wl, inputs, args.steps, args.warmup, prec, line_products, admm)
    line = {
        "metric": "TLR-MDD grad iters/s",
        "value": run["value"],
        "unit": "grad-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": dict(run["config"], precision=prec_name),
        "roofline": run["roofline"],
        "hbm_passes": run["hbm_passes"],
        "mfma_frac_all_gemms": run["mfma_frac_all_gemms"],
        "kernels": run["kernels"],
        "objective": run["objective"],
    }
    if args.workload == "batched" and not admm and args.nfreq is None and args.extra:
        log("nr 64 parity workload: microseconds per iteration")
        line["small_workload"] = small_latency(tl, torch, prec, args)
        log("nr 4096 workload (32 frequencies, inputs generated on the device)")
        wl3 = synth.large()
        inputs3 = device_inputs(wl3, torch, tl, len(wl3.freqs))
        run3 = measure_workload(tl, torch, args, wl3, inputs3, args.large_steps, 1, prec, line_products, False)
        del inputs3
        line["large_workload"] = {k: run3[k] for k in ("value", "unit", "ms_per_step", "steps", "config", "roofline",
                                                      "hbm_passes", "mfma_frac_all_gemms", "kernels", "objective")}
    if not args.no_cpu_baseline and prec != tl.BF16X3 and args.workload == "batched":
        log("timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(line), flush=True)


def device_inputs(wl, torch, tl, nfreq):
    """Inputs of a workload generated on the device (same recipe, torch's device generator)."""
    import synth
    geom = wl.geometry()
    dev = torch.device("cuda")
    Ds, Us, ths, plans = [], [], [], []
    t0 = time.time()
    for i in range(nfreq):
        D, U, th = synth.device_workload_problem(wl, i, dev)
        Ds.append(D)
        Us.append(U)
        ths.append(th)
        plans.append(tl.Plan.from_layout(wl.layout(i), geom.ns))
        if (i + 1) % 8 == 0:
            torch.cuda.synchronize()
            log(f"device inputs {i + 1}/{nfreq} ({time.time() - t0:.1f}s)")
    return geom, Ds, Us, ths, plans


def small_latency(tl, torch, prec, args):
    """The nr 64 parity workload (8 frequencies, 50 iterations) as one batched solve: wall time per
    iteration (launch-latency bound: about 20 launches per iteration)."""
    import synth
    wl = synth.small()
    geom, Ds, Us, ths, plans = build_inputs(wl, torch, tl, len(wl.freqs))
    dev = torch.device("cuda")
    perm = torch.from_numpy(tl.hilbert_order(geom.rec_ix, geom.rec_iy)).to(dev)
    Dh = [tl.permute_columns(D, perm) for D in Ds]
    Uh = [tl.permute_columns(U, perm) for U in Us]
    out = {}
    for label, fn in (
            ("batched_8freq", lambda: tl.solve_batched(plans, Dh, Uh, ths, wl.iters, precision=prec)),
            ("single_freq", lambda: tl.solve(plans[0], Dh[0], Uh[0], ths[0], wl.iters, precision=prec))):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(10):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        med = ts[len(ts) // 2]
        out[label] = {"us_per_iteration": med / wl.iters * 1e6, "ms_per_solve": med * 1e3}
    out["config"] = {"workload": wl.name, "iters": wl.iters, "frequencies": len(wl.freqs)}
    return out


def kernel_table(kt):
    """Per kernel kind: launches, average duration, and (from the library's per-launch work counts) the
    rate of the product form's real flops against its instruction type's peak, the complex-equivalent
    rate (8 m n k), and the algorithmic HBM bytes per second against 8 TB/s."""
    out = {}
    for k, ms in kt.ms.items():
        n = kt.launches[k]
        if n == 0 or ms <= 0:
            continue
        e = {"launches": n, "avg_ms": ms / n}
        sec = ms * 1e-3
        if kt.flops[k] > 0:
            dt = kt.dtype[k]
            e["flop_dtype"] = dt
            e["tflops"] = kt.flops[k] / sec / 1e12
            if dt in PEAK:
                e["frac_peak"] = kt.flops[k] / sec / PEAK[dt]
            e["complex_equiv_tflops"] = kt.cflops[k] / sec / 1e12
        if kt.bytes[k] > 0:
            e["algorithmic_bytes_per_launch"] = kt.bytes[k] / n
            e["gbps"] = kt.bytes[k] / sec / 1e9
            e["frac_hbm"] = kt.bytes[k] / sec / HBM_PEAK
        out[k] = e
    return out


HBM_ROWS = {   # hot-path steps bound by HBM: the kernel kinds that carry them
    "a2_permute": ("permute",), "a2_stage": ("stage",), "a3_assemble_dir": ("assemble_dir",),
    "a6_tile_gradients": ("grad",), "a8_gram": ("gram",), "a8_combine": ("combine",),
    "a7_theta_update": ("theta_update",), "a7_resid_update": ("resid_update",),
}


def measure_workload(tl, torch, args, wl, inputs, steps, warmup, prec, line_products, admm):
    geom, Ds, Us, ths, plans = inputs
    nfreq = len(plans)
    iters = args.iters or wl.iters
    lams = (10.0, 1.0, 0.1)
    if admm:
        iters = len(lams) * args.admm_outer * args.admm_inner
    dev = torch.device("cuda")
    perm = torch.from_numpy(tl.hilbert_order(geom.rec_ix, geom.rec_iy)).to(dev)
    ns, nr = geom.ns, geom.nr
    opts = tl.make_opts(iters, precision=prec, streams=args.streams, line_products=line_products)
    if admm:
        aopts = tl.make_admm_opts(lams, args.admm_outer, args.admm_inner, precision=prec, streams=args.streams,
                                  line_products=line_products)
        ws = torch.empty(tl.admm_workspace_bytes(plans, aopts), dtype=torch.uint8, device=dev)
    else:
        ws = torch.empty(tl.batched_workspace_bytes(plans, opts), dtype=torch.uint8, device=dev)
    out_th = [t.clone() for t in ths]
    out_fh = [torch.empty(iters + 1, dtype=torch.float64, device=dev) for _ in range(nfreq)]
    log(f"{wl.name}: workspace {ws.numel() / 2**30:.2f} GiB, {nfreq} frequencies, {iters} iterations"
        + (f" (ADMM {len(lams)} stages x {args.admm_outer} x {args.admm_inner})" if admm else ""))

    def step():
        nonlocal out_fh
        Dh = [tl.permute_columns(D, perm) for D in Ds]
        Uh = [tl.permute_columns(U, perm) for U in Us]
        if admm:
            _, out_fh = tl.admm_batched(plans, Dh, Uh, ths, lams=lams, outer=args.admm_outer, inner=args.admm_inner,
                                        precision=prec, workspace=ws, streams=args.streams, line_products=line_products)
        else:
            tl.solve_batched(plans, Dh, Uh, ths, iters, precision=prec, workspace=ws, out_thetas=out_th,
                             out_fhist=out_fh, streams=args.streams, line_products=line_products)

    for w in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    with tl.KernelTimer() as kt:
        t0 = time.perf_counter()
        for s in range(steps):
            step()
            torch.cuda.synchronize()
            log(f"step {s + 1}/{steps} done")
        t1 = time.perf_counter()
    elapsed = t1 - t0
    f_final = [float(f[-1].item()) for f in out_fh]
    f_first = [float(f[0].item()) for f in out_fh]
    value = nfreq * iters * steps / elapsed
    forms = [tl.line_form(p, prec, line_products) for p in plans]
    n_tile = sum(1 for f in forms if f[0])
    n_tgrad = sum(1 for f in forms if f[0] == 2)
    nstreams = max(1, min(args.streams, nfreq))
    kernels = kernel_table(kt)
    # the roofline kernel: the matrix-core product kind that takes the most time
    gemm_kinds = [k for k in ("gemm_line", "gemm_adjoint", "line_tile", "grad_tile", "gemm_resid", "resid_tile")
                  if k in kernels and "tflops" in kernels[k]]
    dom_kind = max(gemm_kinds, key=lambda k: kt.ms[k])
    dom = kernels[dom_kind]
    dom_name = {"gemm_line": LINE_KERNEL[args.precision] + " ([a|b] = D [X1|X2], dense line search)",
                "gemm_adjoint": ADJOINT_KERNEL[args.precision] + " (W = D^H r)",
                "line_tile": "cgemm3m_kernel<GM_STORE|GM_LINE, 1> (tile-form line-search stages)",
                "grad_tile": "cgemm3m_kernel<GM_STORE, 1|2> (tile-form gradient products)",
                "gemm_resid": "r = D X - U", "resid_tile": "tile-form residual product"}[dom_kind]
    mode = ("tile_grad" if n_tgrad else "tile") if n_tile else "dense"
    traffic = (measured_traffic(nfreq, wl.name, args.precision, mode, dom_kind) if nstreams == 1 else None)
    roofline = {
        "bound": "mfma",
        "kernel": dom_name,
        "achieved": dom["tflops"], "peak": PEAK[dom["flop_dtype"]] / 1e12, "unit": "TFLOP/s",
        "frac": dom["frac_peak"],
        "flops": "real flops of the product form that runs, true sizes: " + FORM_FLOPS[args.precision]
                 if dom_kind in ("gemm_line", "gemm_adjoint", "gemm_resid") else
                 "real flops of the three-product FP32 form (6 m n k), true ranks",
        "complex_equiv_tflops": dom["complex_equiv_tflops"],
        "traffic": traffic,
        "algorithmic_bytes": dom["algorithmic_bytes_per_launch"],
        "avg_launch_ms": dom["avg_ms"],
        "launches": dom["launches"],
        **({"note": "launches of the %d sub-batches overlap in time: a launch's duration includes "
                    "the sharing of the GPU" % nstreams} if nstreams > 1 else {}),
    }
    mm_flops = sum(kt.flops[k] for k in gemm_kinds if kt.dtype[k] == "f32")
    mm_s = sum(kt.ms[k] for k in gemm_kinds if kt.dtype[k] == "f32") * 1e-3
    hbm = {}
    for row, kinds in HBM_ROWS.items():
        ms = sum(kt.ms[k] for k in kinds)
        b = sum(kt.bytes[k] for k in kinds)
        if ms > 0 and b > 0:
            hbm[row] = {"gbps": b / (ms * 1e-3) / 1e9, "frac_hbm": b / (ms * 1e-3) / HBM_PEAK,
                        "ms_per_step": ms / steps}
    config = {"workload": wl.name if nfreq == len(wl.freqs) else f"{wl.name}[first {nfreq}]",
              "nr": nr, "ns": ns, "frequencies": nfreq, "iters": iters,
              "resid_refresh": tl.RESID_REFRESH, "streams": nstreams,
              "line_products": f"{args.line_products} ({n_tile} of {nfreq} frequencies in tile form"
                               + (f", {n_tgrad} with the gradient in tile form)" if n_tgrad else ")"),
              "optimizer": ("admm(lambda 10,1,0.1; %d x %d L-BFGS(m=5) per stage)" % (args.admm_outer,
                                                                                   args.admm_inner))
              if admm else "lbfgs(m=5)"}
    return {"value": value, "unit": "grad-iters/s", "ms_per_step": elapsed / steps * 1e3, "steps": steps,
            "config": config, "roofline": roofline, "hbm_passes": hbm,
            "mfma_frac_all_gemms": (mm_flops / mm_s / PEAK["f32"]) if mm_s > 0 else None,
            "kernels": kernels,
            "objective": {"f0_mean": sum(f_first) / nfreq, "fT_mean": sum(f_final) / nfreq}}


if __name__ == "__main__":
    main()
