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
(its three products at most 0.6 of the adjoint product: the tile-256 and tile-128 classes here);
--line-products tile keeps the dense gradient, dense the assembled X1, X2
everywhere. Every phase is one launch for all 64 frequencies except the
tile-form products: one dense launch for the frequencies that keep the dense
form, the tile-form stages per (tile size, padded rank) class.

value = grad iterations per second = 64 * 100 * steps / seconds (each grad
iteration: objective gradient, L-BFGS direction, exact line search, update).
The roofline object describes the dominant kernel (the matrix-core product
kind with the most time in one instrumented step before the timed region:
the line-search product [a | b] = D [X1 | X2] of the frequencies whose line
search stays dense), its launches timed with HIP events on their stream over
the timed steps; achieved counts the real flops of the product form that
runs (three-product FP32: 6 m n k, four-product: 8 m n k, BF16 split: 24 m n k
BF16 flops) against that instruction type's peak, complex_equiv_tflops the
8 m n k complex-equivalent rate, traffic the copy-calibrated HBM bytes of the
committed counter runs while the kernel sources are unchanged.
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
    ("fp32_3m", "tile_grad", "gemm_line"): ("cgemm3m_line_traffic_tile.json", ("cgemm3m.hip", "gemm_common.hpp")),
    ("fp32_3m", "tile_grad", "gemm_adjoint"): ("cgemm3m_adjoint_traffic_tile.json",
                                               ("cgemm3m.hip", "gemm_common.hpp")),
    ("bf16x3", "tile_grad", "gemm_line"): ("cgemm_bf16_line_traffic.json", ("cgemm_bf16.hip", "gemm_common.hpp")),
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
    """Poisson stream of per-frequency solves of uneven size: continuous batching (FIFO admission
    by HBM budget, up to --max-active overlapping solves) against the same stream solved one at a
    time, then continuous batching at 0.5x and 0.9x of the measured capacity. Each request's inputs
    are made on the device when it is admitted (same recipe, torch's device generator seeded per
    request), on its own stream, followed by its Hilbert column gather and 100-iteration solve; the
    inputs are freed when the solve completes, so the admission budget covers what requests really
    hold. Results of the saturated runs must agree bit for bit."""
    import synth
    from paper_2412_14973_amd import serve
    prec = precision_info(tl, args.precision)[0]
    line = {"dense": tl.LINE_DENSE, "tile": tl.LINE_TILE, "tile-grad": tl.LINE_TILE_GRAD}[args.line_products]
    dev = torch.device("cuda")
    iters = args.iters or 100
    reqs = synth.request_stream(args.requests, rate=200.0, iters=iters)
    perms = {}
    plans = {}
    for r in reqs:
        if r.n_side not in perms:
            g = synth.make_geometry(r.n_side, r.n_side)
            perms[r.n_side] = torch.from_numpy(tl.hilbert_order(g.rec_ix, g.rec_iy)).to(dev)
        geom = synth.make_geometry(r.n_side, r.n_side, r.ns_mode)
        plans[r.rid] = tl.Plan.from_layout(synth.request_layout(r), geom.ns)

    def make(r):
        def inputs():
            D, U, th, _, _ = synth.device_problem(r, dev)
            pd = perms[r.n_side]
            return tl.permute_columns(D, pd), tl.permute_columns(U, pd), th
        return inputs

    def jobs_for(stream):
        out = []
        for r in stream:
            p = plans[r.rid]
            # transients of making the inputs on the device and the natural-order copies
            make_bytes = synth.device_generate_bytes(p.ns, p.nr)
            req = serve.SolveRequest(p, None, None, None, r.iters, prec, line_products=line, make_inputs=make(r),
                                     make_bytes=make_bytes)
            out.append(serve.Job(rid=r.rid, arrival=r.arrival, payload=req))
        return out

    def run(stream, active, label, budget_gib=None):
        be = serve.GpuBackend(n_streams=max(active, 1))
        jobs = jobs_for(stream)
        torch.cuda.synchronize()
        be.clock = serve.WallClock()
        budget_gib = args.hbm_budget_gib if budget_gib is None else budget_gib
        srv = serve.Server(be, hbm_budget=int(budget_gib * 2 ** 30), max_active=active)
        t0 = time.time()

        def progress(job):
            n = sum(1 for j in jobs if j.finished is not None)
            if n % 16 == 0 or n == len(jobs):
                log(f"{label}: {n}/{len(jobs)} solves done ({time.time() - t0:.0f} s)")
        srv.run(jobs, on_done=progress)
        torch.cuda.synchronize()
        res = serve.summarize(jobs)
        res.update(max_active=active, hbm_budget_gib=budget_gib, peak_footprint_gib=srv.peak_in_use / 2 ** 30,
                   footprint_gib_min_max=[min(j.footprint for j in jobs) / 2 ** 30,
                                          max(j.footprint for j in jobs) / 2 ** 30],
                   admissions_waiting_for_memory=sum(1 for e in srv.log if e[1] == "wait_memory"),
                   offered_rate_per_s=len(stream) / max(stream[-1].arrival - stream[0].arrival, 1e-9))
        log(f"{label}: {res}")
        return res, {j.rid: j.result for j in jobs}

    out = {"metric": "TLR-MDD served solves/s, p50/p99 latency", "requests": len(reqs),
           "arrival_rate_per_s": 200.0, "iters": iters, "precision": args.precision,
           "line_products": args.line_products,
           "forms": [tl.line_form(plans[r.rid], prec, line)[0] for r in reqs],
           "hbm_budget_gib": args.hbm_budget_gib,
           "sizes": [[r.n_side ** 2, (r.n_side ** 2) // (2 if r.ns_mode == "half" else 1), r.d, r.k] for r in reqs],
           "inputs": "made on the device at admission (counted in the footprint), freed at completion"}
    parts = set(args.serving_parts)
    out["parts"] = sorted(parts)
    if "saturated" not in parts:
        if "sub" in parts and args.capacity is None:
            raise SystemExit("--capacity is needed for the sub-capacity runs without the saturated ones")
        out["capacity_solves_per_s"] = args.capacity
        return _sub_capacity(out, run, synth, reqs, iters, args, args.capacity) if "sub" in parts else out
    out["one_at_a_time"], res1 = run(reqs, 1, "one at a time")
    out["continuous"], res2 = run(reqs, args.max_active, "continuous")
    def same(ra, rb):   # bitwise equal results of every request completed in both runs
        common = [k for k in rb if ra.get(k) is not None and rb[k] is not None]
        return bool(common) and all(torch.equal(ra[k]["theta"], rb[k]["theta"]) and
                                    torch.equal(ra[k]["fhist"], rb[k]["fhist"]) for k in common)
    out["bitwise_same_alone_and_in_mix"] = same(res1, res2)
    out["speedup_solves_per_s"] = out["continuous"]["solves_per_s"] / out["one_at_a_time"]["solves_per_s"]
    if args.tight_budget_gib > 0 and "memory" in parts:
        # the same stream under a budget that holds the largest request but not two of them together with
        # others: admission waits on memory
        out["continuous_memory_bound"], res3 = run(reqs, args.max_active, "continuous, memory-bound budget",
                                                   args.tight_budget_gib)
        out["bitwise_same_alone_and_memory_bound"] = same(res1, res3)
        del res3
    del res1, res2
    if "sub" in parts:
        _sub_capacity(out, run, synth, reqs, iters, args, out["continuous"]["solves_per_s"])
    return out


def _sub_capacity(out, run, synth, reqs, iters, args, cap):
    """The first requests of the stream at fractions of the measured capacity (same shapes, slower arrivals)."""
    n_sub = args.sub_capacity_requests
    for frac in args.sub_capacity:
        rate = frac * cap
        stream = synth.request_stream(n_sub, rate=rate, iters=iters)
        assert [(r.n_side, r.ns_mode, r.d, r.k) for r in stream] == [(r.n_side, r.ns_mode, r.d, r.k) for r in reqs[:n_sub]]
        out[f"continuous_at_{frac:g}x_capacity"], _ = run(stream, args.max_active, f"continuous at {frac:g}x capacity")
        out[f"continuous_at_{frac:g}x_capacity"]["arrival_rate_per_s"] = rate
        if frac == min(args.sub_capacity) and args.sub_capacity_alone:
            out[f"one_at_a_time_at_{frac:g}x_capacity"], _ = run(stream, 1, f"one at a time at {frac:g}x capacity")
            out[f"one_at_a_time_at_{frac:g}x_capacity"]["arrival_rate_per_s"] = rate
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
    """Mixed-precision error table on the 64 x 64-receiver problem (nr 4096, ns 2048, tile 256,
    rank 32, 100 iterations) at the given SNRs and frequency indices: the three-product FP32 solve
    with the tile-form line search and gradient (the bench's default line), the four-product FP32
    solve with the dense forms, and the BF16 hi+lo split, each against the FP64 oracle's solve, with
    the oracle's predicted floors of rel_f beside them. The oracle's solves are read from
    --oracle-refs (files of tests/golden/make_error_table_refs.py --full) when present there, else
    run here."""
    import numpy as np

    import oracle as O
    import synth
    iters = args.iters or 100
    rows = []
    variants = [("fp32_3m_tile_forms", tl.FP32_3M, tl.LINE_TILE_GRAD), ("fp32_dense", tl.FP32, tl.LINE_DENSE),
                ("bf16x3", tl.BF16X3, tl.LINE_TILE_GRAD)]
    for snr in [float(v) for v in args.error_snrs.split(",")]:
        for f_idx in [int(v) for v in args.error_freqs.split(",")]:
            wl = synth.large(snr_db=snr, config_id=4)
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
            for name, prec, line in variants:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                thT, fh = tl.solve(plan, D, U, th, iters, precision=prec, line_products=line)
                torch.cuda.synchronize()
                res[name] = (thT.cpu().numpy().astype(np.complex128), time.perf_counter() - t0)
                log(f"snr {snr} f {f_idx}: {name} solve {res[name][1]:.2f} s")
            operm = O.hilbert_order(geom.rec_ix, geom.rec_iy)
            Do = D64.astype(np.complex128)[:, operm]
            Uo = U64.astype(np.complex128)[:, operm]
            path = os.path.join(args.oracle_refs, f"error_table_nr4096_snr{int(snr)}_f{f_idx}.npz") \
                if args.oracle_refs else None
            if path and os.path.exists(path):
                ref = np.load(path)
                th_or, t_or = ref["theta"], float(ref["oracle_s"])
                floors = (float(ref["floor_fp32"]), float(ref["floor_bf16_split"]))
                log(f"snr {snr} f {f_idx}: oracle solve read from {path}")
            else:
                t0 = time.perf_counter()
                th_or = O.solve(T, Do, Uo, th64.astype(np.complex128), iters=iters).theta
                t_or = time.perf_counter() - t0
                Xr = O.assemble(T, th_or)
                r_or = Do @ Xr - Uo
                floors = (O.predicted_objective_floor(Do, Xr, r_or, 2.0 ** -24),
                          O.predicted_objective_floor(Do, Xr, r_or, 2.0 ** -16))
                log(f"snr {snr} f {f_idx}: oracle {t_or:.1f} s")
            fo = O.objective(T, Do, Uo, th_or)[0]
            Xo = O.assemble(T, th_or)
            for name, (thg, tg) in res.items():
                fg = O.objective(T, Do, Uo, thg)[0]
                rows.append({"snr_db": snr, "freq_index": f_idx, "freq_hz": float(wl.freqs[f_idx]),
                             "precision": name, "iters": iters,
                             "rel_f": abs(fg - fo) / fo,
                             "rel_X": float(np.linalg.norm(O.assemble(T, thg) - Xo) / np.linalg.norm(Xo)),
                             "rel_theta": float(np.linalg.norm(thg - th_or) / np.linalg.norm(th_or)),
                             "predicted_floor_rel_f": floors[1] if name.startswith("bf16") else floors[0],
                             "bar": 5e-3 if name.startswith("bf16") else 1e-5,
                             "f_oracle": fo, "f_gpu": fg, "gpu_s": tg, "oracle_s": t_or})
                log(f"  {rows[-1]}")
    return {"error_table": rows,
            "workload": "nr4096_ns2048_d256_k32 (config 4 seeds; frequency indices of the 32 over 5-35 Hz)",
            "floors": "predicted_floor_rel_f: oracle.predicted_objective_floor (2 sqrt(nr) u || |D||X| || / ||r||; "
                      "u = 2^-24 for the FP32 forms, 2^-16 for the BF16 split), an upper estimate"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["batched", "large", "serving", "estimate", "tlr"], default="batched")
    ap.add_argument("--estimate-freqs", type=int, default=6, help="estimate: frequencies sampled over the band")
    ap.add_argument("--bench-lambda", type=float, default=3.0, help="estimate: Tikhonov lambda of the benchmark solve")
    ap.add_argument("--requests", type=int, default=128, help="serving: requests in the Poisson stream")
    ap.add_argument("--sub-capacity", type=lambda v: [float(x) for x in v.split(",") if x], default=[0.5, 0.9],
                    help="serving: also serve the stream at these fractions of the measured capacity")
    ap.add_argument("--no-sub-capacity-alone", dest="sub_capacity_alone", action="store_false",
                    help="serving: skip the one-at-a-time run at the lowest sub-capacity rate")
    ap.add_argument("--sub-capacity-requests", type=int, default=32,
                    help="serving: requests (the stream's first ones) of the sub-capacity runs")
    ap.add_argument("--serving-parts", type=lambda v: [x for x in v.split(",") if x],
                    default=["saturated", "memory", "sub"],
                    help="serving: saturated (one at a time and continuous at 200/s), memory (continuous under "
                         "--tight-budget-gib), sub (the sub-capacity rates)")
    ap.add_argument("--capacity", type=float, default=None,
                    help="serving: measured capacity (solves/s) for the sub-capacity runs without the saturated ones")
    ap.add_argument("--max-active", type=int, default=4, help="serving: concurrent solves")
    ap.add_argument("--hbm-budget-gib", type=float, default=96.0, help="serving: admission budget")
    ap.add_argument("--tight-budget-gib", type=float, default=64.0,
                    help="serving: also serve the saturated stream under this budget (0: skip)")
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
    ap.add_argument("--error-freqs", default="0,10,21,31", help="error table: frequency indices of the 32")
    ap.add_argument("--oracle-refs", default=None,
                    help="error table: directory of the oracle's reference solves "
                         "(tests/golden/make_error_table_refs.py --full --out DIR)")
    ap.add_argument("--line-products", choices=["dense", "tile", "tile-grad"], default="tile-grad",
                    help="line search products from the assembled X1, X2, or in tile form where cheaper "
                         "(tile-grad: the gradient's products too)")
    ap.add_argument("--streams", type=int, default=1,
                    help="batched solve: sub-batches on their own streams (problem i in sub-batch i %% streams)")
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help="batched workload: skip the nr 64 latency and nr 4096 throughput objects")
    ap.add_argument("--large-steps", type=int, default=2, help="timed steps of the nr 4096 object")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: frequencies are independent solves; "
              "multi-GPU sharding is not implemented (run with --gpus 1)", file=sys.stderr)
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
        "timing": run["timing"],
        "objective": run["objective"],
    }
    if args.workload == "batched" and not admm and args.nfreq is None and args.extra:
        log("device copy reference")
        line["copy_reference"] = copy_reference(torch)
        log("tlrmdd_grad calls on the same inputs")
        line["grad_calls"] = grad_calls(tl, torch, inputs, prec)
        log("nr 64 parity workload: microseconds per iteration")
        line["small_workload"] = small_latency(tl, torch, prec, args)
        log("nr 4096 workload (32 frequencies, inputs generated on the device)")
        wl3 = synth.large()
        inputs3 = device_inputs(wl3, torch, tl, len(wl3.freqs))
        run3 = measure_workload(tl, torch, args, wl3, inputs3, args.large_steps, 1, prec, line_products, False)
        del inputs3
        line["large_workload"] = {k: run3[k] for k in ("value", "unit", "ms_per_step", "steps", "config", "roofline",
                                                      "hbm_passes", "mfma_frac_all_gemms", "kernels", "timing",
                                                      "objective")}
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


def copy_reference(torch, mib=1024, reps=5):
    """A plain device-to-device copy (torch's copy kernel, `mib` MiB read and written per copy), timed
    with events: the streaming rate this GPU reaches in practice, beside which the HBM-bound passes
    (hbm_passes) are read."""
    src = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    b = 2.0 * (mib << 20)
    del src, dst
    return {"gbps": b / (ms * 1e-3) / 1e9, "frac_hbm": b / (ms * 1e-3) / HBM_PEAK, "ms": ms,
            "bytes_per_copy": b,
            "note": "torch copy_ of %d MiB (read + write), mean of %d: a library copy kernel, not tuned "
                    "here; passes whose vectors partly stay in the 256 MB memory-side cache between kernels "
                    "(theta-sized ones) can exceed it" % (mib, reps)}


def grad_calls(tl, torch, inputs, prec, passes=3):
    """tlrmdd_grad called once per frequency of the workload (objective and gradient of one problem per
    call: assembly, r = D X - U, W = D^H r, tile contractions, with D staged per call), calls per second
    of wall time over `passes` passes of all frequencies."""
    geom, Ds, Us, ths, plans = inputs
    dev = torch.device("cuda")
    perm = torch.from_numpy(tl.hilbert_order(geom.rec_ix, geom.rec_iy)).to(dev)
    Dh = [tl.permute_columns(D, perm) for D in Ds]
    Uh = [tl.permute_columns(U, perm) for U in Us]
    ws = torch.empty(max(p.workspace_bytes(tl._lib.OP_GRAD) for p in plans), dtype=torch.uint8, device=dev)
    for p, D, U, th in zip(plans, Dh, Uh, ths):   # warm-up pass
        tl.grad(p, D, U, th, precision=prec, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(passes):
        for p, D, U, th in zip(plans, Dh, Uh, ths):
            tl.grad(p, D, U, th, precision=prec, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = passes * len(plans)
    ns, nr = geom.ns, geom.nr
    return {"calls_per_s": n / dt, "ms_per_call": dt / n * 1e3, "calls": n,
            "dense_products_per_call": 2,
            "complex_equiv_tflops_of_the_two_products": 2 * 8.0 * ns * nr * nr * n / dt / 1e12,
            "note": "one frequency per call, D staged per call; inputs resident in HBM"}


def small_latency(tl, torch, prec, args):
    """The nr 64 parity workload (8 frequencies, 50 iterations) as one batched solve and one frequency
    alone: wall time per iteration (launch-latency bound: about 20 launches per iteration), called
    through the library and replayed as recorded HIP graphs."""
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
    # the same solves recorded once as HIP graphs and replayed (theta restored before each replay;
    # the restoring copies are inside the timed region)
    dev_fh = [torch.empty(wl.iters + 1, dtype=torch.float64, device=dev) for _ in ths]
    thb = [t.clone() for t in ths]
    gb = tl.solve_batched_graph(plans, Dh, Uh, thb, dev_fh, wl.iters, precision=prec)
    th1 = ths[0].clone()
    g1 = tl.solve_graph(plans[0], Dh[0], Uh[0], th1, dev_fh[0], wl.iters, precision=prec)

    def replay_b():
        for t, t0 in zip(thb, ths):
            t.copy_(t0)
        gb.launch()

    def replay_1():
        th1.copy_(ths[0])
        g1.launch()
    for label, fn in (("graph_batched_8freq", replay_b), ("graph_single_freq", replay_1)):
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


TIMING_NOTE = ("kernels, hbm_passes, mfma_frac_all_gemms: one instrumented step before the timed region, every "
               "launch between two HIP events on its stream; roofline: the launches of its kernel kind alone "
               "carry events over the timed steps")

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
    # one instrumented step before the timed region: every launch between two events gives the
    # per-kind table and picks the roofline kind; two event records per launch cost about 2 % of a
    # step, so inside the timed region only the roofline kind's launches carry events
    with tl.KernelTimer() as kt:
        step()
        torch.cuda.synchronize()
    log("instrumented step done")
    kernels = kernel_table(kt)
    gemm_kinds = [k for k in ("gemm_line", "gemm_adjoint", "line_tile", "grad_tile", "gemm_resid", "resid_tile")
                  if k in kernels and "tflops" in kernels[k]]
    dom_kind = max(gemm_kinds, key=lambda k: kt.ms[k])
    torch.cuda.synchronize()
    with tl.KernelTimer(kinds=[dom_kind]) as kt_dom:
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
    # the roofline kernel: the matrix-core product kind that took the most time in the instrumented
    # step, with its launches timed over the timed region
    dom = kernel_table(kt_dom)[dom_kind]
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
                        "ms_per_step": ms}
            fl = sum(kt.flops[k] for k in kinds)
            if fl > 0:
                # tile products on the FP32 matrix cores beside the HBM traffic: the nearer roof binds
                fm = fl / (ms * 1e-3) / PEAK["f32"]
                hbm[row].update(tflops=fl / (ms * 1e-3) / 1e12, frac_mfma=fm,
                                bound="mfma" if fm > hbm[row]["frac_hbm"] else "hbm")
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
            "timing": TIMING_NOTE,
            "objective": {"f0_mean": sum(f_first) / nfreq, "fT_mean": sum(f_final) / nfreq}}


if __name__ == "__main__":
    main()
