"""Benchmark of the SymNMF hot path on one MI355X.

A step is one full solver iteration: the S.H row-panel stream, the fused
gradient + AdaGrad update with FP64 partials, and the finalize reduction that
yields f(H_t), E_t, the KKT measure and Gram(H_{t+1}).  Default workload: the
single-GPU |corr| configuration - n = 100000 instruments, k = 32, S built on the
GPU from T = 2500 synthetic returns (generated on the CPU, seed 0) with 32
overlapping groups and a market factor (loading 0.4), FP32 S (40 GB) resident
in HBM, projected AdaGrad.  The S build is timed separately and is not part of
a step.

Besides the headline FP32 step rate, the JSON line carries
* ``storage``: the same step on BF16 and FP8 storage of the same S, each with
  its stream kernel's roofline fraction;
* ``time_to_tolerance``: FP32 vs BF16 storage, ADMM (the method that reaches
  the FP64 reference), time to (f(H_t) - f_ref) / f_ref <= 1e-4 with f_ref the
  committed FP64 oracle reference of this instance, and each result's
  subspace error against an FP64 reference factor computed on the device;
* ``cpu_baseline``: the FP64 oracle timed on a row sample of the same S.

Prints one JSON line.  Only one GPU is used: --gpus N with N > 1 exits with a
message.  Other studies (time to tolerance of more variants, the learned warm
start, K-means) are in studies.py.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DTYPE_NAMES = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8e4m3", "fp64": "f64"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stream_bytes(n_rows, n, k, sbytes):
    """Algorithmic HBM bytes of one S.H launch: S once, H once, S.H out."""
    return n_rows * n * sbytes + n * k * 4 + n_rows * k * 4


def step_bytes(n_rows, n, k, sbytes):
    """Algorithmic bytes of a full AdaGrad step: the S.H stream plus the update
    (read H_t, S.H, G; write H_{t+1}, G)."""
    return stream_bytes(n_rows, n, k, sbytes) + n_rows * k * 4 * 5


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("stream.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2607_24518_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload_key):
    """HBM traffic per stream launch from committed rocprofv3 PMC summaries, if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "stream_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = data.get(workload_key)
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(X_host, k, H0, eta, rows, steps, total_rows):
    """The FP64 oracle on a row panel of the same S: build the panel (not
    timed), then time `steps` oracle iterations restricted to those rows and
    scale to the total_rows of one step."""
    import numpy as np
    import oracle as o
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    n = X_host.shape[1]
    t0 = time.time()
    Z = o.standardise_columns(X_host)
    Sp = o.abs_corr_panel(Z, 0, rows)
    del Z
    build_s = time.time() - t0
    H = H0.astype(np.float64)
    G = np.zeros((rows, k))
    t0 = time.time()
    for _ in range(steps):
        g = o.gradient_panel(Sp, H, 0)
        Hr, G = o.adagrad_update(H[:rows], G, g, eta, 1e-10)
        H[:rows] = Hr
    dt = (time.time() - t0) / steps
    per_full_step = dt * total_rows / rows
    return {"value": 1.0 / per_full_step, "unit": "iters/s", "cores": int(cores), "kind": "oracle",
            "sample": f"FP64 oracle AdaGrad iterations on rows [0,{rows}) of the n={n} |corr| S "
                      f"({steps} timed steps, {dt:.3f} s each), scaled by {total_rows}/{rows}; panel build "
                      f"{build_s:.1f} s not timed"}



def timed_steps(sym, torch, ctx, S, k, params, H0, warmup, steps):
    """W untimed steps, then K steps between two events on the library stream
    (bracketed by device synchronisation); per-kernel HIP-event times of the
    timed steps from the library's profiling hook."""
    st = sym.symnmf_state_create(ctx, S, k, params, H0)
    for _ in range(warmup):
        sym.symnmf_step(ctx, S, st, want_stats=False)
    torch.cuda.synchronize()
    sym.symnmf_profile(ctx, True, read=False)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        sym.symnmf_step(ctx, S, st, want_stats=False)
    stop.record()
    torch.cuda.synchronize()
    prof = sym.symnmf_profile(ctx, False)
    last = sym.symnmf_state_stats(ctx, st)
    del st
    return start.elapsed_time(stop) / steps, prof, last


def roofline(prof, rows, n, k, dtype, workload):
    sbytes = {"fp32": 4, "bf16": 2, "fp8": 1}[dtype]
    s_ms, s_cnt = prof["stream"]
    s_avg = s_ms / max(s_cnt, 1)
    alg = stream_bytes(rows, n, k, sbytes)
    achieved = alg / (s_avg * 1e-3) / 1e9
    return {"kernel": "stream_mfma_" + {"fp32": "f32", "bf16": "lp_bf16", "fp8": "lp_fp8"}[dtype],
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(workload),
            "avg_launch_ms": round(s_avg, 4), "alg_bytes_per_launch": alg}


def ttt_leg(sym, torch, ctx, X, stores, k, H0, max_steps):
    """FP32 vs BF16 storage, ADMM, time to 1e-4 of the committed FP64 oracle
    reference, and FP32 from the network-free warm start (sketch S Omega of
    width 64 and its canonical coordinates; the trained network needs a
    training run of its own, in the warm-start study); subspace errors
    against the device FP64 ADMM run from the same H0 (the oracle's run
    repeated on the device)."""
    import studies

    n = H0.shape[0]
    ref = studies.committed_reference(0, n, 2500, 32, k, 0)
    if ref is None:
        return None
    f_dev, _, Wref, ref_s, _, _ = studies.fp64_reference(ctx, X, 0, k, H0, {"kind": 0},
                                                         [[(f"admm{ref['rho']:g}", ref["iterations"])]])
    f_ref = ref["f_ref"]
    S32 = stores["fp32"]

    def objective_of(H):
        return sym.symnmf_objective(ctx, S32, H, k)[0]

    every = 2
    store = torch.empty(max_steps // every, n, k, device=H0.device)
    eta = math.sqrt(S32.desc.mean / k)
    out = {"tol": 1e-4, "f_ref": f_ref, "method": "ADMM, rho 500",
           "reference": f"FP64 oracle ADMM from the same H0, {ref['iterations']} iterations (tests/golden)",
           "reference_factor": {"what": "device FP64 ADMM, same run", "f": f_dev,
                                "rel_to_f_ref": (f_dev - f_ref) / f_ref, "seconds": round(ref_s, 2)},
           "variants": {}}
    inits = {"fp32": lambda H: H.copy_(H0), "bf16": lambda H: H.copy_(H0),
             "fp32_warm_coords": lambda H: sym.symnmf_warm_start(ctx, S32, None, 64, k, 7, H)}
    for name, init in inits.items():
        dt = name.split("_")[0]
        e = studies.ttt_run(ctx, stores[dt], k, studies.variant_params(dt + "-admm", eta),
                            init, objective_of, f_ref, 1e-4, max_steps, every, store)
        e.pop("times")
        nsave = max_steps // every
        e["subspace_error_final"] = sym.symnmf_subspace_error(ctx, store[nsave - 1], Wref)
        if "iters" in e:
            e["subspace_error_at_tol"] = sym.symnmf_subspace_error(ctx, store[e["iters"] // every - 1], Wref)
        out["variants"][name] = e
        log(f"time to tolerance {name}: {e}")
    a = out["variants"]["fp32"].get("seconds")
    for name, key in (("bf16", "bf16_speedup"), ("fp32_warm_coords", "warm_coords_speedup")):
        b = out["variants"][name].get("seconds")
        if a and b:
            out[key] = round(a / b, 3)
    del store
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--T", type=int, default=2500)
    ap.add_argument("--groups", type=int, default=32)
    ap.add_argument("--family", default="overlap", choices=["overlap", "panel"],
                    help="returns generator: overlapping groups (n = 1e5 workload) or the column-block panel")
    ap.add_argument("--rows", type=int, default=0, help="row-panel share of S (0: all n rows)")
    ap.add_argument("--row0", type=int, default=0, help="first row of the share")
    ap.add_argument("--no-read-probe", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-rows", type=int, default=8192)
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-storage", action="store_true", help="skip the BF16 / FP8 step-rate records")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-tolerance record")
    ap.add_argument("--ttt-max", type=int, default=1000, help="ADMM iterations traced per storage type")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run the library's plain copy kernel over this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.copy_probe > 0:
        import torch
        import paper_2607_24518_amd as sym
        nbytes = int(args.copy_probe * (1 << 30)) // 16 * 16
        src = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        ctx = sym.symnmf_create(0)
        for _ in range(3):
            sym.symnmf_probe_copy(ctx, src, dst, nbytes)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "dispatches": 3}), flush=True)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; row sharding over several GPUs is designed "
                                   "but not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2607_24518_amd as sym
    import synth

    dev = torch.device("cuda:0")
    n, k = args.n, args.k
    rows = args.rows if args.rows > 0 else n - args.row0
    default = (args.family == "overlap" and rows == n and (n, k, args.T, args.groups, args.seed) ==
               (100000, 32, 2500, 32, 0))
    log(f"generating returns T={args.T} n={n} groups={args.groups} ({args.family}) on the CPU")
    if args.family == "panel":
        Xh = synth.panel_returns(args.seed, T=args.T, n=n, groups=args.groups).X
    else:
        Xh = synth.overlap_returns(args.seed, T=args.T, n=n, groups=args.groups).X
    X = Xh.to(dev)
    ctx = sym.symnmf_create(0)
    torch.cuda.synchronize()
    t0 = time.time()
    S = sym.symnmf_build_S(ctx, X, kind=sym.ABS_CORR, dtype=sym.DTYPES[args.dtype], row0=args.row0, rows=rows,
                           fp8_panel_rows=256)
    build_s = time.time() - t0
    log(f"S built in {build_s:.2f} s (rows={rows} fro2={S.desc.fro2:.6e} mean={S.desc.mean:.6f})")
    H0 = torch.empty(n, k, device=dev)
    sym.symnmf_init_H(ctx, S, k, 0, H0)
    eta = math.sqrt(S.desc.mean / k)
    params = sym.symnmf_params_default(eta=eta, max_iter=10 ** 9)
    ms_step, prof, last = timed_steps(sym, torch, ctx, S, k, params, H0, args.warmup, args.steps)
    log(f"{args.steps} steps: {ms_step:.3f} ms/step; kernels {prof}; last E={last.E:.6e} kkt={last.kkt:.3e}")
    workload = (f"abs_corr_n{n}_k{k}_T{args.T}_{args.dtype}" if rows == n else
                f"abs_corr_panel_rows{rows}_n{n}_k{k}_T{args.T}_{args.dtype}")
    roof = roofline(prof, rows, n, k, args.dtype, workload)
    sbytes = {"fp32": 4, "bf16": 2, "fp8": 1}[args.dtype]
    step_gbs = step_bytes(rows, n, k, sbytes) / (ms_step * 1e-3) / 1e9
    if not args.no_read_probe:
        nbytes = 8 << 30
        src = torch.zeros(nbytes // 4, dtype=torch.float32, device=dev)
        sink = torch.empty(1 << 16, dtype=torch.int32, device=dev)
        sym.symnmf_probe_read(ctx, src, sink, nbytes)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            sym.symnmf_probe_read(ctx, src, sink, nbytes)
        ev1.record()
        torch.cuda.synchronize()
        read_ceiling = round(nbytes * 5 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 1)
        del src, sink
        roof["read_ceiling_gbs"] = read_ceiling
        roof["frac_of_read_ceiling"] = round(roof["achieved"] / read_ceiling, 4)
        log(f"plain read probe: {read_ceiling} GB/s")

    storage, stores = None, {args.dtype: S}
    if default and args.dtype == "fp32" and not args.no_storage:
        storage = {}
        for dname in ("bf16", "fp8"):
            t0 = time.time()
            Sd = sym.symnmf_build_S(ctx, X, kind=sym.ABS_CORR, dtype=sym.DTYPES[dname], fp8_panel_rows=256)
            b_s = time.time() - t0
            ms_d, prof_d, last_d = timed_steps(sym, torch, ctx, Sd, k, params, H0, args.warmup, args.steps)
            rf = roofline(prof_d, n, n, k, dname, f"abs_corr_n{n}_k{k}_T{args.T}_{dname}")
            storage[dname] = {"value": round(1000.0 / ms_d, 3), "unit": "iters/s", "ms_per_step": round(ms_d, 4),
                              "build_S_s": round(b_s, 3), "roofline": rf}
            stores[dname] = Sd
            log(f"{dname}: {ms_d:.3f} ms/step, stream {rf['avg_launch_ms']} ms = {rf['frac']:.3f} of HBM peak")
        del stores["fp8"]
        torch.cuda.empty_cache()

    ttt = None
    if default and args.dtype == "fp32" and not args.no_ttt and "bf16" in stores:
        ttt = ttt_leg(sym, torch, ctx, X, stores, k, H0, args.ttt_max)
    del X, stores
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(Xh.double().numpy(), k, H0.double().cpu().numpy(), eta, min(args.cpu_rows, rows),
                           args.cpu_steps, rows)
        log(f"cpu baseline {cpu}")

    out = {
        "metric": "SymNMF iters/s + HBM GB/s (n=1e5,k=32); time-to-rel-obj-tol, FP32 vs BF16/warm",
        "value": round(1000.0 / ms_step, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_NAMES[args.dtype],
        "data": "synthetic",
        "config": {"workload": workload, "kind": "abs_corr", "family": args.family, "n": n, "row0": args.row0,
                   "rows": rows, "k": k, "T": args.T, "groups": args.groups, "market_loading": 0.4,
                   "S_storage": args.dtype, "method": "projected AdaGrad", "eta": eta},
        "hbm_gb_s": round(step_gbs, 1),
        "build_S_s": round(build_s, 3),
        "kernel_ms": {kname: round(v[0] / max(v[1], 1), 4) for kname, v in prof.items() if v[1]},
        "roofline": roof,
        "storage": storage,
        "time_to_tolerance": ttt,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
