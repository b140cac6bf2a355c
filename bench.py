"""Benchmark of the SymNMF hot path on one MI355X.

A step is one full solver iteration: the S.H row-panel stream, the fused
gradient + AdaGrad update with FP64 partials, and the finalize reduction that
yields f(H_t), E_t, the KKT measure and Gram(H_{t+1}).  Default workload: the
single-GPU |corr| configuration - n = 100000 instruments, k = 32, S built on the
GPU from T = 2500 synthetic returns with 32 overlapping groups and a market
factor (loading 0.4), FP32 S (40 GB) resident in HBM, projected AdaGrad.
The S build is timed separately and is not part of a step.

Prints one JSON line (see --help).  Only one GPU is used: --gpus N with N > 1
exits with a message.
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


def ttt_trace(ctx, S, k, params, init, max_steps, every, store, S_hi=None, tau_switch=None):
    """Iterate from init(H) for max_steps with every rule of the solve applied
    at the checks (symnmf_solve_trace), keeping every ``every``-th iterate in
    ``store``.  With S_hi, the precision ladder: the state moves from S to
    S_hi at the first check whose stagnation measure is below tau_switch
    (symnmf_solve_trace_ladder).  Returns (seconds of every kept iterate from
    the start of the initialisation, first certified t or -1, initialisation
    seconds, switch t or -1); times come from HIP events on the solver
    stream."""
    import torch
    import paper_2607_24518_amd as sym

    n = S.desc.n
    nsave = max_steps // every
    torch.cuda.synchronize()
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev_a.record()
    H = torch.empty(n, k, device=store.device)
    init(H)
    st = sym.symnmf_state_create(ctx, S, k, params, H)
    ev_b.record()
    switched = -1
    if S_hi is None:
        ms, certified = sym.symnmf_solve_trace(ctx, S, st, nsave * every, every, store)
    else:
        ms, certified, switched = sym.symnmf_solve_trace_ladder(ctx, S, S_hi, st, nsave * every, every, store,
                                                                tau_switch)
    torch.cuda.synchronize()
    t_init = ev_a.elapsed_time(ev_b) / 1000.0
    del st
    return [t_init + m / 1000.0 for m in ms], certified, t_init, switched


def ttt_scan(objective_of, store, nsave, f_ref, tol, every, times):
    """First kept iterate with (objective_of(H) - f_ref) / f_ref <= tol: a coarse scan
    every 32 kept iterates, then bisection inside the first bracket (the
    objective of these runs decreases except for small oscillations)."""
    cache = {}

    def rel(j):
        if j not in cache:
            cache[j] = (objective_of(store[j]) - f_ref) / f_ref
        return cache[j]

    hit = None
    prev = -1
    for j in list(range(31, nsave, 32)) + [nsave - 1]:
        if rel(j) <= tol:
            lo, hi = prev + 1, j
            while lo < hi:
                mid = (lo + hi) // 2
                if rel(mid) <= tol:
                    hi = mid
                else:
                    lo = mid + 1
            hit = lo
            break
        prev = j
    entry = {"final_rel": rel(nsave - 1), "steps_run": nsave * every, "rel_first_kept": rel(0)}
    if hit is not None:
        entry.update(iters=(hit + 1) * every, seconds=times[hit])
    return entry


def ttt_run(ctx, S, k, params, init, objective_of, f_ref, tol, max_steps, every, store, S_hi=None,
            tau_switch=None):
    """Trace from init(H), then the time to (objective_of(H_t) - f_ref) / f_ref <= tol."""
    times, certified, t_init, switched = ttt_trace(ctx, S, k, params, init, max_steps, every, store, S_hi,
                                                   tau_switch)
    entry = ttt_scan(objective_of, store, max_steps // every, f_ref, tol, every, times)
    entry.update(init_seconds=round(t_init, 4), certified_at=certified, times=times)
    if S_hi is not None:
        entry.update(switched_at=switched)
    return entry


METHODS = {"adagrad": 0, "rmsprop": 1, "piecewise": 2, "rowsvrg": 3, "blocksvrg": 4, "admm": 5, "adam": 6,
           "nadam": 7, "adan": 8, "mu": 9}
# step size of each Adam-type rule in units of sqrt(mean(S) / k), from an oracle
# sweep on the 512-instrument instance (c in {0.01, 0.03, 0.1, 0.3}: the value
# with the smallest KKT measure after 5000 iterations)
ADAM_ETA = {"adam": 0.1, "nadam": 0.03, "adan": 0.01}


def variant_params(variant, eta_base, seed=0):
    """Solver parameters of a variant name "<storage>[-<method>][-softplus][-principal]";
    "admm<rho>" selects ADMM with that penalty (plain "admm": rho = 500)."""
    import paper_2607_24518_amd as sym

    parts = variant.split("-")
    rho = 500.0
    for q in parts[1:]:
        if q.startswith("admm") and q[4:]:
            rho = float(q[4:])
    parts = ["admm" if q.startswith("admm") else q for q in parts]
    method = next((q for q in parts[1:] if q in METHODS), "adagrad")
    kw = dict(method=METHODS[method], eta=eta_base, softplus=int("softplus" in parts), max_iter=10 ** 9, seed=seed)
    if method == "admm":
        kw.update(rho=rho)
    if method == "rmsprop":
        kw.update(eta=0.03 * eta_base, eps=1e-8, alpha=0.99, mu=0.5)
    if method in ADAM_ETA:
        kw.update(eta=ADAM_ETA[method] * eta_base)
    if method == "adan":
        kw.update(beta1=0.98, beta2=0.92, beta3=0.99)
    if method == "mu":
        kw.update(eps=2.0 ** -23)
    if method in ("rowsvrg", "blocksvrg"):
        kw.update(block_rows=1024, snapshot_s=10, delta=10, phi0=0.75, row_frac=0.5)
    if "principal" in parts:            # Block-SVRG with J = I
        kw.update(independent_blocks=0)
    return sym.symnmf_params_default(**kw)


def ttt_instance(args, dev):
    """Returns of the time-to-tolerance workload and the S kind."""
    import synth

    if args.ttt_kind == "tpdm":
        inst = synth.tpdm_returns(args.seed, T=args.T, n=args.n, groups=args.groups, nu=2.5, common=True,
                                  device=dev)
        return inst.X, 1
    return synth.overlap_returns(args.seed, T=args.T, n=args.n, groups=args.groups, device=dev).X, 0


def time_to_tolerance(args):
    """Time to (f_S(H_t) - f_ref) / f_ref <= tol for several variants (storage,
    method) of the same instance and initial H.

    f_S is the objective on the FP32-stored S (MFMA products, FP64 sums across
    chunks) whatever S the variant iterates on; f_ref is the objective of the
    FP32 AdaGrad reference run certified by the stop rule (or stopped at
    --ttt-ref-iters).  Every variant's iterates are kept in HBM and evaluated
    after its timed run; the time of iterate H_t runs from the start of its
    initialisation to the copy of H_t (HIP events on the solver stream), with
    every check-time rule of the method applied.
    """
    import torch
    import paper_2607_24518_amd as sym

    dev = torch.device("cuda:0")
    n, k = args.n, args.k
    X, kind = ttt_instance(args, dev)
    ctx = sym.symnmf_create(0)
    build = dict(kind=kind, q=0.05, lower_tail=1, fp8_panel_rows=256)
    stores = {"fp32": sym.symnmf_build_S(ctx, X, dtype=sym.S_FP32, **build)}
    variants = [v for v in args.ttt_variants.split(",") if v]
    for v in variants:
        for dt in v.split("-")[0].split(">"):       # "fp8>bf16": the precision ladder
            if dt not in stores:
                stores[dt] = sym.symnmf_build_S(ctx, X, dtype=sym.DTYPES[dt], **build)
    del X
    S32 = stores["fp32"]
    eta = math.sqrt(S32.desc.mean / k)

    def objective_of(H):
        return sym.symnmf_objective(ctx, S32, H, k)[0]

    f_ref, rs, conv = reference_solve(ctx, S32, k, eta, 1, args.ttt_ref_iters)
    results = {"f_ref": f_ref, "ref_iters": int(rs.t), "ref_certified": bool(conv), "tol": args.ttt_tol,
               "variants": {}}
    every = max(1, args.ttt_save_every)
    store = torch.empty(args.ttt_max // every, n, k, device=dev)
    for v in variants:
        ladder = v.split("-")[0].split(">")
        S = stores[ladder[0]]
        S_hi = stores[ladder[1]] if len(ladder) > 1 else None
        entry = ttt_run(ctx, S, k, variant_params(v, eta), lambda H: sym.symnmf_init_H(ctx, S, k, 1, H), objective_of,
                        f_ref, args.ttt_tol, args.ttt_max, every, store, S_hi, args.ttt_switch)
        entry.pop("times")
        results["variants"][v] = entry
        log(f"variant {v}: {entry}")
    return results


def reference_solve(ctx, S, k, eta, seed, max_iter, H_out=None):
    """FP32 AdaGrad from the counter-RNG init until the stop rule certifies an
    iterate; returns (f of the certified iterate, final stats, certified)."""
    import torch
    import paper_2607_24518_amd as sym

    n = S.desc.n
    t0 = time.time()
    H0 = torch.empty(n, k, device="cuda:0")
    sym.symnmf_init_H(ctx, S, k, seed, H0)
    p = sym.symnmf_params_default(eta=eta, max_iter=max_iter)
    st = sym.symnmf_state_create(ctx, S, k, p, H0)
    Hr = H_out if H_out is not None else torch.empty(n, k, device="cuda:0")
    rs, conv = sym.symnmf_solve_to_tol(ctx, S, st, H_out=Hr)
    f_ref = sym.symnmf_objective(ctx, S, Hr, k)[0]
    del st
    log(f"reference: n={n} t={rs.t} converged={conv} E={rs.E:.6e} kkt={rs.kkt:.3e} f_ref={f_ref:.9e} "
        f"({time.time() - t0:.1f} s)")
    return f_ref, rs, conv


WARM_WIDTH, WARM_HIDDEN, WARM_OMEGA_SEED = 64, 256, 7


def warm_start_study(args):
    """Learned warm start against random initialisation.

    Training: for every training seed the returns are generated, S (FP32) is
    built and solved from the network-free warm start (stop rule or
    --warm-solve-iters), and the pair (canonical sketch coordinates, solved H)
    is kept on the device;
    the network is then trained with the scale-free Gram loss.
    Evaluation on held-out seeds (and optionally on the n = 100000 |corr|
    workload): time to relative objective tolerance from (a) the random init,
    (b) the network-free coordinates, (c) the network, each timed from the
    start of its initialisation (sketch, coordinates and network included);
    f_ref is the objective of the random-init run's certified iterate (or of
    its last iterate when the stop rule does not certify one).  A
    warm run that has not reached the tolerance within twice the random run's
    iterations falls back to the random run, and its time counts both.
    """
    import numpy as np
    import torch
    import paper_2607_24518_amd as sym
    import synth

    dev = torch.device("cuda:0")
    ctx = sym.symnmf_create(0)
    k, n = args.warm_k, args.warm_n
    W, HID = WARM_WIDTH, WARM_HIDDEN

    def returns(seed, n_cols):
        if args.warm_family == "panel":
            return synth.panel_returns(seed, T=args.warm_T, n=n_cols, groups=args.warm_groups, block=65536,
                                       device=dev).X
        return synth.overlap_returns(seed, T=args.warm_T, n=n_cols, groups=args.warm_groups, device=dev).X

    def features(S, nn):
        Y = torch.empty(nn, W, device=dev)
        sym.symnmf_sketch(ctx, S, WARM_OMEGA_SEED, W, Y)
        Xc = torch.empty(nn, W, device=dev)
        sym.symnmf_canonical(ctx, Y, k, Xc)
        return Xc

    out = {"family": args.warm_family, "n_train": args.warm_sizes or n, "n_heldout": n, "k": k, "T": args.warm_T,
           "groups": args.warm_groups, "width": W, "hidden": HID}
    # 1. training pairs
    t0 = time.time()
    pairs = []
    train_seeds = list(range(args.warm_seed0, args.warm_seed0 + args.warm_train))
    ref_iters = []
    sizes = [int(v) for v in args.warm_sizes.split(",")] if args.warm_sizes else [n]
    for i, seed in enumerate(train_seeds):
        ni = sizes[i % len(sizes)]
        X = returns(seed, ni)
        S = sym.symnmf_build_S(ctx, X, dtype=sym.S_FP32)
        del X
        eta = math.sqrt(S.desc.mean / k)
        # target: the solver's factorization from the network-free warm start
        # (it reaches lower objectives than random initialisation)
        H0 = torch.empty(ni, k, device=dev)
        sym.symnmf_warm_start(ctx, S, None, W, k, WARM_OMEGA_SEED, H0)
        st = sym.symnmf_state_create(ctx, S, k, sym.symnmf_params_default(eta=eta, max_iter=args.warm_solve_iters),
                                     H0)
        Hs = torch.empty(ni, k, device=dev)
        rs, conv = sym.symnmf_solve_to_tol(ctx, S, st, H_out=Hs)
        del st
        ref_iters.append(int(rs.t))
        pairs.append((features(S, ni), Hs))
        del S
        if (i + 1) % 10 == 0 or i + 1 == len(train_seeds):
            log(f"training instance {i + 1}/{len(train_seeds)} solved (t={rs.t} conv={conv} E={rs.E:.4e}) "
                f"{time.time() - t0:.0f} s")
    out["train_solve_iters_median"] = float(np.median(ref_iters))
    out["train_data_seconds"] = round(time.time() - t0, 1)
    # 2. training
    t0 = time.time()
    params = torch.empty(sym.symnmf_mlp_param_count(W, HID, k), device=dev)
    sym.symnmf_mlp_init(ctx, W, HID, k, args.warm_seed0, params)
    net = sym.symnmf_mlp_create(ctx, W, HID, k, params)
    rng = np.random.default_rng(args.warm_seed0)
    hist = []
    steps_total = args.warm_epochs * len(pairs)
    step = 0
    for ep in range(args.warm_epochs):
        losses = []
        for j in rng.permutation(len(pairs)):
            lr = args.warm_lr * 0.5 * (1.0 + math.cos(math.pi * step / steps_total))   # cosine decay
            losses.append(sym.symnmf_mlp_train_step(ctx, net, pairs[j][0], pairs[j][1], lr=lr,
                                                    weight_decay=args.warm_wd, loss_kind=1))
            step += 1
        hist.append(float(np.mean(losses)))
        if ep % 5 == 0 or ep + 1 == args.warm_epochs:
            log(f"epoch {ep}: mean Gram loss {hist[-1]:.5f} ({time.time() - t0:.0f} s)")
    out["train_loss_first_epoch"] = hist[0]
    out["train_loss_last_epoch"] = hist[-1]
    out["train_seconds"] = round(time.time() - t0, 1)
    del pairs
    torch.cuda.empty_cache()

    # 3. evaluation
    def evaluate(S, k_eval, model, label, seed, rand_steps, warm_steps, extra=None):
        """random init run first (it is also the reference: f_ref is its
        certified iterate, or its last one), then the two warm starts; with
        ``extra`` ({name: S stored otherwise}) the three initialisations are
        also run on those stores, evaluated on S."""
        nn = S.desc.n
        eta = math.sqrt(S.desc.mean / k_eval)
        params = variant_params("fp32", eta)

        def objective_of(H):
            return sym.symnmf_objective(ctx, S, H, k_eval)[0]

        every = 2
        store = torch.empty(rand_steps // every, nn, k_eval, device=dev)
        times, cert, t_init, _ = ttt_trace(ctx, S, k_eval, params, lambda H: sym.symnmf_init_H(ctx, S, k_eval, seed, H),
                                        rand_steps, every, store)
        ref_slot = (cert + 1) // every - 1 if cert >= 0 else rand_steps // every - 1
        f_ref = objective_of(store[ref_slot])
        res = {"f_ref": f_ref, "ref_iters": (ref_slot + 1) * every, "ref_certified": cert >= 0}
        res["random"] = ttt_scan(objective_of, store, rand_steps // every, f_ref, args.ttt_tol, every, times)
        inits = {
            "coords": lambda H: sym.symnmf_warm_start(ctx, S, None, W, k_eval, WARM_OMEGA_SEED, H),
            "mlp": lambda H: sym.symnmf_warm_start(ctx, S, model, W, k_eval, WARM_OMEGA_SEED, H),
        }
        r_it, r_s = res["random"].get("iters"), res["random"].get("seconds")
        for name, init in inits.items():
            wt, wcert, w_init, _ = ttt_trace(ctx, S, k_eval, params, init, warm_steps, every, store)
            e = ttt_scan(objective_of, store, warm_steps // every, f_ref, args.ttt_tol, every, wt)
            e["init_seconds"] = round(w_init, 4)
            if r_it is not None:
                if e.get("iters") is None or e["iters"] > 2 * r_it:
                    # fallback: the warm run is abandoned after 2x the random
                    # iterations (or its cap) and the random run is started
                    idx = min(2 * r_it // every, len(wt)) - 1
                    e["fallback"] = True
                    e["seconds_with_fallback"] = wt[idx] + r_s
                else:
                    e["fallback"] = False
                    e["seconds_with_fallback"] = e["seconds"]
                e["speedup_vs_random"] = round(r_s / e["seconds_with_fallback"], 3)
            res[name] = e
        for xname, Sx in (extra or {}).items():
            xinits = {
                "random": lambda H: sym.symnmf_init_H(ctx, Sx, k_eval, seed, H),
                "coords": lambda H: sym.symnmf_warm_start(ctx, Sx, None, W, k_eval, WARM_OMEGA_SEED, H),
                "mlp": lambda H: sym.symnmf_warm_start(ctx, Sx, model, W, k_eval, WARM_OMEGA_SEED, H),
            }
            for name, init in xinits.items():
                steps = rand_steps if name == "random" else warm_steps
                wt, _, w_init, _ = ttt_trace(ctx, Sx, k_eval, params, init, steps, every, store)
                e = ttt_scan(objective_of, store, steps // every, f_ref, args.ttt_tol, every, wt)
                e["init_seconds"] = round(w_init, 4)
                if r_s is not None and e.get("seconds"):
                    e["speedup_vs_fp32_random"] = round(r_s / e["seconds"], 3)
                res[f"{xname}-{name}"] = e
        del store
        log(f"{label}: " + json.dumps(res))
        return res

    held = []
    for seed in range(args.warm_heldout0, args.warm_heldout0 + args.warm_heldout):
        X = returns(seed, n)
        S = sym.symnmf_build_S(ctx, X, dtype=sym.S_FP32)
        del X
        held.append(evaluate(S, k, net, f"held-out seed {seed}", seed, args.warm_max, args.warm_warm_max))
        del S
    out["heldout"] = held
    for name in ("coords", "mlp"):
        sp = [h[name]["speedup_vs_random"] for h in held if "speedup_vs_random" in h[name]]
        if sp:
            out[f"{name}_speedup_median"] = float(np.median(sp))
            out[f"{name}_wins"] = int(sum(1 for v in sp if v > 1.0))
            out[f"{name}_fallbacks"] = int(sum(1 for h in held if h[name].get("fallback")))
    if args.warm_c3:
        X = synth.overlap_returns(0, T=2500, n=100000, groups=32, device=dev).X
        S = sym.symnmf_build_S(ctx, X, dtype=sym.S_FP32)
        extra = {dt: sym.symnmf_build_S(ctx, X, dtype=sym.DTYPES[dt], fp8_panel_rows=256)
                 for dt in args.warm_c3_dtypes.split(",") if dt and dt != "fp32"}
        del X
        out["c3_abs_corr_n100000"] = evaluate(S, k, net, "n=100000 |corr|", 1, args.warm_c3_max, args.warm_c3_max,
                                              extra)
    return out


def kmeans_cpu_baseline(X_host, K, rows):
    """The FP64 oracle's Lloyd step (assignment against K unit centroids and
    the cluster-sum update) on rows [0, rows) of the |corr| S, scaled to all
    n rows; the panel build is not timed."""
    import numpy as np
    import oracle as o
    import oracle.kmeans_oracle as km
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    n = X_host.shape[1]
    Z = o.standardise_columns(X_host)
    Sp = o.abs_corr_panel(Z, 0, rows)
    del Z
    Shat, _ = km.unit_rows(Sp)
    rng = np.random.default_rng(0)
    C = rng.random((K, n))
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    t0 = time.time()
    reps = 8
    for _ in range(reps):
        labels, _, _ = km.assign(Shat, C)
        C = km.centroids(Shat, labels, K, C)
    dt = (time.time() - t0) / reps
    per_iter = dt * n / rows
    return {"value": per_iter, "unit": "s/iteration", "cores": int(cores), "kind": "oracle",
            "sample": f"FP64 oracle Lloyd iterations (assignment + update) on rows [0,{rows}) of the n={n} |corr| S "
                      f"at K={K} ({reps} timed, {dt:.3f} s each), scaled by {n}/{rows}"}


def logspace_study(args):
    """Projected (P) vs softplus (L) convergence counts on the appendix's
    benchmark matrices, as in the paper's LogSpace table: runs satisfying the
    three-criterion stop rule within --logspace-budget iterations, out of
    3 seeds x 2 matrix types per size, k = floor(sqrt(n)) (capped at 64)."""
    import torch
    import paper_2607_24518_amd as sym
    import synth
    dev = torch.device("cuda:0")
    ctx = sym.symnmf_create(0)
    sizes = [int(v) for v in args.logspace_sizes.split(",")]
    methods = {"rmsprop": dict(method=sym.RMSPROP, c=0.03, eps=1e-8, alpha=0.99, mu=0.5),
               "adam": dict(method=sym.ADAM, c=ADAM_ETA["adam"]),
               "adagrad": dict(method=sym.ADAGRAD, c=1.0)}
    table, runs = {}, []
    for n in sizes:
        k = min(math.isqrt(n), 64)
        for kind in ("corr", "tpdm"):
            for seed in (7, 42, 99):
                X = synth.paper_benchmark(seed, n, kind, device=dev).X
                if kind == "corr":
                    S = sym.symnmf_build_S(ctx, X, kind=sym.ABS_CORR, dtype=sym.S_FP32)
                else:
                    S = sym.symnmf_build_S(ctx, X, kind=sym.TPDM, dtype=sym.S_FP32, q=0.01, lower_tail=0,
                                           raw_marginals=1)
                del X
                H0 = torch.empty(n, k, device=dev)
                sym.symnmf_init_H(ctx, S, k, seed, H0)
                base = math.sqrt(S.desc.mean / k)
                for name, m in methods.items():
                    for form in (0, 1):
                        kw = {q: v for q, v in m.items() if q != "c"}
                        p = sym.symnmf_params_default(eta=m["c"] * base, softplus=form, max_iter=args.logspace_budget,
                                                      seed=seed, **kw)
                        st = sym.symnmf_state_create(ctx, S, k, p, H0)
                        t0 = time.perf_counter()
                        try:
                            stats, conv = sym.symnmf_solve_to_tol(ctx, S, st)
                        except sym.SymnmfError as e:     # e.g. a non-finite gradient: not converged
                            log(f"logspace n={n} {kind} seed={seed} {name} form={form}: {e}")
                            stats, conv = sym.symnmf_state_stats(ctx, st), False
                        wall = time.perf_counter() - t0
                        key = f"n{n}_{name}_{'L' if form else 'P'}"
                        table[key] = table.get(key, 0) + int(bool(conv))
                        rec = {"n": n, "k": k, "kind": kind, "seed": seed, "method": name, "form": "L" if form else "P",
                               "converged": bool(conv), "t": int(stats.t), "E": stats.E, "kkt": stats.kkt,
                               "seconds": round(wall, 3)}
                        runs.append(rec)
                        log(f"logspace {rec}")
                        del st
                del S
                torch.cuda.empty_cache()
    return {"converged_of_6": table, "runs": runs}


def phase1_study(args):
    """The paper's Phase-1 protocol on the appendix's benchmark matrices: for
    n in --phase1-sizes, both matrix types and seeds 7, 42, 99 (6 runs per
    size), every method solves with the three-criterion stop rule within
    --logspace-budget iterations; reports the runs certified and the mean wall
    time of the certified runs (the paper's Phase-1 table, one GPU).
    k = floor(sqrt(n)), capped at 64."""
    import torch
    import paper_2607_24518_amd as sym
    import synth
    dev = torch.device("cuda:0")
    ctx = sym.symnmf_create(0)
    sizes = [int(v) for v in args.phase1_sizes.split(",")]
    svrg = dict(block_rows=256, snapshot_s=10, delta=10, phi0=0.75, row_frac=0.5)
    methods = {
        "admm": dict(method=sym.ADMM, c=1.0, rho=500.0),
        "rmsprop": dict(method=sym.RMSPROP, c=0.03, eps=1e-8, alpha=0.99, mu=0.5),
        "blocksvrg": dict(method=sym.BLOCK_SVRG, c=1.0, **svrg),
        "adagrad": dict(method=sym.ADAGRAD, c=1.0),
        "rowsvrg": dict(method=sym.ROW_SVRG, c=1.0, **svrg),
        "piecewise": dict(method=sym.PIECEWISE_ADAGRAD, c=1.0),
        "adan": dict(method=sym.ADAN, c=ADAM_ETA["adan"], beta1=0.98, beta2=0.92, beta3=0.99),
        "adam": dict(method=sym.ADAM, c=ADAM_ETA["adam"]),
        "nadam": dict(method=sym.NADAM, c=ADAM_ETA["nadam"]),
        "mu": dict(method=sym.MU, c=1.0, eps=2.0 ** -23),
    }
    runs = []
    for n in sizes:
        k = min(math.isqrt(n), 64)
        for kind in ("corr", "tpdm"):
            for seed in (7, 42, 99):
                X = synth.paper_benchmark(seed, n, kind, device=dev).X
                if kind == "corr":
                    S = sym.symnmf_build_S(ctx, X, kind=sym.ABS_CORR, dtype=sym.S_FP32)
                else:
                    S = sym.symnmf_build_S(ctx, X, kind=sym.TPDM, dtype=sym.S_FP32, q=0.01, lower_tail=0,
                                           raw_marginals=1)
                del X
                H0 = torch.empty(n, k, device=dev)
                sym.symnmf_init_H(ctx, S, k, seed, H0)
                base = math.sqrt(S.desc.mean / k)
                for name, m in methods.items():
                    kw = {q: v for q, v in m.items() if q != "c"}
                    p = sym.symnmf_params_default(eta=m["c"] * base, max_iter=args.logspace_budget, seed=seed, **kw)
                    st = sym.symnmf_state_create(ctx, S, k, p, H0)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    try:
                        stats, conv = sym.symnmf_solve_to_tol(ctx, S, st)
                    except sym.SymnmfError as e:
                        log(f"phase1 n={n} {kind} seed={seed} {name}: {e}")
                        stats, conv = sym.symnmf_state_stats(ctx, st), False
                    wall = time.perf_counter() - t0
                    rec = {"n": n, "k": k, "kind": kind, "seed": seed, "method": name, "converged": bool(conv),
                           "t": int(stats.t), "E": stats.E, "kkt": stats.kkt, "seconds": round(wall, 4)}
                    runs.append(rec)
                    log(f"phase1 {rec}")
                    del st
                del S
                torch.cuda.empty_cache()
    table = {}
    for name in methods:
        row = {}
        for n in sizes:
            rr = [r for r in runs if r["method"] == name and r["n"] == n]
            ok = [r for r in rr if r["converged"]]
            row[str(n)] = {"converged": f"{len(ok)}/{len(rr)}",
                           "wall_s": round(sum(r["seconds"] for r in ok) / len(ok), 3) if ok else None,
                           "iters": round(sum(r["t"] for r in ok) / len(ok), 1) if ok else None}
        table[name] = row
    return {"table": table, "runs": runs}


def kmeans_paper_benchmark(args, ctx, Ks):
    """K-means on the appendix's own benchmark matrices (floor(sqrt(n))
    groups plus the common factor, 40000 samples; |corr| and the raw-marginal
    TPDM with the top 1 % of samples), one instance and seeding per seed, as
    in the paper's K-means table (means over seeds 7, 42, 99)."""
    import torch
    import paper_2607_24518_amd as sym
    import synth
    dev = torch.device("cuda:0")
    n = args.n
    runs = []
    for kind in args.kmeans_kinds.split(","):
        for seed in [int(v) for v in args.kmeans_seeds.split(",")]:
            log(f"paper benchmark {kind} n={n} seed={seed}")
            X = synth.paper_benchmark(seed, n, kind, device=dev).X
            torch.cuda.synchronize()
            for dname in args.kmeans_dtypes.split(","):
                if kind == "corr":
                    S = sym.symnmf_build_S(ctx, X, kind=sym.ABS_CORR, dtype=sym.DTYPES[dname])
                else:
                    S = sym.symnmf_build_S(ctx, X, kind=sym.TPDM, dtype=sym.DTYPES[dname], q=0.01, lower_tail=0,
                                           raw_marginals=1)
                spec = None
                if dname == "fp32":
                    t0 = time.perf_counter()
                    spec = sym.symnmf_spectral(ctx, S, max_iter=300, tol=1e-9)
                    spec["seconds"] = round(time.perf_counter() - t0, 3)
                    spec["bound"] = (spec["r_eff"] - 1.0) ** 2
                    log(f"spectral {kind} seed={seed}: {spec}")
                for K in Ks:
                    labels = torch.zeros(n, dtype=torch.int32, device=dev)
                    for rep in range(args.kmeans_reps):
                        t0 = time.perf_counter()
                        rows = (sym.symnmf_kmeans_seed_pp(ctx, S, K, seed) if args.kmeans_seeding == "kpp"
                                else None)
                        seed_s = time.perf_counter() - t0
                        st = sym.symnmf_kmeans(ctx, S, K, labels, seed=seed, init_rows=rows, tol=1e-4,
                                               max_iter=args.kmeans_max_iter, allow_notconv=True)
                        wall = time.perf_counter() - t0
                    sil = sym.symnmf_silhouette(ctx, S, labels, K)
                    rec = {"kind": kind, "seed": seed, "S_storage": dname, "K": K, "seconds": round(wall, 4),
                           "seeding": args.kmeans_seeding, "seeding_s": round(seed_s, 4),
                           "iters": st["iters"], "converged": bool(st["converged"]), "J": st["J"],
                           "silhouette": round(sil, 4), "spectral": spec}
                    log(f"kmeans {rec}")
                    runs.append(rec)
                del S
                torch.cuda.empty_cache()
            del X
            torch.cuda.empty_cache()
    means = {}
    for r in runs:
        key = f"{r['kind']}_{r['S_storage']}_K{r['K']}"
        means.setdefault(key, []).append(r)
    def mean_spec(v, key):
        vals = [r["spectral"][key] for r in v if r.get("spectral")]
        return round(sum(vals) / len(vals), 4) if vals else None

    summary = {k: {"seconds": round(sum(r["seconds"] for r in v) / len(v), 4),
                   "seeding_s": round(sum(r["seeding_s"] for r in v) / len(v), 4),
                   "lambda1": mean_spec(v, "lambda1"), "r_eff": mean_spec(v, "r_eff"),
                   "collapse": mean_spec(v, "collapse"), "bound": mean_spec(v, "bound"),
                   "iters": round(sum(r["iters"] for r in v) / len(v), 2),
                   "silhouette": round(sum(r["silhouette"] for r in v) / len(v), 4),
                   "converged": all(r["converged"] for r in v), "seeds": len(v)} for k, v in means.items()}
    return {"runs": runs, "means": summary}


def kmeans_bench(args):
    """Spherical K-means on the rows of the n = 10^5 |corr| S: wall time of
    symnmf_kmeans to the stop rule (relative drop of sum(1 - cos) below 1e-4)
    and of the silhouette, per storage type and cluster count."""
    import torch
    import paper_2607_24518_amd as sym
    import synth
    dev = torch.device("cuda:0")
    n = args.n
    ctx = sym.symnmf_create(0)
    Ks = [int(v) for v in args.kmeans.split(",") if v]
    runs = []
    if args.kmeans_family == "paper":
        return kmeans_paper_benchmark(args, ctx, Ks)
    log(f"generating returns T={args.T} n={n} groups={args.groups}")
    X = synth.overlap_returns(args.seed, T=args.T, n=n, groups=args.groups, device=dev).X
    for dname in args.kmeans_dtypes.split(","):
        S = sym.symnmf_build_S(ctx, X, kind=sym.ABS_CORR, dtype=sym.DTYPES[dname], fp8_panel_rows=256)
        torch.cuda.synchronize()
        sbytes = {"fp32": 4, "bf16": 2, "fp8": 1}[dname]
        for K in Ks:
            labels = torch.zeros(n, dtype=torch.int32, device=dev)
            w = 16 if K <= 16 else (32 if K <= 32 else 64)
            slices = (K + w - 1) // w
            for rep in range(args.kmeans_reps):
                t0 = time.perf_counter()
                rows = (sym.symnmf_kmeans_seed_pp(ctx, S, K, args.kmeans_seed) if args.kmeans_seeding == "kpp"
                        else None)
                seed_s = time.perf_counter() - t0
                st = sym.symnmf_kmeans(ctx, S, K, labels, seed=args.kmeans_seed, init_rows=rows, tol=1e-4,
                                       max_iter=args.kmeans_max_iter, allow_notconv=True)
                wall = time.perf_counter() - t0
            t0 = time.perf_counter()
            sil = sym.symnmf_silhouette(ctx, S, labels, K)
            sil_s = time.perf_counter() - t0
            passes = 2 * slices * (st["iters"] + 1)            # stream passes of the Lloyd iterations
            rec = {"S_storage": dname, "K": K, "slice_width": w, "slices": slices, "seconds": round(wall, 4),
                   "seeding": args.kmeans_seeding, "seeding_s": round(seed_s, 4),
                   "iters": st["iters"], "converged": bool(st["converged"]), "J0": st["J0"], "J": st["J"],
                   "empty_clusters": st["empty"], "silhouette": round(sil, 5), "silhouette_s": round(sil_s, 4),
                   "stream_passes": passes, "ms_per_pass_incl_overheads": round(1e3 * wall / (passes + 1), 3),
                   "S_GB_per_pass": round(n * n * sbytes / 1e9, 2)}
            log(f"kmeans {rec}")
            runs.append(rec)
        del S
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        Kc = Ks[0]
        cpu = kmeans_cpu_baseline(X.double().cpu().numpy(), Kc, min(args.cpu_rows, n))
        log(f"cpu baseline {cpu}")
    return {"runs": runs, "cpu_baseline": cpu}


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
    ap.add_argument("--no-read-probe", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-rows", type=int, default=8192)
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run the library's plain copy kernel over this many GiB (counter calibration)")
    ap.add_argument("--ttt", action="store_true", help="time-to-tolerance comparison instead of the step rate")
    ap.add_argument("--ttt-variants", default="fp32,bf16,fp8,fp32-softplus")
    ap.add_argument("--ttt-kind", default="abs_corr", choices=["abs_corr", "tpdm"])
    ap.add_argument("--ttt-tol", type=float, default=1e-4)
    ap.add_argument("--ttt-switch", type=float, default=1e-5,
                    help="precision ladder (variants 'lo>hi-...'): move to the precise storage at the first check "
                         "whose stagnation measure (E_{t-delta} - E_t) / E_0 is below this")
    ap.add_argument("--ttt-max", type=int, default=6000)
    ap.add_argument("--ttt-save-every", type=int, default=2)
    ap.add_argument("--ttt-ref-iters", type=int, default=8000)
    ap.add_argument("--warm", action="store_true", help="learned warm start study instead of the step rate")
    ap.add_argument("--warm-family", default="panel", choices=["panel", "overlap"])
    ap.add_argument("--warm-n", type=int, default=20000)
    ap.add_argument("--warm-sizes", default="", help="training instance sizes, cycled (default: --warm-n)")
    ap.add_argument("--warm-k", type=int, default=64)
    ap.add_argument("--warm-T", type=int, default=1000)
    ap.add_argument("--warm-groups", type=int, default=64)
    ap.add_argument("--warm-train", type=int, default=200)
    ap.add_argument("--warm-seed0", type=int, default=1000)
    ap.add_argument("--warm-heldout", type=int, default=20)
    ap.add_argument("--warm-heldout0", type=int, default=2000)
    ap.add_argument("--warm-solve-iters", type=int, default=1500)
    ap.add_argument("--warm-ref-iters", type=int, default=8000)
    ap.add_argument("--warm-epochs", type=int, default=40)
    ap.add_argument("--warm-lr", type=float, default=1e-3)
    ap.add_argument("--warm-wd", type=float, default=1e-4)
    ap.add_argument("--warm-max", type=int, default=8000, help="steps of the random-init (reference) run")
    ap.add_argument("--warm-warm-max", type=int, default=3000, help="steps of each warm-started run")
    ap.add_argument("--warm-c3", action="store_true", help="also evaluate on the n=100000 |corr| workload")
    ap.add_argument("--warm-c3-max", type=int, default=6000)
    ap.add_argument("--warm-c3-dtypes", default="fp32", help="storage types of the n=100000 evaluation, e.g. fp32,bf16")
    ap.add_argument("--kmeans", default="", help="spherical K-means study instead of the step rate: cluster counts, "
                                                 "e.g. 32,316")
    ap.add_argument("--kmeans-dtypes", default="fp32,bf16")
    ap.add_argument("--kmeans-seed", type=int, default=7)
    ap.add_argument("--kmeans-max-iter", type=int, default=100)
    ap.add_argument("--kmeans-reps", type=int, default=2, help="runs per case; the last is reported")
    ap.add_argument("--kmeans-family", default="overlap", choices=["overlap", "paper"],
                    help="overlapping-groups returns, or the appendix's benchmark matrices (--kmeans-kinds)")
    ap.add_argument("--kmeans-kinds", default="corr,tpdm")
    ap.add_argument("--kmeans-seeding", default="forgy", choices=["forgy", "kpp"],
                    help="Forgy rows or k-means++ rows (symnmf_kmeans_seed_pp, timed with the run)")
    ap.add_argument("--kmeans-seeds", default="7,42,99")
    ap.add_argument("--logspace", action="store_true", help="projected vs softplus convergence counts instead of the "
                                                           "step rate")
    ap.add_argument("--logspace-sizes", default="100,1000,10000")
    ap.add_argument("--logspace-budget", type=int, default=20000)
    ap.add_argument("--phase1", action="store_true", help="the paper's Phase-1 table (every method, n <= 1e4) "
                                                         "instead of the step rate")
    ap.add_argument("--phase1-sizes", default="100,1000,10000")
    args = ap.parse_args()

    if args.phase1:
        res = phase1_study(args)
        print(json.dumps({"metric": "runs certified by the stop rule and mean wall time of the certified runs",
                          "unit": "s", "n_gpus": 1, "data": "synthetic", "budget": args.logspace_budget, **res}),
              flush=True)
        return

    if args.logspace:
        res = logspace_study(args)
        print(json.dumps({"metric": "runs certified by the stop rule within the iteration budget, projected vs "
                                    "softplus", "unit": "runs of 6", "n_gpus": 1, "data": "synthetic",
                          "budget": args.logspace_budget, **res}), flush=True)
        return

    if args.kmeans:
        res = kmeans_bench(args)
        print(json.dumps({"metric": "spherical K-means on the rows of S: wall time to the stop rule", "unit": "s",
                          "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": (f"paper_benchmark_n{args.n}_T40000" if args.kmeans_family == "paper"
                                                  else f"abs_corr_n{args.n}_T{args.T}_groups{args.groups}"),
                                     "stop": "relative drop of sum(1 - cos) below 1e-4"},
                          **res}), flush=True)
        return

    if args.warm:
        res = warm_start_study(args)
        print(json.dumps({"metric": "time to relative objective tolerance, learned warm start vs random init",
                          "unit": "s", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                          "tol": args.ttt_tol, **res}), flush=True)
        return

    if args.ttt:
        res = time_to_tolerance(args)
        base = res["variants"].get("fp32", {}).get("seconds")
        for v in res["variants"].values():
            if base and v.get("seconds"):
                v["speedup_vs_fp32"] = round(base / v["seconds"], 3)
        print(json.dumps({"metric": "time to relative objective tolerance", "unit": "s",
                          "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": f"{args.ttt_kind}_n{args.n}_k{args.k}_T{args.T}",
                                     "reference_method": "AdaGrad"},
                          **res}), flush=True)
        return

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

    import numpy as np
    import torch
    import paper_2607_24518_amd as sym
    import synth

    dev = torch.device("cuda:0")
    n, k = args.n, args.k
    rows = args.rows if args.rows > 0 else n
    log(f"generating returns T={args.T} n={n} groups={args.groups} ({args.family})")
    if args.family == "panel":
        X = synth.panel_returns(args.seed, T=args.T, n=n, groups=args.groups, device=dev).X
    else:
        X = synth.overlap_returns(args.seed, T=args.T, n=n, groups=args.groups, device=dev).X
    ctx = sym.symnmf_create(0)
    dt = sym.DTYPES[args.dtype]
    torch.cuda.synchronize()
    t0 = time.time()
    S = sym.symnmf_build_S(ctx, X, kind=sym.ABS_CORR, dtype=dt, rows=rows, fp8_panel_rows=256)
    build_s = time.time() - t0
    log(f"S built in {build_s:.2f} s (rows={rows} fro2={S.desc.fro2:.6e} mean={S.desc.mean:.6f})")
    H0 = torch.empty(n, k, device=dev)
    sym.symnmf_init_H(ctx, S, k, 1, H0)
    eta = math.sqrt(S.desc.mean / k)
    params = sym.symnmf_params_default(eta=eta, max_iter=10 ** 9)
    st = sym.symnmf_state_create(ctx, S, k, params, H0)

    for _ in range(args.warmup):
        sym.symnmf_step(ctx, S, st, want_stats=False)
    torch.cuda.synchronize()
    sym.symnmf_profile(ctx, True, read=False)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        sym.symnmf_step(ctx, S, st, want_stats=False)
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    prof = sym.symnmf_profile(ctx, False)
    last = sym.symnmf_state_stats(ctx, st)
    ms_step = total_ms / args.steps
    log(f"{args.steps} steps: {ms_step:.3f} ms/step; kernels {prof}; last E={last.E:.6e} kkt={last.kkt:.3e}")

    sbytes = {"fp32": 4, "bf16": 2, "fp8": 1}[args.dtype]
    s_ms, s_cnt = prof["stream"]
    s_avg = s_ms / max(s_cnt, 1)
    alg = stream_bytes(rows, n, k, sbytes)
    achieved = alg / (s_avg * 1e-3) / 1e9
    workload = (f"abs_corr_n{n}_k{k}_T{args.T}_{args.dtype}" if rows == n else
                f"abs_corr_panel_rows{rows}_n{n}_k{k}_T{args.T}_{args.dtype}")
    traffic = load_traffic(workload)
    roof = {"kernel": "stream_mfma_" + ("f32" if args.dtype == "fp32" else ("lp_bf16" if args.dtype == "bf16" else "lp_fp8")),
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "avg_launch_ms": round(s_avg, 4), "alg_bytes_per_launch": alg}
    step_gbs = step_bytes(rows, n, k, sbytes) / (ms_step * 1e-3) / 1e9
    read_ceiling = None
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
        roof["frac_of_read_ceiling"] = round(achieved / read_ceiling, 4)
        log(f"plain read probe: {read_ceiling} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        Xh = X.double().cpu().numpy()
        H0h = H0.double().cpu().numpy()
        cpu = cpu_baseline(Xh, k, H0h, eta, min(args.cpu_rows, rows), args.cpu_steps, rows)
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
        "config": {"workload": workload, "kind": "abs_corr", "family": args.family, "n": n, "rows": rows, "k": k,
                   "T": args.T, "groups": args.groups, "market_loading": 0.4, "S_storage": args.dtype,
                   "method": "projected AdaGrad", "eta": eta},
        "hbm_gb_s": round(step_gbs, 1),
        "build_S_s": round(build_s, 3),
        "kernel_ms": {kname: round(v[0] / max(v[1], 1), 4) for kname, v in prof.items() if v[1]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
