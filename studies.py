"""Measurement studies of the SymNMF library on one MI355X, beside the step-rate
benchmark of bench.py:

* ``--ttt``: time to a relative objective tolerance, (f(H_t) - f_ref) / f_ref
  <= tol, for several variants (storage of S, method, precision ladder) of
  one instance and one initial factor; f_ref is the FP64 oracle's reference
  objective where one is committed (tests/golden), else the lowest objective
  of an FP64 ADMM run on the device; every result also gets its subspace
  error against an FP64 reference factor;
* ``--warm``: the learned warm start against random initialisation;
* ``--kmeans``: spherical K-means on the rows of S;
* ``--logspace``: projected vs softplus convergence counts on the appendix's
  benchmark matrices.

Each prints one JSON line on stdout; progress goes to stderr.  The library is
the only compute path used here (no oracle).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(f"[studies] {msg}", file=sys.stderr, flush=True)


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
            tau_switch=None, more_tols=()):
    """Trace from init(H), then the time to (objective_of(H_t) - f_ref) / f_ref <= tol
    (and to each of ``more_tols``, under "at_tol")."""
    times, certified, t_init, switched = ttt_trace(ctx, S, k, params, init, max_steps, every, store, S_hi,
                                                   tau_switch)
    entry = ttt_scan(objective_of, store, max_steps // every, f_ref, tol, every, times)
    if more_tols:
        entry["at_tol"] = {}
        for t2 in more_tols:
            e2 = ttt_scan(objective_of, store, max_steps // every, f_ref, t2, every, times)
            entry["at_tol"][f"{t2:g}"] = {q: e2[q] for q in ("iters", "seconds") if q in e2} or None
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
    """Solver parameters of a variant name "<storage>[-<method>][-softplus][-principal][-eta<c>]";
    "admm<rho>" selects ADMM with that penalty (plain "admm": rho = 500); "eta<c>"
    multiplies the method's step size by c."""
    import paper_2607_24518_amd as sym

    parts = variant.split("-")
    rho, eta_mul = 500.0, 1.0
    for q in parts[1:]:
        if q.startswith("admm") and q[4:]:
            rho = float(q[4:])
        if q.startswith("eta") and q[3:]:
            eta_mul = float(q[3:])
    eta_base = eta_base * eta_mul
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


def ttt_instance(args):
    """Returns of the time-to-tolerance workload and the S kind.  The |corr|
    panel is generated on the CPU (the instance the oracle's committed
    reference was computed on); the TPDM panel (T x n = 2e9 Student-t draws,
    no oracle reference at this size) on the GPU."""
    import synth

    if args.ttt_kind == "tpdm":
        inst = synth.tpdm_returns(args.seed, T=args.T, n=args.n, groups=args.groups, nu=2.5, common=True,
                                  device="cuda:0")
        return inst.X, 1
    return synth.overlap_returns(args.seed, T=args.T, n=args.n, groups=args.groups, device="cpu").X, 0


GOLDEN = os.path.join(ROOT, "tests", "golden")


def committed_reference(kind, n, T, groups, k, seed):
    """The FP64 oracle's reference run of this workload, if one is committed
    (tests/golden/*_reference.json, written by the oracle-only script next
    to it), else None."""
    name = {0: "abs_corr", 1: "tpdm"}[kind]
    path = os.path.join(GOLDEN, f"{name}_n{n}_k{k}_reference.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if (d["n"], d["T"], d["groups"], d["k"], d["seed"]) != (n, T, groups, k, seed) or not d.get("complete"):
        return None
    return d


def init_factor(ctx, S, k, seed, H, mean=None):
    """Counter-RNG initial factor H0 = u sqrt(mean / k) (symnmf_init_H); with
    ``mean`` given, the scale uses that mean instead of the stored S's (so a
    device run starts from the oracle's H0 bit for bit)."""
    import ctypes
    import paper_2607_24518_amd as sym

    if mean is None:
        return sym.symnmf_init_H(ctx, S, k, seed, H)
    d = sym.symnmf_S()
    ctypes.memmove(ctypes.byref(d), ctypes.byref(S.desc), ctypes.sizeof(d))
    d.mean = mean
    return sym.symnmf_init_H(ctx, sym.Matrix(d, S.buf), k, seed, H)


def fp64_reference(ctx, X, kind, k, H0, build, plans):
    """FP64 runs (FP64 storage and state) from H0.  ``plans``: list of
    reference plans, each a list of stages (variant name, iterations) run one
    after the other, every stage starting from the previous stage's last
    iterate (e.g. [("admm500", 1500)] or [("adam", 12000), ("admm50", 3000)]).
    The plan that ends lowest is the reference: (objective of its last
    iterate, lowest objective it saw, its last iterate as FP32 n x k, seconds,
    its description, the relative drop of f over its last 1000 iterations)."""
    import torch
    import paper_2607_24518_amd as sym

    t0 = time.time()
    S64 = sym.symnmf_build_S(ctx, X, dtype=sym.S_FP64, **build)
    eta = math.sqrt(S64.desc.mean / k)
    best_run = None
    for plan in plans:
        W = H0.double().clone()
        best, hist = math.inf, []
        for name, iters in plan:
            st = sym.symnmf_state_create(ctx, S64, k, variant_params("fp64-" + name, eta), W)
            for t in range(iters):
                s = sym.symnmf_step(ctx, S64, st, want_stats=(t % 10 == 0 or t == iters - 1))
                if s is not None:
                    best = min(best, s.f)
                    hist.append(s.f)
                    if t % 1000 == 0:
                        log(f"FP64 reference {name} t={t} f={s.f:.12e} kkt={s.kkt:.3e}")
            sym.symnmf_state_read(ctx, st, 0, W)
            del st
        f_last = sym.symnmf_objective(ctx, S64, W, k)[0]
        drop = (hist[-101] - hist[-1]) / hist[-1] if len(hist) > 100 else float("nan")
        desc = " then ".join(f"{name} x {iters}" for name, iters in plan)
        log(f"FP64 reference [{desc}]: last f={f_last:.12e}, drop over the last 1000 iterations {drop:.2e}")
        if best_run is None or f_last < best_run[0]:
            best_run = (f_last, min(best, f_last), W.float().contiguous(), desc, drop)
        del W
    del S64
    torch.cuda.empty_cache()
    return best_run[0], best_run[1], best_run[2], time.time() - t0, best_run[3], best_run[4]


def time_to_tolerance(args):
    """Time to (f(H_t) - f_ref) / f_ref <= tol for several variants (storage,
    method) of the same instance and initial H0.

    f(H_t) is the objective on the FP32-stored S (MFMA products, FP64 sums
    across chunks) whatever S the variant iterates on.  f_ref: the committed
    FP64 oracle reference of the workload if there is one (the device repeats
    the oracle's FP64 ADMM run from the same H0 and reports how close it
    lands), else the last objective of a device FP64 ADMM run of
    --ttt-ref-iters iterations.  The reference factor of the subspace errors
    is that device FP64 run's last iterate.  Every variant's iterates are
    kept in HBM and judged after its timed run; the time of iterate H_t runs
    from the start of its initialisation to the copy of H_t (HIP events on
    the solver stream), with every check-time rule of the method applied.
    """
    import numpy as np
    import torch
    import paper_2607_24518_amd as sym

    dev = torch.device("cuda:0")
    n, k = args.n, args.k
    Xh, kind = ttt_instance(args)
    X = Xh.to(dev)
    del Xh
    ctx = sym.symnmf_create(0)
    build = dict(kind=kind, q=0.05, lower_tail=1, fp8_panel_rows=256)
    stores = {"fp32": sym.symnmf_build_S(ctx, X, dtype=sym.S_FP32, **build)}
    variants = [v for v in args.ttt_variants.split(",") if v]
    S32 = stores["fp32"]
    ref = committed_reference(kind, n, args.T, args.groups, k, args.seed)
    mean = ref["mean"] if ref else None
    H0 = torch.empty(n, k, device=dev)
    init_factor(ctx, S32, k, 0, H0, mean)
    if ref:
        plans = [[(f"admm{ref['rho']:g}", ref["iterations"])]]
    else:
        plans = [[(st.split(":")[0], int(st.split(":")[1])) for st in pl.split("+")]
                 for pl in args.ttt_ref_plans.split(",")]
    if args.ttt_ref_load:
        # the device FP64 reference of an earlier run of the same workload and plans
        z = np.load(args.ttt_ref_load)
        assert str(z["plans"]) == repr(plans) and int(z["n"]) == n and int(z["k"]) == k, "another reference"
        f_dev, f_dev_best, ref_s, ref_desc, ref_drop = (float(z["f_dev"]), float(z["f_dev_best"]), float(z["seconds"]),
                                                        str(z["desc"]) + " (loaded)", float(z["drop"]))
        Wref = torch.from_numpy(z["W"]).to(dev)
    else:
        f_dev, f_dev_best, Wref, ref_s, ref_desc, ref_drop = fp64_reference(ctx, X, kind, k, H0, build, plans)
        if args.ttt_ref_save:
            np.savez(args.ttt_ref_save, f_dev=f_dev, f_dev_best=f_dev_best, W=Wref.cpu().numpy(), seconds=ref_s,
                     desc=ref_desc, drop=ref_drop, plans=repr(plans), n=n, k=k)
    if ref:
        f_ref = ref["f_ref"]
        results = {"f_ref": f_ref, "reference": f"FP64 oracle ADMM (rho {ref['rho']:g}) after {ref['iterations']} "
                                                f"iterations (tests/golden)",
                   "device_fp64_same_run": {"f": f_dev, "rel_to_f_ref": (f_dev - f_ref) / f_ref,
                                            "seconds": round(ref_s, 2)}}
    else:
        f_ref = f_dev_best
        results = {"f_ref": f_ref, "reference": f"device FP64 run from H0: {ref_desc} (the lowest of the plans "
                                                f"{args.ttt_ref_plans})",
                   "reference_last_1000_drop": ref_drop, "reference_seconds": round(ref_s, 2)}
    log(f"f_ref {f_ref:.12e}; device FP64 run {f_dev:.12e}")
    if args.ttt_ref_only:
        return results
    results.update(tol=args.ttt_tol, variants={})
    for v in variants:
        for dt in v.split("-")[0].split(">"):       # "fp8>bf16": the precision ladder
            if dt not in stores:
                stores[dt] = sym.symnmf_build_S(ctx, X, dtype=sym.DTYPES[dt], **build)
    del X
    eta = math.sqrt(S32.desc.mean / k)

    def objective_of(H):
        return sym.symnmf_objective(ctx, S32, H, k)[0]

    every = max(1, args.ttt_save_every)
    store = torch.empty(args.ttt_max // every, n, k, device=dev)
    for v in variants:
        ladder = v.split("-")[0].split(">")
        S = stores[ladder[0]]
        S_hi = stores[ladder[1]] if len(ladder) > 1 else None
        entry = ttt_run(ctx, S, k, variant_params(v, eta), lambda H: H.copy_(H0), objective_of,
                        f_ref, args.ttt_tol, args.ttt_max, every, store, S_hi, args.ttt_switch,
                        [float(x) for x in args.ttt_tols.split(",") if x])
        entry.pop("times")
        nsave = args.ttt_max // every
        entry["subspace_error_final"] = sym.symnmf_subspace_error(ctx, store[nsave - 1], Wref)
        entry["below_reference"] = entry["final_rel"] < 0.0
        if "iters" in entry:
            entry["subspace_error_at_tol"] = sym.symnmf_subspace_error(ctx, store[entry["iters"] // every - 1], Wref)
        results["variants"][v] = entry
        log(f"variant {v}: {entry}")
    return results


WARM_WIDTH, WARM_HIDDEN, WARM_OMEGA_SEED = 64, 256, 7


def warm_start_study(args):
    """Learned warm start against random initialisation and against the
    network-free start, with ADMM (rho 500) as the solver.

    Training: for every training seed the returns are generated, S (FP32) is
    built and solved by ADMM from the network-free start (stop rule or
    --warm-solve-iters), and the pair (canonical sketch coordinates, solved H)
    is kept on the device.  The network has the residual output
    A = max(C + z, 0) (C the coordinates, z its last layer), starts with a
    zero last layer - i.e. exactly at the network-free start - and is trained
    with the scale-free Gram loss.
    Evaluation on held-out seeds: f_ref is the lowest objective of two
    reference runs of --warm-ref-iters ADMM iterations (from random init and
    from the network-free start; FP32 state, FP64-accumulated objective -
    the FP64 state stops at k = 32); then the time to (f(H_t) - f_ref) / f_ref
    <= tol from (a) random init, (b) the network-free coordinates, (c) the
    network, each timed from the start of its initialisation (sketch,
    coordinates and network included).  A warm run that has not reached the
    tolerance within twice the random run's iterations falls back to the
    random run, and its time counts both.  Optionally the same on the
    n = 100000 |corr| workload (k = 32 model) against its committed FP64
    oracle reference.
    """
    import numpy as np
    import torch
    import paper_2607_24518_amd as sym
    import synth

    dev = torch.device("cuda:0")
    ctx = sym.symnmf_create(0)
    k, n = args.warm_k, args.warm_n
    W, HID = WARM_WIDTH, WARM_HIDDEN
    tols = [float(x) for x in args.ttt_tols.split(",") if x]

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

    def admm_params(S, max_iter=10 ** 9):
        return sym.symnmf_params_default(method=sym.ADMM, rho=500.0, max_iter=max_iter)

    out = {"family": args.warm_family, "n_train": args.warm_sizes or n, "n_heldout": n, "k": k, "T": args.warm_T,
           "groups": args.warm_groups, "width": W, "hidden": HID, "solver": "ADMM, rho 500",
           "network_output": "residual: max(C + z, 0), zero last layer at the start"}
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
        H0 = torch.empty(ni, k, device=dev)
        sym.symnmf_warm_start(ctx, S, None, W, k, WARM_OMEGA_SEED, H0)
        st = sym.symnmf_state_create(ctx, S, k, admm_params(S, args.warm_solve_iters), H0)
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
    params[HID * W + HID * HID: HID * W + HID * HID + k * HID].zero_()          # W3 = 0
    params[-k:].zero_()                                                         # b3 = 0
    net = sym.symnmf_mlp_create(ctx, W, HID, k, params)
    sym.symnmf_mlp_set_output(ctx, net, True)
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
    def evaluate(S, k_eval, model, label, seed, ref_steps, steps, f_ref_given=None, W_ref=None):
        nn = S.desc.n
        params = admm_params(S)

        def objective_of(H):
            return sym.symnmf_objective(ctx, S, H, k_eval)[0]

        inits = {
            "random": lambda H: sym.symnmf_init_H(ctx, S, k_eval, seed, H),
            "coords": lambda H: sym.symnmf_warm_start(ctx, S, None, W, k_eval, WARM_OMEGA_SEED, H),
            "mlp": lambda H: sym.symnmf_warm_start(ctx, S, model, W, k_eval, WARM_OMEGA_SEED, H),
        }
        res = {}
        if f_ref_given is None:
            refs = []
            for name in ("random", "coords"):
                Hr = torch.empty(nn, k_eval, device=dev)
                inits[name](Hr)
                st = sym.symnmf_state_create(ctx, S, k_eval, params, Hr)
                for _ in range(ref_steps):
                    sym.symnmf_step(ctx, S, st, want_stats=False)
                sym.symnmf_state_read(ctx, st, 0, Hr)
                del st
                refs.append(objective_of(Hr))
            f_ref = min(refs)
            res["reference_runs"] = {"random": refs[0], "coords": refs[1], "iterations": ref_steps}
        else:
            f_ref = f_ref_given
        res["f_ref"] = f_ref
        every = 2
        store = torch.empty(steps // every, nn, k_eval, device=dev)
        for name, init in inits.items():
            H0 = torch.empty(nn, k_eval, device=dev)
            init(H0)
            f0 = objective_of(H0)
            wt, _, w_init, _ = ttt_trace(ctx, S, k_eval, params, init, steps, every, store)
            e = ttt_scan(objective_of, store, steps // every, f_ref, args.ttt_tol, every, wt)
            e["init_seconds"] = round(w_init, 4)
            e["rel_initial"] = (f0 - f_ref) / f_ref
            if W_ref is not None:
                e["subspace_error_final"] = sym.symnmf_subspace_error(ctx, store[steps // every - 1], W_ref)
                if e.get("iters"):
                    e["subspace_error_at_tol"] = sym.symnmf_subspace_error(ctx, store[e["iters"] // every - 1],
                                                                           W_ref)
            e["at_tol"] = {}
            for t2 in tols:
                e2 = ttt_scan(objective_of, store, steps // every, f_ref, t2, every, wt)
                e["at_tol"][f"{t2:g}"] = {q: e2[q] for q in ("iters", "seconds") if q in e2} or None
            e["times"] = wt
            res[name] = e
        r = res["random"]
        r_it, r_s = r.get("iters"), r.get("seconds")
        for name in ("coords", "mlp"):
            e = res[name]
            if r_it is not None:
                if e.get("iters") is None or e["iters"] > 2 * r_it:
                    idx = min(2 * r_it // every, len(e["times"])) - 1
                    e["fallback"] = True
                    e["seconds_with_fallback"] = e["times"][idx] + r_s
                else:
                    e["fallback"] = False
                    e["seconds_with_fallback"] = e["seconds"]
                e["speedup_vs_random"] = round(r_s / e["seconds_with_fallback"], 3)
        for e in res.values():
            if isinstance(e, dict):
                e.pop("times", None)
        del store
        log(f"{label}: " + json.dumps(res))
        return res

    held = []
    for seed in range(args.warm_heldout0, args.warm_heldout0 + args.warm_heldout):
        X = returns(seed, n)
        S = sym.symnmf_build_S(ctx, X, dtype=sym.S_FP32)
        del X
        held.append(evaluate(S, k, net, f"held-out seed {seed}", seed, args.warm_ref_iters, args.warm_max))
        del S
    out["heldout"] = held
    for name in ("coords", "mlp"):
        sp = [h[name]["speedup_vs_random"] for h in held if "speedup_vs_random" in h[name]]
        if sp:
            out[f"{name}_speedup_median"] = float(np.median(sp))
            out[f"{name}_wins"] = int(sum(1 for v in sp if v > 1.0))
            out[f"{name}_fallbacks"] = int(sum(1 for h in held if h[name].get("fallback")))
        out[f"{name}_reached"] = int(sum(1 for h in held if h[name].get("iters") is not None))
    out["random_reached"] = int(sum(1 for h in held if h["random"].get("iters") is not None))
    both = [(h["coords"]["seconds"], h["mlp"]["seconds"]) for h in held
            if h["coords"].get("seconds") and h["mlp"].get("seconds")]
    if both:
        out["mlp_vs_coords_speedup_median"] = float(np.median([a / b for a, b in both]))
    if args.warm_c3:
        ref = committed_reference(0, 100000, 2500, 32, k, 0)
        X = synth.overlap_returns(0, T=2500, n=100000, groups=32, device="cpu").X.to(dev)
        S = sym.symnmf_build_S(ctx, X, dtype=sym.S_FP32)
        W_ref = None
        if ref:
            # reference factor of the subspace errors: the oracle's FP64 ADMM run
            # repeated on the device from the oracle's H0
            H0 = torch.empty(100000, k, device=dev)
            init_factor(ctx, S, k, 0, H0, ref["mean"])
            f_dev, _, W_ref, _, _, _ = fp64_reference(ctx, X, 0, k, H0, {"kind": 0},
                                                      [[(f"admm{ref['rho']:g}", ref["iterations"])]])
            out["c3_device_fp64_same_run_rel"] = (f_dev - ref["f_ref"]) / ref["f_ref"]
            del H0
        del X
        out["c3_abs_corr_n100000"] = evaluate(S, k, net, "n=100000 |corr|", 0, args.warm_ref_iters,
                                              args.warm_c3_max, ref["f_ref"] if ref else None, W_ref)
    return out


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
    return {"runs": runs}



def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--T", type=int, default=2500)
    ap.add_argument("--groups", type=int, default=32)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--ttt", action="store_true", help="time-to-tolerance comparison")
    ap.add_argument("--ttt-variants", default="fp32-admm,bf16-admm,fp8-admm,fp32,bf16,fp32-adam,bf16-adam")
    ap.add_argument("--ttt-kind", default="abs_corr", choices=["abs_corr", "tpdm"])
    ap.add_argument("--ttt-tol", type=float, default=1e-4)
    ap.add_argument("--ttt-switch", type=float, default=1e-5,
                    help="precision ladder (variants 'lo>hi-...'): move to the precise storage at the first check "
                         "whose stagnation measure (E_{t-delta} - E_t) / E_0 is below this")
    ap.add_argument("--ttt-max", type=int, default=6000)
    ap.add_argument("--ttt-save-every", type=int, default=2)
    ap.add_argument("--ttt-ref-plans", default="admm500:3000,admm50:3000",
                    help="device FP64 reference runs where no oracle reference is committed: comma-separated plans, "
                         "each a '+'-joined list of method:iterations stages")
    ap.add_argument("--ttt-tols", default="1e-2,1e-3", help="further tolerances scanned on the same runs")
    ap.add_argument("--ttt-ref-save", default="", help="save the device FP64 reference (f, factor) to this .npz")
    ap.add_argument("--ttt-ref-load", default="", help="use the device FP64 reference saved by --ttt-ref-save")
    ap.add_argument("--ttt-ref-only", action="store_true", help="stop after the reference run")
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
    ap.add_argument("--warm-ref-iters", type=int, default=3000, help="ADMM iterations of each reference run")
    ap.add_argument("--warm-epochs", type=int, default=40)
    ap.add_argument("--warm-lr", type=float, default=1e-3)
    ap.add_argument("--warm-wd", type=float, default=1e-4)
    ap.add_argument("--warm-max", type=int, default=1500, help="ADMM steps traced from each initialisation")
    ap.add_argument("--warm-c3", action="store_true", help="also evaluate on the n=100000 |corr| workload")
    ap.add_argument("--warm-c3-max", type=int, default=1500)
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
    args = ap.parse_args()
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
        base = res.get("variants", {}).get("fp32-admm", {}).get("seconds")
        for v in res.get("variants", {}).values():
            if base and v.get("seconds"):
                v["speedup_vs_fp32_admm"] = round(base / v["seconds"], 3)
        print(json.dumps({"metric": "time to relative objective tolerance", "unit": "s",
                          "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": f"{args.ttt_kind}_n{args.n}_k{args.k}_T{args.T}"}, **res}),
              flush=True)
        return
    ap.error("choose a study: --ttt, --warm, --kmeans or --logspace")


if __name__ == "__main__":
    main()
