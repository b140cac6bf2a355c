"""Trajectory parity at the benchmark's full size: |corr| n = 100000, k = 32,
T = 2500 (32 overlapping groups, market loading 0.4, returns generated on the
CPU with seed 0), in the launch configuration the benchmark times.

The FP64 oracle's first 30 iterations from the float32 counter-RNG H0 are in
tests/golden/abs_corr_n100000_k32_trajectory.json (written by
make_abs_corr_n100000_fixture.py, which calls only the oracle and the input
generator; S held as float32-rounded entries, every product FP64):
* projected AdaGrad on FP32 storage: f(H_t) of every iterate within 1e-5
  relative of the oracle's (the FP32 target at this size, eq. trace_loss),
  and the sampled rows of H_30;
* ADMM on FP64 storage with an FP64 state - the path that produces the
  time-to-tolerance reference factor: f(W_t) of every iterate to 1e-6
  relative and sampled rows of W_30 and U_30 to 1e-5 of max W.  The oracle's
  S is the float32 rounding of the FP64 S the library builds here, which
  alone moves f by |2 <S - H H^T, dS>| <= 2 sqrt(f) 2^-24 ||S||_F, about
  8e-7 relative on this workload;
* ADMM on FP32 storage: f(W_t) within 1e-4 relative.  ADMM carries the S.W
  products into W itself (eq. admm_H), so the rounding of the FP32 sums over
  10^5 terms (about sqrt(10^5 / 4) 2^-24 ~ 1e-5 per entry) moves every step
  by ~1e-6 in f, and the steps add up (4e-5 after 30 steps measured; an FP64
  run from H0 perturbed by 1e-7 stays within 2e-7, so the iteration does not
  amplify errors: the FP32 sums are the cause).  AdaGrad normalises its step
  by the accumulator and stays within 1e-6.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as o
import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev, from_dev, to_dev  # noqa: E402

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "abs_corr_n100000_k32_trajectory.json")


@pytest.fixture(scope="module")
def fx():
    with open(FIXTURE) as fh:
        d = json.load(fh)
    X = synth.overlap_returns(d["seed"], T=d["T"], n=d["n"], groups=d["groups"], device="cpu").X.numpy()
    ck = d["X_checksums"]
    assert [float(X[t, j]) for t, j in ((0, 0), (17, 4242), (2499, 99999), (1234, 56789))] == ck["samples"], \
        "the returns generator gives another panel on this machine: the fixture does not apply"
    Xd = X.astype(np.float64)
    assert float(Xd.sum()) == pytest.approx(ck["sum"], rel=1e-12)
    del Xd
    c = ctx()
    Xg = to_dev(X)
    del X
    H0 = o.init_H(d["mean"], d["n"], d["k"], d["init_seed"], as_float32=True)
    return d, c, Xg, H0


def _run(c, S, k, params, H0, steps, f64=False):
    st = sym.symnmf_state_create(c, S, k, params, to_dev(H0, torch.float64 if f64 else torch.float32))
    f = [sym.symnmf_step(c, S, st).f for _ in range(steps)]
    return st, np.array(f)


def test_fp32_adagrad_trajectory_at_full_size(fx):
    d, c, Xg, H0 = fx
    n, k, N = d["n"], d["k"], d["steps"]
    S = sym.symnmf_build_S(c, Xg, dtype=sym.S_FP32)
    assert S.desc.mean == pytest.approx(d["mean"], rel=1e-6)
    st, f = _run(c, S, k, sym.symnmf_params_default(eta=d["eta"]), H0, N)
    ref = np.array(d["adagrad"]["f"])
    rel = np.abs(f - ref) / ref
    print("FP32 AdaGrad, relative objective error per step: max %.3e at t=%d" % (rel.max(), rel.argmax()))
    assert rel.max() <= 1e-5
    H = torch.empty(n, k, device=dev())
    sym.symnmf_state_read(c, st, 0, H)
    rows = np.array(d["rows"])
    Hr = from_dev(H)[rows]
    Hr_ref = np.array(d["adagrad"]["H_rows"])
    dev_max = np.max(np.abs(Hr - Hr_ref)) / np.max(np.abs(Hr_ref))
    print("FP32 AdaGrad, sampled rows of H_30: max deviation %.3e of max |H|" % dev_max)
    assert dev_max <= 1e-3
    ADMM = sym.symnmf_params_default(method=sym.ADMM, rho=d["rho"])
    _, fa = _run(c, S, k, ADMM, H0, N)
    ref = np.array(d["admm"]["f"])
    rel = np.abs(fa - ref) / ref
    print("FP32 ADMM, relative objective error per step: max %.3e" % rel.max())
    assert rel.max() <= 1e-4


def test_fp64_admm_trajectory_at_full_size(fx):
    d, c, Xg, H0 = fx
    n, k, N = d["n"], d["k"], d["steps"]
    S = sym.symnmf_build_S(c, Xg, dtype=sym.S_FP64)
    assert S.desc.fro2 == pytest.approx(d["fro2"], rel=1e-6)
    st, f = _run(c, S, k, sym.symnmf_params_default(method=sym.ADMM, rho=d["rho"]), H0.astype(np.float64), N,
                 f64=True)
    ref = np.array(d["admm"]["f"])
    rel = np.abs(f - ref) / ref
    print("FP64 ADMM on FP64 S, relative objective error per step: max %.3e" % rel.max())
    assert rel.max() <= 1e-6
    W = torch.empty(n, k, dtype=torch.float64, device=dev())
    U = torch.empty(n, k, dtype=torch.float64, device=dev())
    sym.symnmf_state_read(c, st, 0, W)
    sym.symnmf_state_read(c, st, 3, U)
    rows = np.array(d["rows"])
    Wr, Ur = from_dev(W)[rows], from_dev(U)[rows]
    Wref, Uref = np.array(d["admm"]["H_rows"]), np.array(d["admm"]["U_rows"])
    print("FP64 ADMM rows: W %.3e, U %.3e of max |W|" % (np.max(np.abs(Wr - Wref)) / np.max(Wref),
                                                        np.max(np.abs(Ur - Uref)) / np.max(Wref)))
    assert np.max(np.abs(Wr - Wref)) <= 1e-5 * np.max(Wref)
    assert np.max(np.abs(Ur - Uref)) <= 1e-5 * np.max(Wref)


REFERENCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "abs_corr_n100000_k32_reference.json")


def test_fp64_admm_reference_run_at_full_size(fx, capsys):
    """The whole reference run of the time-to-tolerance results: 1500 FP64
    ADMM iterations (rho 500) from the oracle's H0 on FP64 storage, compared
    with the oracle's run (tests/golden/abs_corr_n100000_k32_reference.json,
    written by the oracle-only script beside it) at every 10th iterate it
    recorded, and its final objective f_ref.  Bound: the oracle solves the
    problem of the float32-rounded S, which moves f by at most
    2 sqrt(f) 2^-24 ||S||_F, about 8e-7 relative here; the runs are not
    chaotic (an FP64 run from H0 perturbed by 1e-7 stays within 2e-7)."""
    d, c, Xg, H0 = fx
    with open(REFERENCE) as fh:
        ref = json.load(fh)
    assert ref["complete"] and (ref["n"], ref["T"], ref["groups"], ref["k"], ref["seed"], ref["init_seed"]) == \
        (d["n"], d["T"], d["groups"], d["k"], d["seed"], d["init_seed"])
    assert ref["mean"] == d["mean"]
    n, k = d["n"], d["k"]
    S = sym.symnmf_build_S(c, Xg, dtype=sym.S_FP64)
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(method=sym.ADMM, rho=ref["rho"]),
                                 to_dev(H0, torch.float64))
    trace = {e["t"]: e["f"] for e in ref["trace"]}
    worst = 0.0
    for t in range(ref["iterations"]):
        s = sym.symnmf_step(c, S, st, want_stats=(t in trace or t == ref["iterations"] - 1))
        if t in trace:
            assert s.t == t
            worst = max(worst, abs(s.f - trace[t]) / trace[t])
        if t % 300 == 0:
            with capsys.disabled():
                print(f"[reference run] t={t} worst relative difference so far {worst:.2e}", flush=True)
    rel_final = abs(s.f - ref["f_ref"]) / ref["f_ref"]
    with capsys.disabled():
        print(f"[reference run] {len(trace)} recorded iterates: max relative difference {worst:.3e}; "
              f"final f {s.f:.12e} vs f_ref {ref['f_ref']:.12e} ({rel_final:.2e})", flush=True)
    assert worst <= 1e-6
    assert rel_final <= 1e-6


def test_fp32_admm_ends_at_the_oracle_reference(fx):
    """FP32 storage and state at the benchmark's size: 1500 ADMM iterations
    from the oracle's H0, and the objective of the final iterate within 1e-5
    of the oracle's f_ref - the FP32 bar of a relative objective.  The final
    iterate is judged by symnmf_objective (FP64 sums across chunks): the
    step's own statistic sums the FP32 S.W products of the update, and the
    trace form cancels to about 1.7e-5 relative there (eq. trace_loss; the
    oracle pins show the same cancellation of the trace form in FP32).  Step
    to step the FP32 trajectory drifts from the FP64 one (reading of eq.
    admm_H: 4e-5 after 30 steps), but both converge to the same minimum."""
    d, c, Xg, H0 = fx
    with open(REFERENCE) as fh:
        ref = json.load(fh)
    n, k, N = d["n"], d["k"], ref["iterations"]
    S = sym.symnmf_build_S(c, Xg, dtype=sym.S_FP32)
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(method=sym.ADMM, rho=ref["rho"]), to_dev(H0))
    for _ in range(N):
        sym.symnmf_step(c, S, st, want_stats=False)
    W = torch.empty(n, k, device=dev())
    sym.symnmf_state_read(c, st, 0, W)
    f, _ = sym.symnmf_objective(c, S, W, k)
    rel = (f - ref["f_ref"]) / ref["f_ref"]
    print(f"FP32 ADMM after {N} iterations: f {f:.12e}, f_ref {ref['f_ref']:.12e}, relative {rel:.2e}")
    assert abs(rel) <= 1e-5
