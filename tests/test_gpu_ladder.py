"""The precision ladder: a solver state moved from one storage of S to
another (symnmf_state_rebind) and the laddered trace
(symnmf_solve_trace_ladder), through the C ABI.

A state rebound before its first step must follow, bit for bit, the
trajectory of a state created on the new storage (the launch shape and the
buffers follow the storage type, in both directions of the image size).  The
laddered trace must equal the same steps taken by hand: steps on the low
storage up to the switch check, a rebind, the rest on the high storage.
Moving from FP8 to FP32 storage must end below the objective (on the FP32 S)
that FP8 storage alone reaches."""
import math

import numpy as np
import pytest
import torch

import oracle as o
import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev, from_dev, stored_numpy, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def stores():
    X = synth.c1_instance(0, T=2000, n=700, groups=7).X
    c = ctx()
    out = {dt: sym.symnmf_build_S(c, to_dev(X.numpy()), dtype=sym.DTYPES[dt], fp8_panel_rows=128)
           for dt in ("fp32", "bf16", "fp8")}
    return out


def _params(S, k, **kw):
    kw.setdefault("eta", math.sqrt(S.desc.mean / k))
    return sym.symnmf_params_default(max_iter=10 ** 9, **kw)


def _run(c, S, st, steps):
    fs = [sym.symnmf_step(c, S, st).f for _ in range(steps)]
    H = torch.empty(S.desc.n, st.k, device=dev())
    sym.symnmf_state_read(c, st, 0, H)
    return fs, from_dev(H)


@pytest.mark.parametrize("k", [16, 32, 64, 8])
@pytest.mark.parametrize("src,dst", [("fp8", "fp32"), ("fp32", "fp8"), ("bf16", "fp32"), ("fp32", "bf16")])
def test_rebind_before_the_first_step_equals_a_fresh_state(stores, src, dst, k):
    c = ctx()
    n = stores["fp32"].desc.n
    H0 = torch.empty(n, k, device=dev())
    sym.symnmf_init_H(c, stores["fp32"], k, 3, H0)
    fresh = sym.symnmf_state_create(c, stores[dst], k, _params(stores["fp32"], k), H0)
    moved = sym.symnmf_state_create(c, stores[src], k, _params(stores["fp32"], k), H0)
    sym.symnmf_state_rebind(c, moved, stores[dst])
    f_a, H_a = _run(c, stores[dst], fresh, 25)
    f_b, H_b = _run(c, stores[dst], moved, 25)
    assert f_a == f_b
    assert np.array_equal(H_a, H_b)


@pytest.mark.parametrize("src,dst", [("fp32", "fp8"), ("fp8", "fp32")])
def test_rebind_block_svrg_equals_a_fresh_state(stores, src, dst):
    """Block-SVRG keeps a second image (of 2H for the doubly covered blocks):
    both images follow the storage type, sampled steps included."""
    c = ctx()
    n, k = stores["fp32"].desc.n, 32
    kw = dict(method=sym.BLOCK_SVRG, block_rows=256, snapshot_s=5, delta=10, phi0=0.5)
    H0 = torch.empty(n, k, device=dev())
    sym.symnmf_init_H(c, stores["fp32"], k, 7, H0)
    fresh = sym.symnmf_state_create(c, stores[dst], k, _params(stores["fp32"], k, **kw), H0)
    moved = sym.symnmf_state_create(c, stores[src], k, _params(stores["fp32"], k, **kw), H0)
    sym.symnmf_state_rebind(c, moved, stores[dst])
    f_a, H_a = _run(c, stores[dst], fresh, 23)
    f_b, H_b = _run(c, stores[dst], moved, 23)
    assert [x == y or (math.isnan(x) and math.isnan(y)) for x, y in zip(f_a, f_b)] == [True] * 23
    assert np.array_equal(H_a, H_b)


def test_rebind_rejects_another_matrix_or_precision(stores):
    c = ctx()
    X = synth.c1_instance(1, T=500, n=400, groups=4).X.numpy()
    other = sym.symnmf_build_S(c, to_dev(X), dtype=sym.S_FP32)
    H0 = torch.full((700, 8), 0.05, device=dev())
    st = sym.symnmf_state_create(c, stores["fp32"], 8, _params(stores["fp32"], 8), H0)
    with pytest.raises(sym.SymnmfError) as e:
        sym.symnmf_state_rebind(c, st, other)
    assert e.value.code == sym.EINVAL
    S64 = sym.symnmf_S_load(c, to_dev(o.abs_corr(synth.c1_instance(0, T=2000, n=700, groups=7).X.double().numpy()),
                                      torch.float64), dtype=sym.S_FP64)
    with pytest.raises(sym.SymnmfError) as e:
        sym.symnmf_state_rebind(c, st, S64)
    assert e.value.code == sym.EINVAL
    # the state still works on its own storage
    sym.symnmf_step(c, stores["fp32"], st)


@pytest.mark.parametrize("method", ["adagrad", "adam", "admm"])
def test_ladder_trace_equals_the_same_steps_by_hand(stores, method):
    """(Methods without check-time rules, so that plain steps are the same
    iteration as the trace.)"""
    c = ctx()
    S8, S32 = stores["fp8"], stores["fp32"]
    n, k, steps = S32.desc.n, 32, 120
    kw = {}
    if method == "adam":
        kw = dict(method=sym.ADAM, eta=0.1 * math.sqrt(S32.desc.mean / k))
    elif method == "admm":
        kw = dict(method=sym.ADMM, rho=500.0)
    H0 = torch.empty(n, k, device=dev())
    sym.symnmf_init_H(c, S32, k, 5, H0)
    st = sym.symnmf_state_create(c, S8, k, _params(S32, k, **kw), H0)
    store = torch.empty(steps, n, k, device=dev())
    # tau_switch = 1: the first check with a stagnation measure at t >= warmup (50)
    ms, cert, sw = sym.symnmf_solve_trace_ladder(c, S8, S32, st, steps, 1, store, 1.0)
    assert sw == 50 and len(ms) == steps and all(b >= a for a, b in zip(ms, ms[1:]))
    hand = sym.symnmf_state_create(c, S8, k, _params(S32, k, **kw), H0)
    Hh = torch.empty(n, k, device=dev())
    for t in range(steps):
        if t == sw + 1:
            sym.symnmf_state_rebind(c, hand, S32)
        sym.symnmf_step(c, S32 if t > sw else S8, hand)
        if t in (sw - 1, sw, sw + 1, steps - 1):
            sym.symnmf_state_read(c, hand, 0, Hh)
            assert torch.equal(Hh, store[t]), t


def test_ladder_ends_below_fp8_alone(stores):
    """On the FP32 S, FP8 storage alone stalls at the objective of the
    rounded problem; the ladder continues on the FP32 storage below it."""
    c = ctx()
    S8, S32 = stores["fp8"], stores["fp32"]
    n, k, steps = S32.desc.n, 32, 1500
    H0 = torch.empty(n, k, device=dev())
    sym.symnmf_init_H(c, S32, k, 1, H0)
    store = torch.empty(1, n, k, device=dev())
    st8 = sym.symnmf_state_create(c, S8, k, _params(S32, k), H0)
    sym.symnmf_solve_trace(c, S8, st8, steps, steps, store)
    f8 = sym.symnmf_objective(c, S32, store[0], k)[0]
    stl = sym.symnmf_state_create(c, S8, k, _params(S32, k), H0)
    _, _, sw = sym.symnmf_solve_trace_ladder(c, S8, S32, stl, steps, steps, store, 1e-4)
    fl = sym.symnmf_objective(c, S32, store[0], k)[0]
    assert 0 < sw < steps and fl < f8


@pytest.mark.parametrize("method", ["adagrad", "admm"])
@pytest.mark.parametrize("lo,hi", [("fp8", "fp32"), ("fp8", "bf16"), ("bf16", "fp32")])
def test_ladder_matches_the_oracle(lo, hi, method):
    """The laddered trace against the FP64 oracle taking the same iteration on
    the same stored matrices (decoded), moved by Solver.rebind after the
    switch check: the objective of the final iterate on the precise storage to
    1e-5 relative (the FP32 bar).  ADMM carries its dual U across the move."""
    X = synth.c1_instance(0).X.numpy()
    c = ctx()
    S_lo = sym.symnmf_build_S(c, to_dev(X), dtype=sym.DTYPES[lo], fp8_panel_rows=128)
    S_hi = sym.symnmf_build_S(c, to_dev(X), dtype=sym.DTYPES[hi], fp8_panel_rows=128)
    A_lo, A_hi = stored_numpy(S_lo), stored_numpy(S_hi)
    n, k, steps = 512, 8, 100
    H0 = o.init_H(A_hi.mean(), n, k, 0, as_float32=True)
    eta = math.sqrt(A_hi.mean() / k)
    gpu_kw, orc_kw = (dict(method=sym.ADMM, rho=500.0), dict(method=o.ADMM, rho=500.0)) if method == "admm" else ({}, {})
    st = sym.symnmf_state_create(c, S_lo, k, sym.symnmf_params_default(eta=eta, max_iter=10 ** 9, **gpu_kw),
                                 to_dev(H0))
    store = torch.empty(1, n, k, device=dev())
    _, _, sw = sym.symnmf_solve_trace_ladder(c, S_lo, S_hi, st, steps, steps, store, 1.0)
    assert sw == 50
    solver = o.Solver(A_lo, k, o.Params(eta=eta, **orc_kw), H0.astype(np.float64))
    for t in range(steps):
        if t == sw + 1:
            solver.rebind(A_hi)
        solver.step()
    f_gpu = o.objective_trace(A_hi, from_dev(store[0]).astype(np.float64))
    f_orc = o.objective_trace(A_hi, solver.H)
    assert abs(f_gpu - f_orc) / f_orc <= 1e-5
