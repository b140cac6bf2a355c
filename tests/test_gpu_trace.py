"""symnmf_solve_trace against the other entry points: the kept iterates are the
ones symnmf_solve_to_tol reaches with the same rules (Piecewise resets and
Block-SVRG growth included, and asserted to happen), bit for bit, and the
stop-rule certification time agrees with the oracle's."""
import math

import numpy as np
import pytest
import torch

import oracle as o
import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev, from_dev, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def c1():
    X = synth.c1_instance(0).X.numpy()
    c = ctx()
    S = sym.symnmf_build_S(c, to_dev(X), dtype=sym.S_FP32)
    return c, S


@pytest.mark.parametrize("method", [sym.ADAGRAD, sym.PIECEWISE_ADAGRAD, sym.BLOCK_SVRG])
def test_trace_iterates_equal_solve_to_tol(c1, method):
    """tau_g_inf = 1e-12 keeps the stop rule from certifying (no early stop),
    tau_stag = 1e-4 lets stagnation be detected: a Piecewise reset fires
    (near t = 80, then resets switch off) and Block-SVRG grows phi from 0.25
    to 1 (near t = 150 and 190) inside the 300 traced iterations."""
    c, S = c1
    n, k = 512, 8
    eta = math.sqrt(S.desc.mean / k)
    kw = dict(method=method, eta=eta, tau_g_inf=1e-12, tau_stag=1e-4)
    if method == sym.BLOCK_SVRG:
        kw.update(block_rows=256, snapshot_s=10, delta=10, phi0=0.25)
    H0 = torch.empty(n, k, device=dev())
    sym.symnmf_init_H(c, S, k, 3, H0)
    steps, every = 300, 30
    store = torch.empty(steps // every, n, k, device=dev())
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(max_iter=10 ** 9, **kw), H0)
    ms, cert = sym.symnmf_solve_trace(c, S, st, steps, every, store)
    assert len(ms) == steps // every and all(b >= a for a, b in zip(ms, ms[1:]))
    ctl = sym.symnmf_state_control(c, st)
    if method == sym.PIECEWISE_ADAGRAD:
        assert ctl.pw_resets >= 1
        assert any(x.reset_fired for x in sym.symnmf_state_checks(c, st))
    if method == sym.BLOCK_SVRG:
        assert ctl.phi == 1.0
    for j in (0, 4, 9):
        t = (j + 1) * every
        st2 = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(max_iter=t, **kw), H0)
        H = torch.empty(n, k, device=dev())
        _, conv = sym.symnmf_solve_to_tol(c, S, st2, H_out=H)
        assert not conv
        assert torch.equal(H, store[j]), (method, t)


def test_trace_certification_matches_oracle_stop_rule():
    """The first certified check of the trace is the oracle's stop iteration
    (t = 1340 here; FP64 storage and state, so decisions are taken on the same
    values)."""
    X = synth.c1_instance(0).X.numpy()
    S_ref = o.abs_corr(o.standardise_columns(X))
    n, k = 512, 8
    eta = math.sqrt(S_ref.mean() / k)
    H0 = o.init_H(S_ref.mean(), n, k, 0, as_float32=True)
    _, res = o.Solver(S_ref, k, o.Params(eta=eta, tau_g_inf=1e-7, tau_E=0.2, max_iter=3000), H0).solve(max_iter=3000)
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(S_ref, torch.float64), dtype=sym.S_FP64)
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(eta=eta, tau_g_inf=1e-7, tau_E=0.2,
                                                               max_iter=10 ** 9),
                                 to_dev(H0, torch.float64))
    store = torch.empty(300, n, k, dtype=torch.float64, device=dev())
    _, cert = sym.symnmf_solve_trace(c, S, st, 3000, 10, store)
    assert res.converged and cert == res.t


def test_probes_copy_and_read():
    """The bandwidth probes: the copy reproduces its input; the read folds
    every 16-byte vector with XOR (all-zero input gives all-zero words)."""
    c = ctx()
    n = 1 << 20
    src = torch.arange(n, dtype=torch.float32, device=dev())
    dst = torch.empty_like(src)
    sym.symnmf_probe_copy(c, src, dst)
    assert torch.equal(src, dst)
    zeros = torch.zeros(n, dtype=torch.float32, device=dev())
    sink = torch.full((4096,), -1, dtype=torch.int32, device=dev())
    sym.symnmf_probe_read(c, zeros, sink)
    torch.cuda.synchronize()
    assert int(sink.abs().sum()) == 0
