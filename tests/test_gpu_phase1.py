"""Parity of the Adam, NAdam, Adan and dampened multiplicative (MU) update
modes of the fused update kernel (HIP, through the C ABI) with the FP64
oracle.

FP64 storage and state: whole trajectories (objective of every iterate to
1e-10, final H to 1e-9), projected and softplus forms.  FP32 state on FP32
storage: the objective after 300 iterations to 1e-5 relative.  Every stream
kind (FP32 k = 16/32/64, BF16, FP8): one step against the oracle's rule applied
to the stored S (2e-5 of the largest entry, the FP32 accumulation bound)."""
import math

import numpy as np
import pytest
import torch

import oracle as o
import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev, from_dev, stored_numpy, to_dev  # noqa: E402

RULES = {"adam": (sym.ADAM, o.ADAM), "nadam": (sym.NADAM, o.NADAM), "adan": (sym.ADAN, o.ADAN),
         "mu": (sym.MU, o.MU)}


def _betas(rule):
    return dict(beta1=0.98, beta2=0.92, beta3=0.99) if rule == "adan" else dict(beta1=0.9, beta2=0.999, beta3=0.99)


@pytest.fixture(scope="module")
def c1():
    X = synth.c1_instance(0).X.numpy()
    return X, o.abs_corr(X)


def _params(rule, S_mean, k, softplus=0):
    eta = 0.1 * math.sqrt(S_mean / k)
    eps = 2.0 ** -23 if rule == "mu" else 1e-10
    gm, om = RULES[rule]
    return (sym.symnmf_params_default(method=gm, softplus=softplus, eta=eta, eps=eps, max_iter=10 ** 9, **_betas(rule)),
            o.Params(method=om, softplus=bool(softplus), eta=eta, eps=eps, **_betas(rule)))


@pytest.mark.parametrize("rule,softplus", [("adam", 0), ("nadam", 0), ("adan", 0), ("mu", 0),
                                           ("adam", 1), ("nadam", 1), ("adan", 1)])
def test_fp64_trajectory_matches_oracle(c1, rule, softplus):
    X, Sref = c1
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(Sref, torch.float64), dtype=sym.S_FP64)
    k = 8
    H0 = o.init_H(Sref.mean(), 512, k, 4)
    gp, op = _params(rule, Sref.mean(), k, softplus)
    st = sym.symnmf_state_create(c, S, k, gp, to_dev(H0, torch.float64))
    solver = o.Solver(Sref, k, op, H0)
    for t in range(300):
        s = sym.symnmf_step(c, S, st)
        r = solver.step()
        assert s.f == pytest.approx(r.f, rel=1e-10), t
        assert s.kkt == pytest.approx(r.kkt, rel=1e-7, abs=1e-14), t
    H = torch.empty(512, k, dtype=torch.float64, device=dev())
    sym.symnmf_state_read(c, st, 0, H)
    assert np.max(np.abs(from_dev(H) - solver.H)) < 1e-9 * max(1.0, np.max(solver.H))
    assert r.f < o.objective_trace(Sref, H0)


@pytest.mark.parametrize("rule", ["adam", "adan"])
def test_state_buffers_after_two_steps(c1, rule):
    X, Sref = c1
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(Sref, torch.float64), dtype=sym.S_FP64)
    k = 8
    H0 = o.init_H(Sref.mean(), 512, k, 5)
    gp, op = _params(rule, Sref.mean(), k)
    st = sym.symnmf_state_create(c, S, k, gp, to_dev(H0, torch.float64))
    solver = o.Solver(Sref, k, op, H0)
    for _ in range(2):
        sym.symnmf_step(c, S, st)
        solver.step()
    buf = torch.empty(512, k, dtype=torch.float64, device=dev())
    want = {2: solver.nv if rule == "adan" else solver.G, 3: solver.m}
    if rule == "adan":
        want.update({7: solver.d, 8: solver.g_prev})
    for which, ref in want.items():
        sym.symnmf_state_read(c, st, which, buf)
        got = from_dev(buf)
        assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref)), which


@pytest.mark.parametrize("rule", ["adam", "nadam", "adan", "mu"])
def test_fp32_state_matches_oracle_objective(c1, rule):
    X, Sref = c1
    c = ctx()
    S = sym.symnmf_build_S(c, to_dev(X), dtype=sym.S_FP32)
    k = 8
    H0 = o.init_H(Sref.mean(), 512, k, 0, as_float32=True)
    gp, op = _params(rule, Sref.mean(), k)
    st = sym.symnmf_state_create(c, S, k, gp, to_dev(H0))
    for _ in range(300):
        sym.symnmf_step(c, S, st, want_stats=False)
    H = torch.empty(512, k, device=dev())
    sym.symnmf_state_read(c, st, 0, H)
    solver = o.Solver(Sref, k, op, H0)
    for _ in range(300):
        solver.step()
    S64 = sym.symnmf_S_load(c, to_dev(Sref, torch.float64), dtype=sym.S_FP64)
    f_gpu, _ = sym.symnmf_objective(c, S64, to_dev(from_dev(H), torch.float64), k)
    f_orc = o.objective_trace(Sref, solver.H)
    assert abs(f_gpu - f_orc) / f_orc <= 1e-5


@pytest.mark.parametrize("dtype,k", [("fp32", 16), ("fp32", 32), ("fp32", 64), ("bf16", 32), ("fp8", 32), ("fp32", 5)])
@pytest.mark.parametrize("rule", ["adam", "nadam", "adan", "mu"])
def test_single_step_every_stream_kind(c1, dtype, k, rule):
    X, Sref = c1
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(Sref, torch.float64), dtype=sym.DTYPES[dtype], fp8_panel_rows=128)
    Sq = stored_numpy(S)
    H0 = o.init_H(Sref.mean(), 512, k, 3, as_float32=True).astype(np.float64)
    gp, op = _params(rule, Sref.mean(), k)
    st = sym.symnmf_state_create(c, S, k, gp, to_dev(H0))
    sym.symnmf_step(c, S, st)
    H1 = torch.empty(512, k, device=dev())
    sym.symnmf_state_read(c, st, 0, H1)
    solver = o.Solver(Sq, k, op, H0)
    solver.step()
    scale = np.max(np.abs(solver.H))
    if rule == "mu":
        tol = 2e-5 * scale
    else:
        # the first Adam-type step is eta * g / (|g| + eps): entries whose
        # gradient is within FP32 accumulation error of zero may move either
        # way, so compare where |g| clears that error
        g = o.gradient(Sq, H0)
        clear = np.abs(g) > 2e-5 * np.max(np.abs(g))
        diff = np.abs(from_dev(H1) - solver.H)
        assert np.max(diff[clear]) <= 2e-5 * scale
        assert np.max(diff) <= 2.0 * gp.eta * (1.0 + gp.beta1) + 1e-6
        return
    assert np.max(np.abs(from_dev(H1) - solver.H)) <= tol


def test_rejects_mu_softplus_and_bad_betas(c1):
    _, Sref = c1
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(Sref, torch.float64))
    H0 = torch.full((512, 4), 0.05, device=dev())
    for kw in (dict(method=sym.MU, softplus=1), dict(method=sym.ADAM, beta1=1.0), dict(method=sym.ADAN, beta3=-0.1),
               dict(method=sym.NADAM, beta2=1.5), dict(method=10)):
        with pytest.raises(sym.SymnmfError) as e:
            sym.symnmf_state_create(c, S, 4, sym.symnmf_params_default(**kw), H0)
        assert e.value.code == sym.EINVAL


def test_mu_certifies_a_planted_factorisation():
    """The dampened multiplicative update driven to the stop rule on an exact
    S = H* H*^T: the same certified iteration as the oracle (1730 with
    tau_g_inf = 1e-5) and the planted subspace."""
    Hs = synth.planted_factor(3, 300, 4).numpy()
    Snp = Hs @ Hs.T
    H0 = o.init_H(Snp.mean(), 300, 4, 1)
    kw = dict(eps=1e-30, max_iter=20000, tau_g_inf=1e-5)
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(Snp, torch.float64), dtype=sym.S_FP64)
    st = sym.symnmf_state_create(c, S, 4, sym.symnmf_params_default(method=sym.MU, **kw), to_dev(H0, torch.float64))
    W = torch.empty(300, 4, dtype=torch.float64, device=dev())
    stats, conv = sym.symnmf_solve_to_tol(c, S, st, H_out=W)
    Ho, ost = o.Solver(Snp, 4, o.Params(method=o.MU, **kw), H0).solve()
    assert conv and ost.converged and stats.t == ost.t
    assert stats.E < 1e-5 and o.subspace_error(from_dev(W), Hs) < 1e-2
