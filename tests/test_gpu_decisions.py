"""The check-time rules of the HIP solve loop against the oracle, on runs in
which they act: Piecewise AdaGrad resets that fire and then switch off
(appendix "Detailed Algorithm Descriptions", Piecewise AdaGrad), and
Block-SVRG AdaptGrow growing its coverage phi from 0.25 to 1 (same appendix,
Block-SVRG AdaptGrow).  FP64 storage and state, so both sides decide on the
same values up to summation order (1e-10 relative); the instances were chosen
so every decision clears its threshold by at least 0.8 %.  Each test also
asserts, on the oracle side, that the events took place."""
import math

import numpy as np
import pytest
import torch

import oracle as o
import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev, from_dev, to_dev  # noqa: E402


def _compare_checks(gpu_checks, oracle_history, delta):
    ochecks = [h for h in oracle_history if h.t % delta == 0]
    assert len(gpu_checks) == len(ochecks)
    for a, b in zip(gpu_checks, ochecks):
        assert a.t == b.t
        assert bool(a.reset_fired) == b.reset_fired, a.t
        assert bool(a.converged) == b.converged, a.t
        assert a.phi == b.phi, a.t
        assert a.E == pytest.approx(b.E, rel=1e-10), a.t
        assert a.kkt == pytest.approx(b.kkt, rel=1e-8), a.t
        if not math.isnan(b.stag):
            assert a.stag == pytest.approx(b.stag, rel=1e-6, abs=1e-12), a.t


def test_piecewise_resets_fire_and_disable_like_the_oracle():
    """520-instrument |corr| instance, k = 3: two resets (checks 310 and 340),
    then a refused one that turns resets off; 1500 iterations."""
    S_np = o.abs_corr(synth.c1_instance(2, T=600, n=520, groups=6).X.numpy())
    n, k = 520, 3
    H0 = o.init_H(S_np.mean(), n, k, 1)
    eta = 0.1 * math.sqrt(S_np.mean() / k)
    kw = dict(eta=eta, max_iter=1500, tau_stag=1e-3, tau_g_inf=1e-5)
    solver = o.Solver(S_np, k, o.Params(method=o.PIECEWISE_ADAGRAD, **kw), H0)
    Ho, ost = solver.solve()
    fired = [h.t for h in solver.history if h.reset_fired]
    assert fired == [310, 340] and not solver.pw_enabled       # the events this test is about
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(S_np, torch.float64), dtype=sym.S_FP64)
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(method=sym.PIECEWISE_ADAGRAD, **kw),
                                 to_dev(H0, torch.float64))
    H = torch.empty(n, k, dtype=torch.float64, device=dev())
    stats, conv = sym.symnmf_solve_to_tol(c, S, st, H_out=H)
    # not certified within max_iter: the library reports the last check (t = 1490)
    assert not conv and not ost.converged and stats.t == 1490
    _compare_checks(sym.symnmf_state_checks(c, st), solver.history, 10)
    ctl = sym.symnmf_state_control(c, st)
    assert ctl.pw_resets == 2 and ctl.pw_enabled == 0
    assert np.max(np.abs(from_dev(H) - Ho)) < 1e-8 * np.max(Ho)


@pytest.mark.parametrize("indep,c_grow,grows,stop", [(1, 10.0, [(221, 0.5), (311, 1.0)], 490),
                                                      (0, 3.0, [(251, 0.5), (281, 1.0)], 440)])
def test_adaptgrow_phi_growth_matches_the_oracle(indep, c_grow, grows, stop):
    """1300-instrument |corr| instance, k = 8, 256-row blocks, phi0 = 0.25,
    s = 5: phi doubles twice at the oracle's checks (independent I, J or
    I = J), and the stop rule certifies the same iterate."""
    S_np = o.abs_corr(synth.c1_instance(2, T=600, n=1300, groups=8).X.numpy())
    n, k = 1300, 8
    H0 = o.init_H(S_np.mean(), n, k, 3)
    eta = 0.3 * math.sqrt(S_np.mean() / k)
    kw = dict(eta=eta, max_iter=800, tau_stag=6e-3, block_rows=256, snapshot_s=5, delta=10, seed=17, phi0=0.25,
              c_grow=c_grow)
    solver = o.Solver(S_np, k, o.Params(method=o.BLOCK_SVRG, independent_blocks=bool(indep), **kw), H0)
    Ho, ost = solver.solve()
    phis = [(h.t, h.phi) for h in solver.history]
    assert [phis[i] for i in range(1, len(phis)) if phis[i][1] != phis[i - 1][1]] == grows
    assert ost.converged and ost.t == stop
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(S_np, torch.float64), dtype=sym.S_FP64)
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(method=sym.BLOCK_SVRG, independent_blocks=indep,
                                                                     **kw),
                                 to_dev(H0, torch.float64))
    H = torch.empty(n, k, dtype=torch.float64, device=dev())
    stats, conv = sym.symnmf_solve_to_tol(c, S, st, H_out=H)
    assert conv and stats.t == stop
    _compare_checks(sym.symnmf_state_checks(c, st), solver.history, 10)
    assert sym.symnmf_state_control(c, st).phi == 1.0
    assert np.max(np.abs(from_dev(H) - Ho)) < 1e-8 * np.max(Ho)
