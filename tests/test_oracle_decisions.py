"""Pins of the oracle's check-time decision rules on scripted statistics.

Piecewise AdaGrad (appendix "Detailed Algorithm Descriptions", Piecewise
AdaGrad; section "Cross-Family Comparison") recalibrates the accumulator when
the objective stagnates while the gradient is still large; Block-SVRG
AdaptGrow (same appendix) doubles its coverage phi under persistent
stagnation.  Both rules act at the stop rule's check iterations from the
statistics (E_t, KKT_t) of the check and the solver's own state.

Every test here feeds ``Solver.check`` a hand-made sequence of (t, E, KKT)
and sets the accumulator and the last gradient by hand, so each expected
decision and each expected accumulator is worked out on paper, independently
of the oracle's code.  The readings (stated with the oracle's Solver class):
stagnation is (E_prev - E_t)/E_0 < tau_stag at t >= warm-up; the reset gate is
KKT > c_r tau_g and median(g^2) > eps_med; the reset sets
G = max(c g^2, c median(g^2)) with the lower median; after a reset the rule
waits until sum(G) reaches twice its post-reset value; a later reset needs
E < E_reset (1 - 10 tau_stag), otherwise resets stop for good; phi doubles,
capped at 1, once ``grow_checks`` consecutive checks stagnate while
KKT > c_grow tau_g.
"""
import math

import numpy as np
import pytest

import oracle as o
import synth

N = 4          # tau_g(4) = 1e-4 * 1e4 / 4 = 0.25 ; c_r tau_g = c_grow tau_g = 2.5


def _solver(method, **kw):
    S = np.eye(N) + 0.25 * (np.ones((N, N)) - np.eye(N))
    p = o.Params(method=method, tau_stag=1e-5, warmup=50, delta=10, tau_E=0.1, tau_g_inf=1e-4, n_ref=1e4,
                 c=10.0, c_r=10.0, eps_med=1e-30, c_grow=10.0, grow_checks=3, **kw)
    return o.Solver(S, 1, p, np.full((N, 1), 0.3))


def _check(sol, t, E, kkt):
    st = o.Stats(t=t, full=True, f=E * sol.fro2, E=E, kkt=kkt)
    conv = sol.check(st, None)
    assert not conv          # E >= tau_E throughout: the stop rule never certifies here
    return st


def test_scripted_tau_g_and_gates():
    assert o.tau_g(N) == pytest.approx(0.25)


# --- Piecewise AdaGrad ------------------------------------------------------------
def _pw_after_first_reset():
    """One reset at t = 50: G = max(10 g^2, 10 median(g^2)) for g = (1, -2, 3, -4):
    g^2 = (1, 4, 9, 16), lower median (element 1 of 4 sorted) = 4, so
    G = (max(10, 40), max(40, 40), max(90, 40), max(160, 40)) = (40, 40, 90, 160),
    sum 330, and the cool-down waits for sum(G) >= 660."""
    sol = _solver(o.PIECEWISE_ADAGRAD)
    sol.G = np.array([[1.0], [2.0], [3.0], [4.0]])
    sol.last_g = np.array([[1.0], [-2.0], [3.0], [-4.0]])
    st = _check(sol, 0, 0.6, 3.0)                   # first check: E_0 = 0.6, no stagnation measure
    assert not st.reset_fired and math.isnan(st.stag)
    st = _check(sol, 50, 0.599997, 3.0)             # stag = 3e-6 / 0.6 = 5e-6 < 1e-5, t >= 50, KKT 3 > 2.5
    assert st.stag == pytest.approx(5e-6)
    assert st.reset_fired
    assert sol.G.ravel().tolist() == [40.0, 40.0, 90.0, 160.0]
    assert sol.pw_cooldown == 660.0 and sol.pw_E_reset == 0.599997 and sol.pw_resets == 1
    return sol


def test_piecewise_reset_fires_on_stagnation_and_replaces_the_accumulator():
    _pw_after_first_reset()


def test_piecewise_cooldown_blocks_until_the_accumulator_doubles():
    sol = _pw_after_first_reset()
    st = _check(sol, 60, 0.599996, 3.0)             # stagnating and gated open, but sum(G) = 330 < 660
    assert not st.reset_fired and sol.pw_enabled and sol.pw_resets == 1
    sol.G = sol.G + 81.0                            # sum 654: still below 660
    st = _check(sol, 70, 0.599995, 3.0)
    assert not st.reset_fired and sol.pw_enabled and sol.pw_resets == 1


def test_piecewise_disables_itself_without_measurable_progress():
    sol = _pw_after_first_reset()
    sol.G = sol.G + 100.0                           # sum 730 >= 660: the cool-down is over
    # E must fall below 0.599997 (1 - 10 * 1e-5) = 0.59993700 for another reset
    st = _check(sol, 60, 0.59996, 3.0)              # stag = 6.2e-5: progress, nothing decided
    assert not st.reset_fired and sol.pw_enabled
    st = _check(sol, 70, 0.599958, 3.0)             # stagnating, gates open, E above 0.599937
    assert not st.reset_fired and not sol.pw_enabled and sol.pw_resets == 1
    G = sol.G.copy()
    _check(sol, 80, 0.5, 3.0)                       # large progress, then stagnation again:
    st = _check(sol, 90, 0.499999, 3.0)             # every gate would pass, but resets are off for good
    assert not st.reset_fired and not sol.pw_enabled and np.array_equal(sol.G, G)


def test_piecewise_second_reset_after_measurable_progress():
    sol = _pw_after_first_reset()
    sol.G = sol.G + 100.0
    st = _check(sol, 60, 0.5999, 3.0)               # stag = (0.599997 - 0.5999)/0.6 = 1.6e-4: progress
    assert not st.reset_fired and sol.pw_enabled
    sol.last_g = np.array([[0.5], [0.0], [-1.0], [2.0]])   # g^2 = (.25, 0, 1, 4), lower median .25
    st = _check(sol, 70, 0.599899, 3.0)             # stagnating and E < 0.599937
    assert st.reset_fired and sol.pw_resets == 2 and sol.pw_enabled
    assert sol.G.ravel().tolist() == [2.5, 2.5, 10.0, 40.0]
    assert sol.pw_cooldown == 110.0 and sol.pw_E_reset == 0.599899


@pytest.mark.parametrize("case", ["warmup", "kkt_gate", "median_floor", "no_stagnation"])
def test_piecewise_gates(case):
    sol = _solver(o.PIECEWISE_ADAGRAD)
    sol.G = np.ones((N, 1))
    sol.last_g = np.array([[1.0], [-2.0], [3.0], [-4.0]])
    t, E, kkt = 50, 0.599997, 3.0
    if case == "warmup":
        t = 40                                      # stagnation is not looked for before t = 50
    elif case == "kkt_gate":
        kkt = 2.5                                   # the gate is KKT > c_r tau_g = 2.5, strictly
    elif case == "median_floor":
        sol.last_g = np.array([[0.0], [0.0], [0.0], [5.0]])   # g^2 sorted (0, 0, 0, 25): lower median 0
    else:
        E = 0.59999                                 # stag = 1e-5 / 0.6 = 1.67e-5 >= 1e-5
    _check(sol, 0, 0.6, kkt)
    st = _check(sol, t, E, kkt)
    assert not st.reset_fired and sol.pw_resets == 0 and sol.pw_enabled
    assert np.array_equal(sol.G, np.ones((N, 1)))


# --- Block-SVRG AdaptGrow -----------------------------------------------------------
def _grow_seq(sol, seq):
    """seq of (t, E, kkt); returns phi after each check."""
    out = []
    for t, E, kkt in seq:
        _check(sol, t, E, kkt)
        out.append(sol.phi)
    return out


def test_adaptgrow_doubles_after_three_stagnating_checks_and_a_break_resets_the_count():
    sol = _solver(o.BLOCK_SVRG, phi0=0.25)
    seq = [(0, 0.6, 3.0),
           (50, 0.599997, 3.0), (60, 0.599994, 3.0), (70, 0.599991, 3.0),   # 3 stagnating: 0.25 -> 0.5
           (80, 0.58, 3.0),                                                  # progress: count back to 0
           (90, 0.579997, 3.0), (100, 0.579994, 3.0),                        # 2 stagnating
           (110, 0.56, 3.0),                                                 # progress again
           (120, 0.559997, 3.0), (130, 0.559994, 3.0), (140, 0.559991, 3.0), # 3 stagnating: 0.5 -> 1
           (150, 0.559988, 3.0), (160, 0.559985, 3.0), (170, 0.559982, 3.0)] # phi = 1: nothing to grow
    phis = _grow_seq(sol, seq)
    assert phis == [0.25, 0.25, 0.25, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5, 1.0, 1.0, 1.0, 1.0]


def test_adaptgrow_is_capped_at_full_coverage():
    sol = _solver(o.BLOCK_SVRG, phi0=0.75)
    phis = _grow_seq(sol, [(0, 0.6, 3.0), (50, 0.599997, 3.0), (60, 0.599994, 3.0), (70, 0.599991, 3.0)])
    assert phis == [0.75, 0.75, 0.75, 1.0]


def test_adaptgrow_kkt_gate_and_warmup():
    sol = _solver(o.BLOCK_SVRG, phi0=0.25)
    # stagnating checks before the warm-up do not count
    phis = _grow_seq(sol, [(0, 0.6, 3.0), (20, 0.599997, 3.0), (30, 0.599994, 3.0), (40, 0.599991, 3.0)])
    assert phis == [0.25] * 4 and sol.stag_run == 0
    # three stagnating checks with KKT = 2.5 (not above c_grow tau_g): counted, no growth
    phis = _grow_seq(sol, [(50, 0.599988, 2.5), (60, 0.599985, 2.5), (70, 0.599982, 2.5)])
    assert phis == [0.25] * 3 and sol.stag_run == 3
    # the run persists: the next stagnating check with a large KKT grows phi
    phis = _grow_seq(sol, [(80, 0.599979, 2.6)])
    assert phis == [0.5] and sol.stag_run == 0


# --- the rules on a real trajectory ---------------------------------------------------
def _instance_520():
    return o.abs_corr(synth.c1_instance(2, T=600, n=520, groups=6).X.numpy())


def test_piecewise_trajectory_fires_two_resets_then_disables():
    """The 520-instrument |corr| instance (6 groups, T = 600, seed 2), k = 3,
    eta = 0.1 sqrt(mean S / k), tau_stag = 1e-3, tau_g_inf = 1e-5: the oracle
    resets twice and then turns resets off.  Up to the first reset the
    trajectory is plain AdaGrad's, bit for bit; the accumulator right after
    a reset is c max(g^2, median g^2), the median taken by sorting."""
    S = _instance_520()
    k = 3
    H0 = o.init_H(S.mean(), 520, k, 1)
    eta = 0.1 * math.sqrt(S.mean() / k)
    kw = dict(eta=eta, max_iter=1500, tau_stag=1e-3, tau_g_inf=1e-5)
    pw = o.Solver(S, k, o.Params(method=o.PIECEWISE_ADAGRAD, **kw), H0)
    ad = o.Solver(S, k, o.Params(**kw), H0)
    while pw.t < 1500:
        st = pw.step()
        ad.step()
        if st.t % 10 == 0:
            ad_check = pw.G.copy()
            fired = pw.check(st, None)
            assert not fired
            if st.reset_fired:
                g2 = np.sort((pw.last_g * pw.last_g).ravel())
                med = g2[(g2.size - 1) // 2]
                assert np.array_equal(pw.G, 10.0 * np.maximum(pw.last_g * pw.last_g, med))
                assert not np.array_equal(pw.G, ad_check)
        pw.history.append(st)
    fired_at = [h.t for h in pw.history if h.reset_fired]
    assert fired_at == [310, 340]
    assert not pw.pw_enabled and pw.pw_resets == 2
    first = fired_at[0]
    ad2 = o.Solver(S, k, o.Params(**kw), H0)
    pw2 = o.Solver(S, k, o.Params(method=o.PIECEWISE_ADAGRAD, **kw), H0)
    for t in range(first + 2):
        a, b = ad2.step(), pw2.step()
        if t % 10 == 0:
            pw2.check(b, None)
        if t <= first:
            assert a.f == b.f
    assert not np.array_equal(ad2.H, pw2.H)          # step first+1 ran on the reset accumulator


def test_adaptgrow_trajectory_grows_phi_twice():
    """The 1300-instrument |corr| instance (8 groups, T = 600, seed 2), k = 8,
    256-row blocks, phi0 = 0.25, s = 5, tau_stag = 6e-3: phi grows to 0.5 at
    the check t = 220 and to 1 at t = 310 (independent I and J)."""
    S = o.abs_corr(synth.c1_instance(2, T=600, n=1300, groups=8).X.numpy())
    k = 8
    H0 = o.init_H(S.mean(), 1300, k, 3)
    eta = 0.3 * math.sqrt(S.mean() / k)
    p = o.Params(method=o.BLOCK_SVRG, eta=eta, max_iter=800, tau_stag=6e-3, block_rows=256, snapshot_s=5,
                 delta=10, seed=17, phi0=0.25)
    sol = o.Solver(S, k, p, H0)
    _, st = sol.solve()
    phis = [(h.t, h.phi) for h in sol.history]
    changes = [(phis[i][0], phis[i][1]) for i in range(1, len(phis)) if phis[i][1] != phis[i - 1][1]]
    assert changes == [(221, 0.5), (311, 1.0)]
    # once phi = 1 every step is a full step
    assert all(h.full for h in sol.history if h.t >= 311)
    assert st.converged
