"""Pins of the oracle's Adam, NAdam, Adan and dampened-MU rules (CPU).

Adam is checked against torch.optim.Adam (a library implementation of the
same rule), Adan against it too through the special case beta2 = 0 (no
difference term: Adan is then Adam with the second-moment decay beta3), and
all three against closed forms for a constant gradient, where the bias
correction must make every average equal the gradient.  The multiplicative
update is pinned by its exact fixed point at a planted factorisation, the
monotone objective of the dampened rule (He et al. 2011), and the scalar case
whose fixed point is sqrt(s)."""
import math

import numpy as np
import pytest
import torch

import oracle as o
import synth


def _torch_adam(x0, grads, lr, b1, b2, eps):
    p = torch.nn.Parameter(torch.tensor(x0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=lr, betas=(b1, b2), eps=eps)
    out = []
    for g in grads:
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        out.append(p.detach().numpy().copy())
    return out


def test_adam_matches_torch_adam():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((7, 5))
    grads = [rng.standard_normal((7, 5)) for _ in range(6)]
    ref = _torch_adam(x, grads, 0.01, 0.9, 0.999, 1e-8)
    m, v = np.zeros_like(x), np.zeros_like(x)
    for t, g in enumerate(grads, start=1):
        x, m, v = o.adam_update(x, m, v, g, t, 0.01, 1e-8, 0.9, 0.999, project=False)
        assert np.allclose(x, ref[t - 1], rtol=0, atol=1e-14)


def test_adan_without_difference_term_is_adam_with_beta3():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((6, 4))
    grads = [rng.standard_normal((6, 4)) for _ in range(6)]
    ref = _torch_adam(x, grads, 0.02, 0.8, 0.95, 1e-8)
    m, d, nv, gp = np.zeros_like(x), np.zeros_like(x), np.zeros_like(x), None
    for t, g in enumerate(grads, start=1):
        x, m, d, nv = o.adan_update(x, m, d, nv, g, gp, t, 0.02, 1e-8, 0.8, 0.0, 0.95, project=False)
        gp = g
        assert np.allclose(x, ref[t - 1], rtol=0, atol=1e-14)


@pytest.mark.parametrize("rule", ["adam", "nadam", "adan"])
def test_constant_gradient_closed_forms(rule):
    # with g constant every bias-corrected average equals g (m_t = (1 - b1^t) g)
    g = np.array([[0.3, -2.0], [1e-3, 5.0]])
    eta, eps, b1, b2, b3 = 0.1, 1e-9, 0.9, 0.99, 0.999
    x = np.zeros_like(g)
    m, v, d, nv, gp = np.zeros_like(g), np.zeros_like(g), np.zeros_like(g), np.zeros_like(g), None
    for t in range(1, 8):
        x_old = x
        if rule == "adan":
            x, m, d, nv = o.adan_update(x, m, d, nv, g, gp, t, eta, eps, b1, b2, b3, project=False)
            gp = g
            scale = 1.0
        else:
            x, m, v = o.adam_update(x, m, v, g, t, eta, eps, b1, b2, nesterov=rule == "nadam", project=False)
            scale = b1 + (1.0 - b1) / (1.0 - b1 ** t) if rule == "nadam" else 1.0
        assert np.allclose(x_old - x, eta * scale * g / (np.abs(g) + eps), rtol=1e-12, atol=0)


def test_adan_difference_term_on_a_two_step_sequence():
    # g1 then g2 (scalars): d_2 = (1 - b2)(g2 - g1), the step carries b2 d_2 / (1 - b2^2)
    g1, g2 = 1.0, 3.0
    eta, eps, b1, b2, b3 = 1.0, 0.0, 0.5, 0.5, 0.5
    x, m, d, nv = o.adan_update(np.zeros(1), np.zeros(1), np.zeros(1), np.zeros(1), np.array([g1]), None, 1,
                                eta, eps, b1, b2, b3, project=False)
    x2, *_ = o.adan_update(x, m, d, nv, np.array([g2]), np.array([g1]), 2, eta, eps, b1, b2, b3, project=False)
    # by hand: m2 = 0.25 g1 + 0.5 g2 = 1.75 -> /0.75; d2 = 0.5 * 2 = 1 -> 0.5 * 1 / 0.75;
    # n2 = 0.5 * 0.5 * 1 + 0.5 * (3 + 1)^2 = 8.25 -> /0.75 = 11
    expect = (1.75 / 0.75 + 0.5 / 0.75) / math.sqrt(11.0)
    assert float(x[0] - x2[0]) == pytest.approx(expect, rel=1e-14)


def test_mu_fixed_point_monotone_and_scalar_limit():
    # exact factorisation: SH = H (H^T H), so the rule returns H (up to eps)
    H = synth.planted_factor(0, 40, 4).numpy()
    S = H @ H.T
    H1 = o.mu_update(H, S @ H, H @ (H.T @ H), 1e-300)   # eps only guards all-zero rows
    assert np.allclose(H1, H, rtol=1e-12, atol=1e-15)
    # dampened rule: the objective never increases and H stays non-negative
    rng = np.random.default_rng(2)
    X = np.abs(rng.standard_normal((60, 20)))
    S = X @ X.T / 20
    H = rng.random((60, 5))
    f_prev = o.objective_trace(S, H)
    for _ in range(100):
        H = o.mu_update(H, S @ H, H @ (H.T @ H), 2.0 ** -23)
        f = o.objective_trace(S, H)
        assert f <= f_prev * (1 + 1e-12) and np.all(H >= 0)
        f_prev = f
    # n = k = 1: h <- h (1 + s h / (h^3 + eps)) / 2 converges to sqrt(s)
    h = np.array([[0.1]])
    for _ in range(200):
        h = o.mu_update(h, np.array([[9.0]]) @ h, h @ (h.T @ h), 0.0)
    assert float(h[0, 0]) == pytest.approx(3.0, rel=1e-12)


@pytest.mark.parametrize("method", [o.ADAM, o.NADAM, o.ADAN, o.MU])
def test_solver_runs_each_rule_and_decreases_the_objective(method):
    inst = synth.c1_instance(0, T=800, n=200, groups=4)
    S = o.abs_corr(inst.X.double().numpy())
    k = 4
    H0 = o.init_H(S.mean(), 200, k, 3)
    eta = 0.1 * math.sqrt(S.mean() / k)
    p = o.Params(method=method, eta=eta, eps=2.0 ** -23 if method == o.MU else 1e-10,
                 beta1=0.98 if method == o.ADAN else 0.9, beta2=0.92 if method == o.ADAN else 0.999)
    sol = o.Solver(S, k, p, H0)
    f0 = o.objective_trace(S, H0)
    stats = [sol.step() for _ in range(60)]
    assert stats[-1].f < 0.5 * f0 and np.all(sol.H >= 0)
    # the first step of Adam / NAdam / Adan moves every entry by eta (or
    # (1 + b1) eta for NAdam) in the direction of -g, then clamps
    if method != o.MU:
        g0 = o.gradient(S, H0)
        scale = 1.0 + p.beta1 if method == o.NADAM else 1.0
        sol2 = o.Solver(S, k, p, H0)
        sol2.step()
        expect = np.maximum(H0 - eta * scale * g0 / (np.abs(g0) + p.eps), 0.0)
        assert np.allclose(sol2.H, expect, rtol=1e-12, atol=1e-15)


def test_softplus_forms_keep_h_positive():
    inst = synth.c1_instance(0, T=800, n=150, groups=3)
    S = o.abs_corr(inst.X.double().numpy())
    H0 = o.init_H(S.mean(), 150, 3, 1)
    for method in (o.ADAM, o.NADAM, o.ADAN):
        sol = o.Solver(S, 3, o.Params(method=method, softplus=True, eta=0.05), H0)
        for _ in range(30):
            st = sol.step()
        assert np.all(sol.H > 0) and st.f < o.objective_trace(S, H0)
    with pytest.raises(ValueError):
        o.Solver(S, 3, o.Params(method=o.MU, softplus=True), H0)


def test_rebind_keeps_the_iteration_and_moves_it_to_the_new_matrix():
    """The precision ladder's move (Solver.rebind): onto a copy of S it changes
    nothing; onto another matrix S2 the next step is the AdaGrad rule with the
    carried accumulator and the gradient of S2, E is measured on S2, and the
    stagnation reference restarts (the first check after the move has none)."""
    inst = synth.c1_instance(2, T=600, n=120, groups=3)
    S = o.abs_corr(inst.X.double().numpy())
    rng = np.random.default_rng(4)
    S2 = S + 0.01 * np.abs(rng.standard_normal(S.shape))
    S2 = 0.5 * (S2 + S2.T)
    k = 3
    H0 = o.init_H(S.mean(), 120, k, 2)
    p = o.Params(eta=math.sqrt(S.mean() / k))
    a, b = o.Solver(S, k, p, H0), o.Solver(S, k, p, H0)
    for _ in range(20):
        a.step()
        b.step()
    a.rebind(S.copy())
    for _ in range(20):
        a.step()
        b.step()
    assert np.array_equal(a.H, b.H) and a.E0 == b.E0
    c = o.Solver(S, k, p, H0)
    for _ in range(20):
        c.step()
    H20, G20 = c.H.copy(), c.G.copy()
    c.E_prev = 0.3                                    # as if a check had run
    c.rebind(S2)
    assert c.E_prev is None and c.fro2 == pytest.approx(float((S2 * S2).sum()), rel=1e-15)
    st = c.step()
    g = 4.0 * (H20 @ (H20.T @ H20) - S2 @ H20)
    H_exp, _ = o.adagrad_update(H20, G20, g, p.eta, p.eps)
    assert np.allclose(c.H, H_exp, rtol=1e-13, atol=1e-15)
    assert st.E == pytest.approx(float(((S2 - H20 @ H20.T) ** 2).sum()) / float((S2 * S2).sum()), rel=1e-10)
    with pytest.raises(ValueError):
        c.rebind(S2[:10, :10])


def test_rebind_carries_the_admm_dual():
    """ADMM under the ladder's move: the dual U and the iterate W are carried,
    and the next step is the ADMM update (eqs. admm_H, admm_W, admm_U) of the
    new matrix from them."""
    inst = synth.c1_instance(2, T=600, n=120, groups=3)
    S = o.abs_corr(inst.X.double().numpy())
    rng = np.random.default_rng(6)
    S2 = S + 0.01 * np.abs(rng.standard_normal(S.shape))
    S2 = 0.5 * (S2 + S2.T)
    k = 8
    H0 = o.init_H(S.mean(), 120, k, 2)
    p = o.Params(method=o.ADMM, rho=50.0)              # an active dual: clipped entries by t = 40
    a = o.Solver(S, k, p, H0)
    for _ in range(40):
        a.step()
    W40, U40 = a.H.copy(), a.U.copy()
    assert np.count_nonzero(U40) > 100
    a.rebind(S2)
    a.step()
    W_exp, U_exp = o.admm_update(S2, W40, U40, 50.0)
    assert np.array_equal(a.H, W_exp) and np.array_equal(a.U, U_exp)
