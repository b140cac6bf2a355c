"""Pins of the warm-start oracle (CPU): finite differences of the network and
the Gram loss, the loss's permutation invariance and closed forms."""
import math

import numpy as np
import pytest
import scipy.stats

import oracle as o
import oracle.warmstart_oracle as w
import synth


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-6, 6, 101)
    assert np.allclose(w.gelu(x), x * scipy.stats.norm.cdf(x), rtol=1e-14, atol=1e-300)
    h = 1e-6
    assert np.allclose((w.gelu(x + h) - w.gelu(x - h)) / (2 * h), w.gelu_grad(x), rtol=1e-7, atol=1e-9)


def test_omega_is_standard_normal_and_deterministic():
    Om = w.omega(5, 4000, 64)
    assert Om.shape == (4000, 64)
    assert abs(Om.mean()) < 0.01 and abs(Om.std() - 1.0) < 0.01
    assert scipy.stats.kstest(Om.ravel()[:20000], "norm").pvalue > 1e-3
    assert np.array_equal(Om, w.omega(5, 4000, 64))


def test_gram_loss_is_permutation_invariant_and_matches_explicit_form():
    g = np.random.default_rng(0)
    A, B = g.random((50, 6)), g.random((50, 6))
    L, _ = w.gram_loss(A, B)
    explicit = ((A @ A.T - B @ B.T) ** 2).sum() / ((B.T @ B) ** 2).sum()
    assert L == pytest.approx(explicit, rel=1e-12)
    P = np.eye(6)[[3, 1, 5, 0, 2, 4]]
    assert w.gram_loss(A @ P, B)[0] == pytest.approx(L, rel=1e-12)
    assert w.gram_loss(A, B @ P)[0] == pytest.approx(L, rel=1e-12)
    assert w.gram_loss(B @ P, B)[0] == pytest.approx(0.0, abs=1e-14)


def test_scale_free_gram_loss_is_the_best_scalar_fit():
    g = np.random.default_rng(2)
    A, B = g.random((40, 5)), g.random((40, 5))
    L, dA = w.gram_cos_loss(A, B)
    # brute force over the scalar c of c A A^T
    cs = np.linspace(0.0, 3.0, 30001)
    M, N = A @ A.T, B @ B.T
    res = ((M * M).sum() * cs ** 2 - 2 * (M * N).sum() * cs + (N * N).sum()) / (N * N).sum()
    assert L == pytest.approx(res.min(), abs=1e-9)
    assert w.gram_cos_loss(3.7 * A, 0.2 * B)[0] == pytest.approx(L, rel=1e-12)
    assert w.gram_cos_loss(B[:, [2, 0, 1, 4, 3]], B)[0] == pytest.approx(0.0, abs=1e-14)
    h = 1e-6
    for idx in [(0, 0), (7, 3), (39, 4)]:
        Ap, Am = A.copy(), A.copy()
        Ap[idx] += h
        Am[idx] -= h
        fd = (w.gram_cos_loss(Ap, B)[0] - w.gram_cos_loss(Am, B)[0]) / (2 * h)
        assert fd == pytest.approx(dA[idx], rel=1e-6, abs=1e-12)


@pytest.mark.parametrize("residual", [False, True])
def test_network_and_loss_gradients_match_finite_differences(residual):
    g = np.random.default_rng(1)
    P = w.init_params(4, seed=3, width=8, hidden=16)
    X = g.normal(size=(20, 8))
    B = g.random((20, 4))

    def loss(P):
        A, _ = w.forward(P, X, residual)
        return w.gram_loss(A, B)[0]

    A, cache = w.forward(P, X, residual)
    if residual:   # no entry of C + z at the kink of max(., 0), where the derivative jumps
        assert np.min(np.abs(X[:, :4] + cache["z3"])) > 1e-4
        assert 0 < np.mean(A > 0) < 1
    _, dA = w.gram_loss(A, B)
    G = w.backward(P, cache, dA)
    h = 1e-6
    for name in P:
        flat = P[name].ravel()
        for idx in list(range(0, flat.size, max(1, flat.size // 7)))[:7]:
            Pp = {kk: vv.copy() for kk, vv in P.items()}
            Pm = {kk: vv.copy() for kk, vv in P.items()}
            Pp[name].ravel()[idx] += h
            Pm[name].ravel()[idx] -= h
            fd = (loss(Pp) - loss(Pm)) / (2 * h)
            assert fd == pytest.approx(G[name].ravel()[idx], rel=1e-5, abs=1e-9), (name, idx)


def test_adamw_first_step_closed_form():
    P = {"W1": np.array([[1.0, -2.0]]), "b1": np.array([0.5])}
    G = {"W1": np.array([[0.3, -0.1]]), "b1": np.array([2.0])}
    state = {}
    Q = w.adamw_step({k: v.copy() for k, v in P.items()}, G, state, 1, lr=0.01, wd=0.1, eps=1e-12)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> step lr * sign(g); decay lr * wd * W
    assert np.allclose(Q["W1"], P["W1"] * (1 - 0.001) - 0.01 * np.sign(G["W1"]), atol=1e-12)
    assert np.allclose(Q["b1"], P["b1"] - 0.01 * np.sign(G["b1"]), atol=1e-12)


def test_alpha_rescale_minimises_scaled_objective():
    Hs = synth.planted_factor(2, 80, 4).numpy()
    S = Hs @ Hs.T
    A = Hs * 0.37
    a = w.alpha_rescale(S, A)
    assert a == pytest.approx(1 / 0.37, rel=1e-10)
    f = lambda s: o.objective_explicit(S, s * A)
    assert f(a) <= min(f(a * 1.01), f(a * 0.99))


def test_spa_recovers_anchor_rows_of_a_separable_factor():
    Hs = synth.planted_factor(4, 200, 5).numpy()
    g = np.random.default_rng(0)
    Z = Hs @ g.normal(size=(5, 5))            # a separable matrix in a random basis
    idx = w.spa(Z, 5)
    assert sorted(idx.tolist()) == [0, 1, 2, 3, 4]    # the scaled unit rows of H*
    X, anchors = w.canonical_coordinates(Hs @ g.normal(size=(5, 64)), 5, width=8)
    # in the anchor basis the coordinates reproduce H* up to column scaling and permutation
    C = X[:, :5]
    assert o.subspace_error(C, Hs) < 1e-6          # FP64 cancellation floor ~2e-8
    assert sorted(anchors.tolist()) == [0, 1, 2, 3, 4]
    assert np.all(C > -1e-8)


def test_residual_network_with_zero_last_layer_is_the_network_free_start():
    """A = max(C + z, 0): with W3 = 0 and b3 = 0 the network returns the
    coordinates clipped at zero, the start without a network; the gradient
    then reaches W3 only through the rows and columns where C > 0."""
    g = np.random.default_rng(4)
    P = w.init_params(5, seed=2, width=8, hidden=16)
    P["W3"][:] = 0.0
    P["b3"][:] = 0.0
    X = g.normal(size=(30, 8))
    A, cache = w.forward(P, X, residual=True)
    assert np.array_equal(A, np.maximum(X[:, :5], 0.0))
    B = g.random((30, 5))
    _, dA = w.gram_loss(A, B)
    G = w.backward(P, cache, dA)
    mask = X[:, :5] > 0.0
    assert np.allclose(G["W3"], (dA * mask).T @ cache["a2"], rtol=1e-13, atol=1e-15)
    assert np.allclose(G["b3"], (dA * mask).sum(axis=0), rtol=1e-13, atol=1e-15)
