"""GPU parity of the learned warm start against the FP64 warm-start oracle:
sketch, canonical coordinates, network forward (FP32 and BF16 weights), one
training step (loss, gradients, AdamW update) and the composed warm start.
Inputs are seeded (synth, numpy generators); every expected value comes from
the oracle."""
import math

import numpy as np
import pytest
import torch

import oracle as o
import oracle.warmstart_oracle as w
import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev, from_dev, to_dev  # noqa: E402

WIDTH, HIDDEN = 64, 256


def _flat(P):
    """The ABI's parameter order: W1, W2, W3, b1, b2, b3."""
    return np.concatenate([P[n].ravel() for n in ("W1", "W2", "W3", "b1", "b2", "b3")])


def _unflat(v, width, hidden, k):
    shapes = [("W1", (hidden, width)), ("W2", (hidden, hidden)), ("W3", (k, hidden)),
              ("b1", (hidden,)), ("b2", (hidden,)), ("b3", (k,))]
    out, off = {}, 0
    for name, shp in shapes:
        size = int(np.prod(shp))
        out[name] = v[off: off + size].reshape(shp)
        off += size
    return out


def _params32(k, seed, width=WIDTH, hidden=HIDDEN):
    """Seeded parameters rounded to float32 (the values both sides use)."""
    P = w.init_params(k, seed=seed, width=width, hidden=hidden)
    P["b1"] = np.random.default_rng(seed + 1).normal(scale=0.1, size=hidden)
    P["b3"] = np.random.default_rng(seed + 2).normal(scale=0.1, size=k)
    return {n: v.astype(np.float32).astype(np.float64) for n, v in P.items()}


@pytest.fixture(scope="module")
def corr600():
    X = synth.c1_instance(3, T=2000, n=600, groups=8).X.numpy()
    return o.abs_corr(X)


@pytest.mark.parametrize("dtype", ["fp32", "bf16", "fp8"])
def test_sketch_matches_oracle(corr600, dtype):
    S = corr600
    n = S.shape[0]
    c = ctx()
    Sd = sym.symnmf_S_load(c, to_dev(S, torch.float64), dtype=sym.DTYPES[dtype], fp8_panel_rows=256)
    Y = torch.empty(n, WIDTH, device=dev())
    sym.symnmf_sketch(c, Sd, 17, WIDTH, Y)
    Om = w.omega(17, n, WIDTH)
    Sq, _ = o.quantise(S, dtype, panel_rows=256)
    ref = Sq @ Om
    bound = np.abs(Sq) @ np.abs(Om)
    # FP32 products and sums over n = 600 terms (the H operand enters the BF16 and
    # FP8 kinds as three BF16 planes whose sum is exact to ~2^-24)
    err = np.abs(from_dev(Y) - ref)
    assert np.all(err <= 2e-5 * bound + 1e-6), float(np.max(err / (bound + 1e-30)))


def test_omega_definition_through_identity_sketch():
    """With S = I the sketch is Omega itself: Box-Muller values of the counter
    generator, checked against the oracle element by element."""
    n = 300
    c = ctx()
    Sd = sym.symnmf_S_load(c, to_dev(np.eye(n), torch.float64), dtype=sym.S_FP32)
    Y = torch.empty(n, WIDTH, device=dev())
    sym.symnmf_sketch(c, Sd, 5, WIDTH, Y)
    assert np.max(np.abs(from_dev(Y) - w.omega(5, n, WIDTH))) < 2e-6


def _sketch_input(S, k, seed):
    """A float32 sketch computed by the oracle (an input of both sides)."""
    return (S @ w.omega(seed, S.shape[0], WIDTH)).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("case", ["planted", "corr"])
def test_canonical_matches_oracle(corr600, case):
    if case == "planted":
        Hs = synth.planted_factor(6, 700, 7).numpy()
        S, k = Hs @ Hs.T, 7
    else:
        S, k = corr600, 8
    Y = _sketch_input(S, k, 9)
    Xr, anch_r = w.canonical_coordinates(Y, k, WIDTH)
    c = ctx()
    X = torch.empty(Y.shape[0], WIDTH, device=dev())
    anchors = torch.empty(k, dtype=torch.int64, device=dev())
    sym.symnmf_canonical(c, to_dev(Y), k, X, anchors)
    assert anchors.cpu().tolist() == anch_r.tolist()
    Xg = from_dev(X)
    assert np.all(Xg[:, k:] == 0.0)
    assert np.max(np.abs(Xg - Xr)) <= 1e-7 * max(1.0, np.max(np.abs(Xr)))
    # the anchor rows map to the unit rows
    assert np.max(np.abs(Xg[anch_r, :k] - np.eye(k))) < 1e-9


def test_canonical_rejects_rank_deficient_sketch():
    Y = np.zeros((200, WIDTH))
    Y[:, :3] = np.random.default_rng(0).random((200, 3))
    c = ctx()
    X = torch.empty(200, WIDTH, device=dev())
    with pytest.raises(sym.SymnmfError) as e:
        sym.symnmf_canonical(c, to_dev(Y), 5, X)
    assert e.value.code == sym.ENUMERIC


@pytest.mark.parametrize("k,m", [(16, 1000), (5, 333), (64, 130)])
@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("residual", [False, True])
def test_mlp_forward_matches_oracle(k, m, bf16, residual):
    P = _params32(k, seed=k)
    Xin = np.random.default_rng(m).normal(size=(m, WIDTH)).astype(np.float32).astype(np.float64)
    ref, _ = w.forward(w.bf16_weights(P) if bf16 else P, Xin, residual)
    c = ctx()
    net = sym.symnmf_mlp_create(c, WIDTH, HIDDEN, k, to_dev(_flat(P)))
    sym.symnmf_mlp_set_output(c, net, residual)
    A = torch.empty(m, k, device=dev())
    sym.symnmf_mlp_forward(c, net, to_dev(Xin), A, bf16_weights=bf16)
    # FP32 activations and sums over 256 terms: relative 1e-5 of the layer scale
    assert np.max(np.abs(from_dev(A) - ref)) <= 2e-5 * max(1.0, np.max(np.abs(ref)))


def test_mlp_init_matches_oracle():
    k = 12
    c = ctx()
    buf = torch.empty(sym.symnmf_mlp_param_count(WIDTH, HIDDEN, k), device=dev())
    sym.symnmf_mlp_init(c, WIDTH, HIDDEN, k, 3, buf)
    got = _unflat(from_dev(buf), WIDTH, HIDDEN, k)
    ref = w.init_params_counter(k, 3, WIDTH, HIDDEN)
    for name in ref:
        assert np.max(np.abs(got[name] - ref[name])) <= 1e-7 * max(1.0, np.max(np.abs(ref[name]))), name


@pytest.mark.parametrize("loss_kind,residual", [(0, False), (1, False), (1, True)])
def test_mlp_train_step_matches_oracle(loss_kind, residual):
    k, m = 8, 1500
    P = _params32(k, seed=4)
    g = np.random.default_rng(7)
    Xin = g.normal(size=(m, WIDTH)).astype(np.float32).astype(np.float64)
    B = g.random((m, k)).astype(np.float32).astype(np.float64)
    A, cache = w.forward(P, Xin, residual)
    if residual:   # the FP32 side takes the same side of max(., 0) wherever C + z is not within its noise
        assert np.mean(np.abs(Xin[:, :k] + cache["z3"]) < 1e-4) < 1e-3
    L_ref, dA = (w.gram_loss if loss_kind == 0 else w.gram_cos_loss)(A, B)
    G_ref = w.backward(P, cache, dA)
    lr, wd = 1e-3, 1e-2
    P_ref = w.adamw_step({n: v.copy() for n, v in P.items()}, G_ref, {}, 1, lr=lr, wd=wd, eps=1e-8)
    c = ctx()
    net = sym.symnmf_mlp_create(c, WIDTH, HIDDEN, k, to_dev(_flat(P)))
    sym.symnmf_mlp_set_output(c, net, residual)
    L = sym.symnmf_mlp_train_step(c, net, to_dev(Xin), to_dev(B), lr=lr, weight_decay=wd, eps=1e-8,
                                  loss_kind=loss_kind)
    assert L == pytest.approx(L_ref, rel=1e-5)
    buf = torch.empty(net.count, device=dev())
    G = _unflat(from_dev(sym.symnmf_mlp_read(c, net, "grad", buf)), WIDTH, HIDDEN, k)
    Pn = _unflat(from_dev(sym.symnmf_mlp_read(c, net, "params", buf)), WIDTH, HIDDEN, k)
    for name in G_ref:
        scale = np.max(np.abs(G_ref[name]))
        assert np.max(np.abs(G[name] - G_ref[name])) <= 1e-3 * scale, name
        # the first AdamW step moves each entry by about lr sign(g): compare where
        # the sign is decided well above the FP32 gradient error
        sure = np.abs(G_ref[name]) > 1e-2 * scale
        assert np.max(np.abs(Pn[name] - P_ref[name])[sure]) <= 1e-6, name
        assert np.max(np.abs(Pn[name] - P[name])) <= lr * (1 + wd * np.max(np.abs(P[name]))) * 1.001 + 1e-7


def test_mlp_training_fits_a_planted_target():
    """Property at any size: repeated steps on one instance drive the Gram loss down."""
    k, m = 6, 4000
    c = ctx()
    P = _params32(k, seed=1)
    g = np.random.default_rng(3)
    Xin = g.normal(size=(m, WIDTH))
    B = np.maximum(Xin[:, :k] @ g.normal(size=(k, k)), 0.0)
    net = sym.symnmf_mlp_create(c, WIDTH, HIDDEN, k, to_dev(_flat(P)))
    Xd, Bd = to_dev(Xin), to_dev(B)
    losses = [sym.symnmf_mlp_train_step(c, net, Xd, Bd, lr=1e-3) for _ in range(300)]
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])


@pytest.mark.parametrize("with_net,residual", [(False, False), (True, False), (True, True)])
def test_warm_start_matches_oracle(with_net, residual):
    Hs = synth.planted_factor(8, 700, 6).numpy()
    S = Hs @ Hs.T
    k = 6
    P = _params32(k, seed=11) if with_net else None
    if residual:                       # a small correction on top of the coordinates
        P["W3"] = (P["W3"] * 0.05).astype(np.float32).astype(np.float64)
    ref, _ = w.warm_start(S.astype(np.float32).astype(np.float64), k, 21, P, WIDTH, residual)
    c = ctx()
    Sd = sym.symnmf_S_load(c, to_dev(S, torch.float64), dtype=sym.S_FP32)
    net = sym.symnmf_mlp_create(c, WIDTH, HIDDEN, k, to_dev(_flat(P))) if with_net else None
    if net is not None:
        sym.symnmf_mlp_set_output(c, net, residual)
    H0 = torch.empty(700, k, device=dev())
    sym.symnmf_warm_start(c, Sd, net, WIDTH, k, 21, H0)
    # the GPU sketch is FP32 (relative ~1e-6), carried through the anchor solve
    assert np.max(np.abs(from_dev(H0) - ref)) <= 1e-4 * np.max(np.abs(ref))


def test_residual_network_with_zero_last_layer_is_the_network_free_start(corr600):
    """A residual network whose last layer (weights and bias) is zero adds
    nothing to the coordinates: the warm start is the network-free one, bit
    for bit (the starting point of every training run)."""
    k = 8
    c = ctx()
    P = _params32(k, seed=4)
    P["W3"] = np.zeros_like(P["W3"])
    P["b3"] = np.zeros_like(P["b3"])
    net = sym.symnmf_mlp_create(c, WIDTH, HIDDEN, k, to_dev(_flat(P)))
    sym.symnmf_mlp_set_output(c, net, True)
    S = sym.symnmf_S_load(c, to_dev(corr600, torch.float64), dtype=sym.S_FP32)
    Ha, Hb = torch.empty(600, k, device=dev()), torch.empty(600, k, device=dev())
    sym.symnmf_warm_start(c, S, net, WIDTH, k, 9, Ha)
    sym.symnmf_warm_start(c, S, None, WIDTH, k, 9, Hb)
    assert torch.equal(Ha, Hb)


def test_warm_start_without_network_recovers_planted_subspace():
    """On an exactly separable S = H* H*^T the network-free coordinates are
    H* up to column scaling: the subspace error is at rounding level."""
    Hs = synth.planted_factor(2, 900, 8).numpy()
    c = ctx()
    Sd = sym.symnmf_S_load(c, to_dev(Hs @ Hs.T, torch.float64), dtype=sym.S_FP32)
    H0 = torch.empty(900, 8, device=dev())
    sym.symnmf_warm_start(c, Sd, None, WIDTH, 8, 3, H0)
    assert o.subspace_error(from_dev(H0), Hs) < 1e-4


def test_subspace_error_matches_oracle():
    g = np.random.default_rng(5)
    n, k = 1000, 10
    A = g.random((n, k)).astype(np.float32).astype(np.float64)
    B = g.random((n, k)).astype(np.float32).astype(np.float64)
    c = ctx()
    got = sym.symnmf_subspace_error(c, to_dev(A), to_dev(B))
    assert got == pytest.approx(o.subspace_error(A, B), abs=1e-9)
    # same span (B = A R): zero up to the cancellation floor of the formula
    R = g.normal(size=(k, k))
    AR = (A @ R).astype(np.float32).astype(np.float64)
    assert sym.symnmf_subspace_error(c, to_dev(A), to_dev(AR)) < 1e-5
    # orthogonal spans: 1
    E = np.zeros((n, 4))
    F = np.zeros((n, 4))
    E[np.arange(4), np.arange(4)] = 1.0
    F[4 + np.arange(4), np.arange(4)] = 1.0
    assert sym.symnmf_subspace_error(c, to_dev(E), to_dev(F)) == pytest.approx(1.0, abs=1e-12)
