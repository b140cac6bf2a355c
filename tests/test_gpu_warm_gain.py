"""What the trained network gains: a small end-to-end run of the learned warm
start at test size.  A network is trained on the solver's own factorizations
of generated instances and compared, on a held-out instance, with random
initialisation by the iterations needed to reach the random run's final
objective within 1e-4 (kept iterates judged with the FP64-accumulating
objective).  The network-free coordinates are reported beside it."""
import math

import pytest
import torch

import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev  # noqa: E402

W, HID, K, N, T, GROUPS = 64, 256, 16, 2048, 1000, 16


def _S(c, seed):
    X = synth.panel_returns(seed, T=T, n=N, groups=GROUPS, block=65536, device=dev()).X
    return sym.symnmf_build_S(c, X, dtype=sym.S_FP32)


def _iters_to(c, S, H0, steps, f_ref, tol=1e-4):
    """Iterations from H0 until f(H_t) <= f_ref (1 + tol), or None."""
    eta = math.sqrt(S.desc.mean / K)
    st = sym.symnmf_state_create(c, S, K, sym.symnmf_params_default(eta=eta, max_iter=10 ** 9), H0)
    store = torch.empty(steps // 10, N, K, device=dev())
    sym.symnmf_solve_trace(c, S, st, steps, 10, store)
    for j in range(store.shape[0]):
        f, _ = sym.symnmf_objective(c, S, store[j], K)
        if (f - f_ref) / f_ref <= tol:
            return (j + 1) * 10
    return None


def test_trained_network_beats_random_initialisation():
    c = ctx()
    # training pairs: canonical coordinates and the solver's factorization
    pairs = []
    for seed in range(100, 124):
        S = _S(c, seed)
        H0 = torch.empty(N, K, device=dev())
        sym.symnmf_warm_start(c, S, None, W, K, 7, H0)
        eta = math.sqrt(S.desc.mean / K)
        st = sym.symnmf_state_create(c, S, K, sym.symnmf_params_default(eta=eta, max_iter=1000), H0)
        Hs = torch.empty(N, K, device=dev())
        sym.symnmf_solve_to_tol(c, S, st, H_out=Hs)
        Y = torch.empty(N, W, device=dev())
        sym.symnmf_sketch(c, S, 7, W, Y)
        Xc = torch.empty(N, W, device=dev())
        sym.symnmf_canonical(c, Y, K, Xc)
        pairs.append((Xc, Hs))
    params = torch.empty(sym.symnmf_mlp_param_count(W, HID, K), device=dev())
    sym.symnmf_mlp_init(c, W, HID, K, 1, params)
    net = sym.symnmf_mlp_create(c, W, HID, K, params)
    losses = []
    for ep in range(15):
        for Xc, Hs in pairs:
            losses.append(sym.symnmf_mlp_train_step(c, net, Xc, Hs, lr=1e-3, loss_kind=1))
    first = sum(losses[: len(pairs)]) / len(pairs)
    last = sum(losses[-len(pairs):]) / len(pairs)
    assert last < first
    # held-out instance: the random run defines f_ref
    S = _S(c, 999)
    Hr = torch.empty(N, K, device=dev())
    sym.symnmf_init_H(c, S, K, 5, Hr)
    eta = math.sqrt(S.desc.mean / K)
    st = sym.symnmf_state_create(c, S, K, sym.symnmf_params_default(eta=eta, max_iter=4000), Hr)
    Hf = torch.empty(N, K, device=dev())
    stats, _ = sym.symnmf_solve_to_tol(c, S, st, H_out=Hf)
    f_ref, _ = sym.symnmf_objective(c, S, Hf, K)
    it_random = _iters_to(c, S, Hr, int(stats.t) + 10, f_ref)
    Hm = torch.empty(N, K, device=dev())
    sym.symnmf_warm_start(c, S, net, W, K, 7, Hm)
    it_mlp = _iters_to(c, S, Hm, 4000, f_ref)
    Hc = torch.empty(N, K, device=dev())
    sym.symnmf_warm_start(c, S, None, W, K, 7, Hc)
    it_coords = _iters_to(c, S, Hc, 4000, f_ref)
    print(f"[warm gain] iterations to f_ref(1+1e-4): random {it_random}, network {it_mlp}, "
          f"coordinates {it_coords}; loss {first:.4f} -> {last:.4f}", flush=True)
    assert it_random is not None and it_mlp is not None
    assert it_mlp < it_random
