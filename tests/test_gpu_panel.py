"""Solver states on a row panel of S - one GPU's share of a row-sharded S (the
paper's n = 10^6 runs shard S by rows; section "Computational Methodology").

A panel state updates the rows [row0, row0 + rows) of H and keeps the other
rows fixed; its gradient is rows [row0, row0 + rows) of 4 (H (H^T H) - S H)
with the Gram of the whole H (the fixed rows' share computed once).  The
oracle side is oracle.gradient_panel on the decoded stored panel, with the
AdaGrad rule applied to the panel rows only.
* small n (600), panels that start inside a storage tile (row0 = 130) or at
  an FP8 scale-panel boundary, FP32 / BF16 / FP8 storage, k = 16..64: three
  steps, every row of H compared;
* the real share shape: rows [12500, 25000) of the n = 10^6 |corr| S from
  T = 1000 returns (64 groups + market), BF16 storage (25 GB), k = 64: one
  step, sampled rows of the stored panel, the gradient and H_1 compared with
  the oracle row by row, rows outside the panel unchanged.
"""
import math

import numpy as np
import pytest
import torch

import oracle as o
import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev, from_dev, stored_numpy, to_dev  # noqa: E402


def _oracle_panel_steps(Sq, row0, H0, eta, eps, steps):
    H = H0.astype(np.float64).copy()
    rows = Sq.shape[0]
    G = np.zeros((rows, H.shape[1]))
    for _ in range(steps):
        g = o.gradient_panel(Sq, H, row0)
        Hp, G = o.adagrad_update(H[row0:row0 + rows], G, g, eta, eps)
        H[row0:row0 + rows] = Hp
    return H


@pytest.mark.parametrize("dtype,row0,rows,k", [("fp32", 130, 300, 64), ("bf16", 130, 300, 64),
                                               ("fp8", 128, 256, 32), ("fp32", 300, 300, 16),
                                               ("bf16", 0, 256, 32)])
def test_panel_state_steps_match_oracle(dtype, row0, rows, k):
    X = synth.c1_instance(0, T=700, n=600, groups=6).X.numpy()
    c = ctx()
    S = sym.symnmf_build_S(c, to_dev(X), dtype=sym.DTYPES[dtype], row0=row0, rows=rows, fp8_panel_rows=128)
    Sq = stored_numpy(S)
    assert Sq.shape == (rows, 600)
    ref_full = o.abs_corr(X)
    assert np.max(np.abs(Sq - ref_full[row0:row0 + rows])) < (2e-6 if dtype == "fp32" else 0.07)
    H0 = o.init_H(ref_full.mean(), 600, k, 5, as_float32=True)
    eta, eps = 0.5 * math.sqrt(ref_full.mean() / k), 1e-10
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(eta=eta, eps=eps), to_dev(H0))
    for _ in range(3):
        sym.symnmf_step(c, S, st, want_stats=False)
    H = torch.empty(600, k, device=dev())
    sym.symnmf_state_read(c, st, 0, H)
    H = from_dev(H)
    H_ref = _oracle_panel_steps(Sq, row0, H0, eta, eps, 3)
    out = np.ones(600, dtype=bool)
    out[row0:row0 + rows] = False
    assert np.array_equal(H[out], H0[out])                      # rows outside the panel stay fixed
    p = slice(row0, row0 + rows)
    # three AdaGrad steps in FP32: the first moves every entry by eta sign(g), so an
    # entry whose gradient is within FP32 noise of zero can go the other way
    close = np.abs(H[p] - H_ref[p]) <= 2e-4 * np.max(np.abs(H_ref[p]))
    assert close.mean() >= 0.999, close.mean()
    g = torch.empty(rows, k, device=dev())
    sym.symnmf_state_read(c, st, 6, g)                          # gradient of the last step, panel rows
    # the last step's gradient from the GPU's H_2 (read as the previous iterate)
    H2 = torch.empty(600, k, device=dev())
    sym.symnmf_state_read(c, st, 1, H2)
    g_ref = o.gradient_panel(Sq, from_dev(H2), row0)
    assert np.max(np.abs(from_dev(g) - g_ref)) <= 2e-5 * np.max(np.abs(g_ref))


def _stored_rows_tiled(S, rows):
    """Decoded stored rows (FP32 / BF16 tiled storage) gathered on the device."""
    d = S.desc
    E = {sym.S_FP32: 4, sym.S_BF16: 8}[d.dtype]
    W, NS = 4 * E, 256 // (4 * E)
    cols = np.arange(d.n)
    C, cc = np.divmod(cols, 256)
    s, rem = np.divmod(cc, W)
    lg, e = np.divmod(rem, E)
    if d.dtype == sym.S_FP32:
        flat = S.buf[: d.rows_pad * d.ld * 4].view(torch.float32)
    else:
        flat = S.buf[: d.rows_pad * d.ld * 2].view(torch.bfloat16)
    out = []
    for r in rows:
        R, rr = divmod(int(r) - d.row0, 256)
        wv, rg, lr = rr >> 6, (rr >> 4) & 3, rr & 15
        in_tile = (((wv * NS + s) * 4 + rg) * 64 + (lg * 16 + lr)) * E + e
        idx = (R * (d.ld // 256) + C) * 65536 + in_tile
        for j in (0, 1, 777, d.n - 1):
            assert idx[j] == sym.symnmf_S_offset(int(r) - d.row0, j, d.rows_pad, d.ld, d.dtype)
        out.append(flat[torch.from_numpy(idx).to(flat.device)].double().cpu().numpy())
    return np.stack(out)


def test_row_share_of_n_1e6_at_full_shape():
    n, T, groups, k = 1_000_000, 1000, 64, 64
    row0, rows = 12500, 12500
    X = synth.panel_returns(0, T=T, n=n, groups=groups).X
    c = ctx()
    S = sym.symnmf_build_S(c, X.to(dev()), dtype=sym.S_BF16, row0=row0, rows=rows)
    assert S.desc.rows == rows and S.desc.row0 == row0
    Xh = X.numpy()
    del X
    Z = o.standardise_columns(Xh)
    del Xh
    rng = np.random.default_rng(1)
    sample = np.unique(np.concatenate([[row0, row0 + 255, row0 + 256, row0 + rows - 1],
                                       row0 + rng.integers(0, rows, 12)]))
    ref_rows = np.stack([o.abs_corr_panel(Z, int(r), 1)[0] for r in sample])
    del Z
    got = _stored_rows_tiled(S, sample)
    # BF16 of the split-precision FP32 GEMM: within half an ulp of S plus the GEMM error
    ulp = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(ref_rows), 1e-30))) - 7)
    assert np.all(np.abs(got - ref_rows) <= 0.5 * ulp + 2e-6)
    H0 = synth.random_state(11, (n, k), 0.0, 0.03).numpy().astype(np.float64)
    eta, eps = 0.01, 1e-10
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(eta=eta, eps=eps), to_dev(H0))
    sym.symnmf_step(c, S, st, want_stats=False)
    g = torch.empty(rows, k, device=dev())
    H1 = torch.empty(n, k, device=dev())
    sym.symnmf_state_read(c, st, 6, g)
    sym.symnmf_state_read(c, st, 0, H1)
    g, H1 = from_dev(g), from_dev(H1)
    gram = H0.T @ H0
    for i, r in enumerate(sample):
        g_ref = 4.0 * (H0[r] @ gram - got[i] @ H0)
        assert np.max(np.abs(g[r - row0] - g_ref)) <= 2e-5 * np.max(np.abs(g_ref)), r
        h_ref, _ = o.adagrad_update(H0[r], np.zeros(k), g[r - row0], eta, eps)
        assert np.max(np.abs(H1[r] - h_ref)) <= 1e-6
    outside = np.concatenate([np.arange(0, row0, 997), np.arange(row0 + rows, n, 9973)])
    assert np.array_equal(H1[outside], H0[outside].astype(np.float32).astype(np.float64))
