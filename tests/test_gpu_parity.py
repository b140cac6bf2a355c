"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Sizes span several 256-row tiles with a ragged tail.  Tolerances:
* FP64 storage / FP64 state: 1e-10 relative (only summation order differs).
* FP32 and the mixed paths: FP32 accumulation of S.H over n terms gives
  relative errors of order sqrt(n) * 2^-24 ~ 1e-6; the gradient is checked at
  2e-5 of its largest entry and the objective at 1e-5 relative, the bound the
  FP32 path is held to.
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


def _corr_instance(n=600, T=700, groups=6, seed=0):
    inst = synth.c1_instance(seed, T=T, n=n, groups=groups)
    return inst.X.numpy()


@pytest.fixture(scope="module")
def X600():
    return _corr_instance()


@pytest.fixture(scope="module")
def S600(X600):
    return o.abs_corr(X600)


def test_fp8_conversion_instruction_matches_e4m3():
    assert sym.symnmf_selfcheck_fp8(ctx()) == 0


# --- S construction ----------------------------------------------------------
@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16", "fp8"])
def test_build_abs_corr(X600, S600, dtype):
    c = ctx()
    S = sym.symnmf_build_S(c, to_dev(X600), kind=sym.ABS_CORR, dtype=sym.DTYPES[dtype], fp8_panel_rows=128)
    M = stored_numpy(S)
    ref = S600
    if dtype == "fp64":
        assert np.max(np.abs(M - ref)) < 1e-13
    elif dtype == "fp32":
        assert np.max(np.abs(M - ref)) < 2e-6
    elif dtype == "bf16":
        # stored = RNE_bf16 of the FP32-accumulated value, which is within 2e-6 of S
        q = o.to_bf16(ref)
        ulp = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(ref), 1e-30))) - 7)
        assert np.all(np.abs(M - ref) <= 0.5 * ulp + 2e-6)
        assert np.all(np.abs(M - q) <= ulp + 4e-6)
        assert np.mean(M == q) > 0.99
    else:
        assert np.all(np.diag(M) == 1.0)
        off = ~np.eye(600, dtype=bool)
        assert np.all(np.abs(M - ref)[off] <= 2.0 ** -4 * np.abs(ref)[off] + 2.0 ** -9 / 448 * 1.2 + 1e-7)
    assert S.desc.fro2 == pytest.approx((ref * ref).sum(), rel=1e-6 if dtype != "fp64" else 1e-12)
    assert S.desc.fro2_stored == pytest.approx((M * M).sum(), rel=1e-9)
    assert S.desc.mean == pytest.approx(ref.mean(), rel=1e-6)
    # upper tiles are computed and stored twice (FP8 rows carry their own panel scale)
    assert np.all(M == M.T) or dtype == "fp8"


@pytest.mark.parametrize("n", [1, 2, 127, 128, 129, 257, 384])
@pytest.mark.parametrize("dtype", ["fp32", "bf16", "fp8"])
def test_build_tile_boundaries(n, dtype):
    """Sizes on both sides of the 128-row output tiles and the 256-row storage
    tiles: the mirrored blocks land where the oracle's entries are, the
    padding stays zero, and (FP8, 100-row scale panels that straddle the
    tiles) every panel's largest off-diagonal entry is coded as 448, which
    only holds if the panel maxima covered the panel's rows in every tile
    and every mirrored block."""
    inst = synth.c1_instance(5, T=300, n=n, groups=1 if n < 8 else 4)
    X = inst.X.numpy()
    ref = o.abs_corr(X)
    c = ctx()
    S = sym.symnmf_build_S(c, to_dev(X), dtype=sym.DTYPES[dtype], fp8_panel_rows=100)
    M = stored_numpy(S)
    assert np.all(np.diag(M) == 1.0)
    if dtype == "fp32":
        assert np.max(np.abs(M - ref)) < 2e-6
        assert np.all(M == M.T)
    elif dtype == "bf16":
        ulp = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(ref), 1e-30))) - 7)
        assert np.all(np.abs(M - ref) <= 0.5 * ulp + 2e-6)
        assert np.all(M == M.T)
    else:
        off = ~np.eye(n, dtype=bool)
        assert np.all(np.abs(M - ref)[off] <= 2.0 ** -4 * np.abs(ref)[off] + 2.0 ** -9 / 448 * 1.2 + 1e-7)
        d = S.desc
        scale = from_dev(S.buf[d.panel_scale - d.data: d.panel_scale - d.data + 4 * ((n + 99) // 100)]
                         .view(torch.float32))
        for p in range(0, n, 100):
            blk = (M[p:p + 100] * scale[p // 100])[off[p:p + 100]]
            if blk.size:
                assert np.max(np.abs(blk)) == pytest.approx(448.0, rel=1e-6), p
    # the tiled buffer holds nothing outside the matrix
    d = S.desc
    E = {"fp32": 4, "bf16": 2, "fp8": 1}[dtype]
    raw = S.buf[: d.rows_pad * d.ld * E]
    nz = int(torch.count_nonzero(raw).item())
    assert nz <= n * n * E


@pytest.mark.parametrize("dtype,row0,rows", [("fp32", 130, 300), ("bf16", 130, 300), ("fp8", 128, 256),
                                             ("fp32", 0, 599)])
def test_build_row_panel_equals_rows_of_full(X600, dtype, row0, rows):
    """A row panel computes every tile of its rows directly; the full square
    build computes the tiles on and above the diagonal and mirrors them, so
    its lower rows must be the same bits (FP8: panels aligned to the scale
    panels, whose maxima then cover the same rows)."""
    c = ctx()
    kw = dict(dtype=sym.DTYPES[dtype], fp8_panel_rows=128)
    full = stored_numpy(sym.symnmf_build_S(c, to_dev(X600), **kw))
    pan = stored_numpy(sym.symnmf_build_S(c, to_dev(X600), row0=row0, rows=rows, **kw))
    assert pan.shape == (rows, 600)
    assert np.array_equal(pan, full[row0:row0 + rows])


@pytest.mark.parametrize("dtype,tol", [("fp64", 1e-12), ("fp32", 3e-6)])
def test_build_tpdm(dtype, tol):
    inst = synth.tpdm_returns(1, T=3001, n=300, groups=4, nu=3.0)
    X = inst.X.numpy()
    X[:, :40] = np.round(X[:, :40], 1)          # many ties in some columns
    ref = o.tpdm(X, q=0.05, lower_tail=True)
    S = sym.symnmf_build_S(ctx(), to_dev(X), kind=sym.TPDM, dtype=sym.DTYPES[dtype], q=0.05, lower_tail=1)
    M = stored_numpy(S)
    assert np.max(np.abs(M - ref)) < tol
    assert np.all(np.diag(M) == 1.0)


@pytest.mark.parametrize("dtype,tol", [("fp64", 1e-12), ("fp32", 3e-6)])
def test_build_tpdm_raw_marginals(dtype, tol):
    """The appendix's benchmark construction: polar transform of the Pareto
    factor-model samples as generated (no rank step); the lower tail of -X is
    the upper tail of X."""
    X = synth.paper_benchmark(3, 300, "tpdm", T=8000).X.numpy()
    ref = o.tpdm(X, q=0.01, lower_tail=False, raw_marginals=True)
    c = ctx()
    S = sym.symnmf_build_S(c, to_dev(X), kind=sym.TPDM, dtype=sym.DTYPES[dtype], q=0.01, lower_tail=0,
                           raw_marginals=1)
    M = stored_numpy(S)
    assert np.max(np.abs(M - ref)) < tol
    assert np.all(np.diag(M) == 1.0)
    S2 = sym.symnmf_build_S(c, to_dev(-X), kind=sym.TPDM, dtype=sym.DTYPES[dtype], q=0.01, lower_tail=1,
                            raw_marginals=1)
    assert np.array_equal(stored_numpy(S2), M)


def test_build_tpdm_raw_marginals_paper_sample_count():
    """40000 samples (beyond the rank transform's limit), n = 1000, top 1 %:
    the matrix of the paper's spectral table at n = 1000."""
    X = synth.paper_benchmark(7, 1000, "tpdm").X.numpy()
    ref = o.tpdm(X, q=0.01, lower_tail=False, raw_marginals=True)
    c = ctx()
    S = sym.symnmf_build_S(c, to_dev(X), kind=sym.TPDM, dtype=sym.S_FP32, q=0.01, lower_tail=0, raw_marginals=1)
    assert np.max(np.abs(stored_numpy(S) - ref)) < 3e-6
    with pytest.raises(sym.SymnmfError) as e:            # the rank transform stops at T = 32768
        sym.symnmf_build_S(c, to_dev(X), kind=sym.TPDM, q=0.01, lower_tail=0)
    assert e.value.code == sym.EUNSUPPORTED
    with pytest.raises(sym.SymnmfError) as e:            # raw marginals need X >= 0 in the tail orientation
        sym.symnmf_build_S(c, to_dev(X), kind=sym.TPDM, q=0.01, lower_tail=1, raw_marginals=1)
    assert e.value.code == sym.EINVAL


def test_build_rejects_constant_column_and_bad_shapes():
    X = np.random.default_rng(0).random((50, 20)).astype(np.float32)
    X[:, 3] = 2.0
    with pytest.raises(sym.SymnmfError) as e:
        sym.symnmf_build_S(ctx(), to_dev(X))
    assert e.value.code == sym.EINVAL
    with pytest.raises(sym.SymnmfError):
        sym.symnmf_build_S(ctx(), to_dev(X[:, :5] + np.arange(5, dtype=np.float32)), row0=3, rows=5)
    with pytest.raises(sym.SymnmfError):
        sym.symnmf_build_S(ctx(), to_dev(X[:1]))                          # T < 2
    with pytest.raises(sym.SymnmfError):
        sym.symnmf_build_S(ctx(), to_dev(X[:10, :4] + 1.0), kind=sym.TPDM, q=0.05)   # floor(qT) = 0


def test_build_and_load_report_nonfinite_input():
    """A NaN or infinity in X (either kind of S) or in a loaded S is a numeric
    error, not a zero-variance column."""
    c = ctx()
    X = np.random.default_rng(0).random((60, 30)).astype(np.float32)
    for bad in (float("nan"), float("inf")):
        Xb = X.copy()
        Xb[17, 11] = bad
        for kw in (dict(kind=sym.ABS_CORR), dict(kind=sym.TPDM, q=0.2)):
            with pytest.raises(sym.SymnmfError) as e:
                sym.symnmf_build_S(c, to_dev(Xb), **kw)
            assert e.value.code == sym.ENUMERIC, (bad, kw)
    Snp = o.abs_corr(X.astype(np.float64))
    Snp[4, 9] = float("nan")
    for dtype in (sym.S_FP64, sym.S_FP32, sym.S_BF16, sym.S_FP8):
        with pytest.raises(sym.SymnmfError) as e:
            sym.symnmf_S_load(c, to_dev(Snp, torch.float64), dtype=dtype, fp8_panel_rows=16)
        assert e.value.code == sym.ENUMERIC


def test_init_H_matches_oracle(S600):
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(S600, torch.float64), dtype=sym.S_FP32)
    H = torch.empty(600, 32, device=dev())
    sym.symnmf_init_H(c, S, 32, 1234, H)
    ref = o.init_H(S.desc.mean, 600, 32, 1234, as_float32=True)
    assert np.array_equal(from_dev(H), ref)


# --- one step: gradient, statistics and update ------------------------------
def _one_step(Snp, k, dtype, params, seed=0, panel_rows=128):
    c = ctx()
    n = Snp.shape[0]
    S = sym.symnmf_S_load(c, to_dev(Snp, torch.float64), dtype=sym.DTYPES[dtype], fp8_panel_rows=panel_rows)
    Sq = stored_numpy(S)
    f64 = dtype == "fp64"
    H0 = o.init_H(Snp.mean(), n, k, seed, as_float32=not f64)
    st = sym.symnmf_state_create(c, S, k, params, to_dev(H0, torch.float64 if f64 else torch.float32))
    stats = sym.symnmf_step(c, S, st)
    tdt = torch.float64 if f64 else torch.float32
    g = torch.empty(n, k, dtype=tdt, device=dev())
    H1 = torch.empty(n, k, dtype=tdt, device=dev())
    G = torch.empty(n, k, dtype=tdt, device=dev())
    sym.symnmf_state_read(c, st, 6, g)
    sym.symnmf_state_read(c, st, 0, H1)
    sym.symnmf_state_read(c, st, 2, G)
    return Sq, H0, stats, from_dev(g), from_dev(H1), from_dev(G), st, S


@pytest.mark.parametrize("dtype,k", [("fp32", 8), ("fp32", 16), ("fp32", 32), ("fp32", 64), ("fp32", 5),
                                     ("bf16", 32), ("bf16", 16), ("bf16", 64), ("fp8", 32), ("fp8", 64),
                                     ("fp64", 8), ("fp64", 32)])
def test_single_step_parity(S600, dtype, k):
    eta, eps = 0.05, 1e-10
    p = sym.symnmf_params_default(eta=eta, eps=eps)
    Sq, H0, stats, g, H1, G, _, _ = _one_step(S600, k, dtype, p)
    g_ref = o.gradient(Sq, H0)
    tol = 1e-11 if dtype == "fp64" else 2e-5
    assert np.max(np.abs(g - g_ref)) <= tol * np.max(np.abs(g_ref))
    f_ref = o.objective_trace(Sq, H0)
    assert stats.full == 1
    assert stats.f == pytest.approx(f_ref, rel=1e-12 if dtype == "fp64" else 1e-6)
    assert stats.E == pytest.approx(f_ref / (Sq * Sq).sum(), rel=1e-12 if dtype == "fp64" else 1e-6)
    assert stats.kkt == pytest.approx(o.kkt_measure(g_ref, H0), rel=1e-10 if dtype == "fp64" else 1e-4)
    # the update kernel applies the AdaGrad rule to its own gradient
    H_upd, G_upd = o.adagrad_update(H0, np.zeros_like(H0), g, eta, eps)
    atol = 1e-14 if dtype == "fp64" else 1e-6 * max(1.0, np.max(np.abs(H0)))
    assert np.max(np.abs(G - G_upd)) <= (1e-14 if dtype == "fp64" else 1e-6) * np.max(G_upd)
    assert np.max(np.abs(H1 - H_upd)) <= atol


@pytest.mark.parametrize("method,softplus", [("rmsprop", 0), ("adagrad", 1), ("rmsprop", 1)])
def test_update_rules_parity(S600, method, softplus):
    m = sym.RMSPROP if method == "rmsprop" else sym.ADAGRAD
    p = sym.symnmf_params_default(method=m, softplus=softplus, eta=0.01, eps=1e-8, alpha=0.99, mu=0.5)
    Sq, H0, stats, g, H1, G, st, S = _one_step(S600, 16, "fp64", p)
    if softplus:
        theta = o.softplus_inverse(H0)
        Hs = o.softplus(theta)
        g_ref = o.gradient(Sq, Hs)
        assert np.max(np.abs(g - g_ref)) <= 1e-10 * np.max(np.abs(g_ref))
        gt = g * o.sigmoid(theta)
        if m == sym.RMSPROP:
            th, _, _ = o.rmsprop_update(theta, 0 * theta, 0 * theta, gt, 0.01, 1e-8, 0.99, 0.5, project=False)
        else:
            th, _ = o.adagrad_update(theta, 0 * theta, gt, 0.01, 1e-8, project=False)
        assert np.max(np.abs(H1 - o.softplus(th))) < 1e-12
        assert stats.kkt == pytest.approx(o.kkt_measure(g_ref, Hs, softplus=True), rel=1e-10)
    else:
        Hr, v, mm = o.rmsprop_update(H0, 0 * H0, 0 * H0, g, 0.01, 1e-8, 0.99, 0.5)
        assert np.max(np.abs(H1 - Hr)) < 1e-13
        assert np.max(np.abs(G - v)) <= 1e-13 * np.max(v)


# --- trajectories ---------------------------------------------------------
def _run_gpu(Snp_or_S, k, params, H0, steps, dtype="fp64"):
    c = ctx()
    S = Snp_or_S if isinstance(Snp_or_S, sym.Matrix) else sym.symnmf_S_load(
        c, to_dev(Snp_or_S, torch.float64), dtype=sym.DTYPES[dtype])
    f64 = S.desc.dtype == sym.S_FP64
    st = sym.symnmf_state_create(c, S, k, params, to_dev(H0, torch.float64 if f64 else torch.float32))
    hist = [sym.symnmf_step(c, S, st) for _ in range(steps)]
    H = torch.empty(S.desc.n, k, dtype=torch.float64 if f64 else torch.float32, device=dev())
    sym.symnmf_state_read(c, st, 0, H)
    return hist, from_dev(H), S


def test_c1_fp64_trajectory_matches_oracle():
    """Plain projected AdaGrad in FP64 on the 512-instrument |corr| instance
    (8 planted groups, T = 2000, seed 0), 500 iterations."""
    X = synth.c1_instance(0).X.numpy()
    ref_S = o.abs_corr(X)
    c = ctx()
    S = sym.symnmf_build_S(c, to_dev(X), dtype=sym.S_FP64)
    assert np.max(np.abs(stored_numpy(S) - ref_S)) < 1e-13
    k = 8
    eta = math.sqrt(ref_S.mean() / k)
    H0 = o.init_H(ref_S.mean(), 512, k, 0)
    p = sym.symnmf_params_default(eta=eta, max_iter=500)
    hist, H, _ = _run_gpu(S, k, p, H0, 500)
    solver = o.Solver(ref_S, k, o.Params(eta=eta, max_iter=500), H0)
    ohist = [solver.step() for _ in range(500)]
    for t in (0, 1, 10, 100, 499):
        assert hist[t].f == pytest.approx(ohist[t].f, rel=1e-10)
    assert np.max(np.abs(H - solver.H)) < 1e-9
    assert o.subspace_error(H, solver.H) < 1e-6      # FP64 cancellation floor ~1.5e-8


def test_c1_fp32_matches_oracle_objective():
    X = synth.c1_instance(0).X.numpy()
    ref_S = o.abs_corr(X)
    c = ctx()
    S = sym.symnmf_build_S(c, to_dev(X), dtype=sym.S_FP32)
    k = 8
    eta = math.sqrt(ref_S.mean() / k)
    H0 = o.init_H(ref_S.mean(), 512, k, 0, as_float32=True)
    hist, H, _ = _run_gpu(S, k, sym.symnmf_params_default(eta=eta), H0, 500)
    solver = o.Solver(ref_S, k, o.Params(eta=eta), H0)
    for _ in range(500):
        solver.step()
    f_gpu, _ = sym.symnmf_objective(c, sym.symnmf_S_load(c, to_dev(ref_S, torch.float64), dtype=sym.S_FP64),
                                    to_dev(H, torch.float64), k)
    f_orc = o.objective_trace(ref_S, solver.H)
    assert abs(f_gpu - f_orc) / f_orc <= 1e-5
    assert o.subspace_error(H, solver.H) < 1e-3


@pytest.mark.parametrize("method,extra", [
    ("row", dict(row_frac=0.5)),
    ("block", dict(phi0=0.5, independent_blocks=1)),
    ("block", dict(phi0=0.25, independent_blocks=0)),
])
def test_svrg_trajectories_fp64(method, extra):
    X = _corr_instance(n=1300, T=600, groups=8, seed=2)
    Snp = o.abs_corr(X)
    k = 16
    H0 = o.init_H(Snp.mean(), 1300, k, 3)
    eta = 0.5 * math.sqrt(Snp.mean() / k)
    m = sym.ROW_SVRG if method == "row" else sym.BLOCK_SVRG
    p = sym.symnmf_params_default(method=m, eta=eta, block_rows=256, snapshot_s=5, delta=10, seed=17, **extra)
    hist, H, _ = _run_gpu(Snp, k, p, H0, 33)
    op = o.Params(method=o.ROW_SVRG if method == "row" else o.BLOCK_SVRG, eta=eta, block_rows=256, snapshot_s=5,
                  delta=10, seed=17, row_frac=extra.get("row_frac", 0.5), phi0=extra.get("phi0", 0.75),
                  independent_blocks=bool(extra.get("independent_blocks", 1)))
    solver = o.Solver(Snp, k, op, H0)
    ohist = [solver.step() for _ in range(33)]
    for a, b in zip(hist, ohist):
        assert bool(a.full) == b.full
        if b.full:
            assert a.f == pytest.approx(b.f, rel=1e-10)
    assert np.max(np.abs(H - solver.H)) < 1e-9


@pytest.mark.parametrize("dtype,k,indep", [("fp32", 16, 1), ("fp32", 32, 1), ("bf16", 32, 1), ("bf16", 32, 0),
                                           ("fp8", 32, 1), ("fp8", 32, 0), ("fp8", 16, 1)])
def test_block_svrg_mfma_path(dtype, k, indep):
    """Sampled Block-SVRG steps on every storage type, independent I and J or
    I = J.  On FP8 storage the diagonal is kept apart from the codes, so the
    update has to give S_ii h_i the weight of column i in the row's block
    gradient: 0 for rows in I only or J only, 2 for rows in both (every
    sampled row when I = J)."""
    X = _corr_instance(n=1300, T=600, groups=8, seed=2)
    Snp = o.abs_corr(X)
    H0 = o.init_H(Snp.mean(), 1300, k, 3, as_float32=True)
    eta = 0.5 * math.sqrt(Snp.mean() / k)
    p = sym.symnmf_params_default(method=sym.BLOCK_SVRG, eta=eta, block_rows=256, snapshot_s=4, delta=8, seed=5,
                                  phi0=0.5, independent_blocks=indep)
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(Snp, torch.float64), dtype=sym.DTYPES[dtype], fp8_panel_rows=128)
    Sq = stored_numpy(S)
    hist, H, _ = _run_gpu(S, k, p, H0, 6)
    op = o.Params(method=o.BLOCK_SVRG, eta=eta, block_rows=256, snapshot_s=4, delta=8, seed=5, phi0=0.5,
                  independent_blocks=bool(indep))
    solver = o.Solver(Sq, k, op, H0)
    kinds = []
    for _ in range(6):
        kinds.append(solver.step_kind())
        solver.step()
    assert kinds.count("block") >= 3
    assert np.max(np.abs(H - solver.H)) < 2e-4 * np.max(np.abs(solver.H))


# --- order statistics, Piecewise reset, objective ---------------------------
# --- ADMM (appendix family 6) ---------------------------------------------------
def test_admm_fp64_trajectory_matches_oracle(S600):
    """300 ADMM iterations in FP64 storage and state: the objective of every
    W_t and the final W and U agree with the oracle to summation order."""
    c = ctx()
    k, rho = 8, 20.0
    S = sym.symnmf_S_load(c, to_dev(S600, torch.float64), dtype=sym.S_FP64)
    H0 = o.init_H(S600.mean(), 600, k, 2)
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(method=sym.ADMM, rho=rho, max_iter=10 ** 9),
                                 to_dev(H0, torch.float64))
    solver = o.Solver(S600, k, o.Params(method=o.ADMM, rho=rho), H0)
    for t in range(300):
        s = sym.symnmf_step(c, S, st)
        r = solver.step()
        assert s.f == pytest.approx(r.f, rel=1e-10), t
        assert s.kkt == pytest.approx(r.kkt, rel=1e-8, abs=1e-14), t
    W = torch.empty(600, k, dtype=torch.float64, device=dev())
    U = torch.empty(600, k, dtype=torch.float64, device=dev())
    sym.symnmf_state_read(c, st, 0, W)
    sym.symnmf_state_read(c, st, 3, U)
    W, U = from_dev(W), from_dev(U)
    assert np.max(np.abs(W - solver.H)) < 1e-9 * np.max(solver.H)
    assert np.max(np.abs(U - solver.U)) < 1e-9 * max(np.max(np.abs(solver.U)), 1e-30) + 1e-15
    assert np.all(U <= 0.0) and np.all(W >= 0.0) and np.all(W * U == 0.0)


@pytest.mark.parametrize("dtype,k", [("fp32", 16), ("fp32", 32), ("fp32", 64), ("bf16", 32), ("fp8", 32), ("fp32", 5)])
def test_admm_single_step_parity(S600, dtype, k):
    """One ADMM step on the stored S (every stream kernel and the k x k
    inverse): W_1 and U_1 against the oracle's update from the same W_0."""
    c = ctx()
    rho = 50.0
    S = sym.symnmf_S_load(c, to_dev(S600, torch.float64), dtype=sym.DTYPES[dtype], fp8_panel_rows=128)
    Sq = stored_numpy(S)
    H0 = o.init_H(S600.mean(), 600, k, 3, as_float32=True)
    st = sym.symnmf_state_create(c, S, k, sym.symnmf_params_default(method=sym.ADMM, rho=rho), to_dev(H0))
    stats = sym.symnmf_step(c, S, st)
    W1 = torch.empty(600, k, device=dev())
    U1 = torch.empty(600, k, device=dev())
    sym.symnmf_state_read(c, st, 0, W1)
    sym.symnmf_state_read(c, st, 3, U1)
    W_ref, U_ref = o.admm_update(Sq, H0.astype(np.float64), np.zeros((600, k)), rho)
    scale = np.max(np.abs(W_ref))
    assert np.max(np.abs(from_dev(W1) - W_ref)) <= 2e-5 * scale
    assert np.max(np.abs(from_dev(U1) - U_ref)) <= 2e-5 * scale
    assert stats.f == pytest.approx(o.objective_trace(Sq, H0.astype(np.float64)), rel=1e-6)


def test_admm_certifies_planted_factorisation_like_the_oracle():
    Hs = synth.planted_factor(3, 300, 4).numpy()
    Snp = Hs @ Hs.T
    H0 = o.init_H(Snp.mean(), 300, 4, 1)
    kw = dict(rho=2.0, max_iter=5000, tau_g_inf=1e-10)
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(Snp, torch.float64), dtype=sym.S_FP64)
    st = sym.symnmf_state_create(c, S, 4, sym.symnmf_params_default(method=sym.ADMM, **kw), to_dev(H0, torch.float64))
    W = torch.empty(300, 4, dtype=torch.float64, device=dev())
    stats, conv = sym.symnmf_solve_to_tol(c, S, st, H_out=W)
    Wo, ost = o.Solver(Snp, 4, o.Params(method=o.ADMM, **kw), H0).solve()
    assert conv and ost.converged and stats.t == ost.t
    assert stats.E < 1e-12
    assert o.subspace_error(from_dev(W), Hs) < 1e-6


def test_admm_rejects_softplus_and_bad_rho(S600):
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(S600, torch.float64))
    H0 = torch.full((600, 4), 0.05, device=dev())
    for kw in (dict(rho=0.0), dict(rho=-1.0), dict(softplus=1)):
        with pytest.raises(sym.SymnmfError) as e:
            sym.symnmf_state_create(c, S, 4, sym.symnmf_params_default(method=sym.ADMM, **kw), H0)
        assert e.value.code == sym.EINVAL


def test_median_sq_matches_oracle():
    g = np.random.default_rng(3).normal(size=100003).astype(np.float32)
    g[:50] = 0.0
    med = sym.symnmf_median_sq(ctx(), to_dev(g))
    ref = o.lower_median(g.astype(np.float64) ** 2)
    assert med == np.float32(ref)


def test_piecewise_reset_matches_formula(S600):
    p = sym.symnmf_params_default(method=sym.PIECEWISE_ADAGRAD, eta=0.05)
    Sq, H0, stats, g, H1, G, st, S = _one_step(S600, 16, "fp64", p)
    med = sym.symnmf_piecewise_reset(ctx(), st, 10.0)
    assert med == np.float32(o.lower_median(g * g))
    Gn = torch.empty(600, 16, dtype=torch.float64, device=dev())
    sym.symnmf_state_read(ctx(), st, 2, Gn)
    assert np.max(np.abs(from_dev(Gn) - o.piecewise_reset(g, 10.0))) <= 1e-12 * np.max(np.abs(from_dev(Gn)))


def test_solve_to_tol_certifies_planted_factorisation():
    Hs = synth.planted_factor(3, 300, 4).numpy()
    Snp = Hs @ Hs.T
    H0 = o.init_H(Snp.mean(), 300, 4, 1)
    eta = math.sqrt(Snp.mean() / 4)
    # KKT gate 1e-10 * (1e4/300): well above the FP64 noise of the gradient, so
    # both sides take the same stop decision at the same check
    p = sym.symnmf_params_default(eta=eta, max_iter=20000, tau_g_inf=1e-10)
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(Snp, torch.float64), dtype=sym.S_FP64)
    st = sym.symnmf_state_create(c, S, 4, p, to_dev(H0, torch.float64))
    H = torch.empty(300, 4, dtype=torch.float64, device=dev())
    stats, conv = sym.symnmf_solve_to_tol(c, S, st, H_out=H)
    Ho, ost = o.Solver(Snp, 4, o.Params(eta=eta, max_iter=20000, tau_g_inf=1e-10), H0).solve()
    assert conv and ost.converged and stats.t == ost.t
    assert stats.E < 1e-12 and stats.kkt < 1e-10 * 1e4 / 300
    assert o.subspace_error(from_dev(H), Hs) < 1e-6


def test_stop_rule_rejects_zero_factor_through_the_loss_gate():
    """From H = 0 the gradient, the KKT measure and the progress are all zero;
    the loss gate alone keeps the stop rule from certifying it, as in the
    oracle (opened gate: certified at the first check past the warm-up)."""
    c = ctx()
    Snp = o.abs_corr(_corr_instance(n=300, T=200, groups=3, seed=4))
    S = sym.symnmf_S_load(c, to_dev(Snp, torch.float64), dtype=sym.S_FP32)
    H0 = torch.zeros(300, 4, device=dev())
    st = sym.symnmf_state_create(c, S, 4, sym.symnmf_params_default(eta=0.05, max_iter=300), H0)
    stats, conv = sym.symnmf_solve_to_tol(c, S, st)
    # 300 steps evaluate H_0 .. H_299: the last check is t = 290
    assert not conv and stats.t == 290 and stats.E == pytest.approx(1.0, rel=1e-12) and stats.kkt == 0.0
    st = sym.symnmf_state_create(c, S, 4, sym.symnmf_params_default(eta=0.05, max_iter=300, tau_E=1.5), H0)
    stats, conv = sym.symnmf_solve_to_tol(c, S, st)
    _, ost = o.Solver(Snp, 4, o.Params(eta=0.05, max_iter=300, tau_E=1.5), np.zeros((300, 4))).solve()
    assert conv and ost.converged and stats.t == ost.t == 50


def test_objective_near_exact_factorisation():
    """E ~ 1e-6: the trace terms cancel to six digits, and the FP64-accumulating
    objective still matches the explicit n x n residual."""
    Hs = synth.planted_factor(5, 700, 6).numpy()
    Snp = Hs @ Hs.T
    H = Hs * (1.0 + 1e-3 * np.random.default_rng(3).standard_normal(Hs.shape))
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(Snp, torch.float64), dtype=sym.S_FP64)
    f, E = sym.symnmf_objective(c, S, to_dev(H, torch.float64), 6)
    f_ex = o.objective_explicit(Snp, H)
    assert 1e-7 < f_ex / (Snp * Snp).sum() < 1e-5
    assert f == pytest.approx(f_ex, rel=1e-8)


def test_objective_fp64_accumulation(S600):
    c = ctx()
    for dtype in ("fp32", "bf16", "fp8"):
        S = sym.symnmf_S_load(c, to_dev(S600, torch.float64), dtype=sym.DTYPES[dtype], fp8_panel_rows=100)
        Sq = stored_numpy(S)
        H = np.random.default_rng(1).random((600, 24)) * 0.1
        f, E = sym.symnmf_objective(c, S, to_dev(H, torch.float64), 24)
        ref = o.objective_trace(Sq, H)
        assert f == pytest.approx(ref, rel=1e-12)
        assert E == pytest.approx(ref / (Sq * Sq).sum(), rel=1e-12)


@pytest.mark.parametrize("dtype,k", [("fp32", 16), ("fp32", 32), ("bf16", 32), ("fp8", 16), ("fp32", 24)])
def test_objective_float32_H(S600, dtype, k):
    """float32 H: MFMA products summed in FP32 within a 256-column chunk and in
    FP64 across chunks (k = 16, 32), or the all-FP64 path (other k)."""
    c = ctx()
    S = sym.symnmf_S_load(c, to_dev(S600, torch.float64), dtype=sym.DTYPES[dtype], fp8_panel_rows=100)
    Sq = stored_numpy(S)
    H = (np.random.default_rng(2).random((600, k)) * 0.1).astype(np.float32)
    f, E = sym.symnmf_objective(c, S, to_dev(H, torch.float32), k)
    ref = o.objective_trace(Sq, H.astype(np.float64))
    assert f == pytest.approx(ref, rel=1e-7)


# --- edge cases ----------------------------------------------------------------
@pytest.mark.parametrize("n", [1300, 2600])
@pytest.mark.parametrize("dtype,k", [("fp32", 32), ("bf16", 64), ("fp8", 64)])
def test_full_step_with_aligned_pair_segments(n, dtype, k):
    """3 and 6 tile pairs: the full-step stream then launches 255 and 252
    work-groups, each a whole chunk segment of one pair (ragged last tile)."""
    Snp = o.abs_corr(_corr_instance(n=n, T=300, groups=5, seed=2))
    Sq, H0, stats, g, _, _, _, _ = _one_step(Snp, k, dtype, sym.symnmf_params_default(eta=0.05))
    g_ref = o.gradient(Sq, H0)
    assert np.max(np.abs(g - g_ref)) <= 2e-5 * np.max(np.abs(g_ref))
    assert stats.f == pytest.approx(o.objective_trace(Sq, H0), rel=1e-6)


def test_tiny_and_degenerate_shapes():
    c = ctx()
    X = _corr_instance(n=37, T=50, groups=3, seed=9)
    Snp = o.abs_corr(X)
    for k in (1, 5):
        Sq, H0, stats, g, H1, G, _, _ = _one_step(Snp, k, "fp32", sym.symnmf_params_default(eta=0.01))
        g_ref = o.gradient(Sq, H0)
        assert np.max(np.abs(g - g_ref)) <= 2e-5 * np.max(np.abs(g_ref))
    S = sym.symnmf_S_load(c, to_dev(Snp, torch.float64))
    H0 = torch.zeros(37, 4, device=dev())
    st = sym.symnmf_state_create(c, S, 4, sym.symnmf_params_default(), H0)
    s = sym.symnmf_step(c, S, st)
    assert s.E == pytest.approx(1.0) and s.kkt == 0.0    # H = 0: zero gradient, E = 1
    for bad_k in (0, 65, 38):
        with pytest.raises(sym.SymnmfError) as e:
            sym.symnmf_state_create(c, S, bad_k, sym.symnmf_params_default(), torch.zeros(37, 65, device=dev()))
        assert e.value.code == sym.EINVAL
    with pytest.raises(sym.SymnmfError):
        sym.symnmf_state_create(c, S, 4, sym.symnmf_params_default(method=sym.ROW_SVRG, delta=7, snapshot_s=5), H0)


def test_nonfinite_input_is_reported():
    c = ctx()
    Snp = o.abs_corr(_corr_instance(n=100, T=80, groups=2, seed=1))
    S = sym.symnmf_S_load(c, to_dev(Snp, torch.float64))
    H0 = torch.full((100, 4), 0.1, device=dev())
    H0[7, 2] = float("nan")
    st = sym.symnmf_state_create(c, S, 4, sym.symnmf_params_default(), H0)
    with pytest.raises(sym.SymnmfError) as e:
        sym.symnmf_step(c, S, st)
    assert e.value.code == sym.ENUMERIC
