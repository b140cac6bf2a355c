"""Plain FP64 CPU oracle for the SymNMF hot path.

TEST INFRASTRUCTURE ONLY.  This module is the reference that the HIP path
is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never calls it,
and it shares no code with the HIP path (the only shared module is
``synth``, which makes inputs and holds none of the method's arithmetic).

Everything is written for readability against the paper, in float64, with
numpy primitives (matmul, sort) as the only library steps:

* S construction: absolute Pearson correlation (benchmark appendix,
  correlation construction) and the empirical tail pairwise dependence matrix
  (section "Empirical Estimation" and the appendix TPDM construction).
* Objective in trace-identity form (eq. trace_loss) and, for small n, the
  explicit n x n residual (eq. symnmf); gradient 4(H(H^T H) - SH)
  (section "Memory-Efficient Loss Reformulation").
* Update rules of appendix "Detailed Algorithm Descriptions", family 3:
  AdaGrad, RMSprop, Adam, NAdam, Adan, their softplus (LogSpace) forms
  (eq. logspace_grad), Piecewise AdaGrad, Row-Stochastic SVRG, Block-SVRG
  AdaptGrow; family 1, the dampened multiplicative update; and family 6, ADMM
  (eqs. admm_H, admm_W, admm_U).
* The three-criterion stop rule (eqs. proj_grad, loss_gate, kkt_stop,
  kkt_scaled, obj_stag, conv_and).

Where the paper is silent the reading taken is stated next to the code.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Counter-based random numbers (SplitMix64, Steele, Lea & Flood, OOPSLA 2014).
# The method draws random numbers in two places: the initial H (section
# "Initialization and seeds") and the row / block index sets of the
# stochastic AdaGrad variants.  Both sides implement this one published
# generator; the value for counter c under key s is the SplitMix64 output
# of state s after c+1 increments.
# ---------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(key, counter):
    """SplitMix64 output number ``counter`` (0-based) of the stream seeded by ``key``."""
    with np.errstate(over="ignore"):
        z = np.uint64(key) + (np.asarray(counter, dtype=np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform24(key, counter):
    """Uniform in [0, 1) with 24 random bits: (top 24 bits of the draw) * 2^-24."""
    return (splitmix64(key, counter) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24


def stream_key(seed: int, t: int, stream: int) -> int:
    """Key of the index-set draw for iteration t (stream 0 = I, stream 1 = J)."""
    base = int(splitmix64(np.uint64(seed & (2**64 - 1)), np.uint64(2 * t + stream)))
    return base


def sample_blocks(seed: int, t: int, stream: int, nblocks: int, m: int) -> np.ndarray:
    """m distinct block indices out of nblocks, sorted ascending.

    Uniform sampling without replacement by a partial Fisher-Yates shuffle
    (Knuth, TAOCP vol. 2, Algorithm P): for i = 0..m-1 swap position i with
    position i + (u_i * (nblocks - i)) where u_i is the i-th 24-bit uniform of
    the stream keyed by (seed, t, stream).
    """
    key = stream_key(seed, t, stream)
    a = list(range(nblocks))
    for i in range(m):
        u = float(uniform24(key, i))
        j = i + int(u * (nblocks - i))
        a[i], a[j] = a[j], a[i]
    return np.array(sorted(a[:m]), dtype=np.int64)


# ---------------------------------------------------------------------------
# S construction
# ---------------------------------------------------------------------------
def standardise_columns(X):
    """Centre each column and scale it to unit Euclidean norm, in FP64.

    With Z = standardise_columns(X), Z^T Z is exactly the Pearson sample
    correlation (the normalisation constant of the covariance cancels).
    A constant column has no correlation and is rejected.
    """
    X = np.asarray(X, dtype=np.float64)
    D = X - X.mean(axis=0)
    c = np.sqrt((D * D).sum(axis=0))
    if np.any(c == 0.0):
        raise ValueError("zero-variance column")
    return D / c


def abs_corr(X):
    """S_ij = |C_ij|, C the Pearson sample correlation of the columns of X,
    with S_ii = 1 exactly (appendix, correlation construction)."""
    Z = standardise_columns(X)
    S = np.abs(Z.T @ Z)
    np.fill_diagonal(S, 1.0)
    return S


def abs_corr_panel(Z, row0: int, rows: int):
    """Rows [row0, row0+rows) of |corr| from the standardised columns Z
    (Z = standardise_columns(X)), S_ii = 1: the same definition as abs_corr,
    evaluated for a row panel only."""
    P = np.abs(Z[:, row0:row0 + rows].T @ Z)
    r = np.arange(rows)
    P[r, r + row0] = 1.0
    return P


class StoredRows:
    """A dense S too large for FP64 host memory (n = 10^5: 80 GB), held as
    float32 - every entry rounded once from its FP64 value - and used with
    FP64 arithmetic only: S @ H converts one slab of rows at a time to FP64
    and multiplies it by the FP64 H (a library matmul), so the product is the
    FP64 product of the stored entries.  ||S||_F^2 and the mean are FP64 sums
    of the stored entries.  A solver run on a StoredRows solves the problem
    of the float32-rounded matrix exactly in FP64 (the rounding moves S by at
    most 2^-24 relative per entry)."""

    SLAB = 128

    def __init__(self, data32):
        self.data = data32
        self.shape = data32.shape
        self.fro2 = 0.0
        self.sum = 0.0
        for r0 in range(0, self.shape[0], 4096):
            blk = self.data[r0:r0 + 4096].astype(np.float64)
            self.fro2 += float((blk * blk).sum())
            self.sum += float(blk.sum())

    @classmethod
    def abs_corr(cls, X, panel_rows: int = 1024):
        """|corr| of the columns of X (same definition as abs_corr), built
        row panel by row panel from the standardised columns in FP64."""
        Z = standardise_columns(X)
        n = Z.shape[1]
        data = np.empty((n, n), dtype=np.float32)
        for r0 in range(0, n, panel_rows):
            rows = min(panel_rows, n - r0)
            data[r0:r0 + rows] = abs_corr_panel(Z, r0, rows)
        return cls(data)

    def mean(self):
        return self.sum / (self.shape[0] * self.shape[1])

    def rows(self, r0: int, r1: int):
        return self.data[r0:r1].astype(np.float64)

    def __matmul__(self, H):
        from concurrent.futures import ThreadPoolExecutor
        from threadpoolctl import threadpool_limits
        H = np.asarray(H, dtype=np.float64)
        out = np.empty((self.shape[0], H.shape[1]))

        def slab(r0):
            out[r0:r0 + self.SLAB] = self.data[r0:r0 + self.SLAB].astype(np.float64) @ H

        with threadpool_limits(1), ThreadPoolExecutor() as ex:
            list(ex.map(slab, range(0, self.shape[0], self.SLAB)))
        return out


def gradient_panel(S_panel, H, row0: int):
    """Rows [row0, row0+rows) of grad f = 4 (H (H^T H) - S H) from the
    matching row panel of S and the full H."""
    rows = S_panel.shape[0]
    return 4.0 * (H[row0:row0 + rows] @ (H.T @ H) - S_panel @ H)


def rank_columns(X):
    """Rank 1..T of every entry within its column; ties go to the lower row."""
    X = np.asarray(X)
    T, n = X.shape
    order = np.argsort(X, axis=0, kind="stable")
    R = np.empty((T, n), dtype=np.int64)
    R[order, np.arange(n)[None, :]] = np.arange(1, T + 1)[:, None]
    return R


def pareto2_from_ranks(R, T):
    """Empirical-CDF transform to Pareto(alpha=2) margins: P(X > x) = x^-2,
    i.e. x = (1 - F)^(-1/2) with F = r / (T + 1) (section "Empirical
    Estimation": marginals are transformed to Pareto(2) form)."""
    return (1.0 - np.asarray(R, dtype=np.float64) / (T + 1.0)) ** -0.5


def tpdm(X, q: float, lower_tail: bool = True, return_parts: bool = False, raw_marginals: bool = False):
    """Empirical TPDM, unit-diagonal normalised.

    Steps (section "Empirical Estimation"; appendix TPDM construction):
    1. one-sided tail: the lower tail of X is the upper tail of -X;
    2. rank-transform each column to Pareto(2) margins (skipped when
       raw_marginals: the appendix's benchmark matrices apply the polar
       transform to the Pareto(2) factor-model samples as generated);
    3. polar coordinates of every sample: r_t = ||x_t||_2, w_t = x_t / r_t;
    4. keep the n_exc = floor(q T) samples with the largest r_t (ties go to
       the lower sample index); their w_t are the rows of Omega;
    5. S~ = (n / n_exc) Omega^T Omega and S = D^-1/2 S~ D^-1/2, D = diag(S~).
    """
    X = np.asarray(X, dtype=np.float64)
    T, n = X.shape
    Y = -X if lower_tail else X
    P = Y if raw_marginals else pareto2_from_ranks(rank_columns(Y), T)
    r = np.sqrt((P * P).sum(axis=1))
    n_exc = int(math.floor(q * T))
    if n_exc < 1:
        raise ValueError("no exceedances: q*T < 1")
    order = np.lexsort((np.arange(T), -r))      # largest r first, then lower t
    sel = np.sort(order[:n_exc])
    Omega = P[sel] / r[sel, None]
    St = (n / n_exc) * (Omega.T @ Omega)
    d = np.sqrt(np.diag(St))
    S = St / np.outer(d, d)
    np.fill_diagonal(S, 1.0)
    if return_parts:
        return S, dict(P=P, r=r, sel=sel, Omega=Omega, St=St)
    return S


def tpdm_rows(X, q: float, rows, lower_tail: bool = True, col_block: int = 2048):
    """Rows ``rows`` of tpdm(X, q, lower_tail), for sizes where neither the
    n x n matrix nor the T x n Pareto margins fit in FP64 host memory
    (n = 10^5, T = 2 10^4: 80 GB and 16 GB).

    The same five steps as tpdm (section "Empirical Estimation"), taken a
    block of columns at a time where the definition is per column: the rank
    transform of step 2 is per column, so it is done block by block; the
    radii of step 3 are sums over all columns, accumulated over the blocks;
    after the selection of step 4 the blocks are transformed again and only
    the selected samples kept.  Step 5 then needs only the selected rows
    Omega (n_exc x n) and the row norms of its columns:
    S_ij = St_ij / sqrt(St_ii St_jj), St = (n / n_exc) Omega^T Omega.
    """
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    T, n = X.shape
    rows = np.asarray(rows, dtype=np.int64)
    sign = -1.0 if lower_tail else 1.0
    blocks = [(c0, min(c0 + col_block, n)) for c0 in range(0, n, col_block)]

    def margins(b):
        Y = sign * np.asarray(X[:, b[0]:b[1]], dtype=np.float64)
        return pareto2_from_ranks(rank_columns(Y), T)

    def sq_norms(b):
        P = margins(b)
        return (P * P).sum(axis=1)

    import os
    with threadpool_limits(1), ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        r2 = np.zeros(T)
        for part in ex.map(sq_norms, blocks):
            r2 += part
        r = np.sqrt(r2)
        n_exc = int(math.floor(q * T))
        if n_exc < 1:
            raise ValueError("no exceedances: q*T < 1")
        order = np.lexsort((np.arange(T), -r))
        sel = np.sort(order[:n_exc])
        Omega = np.empty((n_exc, n))

        def angular(b):
            Omega[:, b[0]:b[1]] = margins(b)[sel] / r[sel, None]

        list(ex.map(angular, blocks))
    St_rows = (n / n_exc) * (Omega[:, rows].T @ Omega)
    d = np.sqrt((n / n_exc) * (Omega * Omega).sum(axis=0))
    S = St_rows / np.outer(d[rows], d)
    S[np.arange(rows.size), rows] = 1.0
    return S


# ---------------------------------------------------------------------------
# Storage formats (not in the paper: the paper runs fp32 and leaves half
# precision open).  Round-to-nearest-even to a given significand width.
# ---------------------------------------------------------------------------
def _round_sig(x, sig_bits: int, min_normal_exp: int):
    """Round to ``sig_bits`` significand bits (implicit bit included), nearest
    even; below 2^min_normal_exp round to the fixed subnormal spacing."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0.0
    e = np.floor(np.log2(np.abs(x[nz])))
    # guard log2 rounding near powers of two
    e = np.where(np.abs(x[nz]) >= 2.0 ** (e + 1), e + 1, e)
    e = np.where(np.abs(x[nz]) < 2.0 ** e, e - 1, e)
    e = np.maximum(e, min_normal_exp)
    quantum = 2.0 ** (e - (sig_bits - 1))
    out[nz] = np.rint(x[nz] / quantum) * quantum     # np.rint rounds half to even
    return out


def to_bf16(x):
    """bfloat16 value (8 significand bits, normal exponent >= -126), RNE."""
    return _round_sig(x, 8, -126)


FP8_MAX = 448.0


def to_fp8_e4m3(x):
    """OCP FP8 E4M3 value: 4 significand bits, normal exponent >= -6,
    subnormal spacing 2^-9, saturating at +-448, RNE."""
    y = _round_sig(x, 4, -6)
    return np.clip(y, -FP8_MAX, FP8_MAX)


def quantise(S, dtype: str, panel_rows: int = 256, row0: int = 0):
    """The matrix a solver sees when S is stored in ``dtype``.

    'fp64'/'fp32'/'bf16' round every entry; 'fp8' stores round(S * scale_p)
    off the diagonal and keeps S_ii exactly.  Returns (S_q, scales or None).
    """
    S = np.asarray(S, dtype=np.float64)
    if dtype == "fp64":
        return S.copy(), None
    if dtype == "fp32":
        return S.astype(np.float32).astype(np.float64), None
    if dtype == "bf16":
        return to_bf16(S), None
    if dtype == "fp8":
        sc = fp8_panel_scales(S, panel_rows, row0)
        rows = S.shape[0]
        Sq = np.empty_like(S)
        for p in range(len(sc)):
            sl = slice(p * panel_rows, min((p + 1) * panel_rows, rows))
            Sq[sl] = to_fp8_e4m3(S[sl] * sc[p]) / sc[p]
        r = np.arange(rows)
        Sq[r, r + row0] = S[r, r + row0]
        return Sq, sc
    raise ValueError(dtype)


def fp8_panel_scales(S, panel_rows: int, row0: int = 0):
    """Scale of each row panel: 448 / (largest off-diagonal |S_ij| in it).

    S may be a row panel whose first row is global row ``row0``.  The unit
    diagonal is kept out of the stored codes (it would saturate) and is added
    back exactly by the consumer of the panel.
    """
    n_rows, n = S.shape
    scales = []
    for p0 in range(0, n_rows, panel_rows):
        blk = np.abs(np.array(S[p0:p0 + panel_rows], dtype=np.float64))
        rows = np.arange(p0, min(p0 + panel_rows, n_rows))
        blk[rows - p0, rows + row0] = 0.0
        m = blk.max() if blk.size else 0.0
        scales.append(FP8_MAX / m if m > 0 else 1.0)
    return np.array(scales)


# ---------------------------------------------------------------------------
# Initial factor (section "Initialization and seeds"): entries U[0, sqrt(mean(S)/k)].
# ---------------------------------------------------------------------------
def init_H(S_mean: float, n: int, k: int, seed: int, as_float32: bool = False):
    """H0_ij = u_ij * sqrt(S_mean / k), u_ij the 24-bit uniform of counter i*k+j.

    ``as_float32`` returns the value a float32 implementation stores: the
    scale rounded to float32, the product rounded to float32.
    """
    u = uniform24(np.uint64(seed & (2**64 - 1)), np.arange(n * k, dtype=np.uint64)).reshape(n, k)
    scale = math.sqrt(S_mean / k)
    if as_float32:
        return (u.astype(np.float32) * np.float32(scale)).astype(np.float64)
    return u * scale


# ---------------------------------------------------------------------------
# Objective, gradient, stationarity
# ---------------------------------------------------------------------------
def objective_explicit(S, H):
    """f(H) = ||S - H H^T||_F^2 with the n x n residual formed (eq. symnmf)."""
    R = np.asarray(S, dtype=np.float64) - H @ H.T
    return float((R * R).sum())


def objective_trace(S, H, SH=None):
    """f(H) = ||S||_F^2 - 2 tr(H^T S H) + ||H^T H||_F^2 (eq. trace_loss)."""
    if isinstance(S, StoredRows):
        fro2 = S.fro2
    else:
        S = np.asarray(S, dtype=np.float64)
        fro2 = float((S * S).sum())
    SH = S @ H if SH is None else SH
    G = H.T @ H
    return float(fro2 - 2.0 * (H * SH).sum() + (G * G).sum())


def gradient(S, H, SH=None):
    """grad f = 4 (H (H^T H) - S H), H^T H formed first (right to left)."""
    SH = np.asarray(S, dtype=np.float64) @ H if SH is None else SH
    return 4.0 * (H @ (H.T @ H) - SH)


def projected_gradient(g, H):
    """eq. proj_grad: g where H > 0, min(0, g) where H = 0."""
    return np.where(H > 0.0, g, np.minimum(g, 0.0))


def kkt_measure(g, H, softplus: bool = False):
    """||grad_proj||_F / (n k) (eq. kkt_stop).  For H = softplus(Theta) > 0 the
    projected gradient is the H-space gradient itself (LogSpace adaptation)."""
    pg = g if softplus else projected_gradient(g, H)
    return float(np.sqrt((pg * pg).sum()) / H.size)


def tau_g(n: int, tau_inf: float = 1e-4, n_ref: float = 1e4) -> float:
    """eq. kkt_scaled: tau_g(n) = tau_inf * max(1, n_ref / n)."""
    return tau_inf * max(1.0, n_ref / n)


def subspace_error(A, B):
    """||P_A - P_B||_F / sqrt(2k), P the orthogonal projector onto range(.).
    Invariant to column permutations, so it compares SymNMF solutions that
    are identical up to the permutation ambiguity (section Identifiability)."""
    def basis(M):
        Q, _ = np.linalg.qr(np.asarray(M, dtype=np.float64))
        return Q
    QA, QB = basis(A), basis(B)
    k = QA.shape[1]
    d2 = 2 * k - 2.0 * float(((QA.T @ QB) ** 2).sum())
    return math.sqrt(max(d2, 0.0) / (2 * k))


# ---------------------------------------------------------------------------
# Softplus reparameterisation (section "Constraint Handling Strategies")
# ---------------------------------------------------------------------------
def softplus(theta):
    return np.maximum(theta, 0.0) + np.log1p(np.exp(-np.abs(theta)))


def sigmoid(theta):
    return 0.5 * (1.0 + np.tanh(0.5 * theta))


def softplus_inverse(h, floor: float = 1e-12):
    """Theta0 with softplus(Theta0) = max(H0, floor) (reading: the paper does not
    say how Theta is initialised)."""
    h = np.maximum(np.asarray(h, dtype=np.float64), floor)
    return np.where(h > 20.0, h + np.log(-np.expm1(-h)), np.log(np.expm1(np.minimum(h, 20.0))))


# ---------------------------------------------------------------------------
# Update rules (appendix, family 3), one iteration given the gradient g of H_t.
# ---------------------------------------------------------------------------
def adagrad_update(X, G, g, eta, eps, project=True):
    """G_t = G_{t-1} + g*g ;  X <- [X - eta g / (sqrt(G_t) + eps)]_+ ."""
    G = G + g * g
    X = X - eta * g / (np.sqrt(G) + eps)
    return (np.maximum(X, 0.0) if project else X), G


def rmsprop_update(X, v, m, g, eta, eps, alpha, mu, project=True):
    """v = alpha v + (1-alpha) g^2 ; m = mu m + eta g/(sqrt(v)+eps) ; X <- [X - m]_+ .
    The momentum buffer is kept as is when the clamp acts (reading)."""
    v = alpha * v + (1.0 - alpha) * g * g
    m = mu * m + eta * g / (np.sqrt(v) + eps)
    X = X - m
    return (np.maximum(X, 0.0) if project else X), v, m


def adam_update(X, m, v, g, t, eta, eps, beta1, beta2, nesterov=False, project=True):
    """Adam (appendix family 3), step t = 1, 2, ...:
    m = b1 m + (1-b1) g ; v = b2 v + (1-b2) g^2 ; m^ = m/(1-b1^t) ; v^ = v/(1-b2^t) ;
    X <- [X - eta m^ / (sqrt(v^) + eps)]_+ .
    NAdam (nesterov=True) uses b1 m^ + (1-b1) g/(1-b1^t) in place of m^."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    if nesterov:
        mhat = beta1 * mhat + (1.0 - beta1) * g / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    X = X - eta * mhat / (np.sqrt(vhat) + eps)
    return (np.maximum(X, 0.0) if project else X), m, v


def adan_update(X, m, d, nv, g, g_prev, t, eta, eps, beta1, beta2, beta3, project=True):
    """Adan (Xie et al., "Adan: Adaptive Nesterov Momentum Algorithm", 2023,
    Algorithm 1), written with the beta's as decay factors and bias-corrected
    averages; the three buffers are the gradient average m, the average d of
    gradient differences and the second moment nv of the Nesterov-corrected
    gradient.  With diff = g - g_prev (0 at the first step, g_prev = None):
    m = b1 m + (1-b1) g ; d = b2 d + (1-b2) diff ; nv = b3 nv + (1-b3)(g + b2 diff)^2 ;
    X <- [X - eta (m/(1-b1^t) + b2 d/(1-b2^t)) / (sqrt(nv/(1-b3^t)) + eps)]_+ ."""
    diff = np.zeros_like(g) if g_prev is None else g - g_prev
    m = beta1 * m + (1.0 - beta1) * g
    d = beta2 * d + (1.0 - beta2) * diff
    u = g + beta2 * diff
    nv = beta3 * nv + (1.0 - beta3) * u * u
    step = (m / (1.0 - beta1 ** t) + beta2 * d / (1.0 - beta2 ** t)) / (np.sqrt(nv / (1.0 - beta3 ** t)) + eps)
    X = X - eta * step
    return (np.maximum(X, 0.0) if project else X), m, d, nv


def mu_update(H, SH, HG, eps):
    """Dampened multiplicative update (appendix family 1, He et al. 2011):
    H <- (1/2) H * (1 + SH / (H (H^T H) + eps)), eps = fp32 machine epsilon in
    the paper.  Keeps H >= 0 without a projection."""
    return 0.5 * H * (1.0 + SH / (HG + eps))


def admm_update(S, W, U, rho, SW=None):
    """One ADMM iteration (appendix family 6): the least-squares H of the
    bilinear surrogate ||S - H W^T||^2 with consensus penalty (eq. admm_H),
    the projection of H + U onto the non-negative orthant (eq. admm_W) and the
    scaled dual ascent (eq. admm_U).  Returns (W_next, U_next)."""
    SW = S @ W if SW is None else SW
    k = W.shape[1]
    M = 2.0 * (W.T @ W) + rho * np.eye(k)
    H = np.linalg.solve(M, (2.0 * SW + rho * (W - U)).T).T   # H M = 2 S W + rho (W - U)
    W_next = np.maximum(H + U, 0.0)
    return W_next, U + H - W_next


def lower_median(x):
    """Lower middle order statistic: element floor((m-1)/2) of the sorted values."""
    x = np.asarray(x, dtype=np.float64).ravel()
    return float(np.partition(x, (x.size - 1) // 2)[(x.size - 1) // 2])


def piecewise_reset(g, c):
    """Accumulator recalibration of Piecewise AdaGrad:
    G_i <- max(c g_i^2, c median(g^2))."""
    g2 = g * g
    return np.maximum(c * g2, c * lower_median(g2))


# ---------------------------------------------------------------------------
# Solver (state machine shared by every method).
# ---------------------------------------------------------------------------
ADAGRAD, RMSPROP, PIECEWISE_ADAGRAD, ROW_SVRG, BLOCK_SVRG, ADMM, ADAM, NADAM, ADAN, MU = range(10)


@dataclass
class Params:
    method: int = ADAGRAD
    softplus: bool = False
    eta: float = 0.02
    eps: float = 1e-10
    alpha: float = 0.99
    mu: float = 0.5
    c: float = 10.0            # Piecewise reset scale
    c_r: float = 10.0          # Piecewise gradient-margin gate
    eps_med: float = 1e-30     # Piecewise median floor
    row_frac: float = 0.5      # Row-SVRG |I| / n
    phi0: float = 0.75         # Block-SVRG initial coverage
    c_grow: float = 10.0       # AdaptGrow: grow only while KKT > c_grow * tau_g
    grow_checks: int = 3       # AdaptGrow: consecutive stagnating checks
    snapshot_s: int = 10
    block_rows: int = 1024
    independent_blocks: bool = True
    delta: int = 10
    warmup: int = 50
    max_iter: int = 1000
    tau_E: float = 0.1
    tau_g_inf: float = 1e-4
    n_ref: float = 1e4
    tau_stag: float = 1e-5
    seed: int = 0
    rho: float = 500.0         # ADMM consensus penalty
    beta1: float = 0.9         # Adam / NAdam / Adan first-moment decay
    beta2: float = 0.999       # Adam / NAdam second moment; Adan difference average
    beta3: float = 0.99        # Adan second moment


@dataclass
class Stats:
    t: int
    full: bool
    f: float = float("nan")
    E: float = float("nan")
    kkt: float = float("nan")
    stag: float = float("nan")
    phi: float = 1.0
    reset_fired: bool = False
    converged: bool = False


class Solver:
    """Plain FP64 SymNMF solver following the appendix update rules and the
    three-criterion stop rule.

    Iteration t reads H_t, forms g_t, records the statistics of H_t (full
    steps only: a sub-sampled step does not see all of S H) and writes
    H_{t+1}.  Readings where the paper is silent:

    * AdaGrad / RMSprop start from zero accumulators; eps is added outside
      the square root, as written in the appendix.
    * Piecewise AdaGrad: the reset is decided at a check iteration t from
      the statistics of H_t and replaces the accumulator after step t, so step
      t+1 adds g_{t+1}^2 to the recalibrated values.  Stagnation detection
      stays off until sum(G) reaches twice its post-reset value; a later
      reset fires only if E fell below E_at_last_reset * (1 - 10 tau),
      otherwise resets are disabled for good.
    * Row-Stochastic SVRG: snapshot (full) steps at t = 0 mod s; in between,
      the rows of ceil(row_frac * N_b) sampled blocks take their exact
      gradient and every other row takes its snapshot gradient mu.
    * Block-SVRG AdaptGrow: snapshot steps at t = 0 mod s and every step once
      phi = 1; otherwise I and J are ceil(sqrt(phi) N_b) sampled blocks each
      (J = I when ``independent_blocks`` is off); rows in I get
      2(H_I (H_J^T H_J) - S_IJ H_J), rows in J get 2(H_J (H_I^T H_I) - S_JI H_I)
      (rows in both get the sum), rows in neither take mu.  phi doubles (capped
      at 1) after ``grow_checks`` consecutive stagnating checks while the KKT
      measure is above c_grow * tau_g.
    * ADMM: W is the iterate (H_t above), U the scaled dual, both starting at
      (H0, 0); step t records the statistics of W_t (the paper tracks
      convergence on the feasible factor) and applies eqs. admm_H, admm_W,
      admm_U in that order.
    * Adam / NAdam / Adan: zero buffers, bias correction with the step count
      t + 1; Adan's first gradient difference is zero.  MU has no step size
      and no softplus form.
    """

    def __init__(self, S, k: int, params: Params, H0):
        if isinstance(S, StoredRows):       # full steps only (S @ H); see StoredRows
            self.S = S
            self.fro2 = S.fro2
        else:
            self.S = np.asarray(S, dtype=np.float64)
            self.fro2 = float((self.S * self.S).sum())
        self.n = self.S.shape[0]
        self.k = k
        self.p = params
        self.H = np.array(H0, dtype=np.float64).reshape(self.n, k)
        self.theta = softplus_inverse(self.H) if params.softplus else None
        if params.softplus:
            self.H = softplus(self.theta)
        self.G = np.zeros_like(self.H)       # AdaGrad accumulator (or RMSprop v)
        self.m = np.zeros_like(self.H)       # RMSprop momentum
        self.U = np.zeros_like(self.H)       # ADMM scaled dual
        self.d = np.zeros_like(self.H)       # Adan average of gradient differences
        self.nv = np.zeros_like(self.H)      # Adan second moment
        self.g_prev = None                   # Adan previous gradient
        if params.method == MU and params.softplus:
            raise ValueError("MU keeps H >= 0 by construction and has no softplus form")
        self.mu_snap = None
        self.t = 0
        self.phi = params.phi0 if params.method == BLOCK_SVRG else 1.0
        self.nb = -(-self.n // params.block_rows)
        self.E0 = None
        self.E_prev = None
        self.stag_run = 0
        self.pw_enabled = True
        self.pw_cooldown = None
        self.pw_E_reset = None
        self.pw_resets = 0
        self.last_g = None
        self.history = []

    def rebind(self, S):
        """Precision ladder (not in the paper; a remedy for the rounding of
        reduced-precision storage): continue the same iteration - iterate,
        optimiser buffers, t, E_0 - on another storage S of the matrix.  E is
        measured on the stored matrix, so the stagnation reference (E of the
        previous check, the Block-SVRG run of stagnating checks) restarts."""
        S = np.asarray(S, dtype=np.float64)
        if S.shape != self.S.shape:
            raise ValueError("rebind: S has another shape")
        self.S = S
        self.fro2 = float((S * S).sum())
        self.E_prev = None
        self.stag_run = 0

    # -- helpers ---------------------------------------------------------
    def _rows_of(self, blocks):
        br = self.p.block_rows
        mask = np.zeros(self.n, dtype=bool)
        for b in blocks:
            mask[b * br:(b + 1) * br] = True
        return mask

    def step_kind(self):
        p, t = self.p, self.t
        if p.method == ROW_SVRG:
            return "full" if t % p.snapshot_s == 0 else "row"
        if p.method == BLOCK_SVRG:
            return "full" if (self.phi >= 1.0 or t % p.snapshot_s == 0) else "block"
        return "full"

    def sampled_sets(self):
        p, t = self.p, self.t
        kind = self.step_kind()
        if kind == "row":
            m = min(self.nb, math.ceil(p.row_frac * self.nb))
            return sample_blocks(p.seed, t, 0, self.nb, m), None
        if kind == "block":
            m = min(self.nb, math.ceil(math.sqrt(self.phi) * self.nb))
            I = sample_blocks(p.seed, t, 0, self.nb, m)
            J = sample_blocks(p.seed, t, 1, self.nb, m) if p.independent_blocks else I
            return I, J
        return None, None

    def gradient_of_step(self):
        """(g, SH or None, kind) for the current iterate H_t."""
        S, H = self.S, self.H
        kind = self.step_kind()
        if kind == "full":
            SH = S @ H
            return gradient(S, H, SH), SH, kind
        I, J = self.sampled_sets()
        if kind == "row":
            rows = self._rows_of(I)
            g = self.mu_snap.copy()
            g[rows] = 4.0 * (H[rows] @ (H.T @ H) - S[rows] @ H)
            return g, None, kind
        rI, rJ = self._rows_of(I), self._rows_of(J)
        HI, HJ = H[rI], H[rJ]
        g = self.mu_snap.copy()
        g[rI | rJ] = 0.0
        g[rI] += 2.0 * (HI @ (HJ.T @ HJ) - S[np.ix_(rI, rJ)] @ HJ)
        g[rJ] += 2.0 * (HJ @ (HI.T @ HI) - S[np.ix_(rJ, rI)] @ HI)
        return g, None, kind

    # -- one iteration ---------------------------------------------------
    def step(self) -> Stats:
        p = self.p
        g, SH, kind = self.gradient_of_step()
        st = Stats(t=self.t, full=(kind == "full"), phi=self.phi)
        if kind == "full":
            st.f = objective_trace(self.S, self.H, SH)
            st.E = st.f / self.fro2
            st.kkt = kkt_measure(g, self.H, p.softplus)
            if p.method in (ROW_SVRG, BLOCK_SVRG):
                self.mu_snap = g.copy()
        self.last_g = g
        tb = self.t + 1                                        # bias-correction step count
        if p.method == ADMM:
            self.H, self.U = admm_update(self.S, self.H, self.U, p.rho, SH)
        elif p.method == MU:
            self.H = mu_update(self.H, SH, self.H @ (self.H.T @ self.H), p.eps)
        elif p.method in (ADAM, NADAM, ADAN):
            x = self.theta if p.softplus else self.H
            gx = g * sigmoid(self.theta) if p.softplus else g   # eq. logspace_grad
            if p.method == ADAN:
                x, self.m, self.d, self.nv = adan_update(x, self.m, self.d, self.nv, gx, self.g_prev, tb, p.eta,
                                                         p.eps, p.beta1, p.beta2, p.beta3,
                                                         project=not p.softplus)
                self.g_prev = gx
            else:
                x, self.m, self.G = adam_update(x, self.m, self.G, gx, tb, p.eta, p.eps, p.beta1, p.beta2,
                                                nesterov=p.method == NADAM, project=not p.softplus)
            if p.softplus:
                self.theta = x
                self.H = softplus(x)
            else:
                self.H = x
        elif p.softplus:
            g_theta = g * sigmoid(self.theta)                 # eq. logspace_grad
            if p.method == RMSPROP:
                self.theta, self.G, self.m = rmsprop_update(self.theta, self.G, self.m, g_theta,
                                                            p.eta, p.eps, p.alpha, p.mu, project=False)
            else:
                self.theta, self.G = adagrad_update(self.theta, self.G, g_theta, p.eta, p.eps, project=False)
            self.H = softplus(self.theta)
        elif p.method == RMSPROP:
            self.H, self.G, self.m = rmsprop_update(self.H, self.G, self.m, g, p.eta, p.eps, p.alpha, p.mu)
        else:
            self.H, self.G = adagrad_update(self.H, self.G, g, p.eta, p.eps)
        self.t += 1
        return st

    # -- the stop rule and the check-time controls ------------------------
    def check(self, st: Stats, H_prev) -> bool:
        """Apply the stop rule at a check iteration; returns True when converged."""
        p = self.p
        if self.E0 is None:
            self.E0 = st.E
        stag_ok = False
        if self.E_prev is not None:
            st.stag = (self.E_prev - st.E) / self.E0
            stag_ok = st.t >= p.warmup and st.stag < p.tau_stag
        tg = tau_g(self.n, p.tau_g_inf, p.n_ref)
        st.converged = st.E < p.tau_E and st.kkt < tg and stag_ok
        if not st.converged:
            if p.method == PIECEWISE_ADAGRAD:
                st.reset_fired = self._piecewise(st, stag_ok, tg)
            if p.method == BLOCK_SVRG and self.phi < 1.0:
                self.stag_run = self.stag_run + 1 if stag_ok else 0
                if self.stag_run >= p.grow_checks and st.kkt > p.c_grow * tg:
                    self.phi = min(2.0 * self.phi, 1.0)
                    self.stag_run = 0
        self.E_prev = st.E
        return st.converged

    def _piecewise(self, st, stag_ok, tg) -> bool:
        p = self.p
        if self.pw_cooldown is not None and self.G.sum() < self.pw_cooldown:
            return False
        if not (stag_ok and self.pw_enabled):
            return False
        g2med = lower_median(self.last_g * self.last_g)
        if not (st.kkt > p.c_r * tg and g2med > p.eps_med):
            return False
        if self.pw_resets > 0 and not (st.E < self.pw_E_reset * (1.0 - 10.0 * p.tau_stag)):
            self.pw_enabled = False
            return False
        self.G = piecewise_reset(self.last_g, p.c)
        self.pw_cooldown = 2.0 * self.G.sum()
        self.pw_E_reset = st.E
        self.pw_resets += 1
        return True

    def solve(self, max_iter=None, f_target: float = 0.0, rel_tol: float = 1e-4):
        """Iterate until the stop rule certifies an iterate, the objective
        reaches f_target*(1+rel_tol) (when f_target > 0), or max_iter steps.
        Returns (H_certified_or_last, last Stats)."""
        p = self.p
        max_iter = p.max_iter if max_iter is None else max_iter
        st = None
        while self.t < max_iter:
            H_prev = self.H
            st = self.step()
            self.history.append(st)
            if st.full and f_target > 0.0 and (st.f - f_target) / f_target <= rel_tol:
                return H_prev, st
            if st.t % p.delta == 0:
                if not st.full:
                    raise RuntimeError("check iteration without a full step: delta must be a multiple of s")
                if self.check(st, H_prev):
                    return H_prev, st
        return self.H, st
