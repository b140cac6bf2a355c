"""Seeded synthetic inputs for SymNMF: factor-model return panels.

This module only *makes inputs*.  It holds none of the factorisation
arithmetic (no correlation, no tail-dependence estimator, no objective, no
update rule): it draws a non-negative mixing matrix A and returns
``X = Z A^T + noise`` as a T x n float32 panel (rows are samples/days,
columns are instruments), together with the ground-truth labels and the
row permutation that was applied to A.  Both the HIP path and the CPU
oracle consume exactly the same X.

Recipes follow the paper's benchmark-construction appendix (factor model and
mixing matrix paragraph): a common factor with loading mean 0.8 and
Gaussian jitter 0.15, group factors with on-block loadings U[0.6, 1.8],
off-block jitter 0.05, block sizes within +-40% of n/groups, entries clamped
at zero, and rows of A randomly permuted before S is built.  The specific
instance families used by the tests and the benchmark are:

* ``c1_instance``  - 512 instruments, 8 equal planted groups, loadings
  U[0.3, 0.9], Gaussian factors and noise both scaled by 0.5, T = 2000.
* ``tpdm_returns`` - Student-t factors and 0.3 * Student-t noise (heavy
  tailed, so regularly varying), paper mixing recipe, optional common factor.
* ``overlap_returns`` - 32 (or 64) groups where every instrument has a primary
  group and, with probability 0.25, one random secondary group, plus a market
  factor of loading 0.4; Gaussian factors and noise scaled by 0.5.
* ``panel_returns`` - the same recipe generated in column blocks with one seed
  per block, so any column range can be regenerated on its own.
* ``paper_benchmark`` - the appendix's own benchmark matrices: floor(sqrt(n))
  groups plus the common factor, 40000 samples; Gaussian factors and unit
  Gaussian noise for the correlation type, i.i.d. Pareto(2) factors and
  0.3 * Pareto(2) noise for the TPDM type.

Randomness comes from torch's generators inside ``torch.random.fork_rng`` so
the global RNG state is untouched; a given (seed, device type) pair always
yields the same panel.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

__all__ = [
    "Instance", "c1_instance", "tpdm_returns", "overlap_returns",
    "panel_returns", "paper_benchmark", "planted_factor", "random_state",
]


@dataclass
class Instance:
    X: torch.Tensor          # T x n float32 returns panel
    labels: torch.Tensor     # n int64 primary group of each instrument (after permutation)
    perm: torch.Tensor       # n int64: column i of X is row perm[i] of the unpermuted A
    A: torch.Tensor          # n x m float32 mixing matrix after permutation


def _fork(device, seed):
    dev = torch.device(device)
    devices = [dev.index if dev.index is not None else 0] if dev.type == "cuda" else []
    ctx = torch.random.fork_rng(devices=devices)
    return ctx, dev


def _block_sizes(n: int, groups: int, jitter: float) -> torch.Tensor:
    """Sizes within +-jitter of n/groups that add up to n (uses the current RNG)."""
    if jitter == 0.0:
        base = torch.full((groups,), n // groups, dtype=torch.int64)
        base[: n - int(base.sum())] += 1
        return base
    u = 1.0 + jitter * (2.0 * torch.rand(groups, dtype=torch.float64) - 1.0)
    raw = u / u.sum() * n
    sizes = torch.floor(raw).to(torch.int64).clamp_min(1)
    short = n - int(sizes.sum())
    order = torch.argsort(raw - torch.floor(raw), descending=True)
    i = 0
    while short != 0:
        j = int(order[i % groups])
        step = 1 if short > 0 else -1
        if sizes[j] + step >= 1:
            sizes[j] += step
            short -= step
        i += 1
    return sizes


def _student_t(shape, nu: float, device) -> torch.Tensor:
    dist = torch.distributions.StudentT(torch.tensor(float(nu), dtype=torch.float64, device=device))
    return dist.sample(shape).to(torch.float32)


def c1_instance(seed: int = 0, T: int = 2000, n: int = 512, groups: int = 8,
                device="cpu") -> Instance:
    """Equal planted groups, loadings U[0.3,0.9], F and E i.i.d. 0.5*N(0,1)."""
    ctx, dev = _fork(device, seed)
    with ctx:
        torch.manual_seed(seed)
        sizes = _block_sizes(n, groups, 0.0)
        labels0 = torch.repeat_interleave(torch.arange(groups), sizes)
        A0 = torch.zeros(n, groups, dtype=torch.float32)
        A0[torch.arange(n), labels0] = 0.3 + 0.6 * torch.rand(n)
        perm = torch.randperm(n)
        A = A0[perm].contiguous()
        labels = labels0[perm].contiguous()
        F = 0.5 * torch.randn(T, groups, device=dev)
        E = 0.5 * torch.randn(T, n, device=dev)
        X = F @ A.to(dev).T + E
    return Instance(X.contiguous(), labels, perm, A)


def _paper_mixing(n: int, groups: int, common: bool, jitter: float = 0.4) -> tuple:
    """Mixing matrix of the paper's recipe (uses the current CPU RNG)."""
    sizes = _block_sizes(n, groups, jitter)
    labels0 = torch.repeat_interleave(torch.arange(groups), sizes)
    m = groups + (1 if common else 0)
    off = 1 if common else 0
    A0 = 0.05 * torch.randn(n, m)
    A0[torch.arange(n), labels0 + off] = 0.6 + 1.2 * torch.rand(n)
    if common:
        A0[:, 0] = 0.8 + 0.15 * torch.randn(n)
    A0.clamp_(min=0.0)
    perm = torch.randperm(n)
    return A0[perm].contiguous(), labels0[perm].contiguous(), perm


def tpdm_returns(seed: int = 0, T: int = 20000, n: int = 4096, groups: int = 16,
                 nu: float = 3.0, common: bool = False, noise: float = 0.3,
                 device="cpu") -> Instance:
    """Heavy-tailed factor model: Student-t(nu) factors, noise*Student-t(nu) noise."""
    ctx, dev = _fork(device, seed)
    with ctx:
        torch.manual_seed(seed)
        A, labels, perm = _paper_mixing(n, groups, common)
        Z = _student_t((T, A.shape[1]), nu, dev)
        X = Z @ A.to(dev).T
        del Z
        X += noise * _student_t((T, n), nu, dev)
    return Instance(X.contiguous(), labels, perm, A)


def overlap_returns(seed: int = 0, T: int = 2500, n: int = 100000, groups: int = 32,
                    market: float = 0.4, p_second: float = 0.25, scale: float = 0.5,
                    device="cpu") -> Instance:
    """Overlapping groups plus a market factor; Gaussian factors and noise."""
    ctx, dev = _fork(device, seed)
    with ctx:
        torch.manual_seed(seed)
        sizes = _block_sizes(n, groups, 0.4)
        labels0 = torch.repeat_interleave(torch.arange(groups), sizes)
        A0 = torch.zeros(n, groups + 1)
        A0[:, 0] = market
        rows = torch.arange(n)
        A0[rows, labels0 + 1] = 0.3 + 0.6 * torch.rand(n)
        second = torch.rand(n) < p_second
        g2 = torch.randint(0, groups, (n,))
        g2 = torch.where(g2 == labels0, (g2 + 1) % groups, g2)
        val2 = 0.3 + 0.6 * torch.rand(n)
        A0[rows[second], g2[second] + 1] = val2[second]
        perm = torch.randperm(n)
        A = A0[perm].contiguous()
        labels = labels0[perm].contiguous()
        F = scale * torch.randn(T, groups + 1, device=dev)
        X = F @ A.to(dev).T
        X += scale * torch.randn(T, n, device=dev)
    return Instance(X.contiguous(), labels, perm, A)


def panel_returns(seed: int = 0, T: int = 1000, n: int = 1_000_000, groups: int = 64,
                  market: float = 0.4, scale: float = 0.5, block: int = 65536,
                  col0: int = 0, cols: int | None = None, device="cpu") -> Instance:
    """Column-block generated panel: block b of columns uses seed (seed, b).

    Group membership is drawn i.i.d. uniformly per instrument (so no global
    permutation is needed and any column block can be regenerated alone);
    each instrument has one group loading U[0.3, 0.9] plus the market loading.
    The factor path F (T x (groups+1)) is shared by every block and uses
    ``seed`` itself.
    """
    cols = n - col0 if cols is None else cols
    dev = torch.device(device)
    ctx, _ = _fork(device, seed)
    with ctx:
        torch.manual_seed(seed)
        F = scale * torch.randn(T, groups + 1, device=dev)
    X = torch.empty(T, cols, dtype=torch.float32, device=dev)
    labels = torch.empty(cols, dtype=torch.int64)
    A = torch.empty(cols, groups + 1, dtype=torch.float32)
    b0, b1 = col0 // block, (col0 + cols - 1) // block
    for b in range(b0, b1 + 1):
        lo, hi = b * block, min((b + 1) * block, n)
        ctx, _ = _fork(device, seed)
        with ctx:
            torch.manual_seed((seed * 1_000_003 + 7919 * (b + 1)) % (2 ** 63))
            m = hi - lo
            lab = torch.randint(0, groups, (m,))
            Ab = torch.zeros(m, groups + 1)
            Ab[:, 0] = market
            Ab[torch.arange(m), lab + 1] = 0.3 + 0.6 * torch.rand(m)
            Xb = F @ Ab.to(dev).T + scale * torch.randn(T, m, device=dev)
        s0, s1 = max(lo, col0), min(hi, col0 + cols)
        X[:, s0 - col0:s1 - col0] = Xb[:, s0 - lo:s1 - lo]
        labels[s0 - col0:s1 - col0] = lab[s0 - lo:s1 - lo]
        A[s0 - col0:s1 - col0] = Ab[s0 - lo:s1 - lo]
    return Instance(X, labels, torch.arange(col0, col0 + cols), A)


def _pareto2(shape, device) -> torch.Tensor:
    """Standard Pareto(alpha=2) draws, P(X > x) = x^-2 for x >= 1."""
    return (1.0 - torch.rand(shape, dtype=torch.float64, device=device)) ** -0.5


def paper_benchmark(seed: int, n: int, kind: str, T: int = 40000, device="cpu") -> Instance:
    """X = Z A^T + noise with the appendix's mixing matrix (common factor plus
    floor(sqrt(n)) groups).  kind "corr": Z ~ N(0, 1), noise ~ N(0, 1);
    kind "tpdm": Z ~ Pareto(2), noise ~ 0.3 Pareto(2), all i.i.d."""
    if kind not in ("corr", "tpdm"):
        raise ValueError(kind)
    ctx, dev = _fork(device, seed)
    with ctx:
        torch.manual_seed(seed)
        A, labels, perm = _paper_mixing(n, int(math.isqrt(n)), True)
        Ad = A.to(dev, torch.float64)
        if kind == "corr":
            X = torch.randn(T, A.shape[1], dtype=torch.float64, device=dev) @ Ad.T
            X += torch.randn(T, n, dtype=torch.float64, device=dev)
        else:
            X = _pareto2((T, A.shape[1]), dev) @ Ad.T
            X += 0.3 * _pareto2((T, n), dev)
    return Instance(X.float().contiguous(), labels, perm, A)


def planted_factor(seed: int, n: int, k: int, anchor_scale: float = 1.0) -> torch.Tensor:
    """A separable non-negative H* (n x k, float64): the first k rows are
    scaled unit rows (anchors), the rest are sparse non-negative mixtures.
    S = H* H*^T then has an exact rank-k SymNMF with a (near) unique solution."""
    g = torch.Generator().manual_seed(seed)
    H = torch.rand(n, k, generator=g, dtype=torch.float64)
    H *= (torch.rand(n, k, generator=g, dtype=torch.float64) < 0.5)
    H[:k] = anchor_scale * torch.eye(k, dtype=torch.float64)
    H[k:] /= math.sqrt(k)
    return H


def random_state(seed: int, shape, lo: float = 0.0, hi: float = 1.0,
                 dtype=torch.float32) -> torch.Tensor:
    """Uniform test state (e.g. an H or an accumulator) from a seeded CPU generator."""
    g = torch.Generator().manual_seed(seed)
    return (lo + (hi - lo) * torch.rand(*shape, generator=g, dtype=torch.float64)).to(dtype)
