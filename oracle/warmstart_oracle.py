"""FP64 oracle of the learned warm start (not in the paper: a per-row sketch
of S mapped by a small MLP to an initial H row).

TEST INFRASTRUCTURE ONLY - imported by tests/ and the smoke check, never by
the library.

Pieces, in the order the warm start applies them:
1. Gaussian sketch Omega (n x w): Box-Muller (Box & Muller 1958) on pairs of
   53-bit uniforms from SplitMix64 keyed by the seed; Y = S Omega.
2. Canonical coordinates: the top-k eigenpairs (lambda_c, v_c) of Y^T Y give
   whitened coordinates Z = Y V_k Lambda_k^-1/2 (each v_c signed so that
   sum_i (Y v_c)_i^3 > 0); the successive projection algorithm (Gillis &
   Vavasis 2014) picks k anchor rows of Z; rows are expressed in the anchor
   basis, C = Z A^-1, and padded with zeros to the network width.
3. MLP 64 -> 256 -> 256 -> k with exact GELU x Phi(x), softplus output; or,
   in the residual form, A = max(C + z, 0) with C the first k input
   coordinates and z the last layer's output (the network then learns a
   correction to the network-free start max(C, 0), which it reproduces
   exactly when the last layer is zero).
4. Scale: H0 = alpha A with alpha^2 = tr(A^T S A) / ||A^T A||_F^2, the
   minimiser of ||S - alpha^2 A A^T||_F^2 over alpha.
Training: permutation-invariant Gram loss
   L(A, B) = ||A A^T - B B^T||_F^2 = ||A^T A||^2 - 2 ||A^T B||^2 + ||B^T B||^2
with dL/dA = 4 (A (A^T A) - B (B^T A)), divided by ||B^T B||^2; AdamW
(Loshchilov & Hutter 2019) updates.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .symnmf_oracle import splitmix64

# --------------------------------------------------------------------------
# 1. sketch
# --------------------------------------------------------------------------
def uniform53(key, counter):
    """(top 53 bits of SplitMix64 output number counter) * 2^-53, in [0, 1)."""
    return (splitmix64(key, counter) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def omega(seed: int, n: int, width: int):
    """Omega_ij = sqrt(-2 ln(1 - u)) cos(2 pi v), u and v the uniforms of
    counters 2e and 2e + 1, e = i * width + j."""
    e = np.arange(n * width, dtype=np.uint64)
    u = uniform53(np.uint64(seed), 2 * e)
    v = uniform53(np.uint64(seed), 2 * e + np.uint64(1))
    return (np.sqrt(-2.0 * np.log(1.0 - u)) * np.cos(2.0 * math.pi * v)).reshape(n, width)


def sketch(S, Om):
    return np.asarray(S, dtype=np.float64) @ Om


# --------------------------------------------------------------------------
# 2. canonical coordinates
# --------------------------------------------------------------------------
def whiten(Y, k: int):
    """Z = Y V_k Lambda_k^-1/2 with the sign rule; returns (Z, M) with Z = Y M."""
    C = Y.T @ Y
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1][:k]
    lam, V = lam[order], V[:, order]
    proj = Y @ V
    s = np.sign((proj ** 3).sum(axis=0))
    s[s == 0] = 1.0
    M = V * (s / np.sqrt(lam))[None, :]
    return Y @ M, M


def spa(Z, k: int):
    """Successive projection algorithm: k row indices of Z.  At each step the
    row of largest residual norm (lowest index on ties) is taken and every row
    is projected onto the orthogonal complement of it."""
    R = np.array(Z, dtype=np.float64)
    idx = []
    for _ in range(k):
        nr = (R * R).sum(axis=1)
        i = int(np.argmax(nr))
        idx.append(i)
        u = R[i] / math.sqrt(nr[i])
        R = R - np.outer(R @ u, u)
    return np.array(idx)


def canonical_coordinates(Y, k: int, width: int = 64):
    Z, M = whiten(Y, k)
    anchors = spa(Z, k)
    A = Z[anchors]
    C = Z @ np.linalg.inv(A)
    X = np.zeros((Y.shape[0], width))
    X[:, :k] = C
    return X, anchors


# --------------------------------------------------------------------------
# 3. network
# --------------------------------------------------------------------------
def normal_cdf(x):
    """Phi(x) = erfc(-x / sqrt 2) / 2 (no cancellation in the lower tail)."""
    return 0.5 * erfc(-x / math.sqrt(2.0))


def gelu(x):
    return x * normal_cdf(x)


def gelu_grad(x):
    return normal_cdf(x) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def softplus(x):
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def init_params(k: int, seed: int = 0, width: int = 64, hidden: int = 256):
    """W_l ~ N(0, 1/fan_in) (from numpy's seeded generator: an input), b_l = 0."""
    g = np.random.default_rng(seed)
    return {
        "W1": g.normal(size=(hidden, width)) / math.sqrt(width), "b1": np.zeros(hidden),
        "W2": g.normal(size=(hidden, hidden)) / math.sqrt(hidden), "b2": np.zeros(hidden),
        "W3": g.normal(size=(k, hidden)) / math.sqrt(hidden), "b3": np.zeros(k),
    }


def init_params_counter(k: int, seed: int, width: int = 64, hidden: int = 256):
    """W_l = omega(4 seed + 1 + l, fan_out, fan_in) / sqrt(fan_in), b_l = 0:
    the normals of the sketch generator, so a network is reproducible from its
    seed alone."""
    shapes = [(hidden, width), (hidden, hidden), (k, hidden)]
    P = {}
    for l, (r, c) in enumerate(shapes):
        P[f"W{l + 1}"] = omega(4 * seed + 1 + l, r, c) / math.sqrt(c)
    P["b1"], P["b2"], P["b3"] = np.zeros(hidden), np.zeros(hidden), np.zeros(k)
    return P


def forward(P, X, residual: bool = False):
    z1 = X @ P["W1"].T + P["b1"]
    a1 = gelu(z1)
    z2 = a1 @ P["W2"].T + P["b2"]
    a2 = gelu(z2)
    z3 = a2 @ P["W3"].T + P["b3"]
    if residual:
        A = np.maximum(X[:, :z3.shape[1]] + z3, 0.0)
    else:
        A = softplus(z3)
    return A, dict(X=X, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, residual=residual)


def gram_loss(A, B):
    AtA, AtB, BtB = A.T @ A, A.T @ B, B.T @ B
    norm = (BtB * BtB).sum()
    L = ((AtA * AtA).sum() - 2.0 * (AtB * AtB).sum() + norm) / norm
    dA = 4.0 * (A @ AtA - B @ (B.T @ A)) / norm
    return L, dA


def gram_cos_loss(A, B):
    """Scale-free Gram loss: the residual of the best scalar fit,
        min_c ||c A A^T - B B^T||^2 / ||B B^T||^2 = 1 - <A A^T, B B^T>^2 / (||A A^T||^2 ||B B^T||^2),
    with <A A^T, B B^T> = ||A^T B||^2 and ||A A^T|| = ||A^T A||.  With
    a = ||A^T A||^2, b = ||A^T B||^2, c = ||B^T B||^2:
        dL/dA = (4 b / (a c)) ((b / a) A (A^T A) - B (B^T A))."""
    AtA, AtB, BtB = A.T @ A, A.T @ B, B.T @ B
    a, b, c = (AtA * AtA).sum(), (AtB * AtB).sum(), (BtB * BtB).sum()
    L = 1.0 - b * b / (a * c)
    dA = (4.0 * b / (a * c)) * ((b / a) * (A @ AtA) - B @ (B.T @ A))
    return L, dA


def backward(P, cache, dA):
    if cache.get("residual"):
        k = dA.shape[1]
        d3 = dA * (cache["X"][:, :k] + cache["z3"] > 0.0)
    else:
        d3 = dA * sigmoid(cache["z3"])
    g = {"W3": d3.T @ cache["a2"], "b3": d3.sum(axis=0)}
    da2 = d3 @ P["W3"]
    d2 = da2 * gelu_grad(cache["z2"])
    g["W2"] = d2.T @ cache["a1"]
    g["b2"] = d2.sum(axis=0)
    da1 = d2 @ P["W2"]
    d1 = da1 * gelu_grad(cache["z1"])
    g["W1"] = d1.T @ cache["X"]
    g["b1"] = d1.sum(axis=0)
    return g


def adamw_step(P, G, state, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-4):
    """One AdamW step (decoupled weight decay on W only), t = 1, 2, ..."""
    for name in P:
        m = state.setdefault("m_" + name, np.zeros_like(P[name]))
        v = state.setdefault("v_" + name, np.zeros_like(P[name]))
        m[...] = beta1 * m + (1 - beta1) * G[name]
        v[...] = beta2 * v + (1 - beta2) * G[name] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        if name.startswith("W"):
            P[name] = P[name] - lr * wd * P[name]
        P[name] = P[name] - lr * mh / (np.sqrt(vh) + eps)
    return P


# --------------------------------------------------------------------------
# 4. scale
# --------------------------------------------------------------------------
def alpha_rescale(S, A):
    SA = np.asarray(S, dtype=np.float64) @ A
    AtA = A.T @ A
    return math.sqrt(max((A * SA).sum(), 0.0) / (AtA * AtA).sum())


# --------------------------------------------------------------------------
# composed warm start
# --------------------------------------------------------------------------
def bf16_weights(P):
    """The network with W1..W3 rounded to bfloat16 (nearest even), biases kept."""
    from .symnmf_oracle import to_bf16
    return {name: (to_bf16(v) if name.startswith("W") else v) for name, v in P.items()}


def warm_start(S, k: int, seed: int, P=None, width: int = 64, residual: bool = False):
    """H0 = alpha A with A = network(canonical coordinates of S Omega) using the
    BF16-rounded weights, or A = the coordinates clipped at zero when P is None."""
    S = np.asarray(S, dtype=np.float64)
    Y = sketch(S, omega(seed, S.shape[0], width))
    X, anchors = canonical_coordinates(Y, k, width)
    if P is None:
        A = np.maximum(X[:, :k], 0.0)
    else:
        A, _ = forward(bf16_weights(P), X, residual)
    return alpha_rescale(S, A) * A, anchors
