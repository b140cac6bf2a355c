"""Plain FP64 CPU oracle of spherical K-means (Lloyd) on the rows of S.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the product path never
calls it, and it shares no code with the HIP path.

What it follows (paper, section "Clustering"):

* Spherical K-means partitions unit vectors by cosine similarity; the
  centroid of a cluster is the normalised sum of its members, and the
  objective is the total angular dissimilarity, sum_i (1 - cos) (subsection
  "Spherical K-means as constrained SymNMF", Theorem snmf_spkmeans).
* It is run with Lloyd's alternation on the rows of S, which are first
  scaled to unit length; it stops when the relative drop of sum_i (1 - cos)
  falls below 1e-4, which also happens once the assignments are stable
  (subsection "Computational Comparison").
* Partitions are scored by the silhouette with cosine distance (same
  subsection, table tab:kmeans).
* The spectral diagnostic of the collapse of angular clustering on a matrix
  dominated by one common factor: the norm-weighted mean of sin^2 of the
  angle between the rows and the leading eigenvector equals
  (||S||_F^2 - lambda_1^2) / ||S||_F^2 and is bounded by (r_eff - 1)^2 with
  r_eff = tr(S) / lambda_1 (eq. angular_collapse).

Readings where the paper is silent:

* Seeding: the K initial centroids are K distinct rows of S drawn uniformly
  without replacement (Forgy seeding) by a partial Fisher-Yates shuffle
  driven by SplitMix64 (the generator of the rest of the oracle), 53-bit
  uniforms; or k-means++ rows (``kmeanspp_rows``), whose silhouettes come
  much closer to the values the paper prints; an explicit list of rows may
  be given instead.
* Ties in the assignment go to the lowest cluster index.
* A cluster that loses all its members keeps its previous centroid.
* The iteration count is the number of (centroid update, assignment) pairs
  after the initial assignment; the run stops at the first iteration whose
  objective J_t satisfies J_{t-1} - J_t < tol * J_{t-1} (or J_{t-1} = 0).
"""
from __future__ import annotations

import numpy as np

from .symnmf_oracle import splitmix64


def uniform53(key, counter):
    """(top 53 bits of SplitMix64 output number counter) * 2^-53, in [0, 1)."""
    return (splitmix64(key, counter) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def seed_rows(seed: int, n: int, K: int) -> np.ndarray:
    """K distinct rows of [0, n): partial Fisher-Yates shuffle (Knuth, TAOCP
    vol. 2, Algorithm P) - for i = 0..K-1 swap position i with position
    i + floor(u_i (n - i)), u_i the i-th 53-bit uniform of the stream keyed
    by seed.  Returned in draw order (cluster c is seeded by entry c)."""
    if not 1 <= K <= n:
        raise ValueError("need 1 <= K <= n")
    a = np.arange(n, dtype=np.int64)
    key = np.uint64(seed & (2**64 - 1))
    for i in range(K):
        u = float(uniform53(key, i))
        j = min(i + int(u * (n - i)), n - 1)
        a[i], a[j] = a[j], a[i]
    return a[:K].copy()


def kmeanspp_rows(S, K: int, seed: int = 0) -> np.ndarray:
    """k-means++ seeding (Arthur & Vassilvitskii 2007) on the unit rows of S,
    where the squared Euclidean distance of unit vectors is 2 (1 - cos): the
    first seed is row floor(u_0 n); seed i is the smallest j with
    sum_{l <= j} d_l > u_i sum_l d_l, d_l = min over the seeds so far of
    (1 - cos) (negative rounding clamped to 0, and exactly 0 at the seeds),
    u_i the i-th 53-bit uniform of the SplitMix64 stream keyed by seed.  If
    every d is 0 (fewer distinct rows than K), the lowest unchosen row is
    taken."""
    Shat, _ = unit_rows(S)
    n = Shat.shape[0]
    if not 1 <= K <= n:
        raise ValueError("need 1 <= K <= n")
    key = np.uint64(seed & (2**64 - 1))
    first = min(int(float(uniform53(key, 0)) * n), n - 1)
    rows = [first]
    chosen = np.zeros(n, dtype=bool)
    chosen[first] = True
    d = np.where(chosen, 0.0, np.maximum(1.0 - Shat @ Shat[first], 0.0))
    for i in range(1, K):
        total = float(d.sum())
        if total > 0.0:
            target = float(uniform53(key, i)) * total
            j = int(np.searchsorted(np.cumsum(d), target, side="right"))
            j = min(j, n - 1)
        else:
            j = int(np.flatnonzero(~chosen)[0])
        rows.append(j)
        chosen[j] = True
        d = np.where(chosen, 0.0, np.minimum(d, np.maximum(1.0 - Shat @ Shat[j], 0.0)))
    return np.array(rows, dtype=np.int64)


def unit_rows(S):
    """Rows of S scaled to unit Euclidean length, and the row lengths."""
    S = np.asarray(S, dtype=np.float64)
    norms = np.sqrt(np.sum(S * S, axis=1))
    if np.any(norms == 0.0):
        raise ValueError("a zero row of S has no direction")
    return S / norms[:, None], norms


def assign(Shat, C):
    """Lloyd's assignment step.  Shat: n x m unit rows; C: K x m unit
    centroids.  Returns (labels, best cosine, J = sum_i (1 - best cosine)),
    ties to the lowest cluster index (np.argmax returns the first maximum)."""
    cos = Shat @ C.T
    labels = np.argmax(cos, axis=1).astype(np.int64)
    best = cos[np.arange(Shat.shape[0]), labels]
    return labels, best, float(np.sum(1.0 - best))


def centroids(Shat, labels, K: int, C_prev):
    """Lloyd's update step: c_k = (sum of the member rows) / ||that sum||;
    a cluster without members keeps C_prev[k]."""
    C = np.array(C_prev, dtype=np.float64, copy=True)
    for c in range(K):
        members = labels == c
        if not np.any(members):
            continue
        m = Shat[members].sum(axis=0)
        C[c] = m / np.linalg.norm(m)
    return C


def objective(Shat, labels, C):
    """sum_i (1 - cos(s_i, c_{label_i}))."""
    return float(np.sum(1.0 - np.einsum("ij,ij->i", Shat, C[labels])))


def lloyd(S, K: int, seed: int = 0, tol: float = 1e-4, max_iter: int = 100, init_rows=None):
    """Spherical K-means on the rows of S from Forgy seeds.

    Returns a dict with the final labels, centroids (K x n), objective J,
    the objective of every assignment (J_0 first), the iteration count and
    whether the stop rule fired within max_iter."""
    Shat, _ = unit_rows(S)
    n = Shat.shape[0]
    rows = seed_rows(seed, n, K) if init_rows is None else np.asarray(init_rows, dtype=np.int64)
    if rows.shape != (K,) or len(set(rows.tolist())) != K:
        raise ValueError("init_rows must hold K distinct rows")
    C = Shat[rows].copy()
    labels, best, J = assign(Shat, C)
    history = [J]
    converged = False
    it = 0
    while it < max_iter:
        C = centroids(Shat, labels, K, C)
        labels, best, J_new = assign(Shat, C)
        it += 1
        history.append(J_new)
        stop = J <= 0.0 or (J - J_new) < tol * J
        J = J_new
        if stop:
            converged = True
            break
    return {"labels": labels, "C": C, "J": J, "history": history, "iters": it, "converged": converged,
            "best": best, "init_rows": rows}


def cluster_sums(Shat, labels, K: int):
    """m_k = sum of the unit rows in cluster k (K x m) and the cluster sizes."""
    M = np.zeros((K, Shat.shape[1]))
    for c in range(K):
        M[c] = Shat[labels == c].sum(axis=0)
    return M, np.bincount(labels, minlength=K)


def silhouette_cosine(S, labels):
    """Mean silhouette of the partition of the rows of S under the cosine
    distance d(i, j) = 1 - cos(s_i, s_j), from the definition (Rousseeuw
    1987): a(i) is the mean distance to the other members of i's cluster,
    b(i) the smallest mean distance to another non-empty cluster,
    s(i) = (b - a) / max(a, b), and s(i) = 0 for a member of a singleton.
    Brute force over all pairs (small n only)."""
    Shat, _ = unit_rows(S)
    labels = np.asarray(labels, dtype=np.int64)
    n = Shat.shape[0]
    D = 1.0 - Shat @ Shat.T
    present = np.unique(labels)
    if present.size < 2:
        raise ValueError("the silhouette needs at least two non-empty clusters")
    s = np.zeros(n)
    for i in range(n):
        same = labels == labels[i]
        same[i] = False
        if not np.any(same):
            continue
        a = D[i, same].mean()
        b = min(D[i, labels == c].mean() for c in present if c != labels[i])
        s[i] = (b - a) / max(a, b)
    return float(s.mean())


def angular_collapse(S):
    """The collapse diagnostic of eq. angular_collapse for symmetric S.

    Returns (lhs, spectral, bound, r_eff, lambda_1):
    lhs = sum_i ||s_i||^2 sin^2(theta_i) / sum_i ||s_i||^2 with theta_i the
    angle between row i and the leading eigenvector u_1, computed from the
    rows; spectral = (||S||_F^2 - lambda_1^2) / ||S||_F^2;
    bound = (r_eff - 1)^2 with r_eff = tr(S) / lambda_1."""
    S = np.asarray(S, dtype=np.float64)
    lam, U = np.linalg.eigh(S)
    j = int(np.argmax(lam))
    lam1, u1 = float(lam[j]), U[:, j]
    rn2 = np.sum(S * S, axis=1)
    cos2 = (S @ u1) ** 2 / rn2
    lhs = float(np.sum(rn2 * (1.0 - cos2)) / np.sum(rn2))
    fro2 = float(np.sum(S * S))
    spectral = (fro2 - lam1 * lam1) / fro2
    r_eff = float(np.trace(S)) / lam1
    return lhs, spectral, (r_eff - 1.0) ** 2, r_eff, lam1
