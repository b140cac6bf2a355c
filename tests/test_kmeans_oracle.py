"""Pins of the spherical K-means oracle (CPU).

The oracle is checked against what the definitions and the paper fix, not
against itself: the published SplitMix64 outputs, scikit-learn's silhouette,
an exhaustive search over all partitions of a tiny instance, the identity
J = n - sum_k ||m_k|| of the clustering section, Lloyd's monotonicity and
fixed point, exact recovery of planted blocks, and the spectral identity and
bound of eq. angular_collapse (eigenvalues from LAPACK)."""
import itertools
import math

import numpy as np
import pytest
import sklearn.metrics

import oracle.kmeans_oracle as km
import synth
from oracle import abs_corr, tpdm


def _clustered(seed, n_per, groups, dim, spread):
    """Rows scattered around `groups` random directions (a small S stand-in)."""
    g = np.random.default_rng(seed)
    centres = np.zeros((groups, dim))
    for c in range(groups):                      # disjoint supports
        lo, hi = c * dim // groups, (c + 1) * dim // groups
        centres[c, lo:hi] = 1.0 + g.random(hi - lo)
    rows = [centres[c] + spread * g.standard_normal((n_per, dim)) for c in range(groups)]
    X = np.abs(np.concatenate(rows))
    return X, np.repeat(np.arange(groups), n_per)


def test_seed_rows_first_draw_from_published_generator(golden_dir):
    vals = {}
    for line in open(f"{golden_dir}/splitmix64_seed0.txt"):
        if line.startswith("#") or not line.strip():
            continue
        c, v = line.split()
        vals[int(c)] = int(v, 16)
    n = 1000
    rows = km.seed_rows(0, n, 2)
    # first swap position: floor(u_0 n) with u_0 the top 53 bits of output 0
    assert rows[0] == (vals[0] >> 11) * n // 2**53
    # second: position 1 + floor(u_1 (n - 1)); the element there is itself
    # unless the first swap moved it
    j1 = 1 + (vals[1] >> 11) * (n - 1) // 2**53
    assert rows[1] == (0 if j1 == rows[0] else j1)


def test_seed_rows_distinct_uniform_and_full_permutation():
    r = km.seed_rows(11, 5000, 300)
    assert len(set(r.tolist())) == 300 and r.min() >= 0 and r.max() < 5000
    assert sorted(km.seed_rows(3, 64, 64).tolist()) == list(range(64))
    first = np.array([km.seed_rows(s, 10, 1)[0] for s in range(4000)])
    counts = np.bincount(first, minlength=10)
    chi2 = float(((counts - 400.0) ** 2 / 400.0).sum())
    assert chi2 < 30.0          # 9 degrees of freedom: p ~ 4e-4 at 30


def test_silhouette_matches_scikit_learn():
    X, _ = _clustered(1, 20, 4, 30, 0.6)
    S = X @ X.T
    res = km.lloyd(S, 4, seed=2)
    ours = km.silhouette_cosine(S, res["labels"])
    ref = sklearn.metrics.silhouette_score(S, res["labels"], metric="cosine")
    assert ours == pytest.approx(ref, rel=1e-12, abs=1e-14)
    # a singleton cluster scores 0 in both
    labels = res["labels"].copy()
    labels[0] = 4
    assert km.silhouette_cosine(S, labels) == pytest.approx(
        sklearn.metrics.silhouette_score(S, labels, metric="cosine"), rel=1e-12)


def test_objective_is_n_minus_sum_of_cluster_sum_norms():
    # spherical K-means maximises sum_k ||m_k||: with normalised-sum
    # centroids the objective is n - sum_k ||m_k|| for any partition
    X, _ = _clustered(4, 15, 3, 12, 0.8)
    Shat, _ = km.unit_rows(X @ X.T)
    g = np.random.default_rng(0)
    for _ in range(5):
        labels = g.integers(0, 3, Shat.shape[0])
        C = km.centroids(Shat, labels, 3, np.zeros((3, Shat.shape[1])))
        M, _ = km.cluster_sums(Shat, labels, 3)
        expect = Shat.shape[0] - sum(np.linalg.norm(M[c]) for c in range(3))
        assert km.objective(Shat, labels, C) == pytest.approx(expect, rel=1e-13)


def test_lloyd_reaches_the_exhaustive_optimum_of_a_tiny_instance():
    X, truth = _clustered(7, 3, 3, 6, 0.35)
    S = X @ X.T
    Shat, _ = km.unit_rows(S)
    n = Shat.shape[0]
    best, best_lab = math.inf, None
    for lab in itertools.product(range(3), repeat=n):
        lab = np.array(lab)
        if len(set(lab.tolist())) < 3:
            continue
        M, _ = km.cluster_sums(Shat, lab, 3)
        val = n - sum(np.linalg.norm(M[c]) for c in range(3))
        if val < best - 1e-12:
            best, best_lab = val, lab
    # Lloyd's result is never below the optimum, and the best of all
    # seedings reaches it with the same partition (up to cluster names)
    runs = [km.lloyd(S, 3, init_rows=list(rows), tol=1e-12) for rows in itertools.combinations(range(n), 3)]
    assert min(r["J"] for r in runs) >= best - 1e-12
    top = min(runs, key=lambda r: r["J"])
    assert top["J"] == pytest.approx(best, rel=1e-12)
    assert sklearn.metrics.adjusted_rand_score(best_lab, top["labels"]) == 1.0
    assert sklearn.metrics.adjusted_rand_score(truth, top["labels"]) == 1.0


def test_lloyd_is_monotone_and_ends_at_a_fixed_point():
    inst = synth.c1_instance(0, T=2000, n=512, groups=8)
    S = abs_corr(inst.X.double().numpy())
    res = km.lloyd(S, 8, seed=5, tol=1e-15, max_iter=200)
    h = np.array(res["history"])
    assert np.all(np.diff(h) <= 1e-9 * h[0])
    assert res["converged"] and h[-1] == pytest.approx(h[-2], rel=1e-14, abs=0)
    Shat, _ = km.unit_rows(S)
    labels, _, J = km.assign(Shat, res["C"])
    assert np.array_equal(labels, res["labels"]) and J == pytest.approx(res["J"], rel=1e-14)
    C2 = km.centroids(Shat, res["labels"], 8, res["C"])
    assert np.allclose(C2, res["C"], rtol=0, atol=1e-12)


def test_planted_groups_are_recovered_from_one_seed_per_group():
    inst = synth.c1_instance(0, T=2000, n=512, groups=8)
    S = abs_corr(inst.X.double().numpy())
    truth = inst.labels.numpy()
    init = [int(np.flatnonzero(truth == c)[0]) for c in range(8)]
    res = km.lloyd(S, 8, init_rows=init)
    assert np.array_equal(res["labels"], truth)


def test_planted_blocks_exact():
    # block-diagonal S with identical rows inside each block: J = 0 at once
    sizes = [5, 9, 4]
    n = sum(sizes)
    S = np.zeros((n, n))
    o = 0
    for b, s in enumerate(sizes):
        S[o:o + s, o:o + s] = 0.5 + b
        o += s
    res = km.lloyd(S, 3, init_rows=[0, 5, 14])
    assert res["history"][0] < 1e-13 and res["iters"] == 1 and res["converged"]
    assert np.array_equal(res["labels"], np.repeat([0, 1, 2], sizes))
    assert km.silhouette_cosine(S, res["labels"]) == pytest.approx(1.0, abs=1e-14)


def test_empty_cluster_keeps_its_centroid_and_ties_go_low():
    # dyadic unit vectors: every cosine below is exact, so the ties are exact
    Shat = np.array([[0.5, 0.5, 0.5, 0.5], [1.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 1.0]])
    C = np.array([[0.5, 0.5, 0.5, 0.5], [0.5, 0.5, 0.5, 0.5], [0.0, 0.0, 0.0, 1.0]])
    labels, best, J = km.assign(Shat, C)
    assert labels.tolist() == [0, 0, 2] and best.tolist() == [1.0, 0.5, 1.0] and J == 0.5
    C2 = km.centroids(Shat, labels, 3, C)
    assert np.array_equal(C2[1], C[1])                       # no members: kept
    m0 = Shat[0] + Shat[1]
    assert np.allclose(C2[0], m0 / np.linalg.norm(m0), rtol=0, atol=1e-15)


def test_angular_collapse_identity_and_bound():
    inst = synth.tpdm_returns(0, T=4000, n=200, groups=4, nu=3.0, common=True)
    S = tpdm(inst.X.double().numpy(), 0.05)
    lhs, spectral, bound, r_eff, lam1 = km.angular_collapse(S)
    assert lhs == pytest.approx(spectral, rel=1e-10)
    assert lhs <= bound and 1.0 < r_eff < 200
    assert lam1 == pytest.approx(np.linalg.eigvalsh(S)[-1], rel=1e-12)
    # rank one and positive: every row on u_1, no angular spread, r_eff = 1
    u = np.abs(np.random.default_rng(0).standard_normal(50)) + 0.1
    lhs1, spec1, bound1, r1, _ = km.angular_collapse(np.outer(u, u))
    assert abs(lhs1) < 1e-12 and abs(spec1) < 1e-12 and r1 == pytest.approx(1.0, rel=1e-12)


def test_kmeanspp_first_draw_and_second_draw_distribution():
    # the first seed is floor(u_0 n); the second is drawn with probability
    # proportional to 1 - cos to the first (k-means++ on unit vectors)
    X, _ = _clustered(3, 4, 3, 9, 0.3)
    S = X @ X.T
    Shat, _ = km.unit_rows(S)
    n = S.shape[0]
    counts = np.zeros(n)
    first_row = None
    firsts = []
    for seed in range(3000):
        r = km.kmeanspp_rows(S, 2, seed)
        firsts.append(r[0])
        if r[0] == 0:
            counts[r[1]] += 1
    firsts = np.bincount(firsts, minlength=n)
    assert abs(firsts.mean() - 3000 / n) < 1e-9 and firsts.min() > 0.5 * 3000 / n
    d = np.maximum(1.0 - Shat @ Shat[0], 0.0)
    expect = d / d.sum() * counts.sum()
    assert counts[0] == 0
    chi2 = float(((counts - expect)[expect > 0] ** 2 / expect[expect > 0]).sum())
    assert chi2 < 40.0           # 10 degrees of freedom


def test_kmeanspp_seeds_every_planted_group():
    X, truth = _clustered(5, 30, 6, 24, 0.3)
    S = X @ X.T
    hits, forgy = 0, 0
    for seed in range(20):
        rows = km.kmeanspp_rows(S, 6, seed)
        assert len(set(rows.tolist())) == 6
        hits += len(set(truth[rows].tolist())) == 6
        forgy += len(set(truth[km.seed_rows(seed, S.shape[0], 6)].tolist())) == 6
    # uniform draws cover all six groups with probability 6!/6^6 = 1.5 %;
    # distance-weighted draws favour rows far from the seeds so far
    assert hits >= 14 and forgy <= 3
    # duplicate rows only: the zero-distance fallback takes the lowest unchosen rows
    Sd = np.ones((5, 5))
    assert sorted(km.kmeanspp_rows(Sd, 3, 1).tolist()) == sorted(set(km.kmeanspp_rows(Sd, 3, 1).tolist()))
