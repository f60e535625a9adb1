"""Pins of the FP64 oracle to things other than itself (CPU only).

Each test ties one part of the oracle to an independent fact: a hand-derived
worked example, a pure-Python brute force, a library routine (scipy's cdist on
materialised trajectory tensors), the paper's recurrence (Eq. 5) written out
separately, the Gram identity (Eq. 4), exact invariances on integer-valued data,
the k-prefix property (Discussion, "Practical Insight"), the k = 1 matrix-profile
special case (Discussion, "Relation to Matrix Profile"), a planted rare
trajectory, and finite differences of the objective for the gradient.

A plausible slip in the oracle (a dropped term, a wrong sign or index, an
off-by-one exclusion, the wrong tie rule, a transposed operand) fails at least
one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from paper_2603_02059_amd import synth


def _int_fields(T, D, seed, lo=-50, hi=50):
    """Integer-valued fields: every sum the oracle forms is exact in FP64, so
    invariances that only reorder arithmetic must hold bitwise."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(T, D)).astype(np.float64)


# --------------------------------------------------------------------------
# P1: hand-derived worked example (fixture carries its derivation)
# --------------------------------------------------------------------------
def test_worked_example(golden_dir):
    with open(os.path.join(golden_dir, "worked_example.json")) as f:
        g = json.load(f)
    x = np.array(g["x"], dtype=np.float64)[:, None]
    L = g["L"]
    for case in g["cases"]:
        idx, dist, score, gap = oracle.knn(x, L, case["k"])
        np.testing.assert_array_equal(idx, np.array(case["idx"]))
        np.testing.assert_array_equal(dist, np.array(case["dist"], dtype=float))
        np.testing.assert_array_equal(score, np.array(case["score"], dtype=float))
        # the gap decides which set differences the parity rule admits: one
        # division of exact integers, so bitwise
        want = [math.inf if q == "inf" else q[0] / q[1] for q in case["gap"]]
        assert gap.tolist() == want
    gc = g["grad_case"]
    idx, _, _, _ = oracle.knn(x, L, gc["k"])
    grad = oracle.score_grad(x, L, gc["k"], idx, np.array(gc["weights"], float))
    np.testing.assert_array_equal(grad[:, 0], np.array(gc["grad"], dtype=float))


# --------------------------------------------------------------------------
# Pure-Python brute force on a tiny input (no numpy in the arithmetic)
# --------------------------------------------------------------------------
def _py_knn(xs, L, k):
    T = len(xs)
    n = T - L + 1
    out = []
    for t in range(n):
        cands = []
        for j in range(n):
            if abs(t - j) < L:
                continue
            d = 0.0
            for m in range(L):
                for a, b in zip(xs[t + m], xs[j + m]):
                    d += (a - b) * (a - b)
            cands.append((d, j))
        cands.sort()
        best = cands[:k]
        if len(cands) > k:
            dk, dk1 = cands[k - 1][0], cands[k][0]
            gap = (dk1 - dk) / dk if dk > 0 else (math.inf if dk1 > 0 else 0.0)
        else:
            gap = math.inf
        out.append(([j for _, j in best], [d for d, _ in best],
                    sum(d for d, _ in best) / k, gap))
    return out


@pytest.mark.parametrize("T,D,L,k", [(12, 3, 1, 2), (14, 2, 3, 3), (16, 4, 4, 4)])
def test_pure_python_bruteforce(T, D, L, k):
    X = _int_fields(T, D, seed=T * 7 + L)
    ref = _py_knn(X.tolist(), L, k)
    idx, dist, score, gap = oracle.knn(X, L, k)
    for t, (ri, rd, rs, rg) in enumerate(ref):
        assert idx[t].tolist() == ri
        assert dist[t].tolist() == rd
        assert score[t] == rs
        assert gap[t] == rg


# --------------------------------------------------------------------------
# P2: S(i,i) = 0, S and D_L symmetric, bitwise
# --------------------------------------------------------------------------
def test_symmetry_and_zero_diagonal():
    X = synth.random_fields(40, 17, seed=1, scale=3.0, offset=10.0)
    S = oracle.snapshot_dist(X)
    assert np.all(np.diag(S) == 0.0)
    assert np.array_equal(S, S.T)
    Dm = oracle.traj_dist(X, 4)
    assert np.array_equal(Dm, Dm.T)
    assert np.all(np.diag(Dm) == 0.0)


# --------------------------------------------------------------------------
# P3: library brute force on materialised trajectory tensors (Eq. 1 / Eq. 2)
# --------------------------------------------------------------------------
def _materialised(X, L):
    T = X.shape[0]
    return np.stack([X[t:t + L].reshape(-1) for t in range(T - L + 1)])


def _lib_knn(Dm, L, k):
    n = Dm.shape[0]
    idx = np.empty((n, k), dtype=np.int64)
    for t in range(n):
        j = np.arange(n)
        ok = np.abs(j - t) >= L
        order = np.lexsort((j[ok], Dm[t, ok]))
        idx[t] = j[ok][order[:k]]
    return idx


@pytest.mark.parametrize("L", [1, 2, 5])
def test_against_cdist_on_materialised_trajectories(L):
    X = synth.random_fields(90, 11, seed=L, scale=2.0, offset=5.0).astype(np.float64)
    traj = _materialised(X, L)
    ref = cdist(traj, traj, metric="sqeuclidean")
    Dm = oracle.traj_dist(X, L)
    np.testing.assert_allclose(Dm, ref, rtol=1e-12, atol=1e-9)
    k = 4
    idx, dist, score, gap = oracle.knn(X, L, k)
    lib_idx = _lib_knn(ref, L, k)
    clear = gap > 1e-9  # rows whose k-th / (k+1)-th gap is not a rounding tie
    assert clear.mean() > 0.95
    for t in np.nonzero(clear)[0]:
        assert set(idx[t].tolist()) == set(lib_idx[t].tolist())
    np.testing.assert_allclose(score, np.sort(np.where(
        np.abs(np.arange(len(ref))[None] - np.arange(len(ref))[:, None]) >= L, ref, np.inf),
        axis=1)[:, :k].mean(1), rtol=1e-12)


def test_L1_is_snapshot_knn():
    """L = 1: trajectories are snapshots and the exclusion is just j != t."""
    X = synth.random_fields(60, 9, seed=3).astype(np.float64)
    ref = cdist(X, X, metric="sqeuclidean")
    idx, _, score, gap = oracle.knn(X, 1, 3)
    np.fill_diagonal(ref, np.inf)
    ref_sorted = np.sort(ref, axis=1)[:, :3]
    np.testing.assert_allclose(score, ref_sorted.mean(1), rtol=1e-12)
    for t in np.nonzero(gap > 1e-9)[0]:
        assert set(idx[t]) == set(np.argsort(ref[t], kind="stable")[:3])


# --------------------------------------------------------------------------
# P4: the paper's recurrence (Eq. 5) reproduces the oracle's direct sums
# --------------------------------------------------------------------------
def _recurrence(S, L):
    """Eq. 5 written out as the paper's Algorithm 1 runs it: first row by direct
    sums, then D[t, j] = D[t-1, j-1] - S[t-1, j-1] + S[t+L-1, j+L-1]; the first
    column, which the recurrence never reaches, comes from symmetry."""
    T = S.shape[0]
    n = T - L + 1
    Dm = np.zeros((n, n))
    for j in range(n):
        Dm[0, j] = sum(S[m, j + m] for m in range(L))
    for t in range(1, n):
        Dm[t, 0] = Dm[0, t]
        Dm[t, 1:] = Dm[t - 1, :-1] - S[t - 1, :n - 1] + S[t + L - 1, L:L + n - 1]
    return Dm


@pytest.mark.parametrize("L", [1, 3, 7])
def test_recurrence_equals_direct_sum(L):
    X = _int_fields(50, 6, seed=L)
    S = oracle.snapshot_dist(X)
    assert np.array_equal(_recurrence(S, L), oracle.traj_dist(X, L))


# --------------------------------------------------------------------------
# P5: Gram identity (Eq. 4) against the direct differences
# --------------------------------------------------------------------------
def test_gram_identity():
    X = synth.random_fields(64, 33, seed=5, scale=4.0).astype(np.float64)
    N = (X * X).sum(1)
    G = X @ X.T
    S = oracle.snapshot_dist(X)
    np.testing.assert_allclose(N[:, None] + N[None, :] - 2 * G, S, rtol=0,
                               atol=1e-12 * N.max())


# --------------------------------------------------------------------------
# P6-P9: exact invariances (integer-valued data: every sum is exact)
# --------------------------------------------------------------------------
def test_translation_invariance():
    X = _int_fields(48, 7, seed=6)
    a = oracle.knn(X, 3, 4)
    b = oracle.knn(X + 1000.0, 3, 4)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_scaling_by_two():
    X = _int_fields(48, 7, seed=7)
    idx, dist, score, _ = oracle.knn(X, 3, 4)
    idx2, dist2, score2, _ = oracle.knn(2.0 * X, 3, 4)
    assert np.array_equal(idx, idx2)
    assert np.array_equal(4.0 * dist, dist2)
    assert np.array_equal(4.0 * score, score2)


def test_time_reversal():
    X = _int_fields(45, 5, seed=8, lo=-1000, hi=1000)
    L, k = 3, 4
    idx, _, score, gap = oracle.knn(X, L, k)
    idx_r, _, score_r, _ = oracle.knn(X[::-1], L, k)
    n = X.shape[0] - L + 1
    assert np.array_equal(score_r, score[::-1])
    for t in range(n):
        if gap[n - 1 - t] > 0:
            assert set((n - 1 - idx_r[t]).tolist()) == set(idx[n - 1 - t].tolist())


def test_cell_permutation():
    X = _int_fields(40, 12, seed=9)
    perm = np.random.default_rng(0).permutation(12)
    a = oracle.knn(X, 2, 3)
    b = oracle.knn(X[:, perm], 2, 3)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


# --------------------------------------------------------------------------
# P10, P11: k-prefix and the k = 1 matrix profile
# --------------------------------------------------------------------------
def test_k_prefix():
    X = synth.random_fields(70, 8, seed=10).astype(np.float64)
    idx8, dist8, _, _ = oracle.knn(X, 3, 8)
    for kk in (1, 3, 5):
        idx, dist, score, _ = oracle.knn(X, 3, kk)
        assert np.array_equal(idx, idx8[:, :kk])
        assert np.array_equal(dist, dist8[:, :kk])


def test_k1_matrix_profile():
    X = synth.random_fields(70, 8, seed=11).astype(np.float64)
    L = 4
    Dm = oracle.traj_dist(X, L)
    n = Dm.shape[0]
    mask = np.abs(np.arange(n)[None] - np.arange(n)[:, None]) >= L
    mp = np.where(mask, Dm, np.inf).min(1)
    _, _, score, _ = oracle.knn(X, L, 1)
    assert np.array_equal(score, mp)


# --------------------------------------------------------------------------
# P12: a planted off-manifold trajectory is the rarest (tiny workload)
# --------------------------------------------------------------------------
def test_planted_trajectory_is_rarest():
    w = synth.WORKLOADS["tiny"]
    X, starts = synth.make_workload(w)
    _, _, score, _ = oracle.knn(X, w.L, w.k)
    assert int(np.argmax(score)) == starts[0] == 256


# --------------------------------------------------------------------------
# P13: constant series: zero distances, ties broken by the smaller index
# --------------------------------------------------------------------------
def test_constant_series():
    X = np.full((20, 5), 101300.0)
    L, k = 3, 4
    idx, dist, score, _ = oracle.knn(X, L, k)
    assert np.all(dist == 0) and np.all(score == 0)
    n = 20 - L + 1
    for t in range(n):
        first = [j for j in range(n) if abs(t - j) >= L][:k]
        assert idx[t].tolist() == first


def test_rejects_too_few_candidates():
    X = np.zeros((6, 1))
    with pytest.raises(ValueError):
        oracle.knn(X, 2, 3)  # n' = 5 < k + 2L - 1 = 6: the middle row has 2 candidates


# --------------------------------------------------------------------------
# P15/P16: gradient identities and finite differences
# --------------------------------------------------------------------------
def _objective(X, L, k, idx, w):
    """F = sum_t w_t s_t with the neighbour sets held fixed, from pair distances."""
    n = X.shape[0] - L + 1
    ts = np.repeat(np.arange(n), k)
    js = idx.reshape(-1)
    d = oracle.pair_traj_dist(X, L, ts, js).reshape(n, k)
    return float((w * d.mean(1)).sum())


def test_gradient_identities_and_fd():
    X = synth.random_fields(30, 4, seed=12, scale=3.0).astype(np.float64)
    L, k = 3, 3
    idx, _, score, _ = oracle.knn(X, L, k)
    n = X.shape[0] - L + 1
    w = np.random.default_rng(1).uniform(0.5, 2.0, size=n)
    g = oracle.score_grad(X, L, k, idx, w)
    F = float((w * score).sum())
    # translation invariance: the gradient sums to zero over time in every cell
    np.testing.assert_allclose(g.sum(0), 0.0, atol=1e-10 * np.abs(g).max())
    # degree-2 homogeneity (Euler): sum_a <x_a, g_a> = 2F
    np.testing.assert_allclose((X * g).sum(), 2.0 * F, rtol=1e-12)
    # central differences; F is quadratic with N_t fixed, so they are exact up
    # to rounding
    h = 1e-3
    rng = np.random.default_rng(2)
    for _ in range(20):
        a, p = int(rng.integers(0, X.shape[0])), int(rng.integers(0, X.shape[1]))
        Xp, Xm = X.copy(), X.copy()
        Xp[a, p] += h
        Xm[a, p] -= h
        fd = (_objective(Xp, L, k, idx, w) - _objective(Xm, L, k, idx, w)) / (2 * h)
        assert abs(fd - g[a, p]) <= 1e-6 * max(1.0, abs(g[a, p]))


def test_gradient_translation_invariant():
    X = _int_fields(30, 4, seed=13)
    L, k = 2, 3
    idx, _, _, _ = oracle.knn(X, L, k)
    w = np.ones(X.shape[0] - L + 1)
    g1 = oracle.score_grad(X, L, k, idx, w)
    g2 = oracle.score_grad(X + 777.0, L, k, idx, w)
    assert np.array_equal(g1, g2)


def test_gap_is_relative_kth_to_next():
    """The gap of every row against the sorted full row of the trajectory
    matrix, recomputed here from the (k)-th and (k+1)-th order statistics: a
    wrong rank index, a missing exclusion or the wrong denominator fails."""
    X = synth.random_fields(70, 6, seed=15).astype(np.float64)
    L, k = 3, 4
    Dm = cdist(_materialised(X, L), _materialised(X, L), metric="sqeuclidean")
    n = Dm.shape[0]
    _, dist, _, gap = oracle.knn(X, L, k)
    for t in range(n):
        row = np.sort(Dm[t, np.abs(np.arange(n) - t) >= L])
        want = (row[k] - row[k - 1]) / row[k - 1]
        assert gap[t] == pytest.approx(want, rel=1e-9, abs=1e-12)
        assert dist[t, -1] == pytest.approx(row[k - 1], rel=1e-12)


def test_rows_multi_matches_single_length():
    """One pass over L = 1..L_max gives, bit for bit, the rows of each length's
    own direct sums (Eq. 2), and +inf past each length's last trajectory."""
    X = synth.random_fields(60, 7, seed=16, scale=2.0, offset=3.0).astype(np.float64)
    T, Lmax = X.shape[0], 6
    rows = np.array([0, 5, 33, T - Lmax], dtype=np.int64)
    multi = oracle.traj_dist_rows_multi(X, Lmax, rows)
    for L in range(1, Lmax + 1):
        n = T - L + 1
        assert np.array_equal(multi[L - 1, :, :n], oracle.traj_dist_rows(X, L, rows))
        assert np.all(np.isinf(multi[L - 1, :, n:]))
    res = oracle.knn_rows_multi(X, Lmax, 3, rows)
    for L in range(1, Lmax + 1):
        single = oracle.knn_rows(X, L, 3, rows)
        for a, b in zip(res[L - 1], single):
            assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        oracle.traj_dist_rows_multi(X, Lmax, np.array([T - Lmax + 1]))


def test_rows_mode_matches_full():
    X = synth.random_fields(80, 10, seed=14).astype(np.float64)
    L, k = 4, 5
    full = oracle.knn(X, L, k)
    rows = np.array([0, 1, 37, 76], dtype=np.int64)
    idx, dist, score, gap, drows = oracle.knn_rows(X, L, k, rows)
    np.testing.assert_array_equal(drows, oracle.traj_dist(X, L)[rows])
    np.testing.assert_array_equal(idx, full[0][rows])
    np.testing.assert_array_equal(score, full[2][rows])


# --- local intrinsic dimension (Section 5.1, Levina-Bickel MLE) -------------

@pytest.mark.parametrize("d,k,c", [(1.0, 20, 3.0), (5.0, 30, 0.01), (18.0, 40, 1e4),
                                   (2.5, 2, 1.0)])
def test_local_dim_closed_form(d, k, c):
    """Neighbour distances T_j = c j^(1/d) (the spacing of points of a
    d-dimensional set of uniform density) give the closed form
    m_k = (k - 1) d / ((k - 1) ln k - ln (k - 1)!), with ln (k - 1)! from
    lgamma -- a different route from the oracle's sum of log-ratios."""
    import math
    j = np.arange(1, k + 1, dtype=np.float64)
    sq = (c * j ** (1.0 / d)) ** 2  # squared distances, as the lists hold
    m = oracle.local_dim(sq[None, :])[0]
    assert np.isnan(m[0])
    for kk in range(2, k + 1):
        expect = (kk - 1) * d / ((kk - 1) * math.log(kk) - math.lgamma(kk))
        assert m[kk - 1] == pytest.approx(expect, rel=1e-12)


@pytest.mark.parametrize("d", [1, 2, 5, 8])
def test_local_dim_recovers_known_dimension(d):
    """Gaussian samples in a d-dimensional subspace of a 64-cell field, with
    the oracle's own kNN (L = 1): the mean local estimate with k = 20,
    debiased by (k - 2)/(k - 1) as Levina and Bickel note, is within 10% of d.
    A dropped square-root halving would give 2d, a flipped ratio a negative
    value."""
    rng = np.random.default_rng(d)
    N, k = 3000, 20
    Q, _ = np.linalg.qr(rng.standard_normal((64, d)))
    X = rng.standard_normal((N, d)) @ Q.T * 100.0 + 5000.0
    _, dist, _, _ = oracle.knn(X, 1, k)
    m = oracle.local_dim(dist)[:, k - 1]
    assert abs(np.mean(m) * (k - 2) / (k - 1) - d) <= 0.1 * d


def test_local_dim_scale_invariant_and_degenerate():
    rng = np.random.default_rng(3)
    dist = np.sort(rng.uniform(1.0, 50.0, (40, 12)), axis=1)
    m = oracle.local_dim(dist)
    np.testing.assert_allclose(oracle.local_dim(dist * 7.5e6), m, rtol=1e-12)
    # duplicates below a positive k-th distance: estimate 0; all equal: +inf;
    # all zero: NaN
    deg = oracle.local_dim(np.array([[0.0, 0.0, 2.0, 3.0], [4.0, 4.0, 4.0, 4.0],
                                     [0.0, 0.0, 0.0, 0.0]]))
    assert deg[0, 2] == 0.0 and deg[0, 3] == 0.0 and np.isnan(deg[0, 1])
    assert np.all(np.isinf(deg[1, 1:]))
    assert np.all(np.isnan(deg[2]))
