"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times, on sampled rows the oracle computes one by one, plus
properties that hold for every row at any size.

  * full: T = 27394 daily 64 x 128 fields (D = 8192), L = 5, k = 10, all three
    Gram precisions;
  * split: T = 27394, 128 x 256 (D = 32768), BF16x3 against FP16 and FP32;
  * all lengths: L = 1..10 in one sweep at T = 27394, D = 8192;
  * small grid: T = 27394, 4 x 8 (D = 32), where the top-k stage dominates;
  * backward: T = 10957, D = 8192, L = 5, k = 10, the summed score of the 100
    rarest trajectories, against the oracle's analytic gradient and FP64
    central differences (h = 1e-3 Pa) on 64 cells.
"""
import numpy as np
import pytest

import oracle
from paper_2603_02059_amd import synth
from tests.parity import check_rows, gram_norm_tol, precision_tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_DATA = {}


def _say(msg):
    print(msg, flush=True)


def _workload(name):
    if name not in _DATA:
        _say(f"[gpu-full] generating {name}")
        _DATA[name] = synth.make_workload(name)
    return _DATA[name]


def _run(Xn, L_min, L_max, k, prec):
    from paper_2603_02059_amd import traknn as tk
    X = torch.from_numpy(Xn).cuda()
    p = tk.Plan(X.shape[0], X.shape[1], L_min, L_max, k, prec)
    idx, dist = p.knn(X)
    s = p.score(dist)
    torch.cuda.synchronize()
    out = idx.cpu().numpy(), dist.cpu().numpy(), s.cpu().numpy()
    p.close()
    del X
    torch.cuda.empty_cache()
    return out


def _check_all_rows(idx, dist, s, L, k):
    """Properties of every row: in range, outside the exclusion zone, distinct,
    sorted by (distance, index), score = mean of the k distances."""
    n = idx.shape[0]
    t = np.arange(n)[:, None]
    assert np.all((idx >= 0) & (idx < n)), "index out of range"
    assert np.all(np.abs(idx - t) >= L), "exclusion zone violated"
    srt = np.sort(idx, axis=1)
    assert np.all(srt[:, 1:] != srt[:, :-1]), "duplicate neighbour"
    d0, d1 = dist[:, :-1], dist[:, 1:]
    i0, i1 = idx[:, :-1], idx[:, 1:]
    assert np.all((d0 < d1) | ((d0 == d1) & (i0 < i1))), "list not in (distance, index) order"
    assert np.all(np.isfinite(dist)) and np.all(dist >= 0)
    np.testing.assert_allclose(s, dist.mean(axis=1), rtol=1e-14)


def _sample(n, starts, s, m, L):
    rows = set(np.linspace(0, n - 1, m).astype(int).tolist())
    rows |= {0, 1, L, n - 2, n - 1}
    rows |= {st for st in starts if st < n}
    rows |= set(np.argsort(-s, kind="stable")[:8].tolist())
    return np.array(sorted(rows), dtype=np.int64)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fp16"])
def test_full_workload(prec):
    w = synth.WORKLOADS["full"]
    Xn, starts = _workload("full")
    _say(f"[gpu-full] full T={w.T} D={w.D} L={w.L} k={w.k} prec={prec}")
    idx, dist, s = _run(Xn, w.L, w.L, w.k, prec)
    idx, dist, s = idx[0], dist[0], s[0]
    _check_all_rows(idx, dist, s, w.L, w.k)
    rows = _sample(idx.shape[0], starts, s, 40, w.L)
    stats = check_rows(Xn, w.L, w.k, rows, idx[rows], dist[rows], s[rows], precision_tol(prec))
    _say(f"  {stats}")
    # every planted event is found: some trajectory overlapping it ranks
    # among the 5% rarest
    top = set(np.argsort(-s, kind="stable")[: idx.shape[0] // 20].tolist())
    for st in starts:
        assert any(t in top for t in range(st - w.L + 1, st + w.event_len)), st


def test_split_config():
    w = synth.WORKLOADS["split"]
    Xn, starts = _workload("split")
    res = {}
    for prec in ("bf16x3", "fp16", "fp32"):
        _say(f"[gpu-full] split T={w.T} D={w.D} L={w.L} k={w.k} prec={prec}")
        res[prec] = _run(Xn, w.L, w.L, w.k, prec)
    idx, dist, s = (a[0] for a in res["bf16x3"])
    _check_all_rows(idx, dist, s, w.L, w.k)
    rows = _sample(idx.shape[0], starts, s, 24, w.L)
    ref = oracle.knn_rows(Xn, w.L, w.k, rows)
    for prec, (i, d, sc) in res.items():
        stats = check_rows(Xn, w.L, w.k, rows, i[0][rows], d[0][rows], sc[0][rows],
                           precision_tol(prec), ref=ref)
        _say(f"  {prec}: {stats}")
    del _DATA["split"]


def test_all_lengths_sweep():
    w = synth.WORKLOADS["full"]
    Xn, starts = _workload("full")
    Lmax = 10
    _say(f"[gpu-full] sweep L=1..{Lmax} T={w.T} D={w.D} k={w.k}")
    idx, dist, s = _run(Xn, 1, Lmax, w.k, "bf16x3")
    # the same 64 evenly spaced rows (plus both ends, the planted starts and
    # 8 random rows) for every length, all lengths from one oracle pass
    n_last = w.T - Lmax + 1
    rng = np.random.default_rng(11)
    rows = set(np.linspace(0, n_last - 1, 64).astype(int).tolist())
    rows |= {0, 1, n_last - 1} | {st for st in starts if st < n_last}
    rows |= set(rng.integers(0, n_last, 8).tolist())
    rows = np.array(sorted(rows), dtype=np.int64)
    _say(f"  oracle: {rows.size} rows for each of L=1..{Lmax}")
    refs = oracle.knn_rows_multi(Xn, Lmax, w.k, rows)
    for L in range(1, Lmax + 1):
        n = w.T - L + 1
        _check_all_rows(idx[L - 1, :n], dist[L - 1, :n], s[L - 1, :n], L, w.k)
        assert np.all(idx[L - 1, n:] == -1) and np.all(np.isnan(s[L - 1, n:]))
        stats = check_rows(Xn, L, w.k, rows, idx[L - 1][rows], dist[L - 1][rows],
                           s[L - 1][rows], precision_tol("bf16x3"), ref=refs[L - 1])
        _say(f"  L={L}: {stats}")
        # the last rows of each length (only they see the shortest candidate
        # ranges at the end of the series)
        tail = np.arange(n - 3, n)
        check_rows(Xn, L, w.k, tail, idx[L - 1][tail], dist[L - 1][tail], s[L - 1][tail],
                   precision_tol("bf16x3"))
    # the sweep and single-length runs agree bit for bit (same distance
    # matrix; each length's sums started and slid the same way, whether it
    # shares a pass with another length or not)
    for L in (5, 10):
        iL, dL, sL = _run(Xn, L, L, w.k, "bf16x3")
        n = w.T - L + 1
        assert np.array_equal(idx[L - 1, :n], iL[0])
        assert np.array_equal(dist[L - 1, :n], dL[0])
        assert np.array_equal(s[L - 1, :n], sL[0])


@pytest.mark.parametrize("k", [10, 40])
def test_small_grid_full_length(k):
    """A small-D shape (4 x 8 grid, D = 32) at the full length: the Gram is tiny
    and the window/top-k stage dominates. k = 40 is the largest k of the
    paper's intrinsic-dimension estimates. Scores and sets under the stated
    rule; the norm-relative allowance widens only the individual distances."""
    T, L = 27394, 5
    _say(f"[gpu-full] small grid T={T} D=32 L={L} k={k}")
    Xn, starts = synth.make_fields(T, 4, 8, sigma=1.0, n_events=20, event_len=5, seed=4)
    idx, dist, s = _run(Xn, L, L, k, "bf16x3")
    idx, dist, s = idx[0], dist[0], s[0]
    _check_all_rows(idx, dist, s, L, k)
    rows = _sample(idx.shape[0], starts, s, 48, L)
    stats = check_rows(Xn, L, k, rows, idx[rows], dist[rows], s[rows],
                       precision_tol("bf16x3"), norm_tol=gram_norm_tol("bf16x3", 32))
    _say(f"  {stats}")


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_pca13_full_length(prec):
    """The paper's 95%-variance PCA shape (Section 5.1: 13 components, d = 5,
    k = 10): the full workload's fields reduced to their 13 leading principal
    component scores by a randomized SVD, T = 27394. Stated rule for scores
    and sets; the norm-relative allowance widens only individual distances."""
    w = synth.WORKLOADS["full"]
    if "pca13" not in _DATA:
        _say("[gpu-full] generating the 13-component PCA reduction of the full workload")
        _DATA["pca13"] = synth.make_pca_workload(13)
    Xn, starts, frac = _DATA["pca13"]
    _say(f"[gpu-full] pca13 T={w.T} D=13 L={w.L} k={w.k} prec={prec} "
         f"(explained variance {frac:.3f})")
    idx, dist, s = _run(Xn, w.L, w.L, w.k, prec)
    idx, dist, s = idx[0], dist[0], s[0]
    _check_all_rows(idx, dist, s, w.L, w.k)
    rows = _sample(idx.shape[0], starts, s, 48, w.L)
    stats = check_rows(Xn, w.L, w.k, rows, idx[rows], dist[rows], s[rows],
                       precision_tol(prec), norm_tol=gram_norm_tol(prec, 13))
    _say(f"  {stats}")


def test_backward_config():
    w = synth.WORKLOADS["bwd"]
    Xn, _ = synth.make_workload(w)
    L, k = w.L, w.k
    from paper_2603_02059_amd import traknn as tk
    _say(f"[gpu-full] backward T={w.T} D={w.D} L={L} k={k}, 100 rarest, fp32")
    X = torch.from_numpy(Xn).cuda().requires_grad_(True)
    s, idx = tk.score(X, L, k, "fp32")
    sn = s.detach().cpu().numpy()
    rare = np.argsort(-sn, kind="stable")[:100]
    wts = np.zeros_like(sn)
    wts[rare] = 1.0
    (s * torch.from_numpy(wts).cuda()).sum().backward()
    torch.cuda.synchronize()
    g = X.grad.cpu().numpy().astype(np.float64)
    idx = idx.cpu().numpy()
    del X
    torch.cuda.empty_cache()

    g_ref = oracle.score_grad(Xn, L, k, idx, wts)
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    _say(f"  normwise error vs analytic {err:.3e}")
    assert err <= 1e-5

    # FP64 central differences at h = 1e-3 Pa on 64 cells (48 in touched
    # rows, 16 in untouched rows). F is quadratic in X with the neighbour sets
    # fixed, so only the terms that contain the perturbed entry change and the
    # difference over those terms alone is exact up to rounding.
    X64 = Xn.astype(np.float64)
    rng = np.random.default_rng(5)
    touched = np.flatnonzero(np.any(g_ref != 0, axis=1))
    untouched = np.flatnonzero(~np.any(g_ref != 0, axis=1))
    cells = [(int(a), int(rng.integers(0, w.D))) for a in rng.choice(touched, 48, replace=False)]
    cells += [(int(a), int(rng.integers(0, w.D))) for a in rng.choice(untouched, 16, replace=False)]
    h = 1e-3
    gmax = np.abs(g).max()
    worst = 0.0
    for a, p in cells:
        fp = fm = 0.0
        for t in rare:
            for j in idx[t]:
                for m in range(L):
                    if t + m != a and j + m != a:
                        continue
                    xa, xb = X64[t + m, p], X64[j + m, p]
                    for sgn in (1, -1):
                        ya = xa + sgn * h if t + m == a else xa
                        yb = xb + sgn * h if j + m == a else xb
                        term = (ya - yb) ** 2 / k
                        if sgn > 0:
                            fp += term
                        else:
                            fm += term
        fd = (fp - fm) / (2 * h)
        if abs(fd) > 1e-6 * gmax:
            rel = abs(g[a, p] - fd) / abs(fd)
            worst = max(worst, rel)
            assert rel <= 1e-4, (a, p, g[a, p], fd)
        else:
            assert abs(g[a, p]) <= 1e-6 * gmax, (a, p, g[a, p], fd)
    _say(f"  worst relative error vs central differences {worst:.3e}")

    # translation invariance (each cell's gradient sums to zero) and Euler's
    # relation for the degree-2 homogeneous F: sum_a <x_a - mu, g_a> = 2F
    colsum = g.sum(axis=0)
    assert np.all(np.abs(colsum) <= 1e-5 * np.abs(g).sum(axis=0) + 1e-12)
    F = float(sn[rare].sum())
    euler = float(((X64 - X64.mean(axis=0)) * g).sum())
    assert abs(euler - 2 * F) <= 2e-5 * 2 * F, (euler, 2 * F)


def test_local_dim_sweep():
    """The intrinsic dimension study's shape (Section 5.1): one sweep over
    L = 1..5 with k = 40 at the full size, the local dimension for every
    k' <= 40; sampled rows against the oracle's lists and estimator, and the
    mean local dimension over k' in {20, 30, 40} printed per L."""
    from paper_2603_02059_amd import traknn as tk
    w = synth.WORKLOADS["full"]
    Xn, starts = _workload("full")
    k, Lmax = 40, 5
    _say(f"[gpu-full] local dimension sweep L=1..{Lmax} k={k} T={w.T} D={w.D}")
    X = torch.from_numpy(Xn).cuda()
    p = tk.Plan(w.T, w.D, 1, Lmax, k, "bf16x3")
    idx, dist = p.knn(X)
    ld = p.local_dim(dist)
    torch.cuda.synchronize()
    dist_h, ld_h = dist.cpu().numpy(), ld.cpu().numpy()
    p.close()
    del X
    torch.cuda.empty_cache()
    rng = np.random.default_rng(12)
    for L in range(1, Lmax + 1):
        n = w.T - L + 1
        np.testing.assert_allclose(ld_h[L - 1, :n], oracle.local_dim(dist_h[L - 1, :n]),
                                   rtol=1e-12)
        assert np.all(np.isnan(ld_h[L - 1, n:]))
        m = ld_h[L - 1, :n][:, [19, 29, 39]]
        _say(f"  L={L}: mean local dimension {np.mean(m):.2f} +- {np.std(m):.2f}")
        if L in (1, Lmax):
            rows = np.unique(np.concatenate([rng.integers(0, n, 6), [0, n - 1]]))
            r = oracle.knn_rows(Xn, L, k, rows)
            ref = oracle.local_dim(r[1])
            got = ld_h[L - 1][rows]
            err = np.abs(got[:, 1:] - ref[:, 1:])
            tol = 2.0 * ref[:, 1:] ** 2 * 1e-5 + 1e-12 * ref[:, 1:]
            assert np.all(err <= tol), float(err.max())


def test_paper_scaling_default_shape():
    """The default shape of the paper's scaling study (Section 4): T = 27000
    random fields of 180 x 280 (D = 50400), d = 1, k = 1 (the matrix-profile
    case), BF16x3. Every row's list is valid; sampled rows match the oracle."""
    T, H, W, L, k = 27000, 180, 280, 1, 1
    _say(f"[gpu-full] paper scaling default T={T} D={H * W} L={L} k={k}")
    rng = np.random.default_rng(2603)
    Xn = rng.standard_normal((T, H * W), dtype=np.float32)
    idx, dist, s = _run(Xn, L, L, k, "bf16x3")
    idx, dist, s = idx[0], dist[0], s[0]
    _check_all_rows(idx, dist, s, L, k)
    rows = np.unique(np.concatenate([np.linspace(0, T - 1, 14).astype(np.int64), [1, T - 2]]))
    stats = check_rows(Xn, L, k, rows, idx[rows], dist[rows], s[rows], precision_tol("bf16x3"))
    _say(f"  {stats}")
    del Xn
