"""GPU parity of the HIP path against the FP64 oracle (small and ragged cases).

Every call goes through the C ABI (``paper_2603_02059_amd.traknn``). Sizes are
chosen so the oracle finishes in seconds while the kernels still see several
256-row Gram tiles, ragged T and D tails, several 64-diagonal window chunks and
several column splits.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2603_02059_amd import synth
from tests.parity import check_rows, gram_norm_tol, precision_tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _tk():
    from paper_2603_02059_amd import traknn as tk
    return tk


def _say(msg):
    print(msg, flush=True)


def _run(Xn, L, k, prec, L_max=None):
    tk = _tk()
    X = torch.from_numpy(np.ascontiguousarray(Xn, dtype=np.float32)).cuda()
    p = tk.Plan(X.shape[0], X.shape[1], L, L_max, k, prec)
    idx, dist = p.knn(X)
    s = p.score(dist)
    torch.cuda.synchronize()
    out = idx.cpu().numpy(), dist.cpu().numpy(), s.cpu().numpy()
    p.close()
    return out


def _full_check(Xn, L, k, prec, tol=None, norm_tol=0.0):
    tol = precision_tol(prec) if tol is None else tol
    idx, dist, s = _run(Xn, L, k, prec)
    n = Xn.shape[0] - L + 1
    rows = np.arange(n)
    ref = oracle.knn(Xn, L, k)
    Dm = oracle.traj_dist(Xn, L)
    stats = check_rows(Xn, L, k, rows, idx[0], dist[0], s[0], tol,
                       ref=(ref[0], ref[1], ref[2], ref[3], Dm), norm_tol=norm_tol)
    return stats


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16"])
def test_tiny_workload(prec):
    w = synth.WORKLOADS["tiny"]
    _say(f"[gpu] tiny workload T={w.T} D={w.D} L={w.L} k={w.k} prec={prec}")
    Xn, starts = synth.make_workload(w)
    stats = _full_check(Xn, w.L, w.k, prec)
    _say(f"  {stats}")
    idx, dist, s = _run(Xn, w.L, w.k, prec)
    assert int(np.argmax(s[0])) == starts[0]


@pytest.mark.parametrize("T,D,L,k,prec", [
    (700, 1000, 4, 7, "bf16x3"),
    (700, 1000, 1, 1, "fp32"),
    (613, 77, 6, 3, "fp16"),
    # D = 5: BF16x3's hi + lo representation reaches 1e-4 on scores here (the
    # nearest distances are a small fraction of the norms), so FP32
    (300, 5, 2, 9, "fp32"),
    (520, 300, 16, 64, "bf16x3"),
])
def test_ragged_shapes(T, D, L, k, prec):
    _say(f"[gpu] ragged T={T} D={D} L={L} k={k} prec={prec}")
    Xn, _ = synth.make_fields(T, 1, D, sigma=2.0, n_events=2, event_len=L, seed=T + D)
    # off-workload shapes: workload tolerance plus the Gram's norm-relative floor
    stats = _full_check(Xn, L, k, prec, norm_tol=gram_norm_tol(prec, D))
    _say(f"  {stats}")


def test_worked_example(golden_dir):
    with open(os.path.join(golden_dir, "worked_example.json")) as f:
        g = json.load(f)
    x = np.array(g["x"], dtype=np.float32)[:, None]
    # One cell, no averaging over cells: the centred values (up to ~9) are
    # represented to 2^-24 (FP32), 2^-16 (BF16 hi+lo) and 2^-11 (FP16) relative,
    # on differences as small as 3 -> relative distance bounds below.
    for prec, tol in (("fp32", 1e-6), ("bf16x3", 5e-4), ("fp16", 2e-2)):
        for case in g["cases"]:
            _say(f"[gpu] worked example k={case['k']} prec={prec}")
            idx, dist, s = _run(x, g["L"], case["k"], prec)
            assert idx[0].tolist() == case["idx"]
            np.testing.assert_allclose(dist[0], np.array(case["dist"], float), rtol=tol)
            np.testing.assert_allclose(s[0], np.array(case["score"], float), rtol=tol)


def test_constant_series_ties():
    _say("[gpu] constant series")
    Xn = np.full((300, 37), 101300.0, dtype=np.float32)
    L, k = 3, 6
    for prec in ("fp32", "bf16x3", "fp16"):
        idx, dist, s = _run(Xn, L, k, prec)
        ref_idx, _, _, _ = oracle.knn(Xn, L, k)
        assert np.array_equal(idx[0], ref_idx)
        assert np.all(dist[0] == 0) and np.all(s[0] == 0)


def test_planted_trajectory_translation_and_scale():
    """Adding a constant field changes nothing; doubling X quadruples scores."""
    w = synth.WORKLOADS["tiny"]
    _say("[gpu] translation / scaling invariance")
    Xn, starts = synth.make_workload(w)
    i0, d0, s0 = _run(Xn, w.L, w.k, "bf16x3")
    i1, d1, s1 = _run(Xn - 101300.0, w.L, w.k, "bf16x3")
    i2, d2, s2 = _run(2.0 * Xn, w.L, w.k, "bf16x3")
    np.testing.assert_allclose(s1, s0, rtol=2e-5)
    np.testing.assert_allclose(s2, 4.0 * s0, rtol=2e-5)
    assert int(np.argmax(s1[0])) == int(np.argmax(s2[0])) == starts[0]


def test_multi_length_sweep():
    T, D, Lmax, k = 600, 200, 6, 5
    _say(f"[gpu] sweep L=1..{Lmax} T={T} D={D}")
    Xn, _ = synth.make_fields(T, 10, 20, sigma=2.0, n_events=3, event_len=4, seed=5)
    idx, dist, s = _run(Xn, 1, k, "bf16x3", L_max=Lmax)
    S = oracle.snapshot_dist(Xn)
    for L in range(1, Lmax + 1):
        n = T - L + 1
        Dm = oracle.traj_dist_from_snapshot(S, L)
        ref = oracle.knn_from_rows(Dm, np.arange(n), L, k)
        stats = check_rows(Xn, L, k, np.arange(n), idx[L - 1, :n], dist[L - 1, :n],
                           s[L - 1, :n], 1e-5, ref=ref + (Dm,),
                           norm_tol=gram_norm_tol("bf16x3", 200))
        _say(f"  L={L}: {stats}")
        assert np.all(idx[L - 1, n:] == -1) and np.all(np.isinf(dist[L - 1, n:]))
        assert np.all(np.isnan(s[L - 1, n:]))
        # one pass over all lengths = separate single-length runs, bit for bit:
        # the same distance matrix, and each length's sums started and slid
        # the same way whether or not it shares its pass with another length
        i1, d1, s1 = _run(Xn, L, k, "bf16x3")
        assert np.array_equal(idx[L - 1, :n], i1[0])
        assert np.array_equal(dist[L - 1, :n], d1[0])
        assert np.array_equal(s[L - 1, :n], s1[0])


def test_sweep_all_lengths_max_k():
    """L = 1..16 in one call with k = 64 (the largest lengths and list size)."""
    T, D, Lmax, k = 400, 40, 16, 64
    _say(f"[gpu] sweep L=1..{Lmax} k={k} T={T} D={D}")
    Xn, _ = synth.make_fields(T, 5, 8, sigma=1.5, n_events=2, event_len=6, seed=21)
    idx, dist, s = _run(Xn, 1, k, "bf16x3", L_max=Lmax)
    S = oracle.snapshot_dist(Xn)
    for L in range(1, Lmax + 1):
        n = T - L + 1
        Dm = oracle.traj_dist_from_snapshot(S, L)
        ref = oracle.knn_from_rows(Dm, np.arange(n), L, k)
        stats = check_rows(Xn, L, k, np.arange(n), idx[L - 1, :n], dist[L - 1, :n],
                           s[L - 1, :n], 1e-5, ref=ref + (Dm,),
                           norm_tol=gram_norm_tol("bf16x3", D))
        if L in (1, 8, 16):
            _say(f"  L={L}: {stats}")
        assert np.all(idx[L - 1, n:] == -1) and np.all(np.isnan(s[L - 1, n:]))


def test_strided_and_unaligned_inputs():
    """Rows with a stride beyond D (a view into wider rows) and a D that is not a
    multiple of 4 give exactly the results of a contiguous copy."""
    tk = _tk()
    for D, extra in ((96, 12), (77, 0)):
        _say(f"[gpu] strided input D={D} row padding {extra}")
        Xn, _ = synth.make_fields(300, 1, D, sigma=2.0, n_events=1, event_len=3, seed=D)
        wide = np.zeros((300, D + extra + (4 - (D + extra) % 4) % 4), dtype=np.float32)
        wide[:, :D] = Xn
        Xw = torch.from_numpy(wide).cuda()[:, :D]
        Xc = torch.from_numpy(np.ascontiguousarray(Xn)).cuda()
        for prec in ("bf16x3", "fp32"):
            p = tk.Plan(300, D, 3, 3, 6, prec)
            i1, d1 = p.knn(Xw)
            i2, d2 = p.knn(Xc)
            torch.cuda.synchronize()
            assert torch.equal(i1, i2) and torch.equal(d1, d2)
            p.close()


def test_prefix_scores_every_k():
    """Scores for every k' <= k from one search equal separate searches with
    k' neighbours; the last column is the score itself."""
    tk = _tk()
    w = synth.WORKLOADS["tiny"]
    _say("[gpu] prefix scores k'=1..k")
    Xn, _ = synth.make_workload(w)
    X = torch.from_numpy(Xn).cuda()
    k = 8
    p = tk.Plan(w.T, w.D, w.L, w.L, k, "bf16x3")
    idx, dist = p.knn(X)
    sp = p.score_prefix(dist)
    s = p.score(dist)
    torch.cuda.synchronize()
    sp, s = sp.cpu().numpy(), s.cpu().numpy()
    p.close()
    assert np.array_equal(sp[0, :, k - 1], s[0])
    for kk in range(1, k + 1):
        ref = oracle.knn(Xn, w.L, kk)[2]
        np.testing.assert_allclose(sp[0, :, kk - 1], ref, rtol=1e-5)


@pytest.mark.parametrize("T,H,W", [(3000, 8, 16), (27394, 4, 8)])
def test_lists_independent_of_waves_per_block(T, H, W):
    """The planner gives k = 10, 20 and 40 different numbers of waves per
    8-row block (4, 2 and 1 at T = 27394), so their searches split each row's
    diagonals differently. The k nearest are the first k of the 2k nearest
    in (distance, index) order and the window sums are exact, so the first 10
    entries of every k = 20 and k = 40 list equal the k = 10 list bit for
    bit."""
    L = 5
    _say(f"[gpu] list prefixes across k = 10, 20, 40 at T={T} D={H * W}")
    Xn, _ = synth.make_fields(T, H, W, sigma=1.0, n_events=3, event_len=L, seed=T)
    i10, d10, _ = _run(Xn, L, 10, "bf16x3")
    for k in (20, 40):
        ik, dk, _ = _run(Xn, L, k, "bf16x3")
        assert np.array_equal(ik[..., :10], i10), f"k={k}: indices differ from k=10"
        assert np.array_equal(dk[..., :10], d10), f"k={k}: distances differ from k=10"


def test_determinism():
    w = synth.WORKLOADS["tiny"]
    _say("[gpu] determinism")
    Xn, _ = synth.make_workload(w)
    a = _run(Xn, w.L, w.k, "bf16x3")
    b = _run(Xn, w.L, w.k, "bf16x3")
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def _grad_case(Xn, L, k, prec, weights_fn):
    tk = _tk()
    X = torch.from_numpy(Xn).cuda().requires_grad_(True)
    s, idx = tk.score(X, L, k, prec)
    w = weights_fn(s.detach().cpu().numpy())
    (s * torch.from_numpy(w).cuda()).sum().backward()
    torch.cuda.synchronize()
    return X.grad.cpu().numpy().astype(np.float64), idx.cpu().numpy(), w


def test_backward_tiny():
    w = synth.WORKLOADS["tiny"]
    _say("[gpu] backward tiny, top-8 rarest")
    Xn, _ = synth.make_workload(w)

    def top8(s):
        out = np.zeros_like(s)
        out[np.argsort(-s, kind="stable")[:8]] = 1.0
        return out

    g, idx, wts = _grad_case(Xn, w.L, w.k, "bf16x3", top8)
    g_ref = oracle.score_grad(Xn, w.L, w.k, idx, wts)
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    _say(f"  normwise grad error {err:.3e}")
    assert err < 1e-6
    nz = np.abs(g_ref) > 1e-6 * np.abs(g_ref).max()
    assert np.max(np.abs(g - g_ref)[nz] / np.abs(g_ref)[nz]) < 1e-5
    assert np.all(g[~np.any(g_ref != 0, axis=1)] == 0)
    # translation invariance and degree-2 homogeneity of F
    np.testing.assert_allclose(g.sum(0), 0.0, atol=1e-6 * np.abs(g).max() * Xn.shape[0])


def test_autograd_retain_graph_and_small_backward_workspace():
    """TraknnScore frees the forward workspace after the scores exist, keeps
    the plan until the graph is freed (so a retained graph can run backward
    twice) and marks the returned neighbour lists non-differentiable."""
    tk = _tk()
    w = synth.WORKLOADS["tiny"]
    _say("[gpu] autograd: retain_graph, twice")
    Xn, _ = synth.make_workload(w)
    X = torch.from_numpy(Xn).cuda().requires_grad_(True)
    s, idx = tk.score(X, w.L, w.k, "fp32")
    assert not idx.requires_grad
    wts = torch.zeros_like(s)
    wts[::5] = 1.0
    (s * wts).sum().backward(retain_graph=True)
    g1 = X.grad.clone()
    X.grad = None
    (s * wts).sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(g1, X.grad)
    g_ref = oracle.score_grad(Xn, w.L, w.k, idx.cpu().numpy(), wts.cpu().numpy())
    g = g1.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) < 1e-6


def test_backward_all_weights_and_worked_example(golden_dir):
    _say("[gpu] backward, random weights on every trajectory")
    Xn, _ = synth.make_fields(200, 6, 7, sigma=1.5, seed=9)
    rng = np.random.default_rng(3)
    g, idx, wts = _grad_case(Xn, 3, 4, "fp32", lambda s: rng.uniform(-1, 1, s.shape))
    g_ref = oracle.score_grad(Xn, 3, 4, idx, wts)
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert err < 1e-6
    with open(os.path.join(golden_dir, "worked_example.json")) as f:
        gold = json.load(f)
    x = np.array(gold["x"], dtype=np.float32)[:, None]
    gc = gold["grad_case"]
    g, idx, _ = _grad_case(x, gold["L"], gc["k"], "fp32",
                           lambda s: np.array(gc["weights"], dtype=np.float64))
    np.testing.assert_array_equal(g[:, 0], np.array(gc["grad"], dtype=np.float64))


def test_stage_timing():
    tk = _tk()
    w = synth.WORKLOADS["tiny"]
    Xn, _ = synth.make_workload(w)
    X = torch.from_numpy(Xn).cuda()
    p = tk.Plan(w.T, w.D, w.L, w.L, w.k, "bf16x3")
    p.set_timing(True)
    p.knn(X)
    t = p.stage_times()
    assert set(t) == set(tk.STAGES) and all(v >= 0 for v in t.values())
    p.close()


def _dim_tol(m_ref, eps):
    # |d m| <= m^2 eps to first order when every distance of the list moves by
    # at most a relative eps (m = 2(k'-1)/S and |dS| <= 2(k'-1) eps)
    return 2.0 * np.abs(m_ref) ** 2 * eps + 1e-12 * np.abs(m_ref)


def test_local_dim_every_k():
    """Local intrinsic dimension (Section 5.1 estimator) for every k' <= 40
    from one search: on the GPU's own lists it equals the oracle's estimator;
    end to end against the oracle's lists it is within what the 1e-5
    distance tolerance allows; crafted degenerate lists give the same NaN, 0
    and +inf."""
    tk = _tk()
    w = synth.WORKLOADS["tiny"]
    _say("[gpu] local intrinsic dimension k'=1..40")
    Xn, _ = synth.make_workload(w)
    X = torch.from_numpy(Xn).cuda()
    k = 40
    p = tk.Plan(w.T, w.D, w.L, w.L, k, "bf16x3")
    idx, dist = p.knn(X)
    ld = p.local_dim(dist)
    rng = np.random.default_rng(8)
    crafted = np.sort(rng.uniform(1.0, 2.0, (1, p.np0, k)), axis=2)
    crafted[0, 0, :3] = 0.0          # duplicates below positive distances
    crafted[0, 1, :] = 5.0           # all equal
    crafted[0, 2, :] = 0.0           # all zero
    crafted[0, 3, :] *= 1e9          # scale
    ldc = p.local_dim(torch.from_numpy(crafted).cuda())
    torch.cuda.synchronize()
    dist_h, ld_h, ldc_h = dist.cpu().numpy()[0], ld.cpu().numpy()[0], ldc.cpu().numpy()[0]
    p.close()
    np.testing.assert_allclose(ld_h, oracle.local_dim(dist_h), rtol=1e-12)
    np.testing.assert_allclose(ldc_h, oracle.local_dim(crafted[0]), rtol=1e-12)
    assert np.all(np.isnan(ld_h[:, 0]))
    ref = oracle.local_dim(oracle.knn(Xn, w.L, k)[1])
    err = np.abs(ld_h[:, 1:] - ref[:, 1:])
    assert np.all(err <= _dim_tol(ref[:, 1:], 1e-5)), float(err.max())
    _say(f"  mean local dimension k'=20,30,40: "
         f"{[round(float(np.mean(ld_h[:, q - 1])), 2) for q in (20, 30, 40)]}")


@pytest.mark.parametrize("L,k,D", [(1, 1, 1), (2, 2, 3), (5, 10, 64), (16, 1, 7), (16, 64, 33),
                                   (3, 5, 1000)])
def test_smallest_legal_series(L, k, D):
    """T at the smallest value the plan accepts (n' = k + 2L - 1: every row has
    exactly k candidates or more, the middle row exactly k), one block, one
    chunk, every lane at an edge; lists against the oracle exactly (every
    candidate set is forced in the middle row) and the scores within the
    workload tolerance plus the norm-relative floor."""
    T = k + 3 * L - 2
    _say(f"[gpu] smallest legal series T={T} L={L} k={k} D={D}")
    rng = np.random.default_rng(L * 100 + k)
    Xn = (rng.standard_normal((T, D)) * 1000.0 + 101300.0).astype(np.float32)
    tk = _tk()
    with pytest.raises(tk.TraknnError):
        tk.Plan(T - 1, D, L, L, k, "bf16x3")
    for prec in ("fp32", "bf16x3"):
        idx, dist, s = _run(Xn, L, k, prec)
        n = T - L + 1
        ref = oracle.knn(Xn, L, k)
        Dm = oracle.traj_dist(Xn, L)
        stats = check_rows(Xn, L, k, np.arange(n), idx[0], dist[0], s[0], precision_tol(prec),
                           ref=(ref[0], ref[1], ref[2], ref[3], Dm),
                           norm_tol=gram_norm_tol(prec, D))
        _say(f"  {prec}: {stats}")
        # the middle row has exactly k candidates: its set is forced
        mid = (n - 1) // 2
        cands = [j for j in range(n) if abs(j - mid) >= L]
        if len(cands) == k:
            assert sorted(idx[0][mid].tolist()) == cands


def test_hip_graph_capture_replays():
    """The launch sequence allocates nothing and issues no memset, so a caller
    can capture knn + score (whole-matrix and band mode) and the backward in a
    HIP graph. Every replay, with eager work on the same buffers between
    replays, reproduces the eager results exactly."""
    tk = _tk()
    w = synth.WORKLOADS["tiny"]
    _say("[gpu] HIP graph capture and replay")
    Xn, _ = synth.make_workload(w)
    X = torch.from_numpy(Xn).cuda()
    for rb in (0, 64):
        p = tk.Plan(w.T, w.D, w.L, w.L, w.k, "bf16x3", row_batch=rb)
        idx, dist = p.empty_outputs()
        scores = torch.empty((1, p.np0), dtype=torch.float64, device="cuda")
        wts = torch.zeros(p.np0, dtype=torch.float64, device="cuda")
        wts[::7] = 1.0
        gX = torch.empty_like(X)
        p.knn(X, idx, dist)
        p.score(dist, scores)
        p.backward(X, idx[0], wts, grad_X=gX)
        torch.cuda.synchronize()
        ref = [t.clone() for t in (idx, dist, scores, gX)]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # warm-up on a side stream before capture
            p.knn(X, idx, dist)
            p.score(dist, scores)
            p.backward(X, idx[0], wts, grad_X=gX)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            p.knn(X, idx, dist)
            p.score(dist, scores)
            p.backward(X, idx[0], wts, grad_X=gX)
        for rep in range(3):
            idx.fill_(-7)
            dist.fill_(1.5)
            scores.fill_(2.5)
            gX.fill_(3.5)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for a, b in zip((idx, dist, scores, gX), ref):
                assert torch.equal(a, b), (rb, rep)
        del g
        p.close()
