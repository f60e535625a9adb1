"""Benchmark of the TRAKNN hot path on one MI355X.

Workload: T = 27394 daily fields (75 years) of a 64 x 128 grid (D = 8192),
trajectory length L = 5, k = 10 neighbours, synthetic SLP-shaped fields (see
paper_2603_02059_amd/synth.py). One step = one whole pass of the hot path on
device-resident X: centring/conversion, symmetric Gram + distances, window
recurrence + exclusion-zone top-k, merge, scores.

Metric: trajectory pairs per second, n'^2 / step time with n' = T - L + 1.
The headline path is the split BF16x3 Gram; the plain FP32 and single-pass
FP16 paths are timed beside it. One JSON line goes to stdout; progress to
stderr.

``--scaling`` instead times the default shape of the paper's scaling study
(Section 4: T = 27000 random fields of 180 x 280, d = 1, k = 1) as context
and prints one JSON line per precision.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAKS_TFLOPS = {"bf16x3": 2516.6, "fp16": 2516.6, "fp32": 157.3}  # dense MFMA
HBM_PEAK_GBS = 8000.0
GRAM_SOURCES = ("paper_2603_02059_amd/csrc/gram.hip",)
WINDOW_SOURCES = ("paper_2603_02059_amd/csrc/window_topk.hip",)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gram_bf16x3_T27394_D8192_traffic.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(paths=GRAM_SOURCES) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def gram_source_hash() -> str:
    return source_hash(GRAM_SOURCES)


def read_traffic_file() -> dict:
    kv = {}
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    a, b = line.split(":", 1)
                    kv[a.strip()] = b.strip()
    except OSError:
        pass
    return kv


def read_traffic():
    """HBM bytes per Gram launch from the committed rocprofv3 counter summary,
    or None if absent or taken on a different Gram kernel source."""
    kv = read_traffic_file()
    try:
        if kv.get("gram_source_sha256_16") != gram_source_hash():
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_window_traffic():
    """HBM bytes (read + written) per single-length window launch from the same
    summary, or None if absent or taken on a different window kernel source."""
    kv = read_traffic_file()
    try:
        if kv.get("window_source_sha256_16") != source_hash(WINDOW_SOURCES):
            return None
        return float(kv["window1_read_bytes"]) + float(kv["window1_write_bytes"])
    except (KeyError, ValueError):
        return None


def gram_flops(T: int, D: int, prec: str) -> float:
    """Algorithmic flops of one Gram launch: the T(T+1)/2 upper-triangle pairs
    (diagonal included) times 2D, times the 3 products of the split path."""
    passes = 3 if prec == "bf16x3" else 1
    return passes * 2.0 * D * T * (T + 1) / 2.0


def _pass_tiles(T: int, L_max: int, t0: int, nt: int) -> int:
    """Tiles of a band pass of nt trajectories from t0: its ceil(rows / 256)
    block-rows I against the block-columns J >= t0 // 256 + I (the tiles that
    hold entries above the diagonal)."""
    srows = min(nt + L_max - 1, T - t0)
    nbi, nbc = -(-srows // 256), -(-T // 256) - t0 // 256
    return nbi * nbc - nbi * (nbi - 1) // 2


def band_passes(T: int, L_min: int, L_max: int, rb: int, Dpad: int) -> list:
    """The band passes' (t0, rows), as the plan places them: starts on
    multiples of 8, at most rb rows each, minimising the passes' rounds of 256
    tiles plus 1 + 8192 / Dpad rounds per pass, trying for each start the
    longest pass of each of the 16 largest block-row counts (same rule, same
    order of evaluation as the library's planner)."""
    n = T - L_min + 1
    lam = 1.0 + 8192.0 / Dpad
    npos = (n + 7) // 8
    state = lambda t: npos if t >= n else t // 8
    cost, nxt = [0.0] * (npos + 1), [n] * (npos + 1)
    for i in range(npos - 1, -1, -1):
        t0, left = 8 * i, n - 8 * i
        nbi_max = -(-(min(rb, left) + L_max - 1) // 256)
        best, bt1, nbi = None, n, max(1, nbi_max - 15)
        while True:
            nt, last = (nbi * 256 - (L_max - 1)) // 8 * 8, False
            if nt >= rb:
                nt, last = rb, True
            if nt >= left:
                nt, last = left, True
            if nt > 0:
                c = -(-_pass_tiles(T, L_max, t0, nt) // 256) + lam + cost[state(t0 + nt)]
                if best is None or c < best:
                    best, bt1 = c, t0 + nt
            if last:
                break
            nbi += 1
        cost[i], nxt[i] = best, bt1
    out, t = [], 0
    while t < n:
        out.append((t, nxt[state(t)] - t))
        t = nxt[state(t)]
    return out


def band_tiles(T: int, L_min: int, L_max: int, rb: int, Dpad: int) -> int:
    """256 x 256 Gram tiles of all band passes."""
    return sum(_pass_tiles(T, L_max, t0, nt) for t0, nt in band_passes(T, L_min, L_max, rb, Dpad))


def window_bytes(T: int, L: int, rows: int = 8) -> dict:
    """Bytes of S the window/top-k stage must read: the algorithmic figure is
    the upper triangle once (4 T(T+1)/2 B); this design reads every row of S
    (both triangles, so each row's candidates are contiguous) plus the L - 1
    halo rows of each block of `rows` rows."""
    return {"algorithmic_bytes": 4.0 * T * (T + 1) / 2,
            "design_bytes": 4.0 * T * T * (rows + L - 1) / rows}


def time_path(tk, torch, X, w, prec, steps, warmup, row_batch=0):
    p = tk.Plan(w.T, w.D, w.L, w.L, w.k, prec, row_batch=row_batch)
    idx, dist = p.empty_outputs()
    scores = torch.empty((1, p.np0), dtype=torch.float64, device=X.device)
    for _ in range(warmup):
        p.knn(X, idx, dist)
        p.score(dist, scores)
    torch.cuda.synchronize()
    p.set_timing(True)
    stage_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p.knn(X, idx, dist)
        p.score(dist, scores)
        stage_ms.append(p.stage_times())  # waits for this step's last stage event
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    p.set_timing(False)
    out = {
        "prec": prec,
        "ms_per_step": 1e3 * total / steps,
        "stage_ms": {k: float(np.mean([s[k] for s in stage_ms])) for k in stage_ms[0]},
        "idx": idx[0],
        "dist": dist[0],
        "scores": scores[0],
        "ws_bytes": p.ws_bytes,
    }
    p.close()
    return out


def time_sweep(tk, torch, X, w, steps, warmup, L_max=10):
    """The all-lengths configuration: L = 1..L_max in one call on the full
    workload, BF16x3 (one Gram, the window passes two lengths at a time)."""
    p = tk.Plan(w.T, w.D, 1, L_max, w.k, "bf16x3")
    idx, dist = p.empty_outputs()
    scores = torch.empty((p.NL, p.np0), dtype=torch.float64, device=X.device)
    for _ in range(warmup):
        p.knn(X, idx, dist)
        p.score(dist, scores)
    torch.cuda.synchronize()
    p.set_timing(True)
    st = []
    t0 = time.perf_counter()
    for _ in range(steps):
        p.knn(X, idx, dist)
        p.score(dist, scores)
        st.append(p.stage_times())
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    p.set_timing(False)
    out = {"lengths": f"1..{L_max}", "ms_per_call": ms,
           "stage_ms": {k: float(np.mean([s[k] for s in st])) for k in st[0]},
           "idx": idx, "dist": dist, "scores": scores}
    p.close()
    return out


def sweep_parity(Xn, w, sweep, L_max, nrows, starts):
    """Per-length agreement of the sweep with the oracle on the same sampled
    rows for every L = 1..L_max (evenly spaced, plus the planted starts), all
    lengths from one oracle pass over X: set differences (admitted only at
    oracle gaps below 1e-5), maximum distance and score errors."""
    import oracle
    from tests.parity import check_rows

    n_last = w.T - L_max + 1
    rows = set(np.linspace(0, n_last - 1, nrows).astype(int).tolist())
    rows |= {s for s in starts if s < n_last}
    rows = np.array(sorted(rows), dtype=np.int64)
    t0 = time.perf_counter()
    refs = oracle.knn_rows_multi(Xn, L_max, w.k, rows)
    el = time.perf_counter() - t0
    gi = sweep["idx"].cpu().numpy()
    gd = sweep["dist"].cpu().numpy()
    gs = sweep["scores"].cpu().numpy()
    per_L = []
    for L in range(1, L_max + 1):
        try:
            st = check_rows(Xn, L, w.k, rows, gi[L - 1][rows], gd[L - 1][rows],
                            gs[L - 1][rows], 1e-5, ref=refs[L - 1], label=f"bench sweep L={L}")
            ok = True
        except AssertionError as e:  # reported, not hidden
            st, ok = {"error": str(e)[:200]}, False
        per_L.append({"L": L, "pass": ok, "rows": int(rows.size),
                      **{k: st.get(k) for k in ("set_diff_rows", "max_dist_rel_err",
                                                "max_score_rel_err")}})
    return {"rows_per_L": int(rows.size), "oracle_s": el, "per_L": per_L}


def time_small_d(tk, torch, synth, steps, warmup):
    """The PCA-sized shape of the paper's trajectory-space study: T = 27394
    fields of 4 x 8 (D = 32), L = 5, k = 40 (the largest k of its intrinsic-
    dimension estimates), BF16x3; one call is knn plus the local dimension
    for every k' <= k. The Gram is tiny here and the window/top-k stage
    dominates."""
    T, H, W, L, k = 27394, 4, 8, 5, 40
    Xn, _ = synth.make_fields(T, H, W, sigma=1.0, n_events=20, event_len=L, seed=4)
    X = torch.from_numpy(Xn).cuda()
    p = tk.Plan(T, H * W, L, L, k, "bf16x3")
    idx, dist = p.empty_outputs()
    dims = torch.empty((p.NL, p.np0, k), dtype=torch.float64, device=X.device)
    for _ in range(warmup):
        p.knn(X, idx, dist)
        p.local_dim(dist, dims)
    torch.cuda.synchronize()
    p.set_timing(True)
    st = []
    t0 = time.perf_counter()
    for _ in range(steps):
        p.knn(X, idx, dist)
        p.local_dim(dist, dims)
        st.append(p.stage_times())
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    p.set_timing(False)
    stage = {q: float(np.mean([s[q] for s in st])) for q in st[0]}
    n = T - L + 1
    win = window_bytes(T, L)
    m = dims[0, :, [19, 29, 39]].nanmean(dim=0).cpu().numpy()
    out = {"config": f"T={T}, {H}x{W} grid (D={H * W}), L={L}, k={k}, BF16x3, knn + local dimension",
           "ms_per_call": ms, "pairs_per_s": float(n) * n / (ms * 1e-3), "stage_ms": stage,
           "window_design_GBps": win["design_bytes"] / (stage["window_topk"] * 1e-3) / 1e9,
           "mean_local_dim_k20_k30_k40": [float(v) for v in m]}
    p.close()
    del X
    torch.cuda.empty_cache()
    return out


def time_mode(tk, torch, Xn, L, k, prec, mode, steps, warmup):
    """ms per knn call (and the stage split) of one mode and precision."""
    X = torch.from_numpy(Xn).cuda()
    p = tk.Plan(Xn.shape[0], Xn.shape[1], L, L, k, prec, mode=mode)
    idx, dist = p.empty_outputs()
    for _ in range(warmup):
        p.knn(X, idx, dist)
    torch.cuda.synchronize()
    p.set_timing(True)
    st = []
    t0 = time.perf_counter()
    for _ in range(steps):
        p.knn(X, idx, dist)
        st.append(p.stage_times())
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    p.set_timing(False)
    out = {"mode": mode, "prec": prec, "ms_per_call": ms,
           "pairs_per_s": float(Xn.shape[0] - L + 1) ** 2 / (ms * 1e-3),
           "stage_ms": {q: round(float(np.mean([s[q] for s in st])), 4) for q in st[0]},
           "workspace_GiB": p.ws_bytes / 2 ** 30}
    res = (idx[0].cpu().numpy(), dist[0].cpu().numpy())
    p.close()
    del X, idx, dist
    torch.cuda.empty_cache()
    return out, res


def time_fused(tk, torch, synth, Xfull, w, steps, warmup):
    """The fused (S-free) mode beside the matrix mode: the headline workload
    in BF16x3 (and whether its lists and distances equal the matrix mode's
    bit for bit), and the small-D shapes of the PCA comparison (a 4 x 8 grid
    and the full workload's 13 leading principal components) at k = 10 and
    40, where the fused mode also runs in FP64."""
    out = {}
    m, rm = time_mode(tk, torch, Xfull, w.L, w.k, "bf16x3", "matrix", steps, warmup)
    f, rf = time_mode(tk, torch, Xfull, w.L, w.k, "bf16x3", "fused", steps, warmup)
    f["equal_to_matrix_mode"] = bool(np.array_equal(rm[0], rf[0]) and np.array_equal(rm[1], rf[1]))
    out["headline"] = {"shape": f"T={w.T}, D={w.D}, L={w.L}, k={w.k}", "matrix": m, "fused": f}
    log(f"[bench] fused headline: matrix {m['ms_per_call']:.2f} ms, fused {f['ms_per_call']:.2f} ms")
    g32, _ = synth.make_fields(w.T, 4, 8, sigma=1.0, n_events=20, event_len=5, seed=4)
    pca, _, frac = synth.make_pca_workload(13)
    for name, Xn in (("grid 4x8 (D=32)", g32), ("PCA 13 (D=13)", pca)):
        for k in (10, 40):
            row = {}
            for prec, mode in (("bf16x3", "matrix"), ("bf16x3", "fused"), ("fp64", "fused")):
                row[f"{prec}_{mode}"] = time_mode(tk, torch, Xn, w.L, k, prec, mode, steps,
                                                  warmup)[0]
            out[f"{name}, k={k}"] = row
            log(f"[bench] fused {name} k={k}: " + ", ".join(
                f"{q} {v['ms_per_call']:.2f} ms" for q, v in row.items()))
    out["pca13_explained_variance"] = frac
    return out


def time_vendor_gemm(torch, T, D, steps):
    """torch.matmul (hipBLASLt) in BF16 on the Gram's shape padded to whole
    256-row tiles, the full square (2 n^2 D flop): the vendor's rate for a
    plain GEMM of this size, beside which the Gram's counters are read."""
    n = -(-T // 256) * 256
    g = torch.Generator(device="cuda").manual_seed(0)
    a = torch.randn(n, D, dtype=torch.bfloat16, device="cuda", generator=g)
    b = a.t().contiguous()
    c = torch.matmul(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        torch.matmul(a, b, out=c)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    out = {"shape": f"[{n} x {D}] @ [{D} x {n}], bf16 in and out", "ms": ms,
           "tflops": 2.0 * n * n * D / (ms * 1e-3) / 1e12}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def time_backward(tk, torch, synth, steps):
    """The differentiation configuration: T = 10957 daily 64 x 128 fields,
    L = 5, k = 10, FP32 forward, then the backward of the summed score of the
    100 rarest trajectories (neighbour sets held fixed)."""
    w = synth.WORKLOADS["bwd"]
    Xn, _ = synth.make_workload(w)
    X = torch.from_numpy(Xn).cuda()
    p = tk.Plan(w.T, w.D, w.L, w.L, w.k, "fp32")
    idx, dist = p.knn(X)
    s = p.score(dist)[0]
    wts = torch.zeros_like(s)
    wts[torch.argsort(-s)[:100]] = 1.0
    g = p.backward(X, idx[0], wts)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(steps):
        p.knn(X, idx, dist)
    e[1].record()
    for _ in range(steps):
        p.backward(X, idx[0], wts, grad_X=g)
    e[2].record()
    torch.cuda.synchronize()
    out = {"config": f"T={w.T}, D={w.D}, L={w.L}, k={w.k}, FP32, 100 rarest",
           "forward_ms": e[0].elapsed_time(e[1]) / steps,
           "backward_ms": e[1].elapsed_time(e[2]) / steps}
    p.close()
    return out


def cpu_model() -> str | None:
    """The host CPU's model name as /proc/cpuinfo reports it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(Xn, w, budget_s, gidx, gdist, gscore):
    """The FP64 oracle on evenly spaced sample rows, timed on the host cores,
    plus the parity of the GPU rows against it."""
    import oracle
    from tests.parity import check_rows

    n = w.T - w.L + 1
    order = np.linspace(0, n - 1, 4096).astype(np.int64)
    threads = oracle.num_threads()
    done = []
    res = []
    t0 = time.perf_counter()
    batch = 8
    for b in range(0, len(order), batch):
        rows = order[b:b + batch]
        res.append(oracle.knn_rows(Xn, w.L, w.k, rows))
        done.extend(rows.tolist())
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    rows = np.array(done, dtype=np.int64)
    ref = tuple(np.concatenate([r[i] for r in res]) for i in range(5))
    try:
        par = check_rows(Xn, w.L, w.k, rows, gidx[rows], gdist[rows], gscore[rows], 1e-5,
                         ref=ref)
        par["pass"] = True
    except AssertionError as e:  # reported, not hidden
        par = {"pass": False, "rows": len(rows), "error": str(e)[:300]}
    return {
        "value": len(rows) * n / el,
        "unit": "pairs/s",
        "cores": threads,
        "nproc": os.cpu_count(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": f"{len(rows)} evenly spaced rows x {n} candidates each of the same "
                  f"workload (FP64 direct differences, direct L-sums, sorted top-k), "
                  f"{el:.1f} s",
    }, par


def scaling(tk, torch, steps, warmup):
    """Time the default shape of the paper's scaling study (Section 4: T =
    27000 random fields of 180 x 280, d = 1, k = 1; the paper evaluates on
    random data) in BF16x3 and FP32, as context only."""
    T, D, L, k = 27000, 180 * 280, 1, 1
    gen = torch.Generator(device="cuda")
    for prec in ("bf16x3", "fp32"):
        gen.manual_seed(T * 7 + D)
        X = torch.randn((T, D), generator=gen, device="cuda", dtype=torch.float32)
        p = tk.Plan(T, D, L, L, k, prec)
        idx, dist = p.empty_outputs()
        scores = torch.empty((1, p.np0), dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            p.knn(X, idx, dist)
            p.score(dist, scores)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            p.knn(X, idx, dist)
            p.score(dist, scores)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        n = T - L + 1
        line = {"shape": {"T": T, "h": 180, "w": 280, "d": L, "k": k, "prec": prec},
                "D": D, "ms_per_call": ms, "pairs_per_s": n * n / (ms * 1e-3),
                "workspace_GiB": p.ws_bytes / 2 ** 30}
        print(json.dumps(line), flush=True)
        p.close()
        del X, idx, dist, scores
        torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="full")
    ap.add_argument("--compare-steps", type=int, default=3,
                    help="timed steps of the FP32 and FP16 comparison paths")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline (0 = skip)")
    ap.add_argument("--only", default=None, help="time one precision only")
    ap.add_argument("--sweep-rows", type=int, default=64,
                    help="oracle rows per length checked for the all-lengths sweep (0 = skip)")
    ap.add_argument("--no-fused", action="store_true",
                    help="skip the fused-mode comparison")
    ap.add_argument("--no-backward", action="store_true",
                    help="skip the backward timing (T = 10957 configuration)")
    ap.add_argument("--scaling", action="store_true",
                    help="time the paper's scaling-study shapes instead (one JSON line each)")
    ap.add_argument("--band-rows", type=int, default=4088,
                    help="also time band mode (row-batched streaming) with passes of "
                         "this many rows, BF16x3 (0 = skip)")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="also run a plain device copy of this many GiB (counter scale)")
    ap.add_argument("--vendor-gemm", action="store_true",
                    help="also time the vendor BF16 GEMM (torch.matmul) on the Gram's "
                         "square shape, as a reference for the Gram's counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path "
              "(the tile pairs would shard across GPUs with one exchange of partial "
              "neighbour lists).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2603_02059_amd import synth
    from paper_2603_02059_amd import traknn as tk

    if args.scaling:
        scaling(tk, torch, max(1, min(args.steps, 5)), max(1, args.warmup))
        return

    w = synth.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    Xn, starts = synth.make_workload(w)
    log(f"[bench] generated {w.name}: T={w.T} D={w.D} L={w.L} k={w.k} in "
        f"{time.perf_counter() - t0:.1f}s")
    X = torch.from_numpy(Xn).cuda()
    torch.cuda.synchronize()

    if args.calibrate_copy_gib > 0:
        nb = int(args.calibrate_copy_gib * 2 ** 30) // 4
        a = torch.ones(nb, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {4 * nb} bytes done")
        del a, b

    n = w.T - w.L + 1
    pairs = float(n) * float(n)
    precs = [args.only] if args.only else ["bf16x3", "fp32", "fp16"]
    results = {}
    for prec in precs:
        steps = args.steps if prec == precs[0] else args.compare_steps
        log(f"[bench] timing {prec}: {args.warmup} warmup + {steps} steps")
        r = time_path(tk, torch, X, w, prec, steps, args.warmup)
        r["pairs_per_s"] = pairs / (r["ms_per_step"] * 1e-3)
        g = r["stage_ms"]["gram"]
        r["gram_tflops"] = gram_flops(w.T, w.D, prec) / (g * 1e-3) / 1e12
        r["gram_fp32_equiv_tflops"] = gram_flops(w.T, w.D, "fp32") / (g * 1e-3) / 1e12
        log(f"[bench] {prec}: {r['ms_per_step']:.2f} ms/step, "
            f"{r['pairs_per_s']:.3e} pairs/s, stages {r['stage_ms']}, "
            f"gram {r['gram_tflops']:.1f} TFLOP/s")
        results[prec] = r

    vendor = None
    if args.vendor_gemm:
        vendor = time_vendor_gemm(torch, w.T, w.D, max(args.compare_steps, 3))
        log(f"[bench] vendor GEMM: {vendor}")

    band = None
    if args.band_rows > 0 and not args.only:
        log(f"[bench] timing bf16x3 band mode, passes of {args.band_rows} rows: "
            f"{args.warmup} warmup + {args.compare_steps} steps")
        r = time_path(tk, torch, X, w, "bf16x3", args.compare_steps, args.warmup,
                      row_batch=args.band_rows)
        rb = args.band_rows
        Dpad = -(-w.D // 32) * 32  # the BF16x3 Gram's contraction depth
        passes = band_passes(w.T, w.L, w.L, rb, Dpad)
        ntiles = band_tiles(w.T, w.L, w.L, rb, Dpad)
        flops = 3 * 2.0 * Dpad * 256 * 256 * ntiles
        band = {"row_batch": rb, "passes": len(passes),
                "gram_rounds": sum(-(-_pass_tiles(w.T, w.L, t0, nt) // 256) for t0, nt in passes),
                "ms_per_step": r["ms_per_step"],
                "pairs_per_s": pairs / (r["ms_per_step"] * 1e-3),
                "passes_ms": r["stage_ms"]["gram"],
                "mfma_work_vs_algorithmic": flops / gram_flops(w.T, w.D, "bf16x3"),
                "gram_tiles_vs_whole_matrix":
                    ntiles / (-(-w.T // 256) * (-(-w.T // 256) + 1) / 2),
                "workspace_GiB": r["ws_bytes"] / 2 ** 30,
                "whole_matrix_workspace_GiB": results.get("bf16x3", r)["ws_bytes"] / 2 ** 30}
        if "bf16x3" in results:
            a = np.sort(r["idx"].cpu().numpy(), 1)
            b = np.sort(results["bf16x3"]["idx"].cpu().numpy(), 1)
            band["rows_with_whole_matrix_set"] = float(np.all(a == b, axis=1).mean())
        log(f"[bench] band mode: {band}")

    sweep = None
    if not args.only:
        log("[bench] timing the all-lengths sweep L=1..10")
        sweep = time_sweep(tk, torch, X, w, args.compare_steps, args.warmup)
        if args.sweep_rows > 0:
            log(f"[bench] sweep parity: {args.sweep_rows} oracle rows per length")
            sweep["parity"] = sweep_parity(Xn, w, sweep, 10, args.sweep_rows, starts)
        for key in ("idx", "dist", "scores"):
            sweep.pop(key)
        log(f"[bench] sweep: {sweep}")

    small = None
    if not args.only:
        log("[bench] timing the small-D (PCA-sized) shape, k = 40, with the local dimension")
        small = time_small_d(tk, torch, synth, args.compare_steps, args.warmup)
        log(f"[bench] small D: {small}")

    fused = None
    if not args.only and not args.no_fused:
        log("[bench] timing the fused (S-free) mode beside the matrix mode")
        fused = time_fused(tk, torch, synth, Xn, w, args.compare_steps, args.warmup)

    bwd = None
    if not args.no_backward and not args.only:
        log("[bench] timing the backward configuration")
        bwd = time_backward(tk, torch, synth, max(args.compare_steps, 5))
        log(f"[bench] backward: {bwd}")

    head = results[precs[0]]
    hp = head["prec"]
    gidx = head["idx"].cpu().numpy()
    gdist = head["dist"].cpu().numpy()
    gscore = head["scores"].cpu().numpy()
    rarest = np.argsort(-gscore, kind="stable")[:40]
    planted_found = sum(1 for s in starts if s in set(rarest.tolist()))

    cpu, par = None, None
    if args.cpu_budget > 0:
        log(f"[bench] oracle CPU baseline (~{args.cpu_budget:.0f}s) ...")
        cpu, par = cpu_baseline(Xn, w, args.cpu_budget, gidx, gdist, gscore)
        log(f"[bench] cpu baseline {cpu['value']:.3e} pairs/s on {cpu['cores']} threads; "
            f"parity on {par['rows']} rows: {par}")

    gram_ms = head["stage_ms"]["gram"]
    achieved = gram_flops(w.T, w.D, hp) / (gram_ms * 1e-3) / 1e12
    traffic = read_traffic() if hp == "bf16x3" and w.name == "full" else None
    wb = window_bytes(w.T, w.L)
    win_ms = head["stage_ms"]["window_topk"]
    wt = read_window_traffic() if hp == "bf16x3" and w.name == "full" else None
    window_hbm = {"kernel": f"window1_kernel<{w.L}, 1>", "avg_launch_ms": win_ms,
                  "algorithmic_GBps": wb["algorithmic_bytes"] / (win_ms * 1e-3) / 1e9,
                  "design_GBps": wb["design_bytes"] / (win_ms * 1e-3) / 1e9,
                  "counter_bytes": wt,
                  "counter_GBps": wt / (win_ms * 1e-3) / 1e9 if wt else None,
                  "peak_GBps": HBM_PEAK_GBS, **wb}
    line = {
        "metric": "trajectory pairs/sec at T=27394,D=8192,L=5,k=10; Gram MFMA util vs FP32 path",
        "value": head["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3" if hp == "bf16x3" else hp,
        "data": "synthetic SLP-shaped fields (seeded), device-resident",
        "config": {"workload": f"{w.name}: T={w.T} daily fields, {w.H}x{w.W} grid (D={w.D}), "
                               f"L={w.L}, k={w.k}, exclusion |i-j|<{w.L}, {w.n_events} planted "
                               f"{w.event_len}-day dipoles",
                   "T": w.T, "D": w.D, "L": w.L, "k": w.k, "precision": hp,
                   "pairs_per_step": pairs},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAKS_TFLOPS[hp],
                     "unit": "TFLOP/s", "frac": achieved / PEAKS_TFLOPS[hp],
                     "traffic": traffic, "kernel": f"gram_kernel<{hp}>",
                     "avg_launch_ms": gram_ms},
        "cpu_baseline": cpu,
        "stages_ms": {p: {k: round(v, 4) for k, v in r["stage_ms"].items()}
                      for p, r in results.items()},
        "paths": {p: {"ms_per_step": r["ms_per_step"], "pairs_per_s": r["pairs_per_s"],
                      "gram_tflops": r["gram_tflops"],
                      "gram_mfma_frac": r["gram_tflops"] / PEAKS_TFLOPS[p],
                      "gram_fp32_equiv_tflops": r["gram_fp32_equiv_tflops"]}
                  for p, r in results.items()},
        "window_hbm": window_hbm,
        "band_mode": band,
        "sweep": sweep,
        "small_d": small,
        "fused": fused,
        "vendor_gemm": vendor,
        "backward": bwd,
        "parity_sample": par,
        "planted_in_top40": f"{planted_found}/{len(starts)}",
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
