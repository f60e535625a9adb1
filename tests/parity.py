"""Parity rules shared by the GPU tests: compare the HIP path's neighbour lists,
distances and scores with the FP64 oracle on the same seeded inputs.

Neighbour sets are unique except at (near-)ties, so the rule is:
  * the GPU list of each row is sorted by (distance, index), respects the
    exclusion zone |t - j| >= L and stays inside [0, n');
  * every GPU distance matches the oracle's distance of the same pair within
    ``tol`` (relative);
  * the GPU set equals the oracle set, except on rows whose oracle gap
    (delta_{k+1} - delta_k) / delta_k is below ``tol``; there every GPU
    neighbour the oracle did not pick must have an oracle distance within
    ``tol`` of delta_k;
  * scores match within ``tol`` (relative; absolute 0 where the oracle's is 0).

The set and score rules are always exactly these. Off-workload edge cases
(L = 1, k = 1, odd grids) can hold pairs whose distance is a small fraction of
their norms; there the Gram identity (Eq. 4) evaluated with FP32 accumulation
has an error proportional to the norms, not the distance, so those tests add
``norm_tol`` times the pair's sum of centred snapshot norms to the allowance of
each individual neighbour distance (see ``gram_norm_tol``), and to nothing
else. Every call logs its error statistics (``_log_stats``).
"""
from __future__ import annotations

import math

import numpy as np

import oracle


def precision_tol(prec: str) -> float:
    # Score/distance tolerance per Gram precision on SLP-shaped data: 1e-5 for the
    # split BF16x3 path, 1e-3 for the single FP16 pass, and the split path's
    # 1e-5 for the plain FP32 path.
    return {"fp32": 1e-5, "bf16x3": 1e-5, "fp16": 1e-3}[prec]


def gram_norm_tol(prec: str, D: int) -> float:
    """Norm-relative error allowance of d = N_i + N_j - 2G in a precision.

    Accumulation: n roundings of an FP32 running sum bounded by the norms give
    an error ~ sqrt(n) 2^-24 (N_i + N_j) (random-walk model); n = Dpad/2 for
    FP32 MFMA (2 products per step), 3 Dpad/16 for BF16x3 and Dpad/16 for FP16
    (16 products per step). Representation: per-element relative error e of the
    rounded centred field (2^-24, 2^-16 for hi+lo, 2^-11) perturbs d by about
    e sqrt(2/D) (N_i + N_j). Allowance = 4x the first + 8x the second."""
    step = {"fp32": 2, "bf16x3": 16 / 3, "fp16": 16}[prec]
    kdepth = {"fp32": 32, "bf16x3": 32, "fp16": 64}[prec]
    dpad = math.ceil(D / kdepth) * kdepth
    n = dpad / step
    rep = {"fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16, "fp16": 2.0 ** -11}[prec]
    return 4.0 * math.sqrt(n) * 2.0 ** -24 + 8.0 * rep * math.sqrt(2.0 / D)


def snapshot_norms(X) -> np.ndarray:
    """Squared norms of the per-cell centred snapshots (tolerance model only)."""
    Xd = np.asarray(X, dtype=np.float64).reshape(len(X), -1)
    Xc = Xd - Xd.mean(0)
    return (Xc * Xc).sum(1)


def _pair_normsum(N, L, t, js):
    js = np.asarray(js)
    return sum(N[t + m] + N[js + m] for m in range(L))


def _log_stats(stats: dict, label: str | None) -> None:
    """Append one JSON line of error statistics to gpurun_out/parity_stats.jsonl
    (the folder a GPU run brings back) under the running test's name."""
    import json
    import os
    name = label or os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = os.path.join(root, "gpurun_out")
    try:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "parity_stats.jsonl"), "a") as f:
            f.write(json.dumps({"test": name, **stats}) + "\n")
    except OSError:
        pass


def check_rows(X, L: int, k: int, rows, gidx, gdist, gscore, tol: float,
               ref=None, norm_tol: float = 0.0, label: str | None = None) -> dict:
    """Check GPU outputs for ``rows`` (gidx/gdist [len(rows), k], gscore
    [len(rows)]) against the oracle. Returns error statistics, which are also
    logged before any assertion fires.

    The set rule (differences only where the oracle gap is below ``tol``) and
    the score rule (relative error at most ``tol``) are always the stated
    ones. ``norm_tol`` only widens the per-neighbour distance check."""
    rows = np.asarray(rows, dtype=np.int64)
    N = snapshot_norms(X) if norm_tol > 0 else None
    if ref is None:
        ridx, rdist, rscore, rgap, drows = oracle.knn_rows(X, L, k, rows)
    else:
        ridx, rdist, rscore, rgap, drows = ref
    n = drows.shape[1]
    gidx = np.asarray(gidx)
    gdist = np.asarray(gdist, dtype=np.float64)
    gscore = np.asarray(gscore, dtype=np.float64)
    d_errs, s_errs, fails = [], [], []
    set_diff_rows = 0
    min_gap_diff = None
    for r, t in enumerate(rows):
        gi = gidx[r]
        assert np.all((gi >= 0) & (gi < n)), f"row {t}: index out of range {gi}"
        assert np.all(np.abs(gi - t) >= L), f"row {t}: exclusion zone violated {gi}"
        assert len(set(gi.tolist())) == k, f"row {t}: duplicate neighbours {gi}"
        keys = list(zip(gdist[r].tolist(), gi.tolist()))
        assert keys == sorted(keys), f"row {t}: list not in (distance, index) order"
        od = drows[r, gi]
        extra_allow = (norm_tol * _pair_normsum(N, L, t, gi) if norm_tol > 0
                       else np.zeros(k))
        allow = tol * np.abs(od) + extra_allow
        aerr = np.abs(gdist[r] - od)
        scale = np.maximum(np.abs(od), 1e-300)
        derr = np.where(od == 0, np.abs(gdist[r]), aerr / scale)
        d_errs.append(derr)
        if not np.all(aerr <= allow):
            fails.append(f"row {t}: distance error {derr.max():.3e} beyond tolerance "
                         f"(tol {tol}, norm_tol {norm_tol})")
        if set(gi.tolist()) != set(ridx[r].tolist()):
            set_diff_rows += 1
            dk = rdist[r, -1]
            slack = tol * dk  # the stated rule: the oracle gap is below tol
            g = float(rgap[r])
            min_gap_diff = g if min_gap_diff is None else min(min_gap_diff, g)
            if not rgap[r] * dk <= slack:
                fails.append(f"row {t}: neighbour set differs with oracle gap {g:.3e}: "
                             f"gpu {sorted(gi)} oracle {sorted(ridx[r])}")
            extra = [j for j in gi.tolist() if j not in set(ridx[r].tolist())]
            for j in extra:
                if not abs(drows[r, j] - dk) <= slack:
                    fails.append(f"row {t}: gpu neighbour {j} is not a near-tie of the k-th")
        if rscore[r] == 0:
            serr = abs(gscore[r])
        else:
            serr = abs(gscore[r] - rscore[r]) / abs(rscore[r])
        s_errs.append(serr)
        if not serr <= tol:
            fails.append(f"row {t}: score error {serr:.3e} beyond tolerance {tol}")
    dcat = np.concatenate(d_errs) if d_errs else np.zeros(1)
    stats = {"max_dist_rel_err": float(dcat.max()),
             "max_score_rel_err": float(max(s_errs)) if s_errs else 0.0,
             "p99_dist_rel_err": float(np.percentile(dcat, 99)),
             "p99_score_rel_err": float(np.percentile(s_errs, 99)) if s_errs else 0.0,
             "set_diff_rows": set_diff_rows, "rows": len(rows),
             "min_oracle_gap_of_differing_rows": min_gap_diff,
             "tol": tol, "norm_tol": norm_tol, "L": L, "k": k,
             "failures": len(fails)}
    _log_stats(stats, label)
    assert not fails, f"{len(fails)} parity failures; first: " + "; ".join(fails[:3])
    return stats
