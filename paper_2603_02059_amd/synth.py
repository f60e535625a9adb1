"""Seeded synthetic sea-level-pressure-shaped fields (inputs only, no method arithmetic).

This module only draws inputs. It holds none of the distance, recurrence or
neighbour arithmetic, so the FP64 oracle and the GPU path can both be fed from
it without sharing any part of what they compute.

The paper's case study runs on 75 years of daily ERA5 mean sea-level pressure
over Europe (Section 5). That dataset is not available here, so these fields
stand in for it, with the properties the method is sensitive to:

* a ~1e5 Pa offset (101300 Pa), which makes uncentred low-precision Gram
  products cancel catastrophically;
* an annual cycle (800 Pa sinusoid, period 365.25 days, phase 0, uniform in
  space);
* synoptic persistence: AR(1) noise in time with phi = 0.8 (e-folding ~4.5 days,
  the 3-7 day life cycle of a cyclone named in Section 3.1), marginal standard
  deviation 1000 Pa per cell;
* spatial smoothness: each white-noise field is smoothed with a separable,
  periodic Gaussian of sigma_s cells (truncated at 4 sigma) and rescaled so every
  cell has unit variance before the AR(1) step;
* planted rare trajectories: a dipole (+A and -A Gaussian lobes, sigma_d = W/8
  cells, lobe centres 3 sigma_d apart at a random angle around a random centre)
  held fixed over ``event_len`` consecutive days.

Everything is drawn in float64 and cast once to float32 (row-major [T, H*W],
time-major), which is the canonical input of both implementations.

``pca_scores`` reduces such fields to their leading principal components, the
reduced inputs of the paper's PCA comparison (Section 5.1, which keeps 33
components, 99% of the variance of its data, or 13, 95%), by the same kind of
randomized low-rank SVD the paper uses. It is input preparation: the scores
are cast to float32 and then fed to both implementations like any field.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

OFFSET_PA = 101300.0
SEASON_AMP_PA = 800.0
SEASON_PERIOD_DAYS = 365.25
NOISE_STD_PA = 1000.0
AR_PHI = 0.8
EVENT_AMP_PA = 4000.0


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: grid, length, smoothing and planted events."""

    name: str
    T: int
    H: int
    W: int
    sigma: float
    L: int
    k: int
    n_events: int
    event_len: int
    event_starts: tuple | None = None  # fixed starts; None draws them
    seed: int = 0

    @property
    def D(self) -> int:
        return self.H * self.W


# The workloads the method is measured and checked on.  Length and grid follow
# the case study's data (75 years of daily fields, Section 5), trajectory
# duration and k the runs of its PCA comparison (d = 5, k = 10, Section 5.1);
# the tiny one is small enough for the oracle to finish in seconds.
WORKLOADS = {
    "tiny": Workload("tiny", 512, 32, 32, 3.0, 3, 5, 1, 3, (256,)),
    "full": Workload("full", 27394, 64, 128, 6.0, 5, 10, 20, 5),
    "split": Workload("split", 27394, 128, 256, 12.0, 5, 10, 20, 5),
    "bwd": Workload("bwd", 10957, 64, 128, 6.0, 5, 10, 20, 5),
}


def _periodic_gauss_transfer(n: int, sigma: float) -> tuple[np.ndarray, float]:
    """Transfer function of a periodic Gaussian of ``sigma`` cells on ``n`` cells,
    truncated at 4 sigma, and the sum of squares of its wrapped taps."""
    r = int(math.ceil(4.0 * sigma))
    offs = np.arange(-r, r + 1)
    taps = np.exp(-0.5 * (offs / sigma) ** 2)
    taps /= taps.sum()
    wrapped = np.zeros(n)
    np.add.at(wrapped, offs % n, taps)
    return np.fft.fft(wrapped), float((wrapped ** 2).sum())


def _event_starts(T: int, n_events: int, event_len: int, rng) -> list[int]:
    """Starts at least 2*event_len + 30 days apart and event_len from either edge."""
    gap = 2 * event_len + 30
    lo, hi = event_len, T - 2 * event_len
    if n_events == 0:
        return []
    span = hi - lo - (n_events - 1) * gap
    if span < 0:
        raise ValueError("series too short for the requested planted events")
    # sorted uniform draws in the free span, then spread by the minimum gap
    base = np.sort(rng.integers(0, span + 1, size=n_events))
    return [int(lo + b + i * gap) for i, b in enumerate(base)]


def _dipole(H: int, W: int, rng) -> np.ndarray:
    sd = W / 8.0
    half = 1.5 * sd
    cy = rng.uniform(half + sd, H - half - sd) if H > 2 * (half + sd) else H / 2.0
    cx = rng.uniform(half + sd, W - half - sd) if W > 2 * (half + sd) else W / 2.0
    ang = rng.uniform(0.0, 2.0 * math.pi)
    dy, dx = half * math.sin(ang), half * math.cos(ang)
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")

    def lobe(y0, x0):
        return np.exp(-0.5 * ((yy - y0) ** 2 + (xx - x0) ** 2) / sd ** 2)

    return EVENT_AMP_PA * (lobe(cy + dy, cx + dx) - lobe(cy - dy, cx - dx))


def make_fields(T: int, H: int, W: int, sigma: float, n_events: int = 0,
                event_len: int = 1, seed: int = 0, event_starts=None,
                chunk: int = 1024) -> tuple[np.ndarray, list[int]]:
    """Draw the [T, H*W] float32 field sequence and the planted event starts."""
    rng = np.random.default_rng(seed)
    ty, vy = _periodic_gauss_transfer(H, sigma)
    tx, vx = _periodic_gauss_transfer(W, sigma)
    transfer = np.outer(ty, tx)
    rescale = 1.0 / math.sqrt(vy * vx)
    innov = math.sqrt(1.0 - AR_PHI * AR_PHI)

    out = np.empty((T, H * W), dtype=np.float32)
    prev = None
    for c0 in range(0, T, chunk):
        c1 = min(T, c0 + chunk)
        white = rng.standard_normal((c1 - c0, H, W))
        sm = np.fft.ifft2(np.fft.fft2(white) * transfer).real * rescale
        e = np.empty_like(sm)
        for i in range(c1 - c0):
            if prev is None:
                e[i] = sm[i]  # stationary start: unit marginal variance
            else:
                e[i] = AR_PHI * prev + innov * sm[i]
            prev = e[i]
        t = np.arange(c0, c1, dtype=np.float64)
        season = SEASON_AMP_PA * np.sin(2.0 * math.pi * t / SEASON_PERIOD_DAYS)
        block = OFFSET_PA + season[:, None, None] + NOISE_STD_PA * e
        out[c0:c1] = block.reshape(c1 - c0, H * W).astype(np.float32)

    erng = np.random.default_rng(seed + 1)
    if event_starts is None:
        starts = _event_starts(T, n_events, event_len, erng)
    else:
        starts = [int(s) for s in event_starts]
    for s in starts:
        dip = _dipole(H, W, erng).reshape(-1)
        for d in range(event_len):
            if 0 <= s + d < T:
                row = out[s + d].astype(np.float64) + dip
                out[s + d] = row.astype(np.float32)
    return out, starts


def make_workload(w: Workload | str) -> tuple[np.ndarray, list[int]]:
    if isinstance(w, str):
        w = WORKLOADS[w]
    return make_fields(w.T, w.H, w.W, w.sigma, w.n_events, w.event_len, w.seed,
                       w.event_starts)


def pca_scores(X: np.ndarray, n_comp: int, rank: int = 100, power_iters: int = 2,
               seed: int = 0) -> tuple[np.ndarray, float]:
    """Scores of the n_comp leading principal components of the fields X
    [T, D] (rows centred per cell), by a randomized rank-``rank`` SVD with
    ``power_iters`` subspace iterations (Halko et al., the routine behind the
    paper's PCA). Returns float32 scores [T, n_comp], each component's sign
    fixed so that its largest-magnitude score is positive, and the fraction
    of the variance they explain."""
    Xc = np.asarray(X, dtype=np.float64)
    Xc = Xc - Xc.mean(axis=0)
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(Xc @ rng.standard_normal((Xc.shape[1], rank)))
    for _ in range(power_iters):
        Q, _ = np.linalg.qr(Xc.T @ Q)
        Q, _ = np.linalg.qr(Xc @ Q)
    Ub, sv, _ = np.linalg.svd(Q.T @ Xc, full_matrices=False)
    scores = (Q @ Ub[:, :n_comp]) * sv[:n_comp]
    pick = np.abs(scores).argmax(axis=0)
    scores *= np.sign(scores[pick, np.arange(n_comp)])
    frac = float((sv[:n_comp] ** 2).sum() / (Xc * Xc).sum())
    return np.ascontiguousarray(scores, dtype=np.float32), frac


def make_pca_workload(n_comp: int, base: Workload | str = "full"
                      ) -> tuple[np.ndarray, list[int], float]:
    """The base workload's fields reduced to n_comp principal component
    scores: (X [T, n_comp] float32, planted starts, explained variance)."""
    X, starts = make_workload(base)
    Z, frac = pca_scores(X, n_comp)
    return Z, starts, frac


def random_fields(T: int, D: int, seed: int, scale: float = 1.0,
                  offset: float = 0.0) -> np.ndarray:
    """Plain i.i.d. Gaussian [T, D] float32 fields for shape and edge-case tests."""
    rng = np.random.default_rng(seed)
    return (offset + scale * rng.standard_normal((T, D))).astype(np.float32)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
