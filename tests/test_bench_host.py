"""Host-side checks of bench.py (no GPU): the multi-GPU refusal, the
algorithmic work figures its roofline uses, and that every shape it times is
accepted by the planner."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2603_02059_amd import traknn as tk  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_gram_flops():
    # upper triangle with the diagonal: T(T+1)/2 pairs, 2D flop each, x3 for BF16x3
    assert bench.gram_flops(4, 10, "fp32") == 2 * 10 * 10
    assert bench.gram_flops(4, 10, "bf16x3") == 3 * 2 * 10 * 10
    T, D = 27394, 8192
    assert bench.gram_flops(T, D, "bf16x3") == pytest.approx(1.8443e13, rel=1e-4)


def test_window_bytes():
    wb = bench.window_bytes(100, 5, rows=8)
    assert wb["algorithmic_bytes"] == 4.0 * 100 * 101 / 2
    assert wb["design_bytes"] == 4.0 * 100 * 100 * 12 / 8


@pytest.mark.parametrize("Dpad", [8192, 32])
@pytest.mark.parametrize("T,L,rb", [(700, 4, 248), (700, 4, 8), (520, 16, 504), (1000, 2, 512),
                                    (27394, 5, 4088)])
def test_band_tiles(T, L, rb, Dpad):
    # the planned passes: contiguous, starting on multiples of 8, at most rb
    # rows each, covering the n trajectories
    n, nb = T - L + 1, -(-T // 256)
    passes = bench.band_passes(T, L, L, rb, Dpad)
    assert passes[0][0] == 0 and sum(nt for _, nt in passes) == n
    for (t0, nt), (t1, _) in zip(passes, passes[1:] + [(n, 0)]):
        assert t0 % 8 == 0 and 0 < nt <= rb and t0 + nt == t1
    # brute force: pass t0 holds rows t0 .. t0 + srows - 1 in 256-row block-rows
    # aligned to t0 and 256-column blocks aligned to 0; it contracts the tiles
    # with an entry above the diagonal, and together the passes hold every
    # entry (r, c), c > r, that a trajectory window reads
    tiles, rounds, covered = 0, 0, np.zeros(T, bool)
    for t0, nt in passes:
        srows = min(nt + L - 1, T - t0)
        nbi = -(-srows // 256)
        ptiles = 0
        for I in range(nbi):
            r_lo = t0 + 256 * I
            for J in range(nb):
                if 256 * J + 255 > r_lo:  # some column above the tile's first row
                    ptiles += 1
        tiles += ptiles
        rounds += -(-ptiles // 256)
        if T <= 1000:
            r = np.arange(t0, t0 + srows)[:, None]
            c = np.arange(T)[None, :]
            I, J = (r - t0) // 256, c // 256
            # every entry above the diagonal in the pass's rows is in a
            # contracted tile
            assert np.all((J >= t0 // 256 + I) | (c <= r))
            covered[t0:t0 + srows] = True
    assert bench.band_tiles(T, L, L, rb, Dpad) == tiles
    assert T > 1000 or covered.all()
    # the plan costs no more than passes of exactly rb rows (rounds of 256
    # tiles plus 1 + 8192 / Dpad rounds per pass), which it also considers
    lam = 1.0 + 8192.0 / Dpad
    fixed = [(t0, min(rb, n - t0)) for t0 in range(0, n, rb)]
    fixed_cost = sum(-(-bench._pass_tiles(T, L, t0, nt) // 256) + lam for t0, nt in fixed)
    assert rounds + lam * len(passes) <= fixed_cost + 1e-9
    if (T, L, rb, Dpad) == (27394, 5, 4088, 8192):
        assert (len(passes), rounds) == (7, 26)  # fixed passes: 7 and 28


@pytest.mark.parametrize("T,D,L,k,prec,rb", [
    (27394, 8192, 5, 10, "bf16x3", 0), (27394, 8192, 5, 10, "fp32", 0),
    (27394, 8192, 5, 10, "fp16", 0), (27394, 8192, 5, 10, "bf16x3", 4088),
    (10957, 8192, 5, 10, "fp32", 0),
    (27000, 50400, 1, 1, "bf16x3", 0), (27000, 2025, 1, 1, "bf16x3", 0),
    (40000, 50400, 1, 1, "bf16x3", 0), (27000, 50400, 15, 1, "bf16x3", 0),
    (27000, 50400, 1, 50, "bf16x3", 0), (27000, 50625, 1, 1, "bf16x3", 0),
    (27394, 50861, 5, 10, "bf16x3", 0), (27394, 50861, 5, 10, "fp32", 0),
    (27394, 32, 5, 40, "bf16x3", 0),
])
def test_timed_shapes_plan(T, D, L, k, prec, rb):
    h, ws = tk.traknn_plan(T, D, L, L, k, prec, rb)
    tk.traknn_plan_destroy(h)
    # every timed shape fits one MI355X (288 GiB)
    assert ws < 288 * 2 ** 30
