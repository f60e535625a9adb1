"""traknn_knn_noalloc, the entry point for callers that cannot allocate: its
scratch is the library's fixed per-device array, so the caller passes only
inputs and outputs. Called through the C ABI and compared with traknn_knn,
the workspace entry point running the same kernels, on two calls in a row,
the second with a smaller input; and against the oracle's parity rule."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2603_02059_amd import synth
from paper_2603_02059_amd import traknn as tk
from tests.parity import check_rows, precision_tol


def test_noalloc_rejects_plans_beyond_its_scratch():
    """A plan whose workspace exceeds the fixed scratch is refused with its
    own status code before anything touches the device (host-side check)."""
    h, ws = tk.traknn_plan(27394, 8192, 5, 5, 10, "bf16x3")
    try:
        assert ws > tk.NOALLOC_MAX_BYTES
        fake = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced
        rc = tk._lib.traknn_knn_noalloc(h, fake, 8192, fake, fake, None)
        assert rc == tk.TRAKNN_ERR_SCRATCH_LIMIT
        assert "noalloc" in tk.status_string(rc)
    finally:
        tk.traknn_plan_destroy(h)


def _both(Xn, L, k, prec, mode="matrix"):
    """(workspace entry point outputs, allocation-free entry point outputs)."""
    import torch
    T, D = Xn.shape
    X = torch.from_numpy(np.ascontiguousarray(Xn)).cuda()
    p = tk.Plan(T, D, L, L, k, prec, mode=mode)
    assert p.ws_bytes <= tk.NOALLOC_MAX_BYTES
    i1, d1 = p.empty_outputs()
    i2, d2 = p.empty_outputs()
    i2.fill_(-7)
    d2.fill_(1.5)
    tk.traknn_knn(p.handle, X, X.stride(0), p.ws, p.ws_bytes, i1, d1)
    tk.traknn_knn_noalloc(p.handle, X, X.stride(0), i2, d2)
    s2 = p.score(d2)
    torch.cuda.synchronize()
    out = (i1.cpu().numpy(), d1.cpu().numpy(), i2.cpu().numpy(), d2.cpu().numpy(),
           s2.cpu().numpy())
    p.close()
    return out


@pytest.mark.gpu
def test_noalloc_matches_knn_twice_then_smaller():
    print("[gpu] noalloc: tiny workload, then a smaller series", flush=True)
    w = synth.WORKLOADS["tiny"]
    Xa, _ = synth.make_workload(w)
    Xb, _ = synth.make_fields(300, 10, 20, sigma=2.0, n_events=2, event_len=4, seed=17)
    for Xn, L, k, prec in ((Xa, w.L, w.k, "bf16x3"), (Xb, 4, 6, "fp32")):
        print(f"  T={Xn.shape[0]} D={Xn.shape[1]} L={L} k={k} {prec}", flush=True)
        i1, d1, i2, d2, s2 = _both(Xn, L, k, prec)
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2)
        n = Xn.shape[0] - L + 1
        ref = oracle.knn(Xn, L, k)
        Dm = oracle.traj_dist(Xn, L)
        check_rows(Xn, L, k, np.arange(n), i2[0], d2[0], s2[0], precision_tol(prec),
                   ref=(ref[0], ref[1], ref[2], ref[3], Dm), label="noalloc")


@pytest.mark.gpu
def test_noalloc_fused_matches_knn():
    """The fused mode through the allocation-free entry point: its slots,
    bounds and running lists live in the fixed scratch, which keeps the
    previous call's contents, so every slot must be written before it is
    read. A larger series, then a smaller one, in FP64 and BF16x3."""
    print("[gpu] noalloc: fused mode", flush=True)
    Xa, _ = synth.make_fields(1400, 4, 8, sigma=1.0, n_events=3, event_len=5, seed=23)
    Xb, _ = synth.make_fields(700, 4, 8, sigma=1.0, n_events=2, event_len=5, seed=29)
    for Xn, prec in ((Xa, "fp64"), (Xb, "fp64"), (Xa, "bf16x3"), (Xb, "bf16x3")):
        L, k = 5, 8
        print(f"  T={Xn.shape[0]} D={Xn.shape[1]} L={L} k={k} {prec} fused", flush=True)
        i1, d1, i2, d2, s2 = _both(Xn, L, k, prec, mode="fused")
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2)
        if prec == "fp64":
            n = Xn.shape[0] - L + 1
            ref = oracle.knn(Xn, L, k)
            Dm = oracle.traj_dist(Xn, L)
            check_rows(Xn, L, k, np.arange(n), i2[0], d2[0], s2[0], 1e-5,
                       ref=(ref[0], ref[1], ref[2], ref[3], Dm), label="noalloc fused")
