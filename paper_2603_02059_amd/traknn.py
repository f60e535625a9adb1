"""Python binding of the TRAKNN C ABI (``include/traknn.h``).

The functions named ``traknn_*`` mirror the C entry points one to one and only
marshal arguments (device pointers from torch tensors, the current HIP stream);
every step of the computation runs in the library's HIP kernels. Convenience
wrappers (``Plan``, ``knn``, ``score``) allocate outputs and the workspace with
torch on the device, and ``TraknnScore`` exposes the score and its
hand-written backward as a ``torch.autograd.Function``.

There is no fallback: if ``libtraknn.so`` has not been built, importing this
module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtraknn.so")

TRAKNN_OK = 0
TRAKNN_ERR_INVALID_ARG = -1
TRAKNN_ERR_UNSUPPORTED = -2
TRAKNN_ERR_WORKSPACE = -3
TRAKNN_ERR_HIP = -4
TRAKNN_ERR_SCRATCH_LIMIT = -5
NOALLOC_MAX_BYTES = 32 << 20

TRAKNN_FP32 = 0
TRAKNN_BF16X3 = 1
TRAKNN_FP16 = 2
TRAKNN_FP64 = 3
PRECISIONS = {"fp32": TRAKNN_FP32, "bf16x3": TRAKNN_BF16X3, "fp16": TRAKNN_FP16,
              "fp64": TRAKNN_FP64}
TRAKNN_MODE_MATRIX = 0
TRAKNN_MODE_FUSED = 1
MODES = {"matrix": TRAKNN_MODE_MATRIX, "fused": TRAKNN_MODE_FUSED}
MAX_L = 16
MAX_K = 64
STAGES = ("centre_stats", "centre_convert", "gram", "window_topk", "merge")

EXPORTS = ("traknn_plan", "traknn_plan_destroy", "traknn_knn", "traknn_knn_noalloc",
           "traknn_score",
           "traknn_score_prefix", "traknn_local_dim", "traknn_score_backward",
           "traknn_backward_workspace", "traknn_status_string", "traknn_set_timing",
           "traknn_stage_times", "traknn_band_passes")


class TraknnError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} ({code})")


class traknn_config(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int64), ("D", ctypes.c_int64),
                ("L_min", ctypes.c_int32), ("L_max", ctypes.c_int32),
                ("k", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("row_batch", ctypes.c_int64), ("mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it first (python -m "
            "paper_2603_02059_amd.build or __graft_entry__.build()). There is no "
            "CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    lib.traknn_plan.argtypes = [ctypes.POINTER(traknn_config), ctypes.POINTER(vp),
                                ctypes.POINTER(sz)]
    lib.traknn_plan_destroy.argtypes = [vp]
    lib.traknn_knn.argtypes = [vp, vp, i64, vp, sz, vp, vp, vp]
    lib.traknn_knn_noalloc.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.traknn_score.argtypes = [vp, vp, vp, vp]
    lib.traknn_score_prefix.argtypes = [vp, vp, vp, vp]
    lib.traknn_local_dim.argtypes = [vp, vp, vp, vp]
    lib.traknn_score_backward.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp, sz, vp]
    lib.traknn_backward_workspace.argtypes = [vp, ctypes.POINTER(sz)]
    lib.traknn_band_passes.argtypes = [vp, ctypes.POINTER(i64), i64, ctypes.POINTER(i64)]
    lib.traknn_status_string.argtypes = [i32]
    lib.traknn_status_string.restype = ctypes.c_char_p
    lib.traknn_set_timing.argtypes = [vp, i32]
    lib.traknn_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32,
                                       ctypes.POINTER(i32)]
    for name in EXPORTS:
        if name != "traknn_status_string":
            getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()


def status_string(code: int) -> str:
    return _lib.traknn_status_string(int(code)).decode()


def _ck(rc: int, what: str) -> None:
    if rc != TRAKNN_OK:
        raise TraknnError(rc, what)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


# --------------------------------------------------------------------------
# One-to-one wrappers of the C entry points
# --------------------------------------------------------------------------
def traknn_plan(T: int, D: int, L_min: int, L_max: int, k: int,
                precision: int | str = TRAKNN_BF16X3, row_batch: int = 0,
                mode: int | str = TRAKNN_MODE_MATRIX):
    """-> (plan handle, workspace bytes). Pure host call; raises TraknnError."""
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    if isinstance(mode, str):
        mode = MODES[mode]
    cfg = traknn_config(int(T), int(D), int(L_min), int(L_max), int(k),
                        int(precision), int(row_batch), int(mode), 0)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    _ck(_lib.traknn_plan(ctypes.byref(cfg), ctypes.byref(h), ctypes.byref(ws)),
        "traknn_plan")
    return h.value, ws.value


def traknn_plan_destroy(plan) -> None:
    _ck(_lib.traknn_plan_destroy(plan), "traknn_plan_destroy")


def workspace_bytes(T: int, D: int, L_min: int, L_max: int, k: int,
                    precision: int | str = TRAKNN_BF16X3, row_batch: int = 0,
                    mode: int | str = TRAKNN_MODE_MATRIX) -> int:
    """Workspace of a plan, from the planner alone (no GPU involved)."""
    h, ws = traknn_plan(T, D, L_min, L_max, k, precision, row_batch, mode)
    traknn_plan_destroy(h)
    return ws


def row_batch_for(T: int, D: int, L_min: int, L_max: int, k: int,
                  precision: int | str = TRAKNN_BF16X3, *, max_bytes: int) -> int:
    """A row_batch whose workspace fits in max_bytes: 0 (the whole matrix, the
    faster mode) when that fits, else the largest multiple of 8 a bisection
    finds. Band mode's workspace grows with row_batch (both stored copies of
    the band do), up to a wobble of the window's partial lists of a few MB.
    Raises ValueError if even passes of 8 rows do not fit."""
    if workspace_bytes(T, D, L_min, L_max, k, precision, 0) <= max_bytes:
        return 0
    if workspace_bytes(T, D, L_min, L_max, k, precision, 8) > max_bytes:
        raise ValueError(f"no row_batch fits a workspace of {max_bytes} bytes")
    lo, hi = 1, (T - L_min + 1 + 7) // 8  # in units of 8 rows; lo fits
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if workspace_bytes(T, D, L_min, L_max, k, precision, 8 * mid) <= max_bytes:
            lo = mid
        else:
            hi = mid - 1
    return 8 * lo


def traknn_knn(plan, X, ldx: int, ws, ws_bytes: int, nbr_idx, nbr_dist,
               stream=None) -> None:
    _ck(_lib.traknn_knn(plan, _ptr(X), int(ldx), _ptr(ws), int(ws_bytes),
                        _ptr(nbr_idx), _ptr(nbr_dist), _stream(stream)), "traknn_knn")


def traknn_knn_noalloc(plan, X, ldx: int, nbr_idx, nbr_dist, stream=None) -> None:
    _ck(_lib.traknn_knn_noalloc(plan, _ptr(X), int(ldx), _ptr(nbr_idx), _ptr(nbr_dist),
                                _stream(stream)), "traknn_knn_noalloc")


def traknn_score(plan, nbr_dist, scores, stream=None) -> None:
    _ck(_lib.traknn_score(plan, _ptr(nbr_dist), _ptr(scores), _stream(stream)),
        "traknn_score")


def traknn_score_prefix(plan, nbr_dist, scores, stream=None) -> None:
    _ck(_lib.traknn_score_prefix(plan, _ptr(nbr_dist), _ptr(scores), _stream(stream)),
        "traknn_score_prefix")


def traknn_local_dim(plan, nbr_dist, out, stream=None) -> None:
    _ck(_lib.traknn_local_dim(plan, _ptr(nbr_dist), _ptr(out), _stream(stream)),
        "traknn_local_dim")


def traknn_score_backward(plan, X, ldx: int, nbr_idx, grad_scores, grad_X,
                          ldg: int, ws, ws_bytes: int, stream=None) -> None:
    _ck(_lib.traknn_score_backward(plan, _ptr(X), int(ldx), _ptr(nbr_idx),
                                   _ptr(grad_scores), _ptr(grad_X), int(ldg),
                                   _ptr(ws), int(ws_bytes), _stream(stream)),
        "traknn_score_backward")


def traknn_backward_workspace(plan) -> int:
    """Bytes of workspace traknn_score_backward needs (a prefix of the plan's)."""
    b = ctypes.c_size_t()
    _ck(_lib.traknn_backward_workspace(plan, ctypes.byref(b)), "traknn_backward_workspace")
    return b.value


def traknn_band_passes(plan) -> list:
    """Band mode's pass starts as the plan placed them ([] outside band mode)."""
    n = ctypes.c_int64()
    _ck(_lib.traknn_band_passes(plan, None, 0, ctypes.byref(n)), "traknn_band_passes")
    buf = (ctypes.c_int64 * max(n.value, 1))()
    _ck(_lib.traknn_band_passes(plan, buf, n.value, ctypes.byref(n)), "traknn_band_passes")
    return list(buf[:n.value])


def traknn_status_string(code: int) -> str:
    return status_string(code)


def traknn_set_timing(plan, enable: bool) -> None:
    _ck(_lib.traknn_set_timing(plan, 1 if enable else 0), "traknn_set_timing")


def traknn_stage_times(plan) -> list[float]:
    ms = (ctypes.c_double * len(STAGES))()
    n = ctypes.c_int()
    _ck(_lib.traknn_stage_times(plan, ms, len(STAGES), ctypes.byref(n)),
        "traknn_stage_times")
    return [ms[i] for i in range(n.value)]


# --------------------------------------------------------------------------
# Convenience layer (torch allocates device memory; the library computes)
# --------------------------------------------------------------------------
def _as_fields(X: torch.Tensor) -> torch.Tensor:
    if X.dim() > 2:
        X = X.reshape(X.shape[0], -1)
    if X.dim() != 2 or X.dtype != torch.float32 or not X.is_cuda:
        raise ValueError("X must be a float32 CUDA tensor of shape [T, D] or [T, H, W]")
    if X.stride(1) != 1 or X.stride(0) % 4 != 0 or X.data_ptr() % 16 != 0:
        X = X.contiguous()
        if X.shape[1] % 4 != 0:
            pad = torch.zeros(X.shape[0], (X.shape[1] + 3) // 4 * 4, device=X.device,
                              dtype=X.dtype)
            pad[:, :X.shape[1]] = X
            X = pad[:, :X.shape[1]]
    return X


class Plan:
    """A TRAKNN plan plus its device workspace, reusable across calls."""

    def __init__(self, T: int, D: int, L_min: int, L_max: int | None = None,
                 k: int = 10, precision: str | int = "bf16x3", device=None,
                 row_batch: int = 0, mode: str | int = "matrix"):
        """row_batch > 0 (a multiple of 8) streams the distance matrix in bands
        of row_batch trajectory rows instead of holding all T x T of it;
        mode="fused" never stores it (single length)."""
        L_max = L_min if L_max is None else L_max
        self.T, self.D, self.L_min, self.L_max, self.k = T, D, L_min, L_max, k
        self.row_batch = row_batch
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else precision
        self.mode = MODES[mode] if isinstance(mode, str) else mode
        self.handle, self.ws_bytes = traknn_plan(T, D, L_min, L_max, k, self.precision,
                                                 row_batch, self.mode)
        self.bw_bytes = traknn_backward_workspace(self.handle)
        self.device = torch.device(device if device is not None else "cuda")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.NL = L_max - L_min + 1
        self.np0 = T - L_min + 1

    def close(self):
        if self.handle:
            traknn_plan_destroy(self.handle)
            self.handle = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_outputs(self):
        idx = torch.empty((self.NL, self.np0, self.k), dtype=torch.int32, device=self.device)
        dist = torch.empty((self.NL, self.np0, self.k), dtype=torch.float64, device=self.device)
        return idx, dist

    def knn(self, X: torch.Tensor, idx=None, dist=None, stream=None):
        X = _as_fields(X)
        if X.shape != (self.T, self.D):
            raise ValueError(f"X has shape {tuple(X.shape)}, plan expects {(self.T, self.D)}")
        if idx is None:
            idx, dist = self.empty_outputs()
        traknn_knn(self.handle, X, X.stride(0), self.ws, self.ws_bytes, idx, dist, stream)
        return idx, dist

    def score(self, dist: torch.Tensor, scores=None, stream=None):
        if scores is None:
            scores = torch.empty((self.NL, self.np0), dtype=torch.float64, device=self.device)
        traknn_score(self.handle, dist, scores, stream)
        return scores

    def score_prefix(self, dist: torch.Tensor, scores=None, stream=None):
        """Scores for every k' = 1..k: [NL, n', k] float64 (last column = score)."""
        if scores is None:
            scores = torch.empty((self.NL, self.np0, self.k), dtype=torch.float64,
                                 device=self.device)
        traknn_score_prefix(self.handle, dist, scores, stream)
        return scores

    def local_dim(self, dist: torch.Tensor, out=None, stream=None):
        """Local intrinsic dimension (Levina-Bickel MLE) of every trajectory for
        every k' = 1..k: [NL, n', k] float64 (column 0 is NaN)."""
        if out is None:
            out = torch.empty((self.NL, self.np0, self.k), dtype=torch.float64,
                              device=self.device)
        traknn_local_dim(self.handle, dist, out, stream)
        return out

    def band_passes(self):
        """Band mode's pass starts as the plan placed them ([] outside band mode)."""
        return traknn_band_passes(self.handle)

    def release_workspace(self):
        """Free the forward workspace; backward then allocates only the small
        prefix it needs."""
        self.ws = None

    def backward(self, X: torch.Tensor, idx: torch.Tensor, grad_scores: torch.Tensor,
                 grad_X=None, stream=None):
        X = _as_fields(X)
        if grad_X is None:
            grad_X = torch.empty((self.T, self.D), dtype=torch.float32, device=self.device)
        gs = grad_scores.reshape(-1).to(torch.float64).contiguous()
        idx = idx.reshape(-1, self.k).contiguous()
        if self.ws is not None:
            ws, nbytes = self.ws, self.ws_bytes
        else:
            ws = torch.empty(self.bw_bytes, dtype=torch.uint8, device=self.device)
            nbytes = self.bw_bytes
        traknn_score_backward(self.handle, X, X.stride(0), idx, gs, grad_X,
                              grad_X.stride(0), ws, nbytes, stream)
        return grad_X

    def set_timing(self, enable: bool = True):
        traknn_set_timing(self.handle, enable)

    def stage_times(self) -> dict:
        return dict(zip(STAGES, traknn_stage_times(self.handle)))


def knn(X: torch.Tensor, L: int, k: int, precision: str = "bf16x3",
        L_max: int | None = None, row_batch: int = 0, mode: str = "matrix"):
    """Neighbour lists (idx [NL, n', k] int32, dist [NL, n', k] float64)."""
    X = _as_fields(X)
    p = Plan(X.shape[0], X.shape[1], L, L_max, k, precision, device=X.device,
             row_batch=row_batch, mode=mode)
    try:
        return p.knn(X)
    finally:
        p.close()


class TraknnScore(torch.autograd.Function):
    """s = rarity scores (Eq. 3) of every length-L trajectory of X; backward
    gives dF/dX with the neighbour sets held fixed.

    Between forward and backward only the plan handle, X and the neighbour
    lists are kept: the forward workspace (the distance matrix) is freed as
    soon as the scores exist, and backward allocates just the reverse-list
    scratch it needs. The plan is released with the graph, so a backward
    with retain_graph=True can run again."""

    @staticmethod
    def forward(ctx, X: torch.Tensor, L: int, k: int, precision: str = "bf16x3"):
        Xf = _as_fields(X.detach())
        p = Plan(Xf.shape[0], Xf.shape[1], L, L, k, precision, device=Xf.device)
        idx, dist = p.knn(Xf)
        s = p.score(dist)[0]
        p.release_workspace()
        idx0 = idx[0]
        ctx.plan = p
        ctx.shape = X.shape
        ctx.save_for_backward(Xf, idx0)
        ctx.mark_non_differentiable(idx0)
        return s, idx0

    @staticmethod
    def backward(ctx, grad_s, grad_idx):
        Xf, idx0 = ctx.saved_tensors
        g = ctx.plan.backward(Xf, idx0, grad_s.to(torch.float64))
        return g.reshape(ctx.shape), None, None, None


def score(X: torch.Tensor, L: int, k: int, precision: str = "bf16x3"):
    """Rarity scores s [n'] (float64) with autograd support; also returns the
    neighbour lists [n', k]."""
    return TraknnScore.apply(X, L, k, precision)
