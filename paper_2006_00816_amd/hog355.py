"""Python binding of libhog355 (ctypes).

Argument marshalling only: every step of the detector runs in the HIP
kernels of libhog355.so.  PyTorch provides device memory and the stream
(the current torch stream).  There is no fallback: if the library is not
built, or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhog355.so")

HOG_OK = 0
MAX_DETS = 4096
STATIC_SCRATCH_BYTES = 64 << 20
HOG_E_SCRATCH = -8


class HogError(RuntimeError):
    pass


class hog_params(ctypes.Structure):
    _fields_ = [("upsample", ctypes.c_int32), ("thresh", ctypes.c_float), ("iou", ctypes.c_float),
                ("min_face", ctypes.c_int32), ("regions", ctypes.c_void_p), ("score_arith", ctypes.c_int32)]


ARITH_F32 = 0     # HOG_ARITH_F32: FP32 products (the default)
ARITH_F16X3 = 1   # HOG_ARITH_F16X3: each product from three fp16 products of split operands


ALL_LEVELS = 1 << 30
CASCADE = 0x100   # recursive pyramid, or-ed into upsample


def region_windows(h: int, w: int, upsample: int, level: int, region):
    """(r_lo, r_hi, c_lo, c_hi): the anchors of `level` whose windows a
    search region (x0, y0, x1, y1, k_lo, k_hi) lets through, as the kernels
    compute them (host)."""
    reg = (ctypes.c_int32 * 6)(*[int(v) for v in region])
    out = (ctypes.c_int32 * 4)()
    _check(lib().hog_region_windows(h, w, upsample, level, reg, out), "hog_region_windows")
    return tuple(out)


def region_tensor(regions, device="cuda"):
    """Search regions as the int32 [n][6] device tensor the library reads:
    rows (x0, y0, x1, y1, k_lo, k_hi) in frame pixels (half-open) and
    pyramid levels (inclusive)."""
    t = torch.as_tensor(regions, dtype=torch.int32).reshape(-1, 6)
    return t.to(device).contiguous()


class hog_tuning(ctypes.Structure):
    _fields_ = [("fused", ctypes.c_int32), ("queues", ctypes.c_int32), ("wg_per_queue", ctypes.c_int32),
                ("lag_f", ctypes.c_int32), ("lag_s", ctypes.c_int32), ("split", ctypes.c_int32),
                ("nms_rounds", ctypes.c_int32), ("score_rows", ctypes.c_int32), ("stagger", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class hog_constants(ctypes.Structure):
    _fields_ = [("cell_px", ctypes.c_int32), ("bins", ctypes.c_int32), ("features", ctypes.c_int32),
                ("window_cells", ctypes.c_int32), ("min_side", ctypes.c_int32), ("scale_num", ctypes.c_int32),
                ("scale_den", ctypes.c_int32), ("clip", ctypes.c_float), ("eps", ctypes.c_float)]


class hog_filterbank(ctypes.Structure):
    _fields_ = [("nf", ctypes.c_int32), ("rank", ctypes.c_int32), ("W", ctypes.c_void_p), ("row", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("bias", ctypes.c_void_p)]


class FilterBank:
    """nf linear filters with biases, on the device: full filters W
    [nf][10][10][31] (rank 0), or separable row / column factors
    [nf][rank][10][31] with W[f][dr][dc][ch] = sum_i col[f][i][dr][ch] *
    row[f][i][dc][ch] (rank 1..4)."""

    def __init__(self, bias: torch.Tensor, W: torch.Tensor = None, row: torch.Tensor = None,
                 col: torch.Tensor = None):
        self.bias = bias
        self.W, self.row, self.col = W, row, col
        if W is not None:
            self.nf, self.rank = int(W.shape[0]), 0
        else:
            if row is None or col is None or tuple(row.shape) != tuple(col.shape) or row.dim() != 4:
                raise HogError("separable filters need row and col factors of shape [nf][rank][10][31]")
            self.nf, self.rank = int(row.shape[0]), int(row.shape[1])
        self.struct = hog_filterbank(self.nf, self.rank, _ptr(W) if W is not None else None,
                                     _ptr(row) if row is not None else None, _ptr(col) if col is not None else None,
                                     _ptr(bias))


class hog_level(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("cy", ctypes.c_int32), ("cx", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("cols", ctypes.c_int32), ("reserved", ctypes.c_int32), ("sig", ctypes.c_int64),
                ("feat_offset", ctypes.c_int64), ("score_offset", ctypes.c_int64)]


DET_DTYPE = np.dtype([("frame", "i4"), ("filter", "i4"), ("level", "i4"), ("row", "i4"), ("col", "i4"),
                      ("x0", "i4"), ("y0", "i4"), ("x1", "i4"), ("y1", "i4"), ("score", "f4")])

_lib = None


def lib():
    """The loaded library; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HogError(f"{LIB_PATH} is not built (python -m paper_2006_00816_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    f32 = ctypes.c_float
    sig = {
        "hog_version": ([], i32),
        "hog_init": ([], i32),
        "hog_params_default": ([vp], i32),
        "hog_constants_get": ([vp], i32),
        "hog_windows_check": ([i32, i32, i32, i32, i32, vp, i32, vp], i32),
        "hog_strerror": ([i32], ctypes.c_char_p),
        "hog_orientation_table": ([vp, vp], i32),
        "hog_pyramid": ([i32, i32, i32, i32, vp, i32, vp], i32),
        "hog_workspace_bytes": ([i32, i32, i32, i32, i32], sz),
        "hog_features": ([vp, i32, i32, i32, i32, vp, i64, vp, sz, vp], i32),
        "hog_scores": ([vp, i32, i32, i32, i32, vp, vp, i32, vp, i64, vp, sz, vp], i32),
        "hog_scores_bank": ([vp, i32, i32, i32, i32, vp, vp, i64, vp, sz, vp], i32),
        "hog_scores_arith": ([vp, i32, i32, i32, i32, vp, vp, i32, i32, vp, i64, vp, sz, vp], i32),
        "hog_detect_batch_bank": ([vp, vp, i32, i32, i32, i32, i64, vp, vp, i32, vp, vp, sz, vp], i32),
        "hog_graph_create_bank": ([vp, vp, vp, i32, i32, i32, i32, i64, vp, vp, i32, vp, vp, sz, vp], i32),
        "hog_detect": ([vp, vp, i32, i32, i32, vp, vp, i32, vp, i32, vp, vp, sz, vp], i32),
        "hog_detect_batch": ([vp, vp, i32, i32, i32, i32, i64, vp, vp, i32, vp, i32, vp, vp, sz, vp], i32),
        "hog_detect_batch_static": ([vp, vp, i32, i32, i32, i32, i64, vp, vp, i32, vp, i32, vp, vp], i32),
        "hog_track_regions": ([vp, vp, i32, i32, i32, i32, i32, i32, vp, vp], i32),
        "hog_region_windows": ([i32, i32, i32, i32, vp, vp], i32),
        "hog_detect_topk": ([vp, vp, i32, i32, i32, i32, i64, vp, vp, i32, vp, i32, vp, i32, vp, vp, vp, sz, vp],
                            i32),
        "hog_pipeline_create": ([vp, vp, vp, vp, vp, i32], i32),
        "hog_pipeline_submit": ([vp, vp, i32, i64], i32),
        "hog_pipeline_drain": ([vp], i32),
        "hog_pipeline_destroy": ([vp], i32),
        "hog_graph_create": ([vp, vp, vp, i32, i32, i32, i32, i64, vp, vp, i32, vp, i32, vp, vp, sz, vp], i32),
        "hog_graph_launch": ([vp, vp], i32),
        "hog_graph_destroy": ([vp], i32),
        "hog_level_maps": ([vp, i32, i32, i32, i32, i32, vp, vp, vp, vp, sz, vp], i32),
        "hog_orient_bins": ([vp, vp, i64, vp, vp], i32),
        "hog_grad_workspace_bytes": ([i32, i32, i32, i32, i32, i32], sz),
        "hog_window_scores": ([vp, i32, i32, i32, i32, i64, i32, vp, vp, i32, vp, i32, vp, vp, sz, vp], i32),
        "hog_topk_windows": ([vp, i32, i32, i32, i32, i64, i32, vp, vp, i32, i32, vp, vp, vp, sz, vp], i32),
        "hog_filter_backward": ([vp, i32, i32, i32, i32, i64, i32, vp, i32, vp, vp, i32, vp, vp, vp, vp, sz, vp],
                                i32),
        "hog_hinge_loss": ([vp, vp, i32, vp, i32, ctypes.c_float, vp, vp, vp, vp], i32),
        "hog_tuning_get": ([i32, i32, i32, i32, i32, vp], i32),
        "hog_tuning_set": ([i32, i32, i32, i32, i32, vp], i32),
        "hog_autotune": ([vp, vp, i32, i32, i32, i32, i64, vp, vp, i32, vp, i32, vp, vp, sz, i32, vp, vp, vp], i32),
        "hog_profile_enable": ([i32], i32),
        "hog_profile_reset": ([], i32),
        "hog_profile_read": ([ctypes.c_char_p, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _ = f32
    _lib = L
    return L


def _check(st: int, what: str):
    if st != HOG_OK:
        raise HogError(f"{what}: {lib().hog_strerror(st).decode()} ({st})")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise HogError("expected a device tensor")
    if not t.is_contiguous():
        raise HogError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _fptr(t: torch.Tensor):
    """Pointer to uint8 frames whose rows may be padded: unit stride along
    a row; the row pitch and the frame stride come from the tensor's
    strides (the library checks them)."""
    if not t.is_cuda:
        raise HogError("expected a device tensor")
    if t.dtype != torch.uint8 or t.stride(-1) != 1 or any(st < 0 for st in t.stride()):
        raise HogError("frames must be uint8 with unit stride along a row")
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------ host helpers
def params_default():
    p = hog_params()
    _check(lib().hog_params_default(ctypes.byref(p)), "hog_params_default")
    return {"upsample": int(p.upsample), "thresh": float(p.thresh), "iou": float(p.iou)}


def constants():
    c = hog_constants()
    _check(lib().hog_constants_get(ctypes.byref(c)), "hog_constants_get")
    return {k: getattr(c, k) for k, _ in hog_constants._fields_}


def orientation_table():
    c = (ctypes.c_double * 9)()
    s = (ctypes.c_double * 9)()
    _check(lib().hog_orientation_table(c, s), "hog_orientation_table")
    return np.array(c[:]), np.array(s[:])


def pyramid(h: int, w: int, upsample: int = 1, nf: int = 0):
    arr = (hog_level * 32)()
    n = ctypes.c_int(0)
    _check(lib().hog_pyramid(h, w, upsample, nf, arr, 32, ctypes.byref(n)), "hog_pyramid")
    return [{f: getattr(arr[i], f) for f, _ in hog_level._fields_} for i in range(n.value)]


def workspace_bytes(h: int, w: int, upsample: int = 1, n: int = 1, nf: int = 1) -> int:
    b = lib().hog_workspace_bytes(h, w, upsample, n, nf)
    if b == 0:
        raise HogError("hog_workspace_bytes: invalid arguments")
    return int(b)


class Workspace:
    """A device byte buffer that grows to the largest request seen."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = torch.empty(0, dtype=torch.uint8, device=device)

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws = {}


def _ws(ws, nbytes):
    if ws is None:
        dev = torch.cuda.current_device()
        ws = _default_ws.setdefault(dev, Workspace(f"cuda:{dev}"))
    b = ws.get(nbytes)
    return ctypes.c_void_p(b.data_ptr()), ctypes.c_size_t(b.numel())


def _frame_args(frame: torch.Tensor):
    if frame.dtype != torch.uint8 or frame.dim() != 2:
        raise HogError("frame must be a uint8 [h][w] device tensor")
    h, w = frame.shape
    return int(h), int(w), int(frame.stride(0))


# ---------------------------------------------------------------- calls
def features(frame: torch.Tensor, upsample: int = 1, ws=None):
    """31-d features per level: list of (level dict, float32 tensor [cy][cx][31])."""
    h, w, pitch = _frame_args(frame)
    levels = pyramid(h, w, upsample, 0)
    total = sum(l["cy"] * l["cx"] * 31 for l in levels)
    out = torch.empty(max(total, 1), dtype=torch.float32, device=frame.device)
    wp, wn = _ws(ws, workspace_bytes(h, w, upsample, 1, 0))
    _check(lib().hog_features(_fptr(frame), h, w, pitch, upsample, _ptr(out), out.numel(), wp, wn, _stream()),
           "hog_features")
    return [(l, out[l["feat_offset"]:l["feat_offset"] + l["cy"] * l["cx"] * 31].view(l["cy"], l["cx"], 31))
            for l in levels]


def scores(frame: torch.Tensor, W: torch.Tensor, b: torch.Tensor, upsample: int = 1, ws=None, arith=None):
    """Dense window scores per level: list of (level dict, tensor [nf][rows][cols]).
    arith (ARITH_*): through hog_scores_arith; None: hog_scores."""
    h, w, pitch = _frame_args(frame)
    nf = int(W.shape[0])
    levels = pyramid(h, w, upsample, nf)
    total = sum(nf * l["rows"] * l["cols"] for l in levels)
    out = torch.empty(max(total, 1), dtype=torch.float32, device=frame.device)
    wp, wn = _ws(ws, workspace_bytes(h, w, upsample, 1, nf))
    if arith is None:
        _check(lib().hog_scores(_fptr(frame), h, w, pitch, upsample, _ptr(W), _ptr(b), nf, _ptr(out), out.numel(),
                                wp, wn, _stream()), "hog_scores")
    else:
        _check(lib().hog_scores_arith(_fptr(frame), h, w, pitch, upsample, _ptr(W), _ptr(b), nf, int(arith),
                                      _ptr(out), out.numel(), wp, wn, _stream()), "hog_scores_arith")
    return [(l, out[l["score_offset"]:l["score_offset"] + nf * l["rows"] * l["cols"]]
             .view(nf, l["rows"], l["cols"])) for l in levels]


def scores_bank(frame: torch.Tensor, bank: FilterBank, upsample: int = 1, ws=None):
    """Dense window scores per level for a filter bank: list of (level dict,
    tensor [nf][rows][cols])."""
    h, w, pitch = _frame_args(frame)
    nf = bank.nf
    levels = pyramid(h, w, upsample, nf)
    total = sum(nf * l["rows"] * l["cols"] for l in levels)
    out = torch.empty(max(total, 1), dtype=torch.float32, device=frame.device)
    wp, wn = _ws(ws, workspace_bytes(h, w, upsample, 1, nf))
    _check(lib().hog_scores_bank(_fptr(frame), h, w, pitch, upsample, ctypes.byref(bank.struct), _ptr(out),
                                 out.numel(), wp, wn, _stream()), "hog_scores_bank")
    return [(l, out[l["score_offset"]:l["score_offset"] + nf * l["rows"] * l["cols"]]
             .view(nf, l["rows"], l["cols"])) for l in levels]


def detect_batch_bank_into(frames: torch.Tensor, bank: FilterBank, dets: torch.Tensor, n_dets: torch.Tensor,
                           thresh: float = 0.0, iou: float = 0.5, upsample: int = 1, ws=None):
    """Enqueue hog_detect_batch_bank into caller-provided outputs."""
    if frames.dtype != torch.uint8 or frames.dim() != 3:
        raise HogError("frames must be a uint8 [n][h][w] device tensor")
    n, h, w = (int(v) for v in frames.shape)
    prm = _params(thresh, iou, upsample)
    wp, wn = _ws(ws, workspace_bytes(h, w, upsample, n, bank.nf))
    _check(lib().hog_detect_batch_bank(ctypes.byref(prm), _fptr(frames), n, h, w, int(frames.stride(1)),
                                       int(frames.stride(0)), ctypes.byref(bank.struct), _ptr(dets),
                                       int(dets.shape[1]), _ptr(n_dets), wp, wn, _stream()), "hog_detect_batch_bank")


def detect_batch_bank(frames: torch.Tensor, bank: FilterBank, thresh=0.0, iou=0.5, upsample=1, cap=MAX_DETS,
                      ws=None):
    dets, nd = alloc_dets(int(frames.shape[0]), cap, frames.device)
    detect_batch_bank_into(frames, bank, dets, nd, thresh, iou, upsample, ws)
    return dets_to_numpy(dets, nd)


def _params(thresh, iou, upsample, min_face=0, regions=None, n=None, arith=ARITH_F32):
    """hog_params; `regions` is an int32 [n][6] device tensor (see
    region_tensor) or None; `arith` the scoring arithmetic (ARITH_*)."""
    rp = None
    if regions is not None:
        if regions.dtype != torch.int32 or regions.dim() != 2 or regions.shape[1] != 6:
            raise HogError("regions must be an int32 [n][6] device tensor")
        if n is not None and regions.shape[0] < n:
            raise HogError(f"{regions.shape[0]} regions for {n} frames")
        rp = _ptr(regions).value
    return hog_params(upsample, thresh, iou, int(min_face), rp, int(arith))


def detect_batch_into(frames: torch.Tensor, W: torch.Tensor, b: torch.Tensor, dets: torch.Tensor,
                      n_dets: torch.Tensor, thresh: float = 0.0, iou: float = 0.5, upsample: int = 1, ws=None,
                      min_face: int = 0, regions: torch.Tensor = None, arith: int = ARITH_F32):
    """Enqueue hog_detect_batch into caller-provided outputs: dets int32
    [n][cap][10] (hog_det records), n_dets int32 [n].  min_face skips the
    levels whose window spans fewer frame pixels; regions (int32 [n][6],
    device) restricts each frame's search; arith selects the scoring
    arithmetic (ARITH_F32, or ARITH_F16X3: split fp16 operands)."""
    if frames.dtype != torch.uint8 or frames.dim() != 3:
        raise HogError("frames must be a uint8 [n][h][w] device tensor")
    n, h, w = (int(v) for v in frames.shape)
    cap = int(dets.shape[1])
    nf = int(W.shape[0])
    prm = _params(thresh, iou, upsample, min_face, regions, n, arith)
    wp, wn = _ws(ws, workspace_bytes(h, w, upsample, n, nf))
    _check(lib().hog_detect_batch(ctypes.byref(prm), _fptr(frames), n, h, w, int(frames.stride(1)),
                                  int(frames.stride(0)), _ptr(W), _ptr(b), nf, _ptr(dets), cap, _ptr(n_dets),
                                  wp, wn, _stream()), "hog_detect_batch")


def detect_batch_static_into(frames: torch.Tensor, W: torch.Tensor, b: torch.Tensor, dets: torch.Tensor,
                             n_dets: torch.Tensor, thresh: float = 0.0, iou: float = 0.5, upsample: int = 1):
    """Enqueue hog_detect_batch_static (the library's fixed scratch array as
    workspace, no allocation) into caller-provided outputs, as
    detect_batch_into."""
    if frames.dtype != torch.uint8 or frames.dim() != 3:
        raise HogError("frames must be a uint8 [n][h][w] device tensor")
    n, h, w = (int(v) for v in frames.shape)
    prm = _params(thresh, iou, upsample)
    _check(lib().hog_detect_batch_static(ctypes.byref(prm), _fptr(frames), n, h, w, int(frames.stride(1)),
                                         int(frames.stride(0)), _ptr(W), _ptr(b), int(W.shape[0]), _ptr(dets),
                                         int(dets.shape[1]), _ptr(n_dets), _stream()), "hog_detect_batch_static")


def alloc_dets(n: int, cap: int, device="cuda"):
    return (torch.empty((n, cap, 10), dtype=torch.int32, device=device),
            torch.empty(n, dtype=torch.int32, device=device))


def dets_to_numpy(dets: torch.Tensor, n_dets: torch.Tensor):
    """Per frame, a structured numpy array of the written detections."""
    d = dets.cpu().numpy()
    nd = n_dets.cpu().numpy()
    out = []
    for i in range(d.shape[0]):
        m = min(int(nd[i]), d.shape[1])
        out.append(np.ascontiguousarray(d[i, :m]).view(DET_DTYPE).reshape(m))
    return out, nd


def detect(frame: torch.Tensor, W, b, thresh=0.0, iou=0.5, upsample=1, cap=MAX_DETS, ws=None):
    """One frame through hog_detect: (detections, true kept count)."""
    h, w, pitch = _frame_args(frame)
    nf = int(W.shape[0])
    dets, nd = alloc_dets(1, cap, frame.device)
    prm = _params(thresh, iou, upsample)
    wp, wn = _ws(ws, workspace_bytes(h, w, upsample, 1, nf))
    _check(lib().hog_detect(ctypes.byref(prm), _fptr(frame), h, w, pitch, _ptr(W), _ptr(b), nf, _ptr(dets), cap,
                            _ptr(nd), wp, wn, _stream()), "hog_detect")
    out, cnt = dets_to_numpy(dets, nd)
    return out[0], int(cnt[0])


def detect_batch(frames: torch.Tensor, W, b, thresh=0.0, iou=0.5, upsample=1, cap=MAX_DETS, ws=None, min_face=0,
                 regions=None, arith=ARITH_F32):
    dets, nd = alloc_dets(int(frames.shape[0]), cap, frames.device)
    detect_batch_into(frames, W, b, dets, nd, thresh, iou, upsample, ws, min_face, regions, arith)
    return dets_to_numpy(dets, nd)


def track_regions(dets: torch.Tensor, n_dets: torch.Tensor, h: int, w: int, margin: int, span: int,
                  regions: torch.Tensor):
    """Enqueue hog_track_regions: the next frames' search regions (int32
    [n][6], written in place) from the detections of these frames."""
    n, cap = int(dets.shape[0]), int(dets.shape[1])
    if regions.dtype != torch.int32 or tuple(regions.shape) != (n, 6):
        raise HogError("regions must be an int32 [n][6] device tensor")
    _check(lib().hog_track_regions(_ptr(dets), _ptr(n_dets), n, cap, h, w, margin, span, _ptr(regions), _stream()),
           "hog_track_regions")


def tuning_get(h: int, w: int, upsample: int, n: int, nf: int):
    """(schedule dict, True if set for this shape / False for the default)."""
    t = hog_tuning()
    st = lib().hog_tuning_get(h, w, upsample, n, nf, ctypes.byref(t))
    if st < 0:
        _check(st, "hog_tuning_get")
    return t.as_dict(), st == 1


def tuning_set(h: int, w: int, upsample: int, n: int, nf: int, t: dict | None):
    """Set (dict) or clear (None) the schedule of a shape."""
    if t is None:
        _check(lib().hog_tuning_set(h, w, upsample, n, nf, None), "hog_tuning_set")
        return
    tt = hog_tuning(**{"split": 1, "nms_rounds": 3, "score_rows": 0, "stagger": 0,
                       **{k: int(v) for k, v in t.items()}})
    _check(lib().hog_tuning_set(h, w, upsample, n, nf, ctypes.byref(tt)), "hog_tuning_set")


def autotune(frames: torch.Tensor, W, b, cap=MAX_DETS, thresh=0.0, iou=0.5, upsample=1, reps: int = 5, ws=None):
    """Time hog_detect_batch under each candidate schedule on these frames;
    the fastest is kept for the shape.  Returns (schedule dict, ms per call)."""
    n, h, w = (int(v) for v in frames.shape)
    nf = int(W.shape[0])
    dets, nd = alloc_dets(n, cap, frames.device)
    prm = _params(thresh, iou, upsample)
    wp, wn = _ws(ws, workspace_bytes(h, w, upsample, n, nf))
    best = hog_tuning()
    ms = ctypes.c_float()
    _check(lib().hog_autotune(ctypes.byref(prm), _fptr(frames), n, h, w, int(frames.stride(1)), int(frames.stride(0)),
                              _ptr(W), _ptr(b), nf, _ptr(dets), cap, _ptr(nd), wp, wn, reps, ctypes.byref(best),
                              ctypes.byref(ms), _stream()), "hog_autotune")
    return best.as_dict(), float(ms.value)


class BoundGraph:
    """hog_detect_batch over caller-owned buffers (frames uint8 [n][h][w],
    dets int32 [n][cap][10], n_dets int32 [n], workspace tensor) captured
    once as a hipGraph on ``stream``; launch() replays it on a stream."""

    def __init__(self, frames: torch.Tensor, W, b, dets: torch.Tensor, n_dets: torch.Tensor, ws: torch.Tensor,
                 thresh=0.0, iou=0.5, upsample=1, stream=None):
        n, h, w = (int(v) for v in frames.shape)
        nf = int(W.shape[0])
        need = workspace_bytes(h, w, upsample, n, nf)
        if ws.numel() < need:
            raise HogError(f"workspace of {ws.numel()} bytes, {need} needed")
        self.keep = (frames, W, b, dets, n_dets, ws)
        self.prm = _params(thresh, iou, upsample)
        self.handle = ctypes.c_void_p()
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().hog_graph_create(ctypes.byref(self.handle), ctypes.byref(self.prm), _fptr(frames), n, h, w,
                                      int(frames.stride(1)), int(frames.stride(0)), _ptr(W), _ptr(b), nf, _ptr(dets),
                                      int(dets.shape[1]), _ptr(n_dets), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      ctypes.c_void_p(st.cuda_stream)), "hog_graph_create")

    def launch(self, stream=None):
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().hog_graph_launch(self.handle, ctypes.c_void_p(st.cuda_stream)), "hog_graph_launch")

    def close(self):
        if self.handle:
            lib().hog_graph_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DetectGraph:
    """hog_detect_batch captured once as a hipGraph over fixed buffers and
    replayed; refresh ``frames`` in place between replays.  ``bank`` (a
    FilterBank) takes the place of W and b when given."""

    def __init__(self, frames: torch.Tensor, W=None, b=None, cap=MAX_DETS, thresh=0.0, iou=0.5, upsample=1,
                 bank: FilterBank = None, min_face: int = 0, regions: torch.Tensor = None, arith: int = ARITH_F32):
        n, h, w = (int(v) for v in frames.shape)
        if bank is None:
            bank = FilterBank(b, W=W)
        nf = bank.nf
        self.frames, self.bank, self.regions = frames, bank, regions
        self.dets, self.n_dets = alloc_dets(n, cap, frames.device)
        self.ws = torch.empty(workspace_bytes(h, w, upsample, n, nf), dtype=torch.uint8, device=frames.device)
        self.prm = _params(thresh, iou, upsample, min_face, regions, n, arith)
        self.stream = torch.cuda.Stream(device=frames.device)
        self.handle = ctypes.c_void_p()
        torch.cuda.synchronize(frames.device)
        _check(lib().hog_graph_create_bank(ctypes.byref(self.handle), ctypes.byref(self.prm), _fptr(frames), n, h,
                                           w, int(frames.stride(1)), int(frames.stride(0)), ctypes.byref(bank.struct),
                                           _ptr(self.dets), cap, _ptr(self.n_dets),
                                           ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                           ctypes.c_void_p(self.stream.cuda_stream)), "hog_graph_create_bank")

    def launch(self):
        _check(lib().hog_graph_launch(self.handle, _stream()), "hog_graph_launch")

    def close(self):
        if self.handle:
            lib().hog_graph_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ClipStream:
    """Several clips in flight: one captured DetectGraph per input buffer
    (``frames_list``; each graph has its own workspace and outputs), launched
    in turn on as many streams.  While one clip's per-frame NMS holds a few
    compute units, the next clip's histograms and scores run on the others.
    ``launch`` returns the graph just launched; its ``dets`` / ``n_dets`` are
    valid once ``stream_of(graph)`` has completed the launch.  Refill a
    graph's frames on its stream (or after synchronising it) before its next
    launch."""

    def __init__(self, frames_list, W=None, b=None, **kw):
        if not frames_list:
            raise ValueError("ClipStream needs at least one frames buffer")
        self.graphs = [DetectGraph(f, W, b, **kw) for f in frames_list]
        dev = frames_list[0].device
        self.streams = [torch.cuda.Stream(device=dev) for _ in self.graphs]
        self.next = 0

    def __len__(self):
        return len(self.graphs)

    def launch(self):
        i = self.next
        with torch.cuda.stream(self.streams[i]):
            self.graphs[i].launch()
        self.next = (i + 1) % len(self.graphs)
        return self.graphs[i]

    def stream_of(self, graph):
        return self.streams[self.graphs.index(graph)]

    def synchronize(self):
        for s in self.streams:
            s.synchronize()

    def close(self):
        for g in self.graphs:
            g.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_clip_stream(frames_list, W, b, candidates, warmup: int = 10, reps: int = 40, **kw):
    """Time ``reps`` launches of a ClipStream over ``frames_list`` under each
    candidate schedule (dicts for ``tuning_set``); the fastest is set for the
    shape and returned with its ms per clip."""
    n, h, w = (int(v) for v in frames_list[0].shape)
    nf = int(W.shape[0])
    up = int(kw.get("upsample", 1))
    best, best_ms = None, float("inf")
    for t in candidates:
        tuning_set(h, w, up, n, nf, t)
        cs = ClipStream(frames_list, W, b, **kw)
        for _ in range(warmup):
            cs.launch()
        cs.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            cs.launch()
        cs.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        cs.close()
        if ms < best_ms:
            best, best_ms = dict(t), ms
    tuning_set(h, w, up, n, nf, best)
    return best, best_ms


def level_maps(frame: torch.Tensor, level: int, upsample: int = 1, ws=None):
    """(level pixels float32 [h_k][w_k], bins uint8 [h_k][w_k], hist float32 [cy][cx][18])."""
    h, w, pitch = _frame_args(frame)
    lv = pyramid(h, w, upsample, 0)[level]
    px = torch.empty((lv["h"], lv["w"]), dtype=torch.float32, device=frame.device)
    bins = torch.empty((lv["h"], lv["w"]), dtype=torch.uint8, device=frame.device)
    hist = torch.empty((lv["cy"], lv["cx"], 18), dtype=torch.float32, device=frame.device)
    wp, wn = _ws(ws, workspace_bytes(h, w, upsample, 1, 0))
    _check(lib().hog_level_maps(_fptr(frame), h, w, pitch, upsample, level, _ptr(px), _ptr(bins), _ptr(hist),
                                wp, wn, _stream()), "hog_level_maps")
    return px, bins, hist


def orient_bins(gx: torch.Tensor, gy: torch.Tensor) -> torch.Tensor:
    """Orientation bins of int32 gradients (units of 2^-16)."""
    out = torch.empty(gx.shape, dtype=torch.uint8, device=gx.device)
    _check(lib().hog_orient_bins(_ptr(gx), _ptr(gy), gx.numel(), _ptr(out), _stream()), "hog_orient_bins")
    return out


# ------------------------------------------------------------ gradients
def _frames_args(frames: torch.Tensor):
    if frames.dtype != torch.uint8 or frames.dim() != 3:
        raise HogError("frames must be a uint8 [n][h][w] device tensor")
    n, h, w = (int(v) for v in frames.shape)
    return n, h, w, int(frames.stride(1)), int(frames.stride(0))


def grad_workspace_bytes(h, w, upsample, n, nf, n_windows) -> int:
    b = lib().hog_grad_workspace_bytes(h, w, upsample, n, nf, n_windows)
    if b == 0:
        raise HogError("hog_grad_workspace_bytes: invalid arguments")
    return int(b)


def windows_tensor(frame, filt, level, row, col, device="cuda"):
    """hog_window records as an int32 [n][5] tensor."""
    cols = [torch.as_tensor(v, dtype=torch.int32).reshape(-1) for v in (frame, filt, level, row, col)]
    n = max(c.numel() for c in cols)
    cols = [c.expand(n) if c.numel() == 1 else c for c in cols]
    return torch.stack(cols, 1).contiguous().to(device)


def windows_check(windows: torch.Tensor, n: int, h: int, w: int, nf: int, upsample: int = 1):
    """Raises HogError unless every hog_window record (int32 [m][5], any
    device) addresses a frame of the batch, a filter, a level and an anchor
    inside that level (the library's own test, run on a host copy)."""
    if windows.dtype != torch.int32 or windows.dim() != 2 or windows.shape[1] != 5:
        raise HogError("windows must be int32 [m][5] hog_window records")
    host = windows.detach().to("cpu").contiguous()
    bad = ctypes.c_int(-1)
    st = lib().hog_windows_check(h, w, upsample, n, nf, ctypes.c_void_p(host.data_ptr()), int(host.shape[0]),
                                 ctypes.byref(bad))
    if st != HOG_OK:
        i = bad.value
        rec = host[i].tolist() if 0 <= i < host.shape[0] else None
        raise HogError(f"hog_windows_check: window {i} {rec} is outside the batch ({st})")


def window_scores(frames: torch.Tensor, W, b, windows: torch.Tensor, upsample: int = 1, ws=None,
                  check: bool = True):
    """Scores of the listed windows (int32 [m][5] hog_window records)."""
    n, h, w, pitch, stride = _frames_args(frames)
    m = int(windows.shape[0])
    nf = int(W.shape[0])
    if check:
        windows_check(windows, n, h, w, nf, upsample)
    out = torch.empty(m, dtype=torch.float32, device=frames.device)
    wp, wn = _ws(ws, grad_workspace_bytes(h, w, upsample, n, nf, m))
    _check(lib().hog_window_scores(_fptr(frames), n, h, w, pitch, stride, upsample, _ptr(W), _ptr(b), nf,
                                   _ptr(windows), m, _ptr(out), wp, wn, _stream()), "hog_window_scores")
    return out


def topk_windows(frames: torch.Tensor, W, b, k: int = 10, upsample: int = 1, ws=None):
    """The k best windows per frame: (int32 [n][k][5] records, float32 [n][k] scores)."""
    n, h, w, pitch, stride = _frames_args(frames)
    nf = int(W.shape[0])
    win = torch.empty((n, k, 5), dtype=torch.int32, device=frames.device)
    sc = torch.empty((n, k), dtype=torch.float32, device=frames.device)
    wp, wn = _ws(ws, grad_workspace_bytes(h, w, upsample, n, nf, 1))
    _check(lib().hog_topk_windows(_fptr(frames), n, h, w, pitch, stride, upsample, _ptr(W), _ptr(b), nf, k,
                                  _ptr(win), _ptr(sc), wp, wn, _stream()), "hog_topk_windows")
    return win, sc


def detect_topk_into(frames: torch.Tensor, W, b, dets: torch.Tensor, n_dets: torch.Tensor, k: int = 10,
                     thresh: float = 0.0, iou: float = 0.5, upsample: int = 1, ws=None):
    """hog_detect_topk: detections into dets / n_dets and the k best windows
    of every frame, from one forward pass.  Returns (windows int32 [n][k][5],
    scores float32 [n][k])."""
    n, h, w, pitch, stride = _frames_args(frames)
    nf = int(W.shape[0])
    win = torch.empty((n, k, 5), dtype=torch.int32, device=frames.device)
    sc = torch.empty((n, k), dtype=torch.float32, device=frames.device)
    prm = _params(thresh, iou, upsample)
    wp, wn = _ws(ws, grad_workspace_bytes(h, w, upsample, n, nf, 1))
    _check(lib().hog_detect_topk(ctypes.byref(prm), _fptr(frames), n, h, w, pitch, stride, _ptr(W), _ptr(b), nf,
                                 _ptr(dets), int(dets.shape[1]), _ptr(n_dets), k, _ptr(win), _ptr(sc), wp, wn,
                                 _stream()), "hog_detect_topk")
    return win, sc


def filter_backward(frames: torch.Tensor, W, windows: torch.Tensor, dscore: torch.Tensor, upsample: int = 1,
                    pixels: bool = False, dW=None, db=None, ws=None, check: bool = True):
    """(dW, db, dpixels or None) for upstream score gradients dscore [m]."""
    n, h, w, pitch, stride = _frames_args(frames)
    m = int(windows.shape[0])
    nf = int(W.shape[0])
    if check:
        windows_check(windows, n, h, w, nf, upsample)
    dW = torch.zeros_like(W) if dW is None else dW
    db = torch.zeros(nf, dtype=torch.float32, device=frames.device) if db is None else db
    dpix = torch.zeros((n, h, w), dtype=torch.float32, device=frames.device) if pixels else None
    wp, wn = _ws(ws, grad_workspace_bytes(h, w, upsample, n, nf, m))
    _check(lib().hog_filter_backward(_fptr(frames), n, h, w, pitch, stride, upsample, _ptr(W), nf, _ptr(windows),
                                     _ptr(dscore), m, _ptr(dW), _ptr(db), _ptr(dpix) if pixels else None, wp, wn,
                                     _stream()), "hog_filter_backward")
    return dW, db, dpix


def hinge_loss(scores: torch.Tensor, labels: torch.Tensor, W: torch.Tensor, l2: float = 1e-4, dW=None):
    """(loss [1], dscore [n], dW) with dW += 2 l2 W."""
    n = int(scores.numel())
    loss = torch.empty(1, dtype=torch.float32, device=scores.device)
    dscore = torch.empty(n, dtype=torch.float32, device=scores.device)
    dW = torch.zeros_like(W) if dW is None else dW
    _check(lib().hog_hinge_loss(_ptr(scores), _ptr(labels), n, _ptr(W), int(W.shape[0]), ctypes.c_float(l2),
                                _ptr(loss), _ptr(dscore), _ptr(dW), _stream()), "hog_hinge_loss")
    return loss, dscore, dW


class HogScore(torch.autograd.Function):
    """Window scores as a differentiable function of the filters and bias:
    forward hog_window_scores, backward hog_filter_backward (features
    recomputed from the frames)."""

    @staticmethod
    def forward(ctx, W, b, frames, windows, upsample=1):
        ctx.save_for_backward(W, frames, windows)
        ctx.upsample = upsample
        return window_scores(frames, W.detach().contiguous(), b.detach().contiguous(), windows, upsample)

    @staticmethod
    def backward(ctx, dscore):
        W, frames, windows = ctx.saved_tensors
        dW, db, _ = filter_backward(frames, W.detach().contiguous(), windows, dscore.contiguous().float(),
                                    ctx.upsample)
        return dW, db, None, None, None


class HogPixelScore(torch.autograd.Function):
    """Window scores as a differentiable function of the frame pixels, the
    filters and the bias.  ``pixels`` is a float tensor [n][h][w] holding
    integer grey levels 0..255 (the detector's input is 8-bit); forward
    hog_window_scores on those frames, backward hog_filter_backward with
    the pixel gradient (orientation bins and clip decisions held at their
    forward values)."""

    @staticmethod
    def forward(ctx, pixels, W, b, windows, upsample=1):
        if pixels.dim() != 3 or not pixels.is_floating_point():
            raise HogError("pixels must be a float [n][h][w] tensor of grey levels")
        frames = pixels.detach().round().clamp(0, 255).to(torch.uint8)
        if not torch.equal(frames.to(pixels.dtype), pixels.detach()):
            raise HogError("pixels must hold integer grey levels in 0..255")
        ctx.save_for_backward(W, frames, windows)
        ctx.upsample = upsample
        return window_scores(frames, W.detach().contiguous(), b.detach().contiguous(), windows, upsample)

    @staticmethod
    def backward(ctx, dscore):
        W, frames, windows = ctx.saved_tensors
        dW, db, dpix = filter_backward(frames, W.detach().contiguous(), windows, dscore.contiguous().float(),
                                       ctx.upsample, pixels=ctx.needs_input_grad[0])
        return dpix, dW, db, None, None


def pixel_gradient(frames: torch.Tensor, W, windows: torch.Tensor, dscore: torch.Tensor, upsample: int = 1):
    """d(sum_i dscore_i * score_i) / d(frame pixels), float32 [n][h][w]."""
    return filter_backward(frames, W, windows, dscore, upsample, pixels=True)[2]


# ------------------------------------------------------------ profiling
def profile_enable(on: bool = True):
    _check(lib().hog_profile_enable(1 if on else 0), "hog_profile_enable")


def profile_reset():
    _check(lib().hog_profile_reset(), "hog_profile_reset")


def profile_read(kernel: str):
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().hog_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)), "hog_profile_read")
    return ms.value, cnt.value


# ----------------------------------------------------------- host pipeline
CONSUMER_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_int)


class hog_pipeline_config(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int32), ("w", ctypes.c_int32), ("batch", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("cap", ctypes.c_int32), ("consumer_threads", ctypes.c_int32), ("staging", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("consumer", CONSUMER_FN), ("user", ctypes.c_void_p)]


class Pipeline:
    """hog_pipeline: frames from host memory through the detector to a
    consumer called on the library's consumer threads with each batch's
    detections.  consumer(first_frame, dets, n_dets) receives numpy copies
    (DET_DTYPE records [n][cap], int32 [n]); None keeps only counts."""

    def __init__(self, W: torch.Tensor, b: torch.Tensor, h: int, w: int, batch: int, depth: int = 3, cap: int = 64,
                 consumer_threads: int = 1, staging: bool = True, consumer=None, thresh: float = 0.0,
                 iou: float = 0.5, upsample: int = 1, min_face: int = 0):
        self.W, self.b, self.user_fn = W, b, consumer
        self.frames_done = 0

        def _cb(user, first, n, dets, n_dets, cap_):
            nd = np.ctypeslib.as_array(ctypes.cast(n_dets, ctypes.POINTER(ctypes.c_int32)), (n,)).copy()
            self.frames_done += n
            if self.user_fn is not None:
                raw = np.ctypeslib.as_array(ctypes.cast(dets, ctypes.POINTER(ctypes.c_int32)), (n, cap_, 10)).copy()
                self.user_fn(int(first), raw.view(DET_DTYPE).reshape(n, cap_), nd)

        self._cb = CONSUMER_FN(_cb)
        self.cfg = hog_pipeline_config(h, w, batch, depth, cap, consumer_threads, 1 if staging else 0, 0, self._cb,
                                       None)
        self.prm = _params(thresh, iou, upsample, min_face)
        self.handle = ctypes.c_void_p()
        _check(lib().hog_pipeline_create(ctypes.byref(self.handle), ctypes.byref(self.prm), ctypes.byref(self.cfg),
                                         _ptr(W), _ptr(b), int(W.shape[0])), "hog_pipeline_create")

    def submit(self, frames, first_frame: int):
        """frames: host uint8 [n][h][w], a C-contiguous numpy array or a CPU
        tensor (pinned or not)."""
        if isinstance(frames, torch.Tensor):
            if frames.is_cuda or frames.dtype != torch.uint8 or not frames.is_contiguous():
                raise HogError("frames must be a contiguous host uint8 tensor")
            ptr, n = ctypes.c_void_p(frames.data_ptr()), int(frames.shape[0])
        else:
            if frames.dtype != np.uint8 or not frames.flags.c_contiguous:
                raise HogError("frames must be a C-contiguous uint8 array")
            ptr, n = ctypes.c_void_p(frames.ctypes.data), int(frames.shape[0])
        if tuple(frames.shape[1:]) != (self.cfg.h, self.cfg.w):
            raise HogError("frame size differs from the pipeline's")
        _check(lib().hog_pipeline_submit(self.handle, ptr, n, int(first_frame)), "hog_pipeline_submit")

    def drain(self):
        _check(lib().hog_pipeline_drain(self.handle), "hog_pipeline_drain")

    def close(self):
        if self.handle:
            st = lib().hog_pipeline_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            _check(st, "hog_pipeline_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

