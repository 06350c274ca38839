"""Python binding of libsne (include/sne.h): argument marshalling only.

Every step of the estimator runs in the HIP kernels of ``libsne.so``; this
module converts torch tensors (device memory) and Python values into the C
ABI's pointers, pitches and enums.  The raw ``sne_*`` functions mirror the C
names one to one; ``Context`` and the tensor-level helpers below only
allocate outputs with torch and fill in pitches.  If the library is missing
every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Iterable, List, Optional, Sequence, Tuple

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
# SNE_LIBRARY selects another build of the same library (e.g. an experiment)
LIB_PATH = os.environ.get("SNE_LIBRARY", os.path.join(PKG, "libsne.so"))
TUNING_TABLE = os.path.join(PKG, "tuning.txt")  # written by paper_2005_08165_amd.tune
HEADER = os.path.join(os.path.dirname(PKG), "include", "sne.h")

SNE_OK = 0
SNE_ERR_ARG, SNE_ERR_BUDGET, SNE_ERR_STATE = -1, -3, -5
SNE_NOALLOC_MAX_FRAMES = 4096  # include/sne.h
# version tag the library writes into (and requires of) tile-table entries
TILE_CACHE_VERSION = 10200
STATUS = {0: "SNE_OK", -1: "SNE_ERR_ARG", -2: "SNE_ERR_UNSUPPORTED", -3: "SNE_ERR_BUDGET",
          -4: "SNE_ERR_HIP", -5: "SNE_ERR_STATE", -6: "SNE_ERR_FULL", -7: "SNE_ERR_IO"}

KIND = {"depth_f32": 0, "depth_u16": 1, "depth_f16": 2, "disparity_f32": 3}
KIND_DTYPE = {0: torch.float32, 1: torch.uint16, 2: torch.float16, 3: torch.float32}
GRAD = {"fd": 0, "sobel": 1, "scharr": 2, "prewitt": 3, "custom": 4}
AGG = {"mean": 0, "median": 1}
OUT = {"f32": 0, "f16": 1}
OUT_DTYPE = {0: torch.float32, 1: torch.float16}


class SneError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__("%s failed: %s (%d)" % (fn, STATUS.get(status, "?"), status))
        self.status = status


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("u0", ctypes.c_float), ("v0", ctypes.c_float)]


class FrameDesc(ctypes.Structure):
    _fields_ = [("input", ctypes.c_void_p), ("normals", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("in_pitch", ctypes.c_int64), ("out_pitch", ctypes.c_int64),
                ("mask_pitch", ctypes.c_int64), ("k_index", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Tile(ctypes.Structure):
    _fields_ = [("cols_per_lane", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("lanes", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("grad", ctypes.c_int32), ("agg", ctypes.c_int32),
                ("out_type", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch_frames", ctypes.c_int32), ("max_batch_pixels", ctypes.c_int64),
                ("hbm_budget_bytes", ctypes.c_int64), ("queue_capacity", ctypes.c_int64),
                ("use_graphs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("input", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("in_pitch", ctypes.c_int64), ("stream_id", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("t_arrival", ctypes.c_double),
                ("ready", ctypes.c_void_p)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("stream_id", ctypes.c_int32), ("normals", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("t_arrival", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("rejected_full", ctypes.c_uint64),
                ("rejected_budget", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("mean_batch_frames", ctypes.c_double), ("latency_p50", ctypes.c_double),
                ("latency_p90", ctypes.c_double), ("latency_p99", ctypes.c_double),
                ("latency_p999", ctypes.c_double), ("latency_max", ctypes.c_double),
                ("mpix_per_s", ctypes.c_double), ("frames_per_s", ctypes.c_double),
                ("arena_free_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LoadgenConfig(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("n_producers", ctypes.c_int32),
                ("total_rate", ctypes.c_double), ("duration_s", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("frames", ctypes.POINTER(ctypes.c_void_p)),
                ("ring", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("H", ctypes.POINTER(ctypes.c_int32)), ("W", ctypes.POINTER(ctypes.c_int32)),
                ("pitch", ctypes.POINTER(ctypes.c_int64))]


class SimConfig(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch_frames", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_batch_pixels", ctypes.c_int64), ("budget_bytes", ctypes.c_int64),
                ("total_rate", ctypes.c_double), ("duration_s", ctypes.c_double),
                ("gpu_pixels_per_s", ctypes.c_double), ("batch_overhead_s", ctypes.c_double),
                ("tick_s", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("H", ctypes.POINTER(ctypes.c_int32)), ("W", ctypes.POINTER(ctypes.c_int32))]


_lib = None
_vp, _i32, _i64, _int = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int

_SIGS = {
    "sne_version": ([], _int),
    "sne_status_string": ([_int], ctypes.c_char_p),
    "sne_ctx_create": ([ctypes.POINTER(_vp), _int], _int),
    "sne_ctx_destroy": ([_vp], _int),
    "sne_estimate": ([_vp, _vp, _i32, _i32, _i64, ctypes.POINTER(Intrinsics), _int, _int, _int,
                      _int, _vp, _i64, _vp, _i64, _vp], _int),
    "sne_estimate_uniform": ([_vp, _vp, _i32, _i32, _i32, _i64, _i64, ctypes.POINTER(Intrinsics),
                              _int, _int, _int, _int, _vp, _i64, _i64, _vp, _i64, _i64, _vp],
                             _int),
    "sne_estimate_rgbn": ([_vp, _vp, _i32, _i32, _i32, _i64, _i64, ctypes.POINTER(Intrinsics),
                           _int, _int, _int, _vp, _i64, _i64, _vp, _i64, _i64, _vp, _i64, _i64,
                           _vp], _int),
    "sne_set_intrinsics_table": ([_vp, ctypes.POINTER(Intrinsics), _i32], _int),
    "sne_set_gradient_kernel": ([_vp, ctypes.POINTER(ctypes.c_float)], _int),
    "sne_set_gradient_kernel_n": ([_vp, _int, ctypes.POINTER(ctypes.c_float)], _int),
    "sne_estimate_batched": ([_vp, ctypes.POINTER(FrameDesc), _i32, _int, _int, _int, _int, _vp],
                             _int),
    "sne_estimate_batched_noalloc": ([_vp, ctypes.POINTER(FrameDesc), _i32, _int, _int, _int,
                                      _int, _vp], _int),
    "sne_set_tile": ([_vp, ctypes.POINTER(Tile)], _int),
    "sne_get_tile": ([_vp, _i32, _i32, _i32, _int, _int, _int, _int, ctypes.POINTER(Tile)], _int),
    "sne_get_tile_pitched": ([_vp, _i32, _i32, _i32, _i64, _i64, _int, _int, _int, _int,
                              ctypes.POINTER(Tile)], _int),
    "sne_autotune": ([_vp, _i32, _i32, _i32, _int, _int, _int, _int, ctypes.POINTER(Tile)], _int),
    "sne_autotune_pitched": ([_vp, _i32, _i32, _i32, _i64, _i64, _int, _int, _int, _int,
                              ctypes.POINTER(Tile)], _int),
    "sne_row_pitch": ([_i32, _i32], _i64),
    "sne_autotune_batched": ([_vp, ctypes.POINTER(FrameDesc), _i32, _int, _int, _int, _int,
                              ctypes.POINTER(Tile)], _int),
    "sne_autotune_save": ([_vp, ctypes.c_char_p], _int),
    "sne_accuracy": ([_vp, _vp, _int, _vp, _vp, _i32, ctypes.c_int64,
                      ctypes.POINTER(ctypes.c_float), _i32, _vp, _vp], _int),
    "sne_autotune_load": ([_vp, ctypes.c_char_p], _int),
    "sne_server_create": ([ctypes.POINTER(_vp), _vp, ctypes.POINTER(ServerConfig)], _int),
    "sne_server_submit": ([_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], _int),
    "sne_server_poll": ([_vp, ctypes.POINTER(Completion), _i32, ctypes.POINTER(_i32)], _int),
    "sne_server_release": ([_vp, ctypes.c_uint64], _int),
    "sne_server_drain": ([_vp, ctypes.c_double], _int),
    "sne_server_get_stats": ([_vp, ctypes.POINTER(ServerStats)], _int),
    "sne_server_reset_stats": ([_vp], _int),
    "sne_server_now": ([_vp], ctypes.c_double),
    "sne_server_destroy": ([_vp], _int),
    "sne_server_run_open_loop": ([_vp, ctypes.POINTER(LoadgenConfig), ctypes.POINTER(ServerStats)],
                                 _int),
    "sne_bandwidth_probe": ([_int, _vp, _vp, _vp, _i64, _vp], _int),
    "sne_sched_simulate": ([ctypes.POINTER(SimConfig), ctypes.POINTER(ServerStats)], _int),
}


def lib():
    """Load libsne.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsne.so not built: run `python -m paper_2005_08165_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def header_functions() -> List[str]:
    """Names of the functions include/sne.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sne_[a-z_0-9]+)\s*\(", text)))


def check(fn: str, status: int) -> None:
    if status != SNE_OK:
        raise SneError(fn, status)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _on_gpu(*tensors) -> None:
    """Every tensor the library reads or writes must live in device memory:
    a host pointer handed to a kernel would fault the GPU."""
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors passed to the library must be on the GPU, got %s" % t.device)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _sync(stream) -> None:
    """Wait for a torch stream or a raw hipStream_t handle."""
    if isinstance(stream, torch.cuda.Stream):
        stream.synchronize()
        return
    rc = _hip().hipStreamSynchronize(ctypes.c_void_p(int(stream)))
    if rc != 0:
        raise RuntimeError("hipStreamSynchronize failed (%d)" % rc)


def _K(K: Sequence[float]) -> Intrinsics:
    fx, fy, u0, v0 = (float(x) for x in K)
    return Intrinsics(fx, fy, u0, v0)


def _enum(table, key, what):
    if isinstance(key, int):
        return key
    if key not in table:
        raise ValueError("unknown %s %r" % (what, key))
    return table[key]


SNE_LENIENT = 0x100  # include/sne.h


def _kind(kind) -> int:
    """Kind code; a "+lenient" suffix (e.g. "depth_u16+lenient") ORs in
    SNE_LENIENT, the rule for holes and the frame border."""
    if isinstance(kind, int):
        return kind
    base, plus, rule = kind.partition("+")
    code = _enum(KIND, base, "kind")
    if plus:
        if rule != "lenient":
            raise ValueError("unknown kind suffix %r" % rule)
        code |= SNE_LENIENT
    return code


def _dtype(kind_i: int):
    return KIND_DTYPE[kind_i & ~SNE_LENIENT]


def row_pitch(W: int, dtype) -> int:
    """sne_row_pitch: the smallest row pitch (elements) >= W whose rows start
    at 256-byte boundaries, for a 1, 2 or 4-byte dtype."""
    p = lib().sne_row_pitch(int(W), torch.empty((), dtype=dtype).element_size())
    if p < 0:
        check("sne_row_pitch", int(p))
    return int(p)


def pitched_empty(shape: Sequence[int], dtype=torch.float32, device="cuda") -> torch.Tensor:
    """An uninitialised [..., H, W] tensor whose rows are padded to
    row_pitch(W, dtype) elements (a view of the first W columns), the layout
    that keeps every row on a 256-byte boundary."""
    shape = tuple(int(x) for x in shape)
    full = torch.empty(shape[:-1] + (row_pitch(shape[-1], dtype),), dtype=dtype, device=device)
    return full[..., :shape[-1]]


def _row_pitch(t: torch.Tensor) -> int:
    """Row pitch (elements) of a [..., H, W] tensor with unit column stride."""
    if t.stride(-1) != 1:
        raise ValueError("images need a unit column stride")
    return t.stride(-2)


class Context:
    """Owns an sne_ctx bound to one GPU."""

    def __init__(self, device: int = 0, tuning: bool = True):
        """`tuning`: load the shipped tile table (tuning.txt beside this
        module) when it exists; without it tiles come from the heuristic."""
        self._h = ctypes.c_void_p()
        check("sne_ctx_create", lib().sne_ctx_create(ctypes.byref(self._h), int(device)))
        self.device = int(device)
        if tuning and os.path.exists(TUNING_TABLE):
            self.autotune_load(TUNING_TABLE)

    @property
    def handle(self):
        return self._h

    def close(self):
        """Free the context (SneError with SNE_ERR_STATE while a Server on it
        is still open; the context then stays usable)."""
        if self._h:
            check("sne_ctx_destroy", lib().sne_ctx_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tile shapes ---------------------------------------------------------
    def set_tile(self, cols_per_lane: int = 0, rows: int = 0, lanes: int = 64):
        t = Tile(int(cols_per_lane), int(rows), int(lanes))
        check("sne_set_tile", lib().sne_set_tile(self._h, ctypes.byref(t)))

    def get_tile(self, H, W, B=1, kind="depth_f32", grad="fd", agg="mean",
                 out="f32", in_pitch=None, out_pitch=None) -> Tuple[int, int, int]:
        """sne_get_tile_pitched: the shape used for frames at these row
        pitches (elements; dense, i.e. W, by default)."""
        t = Tile()
        check("sne_get_tile_pitched",
              lib().sne_get_tile_pitched(self._h, H, W, B, in_pitch or W, out_pitch or W,
                                         _kind(kind), _enum(GRAD, grad, "grad"),
                                         _enum(AGG, agg, "agg"), _enum(OUT, out, "out"),
                                         ctypes.byref(t)))
        return t.cols_per_lane, t.rows, t.lanes

    def autotune(self, H, W, B=1, kind="depth_f32", grad="fd", agg="mean", out="f32",
                 in_pitch=None, out_pitch=None):
        """sne_autotune_pitched on frames at these row pitches (dense by
        default); returns (cols_per_lane, rows, lanes)."""
        t = Tile()
        check("sne_autotune_pitched",
              lib().sne_autotune_pitched(self._h, H, W, B, in_pitch or W, out_pitch or W,
                                         _kind(kind), _enum(GRAD, grad, "grad"),
                                         _enum(AGG, agg, "agg"), _enum(OUT, out, "out"),
                                         ctypes.byref(t)))
        return t.cols_per_lane, t.rows, t.lanes

    def autotune_batched(self, descs, kind="depth_u16", grad="fd", agg="mean", out="f16"):
        """sne_autotune_batched on a prepared descriptor array (its outputs
        are written); returns (cols_per_lane, rows, lanes)."""
        t = Tile()
        check("sne_autotune_batched",
              lib().sne_autotune_batched(self._h, descs, len(descs), _kind(kind),
                                         _enum(GRAD, grad, "grad"), _enum(AGG, agg, "agg"),
                                         _enum(OUT, out, "out"), ctypes.byref(t)))
        return t.cols_per_lane, t.rows, t.lanes

    def accuracy(self, normals: torch.Tensor, gt: torch.Tensor,
                 mask: Optional[torch.Tensor] = None, phis=(11.25, 22.5, 30.0), stream=None):
        """sne_accuracy: (e_A, [e_P(phi) ...], m) of eq. ea_ep for normals
        [..., 3, H, W] (FP32 or FP16) against ground truth [..., 3, H, W]
        (FP32) over the pixels where mask [..., H, W] is non-zero.  Waits for
        the result."""
        _on_gpu(normals, gt, mask)
        if normals.dtype not in (torch.float32, torch.float16) or gt.dtype != torch.float32:
            raise TypeError("normals FP32/FP16 and ground truth FP32 expected")
        if normals.shape != gt.shape or normals.shape[-3] != 3:
            raise ValueError("normals and ground truth must both be [..., 3, H, W]")
        if not (normals.is_contiguous() and gt.is_contiguous()):
            raise ValueError("contiguous tensors expected")
        frame_px = normals.shape[-1] * normals.shape[-2]
        B = normals.numel() // (3 * frame_px) if frame_px else 0
        if mask is not None:
            if mask.dtype != torch.uint8 or not mask.is_contiguous() or mask.numel() != B * frame_px:
                raise ValueError("mask must be a contiguous uint8 [..., H, W]")
        ph = (ctypes.c_float * max(len(phis), 1))(*[float(p) for p in phis])
        res = torch.empty(2 + len(phis), dtype=torch.float64, device=normals.device)
        check("sne_accuracy",
              lib().sne_accuracy(self._h, normals.data_ptr(), 1 if normals.dtype == torch.float16
                                 else 0, gt.data_ptr(), _ptr(mask), B, frame_px, ph, len(phis),
                                 res.data_ptr(), _stream(stream)))
        if stream is not None:
            _sync(stream)  # res was written there; read it only once it is done
        r = res.cpu().tolist()
        return r[0], r[2:], int(r[1])

    def autotune_save(self, path: str):
        check("sne_autotune_save", lib().sne_autotune_save(self._h, path.encode()))

    def autotune_load(self, path: str):
        check("sne_autotune_load", lib().sne_autotune_load(self._h, path.encode()))

    def set_intrinsics_table(self, Ks: Sequence[Sequence[float]]):
        arr = (Intrinsics * len(Ks))(*[_K(k) for k in Ks])
        check("sne_set_intrinsics_table", lib().sne_set_intrinsics_table(self._h, arr, len(Ks)))

    def set_gradient_kernel(self, kx) -> None:
        """sne_set_gradient_kernel_n: the square K_x (row-major; 3x3, 5x5 or
        7x7) that grad="custom" uses on this context (K_y = K_x^T)."""
        rows = [[float(x) for x in row] for row in kx]
        n = len(rows)
        if any(len(r) != n for r in rows):
            raise ValueError("a square kernel is expected")
        vals = [x for r in rows for x in r]
        arr = (ctypes.c_float * max(len(vals), 1))(*vals)
        check("sne_set_gradient_kernel_n", lib().sne_set_gradient_kernel_n(self._h, n, arr))

    # -- compute -------------------------------------------------------------
    def estimate(self, raw: torch.Tensor, K, kind="depth_f32", grad="fd", agg="mean", out="f32",
                 normals: Optional[torch.Tensor] = None, mask: Optional[torch.Tensor] = None,
                 want_mask: bool = True, stream=None):
        return estimate(raw, K, kind, grad, agg, out, normals, mask, want_mask, stream, ctx=self)

    def estimate_uniform(self, raw: torch.Tensor, K, kind="depth_f32", grad="fd", agg="mean",
                         out="f32", normals=None, mask=None, want_mask=True, stream=None):
        return estimate_uniform(raw, K, kind, grad, agg, out, normals, mask, want_mask, stream,
                                ctx=self)

    def prepare_batched(self, frames: Sequence[torch.Tensor], k_index: Sequence[int],
                        kind="depth_u16", out="f16",
                        normals: Optional[Sequence[torch.Tensor]] = None,
                        masks: Optional[Sequence[Optional[torch.Tensor]]] = None):
        """Descriptor array (host, ctypes) of an uneven batch, reusable across
        launches, with the outputs it points to."""
        kind_i = _kind(kind)
        out_i = _enum(OUT, out, "out")
        n = len(frames)
        if normals is None:
            normals = [torch.empty((3,) + tuple(f.shape[-2:]), dtype=OUT_DTYPE[out_i],
                                   device=f.device) for f in frames]
        if masks is None:
            masks = [torch.empty(tuple(f.shape[-2:]), dtype=torch.uint8, device=f.device)
                     for f in frames]
        descs = (FrameDesc * n)()
        for i, f in enumerate(frames):
            _on_gpu(f, normals[i], masks[i])
            if f.dtype != _dtype(kind_i):
                raise TypeError("frame %d: kind %s needs %s" % (i, kind, _dtype(kind_i)))
            H, W = f.shape[-2:]
            m = masks[i]
            descs[i] = FrameDesc(f.data_ptr(), normals[i].data_ptr(),
                                 None if m is None else m.data_ptr(), H, W, _row_pitch(f),
                                 _row_pitch(normals[i]), 0 if m is None else _row_pitch(m),
                                 int(k_index[i]), 0)
        return descs, normals, masks

    def run_batched(self, descs, kind="depth_u16", grad="fd", agg="mean", out="f16",
                    stream=None):
        """sne_estimate_batched on a prepared descriptor array."""
        check("sne_estimate_batched",
              lib().sne_estimate_batched(self._h, descs, len(descs), _kind(kind),
                                         _enum(GRAD, grad, "grad"), _enum(AGG, agg, "agg"),
                                         _enum(OUT, out, "out"), _stream(stream)))

    def estimate_batched(self, frames: Sequence[torch.Tensor], k_index: Sequence[int],
                         kind="depth_u16", grad="fd", agg="mean", out="f16",
                         normals: Optional[Sequence[torch.Tensor]] = None,
                         masks: Optional[Sequence[Optional[torch.Tensor]]] = None, stream=None):
        """One persistent launch over frames of any sizes.  Returns the lists
        (normals, masks); outputs are allocated unless given."""
        descs, normals, masks = self.prepare_batched(frames, k_index, kind, out, normals, masks)
        self.run_batched(descs, kind, grad, agg, out, stream)
        return normals, masks


class Server:
    """sne_server_*: continuous-batching serving loop on a Context."""

    def __init__(self, ctx: Context, kind="depth_u16", grad="fd", agg="mean", out="f16",
                 max_inflight=3, max_batch_frames=256, max_batch_pixels=64 << 20,
                 hbm_budget_bytes=4 << 30, queue_capacity=65536, use_graphs=True):
        self.ctx = ctx
        self.kind, self.out = _kind(kind), _enum(OUT, out, "out")
        cfg = ServerConfig(self.kind, _enum(GRAD, grad, "grad"), _enum(AGG, agg, "agg"),
                           self.out, max_inflight, max_batch_frames, max_batch_pixels,
                           hbm_budget_bytes, queue_capacity, 1 if use_graphs else 0, 0)
        self._h = ctypes.c_void_p()
        check("sne_server_create",
              lib().sne_server_create(ctypes.byref(self._h), ctx.handle, ctypes.byref(cfg)))
        self._keep = {}   # ticket -> input tensor kept alive until completion

    def submit(self, frame: torch.Tensor, stream_id: int, t_arrival: float = -1.0,
               producer=None) -> int:
        """Queue one frame.  An event is recorded on `producer` (default: the
        current stream), so the batch reads the frame only after the work
        enqueued there so far; frame and event are kept until release."""
        _on_gpu(frame)
        if frame.dtype != _dtype(self.kind):
            raise TypeError("server kind needs %s frames" % _dtype(self.kind))
        H, W = frame.shape
        ev = torch.cuda.Event()
        ev.record(producer if producer is not None else torch.cuda.current_stream(frame.device))
        r = Request(frame.data_ptr(), H, W, _row_pitch(frame), int(stream_id), 0, float(t_arrival),
                    ev.cuda_event)
        t = ctypes.c_uint64()
        check("sne_server_submit", lib().sne_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = (frame, ev)
        return t.value

    def poll(self, max_n: int = 1024):
        buf = (Completion * max_n)()
        n = ctypes.c_int32()
        check("sne_server_poll", lib().sne_server_poll(self._h, buf, max_n, ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]

    def result(self, c: Completion, copy: bool = True):
        """(normals [3,H,W], mask [H,W]) of a completion, copied out of the
        arena (the arena slot is still held until release)."""
        dt = OUT_DTYPE[self.out]
        esz = torch.tensor([], dtype=dt).element_size()
        n = torch.empty((3, c.H, c.W), dtype=dt, device="cuda")
        m = torch.empty((c.H, c.W), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        _memcpy_d2d(n.data_ptr(), c.normals, 3 * c.H * c.W * esz)
        _memcpy_d2d(m.data_ptr(), c.mask, c.H * c.W)
        return n, m

    def release(self, ticket: int):
        check("sne_server_release", lib().sne_server_release(self._h, int(ticket)))
        self._keep.pop(int(ticket), None)

    def drain(self, timeout_s: float = 30.0):
        check("sne_server_drain", lib().sne_server_drain(self._h, float(timeout_s)))

    def stats(self) -> dict:
        st = ServerStats()
        check("sne_server_get_stats", lib().sne_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def reset_stats(self):
        check("sne_server_reset_stats", lib().sne_server_reset_stats(self._h))

    def now(self) -> float:
        return lib().sne_server_now(self._h)

    def run_open_loop(self, frames: Sequence[Sequence[torch.Tensor]], total_rate: float,
                      duration_s: float, seed: int = 5000, n_producers: int = 8) -> dict:
        """frames[s][k]: the device ring of stream s (stream s uses intrinsics
        row s).  Returns the run's statistics."""
        ns = len(frames)
        ring = len(frames[0])
        ptrs = (ctypes.c_void_p * (ns * ring))()
        Hs = (ctypes.c_int32 * ns)()
        Ws = (ctypes.c_int32 * ns)()
        Ps = (ctypes.c_int64 * ns)()
        for s_, fs in enumerate(frames):
            if len(fs) != ring:
                raise ValueError("every stream needs the same ring length")
            Hs[s_], Ws[s_] = fs[0].shape
            Ps[s_] = _row_pitch(fs[0])
            for k, f in enumerate(fs):
                _on_gpu(f)
                if tuple(f.shape) != (Hs[s_], Ws[s_]) or f.dtype != _dtype(self.kind):
                    raise ValueError("stream %d: frames differ in shape or dtype" % s_)
                ptrs[s_ * ring + k] = f.data_ptr()
        cfg = LoadgenConfig(ns, n_producers, float(total_rate), float(duration_s), int(seed),
                            ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)), ring, 0,
                            ctypes.cast(Hs, ctypes.POINTER(ctypes.c_int32)),
                            ctypes.cast(Ws, ctypes.POINTER(ctypes.c_int32)),
                            ctypes.cast(Ps, ctypes.POINTER(ctypes.c_int64)))
        st = ServerStats()
        check("sne_server_run_open_loop",
              lib().sne_server_run_open_loop(self._h, ctypes.byref(cfg), ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self._h:
            lib().sne_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(stream_shapes: Sequence[Tuple[int, int]], total_rate: float, duration_s: float,
             gpu_pixels_per_s: float, batch_overhead_s: float = 20e-6, max_inflight: int = 3,
             max_batch_frames: int = 256, max_batch_pixels: int = 0,
             budget_bytes: int = 4 << 30, tick_s: float = 10e-6, seed: int = 5000) -> dict:
    """sne_sched_simulate: the scheduler against a GPU model (host only)."""
    ns = len(stream_shapes)
    Hs = (ctypes.c_int32 * ns)(*[h for h, _ in stream_shapes])
    Ws = (ctypes.c_int32 * ns)(*[w for _, w in stream_shapes])
    cfg = SimConfig(ns, max_inflight, max_batch_frames, 0, max_batch_pixels, budget_bytes,
                    float(total_rate), float(duration_s), float(gpu_pixels_per_s),
                    float(batch_overhead_s), float(tick_s), int(seed),
                    ctypes.cast(Hs, ctypes.POINTER(ctypes.c_int32)),
                    ctypes.cast(Ws, ctypes.POINTER(ctypes.c_int32)))
    st = ServerStats()
    check("sne_sched_simulate", lib().sne_sched_simulate(ctypes.byref(cfg), ctypes.byref(st)))
    return st.as_dict()


def _memcpy_d2d(dst: int, src: int, nbytes: int):
    """Device-to-device copy of nbytes on the current stream (plumbing)."""
    s = torch.cuda.current_stream()
    hip = _hip()
    rc = hip.hipMemcpyAsync(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes),
                            3, ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise RuntimeError("hipMemcpyAsync failed (%d)" % rc)
    s.synchronize()


_hiplib = None


def _hip():
    global _hiplib
    if _hiplib is None:
        _hiplib = ctypes.CDLL("libamdhip64.so")
        _hiplib.hipMemcpyAsync.restype = ctypes.c_int
        _hiplib.hipStreamSynchronize.restype = ctypes.c_int
    return _hiplib


def _outputs(raw, out_i, normals, mask, want_mask):
    _on_gpu(raw, normals, mask)
    shape = tuple(raw.shape[:-2]) + (3,) + tuple(raw.shape[-2:])
    if normals is None:
        normals = torch.empty(shape, dtype=OUT_DTYPE[out_i], device=raw.device)
    if tuple(normals.shape) != shape or normals.dtype != OUT_DTYPE[out_i]:
        raise ValueError("normals must be %s %s" % (shape, OUT_DTYPE[out_i]))
    if normals.stride(-3) != raw.shape[-2] * _row_pitch(normals):
        raise ValueError("normal channels must be H * row_pitch apart")
    if mask is None and want_mask:
        mask = torch.empty(tuple(raw.shape), dtype=torch.uint8, device=raw.device)
    if mask is not None and (tuple(mask.shape) != tuple(raw.shape) or mask.dtype != torch.uint8):
        raise ValueError("mask must be %s uint8" % (tuple(raw.shape),))
    return normals, mask


def estimate(raw: torch.Tensor, K, kind="depth_f32", grad="fd", agg="mean", out="f32",
             normals=None, mask=None, want_mask=True, stream=None, ctx: Optional[Context] = None):
    """sne_estimate on a [H, W] device tensor; returns (normals [3,H,W], mask)."""
    kind_i, out_i = _kind(kind), _enum(OUT, out, "out")
    if raw.dim() != 2:
        raise ValueError("expected [H, W]")
    if raw.dtype != _dtype(kind_i):
        raise TypeError("kind %s needs %s input" % (kind, _dtype(kind_i)))
    normals, mask = _outputs(raw, out_i, normals, mask, want_mask)
    H, W = raw.shape
    Kc = _K(K)
    st = lib().sne_estimate(None if ctx is None else ctx.handle, raw.data_ptr(), H, W,
                            _row_pitch(raw), ctypes.byref(Kc), kind_i, _enum(GRAD, grad, "grad"),
                            _enum(AGG, agg, "agg"), out_i, normals.data_ptr(),
                            _row_pitch(normals), _ptr(mask),
                            0 if mask is None else _row_pitch(mask), _stream(stream))
    check("sne_estimate", st)
    return normals, mask


def estimate_uniform(raw: torch.Tensor, K, kind="depth_f32", grad="fd", agg="mean", out="f32",
                     normals=None, mask=None, want_mask=True, stream=None,
                     ctx: Optional[Context] = None):
    """sne_estimate_uniform on a [B, H, W] device tensor; returns
    (normals [B,3,H,W], mask [B,H,W])."""
    kind_i, out_i = _kind(kind), _enum(OUT, out, "out")
    if raw.dim() != 3:
        raise ValueError("expected [B, H, W]")
    if raw.dtype != _dtype(kind_i):
        raise TypeError("kind %s needs %s input" % (kind, _dtype(kind_i)))
    normals, mask = _outputs(raw, out_i, normals, mask, want_mask)
    B, H, W = raw.shape
    Kc = _K(K)
    st = lib().sne_estimate_uniform(
        None if ctx is None else ctx.handle, raw.data_ptr(), B, H, W, _row_pitch(raw),
        raw.stride(0), ctypes.byref(Kc), kind_i, _enum(GRAD, grad, "grad"),
        _enum(AGG, agg, "agg"), out_i, normals.data_ptr(), _row_pitch(normals),
        normals.stride(0), _ptr(mask), 0 if mask is None else _row_pitch(mask),
        0 if mask is None else mask.stride(0), _stream(stream))
    check("sne_estimate_uniform", st)
    return normals, mask


def estimate_rgbn(raw: torch.Tensor, K, kind="depth_f32", grad="fd", agg="mean",
                  rgb: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                  mask: Optional[torch.Tensor] = None, stream=None,
                  ctx: Optional[Context] = None) -> torch.Tensor:
    """sne_estimate_rgbn on [B, H, W] depth (or [H, W]): returns the packed
    [B, H, W, 8] FP16 tensor (R, G, B, mask, n_x, n_y, n_z, 0); rgb is a
    [B, H, W, 4] uint8 RGBX tensor or None."""
    kind_i = _kind(kind)
    single = raw.dim() == 2
    if single:
        raw = raw.unsqueeze(0)
        rgb = None if rgb is None else rgb.unsqueeze(0)
        mask = None if mask is None else mask.unsqueeze(0)
    if raw.dim() != 3:
        raise ValueError("expected [B, H, W] or [H, W]")
    if raw.dtype != _dtype(kind_i):
        raise TypeError("kind %s needs %s input" % (kind, _dtype(kind_i)))
    B, H, W = raw.shape
    if rgb is not None and (tuple(rgb.shape) != (B, H, W, 4) or rgb.dtype != torch.uint8 or
                            rgb.stride(-1) != 1 or rgb.stride(-2) != 4):
        raise ValueError("rgb must be a [B, H, W, 4] uint8 tensor with packed pixels")
    if out is None:
        out = torch.empty((B, H, W, 8), dtype=torch.float16, device=raw.device)
    if (tuple(out.shape) != (B, H, W, 8) or out.dtype != torch.float16 or out.stride(-1) != 1
            or out.stride(-2) != 8):
        raise ValueError("out must be a [B, H, W, 8] float16 tensor with packed pixels")
    _on_gpu(raw, rgb, out, mask)
    Kc = _K(K)
    st = lib().sne_estimate_rgbn(
        None if ctx is None else ctx.handle, raw.data_ptr(), B, H, W, _row_pitch(raw),
        raw.stride(0), ctypes.byref(Kc), kind_i, _enum(GRAD, grad, "grad"),
        _enum(AGG, agg, "agg"), _ptr(rgb), 0 if rgb is None else rgb.stride(1),
        0 if rgb is None else rgb.stride(0), out.data_ptr(), out.stride(1) // 8,
        out.stride(0) // 8, _ptr(mask), 0 if mask is None else _row_pitch(mask),
        0 if mask is None else mask.stride(0), _stream(stream))
    check("sne_estimate_rgbn", st)
    return out[0] if single else out


def status_string(code: int) -> str:
    return lib().sne_status_string(int(code)).decode()


def version() -> int:
    return lib().sne_version()


PROBE = {"read": 0, "write": 1, "copy": 2, "stencil": 3}


def bandwidth_probe(mode: str, src: Optional[torch.Tensor], dst: torch.Tensor,
                    mask: Optional[torch.Tensor] = None, n: Optional[int] = None,
                    stream=None) -> None:
    """sne_bandwidth_probe: one streaming launch of a calibration pattern
    over n float elements (default: all of src, or of dst for "write")."""
    _on_gpu(src, dst, mask)
    if n is None:
        n = (dst if src is None else src).numel()
    check("sne_bandwidth_probe",
          lib().sne_bandwidth_probe(_enum(PROBE, mode, "mode"), _ptr(src), dst.data_ptr(),
                                    _ptr(mask), int(n), _stream(stream)))

