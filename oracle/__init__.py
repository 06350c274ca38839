"""FP64 CPU oracle of three-filters-to-normal — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never loads it, and it shares no code with them.

``sne_oracle.c`` holds the arithmetic (see its header for the definition it
follows, Sec. III of the paper); this module builds it with gcc, loads it with
ctypes and marshals numpy arrays.  ``exact.py`` is an independent brute-force
evaluation in rational arithmetic for tiny integer images.  ``accuracy``
evaluates the paper's accuracy metrics e_A and e_P (eq. ea_ep) in numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sne_oracle.c")
LIB = os.path.join(HERE, "libsne_oracle.so")

KINDS = {"depth_f32": 0, "depth_u16": 1, "depth_f16": 2, "disparity_f32": 3,
         "depth_f64": 4, "disparity_f64": 5}
KIND_DTYPE = {"depth_f32": np.float32, "depth_u16": np.uint16, "depth_f16": np.float16,
              "disparity_f32": np.float32, "depth_f64": np.float64,
              "disparity_f64": np.float64}
GRADS = {"fd": 0, "sobel": 1, "scharr": 2, "prewitt": 3}
AGGS = {"mean": 0, "median": 1}
RULES = {"strict": 0, "lenient": 1}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, -O2, OpenMP, no intrinsics)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c11", "-Wall", "-Wextra",
                               "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        common = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                  ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                  ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        lib.orc_estimate.argtypes = common + [dp, ctypes.c_void_p, dp, ctypes.c_void_p,
                                              ctypes.c_int]
        lib.orc_estimate.restype = ctypes.c_int
        lib.orc_estimate_pixels.argtypes = common + [ctypes.c_void_p, ctypes.c_int64, dp,
                                                     ctypes.c_void_p, dp, ctypes.c_void_p,
                                                     ctypes.c_int]
        lib.orc_estimate_pixels.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prep(raw: np.ndarray, kind: str) -> np.ndarray:
    if kind not in KINDS:
        raise ValueError("unknown kind %r" % kind)
    raw = np.ascontiguousarray(raw)
    want = KIND_DTYPE[kind]
    if raw.dtype != want:
        raise TypeError("kind %s needs %s input, got %s" % (kind, np.dtype(want), raw.dtype))
    if raw.ndim != 2:
        raise ValueError("expected a 2-D image")
    return raw


CUSTOM_SIZES = {3: 4, 5: 5, 7: 6}


def _grad(grad):
    """(code, kx) of a gradient filter: a name, or a 3x3, 5x5 or 7x7 K_x
    (custom)."""
    if isinstance(grad, str):
        return GRADS[grad], None
    kx = np.ascontiguousarray(np.asarray(grad, dtype=np.float64))
    if kx.ndim != 2 or kx.shape[0] != kx.shape[1] or kx.shape[0] not in CUSTOM_SIZES:
        raise ValueError("a custom gradient kernel is 3x3, 5x5 or 7x7")
    return CUSTOM_SIZES[kx.shape[0]], kx


def estimate(raw: np.ndarray, kind: str, K: Sequence[float], grad="fd",
             agg: str = "mean", tc: float = 1.0, threads: int = 0, unnorm: bool = False,
             mcount: bool = False, rule: str = "strict"):
    """Normals [3,H,W] float64 and mask [H,W] uint8 of one image.

    ``rule``: "strict" (a fully valid filter window at an interior pixel) or
    "lenient" (valid neighbours only, one-sided gradient lines; see the header
    of sne_oracle.c).  ``grad``: "fd", "sobel", "scharr", "prewitt" or a 3x3,
    5x5 or 7x7 custom K_x (row-major, K_y = K_x^T; Q_i stays the
    8-neighbourhood).

    K = (fx, fy, u0, v0) as the values the caller wants used (pass the FP32
    values a GPU run used to compare like with like).  With ``unnorm`` the
    unnormalised n' = (n_x, n_y, n_z) [3,H,W] is returned too; with ``mcount``
    the number of candidates kept per pixel [H,W] (-1 masked, 0 degenerate)."""
    raw = _prep(raw, kind)
    H, W = raw.shape
    fx, fy, u0, v0 = (float(x) for x in K)
    nrm = np.zeros((3, H, W), np.float64)
    msk = np.zeros((H, W), np.uint8)
    un = np.zeros((3, H, W), np.float64) if unnorm else None
    mc = np.zeros((H, W), np.int32) if mcount else None
    g, kx = _grad(grad)
    rc = _load().orc_estimate(raw.ctypes.data, KINDS[kind], H, W, W, fx, fy, u0, v0, float(tc),
                              g, AGGS[agg], RULES[rule], _dp(kx), _dp(nrm), msk.ctypes.data,
                              _dp(un),
                              None if mc is None else mc.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments (rc=%d)" % rc)
    out = [nrm, msk]
    if unnorm:
        out.append(un)
    if mcount:
        out.append(mc)
    return tuple(out)


def estimate_pixels(raw: np.ndarray, kind: str, K: Sequence[float], pix: np.ndarray,
                    grad="fd", agg: str = "mean", tc: float = 1.0, threads: int = 0,
                    unnorm: bool = False, mcount: bool = False, rule: str = "strict"):
    """Normals [n,3] and mask [n] at flat pixel indices ``pix`` (v*W + u)."""
    raw = _prep(raw, kind)
    H, W = raw.shape
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.size
    fx, fy, u0, v0 = (float(x) for x in K)
    nrm = np.zeros((n, 3), np.float64)
    msk = np.zeros(n, np.uint8)
    un = np.zeros((n, 3), np.float64) if unnorm else None
    mc = np.zeros(n, np.int32) if mcount else None
    g, kx = _grad(grad)
    rc = _load().orc_estimate_pixels(raw.ctypes.data, KINDS[kind], H, W, W, fx, fy, u0, v0,
                                     float(tc), g, AGGS[agg], RULES[rule], _dp(kx),
                                     pix.ctypes.data, n,
                                     _dp(nrm), msk.ctypes.data, _dp(un),
                                     None if mc is None else mc.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments (rc=%d)" % rc)
    out = [nrm, msk]
    if unnorm:
        out.append(un)
    if mcount:
        out.append(mc)
    return tuple(out)


def angular_error_deg(a: np.ndarray, b: np.ndarray, axis: int = 0) -> np.ndarray:
    """Angle between vectors a and b (FP64) as atan2(|a x b|, a.b) in degrees:
    the psi of Sec. IV-A, well conditioned near 0."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    cr = np.cross(a, b, axisa=axis, axisb=axis, axisc=axis)
    return np.degrees(np.arctan2(np.linalg.norm(cr, axis=axis), np.sum(a * b, axis=axis)))


def accuracy(est: np.ndarray, gt: np.ndarray, mask: Optional[np.ndarray] = None,
             phis: Sequence[float] = (11.25, 22.5, 30.0)):
    """Accuracy metrics of eq. ea_ep (Sec. IV-A) in FP64, written as the
    paper defines them: psi_k = arccos(<n_k, g_k> / (|n_k| |g_k|)) in degrees
    over the m pixels evaluated (those with mask != 0; all if mask is None),
    e_A = mean psi_k, e_P(phi) = fraction of pixels with psi_k <= phi.
    est, gt: [..., 3, H, W] (any leading frame axes); mask: [..., H, W].
    Returns (e_A, [e_P(phi) for phi in phis], m); e_A = e_P = 0 when m = 0."""
    n = np.asarray(est, np.float64)
    g = np.asarray(gt, np.float64)
    n = np.moveaxis(n, -3, -1).reshape(-1, 3)
    g = np.moveaxis(g, -3, -1).reshape(-1, 3)
    if mask is not None:
        keep = np.asarray(mask).reshape(-1) != 0
        n, g = n[keep], g[keep]
    m = n.shape[0]
    if m == 0:
        return 0.0, [0.0 for _ in phis], 0
    c = np.sum(n * g, axis=1) / (np.linalg.norm(n, axis=1) * np.linalg.norm(g, axis=1))
    psi = np.degrees(np.arccos(np.clip(c, -1.0, 1.0)))
    return float(psi.mean()), [float(np.mean(psi <= phi)) for phi in phis], m
