"""Python front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of the benchmark.  The product path (the HIP library and its
binding) never imports or calls it.

Functions follow the paper's steps: ``fragments`` (projection, Eq. 5, and
bilinear splatting, Eq. 6, then per-pixel depth order), ``blend_forward``
(Eq. 1 with early termination, Appendix A.6), ``blend_backward`` (its
exact derivative with the termination count held fixed, per-point
bilinear-weighted combination, Appendix A.6), ``blend_weight`` (the per-point
blend weight for the probability updates, combined with the bilinear
weights, Appendix A.6) and ``multisample`` (per-pixel average over several
sampled clouds, Section 3.2).
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# INPC_ORACLE_LIB selects another build of oracle.c (the sanitizer test loads
# the AddressSanitizer/UBSan build through it)
LIB_PATH = os.environ.get("INPC_ORACLE_LIB") or os.path.join(HERE, "liborc.so")


class _Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("near_plane", ctypes.c_float), ("far_plane", ctypes.c_float)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_emit.restype = i64
        L.orc_emit.argtypes = [P, i64, ctypes.POINTER(_Camera), P, P, P, P, i64]
        L.orc_build_lists.restype = ctypes.c_int
        L.orc_build_lists.argtypes = [i64, i64, P, P, P, P, P, P, P, P]
        L.orc_blend_fwd.restype = None
        L.orc_blend_fwd.argtypes = [i64, P, P, P, P, P, ctypes.c_int, i32, dbl, P, P, P, P, P]
        L.orc_blend_bwd.restype = ctypes.c_int
        L.orc_blend_bwd.argtypes = [i64, P, P, P, P, P, ctypes.c_int, i32, P, P, P, i64, P, P]
        L.orc_blend_weight.restype = None
        L.orc_blend_weight.argtypes = [i64, P, P, P, P, P, i64, P]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel regions (timing runs only)."""
    lib().orc_set_num_threads(int(n))


def _cam(cam) -> _Camera:
    d = cam.as_dict() if hasattr(cam, "as_dict") else dict(cam)
    c = _Camera()
    for i, v in enumerate(d["R"]):
        c.R[i] = v
    for i, v in enumerate(d["t"]):
        c.t[i] = v
    c.fx, c.fy, c.cx, c.cy = d["fx"], d["fy"], d["cx"], d["cy"]
    c.width, c.height = d["width"], d["height"]
    c.near_plane, c.far_plane = d["near"], d["far"]
    return c


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Lists:
    """Per-pixel splat lists of one view, concatenated in pixel order."""

    P: int
    start: np.ndarray    # int64 [P+1]
    zbits: np.ndarray    # uint32 [M], float32 bits of view depth
    ids: np.ndarray      # uint32 [M], 4*point + corner
    w: np.ndarray        # float64 [M], bilinear weight
    n_points: int

    @property
    def m(self) -> int:
        return int(self.ids.shape[0])

    def pixels(self) -> np.ndarray:
        return np.repeat(np.arange(self.P, dtype=np.uint64), np.diff(self.start))

    def keys(self, pixel_offset: int = 0) -> np.ndarray:
        """64-bit (pixel << 32 | depth bits) keys of the sorted splats."""
        return ((self.pixels() + np.uint64(pixel_offset)) << np.uint64(32)) | self.zbits.astype(np.uint64)


def emit(xyz: np.ndarray, cam):
    """Unsorted splats of every point in point order: (pixel, zbits, id, w)."""
    xyz = np.ascontiguousarray(xyz, np.float32)
    n = xyz.shape[0]
    c = _cam(cam)
    L = lib()
    m = L.orc_emit(_ptr(xyz), n, ctypes.byref(c), None, None, None, None, 0)
    pix = np.empty(m, np.uint32)
    zb = np.empty(m, np.uint32)
    ids = np.empty(m, np.uint32)
    w = np.empty(m, np.float64)
    m2 = L.orc_emit(_ptr(xyz), n, ctypes.byref(c), _ptr(pix), _ptr(zb), _ptr(ids), _ptr(w), m)
    assert m2 == m
    return pix, zb, ids, w


def fragments(xyz: np.ndarray, cam) -> Lists:
    """Per-pixel splat lists sorted by (depth bits, id)."""
    if xyz.shape[0] >= (1 << 30):
        raise ValueError("splat ids 4*p+corner must fit in 32 bits")
    pix, zb, ids, w = emit(xyz, cam)
    d = cam.as_dict() if hasattr(cam, "as_dict") else dict(cam)
    P = int(d["width"]) * int(d["height"])
    start = np.empty(P + 1, np.int64)
    s_zb = np.empty_like(zb)
    s_id = np.empty_like(ids)
    s_w = np.empty_like(w)
    rc = lib().orc_build_lists(P, pix.shape[0], _ptr(pix), _ptr(zb), _ptr(ids), _ptr(w),
                               _ptr(start), _ptr(s_zb), _ptr(s_id), _ptr(s_w))
    if rc != 0:
        raise RuntimeError("orc_build_lists failed")
    return Lists(P, start, s_zb, s_id, s_w, int(xyz.shape[0]))


def _feat(feat: np.ndarray):
    """float32 features, or bfloat16 given as their uint16 bit patterns."""
    if feat.dtype == np.uint16:
        return np.ascontiguousarray(feat), 1
    return np.ascontiguousarray(feat, np.float32), 0


def blend_forward(lists: Lists, opa: np.ndarray, feat: np.ndarray, tau: float,
                  n_override: Optional[np.ndarray] = None, want_t_after: bool = False):
    """Eq. 1 per pixel.  Returns dict(image [P,F] f64, t_final [P], n_blended [P] i32[, t_after])."""
    opa = np.ascontiguousarray(opa, np.float32)
    fb, is_bf16 = _feat(feat)
    F = int(fb.shape[1])
    image = np.empty((lists.P, F), np.float64)
    t_final = np.empty(lists.P, np.float64)
    nb = np.empty(lists.P, np.int32)
    t_after = np.empty(lists.m, np.float64) if want_t_after else None
    nov = None if n_override is None else np.ascontiguousarray(n_override, np.int32)
    lib().orc_blend_fwd(lists.P, _ptr(lists.start), _ptr(lists.ids), _ptr(lists.w), _ptr(opa),
                        _ptr(fb), is_bf16, F, float(tau), _ptr(nov), _ptr(image), _ptr(t_final),
                        _ptr(nb), _ptr(t_after))
    out = dict(image=image, t_final=t_final, n_blended=nb)
    if want_t_after:
        out["t_after"] = t_after
    return out


def blend_backward(lists: Lists, opa: np.ndarray, feat: np.ndarray, n_blended: np.ndarray,
                   g_img: np.ndarray, g_t: Optional[np.ndarray] = None):
    """Gradients of L = <g_img, image> + <g_t, t_final> w.r.t. features and opacities."""
    opa = np.ascontiguousarray(opa, np.float32)
    fb, is_bf16 = _feat(feat)
    F = int(fb.shape[1])
    N = int(opa.shape[0])
    g_img = np.ascontiguousarray(g_img, np.float32).reshape(lists.P, F)
    gt = None if g_t is None else np.ascontiguousarray(g_t, np.float32).reshape(lists.P)
    nb = np.ascontiguousarray(n_blended, np.int32)
    gf = np.empty((N, F), np.float64)
    go = np.empty(N, np.float64)
    rc = lib().orc_blend_bwd(lists.P, _ptr(lists.start), _ptr(lists.ids), _ptr(lists.w), _ptr(opa),
                             _ptr(fb), is_bf16, F, _ptr(nb), _ptr(g_img), _ptr(gt), N, _ptr(gf),
                             _ptr(go))
    if rc != 0:
        raise RuntimeError("orc_blend_bwd failed")
    return dict(grad_feat=gf, grad_opa=go)


def blend_weight(lists: Lists, opa: np.ndarray, n_blended: np.ndarray) -> np.ndarray:
    """Per-point blend weight b_p = sum_k w_k T_k alpha_k over the point's blended splats."""
    opa = np.ascontiguousarray(opa, np.float32)
    nb = np.ascontiguousarray(n_blended, np.int32)
    out = np.empty(opa.shape[0], np.float64)
    lib().orc_blend_weight(lists.P, _ptr(lists.start), _ptr(lists.ids), _ptr(lists.w), _ptr(opa), _ptr(nb),
                           opa.shape[0], _ptr(out))
    return out


def multisample(xyz, feat, opa, cam, offsets, counts, tau: float = 1e-4, want_samples: bool = False):
    """Multisampled inference (Section 3.2): cloud k = points [offsets[k], +counts[k])
    rendered for ``cam`` with Eq. 1, then per-pixel means of the K images and of
    the K final transmittances (FP64).  Returns dict(image [P,F], t_final [P][, samples])."""
    samples = []
    for o, c in zip(offsets, counts):
        sl = slice(int(o), int(o) + int(c))
        lists = fragments(np.ascontiguousarray(xyz[sl]), cam)
        r = blend_forward(lists, opa[sl], feat[sl], tau, want_t_after=want_samples)
        r["lists"] = lists
        samples.append(r)
    K = len(samples)
    image = sum(s["image"] for s in samples) / K
    t_final = sum(s["t_final"] for s in samples) / K
    out = dict(image=image, t_final=t_final)
    if want_samples:
        out["samples"] = samples
    return out


def render(xyz, feat, opa, cam, tau: float = 1e-4):
    """Convenience: lists + forward for one view; image reshaped to [H,W,F]."""
    lists = fragments(xyz, cam)
    out = blend_forward(lists, opa, feat, tau)
    d = cam.as_dict() if hasattr(cam, "as_dict") else dict(cam)
    H, W = int(d["height"]), int(d["width"])
    F = int(np.asarray(feat).shape[1])
    out["image"] = out["image"].reshape(H, W, F)
    out["t_final"] = out["t_final"].reshape(H, W)
    out["lists"] = lists
    return out
