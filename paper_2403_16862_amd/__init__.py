"""Python binding of the gfx950 bilinear point rasterizer (``libinpc_raster.so``).

Argument marshalling only: every step of the forward and backward pass runs
in the HIP kernels of the library (C ABI in ``include/inpc_raster.h``).
PyTorch provides device memory, the current HIP stream and autograd.  If the
library has not been built this module raises on first use; there is no
fallback path.

Entry points mirror the C ABI:

* ``rasterize(xyz, feat, opa, cam, t_threshold=1e-4, mode="save")`` -- one
  view, differentiable w.r.t. ``feat`` and ``opa`` (Algorithm 1 and the
  backward of Appendix A.6);
* ``rasterize_batched(xyz, feat, opa, views, ...)`` -- many views of uneven
  size and point count in one launch sequence, packed outputs;
* ``sum_view_grads`` -- fold per-view-point gradients onto shared points;
* ``autotune`` / ``load_tuning`` -- the tuning-table search;
* ``debug_fragments`` -- copy the sorted splat list of a forward to the host.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# INPC_RASTER_LIB selects another build of the same sources (the sanitizer
# test loads the build whose host code carries AddressSanitizer/UBSan)
LIB_PATH = os.environ.get("INPC_RASTER_LIB") or os.path.join(HERE, "libinpc_raster.so")

INPC_F32, INPC_BF16 = 0, 1
INPC_SAVE, INPC_RECOMPUTE = 0, 1
ERRORS = {0: "ok", -1: "EINVAL", -2: "EWORKSPACE", -3: "EUNSUPPORTED", -4: "EOVERFLOW", -5: "EHIP",
          -6: "ESCRATCH"}


class InpcError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        super().__init__(f"{what} failed: {ERRORS.get(code, code)}" + (f" ({detail})" if detail else ""))


class CCamera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("near_plane", ctypes.c_float), ("far_plane", ctypes.c_float)]


class CSettings(ctypes.Structure):
    _fields_ = [("t_threshold", ctypes.c_float), ("mode", ctypes.c_int32),
                ("tuning_id", ctypes.c_int32), ("flags", ctypes.c_int32)]


class CView(ctypes.Structure):
    _fields_ = [("cam", CCamera), ("point_offset", ctypes.c_int64),
                ("point_count", ctypes.c_int64), ("pixel_offset", ctypes.c_int64)]


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2403_16862_amd/build.py "
                           "(or __graft_entry__.build()); there is no non-HIP fallback")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    szp = ctypes.POINTER(ctypes.c_size_t)
    cam_p, set_p, view_p = ctypes.POINTER(CCamera), ctypes.POINTER(CSettings), ctypes.POINTER(CView)
    sig = {
        "inpc_plain_sizes": [i64, cam_p, i32, i32, i32, szp, szp, szp],
        "inpc_batched_sizes": [view_p, i32, i64, i32, i32, i32, szp, szp, szp],
        "inpc_rasterize_fwd": [P, P, i32, P, i64, i32, cam_p, set_p, P, P, P, P, sz, P, sz, P],
        "inpc_rasterize_bwd": [P, P, i32, P, i64, i32, cam_p, set_p, P, sz, P, P, P, P, P, P, sz, P],
        "inpc_rasterize_fwd_noalloc": [P, P, i32, P, i64, i32, cam_p, set_p, P, P, P, P],
        "inpc_rasterize_fwd_batched": [P, P, i32, P, i64, i32, view_p, i32, set_p, P, P, P, P, sz, P, sz,
                                       P],
        "inpc_rasterize_bwd_batched": [P, P, i32, P, i64, i32, view_p, i32, set_p, P, sz, P, P, P, P, P,
                                       P, sz, P],
        "inpc_sum_view_grads": [view_p, i32, i64, i32, P, P, P, P, P, sz, P],
        "inpc_multisample_sizes": [i64, cam_p, P, P, i32, i32, i32, szp],
        "inpc_appearance_fwd": [P, P, i64, view_p, i32, P, P, i32, P, sz, P],
        "inpc_sampling_sizes": [i64, szp],
        "inpc_sample_view": [P, P, P, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float, cam_p, i64,
                             ctypes.c_uint64, ctypes.c_uint64, i32, P, P, P, P, sz, P],
        "inpc_sample_global": [P, P, P, i64, ctypes.c_float, ctypes.c_float, i64, ctypes.c_uint64,
                               ctypes.c_uint64, P, P, P, sz, P],
        "inpc_update_probabilities": [P, P, i64, i64, ctypes.c_float, P, P, P, sz, P],
        "inpc_appearance_bwd": [P, P, i64, view_p, i32, P, P, P, P, sz, P],
        "inpc_multisample_fwd": [P, P, i32, P, i64, i32, cam_p, P, P, i32, set_p, P, P, P, sz, P],
        "inpc_tuning_count": [],
        "inpc_tuning_name": [i32],
        "inpc_autotune": [P, P, i32, P, i64, i32, view_p, i32, ctypes.c_float, P, P, P, sz, P, P, P, P, sz,
                          i32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_float), P],
        "inpc_autotune_load": [ctypes.c_char_p],
        "inpc_tuning_for": [view_p, i32, i64, i32, i32],
        "inpc_saved_tuning": [P],
        "inpc_debug_fragments": [view_p, i32, i64, i32, i32, P, sz, P, sz, P, P, i64,
                                 ctypes.POINTER(ctypes.c_int64), P, P],
        "inpc_state_info": [view_p, i32, i64, i32, i32, P, sz, ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_int32), P],
        "inpc_profile_stage_count": [],
        "inpc_profile_stage_name": [i32],
        "inpc_profile_begin": [],
        "inpc_profile_end": [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
        "inpc_error_string": [ctypes.c_int],
        "inpc_last_hip_error": [],
        "inpc_version": [],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.inpc_tuning_name.restype = ctypes.c_char_p
    L.inpc_profile_stage_name.restype = ctypes.c_char_p
    L.inpc_error_string.restype = ctypes.c_char_p
    L.inpc_last_hip_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc < 0:
        detail = lib().inpc_last_hip_error().decode() if rc == -5 else ""
        raise InpcError(rc, what, detail)
    return rc


# ------------------------------------------------------------------ marshalling
def c_camera(cam) -> CCamera:
    """From an object with R, t, fx, fy, cx, cy, width, height, near, far (or a dict)."""
    d = cam.as_dict() if hasattr(cam, "as_dict") else dict(cam)
    c = CCamera()
    R = [float(x) for x in (d["R"].reshape(-1) if hasattr(d["R"], "reshape") else d["R"])]
    t = [float(x) for x in (d["t"].reshape(-1) if hasattr(d["t"], "reshape") else d["t"])]
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = t[i]
    c.fx, c.fy, c.cx, c.cy = d["fx"], d["fy"], d["cx"], d["cy"]
    c.width, c.height = int(d["width"]), int(d["height"])
    c.near_plane = d.get("near", d.get("near_plane", 0.01))
    c.far_plane = d.get("far", d.get("far_plane", 100.0))
    return c


def c_views(cams: Sequence, point_offsets: Sequence[int], point_counts: Sequence[int]):
    arr = (CView * len(cams))()
    pix = 0
    for i, cam in enumerate(cams):
        arr[i].cam = c_camera(cam)
        arr[i].point_offset = int(point_offsets[i])
        arr[i].point_count = int(point_counts[i])
        arr[i].pixel_offset = pix
        pix += arr[i].cam.width * arr[i].cam.height
    return arr, pix


ATTR_PER_VIEW_POINT = 1   # settings flag: features / opacities indexed by view point


def c_settings(t_threshold: float, mode: int, tuning_id: int, flags: int = 0) -> CSettings:
    s = CSettings()
    s.t_threshold = float(t_threshold)
    s.mode = int(mode)
    s.tuning_id = int(tuning_id)
    s.flags = int(flags)
    return s


def _mode(mode) -> int:
    if isinstance(mode, str):
        return {"save": INPC_SAVE, "recompute": INPC_RECOMPUTE}[mode]
    return int(mode)


def _fdt(feat: torch.Tensor) -> int:
    if feat.dtype == torch.float32:
        return INPC_F32
    if feat.dtype == torch.bfloat16:
        return INPC_BF16
    raise TypeError(f"features must be float32 or bfloat16, got {feat.dtype}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _buffer(nbytes: int, device) -> torch.Tensor:
    """Device byte buffer whose data pointer is 256-byte aligned."""
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + max(int(nbytes), 1)]


def _check_points(xyz: torch.Tensor, feat: torch.Tensor, opa: torch.Tensor, n_attr=None):
    """n_attr: rows of feat / opa when they are indexed by view point (else N)."""
    if not (xyz.is_cuda and feat.is_cuda and opa.is_cuda):
        raise ValueError("xyz, feat and opa must be device tensors")
    if xyz.dtype != torch.float32 or opa.dtype != torch.float32:
        raise TypeError("xyz and opacity must be float32")
    if xyz.dim() != 2 or xyz.shape[1] != 3 or feat.dim() != 2 or opa.dim() != 1:
        raise ValueError("expected xyz [N,3], feat [N,F], opa [N]")
    rows = xyz.shape[0] if n_attr is None else n_attr
    if not (rows == feat.shape[0] == opa.shape[0]):
        raise ValueError("feat and opa must have one row per point (per view point with "
                         "attr_per_view_point)")


# ------------------------------------------------------------------ plain calls
def plain_sizes(n: int, cam, F: int, fdt: int, mode: int, ccam: Optional[CCamera] = None):
    a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    cc = ccam if ccam is not None else c_camera(cam)
    _check(lib().inpc_plain_sizes(int(n), ctypes.byref(cc), int(F), int(fdt), int(mode),
                                  ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "inpc_plain_sizes")
    return a.value, b.value, c.value


def batched_sizes(views, n_views: int, n_points: int, F: int, fdt: int, mode: int):
    a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().inpc_batched_sizes(views, int(n_views), int(n_points), int(F), int(fdt), int(mode),
                                    ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "inpc_batched_sizes")
    return a.value, b.value, c.value


@dataclass
class ForwardState:
    """What a forward leaves for its backward (and for debug_fragments)."""

    saved: torch.Tensor
    fwd_ws: Optional[torch.Tensor]
    settings: CSettings
    views: object
    n_views: int
    n_points: int
    F: int
    fdt: int
    plain: bool = False   # made by the plain one-view entry point (inpc_rasterize_fwd)


def rasterize_forward(xyz, feat, opa, cam, t_threshold: float = 1e-4, mode="save",
                      tuning_id: int = -1, keep_workspace: bool = False, blend_weight=None):
    """Forward only; returns (image [H,W,F], t_final [H,W], ForwardState).

    ``blend_weight``: optional float32 [N] device tensor that receives each
    point's blend weight (its splats' T*alpha summed with the bilinear
    weights as factors)."""
    _check_points(xyz, feat, opa)
    xyz, feat, opa = xyz.contiguous(), feat.contiguous(), opa.contiguous()
    cams = [cam]
    views, P = c_views(cams, [0], [xyz.shape[0]])
    return _forward(xyz, feat, opa, views, 1, t_threshold, mode, tuning_id, keep_workspace,
                    (views[0].cam.height, views[0].cam.width), blend_weight, plain=True)


def rasterize_forward_noalloc(xyz, feat, opa, cam, t_threshold: float = 1e-4, tuning_id: int = -1,
                              blend_weight=None):
    """Forward of one view through inpc_rasterize_fwd_noalloc (state and
    workspace in the library's fixed per-GPU scratch, no backward state);
    returns (image [H,W,F], t_final [H,W]).  Only the outputs are allocated
    here, by torch."""
    _check_points(xyz, feat, opa)
    xyz, feat, opa = xyz.contiguous(), feat.contiguous(), opa.contiguous()
    cc = c_camera(cam)
    F = int(feat.shape[1])
    dev = xyz.device
    image = torch.empty((cc.height, cc.width, F), dtype=torch.float32, device=dev)
    t_final = torch.empty((cc.height, cc.width), dtype=torch.float32, device=dev)
    views, _ = c_views([cam], [0], [xyz.shape[0]])
    _check_blend_weight(blend_weight, views, 1, dev)
    st = c_settings(t_threshold, INPC_RECOMPUTE, tuning_id)
    _check(lib().inpc_rasterize_fwd_noalloc(_ptr(xyz), _ptr(feat), _fdt(feat), _ptr(opa), int(xyz.shape[0]), F,
                                            ctypes.byref(cc), ctypes.byref(st), _ptr(image), _ptr(t_final),
                                            _ptr(blend_weight), _stream()), "inpc_rasterize_fwd_noalloc")
    return image, t_final


def rasterize_forward_batched(xyz, feat, opa, views, t_threshold: float = 1e-4, mode="save",
                              tuning_id: int = -1, keep_workspace: bool = False, blend_weight=None,
                              attr_per_view_point: bool = False):
    """Forward of a packed view table (``make_views``); returns packed
    (image [sum P, F], t_final [sum P], ForwardState).  ``blend_weight``:
    optional float32 tensor with one entry per view point."""
    _check_points(xyz, feat, opa, _n_vp(views) if attr_per_view_point else None)
    xyz, feat, opa = xyz.contiguous(), feat.contiguous(), opa.contiguous()
    return _forward(xyz, feat, opa, views, len(views), t_threshold, mode, tuning_id, keep_workspace, None,
                    blend_weight, ATTR_PER_VIEW_POINT if attr_per_view_point else 0)


def _check_blend_weight(bw, views, n_views, dev):
    if bw is None:
        return
    nvp = sum(int(views[i].point_count) for i in range(n_views))
    if (bw.dtype != torch.float32 or bw.numel() != nvp or not bw.is_contiguous()
            or bw.device != dev):
        raise ValueError("blend_weight must be a contiguous float32 tensor with one entry per "
                         "view point, on the points' device")


def _forward(xyz, feat, opa, views, n_views, t_threshold, mode, tuning_id, keep_workspace, img_hw,
             blend_weight=None, flags: int = 0, plain: bool = False):
    """plain: one camera over all points (views[0]), through the plain entry
    points inpc_rasterize_fwd / inpc_rasterize_bwd; else the batched ones."""
    m = _mode(mode)
    fdt = _fdt(feat)
    F = int(feat.shape[1])
    N = int(xyz.shape[0])
    if plain:
        assert n_views == 1 and flags == 0 and views[0].point_offset == 0 and views[0].point_count == N
        fws, sv, _ = plain_sizes(N, None, F, fdt, m, ccam=views[0].cam)
    else:
        fws, sv, _ = batched_sizes(views, n_views, N, F, fdt, m)
    dev = xyz.device
    saved = _buffer(sv, dev)
    ws = _buffer(fws, dev)
    P = sum(views[i].cam.width * views[i].cam.height for i in range(n_views))
    if img_hw is not None:
        image = torch.empty((img_hw[0], img_hw[1], F), dtype=torch.float32, device=dev)
        t_final = torch.empty(img_hw, dtype=torch.float32, device=dev)
    else:
        image = torch.empty((P, F), dtype=torch.float32, device=dev)
        t_final = torch.empty((P,), dtype=torch.float32, device=dev)
    st = c_settings(t_threshold, m, tuning_id, flags)
    _check_blend_weight(blend_weight, views, n_views, dev)
    if plain:
        _check(lib().inpc_rasterize_fwd(_ptr(xyz), _ptr(feat), fdt, _ptr(opa), N, F, ctypes.byref(views[0].cam),
                                        ctypes.byref(st), _ptr(image), _ptr(t_final), _ptr(blend_weight),
                                        _ptr(saved), saved.numel(), _ptr(ws), ws.numel(), _stream()),
               "inpc_rasterize_fwd")
    else:
        _check(lib().inpc_rasterize_fwd_batched(_ptr(xyz), _ptr(feat), fdt, _ptr(opa), N, F, views, n_views,
                                                ctypes.byref(st), _ptr(image), _ptr(t_final),
                                                _ptr(blend_weight), _ptr(saved), saved.numel(), _ptr(ws),
                                                ws.numel(), _stream()),
               "inpc_rasterize_fwd_batched")
    # the backward reads the state with the tuning this forward used
    st.tuning_id = _check(lib().inpc_saved_tuning(_ptr(saved)), "inpc_saved_tuning")
    state = ForwardState(saved, ws if keep_workspace else None, st, views, n_views, N, F, fdt, plain)
    return image, t_final, state


def rasterize_backward(xyz, feat, opa, state: ForwardState, g_img, g_t=None, blend_weight=None):
    """Backward of a forward; returns float32 (grad_feat, grad_opa) per view point.
    ``blend_weight``: optional float32 tensor (one entry per view point) that
    receives the per-point blend weights, computed from the backward's records."""
    g_img = g_img.contiguous().float()
    g_t = None if g_t is None else g_t.contiguous().float()
    nvp = sum(int(state.views[i].point_count) for i in range(state.n_views))
    if state.plain:
        _, _, bws = plain_sizes(state.n_points, None, state.F, state.fdt, state.settings.mode,
                                ccam=state.views[0].cam)
    else:
        _, _, bws = batched_sizes(state.views, state.n_views, state.n_points, state.F, state.fdt,
                                  state.settings.mode)
    dev = xyz.device
    ws = _buffer(bws, dev)
    gf = torch.empty((nvp, state.F), dtype=torch.float32, device=dev)
    go = torch.empty((nvp,), dtype=torch.float32, device=dev)
    _check_blend_weight(blend_weight, state.views, state.n_views, dev)
    if state.plain:
        _check(lib().inpc_rasterize_bwd(_ptr(xyz), _ptr(feat), state.fdt, _ptr(opa), state.n_points, state.F,
                                        ctypes.byref(state.views[0].cam), ctypes.byref(state.settings),
                                        _ptr(state.saved), state.saved.numel(), _ptr(g_img), _ptr(g_t),
                                        _ptr(gf), _ptr(go), _ptr(blend_weight), _ptr(ws), ws.numel(),
                                        _stream()),
               "inpc_rasterize_bwd")
    else:
        _check(lib().inpc_rasterize_bwd_batched(_ptr(xyz), _ptr(feat), state.fdt, _ptr(opa), state.n_points,
                                                state.F, state.views, state.n_views,
                                                ctypes.byref(state.settings), _ptr(state.saved),
                                                state.saved.numel(), _ptr(g_img), _ptr(g_t), _ptr(gf),
                                                _ptr(go), _ptr(blend_weight), _ptr(ws), ws.numel(), _stream()),
               "inpc_rasterize_bwd_batched")
    return gf, go


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, feat, opa, views, n_views, img_hw, t_threshold, mode, tuning_id, fold, flags,
                plain=False):
        image, t_final, state = _forward(xyz, feat, opa, views, n_views, t_threshold, mode, tuning_id,
                                         False, img_hw, None, flags, plain)
        ctx.state = state
        ctx.fold = fold
        ctx.set_materialize_grads(False)
        ctx.save_for_backward(xyz, feat, opa)
        return image, t_final

    @staticmethod
    def backward(ctx, g_img, g_t):
        xyz, feat, opa = ctx.saved_tensors
        st = ctx.state
        if g_img is None and g_t is None:
            return (None,) * 12
        if g_img is None:
            P = sum(st.views[i].cam.width * st.views[i].cam.height for i in range(st.n_views))
            g_img = torch.zeros((P, st.F), dtype=torch.float32, device=xyz.device)
        gf, go = rasterize_backward(xyz, feat, opa, st, g_img, g_t)
        if ctx.fold:
            gf, go = sum_view_grads(st.views, st.n_views, st.n_points, gf, go)
        return None, gf, go, None, None, None, None, None, None, None, None, None


def rasterize(xyz, feat, opa, cam, t_threshold: float = 1e-4, mode="save", tuning_id: int = -1):
    """Differentiable rasterization of one view -> (image [H,W,F], t_final [H,W])."""
    _check_points(xyz, feat, opa)
    xyz, feat, opa = xyz.contiguous(), feat.contiguous(), opa.contiguous()
    views, _ = c_views([cam], [0], [xyz.shape[0]])
    hw = (views[0].cam.height, views[0].cam.width)
    return _Rasterize.apply(xyz, feat, opa, views, 1, hw, t_threshold, mode, tuning_id, False, 0, True)


def make_views(cams: Sequence, point_offsets: Sequence[int], point_counts: Sequence[int]):
    """C view table for the batched calls (views packed in order)."""
    views, _ = c_views(cams, point_offsets, point_counts)
    return views


def _is_identity_layout(views, n_views, n_points) -> bool:
    off = 0
    for i in range(n_views):
        if views[i].point_offset != off:
            return False
        off += views[i].point_count
    return off == n_points


def rasterize_batched(xyz, feat, opa, views, t_threshold: float = 1e-4, mode="save",
                      tuning_id: int = -1, attr_per_view_point: bool = False):
    """Differentiable batched rasterization -> packed (image [sum P,F], t_final [sum P]).

    ``views`` comes from ``make_views``.  Gradients w.r.t. feat/opa are folded
    onto the points (views sharing points are summed in view order).  With
    ``attr_per_view_point`` feat and opa hold one row per view point (views
    in order) and their gradients keep that layout."""
    _check_points(xyz, feat, opa, _n_vp(views) if attr_per_view_point else None)
    xyz, feat, opa = xyz.contiguous(), feat.contiguous(), opa.contiguous()
    n_views = len(views)
    flags = ATTR_PER_VIEW_POINT if attr_per_view_point else 0
    fold = not attr_per_view_point and not _is_identity_layout(views, n_views, xyz.shape[0])
    return _Rasterize.apply(xyz, feat, opa, views, n_views, None, t_threshold, mode, tuning_id, fold, flags)


def sum_view_grads(views, n_views: int, n_points: int, vg_feat, vg_opa):
    F = int(vg_feat.shape[1])
    dev = vg_feat.device
    gf = torch.empty((n_points, F), dtype=torch.float32, device=dev)
    go = torch.empty((n_points,), dtype=torch.float32, device=dev)
    ws = _buffer(256 * n_views, dev)
    _check(lib().inpc_sum_view_grads(views, n_views, int(n_points), F, _ptr(vg_feat.contiguous()),
                                     _ptr(vg_opa.contiguous()), _ptr(gf), _ptr(go), _ptr(ws), ws.numel(),
                                     _stream()), "inpc_sum_view_grads")
    return gf, go


# ---------------------------------------------------------------- appearance
N_RAW = 37   # opacity logit + 9 SH basis functions x 4 channels


def _n_vp(views) -> int:
    return sum(int(views[i].point_count) for i in range(len(views)))


def appearance_forward(xyz, raw, views, feat_dtype=torch.float32):
    """Opacity activation and degree-2 SH features per view point:
    returns (opacity [n_vp] f32, feat [n_vp, 4] in ``feat_dtype``)."""
    if raw.dtype != torch.float32 or raw.dim() != 2 or raw.shape[1] != N_RAW:
        raise TypeError("raw must be float32 [N, 37]")
    if xyz.dtype != torch.float32 or not (xyz.is_cuda and raw.is_cuda):
        raise TypeError("xyz and raw must be float32 device tensors")
    xyz, raw = xyz.contiguous(), raw.contiguous()
    n = _n_vp(views)
    dev = xyz.device
    opa = torch.empty((n,), dtype=torch.float32, device=dev)
    feat = torch.empty((n, 4), dtype=feat_dtype, device=dev)
    ws = _buffer(256 * len(views), dev)
    _check(lib().inpc_appearance_fwd(_ptr(xyz), _ptr(raw), int(xyz.shape[0]), views, len(views), _ptr(opa),
                                     _ptr(feat), _fdt(feat), _ptr(ws), ws.numel(), _stream()),
           "inpc_appearance_fwd")
    return opa, feat


def appearance_backward(xyz, raw, views, g_opa, g_feat):
    """Gradient of the raw rows [N, 37] (view points of a point summed in view order)."""
    xyz, raw = xyz.contiguous(), raw.contiguous()
    dev = xyz.device
    n = _n_vp(views)
    g_opa = (torch.zeros((n,), dtype=torch.float32, device=dev) if g_opa is None
             else g_opa.contiguous().float())
    g_feat = (torch.zeros((n, 4), dtype=torch.float32, device=dev) if g_feat is None
              else g_feat.contiguous().float())
    grad = torch.empty((xyz.shape[0], N_RAW), dtype=torch.float32, device=dev)
    ws = _buffer(256 * len(views), dev)
    _check(lib().inpc_appearance_bwd(_ptr(xyz), _ptr(raw), int(xyz.shape[0]), views, len(views),
                                     _ptr(g_opa), _ptr(g_feat), _ptr(grad), _ptr(ws), ws.numel(), _stream()),
           "inpc_appearance_bwd")
    return grad


class _Appearance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, raw, views):
        opa, feat = appearance_forward(xyz, raw, views)
        ctx.views = views
        ctx.save_for_backward(xyz, raw)
        ctx.set_materialize_grads(False)
        return opa, feat

    @staticmethod
    def backward(ctx, g_opa, g_feat):
        xyz, raw = ctx.saved_tensors
        if g_opa is None and g_feat is None:
            return None, None, None
        return None, appearance_backward(xyz, raw, ctx.views, g_opa, g_feat), None


def appearance(xyz, raw, views):
    """Differentiable appearance step -> (opacity [n_vp], feat [n_vp, 4]) in float32."""
    return _Appearance.apply(xyz, raw, views)


class _ShRaster(torch.autograd.Function):
    """Appearance step fused with the batched rasterizer: gradients flow from
    the image to the raw rows in float32 even when the features are stored as
    bfloat16."""

    @staticmethod
    def forward(ctx, xyz, raw, views, t_threshold, mode, tuning_id, feat_dtype, blend_weight, bw_in_backward):
        opa, feat = appearance_forward(xyz, raw, views, feat_dtype)
        image, t_final, state = _forward(xyz, feat, opa, views, len(views), t_threshold, mode, tuning_id,
                                         False, None, None if bw_in_backward else blend_weight,
                                         ATTR_PER_VIEW_POINT)
        ctx.bw = blend_weight if bw_in_backward else None
        ctx.state = state
        ctx.views = views
        ctx.save_for_backward(xyz, raw, feat, opa)
        ctx.set_materialize_grads(False)
        return image, t_final

    @staticmethod
    def backward(ctx, g_img, g_t):
        xyz, raw, feat, opa = ctx.saved_tensors
        if g_img is None and g_t is None:
            return (None,) * 9
        st = ctx.state
        if g_img is None:
            P = sum(st.views[i].cam.width * st.views[i].cam.height for i in range(st.n_views))
            g_img = torch.zeros((P, st.F), dtype=torch.float32, device=xyz.device)
        gf, go = rasterize_backward(xyz, feat, opa, st, g_img, g_t, ctx.bw)
        return None, appearance_backward(xyz, raw, ctx.views, go, gf), None, None, None, None, None, None, None


def render_sh(xyz, raw, views, t_threshold: float = 1e-4, mode="save", tuning_id: int = -1,
              feat_dtype=torch.float32, blend_weight=None, blend_weight_in_backward: bool = False):
    """Appearance step (opacity activation + degree-2 SH, per view point) then
    batched rasterization -> packed (image [sum P, 4], t_final [sum P]);
    differentiable with respect to ``raw`` [N, 37].  ``blend_weight``: optional
    float32 tensor (one entry per view point) that receives the per-point
    blend weights, written by the forward or (cheaper, for training) by the
    backward when ``blend_weight_in_backward``."""
    if xyz.dtype != torch.float32 or not xyz.is_cuda:
        raise TypeError("xyz must be a float32 device tensor")
    return _ShRaster.apply(xyz.contiguous(), raw.contiguous(), views, t_threshold, mode, tuning_id, feat_dtype,
                           blend_weight, bool(blend_weight_in_backward))


# ---------------------------------------------------------------- octree sampling
class OctreeLeaves:
    """Device arrays of a probability octree's leaves (centre [L,3] f32, level [L] int32,
    prob [L] f32, subdiv [L] f32) and the edge length of a level-0 cube."""

    def __init__(self, centre, level, prob, subdiv, root_size: float):
        self.centre = centre.contiguous().float()
        self.level = level.contiguous().to(torch.int32)
        self.prob = prob.contiguous().float()
        self.subdiv = subdiv.contiguous().float()
        self.root_size = float(root_size)
        self.n = int(self.level.shape[0])
        need = ctypes.c_size_t(0)
        _check(lib().inpc_sampling_sizes(self.n, ctypes.byref(need)), "inpc_sampling_sizes")
        self.ws = _buffer(need.value, self.centre.device)


def sample_view(tree: OctreeLeaves, cam, n_samples: int, seed=(0, 0), lambda_l: float = 0.5,
                tau_d: float = 1e-8, max_rounds: int = 64):
    """Viewpoint-specific samples -> (xyz [n,3], leaf [n] int32, unresolved count tensor [1] int64)."""
    dev = tree.centre.device
    xyz = torch.empty((n_samples, 3), dtype=torch.float32, device=dev)
    leaf = torch.empty((n_samples,), dtype=torch.int32, device=dev)
    unres = torch.empty((1,), dtype=torch.int64, device=dev)
    c = c_camera(cam)
    _check(lib().inpc_sample_view(_ptr(tree.centre), _ptr(tree.level), _ptr(tree.prob), tree.n, tree.root_size,
                                  float(lambda_l), float(tau_d), ctypes.byref(c), int(n_samples),
                                  int(seed[0]), int(seed[1]), int(max_rounds), _ptr(xyz), _ptr(leaf), _ptr(unres),
                                  _ptr(tree.ws), tree.ws.numel(), _stream()), "inpc_sample_view")
    return xyz, leaf, unres


def sample_global(tree: OctreeLeaves, n_samples: int, seed=(0, 0), lambda_l: float = 0.5):
    """Viewpoint-independent extraction -> (xyz [n,3] ordered by leaf, leaf [n] int32)."""
    dev = tree.centre.device
    xyz = torch.empty((n_samples, 3), dtype=torch.float32, device=dev)
    leaf = torch.empty((n_samples,), dtype=torch.int32, device=dev)
    _check(lib().inpc_sample_global(_ptr(tree.centre), _ptr(tree.level), _ptr(tree.prob), tree.n, tree.root_size,
                                    float(lambda_l), int(n_samples), int(seed[0]), int(seed[1]), _ptr(xyz),
                                    _ptr(leaf), _ptr(tree.ws), tree.ws.numel(), _stream()), "inpc_sample_global")
    return xyz, leaf


def update_probabilities(tree: OctreeLeaves, leaf, blend_weight, lambda_u: float = 0.9968):
    """Eq. 2 and Eq. 3 on tree.prob / tree.subdiv in place, from per-point leaves and blend weights."""
    leaf = leaf.contiguous().to(torch.int32)
    bw = blend_weight.contiguous().float()
    if leaf.numel() != bw.numel():
        raise ValueError("one leaf index per blend weight")
    _check(lib().inpc_update_probabilities(_ptr(leaf), _ptr(bw), int(leaf.numel()), tree.n, float(lambda_u),
                                           _ptr(tree.prob), _ptr(tree.subdiv), _ptr(tree.ws), tree.ws.numel(),
                                           _stream()), "inpc_update_probabilities")


# ---------------------------------------------------------------- multisampling
def multisample(xyz, feat, opa, cam, cloud_offsets: Sequence[int], cloud_counts: Sequence[int],
                t_threshold: float = 1e-4, tuning_id: int = -1):
    """Renders K point clouds (ranges of the point arrays) for one camera and
    returns the per-pixel means (image [H,W,F], t_final [H,W])."""
    _check_points(xyz, feat, opa)
    xyz, feat, opa = xyz.contiguous(), feat.contiguous(), opa.contiguous()
    K = len(cloud_offsets)
    if K != len(cloud_counts) or K < 1:
        raise ValueError("need one offset and one count per cloud")
    off = (ctypes.c_int64 * K)(*[int(o) for o in cloud_offsets])
    cnt = (ctypes.c_int64 * K)(*[int(c) for c in cloud_counts])
    c = c_camera(cam)
    F, fdt, N = int(feat.shape[1]), _fdt(feat), int(xyz.shape[0])
    need = ctypes.c_size_t(0)
    _check(lib().inpc_multisample_sizes(N, ctypes.byref(c), off, cnt, K, F, fdt, ctypes.byref(need)),
           "inpc_multisample_sizes")
    dev = xyz.device
    ws = _buffer(need.value, dev)
    image = torch.empty((c.height, c.width, F), dtype=torch.float32, device=dev)
    t_final = torch.empty((c.height, c.width), dtype=torch.float32, device=dev)
    st = c_settings(t_threshold, 1, tuning_id)
    _check(lib().inpc_multisample_fwd(_ptr(xyz), _ptr(feat), fdt, _ptr(opa), N, F, ctypes.byref(c), off, cnt,
                                      K, ctypes.byref(st), _ptr(image), _ptr(t_final), _ptr(ws), ws.numel(),
                                      _stream()), "inpc_multisample_fwd")
    return image, t_final


# ---------------------------------------------------------------- tuning, debug
def tuning_table() -> List[str]:
    L = lib()
    return [L.inpc_tuning_name(i).decode() for i in range(L.inpc_tuning_count())]


def load_tuning(path: str) -> int:
    return _check(lib().inpc_autotune_load(path.encode()), "inpc_autotune_load")


def autotune(xyz, feat, opa, views, t_threshold: float = 1e-4, g_img=None, repeats: int = 3,
             cache_path: Optional[str] = None):
    """Time every tuning-table entry on this problem; returns (best id, ms per call)."""
    n_views = len(views)
    N, F, fdt = int(xyz.shape[0]), int(feat.shape[1]), _fdt(feat)
    fws, sv, bws = batched_sizes(views, n_views, N, F, fdt, INPC_SAVE)
    dev = xyz.device
    saved = _buffer(sv, dev)
    ws = _buffer(max(fws, bws), dev)
    P = sum(views[i].cam.width * views[i].cam.height for i in range(n_views))
    nvp = sum(int(views[i].point_count) for i in range(n_views))
    image = torch.empty((P, F), dtype=torch.float32, device=dev)
    t_final = torch.empty((P,), dtype=torch.float32, device=dev)
    gf = torch.empty((nvp, F), dtype=torch.float32, device=dev)
    go = torch.empty((nvp,), dtype=torch.float32, device=dev)
    ms = ctypes.c_float()
    g = None if g_img is None else g_img.contiguous().float()
    best = _check(lib().inpc_autotune(_ptr(xyz), _ptr(feat), fdt, _ptr(opa), N, F, views, n_views,
                                      float(t_threshold), _ptr(image), _ptr(t_final), _ptr(saved),
                                      saved.numel(), _ptr(g), _ptr(gf), _ptr(go), _ptr(ws), ws.numel(),
                                      int(repeats), cache_path.encode() if cache_path else None,
                                      ctypes.byref(ms), _stream()), "inpc_autotune")
    return best, ms.value


def debug_fragments(state: ForwardState):
    """Sorted (keys uint64, ids uint32) and n_blended per pixel of a SAVE-mode forward
    made with keep_workspace=True."""
    import numpy as np
    if state.fwd_ws is None:
        raise ValueError("forward must be called with keep_workspace=True")
    m = ctypes.c_int64()
    P = sum(state.views[i].cam.width * state.views[i].cam.height for i in range(state.n_views))
    nb = np.empty(P, np.uint32)
    L = lib()
    _check(L.inpc_debug_fragments(state.views, state.n_views, state.n_points, state.F, state.fdt,
                                  _ptr(state.saved), state.saved.numel(), _ptr(state.fwd_ws),
                                  state.fwd_ws.numel(), None, None, 0, ctypes.byref(m),
                                  nb.ctypes.data_as(ctypes.c_void_p), _stream()), "inpc_debug_fragments")
    keys = np.empty(m.value, np.uint64)
    ids = np.empty(m.value, np.uint32)
    _check(L.inpc_debug_fragments(state.views, state.n_views, state.n_points, state.F, state.fdt,
                                  _ptr(state.saved), state.saved.numel(), _ptr(state.fwd_ws),
                                  state.fwd_ws.numel(), keys.ctypes.data_as(ctypes.c_void_p),
                                  ids.ctypes.data_as(ctypes.c_void_p), m.value, ctypes.byref(m), None,
                                  _stream()), "inpc_debug_fragments")
    return keys, ids, nb


def state_info(state: ForwardState):
    """(stored list items, layout): splats and 0 for per-pixel lists, tile
    entries and the tile blend shape (5: 16x16, 6: 8x8) for tile lists."""
    items, layout = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().inpc_state_info(state.views, state.n_views, state.n_points, state.F, state.fdt, _ptr(state.saved),
                                 state.saved.numel(), ctypes.byref(items), ctypes.byref(layout), _stream()),
           "inpc_state_info")
    return int(items.value), int(layout.value)


# --------------------------------------------------------------- stage timing
def profile_begin():
    _check(lib().inpc_profile_begin(), "inpc_profile_begin")


def profile_end():
    """{stage name: (total ms, timed launches)} since profile_begin()."""
    L = lib()
    n = L.inpc_profile_stage_count()
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(L.inpc_profile_end(ms, cnt), "inpc_profile_end")
    return {L.inpc_profile_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(n)}


def fragment_count(state: ForwardState) -> int:
    """Number of splats the forward emitted (synchronises the stream)."""
    m = ctypes.c_int64()
    ws = state.fwd_ws
    _check(lib().inpc_debug_fragments(state.views, state.n_views, state.n_points, state.F, state.fdt,
                                      _ptr(state.saved), state.saved.numel(),
                                      _ptr(ws), ws.numel() if ws is not None else 0, None, None, 0,
                                      ctypes.byref(m), None, _stream()), "fragment_count")
    return int(m.value)


# ------------------------------------------------ batched step with HIP graphs
class BatchedStep:
    """Forward + backward of many views on static device buffers.

    ``run()`` enqueues the batched forward and backward eagerly; ``capture()``
    records the same launch sequence once into a HIP graph (through
    torch.cuda.CUDAGraph) and ``replay()`` relaunches it.  No allocation,
    host synchronisation or memset happens inside the step, so the recorded
    graph is replayable; inputs are read from and outputs written to the
    tensors given at construction.
    """

    def __init__(self, xyz, feat, opa, views, g_img, t_threshold: float = 1e-4, mode="save",
                 tuning_id: int = -1, g_t=None, want_blend_weight: bool = False,
                 attr_per_view_point: bool = False):
        self.xyz, self.feat, self.opa = xyz.contiguous(), feat.contiguous(), opa.contiguous()
        self.views = views
        self.n_views = len(views)
        self.N, self.F, self.fdt = int(xyz.shape[0]), int(feat.shape[1]), _fdt(feat)
        m = _mode(mode)
        self.settings = c_settings(t_threshold, m, tuning_id,
                                   ATTR_PER_VIEW_POINT if attr_per_view_point else 0)
        fws, sv, bws = batched_sizes(views, self.n_views, self.N, self.F, self.fdt, m)
        dev = xyz.device
        self.saved = _buffer(sv, dev)
        self.fwd_ws = _buffer(fws, dev)
        self.bwd_ws = _buffer(bws, dev)
        self.P = sum(views[i].cam.width * views[i].cam.height for i in range(self.n_views))
        self.nvp = sum(int(views[i].point_count) for i in range(self.n_views))
        self.image = torch.empty((self.P, self.F), dtype=torch.float32, device=dev)
        self.t_final = torch.empty((self.P,), dtype=torch.float32, device=dev)
        self.g_img = g_img.contiguous().float()
        self.g_t = None if g_t is None else g_t.contiguous().float()
        self.grad_feat = torch.empty((self.nvp, self.F), dtype=torch.float32, device=dev)
        self.grad_opa = torch.empty((self.nvp,), dtype=torch.float32, device=dev)
        self.blend_weight = (torch.empty((self.nvp,), dtype=torch.float32, device=dev)
                             if want_blend_weight else None)
        self.graph = None

    def forward(self):
        _check(lib().inpc_rasterize_fwd_batched(
            _ptr(self.xyz), _ptr(self.feat), self.fdt, _ptr(self.opa), self.N, self.F, self.views,
            self.n_views, ctypes.byref(self.settings), _ptr(self.image), _ptr(self.t_final),
            None, _ptr(self.saved), self.saved.numel(), _ptr(self.fwd_ws),
            self.fwd_ws.numel(), _stream()),
            "inpc_rasterize_fwd_batched")

    def backward(self):
        _check(lib().inpc_rasterize_bwd_batched(
            _ptr(self.xyz), _ptr(self.feat), self.fdt, _ptr(self.opa), self.N, self.F, self.views,
            self.n_views, ctypes.byref(self.settings), _ptr(self.saved), self.saved.numel(),
            _ptr(self.g_img), _ptr(self.g_t), _ptr(self.grad_feat), _ptr(self.grad_opa),
            _ptr(self.blend_weight), _ptr(self.bwd_ws), self.bwd_ws.numel(), _stream()),
            "inpc_rasterize_bwd_batched")

    def run(self):
        self.forward()
        self.backward()

    def capture(self):
        """Record forward + backward into a HIP graph (after one eager warm-up run)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        torch.cuda.synchronize()
        return self

    def replay(self):
        self.graph.replay()

    def state(self) -> ForwardState:
        return ForwardState(self.saved, self.fwd_ws, self.settings, self.views, self.n_views, self.N,
                            self.F, self.fdt)
