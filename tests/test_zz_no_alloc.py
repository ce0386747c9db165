"""The no-allocation forward (inpc_rasterize_fwd_noalloc: state and
workspace in the library's fixed per-GPU scratch array) against the plain
forward (inpc_rasterize_fwd with caller buffers), through the C ABI, on two
calls in a row, the second with a smaller input: 1M points at 1280x720 with
F=8, then 4,096 points at 128x128 with F=4.  Both calls run the same kernels,
so images, transmittances and blend weights must be equal bit for bit; the
small call is also checked against the FP64 oracle."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2403_16862_amd as pr
import workloads
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _noalloc(x, f, o, cam, bw):
    c = pr.c_camera(cam)
    st = pr.c_settings(1e-4, pr.INPC_RECOMPUTE, -1)
    F = int(f.shape[1])
    img = torch.full((c.height, c.width, F), float("nan"), dtype=torch.float32, device=H.DEV)
    tf = torch.full((c.height, c.width), float("nan"), dtype=torch.float32, device=H.DEV)
    rc = pr.lib().inpc_rasterize_fwd_noalloc(pr._ptr(x), pr._ptr(f), pr._fdt(f), pr._ptr(o), int(x.shape[0]), F,
                                             ctypes.byref(c), ctypes.byref(st), pr._ptr(img), pr._ptr(tf),
                                             pr._ptr(bw), pr._stream())
    assert rc == 0, pr.lib().inpc_error_string(rc)
    return img, tf


def _plain(x, f, o, cam, bw):
    c = pr.c_camera(cam)
    st = pr.c_settings(1e-4, pr.INPC_RECOMPUTE, -1)
    F = int(f.shape[1])
    fws, sv, _ = pr.plain_sizes(int(x.shape[0]), cam, F, pr._fdt(f), pr.INPC_RECOMPUTE)
    saved, ws = pr._buffer(sv, H.DEV), pr._buffer(fws, H.DEV)
    img = torch.empty((c.height, c.width, F), dtype=torch.float32, device=H.DEV)
    tf = torch.empty((c.height, c.width), dtype=torch.float32, device=H.DEV)
    rc = pr.lib().inpc_rasterize_fwd(pr._ptr(x), pr._ptr(f), pr._fdt(f), pr._ptr(o), int(x.shape[0]), F,
                                     ctypes.byref(c), ctypes.byref(st), pr._ptr(img), pr._ptr(tf), pr._ptr(bw),
                                     pr._ptr(saved), saved.numel(), pr._ptr(ws), ws.numel(), pr._stream())
    assert rc == 0, pr.lib().inpc_error_string(rc)
    return img, tf


def test_noalloc_forward_equals_plain_forward_on_two_calls():
    for label, s in (("1M points, 1280x720, F=8", workloads.config2()),
                     ("4096 points, 128x128, F=4", workloads.config1())):
        H.say(f"  no-allocation forward: {label}")
        x, f, o = H.to_dev(s.xyz), H.to_dev(s.feat), H.to_dev(s.opa)
        bw_n = torch.full((s.n,), float("nan"), dtype=torch.float32, device=H.DEV)
        bw_p = torch.empty((s.n,), dtype=torch.float32, device=H.DEV)
        img_n, tf_n = _noalloc(x, f, o, s.cam, bw_n)
        img_p, tf_p = _plain(x, f, o, s.cam, bw_p)
        torch.cuda.synchronize()
        assert torch.equal(img_n, img_p), label
        assert torch.equal(tf_n, tf_p), label
        assert torch.equal(bw_n, bw_p), label
    # the small call against the oracle as well
    L = oracle.fragments(s.xyz, s.cam)
    ref = oracle.blend_forward(L, s.opa, s.feat, 1e-4)
    e = H.rel_err(img_n.reshape(-1, s.F).cpu().numpy(), ref["image"]).max()
    et = H.rel_err(tf_n.reshape(-1).cpu().numpy(), ref["t_final"]).max()
    assert e <= H.REL_TOL and et <= H.REL_TOL, (e, et)
    H.say(f"    equal to the plain forward bit for bit; small call vs oracle: image {e:.2e}, t_final {et:.2e}")
