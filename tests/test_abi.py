"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, answers size queries, and rejects bad arguments on the host
before anything is enqueued."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2403_16862_amd as pr
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "inpc_raster.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(inpc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = pr.lib()
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s


def test_version_and_error_strings():
    L = pr.lib()
    assert L.inpc_version() >= 1
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.inpc_error_string(code)
    assert L.inpc_error_string(-6) != L.inpc_error_string(-99)


def test_tuning_table_is_listed():
    names = pr.tuning_table()
    assert len(names) >= 4 and all(names)


def cam(W=64, H=48):
    return workloads.canonical_camera(W, H)


def test_sizes_scale_with_points_and_pixels():
    a = pr.plain_sizes(1000, cam(), 8, pr.INPC_F32, pr.INPC_SAVE)
    b = pr.plain_sizes(4000, cam(), 8, pr.INPC_F32, pr.INPC_SAVE)
    c = pr.plain_sizes(1000, cam(128, 96), 8, pr.INPC_F32, pr.INPC_SAVE)
    assert all(x > 0 for x in a)
    assert b[0] > a[0] and b[1] > a[1] and b[2] > a[2]
    assert c[1] > a[1]
    r = pr.plain_sizes(1000, cam(), 8, pr.INPC_F32, pr.INPC_RECOMPUTE)
    assert r[1] < a[1]          # recompute keeps only per-pixel state
    assert r[2] > a[2]          # and rebuilds the fragment lists in the backward


def test_sizes_zero_points():
    a = pr.plain_sizes(0, cam(), 4, pr.INPC_F32, pr.INPC_SAVE)
    assert a[1] > 0


def _call_sizes(n=10, F=4, fdt=0, mode=0, c=None):
    cc = pr.c_camera(c or cam())
    x = ctypes.c_size_t()
    return pr.lib().inpc_plain_sizes(n, ctypes.byref(cc), F, fdt, mode, ctypes.byref(x), None, None)


@pytest.mark.parametrize("kw,code", [
    (dict(F=0), -3), (dict(F=65), -3), (dict(fdt=2), -1), (dict(mode=3), -1), (dict(n=-1), -1),
    (dict(n=1 << 28), -4),
])
def test_size_query_rejects(kw, code):
    assert _call_sizes(**kw) == code


def test_camera_validation():
    c = cam()
    bad = [dict(width=0), dict(width=20000), dict(height=-3), dict(near=2.0, far=1.0),
           dict(near=-0.5), dict(fx=float("nan")), dict(far=float("nan"))]
    for b in bad:
        d = c.as_dict()
        d.update(b)
        rc = _call_sizes(c=d)
        assert rc in (-1, -3), (b, rc)
    assert pr.lib().inpc_plain_sizes(10, None, 4, 0, 0, None, None, None) == -1


FAKE = 1 << 20   # never dereferenced: every call below fails validation first


def _fwd(n=100, F=4, st=None, ws_bytes=None, saved_bytes=None, image=FAKE, feat=FAKE, saved=FAKE,
         ws=FAKE, blend_weight=None):
    c = pr.c_camera(cam())
    fws, sv, _ = pr.plain_sizes(n, cam(), F, 0, 0)
    st = st or pr.c_settings(1e-4, 0, -1)
    return pr.lib().inpc_rasterize_fwd(FAKE, feat, 0, FAKE, n, F, ctypes.byref(c), ctypes.byref(st),
                                       image, FAKE, blend_weight, saved,
                                       sv if saved_bytes is None else saved_bytes,
                                       ws, fws if ws_bytes is None else ws_bytes, None)


def test_forward_rejects_small_workspace():
    assert _fwd(ws_bytes=16) == -2
    assert _fwd(saved_bytes=16) == -2


@pytest.mark.parametrize("st", [pr.c_settings(-1.0, 0, -1), pr.c_settings(float("inf"), 0, -1),
                                pr.c_settings(1e-4, 5, -1), pr.c_settings(1e-4, 0, 999)])
def test_forward_rejects_settings(st):
    assert _fwd(st=st) == -1


def test_forward_rejects_unknown_flags():
    st = pr.c_settings(1e-4, 0, -1)
    st.flags = 2
    assert _fwd(st=st) == -1


def test_inpc_log_reports_rejected_calls(capfd, monkeypatch):
    """INPC_LOG set: a rejected call says so on stderr (the line a launched
    call prints with its tuning and sort passes needs a GPU)."""
    monkeypatch.delenv("INPC_LOG", raising=False)
    assert _fwd(ws_bytes=16) == -2
    assert "inpc:" not in capfd.readouterr().err
    monkeypatch.setenv("INPC_LOG", "1")
    assert _fwd(ws_bytes=16) == -2
    assert "inpc: forward rejected: workspace or saved buffer too small" in capfd.readouterr().err
    monkeypatch.setenv("INPC_LOG", "0")
    assert _fwd(ws_bytes=16) == -2
    assert "inpc:" not in capfd.readouterr().err


def test_forward_rejects_null_and_misaligned():
    assert _fwd(image=None) == -1
    assert _fwd(image=FAKE + 4) == -1       # image must be 16-byte aligned
    assert _fwd(feat=FAKE + 8) == -1        # features must be 16-byte aligned
    assert _fwd(saved=FAKE + 16) == -1      # buffers must be 256-byte aligned
    assert _fwd(blend_weight=FAKE + 2) == -1  # per-point blend weights are float32


def test_batched_views_must_be_packed_in_order():
    c1, c2 = cam(32, 16), cam(16, 8)
    views = pr.make_views([c1, c2], [0, 50], [50, 50])
    fws, sv, bws = pr.batched_sizes(views, 2, 100, 4, 0, 0)
    assert fws > 0
    views[1].pixel_offset += 1
    with pytest.raises(pr.InpcError):
        pr.batched_sizes(views, 2, 100, 4, 0, 0)
    views = pr.make_views([c1, c2], [0, 60], [50, 50])   # view 2 runs past the point arrays
    with pytest.raises(pr.InpcError):
        pr.batched_sizes(views, 2, 100, 4, 0, 0)


def test_view_grads_validation():
    views = pr.make_views([cam(8, 8)], [0], [10])
    L = pr.lib()
    rc = L.inpc_sum_view_grads(views, 1, 10, 4, FAKE, FAKE, FAKE, FAKE, FAKE + 8, 4096, None)
    assert rc == -1   # workspace pointer not 256-aligned
    rc = L.inpc_sum_view_grads(views, 1, 10, 4, FAKE, FAKE, FAKE, FAKE, FAKE, 8, None)
    assert rc == -2   # workspace smaller than the view table


def test_multisample_validation():
    c = pr.c_camera(cam())
    off = (ctypes.c_int64 * 2)(0, 50)
    cnt = (ctypes.c_int64 * 2)(50, 50)
    need = ctypes.c_size_t(0)
    L = pr.lib()
    assert L.inpc_multisample_sizes(100, ctypes.byref(c), off, cnt, 2, 4, 0, ctypes.byref(need)) == 0
    assert need.value > 0
    assert L.inpc_multisample_sizes(100, ctypes.byref(c), off, cnt, 0, 4, 0, ctypes.byref(need)) == -1
    bad = (ctypes.c_int64 * 2)(0, 60)      # second cloud runs past the point arrays
    assert L.inpc_multisample_sizes(100, ctypes.byref(c), bad, cnt, 2, 4, 0, ctypes.byref(need)) == -1
    st = pr.c_settings(1e-4, 1, -1)
    args = lambda ws_bytes: (FAKE, FAKE, 0, FAKE, 100, 4, ctypes.byref(c), off, cnt, 2, ctypes.byref(st),
                             FAKE, FAKE, FAKE, ws_bytes, None)
    assert L.inpc_multisample_fwd(*args(need.value - 1)) == -2
    st.mode = 7
    assert L.inpc_multisample_fwd(*args(need.value)) == -1


def test_sampling_validation():
    L = pr.lib()
    need = ctypes.c_size_t(0)
    assert L.inpc_sampling_sizes(0, ctypes.byref(need)) == -1
    assert L.inpc_sampling_sizes((1 << 24) + 1, ctypes.byref(need)) == -3
    assert L.inpc_sampling_sizes(1000, ctypes.byref(need)) == 0 and need.value >= 1000 * 24
    c = pr.c_camera(cam())
    unres = FAKE + 64

    def view(n_leaves=1000, tau_d=1e-8, rounds=8, ws_bytes=None, n=10):
        return L.inpc_sample_view(FAKE, FAKE, FAKE, n_leaves, 16.0, 0.5, tau_d, ctypes.byref(c), n, 1, 2, rounds,
                                  FAKE, FAKE, unres, FAKE, need.value if ws_bytes is None else ws_bytes, None)
    assert view(ws_bytes=need.value - 1) == -2
    assert view(tau_d=0.0) == -1
    assert view(rounds=-1) == -1
    assert view(n=-5) == -1
    assert view(n_leaves=0) == -1
    assert L.inpc_sample_global(FAKE, FAKE, FAKE, 1000, -1.0, 0.5, 10, 1, 2, FAKE, FAKE, FAKE, need.value,
                                None) == -1     # root size must be positive
    assert L.inpc_update_probabilities(FAKE, FAKE, 10, 1000, 0.9968, FAKE, FAKE, FAKE, need.value - 1,
                                       None) == -2


def _gpu_visible() -> bool:
    import torch
    return torch.cuda.is_available()


# The forward below passes validation with pointers that are never valid device
# memory; without a GPU every HIP call fails before anything runs.  Where a GPU
# is visible it is skipped (tests/test_gpu_parity.py covers the same on real
# buffers).
@pytest.mark.skipif(_gpu_visible(), reason="fake pointers may only reach the launch path without a GPU")
def test_backward_uses_the_tuning_of_its_forward(tmp_path):
    L = pr.lib()
    c = pr.c_camera(cam())
    n, F = 100, 4
    fws, sv, bws = pr.plain_sizes(n, cam(), F, 0, 0)
    saved = FAKE + (1 << 24)
    st = pr.c_settings(1e-4, 0, 7)
    rc = L.inpc_rasterize_fwd(FAKE, FAKE, 0, FAKE, n, F, ctypes.byref(c), ctypes.byref(st), FAKE, FAKE, None,
                              saved, sv, FAKE, fws, None)
    assert rc == -5                          # no device: nothing ran, but the arguments were accepted
    assert L.inpc_saved_tuning(saved) == 7
    assert L.inpc_saved_tuning(None) == -1 and L.inpc_saved_tuning(saved + 256) == -1
    # the autotuner's cache changes between forward and backward: the bucket
    # key is the device, view count, ceil(log2) of the view points and of the
    # pixels, F and the feature type
    import json
    views = pr.make_views([cam()], [0], [n])
    lg = lambda x: (int(x) - 1).bit_length()
    bucket = f"gfx950|V1|N{lg(n)}|P{lg(64 * 48)}|F{F}|T0"
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({bucket: 3}))
    assert L.inpc_autotune_load(str(cache).encode()) >= 0
    assert L.inpc_tuning_for(views, 1, n, F, 0) == 3

    def bwd(tid):
        s2 = pr.c_settings(1e-4, 0, tid)
        return L.inpc_rasterize_bwd(FAKE, FAKE, 0, FAKE, n, F, ctypes.byref(c), ctypes.byref(s2), saved, sv,
                                    FAKE, None, FAKE, FAKE, None, FAKE, bws, None)
    assert bwd(3) == -1          # an explicit id other than the forward's is rejected
    assert bwd(0) == -1
    assert bwd(7) == -5          # the forward's id is accepted (then fails for want of a device)
    assert bwd(-1) == -5         # -1 is accepted (it takes the recorded id, not the cache's 3)
    # a state no forward recorded falls back to the cache
    s3 = pr.c_settings(1e-4, 0, -1)
    assert L.inpc_rasterize_bwd(FAKE, FAKE, 0, FAKE, n, F, ctypes.byref(c), ctypes.byref(s3), saved + 512, sv,
                                FAKE, None, FAKE, FAKE, None, FAKE, bws, None) == -5
    cache.write_text(json.dumps({bucket: 0}))
    L.inpc_autotune_load(str(cache).encode())


def test_negative_zero_near_plane_is_accepted():
    d = cam().as_dict()
    d["near"] = -0.0
    assert _call_sizes(c=d) == 0


SCRATCH_BYTES = 256 << 20   # INPC_NOALLOC_SCRATCH_BYTES


def _noalloc(n, F=16, fdt=0, mode=1, camera=None):
    c = pr.c_camera(camera or cam())
    st = pr.c_settings(1e-4, mode, -1)
    return pr.lib().inpc_rasterize_fwd_noalloc(FAKE, FAKE, fdt, FAKE, n, F, ctypes.byref(c), ctypes.byref(st),
                                               FAKE, FAKE, None, None)


def _noalloc_fits(n, camera, F, fdt):
    fws, sv, _ = pr.plain_sizes(n, camera, F, fdt, 1)
    return ((sv + 255) // 256) * 256 + fws <= SCRATCH_BYTES


def test_noalloc_forward_rejects_on_the_host():
    """The no-allocation forward refuses, before touching the device, a
    problem whose recompute-mode state and workspace exceed the fixed
    scratch (INPC_ESCRATCH) and a SAVE-mode request (no state is kept)."""
    hd = workloads.canonical_camera(1920, 1080)
    assert not _noalloc_fits(2_000_000, hd, 16, 0)
    assert _noalloc(2_000_000, camera=hd) == -6
    assert _noalloc(100, mode=0) == -1
    assert _noalloc(100, F=0) == -3
    # the sizes the header quotes as fitting
    assert _noalloc_fits(1_370_000, workloads.canonical_camera(1280, 720), 8, 0)
    assert _noalloc_fits(870_000, hd, 16, 0) and not _noalloc_fits(880_000, hd, 16, 0)
    assert _noalloc_fits(1_190_000, hd, 16, 1) and not _noalloc_fits(1_200_000, hd, 16, 1)
