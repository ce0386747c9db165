"""The plain one-view entry points of the C ABI, driven directly through
ctypes with real device buffers sized by inpc_plain_sizes: Algorithm 1's
Rasterize(C, P, A, F) (inpc_rasterize_fwd) and its backward (Appendix A.6,
inpc_rasterize_bwd), against the FP64 oracle on the 1M-point 1280x720 scene
(F = 8 float32): sorted splat lists bit-exact, image and transmittance within
1e-5 relative, gradients against the oracle's adjoint and central
differences within 1e-3, blend weights from both passes.  Also: RECOMPUTE
equals SAVE bit for bit, and a backward keeps the forward's tuning when the
autotuner's cache changes in between."""

import ctypes
import json

import numpy as np
import pytest
import torch

import oracle
import paper_2403_16862_amd as pr
import workloads
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class PlainRun:
    """Buffers of one plain forward + backward through the C ABI."""

    def __init__(self, s, mode=pr.INPC_SAVE, tuning_id=-1, g_t=None):
        self.s, self.mode = s, mode
        self.N, self.F = s.n, s.F
        self.cam = pr.c_camera(s.cam)
        self.fws, self.sv, self.bws = pr.plain_sizes(self.N, s.cam, self.F, pr.INPC_F32, mode)
        self.x, self.f, self.o = H.to_dev(s.xyz), H.to_dev(s.feat), H.to_dev(s.opa)
        self.saved = pr._buffer(self.sv, H.DEV)
        self.ws = pr._buffer(self.fws, H.DEV)
        self.bwd_ws = pr._buffer(self.bws, H.DEV)
        W, Hh = s.cam.width, s.cam.height
        self.image = torch.empty((Hh, W, self.F), dtype=torch.float32, device=H.DEV)
        self.t_final = torch.empty((Hh, W), dtype=torch.float32, device=H.DEV)
        self.bw_fwd = torch.empty((self.N,), dtype=torch.float32, device=H.DEV)
        self.bw_bwd = torch.empty((self.N,), dtype=torch.float32, device=H.DEV)
        self.g = H.to_dev(s.g_img)
        self.g_t = None if g_t is None else H.to_dev(g_t)
        self.gf = torch.empty((self.N, self.F), dtype=torch.float32, device=H.DEV)
        self.go = torch.empty((self.N,), dtype=torch.float32, device=H.DEV)
        self.settings = pr.c_settings(1e-4, mode, tuning_id)

    def forward(self):
        rc = pr.lib().inpc_rasterize_fwd(
            _p(self.x), _p(self.f), pr.INPC_F32, _p(self.o), self.N, self.F, ctypes.byref(self.cam),
            ctypes.byref(self.settings), _p(self.image), _p(self.t_final), _p(self.bw_fwd), _p(self.saved),
            self.saved.numel(), _p(self.ws), self.ws.numel(), pr._stream())
        assert rc == 0, pr.lib().inpc_error_string(rc)

    def backward(self, settings=None):
        st = settings or self.settings
        return pr.lib().inpc_rasterize_bwd(
            _p(self.x), _p(self.f), pr.INPC_F32, _p(self.o), self.N, self.F, ctypes.byref(self.cam),
            ctypes.byref(st), _p(self.saved), self.saved.numel(), _p(self.g), _p(self.g_t), _p(self.gf),
            _p(self.go), _p(self.bw_bwd), _p(self.bwd_ws), self.bwd_ws.numel(), pr._stream())

    def fragments(self):
        views = pr.make_views([self.s.cam], [0], [self.N])
        st = pr.ForwardState(self.saved, self.ws, self.settings, views, 1, self.N, self.F, pr.INPC_F32)
        return pr.debug_fragments(st)

    def host(self):
        torch.cuda.synchronize()
        return dict(image=self.image.reshape(-1, self.F).cpu().numpy(), t_final=self.t_final.reshape(-1).cpu().numpy(),
                    gf=self.gf.cpu().numpy(), go=self.go.cpu().numpy(), bw_fwd=self.bw_fwd.cpu().numpy(),
                    bw_bwd=self.bw_bwd.cpu().numpy())


@pytest.fixture(scope="module")
def scene2():
    return workloads.config2(g_t=True)


def test_plain_abi_config2_against_oracle(scene2):
    s = scene2
    H.say(f"  plain C ABI: N={s.n} {s.cam.width}x{s.cam.height} F={s.F}, with dL/dT_final")
    run = PlainRun(s, g_t=s.g_t)
    run.forward()
    assert run.backward() == 0
    out = run.host()
    keys, ids, nb = run.fragments()
    L = oracle.fragments(s.xyz, s.cam)
    assert np.array_equal(keys, L.keys()) and np.array_equal(ids, L.ids)
    n_gpu = nb.astype(np.int32)
    ref_t = oracle.blend_forward(L, s.opa, s.feat, 1e-4, want_t_after=True)
    amb = H.termination_ok(L, ref_t["t_after"], n_gpu, ref_t["n_blended"], 1e-4)
    H.say(f"    {L.m} splats bit-exact, ambiguous pixels {amb}")
    H.check_image(dict(image=run.image, t_final=run.t_final), L, s.opa, s.feat, 1e-4, n_gpu)
    P = s.cam.width * s.cam.height
    ref = oracle.blend_backward(L, s.opa, s.feat, n_gpu, s.g_img.reshape(P, s.F), s.g_t.reshape(P))
    H.check_grads(out["gf"], out["go"], ref)
    H.fd_check(L, s.opa, s.feat, n_gpu, s.g_img, s.g_t, out["gf"], out["go"], n_check=64, seed=11)
    H.check_blend_weight(out["bw_fwd"], L, s.opa, n_gpu)
    H.check_blend_weight(out["bw_bwd"], L, s.opa, n_gpu)


def test_plain_abi_recompute_equals_save(scene2):
    s = scene2
    a = PlainRun(s, pr.INPC_SAVE, g_t=s.g_t)
    a.forward()
    assert a.backward() == 0
    ra = a.host()
    del a
    b = PlainRun(s, pr.INPC_RECOMPUTE, g_t=s.g_t)
    b.forward()
    assert b.backward() == 0
    rb = b.host()
    for k in ra:
        assert np.array_equal(ra[k], rb[k]), k
    H.say("    RECOMPUTE == SAVE bit for bit (image, t_final, gradients, blend weights)")


def test_backward_keeps_the_forward_tuning_when_the_cache_changes(tmp_path):
    s = workloads.config1()
    rng = np.random.default_rng(5)
    s.g_img = rng.normal(size=(s.cam.height, s.cam.width, s.F)).astype(np.float32)
    L = pr.lib()
    views = pr.make_views([s.cam], [0], [s.n])
    first = L.inpc_tuning_for(views, 1, s.n, s.F, 0)
    other = len(pr.tuning_table()) - 1            # per-pixel lists, 1 lane: another state layout
    assert other != first
    ref = PlainRun(s, tuning_id=first)
    ref.forward()
    assert ref.backward() == 0
    want = ref.host()
    run = PlainRun(s, tuning_id=-1)
    run.forward()
    assert L.inpc_saved_tuning(_p(run.saved)) == first
    lg = lambda x: (int(x) - 1).bit_length()
    bucket = f"gfx950|V1|N{lg(s.n)}|P{lg(s.cam.width * s.cam.height)}|F{s.F}|T0"
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({bucket: other}))
    try:
        assert L.inpc_autotune_load(str(cache).encode()) >= 0
        assert L.inpc_tuning_for(views, 1, s.n, s.F, 0) == other
        assert run.backward(pr.c_settings(1e-4, pr.INPC_SAVE, other)) == -1   # mismatch: rejected, nothing ran
        assert run.backward() == 0                                           # -1: the forward's tuning
        got = run.host()
    finally:
        cache.write_text(json.dumps({bucket: first}))
        L.inpc_autotune_load(str(cache).encode())
    for k in want:
        assert np.array_equal(want[k], got[k]), k
