"""GPU parity of the appearance step (Section 3.3: opacity activation and
degree-2 SH features per view point) and of its fusion with the rasterizer,
against the FP64 oracle on the same seeded inputs.

Tolerances: the opacity is evaluated in float64 and rounded once (2 ulp of
float32); a feature sum_j Y_j c_j in float32 has error below ~1e-6 times
sum_j |c_j| (|Y_j| <= 1.1, direction error ~1e-7), checked at 1e-5 times
that scale; gradients as for the rasterizer (1e-3 of max(|ref|, 1e-3 rms))."""

import numpy as np
import pytest
import torch

import oracle
import paper_2403_16862_amd as pr
import workloads
from oracle import appearance as A
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _scene(seed, n, W=160, H_=96):
    rng = np.random.default_rng(seed)
    cam0 = workloads.canonical_camera(W, H_)
    xyz = workloads.cluster_points(rng, n, 16, cam0).astype(np.float32)
    raw = workloads.sh_raw(rng, n)
    cams = [workloads.look_at_camera(rng.uniform(-0.5, 0.5, 3), [0, 0, 5], [0, -1, 0], W, H_)
            for _ in range(2)]
    return xyz, raw, cams


def _feat_scale(raw, offs, cnts):
    coef = np.abs(raw[:, 1:].astype(np.float64)).reshape(-1, 9, 4).sum(1)   # [N,4]
    return np.concatenate([coef[o:o + c] for o, c in zip(offs, cnts)])


def test_appearance_forward_views_and_bf16():
    xyz, raw, cams = _scene(21, 50_000)
    offs, cnts = [0, 20_000], [40_000, 30_000]          # points 20000..39999 are in both views
    views = pr.make_views(cams, offs, cnts)
    x, r = H.to_dev(xyz), H.to_dev(raw)
    ref_o, ref_f = A.forward(xyz, raw, cams, offs, cnts)
    scale = _feat_scale(raw, offs, cnts)
    o, f = pr.appearance_forward(x, r, views)
    o, f = o.cpu().numpy(), f.cpu().numpy()
    e_o = np.abs(o - ref_o) / ref_o
    e_f = np.abs(f - ref_f) / scale
    H.say(f"    opacity rel err max {e_o.max():.3e}; feature err / sum|c| max {e_f.max():.3e}")
    assert e_o.max() <= 2.0 ** -22
    assert e_f.max() <= 1e-5
    ob, fb = pr.appearance_forward(x, r, views, torch.bfloat16)
    assert torch.equal(ob.cpu(), torch.from_numpy(o))
    # bfloat16 output = the float32 result rounded to nearest even
    assert torch.equal(fb.cpu(), torch.from_numpy(f).to(torch.bfloat16))


def test_appearance_backward_folds_views():
    xyz, raw, cams = _scene(22, 30_000)
    offs, cnts = [0, 10_000], [25_000, 20_000]
    views = pr.make_views(cams, offs, cnts)
    n_vp = sum(cnts)
    rng = np.random.default_rng(5)
    go = rng.normal(size=n_vp).astype(np.float32)
    gf = rng.normal(size=(n_vp, 4)).astype(np.float32)
    g = pr.appearance_backward(H.to_dev(xyz), H.to_dev(raw), views, H.to_dev(go), H.to_dev(gf))
    g = g.cpu().numpy()
    ref = A.backward(xyz, raw, cams, offs, cnts, go, gf)
    # per-point scale: sum over the point's view rows of |g| (|Y| <= 1.1)
    sc_f = np.zeros((xyz.shape[0], 4))
    sc_o = np.zeros(xyz.shape[0])
    vp = 0
    for o, c in zip(offs, cnts):
        sc_f[o:o + c] += np.abs(gf[vp:vp + c])
        sc_o[o:o + c] += np.abs(go[vp:vp + c]) * A.opacity_grad(raw[o:o + c, 0])
        vp += c
    e_sh = np.abs(g[:, 1:] - ref[:, 1:]).reshape(-1, 9, 4) / np.maximum(sc_f[:, None, :], 1e-30)
    e_o = np.abs(g[:, 0] - ref[:, 0]) / np.maximum(sc_o, 1e-30)
    H.say(f"    grad SH err max {e_sh.max():.3e}; grad logit err max {e_o.max():.3e}")
    assert e_sh.max() <= 1e-5 and e_o.max() <= 1e-5


def test_render_sh_end_to_end_gradients():
    xyz, raw, cams = _scene(23, 40_000)
    offs, cnts = [0, 0], [40_000, 40_000]                # two views of one cloud
    views = pr.make_views(cams, offs, cnts)
    x = H.to_dev(xyz)
    r = H.to_dev(raw).requires_grad_(True)
    bw = torch.empty((sum(cnts),), dtype=torch.float32, device=H.DEV)
    img, tf = pr.render_sh(x, r, views, blend_weight=bw)
    P = [c.width * c.height for c in cams]
    rng = np.random.default_rng(6)
    g_img = rng.normal(size=(sum(P), 4)).astype(np.float32)
    torch.autograd.backward([img], [H.to_dev(g_img)])
    torch.cuda.synchronize()
    grad = r.grad.cpu().numpy()
    # the features and opacities the GPU rendered, and its blend counts
    o_gpu, f_gpu = pr.appearance_forward(x, H.to_dev(raw), views)
    o_gpu, f_gpu = o_gpu.cpu().numpy(), f_gpu.cpu().numpy()
    img2, _, st = pr.rasterize_forward_batched(x, H.to_dev(f_gpu), H.to_dev(o_gpu), views, keep_workspace=True,
                                               attr_per_view_point=True)
    _, _, nb = pr.debug_fragments(st)
    img = img.detach().cpu().numpy()
    assert np.array_equal(img, img2.cpu().numpy())
    g_opa = np.zeros(sum(cnts))
    g_feat = np.zeros((sum(cnts), 4))
    pix = 0
    vp = 0
    for v, cam in enumerate(cams):
        sl = slice(vp, vp + cnts[v])
        L = oracle.fragments(xyz[offs[v]:offs[v] + cnts[v]], cam)
        n = nb[pix:pix + L.P].astype(np.int32)
        ref_t = oracle.blend_forward(L, o_gpu[sl], f_gpu[sl], 1e-4, want_t_after=True)
        H.termination_ok(L, ref_t["t_after"], n, ref_t["n_blended"], 1e-4)
        ref = oracle.blend_forward(L, o_gpu[sl], f_gpu[sl], 1e-4, n_override=n)
        mag = oracle.blend_forward(L, o_gpu[sl], np.abs(f_gpu[sl]), 1e-4, n_override=n)["image"]
        e = np.abs(img[pix:pix + L.P] - ref["image"]) / np.maximum(mag, 1e-12)
        H.say(f"    view {v}: image err / sum T a |c| max {e.max():.3e}")
        assert e.max() <= H.REL_TOL
        H.check_blend_weight(bw[sl].cpu().numpy(), L, o_gpu[sl], n)
        b = oracle.blend_backward(L, o_gpu[sl], f_gpu[sl], n, g_img[pix:pix + L.P])
        g_opa[sl] = b["grad_opa"]
        g_feat[sl] = b["grad_feat"]
        pix += L.P
        vp += cnts[v]
    ref_raw = A.backward(xyz, raw, cams, offs, cnts, g_opa, g_feat)
    e = H.grad_err(grad, ref_raw)
    H.say(f"    grad raw err max {e.max():.3e} p99 {np.quantile(e, 0.99):.3e}")
    assert e.max() <= H.GRAD_TOL
