"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (default tuning):

* 8M points at 1920x1080, F=16 float32, forward + backward through
  torch.autograd.Function: the whole sorted splat list bit-exact, every image
  element and gradient against the oracle, central differences on 64 points;
* the 16-view batched bfloat16 workload as one graph replay, every view
  checked completely against the oracle;
* 32M points (clusters plus a far background shell), 8 poses at 1080p,
  bfloat16 features, forward only: each pose as a plain call, the 8 poses as
  one batched call over aliased views, and the far = 10^3 variant.

The first also checks the per-point blend weights of every point.
"""

import numpy as np
import pytest
import torch

import oracle
import paper_2403_16862_amd as pr
import workloads
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def test_config3_full_autograd_with_fd():
    s = workloads.config3()
    H.say(f"  config 3: N={s.n} {s.cam.width}x{s.cam.height} F={s.F}")
    x = H.to_dev(s.xyz)
    f = H.to_dev(s.feat).requires_grad_(True)
    o = H.to_dev(s.opa).requires_grad_(True)
    img, tf = pr.rasterize(x, f, o, s.cam, 1e-4)
    torch.autograd.backward([img], [H.to_dev(s.g_img)])
    torch.cuda.synchronize()
    gf, go = f.grad.cpu().numpy(), o.grad.cpu().numpy()
    # the splat list of the same forward, via the debug hook
    bw = torch.empty((s.n,), dtype=torch.float32, device=H.DEV)
    _, _, st = pr.rasterize_forward(x, f.detach(), o.detach(), s.cam, 1e-4, keep_workspace=True,
                                    blend_weight=bw)
    keys, ids, nb = pr.debug_fragments(st)
    L = oracle.fragments(s.xyz, s.cam)
    assert np.array_equal(keys, L.keys()) and np.array_equal(ids, L.ids)
    H.say(f"    {L.m} splats bit-exact")
    n_gpu = nb.astype(np.int32)
    ref_t = oracle.blend_forward(L, s.opa, s.feat, 1e-4, want_t_after=True)
    amb = H.termination_ok(L, ref_t["t_after"], n_gpu, ref_t["n_blended"], 1e-4)
    H.say(f"    ambiguous pixels: {amb}")
    run = dict(image=img.detach(), t_final=tf.detach())
    H.check_image(run, L, s.opa, s.feat, 1e-4, n_gpu)
    ref = oracle.blend_backward(L, s.opa, s.feat, n_gpu, s.g_img)
    H.check_grads(gf, go, ref)
    H.fd_check(L, s.opa, s.feat, n_gpu, s.g_img, None, gf, go, n_check=64, seed=3)
    H.check_blend_weight(bw.cpu().numpy(), L, s.opa, n_gpu)


@pytest.fixture(scope="module")
def config4_replay():
    """The 16-view batched bfloat16 workload as one graph replay (the timed
    form): sorted lists, blend counts, images, transmittances and gradients."""
    b = workloads.config4()
    views = pr.make_views(b.cams, b.point_offset, b.point_count)
    g = np.concatenate([gi.reshape(-1, b.F) for gi in b.g_imgs])
    x, o = H.to_dev(b.xyz), H.to_dev(b.opa)
    f = H.to_dev(b.feat).to(torch.bfloat16)
    step = pr.BatchedStep(x, f, o, views, H.to_dev(g))
    step.capture()
    step.replay()
    torch.cuda.synchronize()
    keys, ids, nb = pr.debug_fragments(step.state())
    out = dict(b=b, g=g, keys=keys, ids=ids, nb=nb, img=step.image.cpu().numpy(), tf=step.t_final.cpu().numpy(),
               gf=step.grad_feat.cpu().numpy(), go=step.grad_opa.cpu().numpy(), fbits=H.bf16_bits(b.feat))
    del step, x, o, f
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("view", range(16))
def test_config4_batched_graph_view(config4_replay, view):
    """One of the 16 views of the timed graph replay: splat list bit-exact,
    image and transmittance within 1e-5 of the oracle on the bfloat16-rounded
    features, within 1e-2 of the oracle on the unrounded float32 features,
    gradients against the oracle's adjoint."""
    r = config4_replay
    b, v = r["b"], view
    P_v = [c.width * c.height for c in b.cams]
    pix_off = np.concatenate([[0], np.cumsum(P_v)]).astype(np.int64)
    vp_off = np.concatenate([[0], np.cumsum(b.point_count)]).astype(np.int64)
    vbound = np.searchsorted(r["keys"] >> np.uint64(32), pix_off.astype(np.uint64))   # keys are sorted by pixel
    sl = slice(b.point_offset[v], b.point_offset[v] + b.point_count[v])
    L = oracle.fragments(b.xyz[sl], b.cams[v])
    lo, hi = int(pix_off[v]), int(pix_off[v + 1])
    a, e = int(vbound[v]), int(vbound[v + 1])
    assert np.array_equal(r["keys"][a:e], L.keys(lo))
    assert np.array_equal(r["ids"][a:e].astype(np.int64) - 4 * int(vp_off[v]), L.ids.astype(np.int64))
    n_gpu = r["nb"][lo:hi].astype(np.int32)
    fbits = r["fbits"]
    ref_t = oracle.blend_forward(L, b.opa[sl], fbits[sl], 1e-4, want_t_after=True)
    amb = H.termination_ok(L, ref_t["t_after"], n_gpu, ref_t["n_blended"], 1e-4)
    del ref_t
    ref = oracle.blend_forward(L, b.opa[sl], fbits[sl], 1e-4, n_override=n_gpu)
    e_img = H.rel_err(r["img"][lo:hi], ref["image"]).max()
    e_t = H.rel_err(r["tf"][lo:hi], ref["t_final"]).max()
    assert e_img <= H.REL_TOL and e_t <= H.REL_TOL, (v, e_img, e_t)
    del ref
    unr = oracle.blend_forward(L, b.opa[sl], b.feat[sl], 1e-4, n_override=n_gpu)
    e_unr = float(np.abs(r["img"][lo:hi] - unr["image"]).max())
    assert e_unr <= H.BF16_ABS_TOL, (v, e_unr)
    del unr
    rb = oracle.blend_backward(L, b.opa[sl], fbits[sl], n_gpu, r["g"][lo:hi])
    H.check_grads(r["gf"][vp_off[v]:vp_off[v + 1]], r["go"][vp_off[v]:vp_off[v + 1]], rb)
    H.say(f"    view {v}: {b.cams[v].width}x{b.cams[v].height} N={b.point_count[v]} M={L.m} ambiguous={amb} "
          f"image err {e_img:.2e} t_final err {e_t:.2e} unrounded-feature err {e_unr:.2e}")


@pytest.fixture(scope="module")
def config5_scene():
    return workloads.config5()


def _check_pose(L, opa, feat, fbits, img, tf, n_gpu, label):
    ref_t = oracle.blend_forward(L, opa, fbits, 1e-4, want_t_after=True)
    amb = H.termination_ok(L, ref_t["t_after"], n_gpu, ref_t["n_blended"], 1e-4)
    del ref_t
    ref = oracle.blend_forward(L, opa, fbits, 1e-4, n_override=n_gpu)
    e = H.rel_err(img, ref["image"]).max()
    et = H.rel_err(tf, ref["t_final"]).max()
    assert e <= H.REL_TOL and et <= H.REL_TOL, (label, e, et)
    del ref
    unr = oracle.blend_forward(L, opa, feat, 1e-4, n_override=n_gpu)
    eu = float(np.abs(img - unr["image"]).max())
    assert eu <= H.BF16_ABS_TOL, (label, eu)
    H.say(f"    {label}: M={L.m} blended={int(n_gpu.sum())} ambiguous={amb} image err {e:.2e} "
          f"t_final err {et:.2e} unrounded-feature err {eu:.2e}")


@pytest.fixture(scope="module")
def config5_batched(config5_scene):
    """The 8 poses as one batched call whose views all alias the same points:
    sorted lists, blend counts, images and transmittances on the host."""
    b = config5_scene
    x, o = H.to_dev(b.xyz), H.to_dev(b.opa)
    f = H.to_dev(b.feat).to(torch.bfloat16)
    views = pr.make_views(b.cams, b.point_offset, b.point_count)
    img_b, tf_b, st_b = pr.rasterize_forward_batched(x, f, o, views, 1e-4, "save", keep_workspace=True)
    keys_b, ids_b, nb_b = pr.debug_fragments(st_b)
    out = dict(keys=keys_b, ids=ids_b, nb=nb_b, img=img_b.cpu().numpy(), tf=tf_b.cpu().numpy())
    del st_b, img_b, tf_b, x, o, f
    torch.cuda.empty_cache()
    H.say(f"  config 5: N={b.xyz.shape[0]}, 8 aliased views, {keys_b.shape[0]} splats in the batched call")
    return out


@pytest.mark.parametrize("pose", range(8))
def test_config5_pose_plain_and_aliased_batched(config5_scene, config5_batched, pose):
    """32M points (clusters plus a background shell), 8 poses on a circle,
    bfloat16 features, forward only: this pose as a plain call against the
    oracle, and its view of the batched call over 8 aliased views."""
    b = config5_scene
    v, cam = pose, b.cams[pose]
    n = b.xyz.shape[0]
    x, o = H.to_dev(b.xyz), H.to_dev(b.opa)
    f = H.to_dev(b.feat).to(torch.bfloat16)
    img, tf, st = pr.rasterize_forward(x, f, o, cam, 1e-4, keep_workspace=True)
    keys, ids, nb = pr.debug_fragments(st)
    img, tf = img.reshape(-1, 16).cpu().numpy(), tf.reshape(-1).cpu().numpy()
    del st, x, o, f
    torch.cuda.empty_cache()
    L = oracle.fragments(b.xyz, cam)
    assert np.array_equal(keys, L.keys()) and np.array_equal(ids, L.ids), v
    P = cam.width * cam.height
    bt = config5_batched
    vbound = np.searchsorted(bt["keys"] >> np.uint64(32), np.array([v * P, (v + 1) * P], dtype=np.uint64))
    a, e = int(vbound[0]), int(vbound[1])
    assert np.array_equal(bt["keys"][a:e], L.keys(v * P)), v
    assert np.array_equal(bt["ids"][a:e].astype(np.int64) - 4 * v * n, L.ids.astype(np.int64)), v
    n_gpu = nb.astype(np.int32)
    assert np.array_equal(bt["nb"][v * P:(v + 1) * P], nb), v
    _check_pose(L, b.opa, b.feat, H.bf16_bits(b.feat), img, tf, n_gpu, f"pose {v} plain")
    # the batched call blends the same lists with the same arithmetic
    assert np.array_equal(bt["img"][v * P:(v + 1) * P], img) and np.array_equal(bt["tf"][v * P:(v + 1) * P], tf), v
    H.say(f"    pose {v} batched: lists and blend counts equal the oracle's, image equal to the plain call")


def test_config5_far_plane_1000(config5_scene):
    """The far = 10^3 variant: the background shell (radius 50-200) is no longer culled."""
    import copy
    b = config5_scene
    cam = copy.deepcopy(b.cams[0])
    cam.far = 1000.0
    x, o = H.to_dev(b.xyz), H.to_dev(b.opa)
    f = H.to_dev(b.feat).to(torch.bfloat16)
    img, tf, st = pr.rasterize_forward(x, f, o, cam, 1e-4, keep_workspace=True)
    keys, ids, nb = pr.debug_fragments(st)
    L = oracle.fragments(b.xyz, cam)
    assert np.array_equal(keys, L.keys()) and np.array_equal(ids, L.ids)
    _check_pose(L, b.opa, b.feat, H.bf16_bits(b.feat), img.reshape(-1, 16).cpu().numpy(),
                tf.reshape(-1).cpu().numpy(), nb.astype(np.int32), "pose 0, far 1000")
