"""GPU parity of the per-point blend weight (the sum over a point's blended
splats of w_k T_k alpha_k, Eq. 1 weights combined bilinearly as in
Appendix A.6; the input of the probability updates of Section 3.1) against
the FP64 oracle on the same seeded inputs and the GPU's blend counts."""

import numpy as np
import pytest
import torch

import oracle
import paper_2403_16862_amd as pr
import workloads
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _case(xyz, feat, opa, cam, tau=1e-4, mode="save", tuning_id=-1, bf16=False):
    H.say(f"  case N={xyz.shape[0]} {cam.width}x{cam.height} tau={tau} mode={mode} tuning={tuning_id}")
    lists = oracle.fragments(xyz, cam)
    x, o = H.to_dev(xyz), H.to_dev(opa)
    f = H.to_dev(feat)
    if bf16:
        f = f.to(torch.bfloat16)
    bw = torch.full((xyz.shape[0],), float("nan"), dtype=torch.float32, device=H.DEV)
    img, tf, st = pr.rasterize_forward(x, f, o, cam, tau, mode, tuning_id, keep_workspace=True,
                                       blend_weight=bw)
    img2, tf2, _ = pr.rasterize_forward(x, f, o, cam, tau, mode, tuning_id)
    torch.cuda.synchronize()
    # asking for the weights changes nothing else
    assert torch.equal(img, img2) and torch.equal(tf, tf2)
    if mode == "save":
        n_gpu = H.check_fragments(dict(state=st), lists)
    else:
        n_gpu = oracle.blend_forward(lists, opa, feat, tau)["n_blended"]
    H.check_blend_weight(bw.cpu().numpy(), lists, opa, n_gpu)
    return bw


def test_blend_weight_config1():
    s = workloads.config1()
    _case(s.xyz, s.feat, s.opa, s.cam)


def test_blend_weight_config2_all_tunings():
    s = workloads.config2(n=200_000)
    for tid in range(len(pr.tuning_table())):
        _case(s.xyz, s.feat, s.opa, s.cam, tuning_id=tid)


def test_blend_weight_no_termination_and_bf16():
    s = workloads.config3(n=40_000, width=129, height=65, grads=False)
    _case(s.xyz, s.feat, s.opa, s.cam, tau=0.0, bf16=True)


def test_blend_weight_ragged_and_culled():
    rng = np.random.default_rng(7)
    cam = workloads.canonical_camera(53, 17)
    n = 5000
    xyz = workloads.scenes.cluster_points(rng, n, 6, cam).astype(np.float32)
    xyz[: n // 4, 2] = -1.0          # behind the camera: no splats, weight exactly 0
    feat = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    opa = rng.uniform(0.05, 0.95, n).astype(np.float32)
    bw = _case(xyz, feat, opa, cam).cpu().numpy()
    assert np.all(bw[: n // 4] == 0)


def test_blend_weight_empty_cloud():
    cam = workloads.canonical_camera(16, 8)
    xyz = np.zeros((0, 3), np.float32)
    bw = torch.zeros((0,), dtype=torch.float32, device=H.DEV)
    pr.rasterize_forward(H.to_dev(xyz), H.to_dev(np.zeros((0, 4), np.float32)),
                         H.to_dev(np.zeros(0, np.float32)), cam, blend_weight=bw)
    torch.cuda.synchronize()


def test_blend_weight_batched_aliased_views():
    """Two views of the same points: one weight per view point, each equal to
    the single-view oracle of its view."""
    s = workloads.config2(n=100_000)
    cam2 = workloads.look_at_camera(np.array([0.5, 0.3, -2.5]), np.array([0.0, 0.0, 5.0]),
                                  np.array([0.0, -1.0, 0.0]), 160, 96)
    cams = [s.cam, cam2]
    views = pr.make_views(cams, [0, 0], [s.n, s.n])
    bw = torch.empty((2 * s.n,), dtype=torch.float32, device=H.DEV)
    x, f, o = H.to_dev(s.xyz), H.to_dev(s.feat), H.to_dev(s.opa)
    img, tf, st = pr.rasterize_forward_batched(x, f, o, views, keep_workspace=True, blend_weight=bw)
    torch.cuda.synchronize()
    keys, ids, nb = pr.debug_fragments(st)
    bw = bw.cpu().numpy()
    pix_off = 0
    for v, cam in enumerate(cams):
        L = oracle.fragments(s.xyz, cam)
        n_gpu = nb[pix_off:pix_off + L.P].astype(np.int32)
        H.check_blend_weight(bw[v * s.n:(v + 1) * s.n], L, s.opa, n_gpu)
        pix_off += L.P


def test_blend_weight_in_graph_replay():
    b = workloads.config4(n_views=4, n_min=1e5, n_max=4e5)
    views = pr.make_views(b.cams, b.point_offset, b.point_count)
    g = np.concatenate([gi.reshape(-1, b.F) for gi in b.g_imgs])
    x, o, f = H.to_dev(b.xyz), H.to_dev(b.opa), H.to_dev(b.feat)
    step = pr.BatchedStep(x, f, o, views, H.to_dev(g), want_blend_weight=True)
    step.run()
    torch.cuda.synchronize()
    eager = step.blend_weight.clone()
    step.capture()
    for _ in range(3):
        step.blend_weight.fill_(float("nan"))
        step.replay()
        torch.cuda.synchronize()
        assert torch.equal(step.blend_weight, eager)
    _, _, nb = pr.debug_fragments(step.state())
    P_v = [c.width * c.height for c in b.cams]
    pix_off = np.concatenate([[0], np.cumsum(P_v)]).astype(np.int64)
    vp_off = np.concatenate([[0], np.cumsum(b.point_count)]).astype(np.int64)
    bw = eager.cpu().numpy()
    for v in range(len(b.cams)):
        sl = slice(b.point_offset[v], b.point_offset[v] + b.point_count[v])
        L = oracle.fragments(b.xyz[sl], b.cams[v])
        H.check_blend_weight(bw[vp_off[v]:vp_off[v + 1]], L, b.opa[sl],
                             nb[pix_off[v]:pix_off[v + 1]].astype(np.int32))


@pytest.mark.parametrize("mode", ["save", "recompute"])
def test_blend_weight_from_backward(mode):
    """The backward's per-point reduction yields the same weights (from its own
    T_k alpha_k records) as the forward's optional output."""
    s = workloads.config2(n=300_000)
    lists = oracle.fragments(s.xyz, s.cam)
    x, f, o = H.to_dev(s.xyz), H.to_dev(s.feat), H.to_dev(s.opa)
    img, tf, st = pr.rasterize_forward(x, f, o, s.cam, 1e-4, "save", keep_workspace=True)
    n_gpu = H.check_fragments(dict(state=st), lists)
    img2, tf2, st2 = pr.rasterize_forward(x, f, o, s.cam, 1e-4, mode)
    bw = torch.full((s.n,), float("nan"), dtype=torch.float32, device=H.DEV)
    gf, go = pr.rasterize_backward(x, f, o, st2, H.to_dev(s.g_img), None, bw)
    torch.cuda.synchronize()
    H.check_blend_weight(bw.cpu().numpy(), lists, s.opa, n_gpu)
