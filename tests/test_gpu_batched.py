"""GPU parity of the batched path: many views of uneven size and point count
in one launch sequence, per-view results against the per-view oracle; view
aliasing with gradient folding; HIP-graph replay against eager runs; the
autotuner."""

import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2403_16862_amd as pr
import workloads
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _views_scene(seed, sizes, counts, F=8, shared=False):
    rng = np.random.default_rng(seed)
    cams, xs, offs = [], [], []
    off = 0
    for v, ((W, Hh), n) in enumerate(zip(sizes, counts)):
        cam0 = workloads.canonical_camera(W, Hh)
        if not shared or v == 0:
            pts = workloads.scenes.cluster_points(rng, n, 16, cam0)
            xs.append(pts)
        eye = rng.uniform(-0.3, 0.3, 3)
        target = np.array([0.0, 0.0, 5.0]) + rng.uniform(-0.5, 0.5, 3)
        cams.append(workloads.look_at_camera(eye, target, (0, -1, 0), W, Hh))
        offs.append(0 if shared else off)
        off += n
    xyz = np.concatenate(xs).astype(np.float32)
    N = xyz.shape[0]
    feat = rng.uniform(0, 1, (N, F)).astype(np.float32)
    opa = rng.uniform(0.01, 0.99, N).astype(np.float32)
    counts = [N] * len(sizes) if shared else list(counts)
    return xyz, feat, opa, cams, offs, counts


def _check_batched(xyz, feat, opa, cams, offs, counts, bf16=False, tau=1e-4, tuning_id=-1, seed=0):
    views = pr.make_views(cams, offs, counts)
    P_v = [c.width * c.height for c in cams]
    pix_off = np.concatenate([[0], np.cumsum(P_v)]).astype(np.int64)
    vp_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    rng = np.random.default_rng(seed + 7)
    g_img = rng.normal(size=(int(pix_off[-1]), feat.shape[1])).astype(np.float32)
    x, o = H.to_dev(xyz), H.to_dev(opa)
    f = H.to_dev(feat).to(torch.bfloat16) if bf16 else H.to_dev(feat)
    step = pr.BatchedStep(x, f, o, views, H.to_dev(g_img), tau, "save", tuning_id)
    step.run()
    torch.cuda.synchronize()
    keys, ids, nb = pr.debug_fragments(step.state())
    img = step.image.cpu().numpy()
    tf = step.t_final.cpu().numpy()
    gf = step.grad_feat.cpu().numpy()
    go = step.grad_opa.cpu().numpy()
    ofeat_all = H.bf16_bits(feat) if bf16 else feat
    pix = keys >> np.uint64(32)
    for v, cam in enumerate(cams):
        sl = slice(offs[v], offs[v] + counts[v])
        L = oracle.fragments(xyz[sl], cam)
        lo, hi = int(pix_off[v]), int(pix_off[v + 1])
        sel = (pix >= lo) & (pix < hi)
        assert np.array_equal(keys[sel], L.keys(lo)), f"view {v} keys"
        assert np.array_equal(ids[sel].astype(np.int64) - 4 * int(vp_off[v]), L.ids.astype(np.int64)), \
            f"view {v} ids"
        n_gpu = nb[lo:hi].astype(np.int32)
        ofeat = ofeat_all[sl]
        ref_t = oracle.blend_forward(L, opa[sl], ofeat, tau, want_t_after=True)
        H.termination_ok(L, ref_t["t_after"], n_gpu, ref_t["n_blended"], tau)
        ref = oracle.blend_forward(L, opa[sl], ofeat, tau, n_override=n_gpu)
        e_i = H.rel_err(img[lo:hi], ref["image"])
        e_t = H.rel_err(tf[lo:hi], ref["t_final"])
        assert e_i.max() <= H.REL_TOL and e_t.max() <= H.REL_TOL, (v, e_i.max(), e_t.max())
        rb = oracle.blend_backward(L, opa[sl], ofeat, n_gpu, g_img[lo:hi])
        r0, r1 = int(vp_off[v]), int(vp_off[v + 1])
        H.check_grads(gf[r0:r1], go[r0:r1], rb)
        H.say(f"    view {v}: {cam.width}x{cam.height} N={counts[v]} M={L.m} ok")
    return step, views, g_img


def test_batched_uneven_views_f32():
    sizes = [(64, 48), (97, 61), (33, 129), (150, 40), (1, 1)]
    counts = [20000, 35000, 5000, 60000, 100]
    xyz, feat, opa, cams, offs, counts = _views_scene(1, sizes, counts)
    _check_batched(xyz, feat, opa, cams, offs, counts)


@pytest.mark.parametrize("n_views", [40, 70])
def test_batched_many_small_views(n_views):
    """Up to 64 views the tile emission looks views up in an LDS copy of
    their placement, past that in memory; view points are not aligned to
    blocks, so blocks across two views take the per-thread lookups."""
    rng = np.random.default_rng(100 + n_views)
    sizes = [(int(rng.integers(8, 65)), int(rng.integers(8, 49))) for _ in range(n_views)]
    counts = [int(rng.integers(200, 3000)) for _ in range(n_views)]
    xyz, feat, opa, cams, offs, counts = _views_scene(100 + n_views, sizes, counts)
    _check_batched(xyz, feat, opa, cams, offs, counts)


def test_batched_bf16_and_other_shapes():
    sizes = [(120, 90), (57, 33), (200, 11)]
    counts = [40000, 9000, 15000]
    xyz, feat, opa, cams, offs, counts = _views_scene(2, sizes, counts, F=16)
    for tid in (0, 1, 3):
        _check_batched(xyz, feat, opa, cams, offs, counts, bf16=True, tuning_id=tid)


def test_batched_view_without_points():
    sizes = [(40, 30), (20, 20), (50, 10)]
    counts = [8000, 0, 3000]
    xyz, feat, opa, cams, offs, counts = _views_scene(3, sizes, counts)
    _check_batched(xyz, feat, opa, cams, offs, counts)


def test_aliased_views_fold_gradients():
    # several poses of one shared cloud (as in multi-pose inference); the
    # per-view-point gradients fold onto the points in view order
    sizes = [(80, 60), (64, 64), (100, 50)]
    xyz, feat, opa, cams, offs, counts = _views_scene(4, sizes, [30000] * 3, shared=True)
    step, views, g_img = _check_batched(xyz, feat, opa, cams, offs, counts)
    gf, go = pr.sum_view_grads(views, len(views), xyz.shape[0], step.grad_feat, step.grad_opa)
    torch.cuda.synchronize()
    N = xyz.shape[0]
    exp_f = step.grad_feat.cpu().numpy().reshape(3, N, -1).astype(np.float64).sum(0)
    exp_o = step.grad_opa.cpu().numpy().reshape(3, N).astype(np.float64).sum(0)
    assert np.allclose(gf.cpu().numpy(), exp_f, rtol=1e-6, atol=1e-7)
    assert np.allclose(go.cpu().numpy(), exp_o, rtol=1e-6, atol=1e-7)
    # and through autograd: rasterize_batched folds by itself
    x = H.to_dev(xyz)
    f = H.to_dev(feat).requires_grad_(True)
    o = H.to_dev(opa).requires_grad_(True)
    img, tf = pr.rasterize_batched(x, f, o, views)
    (img * H.to_dev(g_img)).sum().backward()
    torch.cuda.synchronize()
    assert np.array_equal(f.grad.cpu().numpy(), gf.cpu().numpy())
    assert np.array_equal(o.grad.cpu().numpy(), go.cpu().numpy())


def test_graph_replay_matches_eager():
    sizes = [(96, 64), (70, 50), (128, 30)]
    counts = [50000, 20000, 30000]
    xyz, feat, opa, cams, offs, counts = _views_scene(5, sizes, counts, F=16)
    views = pr.make_views(cams, offs, counts)
    rng = np.random.default_rng(0)
    P = sum(c.width * c.height for c in cams)
    g = H.to_dev(rng.normal(size=(P, 16)).astype(np.float32))
    step = pr.BatchedStep(H.to_dev(xyz), H.to_dev(feat).to(torch.bfloat16), H.to_dev(opa), views, g)
    step.run()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (step.image, step.t_final, step.grad_feat, step.grad_opa)]
    step.capture()
    scratch = torch.empty(1 << 20, device="cuda:0")
    for r in range(4):
        for t in (step.image, step.t_final, step.grad_feat, step.grad_opa):
            t.fill_(float("nan"))
        scratch.normal_()                       # unrelated eager work between replays
        torch.cuda.synchronize()
        step.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, (step.image, step.t_final, step.grad_feat, step.grad_opa)):
            assert torch.equal(a, b), f"replay {r} differs from the eager run"


def test_autotune_records_choice(tmp_path):
    sizes = [(96, 64), (70, 50)]
    counts = [40000, 20000]
    xyz, feat, opa, cams, offs, counts = _views_scene(6, sizes, counts, F=16)
    views = pr.make_views(cams, offs, counts)
    P = sum(c.width * c.height for c in cams)
    g = H.to_dev(np.random.default_rng(1).normal(size=(P, 16)).astype(np.float32))
    cache = str(tmp_path / "tune.json")
    best, ms = pr.autotune(H.to_dev(xyz), H.to_dev(feat), H.to_dev(opa), views, g_img=g, repeats=2,
                           cache_path=cache)
    assert 0 <= best < len(pr.tuning_table()) and ms > 0
    d = json.load(open(cache))
    assert best in d.values()
    assert pr.lib().inpc_tuning_for(views, len(views), xyz.shape[0], 16, 0) == best
    assert pr.load_tuning(cache) >= 0
    _check_batched(xyz, feat, opa, cams, offs, counts)   # default (tuned) choice is still exact
