"""GPU parity of the tile-list blend (entries per 8x8 or 16x16 tile, 1, 2 or
4 lanes per pixel, chunks staged in LDS) against the FP64 oracle: the splat
lists rebuilt from the device's sorted tile entries are bit-exact, images and
gradients meet the same tolerances as the per-pixel-list path, RECOMPUTE
equals SAVE bit for bit, one lane per pixel equals the one-lane list blend
bit for bit, and batched views and bfloat16 features work."""

import numpy as np
import pytest
import torch

import oracle
import paper_2403_16862_amd as pr
import workloads
from tests import gpu_helpers as H
from tests.test_gpu_parity import _scene_case

pytestmark = pytest.mark.gpu


# tile tunings under test, by a distinctive part of their table name
VARIANTS = ["4096-key tiles, tile-list blend 8x8 (entries", "tile-list blend 16x16", "8x8, 4 lanes/pixel",
            "8x8, 2 lanes/pixel", "fwd 4 lanes/pixel, bwd 1", "fwd 1 lane/pixel, bwd 2"]
ONE_LANE = VARIANTS[:2]


def tile_tunings():
    return [i for i, n in enumerate(pr.tuning_table()) if "tile-list" in n]


def tuning_named(part):
    hits = [i for i, n in enumerate(pr.tuning_table()) if part in n]
    assert len(hits) == 1, (part, hits)
    return hits[0]


def test_tile_tunings_exist():
    assert len(tile_tunings()) >= len(VARIANTS)
    for v in VARIANTS:
        assert "tile-list" in pr.tuning_table()[tuning_named(v)]


@pytest.mark.parametrize("which", VARIANTS)
def test_tile_config2_fwd_bwd_fd(which):
    tid = tuning_named(which)
    s = workloads.config2(n=400_000)
    _scene_case(s.xyz, s.feat, s.opa, s.cam, tuning_id=tid, fd=32)


@pytest.mark.parametrize("which", VARIANTS)
def test_tile_ragged_sizes_and_feature_widths(which):
    tid = tuning_named(which)
    for (W, Hh, F) in [(1, 1, 4), (17, 33, 3), (300, 7, 16), (129, 65, 64), (97, 61, 20)]:
        rng = np.random.default_rng(W * 7 + Hh)
        cam = workloads.canonical_camera(W, Hh)
        n = 20_000
        xyz = workloads.scenes.cluster_points(rng, n, 8, cam).astype(np.float32)
        feat = rng.uniform(0, 1, (n, F)).astype(np.float32)
        opa = rng.uniform(0.05, 0.95, n).astype(np.float32)
        _scene_case(xyz, feat, opa, cam, tuning_id=tid, seed=W)


@pytest.mark.parametrize("which", VARIANTS)
def test_tile_bf16_ragged_feature_widths(which):
    """bfloat16 features of widths without a vector path (3, 20) and a
    compiled one (16) on ragged image sizes."""
    tid = tuning_named(which)
    for (W, Hh, F) in [(37, 23, 3), (211, 97, 20), (64, 64, 16)]:
        rng = np.random.default_rng(W + 31 * Hh)
        cam = workloads.canonical_camera(W, Hh)
        n = 15_000
        xyz = workloads.scenes.cluster_points(rng, n, 6, cam).astype(np.float32)
        feat = rng.uniform(0, 1, (n, F)).astype(np.float32)
        opa = rng.uniform(0.05, 0.95, n).astype(np.float32)
        _scene_case(xyz, feat, opa, cam, tuning_id=tid, seed=W, bf16=True)


@pytest.mark.parametrize("which", VARIANTS)
def test_tile_tau_zero_opaque_and_gt(which):
    tid = tuning_named(which)
    rng = np.random.default_rng(5)
    cam = workloads.canonical_camera(48, 40)
    n = 8000
    xyz = workloads.scenes.cluster_points(rng, n, 4, cam).astype(np.float32)
    opa = rng.uniform(0.2, 0.9, n).astype(np.float32)
    opa[::5] = 1.0
    feat = rng.uniform(0, 1, (n, 4)).astype(np.float32)
    _scene_case(xyz, feat, opa, cam, tau=0.0, tuning_id=tid, g_t=True, fd=16)


@pytest.mark.parametrize("which", VARIANTS)
def test_tile_bf16(which):
    tid = tuning_named(which)
    s = workloads.config2(n=200_000)
    _scene_case(s.xyz, s.feat, s.opa, s.cam, bf16=True, tuning_id=tid)


@pytest.mark.parametrize("which", VARIANTS)
def test_tile_recompute_equals_save(which):
    tid = tuning_named(which)
    s = workloads.config2(n=300_000)
    rng = np.random.default_rng(1)
    g = rng.normal(size=(s.cam.height * s.cam.width, s.F)).astype(np.float32)
    out = []
    for mode in ("save", "recompute"):
        run = H.gpu_forward(s.xyz, s.feat, s.opa, s.cam, mode=mode, tuning_id=tid)
        gf, go = H.gpu_backward(run, g)
        out.append((run["image"].cpu().numpy(), run["t_final"].cpu().numpy(), gf, go))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("which", ONE_LANE)
@pytest.mark.parametrize("mode", ["save", "recompute"])
def test_tile_matches_list_path_closely(which, mode):
    """Same fragments, same per-pixel float32 recurrence as the 1-lane list
    blend: images agree bit for bit with tuning '1 lane/pixel', and so do the
    gradients (the backward's per-splat float64 chain is the same, and both
    paths combine the per-splat records with the same per-point reduction)."""
    one = [i for i, n in enumerate(pr.tuning_table()) if "1 lane/pixel 8x8" in n][0]
    tid = tuning_named(which)
    s = workloads.config2(n=300_000)
    rng = np.random.default_rng(3)
    g = rng.normal(size=(s.cam.height * s.cam.width, s.F)).astype(np.float32)
    a = H.gpu_forward(s.xyz, s.feat, s.opa, s.cam, tuning_id=one, mode=mode)
    b = H.gpu_forward(s.xyz, s.feat, s.opa, s.cam, tuning_id=tid, mode=mode)
    assert torch.equal(a["image"], b["image"]) and torch.equal(a["t_final"], b["t_final"])
    ga, gb = H.gpu_backward(a, g), H.gpu_backward(b, g)
    assert np.array_equal(ga[0], gb[0]) and np.array_equal(ga[1], gb[1])


@pytest.mark.parametrize("which", VARIANTS)
def test_tile_batched_views_graph(which):
    tid = tuning_named(which)
    b = workloads.config4(n_views=4, n_min=1e5, n_max=4e5)
    views = pr.make_views(b.cams, b.point_offset, b.point_count)
    g = np.concatenate([gi.reshape(-1, b.F) for gi in b.g_imgs])
    x, o = H.to_dev(b.xyz), H.to_dev(b.opa)
    f = H.to_dev(b.feat).to(torch.bfloat16)
    step = pr.BatchedStep(x, f, o, views, H.to_dev(g), tuning_id=tid, want_blend_weight=True)
    step.run()
    torch.cuda.synchronize()
    eager = (step.image.clone(), step.grad_feat.clone(), step.grad_opa.clone(), step.blend_weight.clone())
    step.capture()
    for _ in range(2):
        step.replay()
        torch.cuda.synchronize()
        assert torch.equal(step.image, eager[0]) and torch.equal(step.grad_feat, eager[1])
        assert torch.equal(step.grad_opa, eager[2]) and torch.equal(step.blend_weight, eager[3])
    keys, ids, nb = pr.debug_fragments(step.state())
    P_v = [c.width * c.height for c in b.cams]
    pix_off = np.concatenate([[0], np.cumsum(P_v)]).astype(np.int64)
    vp_off = np.concatenate([[0], np.cumsum(b.point_count)]).astype(np.int64)
    pix = keys >> np.uint64(32)
    fbits = H.bf16_bits(b.feat)
    img = step.image.cpu().numpy()
    gf, go = step.grad_feat.cpu().numpy(), step.grad_opa.cpu().numpy()
    bw = step.blend_weight.cpu().numpy()
    for v in range(len(b.cams)):
        sl = slice(b.point_offset[v], b.point_offset[v] + b.point_count[v])
        L = oracle.fragments(b.xyz[sl], b.cams[v])
        lo, hi = int(pix_off[v]), int(pix_off[v + 1])
        sel = (pix >= lo) & (pix < hi)
        assert np.array_equal(keys[sel], L.keys(lo))
        assert np.array_equal(ids[sel].astype(np.int64) - 4 * int(vp_off[v]), L.ids.astype(np.int64))
        n_gpu = nb[lo:hi].astype(np.int32)
        ref = oracle.blend_forward(L, b.opa[sl], fbits[sl], 1e-4, n_override=n_gpu)
        assert H.rel_err(img[lo:hi], ref["image"]).max() <= H.REL_TOL
        rb = oracle.blend_backward(L, b.opa[sl], fbits[sl], n_gpu, g[lo:hi])
        H.check_grads(gf[vp_off[v]:vp_off[v + 1]], go[vp_off[v]:vp_off[v + 1]], rb)
        H.check_blend_weight(bw[vp_off[v]:vp_off[v + 1]], L, b.opa[sl], n_gpu)


# entries per 8x8 tile around the chunk sizes of the tile blends (64 entries
# per chunk with one lane per 8x8 pixel, 256 with 4 lanes or 16x16 tiles)
CHUNK_COUNTS = [1, 63, 64, 65, 127, 128, 129, 255, 256, 257, 513]


def _chunk_boundary_scene(seed):
    """Points placed so that 8x8 tile i of a 96x64 image (first tile row) is
    touched by exactly CHUNK_COUNTS[i] points, every 2x2 footprint inside its
    tile; the other tiles are empty.  Checked against the oracle's splats."""
    W, Hh = 96, 64
    cam = workloads.canonical_camera(W, Hh)
    rng = np.random.default_rng(seed)
    pts = []
    for i, n in enumerate(CHUNK_COUNTS):
        u = i * 8 + rng.uniform(1.5, 6.5, n)
        v = rng.uniform(1.5, 6.5, n)
        z = rng.uniform(2.0, 10.0, n)
        pts.append(np.stack([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z], 1))
    xyz = np.concatenate(pts)[rng.permutation(sum(CHUNK_COUNTS))].astype(np.float32)
    pix, _, ids, _ = oracle.emit(xyz, cam)
    tile = (pix // W // 8) * (W // 8) + (pix % W) // 8
    pairs = np.unique(tile.astype(np.int64) * (1 << 32) + ids // 4)
    counts = np.bincount(pairs >> 32, minlength=(W // 8) * (Hh // 8))
    assert list(counts[:len(CHUNK_COUNTS)]) == CHUNK_COUNTS and not counts[len(CHUNK_COUNTS):].any()
    return xyz, cam


@pytest.mark.parametrize("which", VARIANTS)
def test_tile_chunk_boundaries(which):
    """Tiles whose entry counts sit on, just below and just above multiples
    of the chunk size (the prefetch of the next chunk's view points and rows
    clamps its indices at the tile's end), with faint splats (every chunk is
    walked) and with dense ones (pixels terminate inside the tile)."""
    tid = tuning_named(which)
    xyz, cam = _chunk_boundary_scene(11)
    rng = np.random.default_rng(12)
    n = xyz.shape[0]
    feat = rng.uniform(0, 1, (n, 16)).astype(np.float32)
    for lo, hi in [(0.01, 0.05), (0.3, 0.95)]:
        opa = rng.uniform(lo, hi, n).astype(np.float32)
        _scene_case(xyz, feat, opa, cam, tuning_id=tid, seed=int(100 * hi), g_t=True)


@pytest.mark.parametrize("which", ONE_LANE)
def test_tile_chunk_boundaries_match_list_path(which):
    one = [i for i, n in enumerate(pr.tuning_table()) if "1 lane/pixel 8x8" in n][0]
    tid = tuning_named(which)
    xyz, cam = _chunk_boundary_scene(13)
    rng = np.random.default_rng(14)
    n = xyz.shape[0]
    feat = rng.uniform(0, 1, (n, 16)).astype(np.float32)
    opa = rng.uniform(0.01, 0.3, n).astype(np.float32)
    g = rng.normal(size=(cam.height * cam.width, 16)).astype(np.float32)
    a = H.gpu_forward(xyz, feat, opa, cam, tuning_id=one)
    b = H.gpu_forward(xyz, feat, opa, cam, tuning_id=tid)
    assert torch.equal(a["image"], b["image"]) and torch.equal(a["t_final"], b["t_final"])
    ga, gb = H.gpu_backward(a, g), H.gpu_backward(b, g)
    assert np.array_equal(ga[0], gb[0]) and np.array_equal(ga[1], gb[1])
