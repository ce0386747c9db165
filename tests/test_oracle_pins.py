"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: worked
examples (tests/golden), closed forms of Eq. 1 and Eq. 6, invariants
(weights summing to one, partition of unity, occlusion, permutation),
a brute-force per-pixel re-derivation, and exact finite differences.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from tests import brute_force

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cam_of(d):
    return workloads.Camera(R=np.asarray(d["R"], np.float32).reshape(3, 3),
                            t=np.asarray(d["t"], np.float32), fx=d["fx"], fy=d["fy"],
                            cx=d["cx"], cy=d["cy"], width=d["width"], height=d["height"],
                            near=d.get("near", 0.01), far=d.get("far", 100.0))


def ident_cam(W=16, H=16, f=1.0, c=0.0, near=0.01, far=100.0):
    return workloads.Camera(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), fx=f, fy=f,
                            cx=c, cy=c, width=W, height=H, near=near, far=far)


def centre_point(x, y, z=1.0):
    """World point landing on the centre of pixel (x, y) of ident_cam (f=1, c=0, z=1)."""
    return [x + 0.5, y + 0.5, z]


def f32bits(x):
    return int(np.asarray(x, np.float32).view(np.uint32))


# --------------------------------------------------------------------- constants
def test_paper_constants_match_workload_defaults():
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert workloads.scenes.TAU == c["transmittance_threshold"]["value"]
    assert workloads.scenes.NEAR == c["near_plane"]["value"]
    assert workloads.scenes.FAR == c["far_plane"]["value"]


# --------------------------------------------------------------- O1: projection
@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "hand_projection.json")))["cases"],
                         ids=lambda c: c["name"])
def test_hand_worked_projection(case):
    cam = cam_of(case["camera"])
    xyz = np.asarray([case["xyz"]], np.float32)
    pix, zb, ids, w = oracle.emit(xyz, cam)
    W = case["camera"]["width"]
    got = sorted(zip(pix.tolist(), ids.tolist(), w.tolist()))
    exp = sorted((f["pixel"][1] * W + f["pixel"][0], f["corner"], f["weight"]) for f in case["fragments"])
    assert got == exp
    assert all(z == f32bits(np.float32(case["xyz"][2]) + np.float32(case["camera"]["t"][2])) for z in zb)


def test_pixel_centre_lands_wholly_in_that_pixel():
    rng = np.random.default_rng(5)
    W = H = 16
    xs, ys = rng.integers(0, W, 50), rng.integers(0, H, 50)
    xyz = np.asarray([centre_point(x, y) for x, y in zip(xs, ys)], np.float32)
    pix, zb, ids, w = oracle.emit(xyz, ident_cam(W, H))
    assert len(pix) == 50
    assert np.all(w == 1.0)
    assert np.all(pix == ys * W + xs)
    assert np.all(ids == 4 * np.arange(50))   # corner 0 of each point


def test_interior_weights_sum_to_one_exactly():
    # u, v at least one pixel away from the top/left border: 1-a is exact in float32
    rng = np.random.default_rng(6)
    W, H = 64, 48
    n = 2000
    xyz = np.stack([rng.uniform(2, W - 2, n), rng.uniform(2, H - 2, n), np.ones(n)], 1).astype(np.float32)
    pix, zb, ids, w = oracle.emit(xyz, ident_cam(W, H))
    p = ids >> 2
    sums = np.bincount(p, weights=w, minlength=n)
    counts = np.bincount(p, minlength=n)
    assert np.all(sums == 1.0)
    # four splats unless the point sits exactly on a centre row/column
    su = xyz[:, 0] - np.float32(0.5)
    sv = xyz[:, 1] - np.float32(0.5)
    on_col = (su - np.floor(su)) == 0
    on_row = (sv - np.floor(sv)) == 0
    exp = np.where(on_col, 1, 2) * np.where(on_row, 1, 2)
    assert np.array_equal(counts, exp)


def test_weights_match_eq6_distances():
    # alpha factor of pixel i is (1-|u-u_i|)(1-|v-v_i|) with u_i the pixel centre
    rng = np.random.default_rng(7)
    W, H = 32, 32
    xyz = np.stack([rng.uniform(0, W, 500), rng.uniform(0, H, 500), np.ones(500)], 1).astype(np.float32)
    pix, zb, ids, w = oracle.emit(xyz, ident_cam(W, H))
    p = ids >> 2
    u = xyz[p, 0].astype(np.float64)
    v = xyz[p, 1].astype(np.float64)
    cx = (pix % W) + 0.5
    cy = (pix // W) + 0.5
    assert np.all(np.abs(u - cx) < 1) and np.all(np.abs(v - cy) < 1)
    ref = (1 - np.abs(u - cx)) * (1 - np.abs(v - cy))
    assert np.allclose(w, ref, rtol=0, atol=1e-6)


def test_border_points_keep_only_in_image_corners():
    W, H = 16, 16
    pts = [[0.25, 8.5, 1], [15.75, 8.5, 1], [8.5, 0.25, 1], [8.5, 15.75, 1], [0.25, 0.25, 1],
           [15.75, 15.75, 1]]
    pix, zb, ids, w = oracle.emit(np.asarray(pts, np.float32), ident_cam(W, H))
    got = sorted(zip((ids >> 2).tolist(), pix.tolist(), w.tolist()))
    exp = sorted([(0, 8 * W + 0, 0.75), (1, 8 * W + 15, 0.75), (2, 0 * W + 8, 0.75), (3, 15 * W + 8, 0.75),
                  (4, 0, 0.5625), (5, 15 * W + 15, 0.5625)])
    assert got == exp


def test_culling_near_far_guard_and_nonfinite():
    W, H = 16, 16
    cam = ident_cam(W, H, near=0.5, far=10.0)
    pts = [[1.0, 1.0, 0.5],            # z == near: culled (strict)
           [1.0, 1.0, 10.0],           # z == far: culled
           [1.0, 1.0, -2.0],           # behind
           [float("nan"), 1.0, 2.0],
           [float("inf"), 1.0, 2.0],
           [1.0, 1.0, float("nan")],
           [-2.2, 2.0, 2.0],           # u = -1.1: outside the guard
           [34.2, 2.0, 2.0],           # u = 17.1: outside
           [-1.2, 2.0, 2.0],           # u = -0.6: inside the guard but both columns off-image
           [1.0, 1.0, 0.5000001]]      # just inside the near plane: kept
    pix, zb, ids, w = oracle.emit(np.asarray(pts, np.float32), cam)
    assert set((ids >> 2).tolist()) == {9}


def test_depth_bits_order_equals_float_order():
    z = np.sort(np.random.default_rng(0).uniform(0.011, 99.0, 10000).astype(np.float32))
    b = z.view(np.uint32)
    assert np.all(np.diff(b.astype(np.int64)) >= 0)


# ------------------------------------------------------- O2: lists and order
def _random_tiny_scene(seed, n=120, W=12, H=10, dup=True):
    rng = np.random.default_rng(seed)
    cam = workloads.look_at_camera(rng.uniform(-0.2, 0.2, 3), (0, 0, 4), (0, -1, 0), W, H, 70.0)
    xyz = rng.uniform(-1.5, 1.5, (n, 3)) + np.array([0, 0, 4.0])
    if dup:
        xyz[n // 2: n // 2 + 10] = xyz[:10]   # exact duplicates: equal depth, ids decide
    xyz[-3] = [np.nan, 0, 4]
    feat = rng.uniform(0, 1, (n, 3))
    opa = rng.uniform(0.05, 0.95, n)
    opa[5] = 1.0
    opa[6] = 0.0
    return xyz.astype(np.float32), feat.astype(np.float32), opa.astype(np.float32), cam


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("tau", [1e-4, 0.0, 0.3])
def test_oracle_matches_brute_force(seed, tau):
    xyz, feat, opa, cam = _random_tiny_scene(seed)
    L = oracle.fragments(xyz, cam)
    o = oracle.blend_forward(L, opa, feat, tau)
    b = brute_force.render(xyz, feat, opa, cam, tau)
    assert np.array_equal(L.keys(), b["keys"])
    assert np.array_equal(L.ids, b["ids"])
    assert np.array_equal(o["n_blended"], b["n_blended"])
    assert np.allclose(o["image"], b["image"], rtol=1e-13, atol=1e-15)
    assert np.allclose(o["t_final"], b["t_final"], rtol=1e-13, atol=1e-15)


def test_sorted_keys_and_multiset():
    s = workloads.config1()
    L = oracle.fragments(s.xyz, s.cam)
    k = L.keys()
    order = np.lexsort((L.ids, k))
    assert np.array_equal(order, np.arange(L.m))
    pix, zb, ids, w = oracle.emit(s.xyz, s.cam)
    assert np.array_equal(np.sort(ids), np.sort(L.ids))
    emitted = (pix.astype(np.uint64) << np.uint64(32)) | zb.astype(np.uint64)
    assert np.array_equal(np.sort(emitted), np.sort(k))


def test_duplicates_ordered_by_ascending_id():
    W = H = 8
    xyz = np.asarray([[3.3, 4.1, 2.0]] * 5, np.float32) * np.asarray([1, 1, 1], np.float32)
    L = oracle.fragments(xyz, ident_cam(W, H, f=2.0))
    for q in range(L.P):
        seg = L.ids[L.start[q]:L.start[q + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)
    assert L.m > 0


def test_permuting_points_permutes_ids_only():
    s = workloads.config1()
    perm = np.random.default_rng(3).permutation(s.n)
    L0 = oracle.fragments(s.xyz, s.cam)
    L1 = oracle.fragments(s.xyz[perm], s.cam)
    o0 = oracle.blend_forward(L0, s.opa, s.feat, 1e-4)
    o1 = oracle.blend_forward(L1, s.opa[perm], s.feat[perm], 1e-4)
    # depths are distinct in config 1, so lists keep their order and images are bit-identical
    assert np.array_equal(o0["image"], o1["image"])
    assert np.array_equal(o0["t_final"], o1["t_final"])
    mapped = 4 * perm[L1.ids >> 2] + (L1.ids & 3)   # point j of the permuted cloud is point perm[j]
    assert np.array_equal(mapped.astype(np.uint32), L0.ids)


# ------------------------------------------------------------ O3: blending
def _stack(pixel_xy, depths, opas, feats, W=8, H=8):
    """Points stacked on the centre of one pixel at the given depths (one splat each, w = 1)."""
    x, y = pixel_xy
    f = 2.0
    xyz = np.asarray([[(x + 0.5) * d / f, (y + 0.5) * d / f, d] for d in depths], np.float32)
    cam = ident_cam(W, H, f=f)
    return xyz, np.asarray(feats, np.float32), np.asarray(opas, np.float32), cam


def test_stack_points_are_single_full_weight_splats():
    xyz, feat, opa, cam = _stack((3, 2), [1.0, 2.0, 4.0], [0.5] * 3, [[1]] * 3)
    pix, zb, ids, w = oracle.emit(xyz, cam)
    assert np.all(pix == 2 * 8 + 3) and np.all(w == 1.0) and len(pix) == 3


def test_single_splat_closed_form():
    xyz, feat, opa, cam = _stack((1, 1), [2.0], [0.3], [[0.25, 0.75]])
    o = oracle.render(xyz, feat, opa, cam)
    q = 1 * 8 + 1
    assert np.allclose(o["image"].reshape(-1, 2)[q], [np.float32(0.3) * 0.25, np.float32(0.3) * 0.75], rtol=1e-15)
    assert o["t_final"].reshape(-1)[q] == 1 - np.float64(np.float32(0.3))
    assert o["n_blended"][q] == 1
    others = np.delete(np.arange(64), q)
    assert np.all(o["image"].reshape(-1, 2)[others] == 0) and np.all(o["t_final"].reshape(-1)[others] == 1)


def test_two_splats_closed_form_and_gradients():
    af, ab, cf, cb = 0.375, 0.625, 0.5, 0.25   # exact in float32
    # back point listed first in the input: order must come from depth
    xyz, feat, opa, cam = _stack((4, 5), [3.0, 1.5], [ab, af], [[cb], [cf]])
    L = oracle.fragments(xyz, cam)
    o = oracle.blend_forward(L, opa, feat, 1e-4)
    q = 5 * 8 + 4
    assert o["image"][q, 0] == af * cf + (1 - af) * ab * cb
    assert o["t_final"][q] == (1 - af) * (1 - ab)
    g = np.zeros((64, 1), np.float32)
    g[q, 0] = 1.0
    gt = np.zeros(64, np.float32)
    gb = oracle.blend_backward(L, opa, feat, o["n_blended"], g, gt)
    # point 1 is the front one
    assert gb["grad_opa"][1] == cf - ab * cb
    assert gb["grad_opa"][0] == (1 - af) * cb
    assert gb["grad_feat"][1, 0] == af
    assert gb["grad_feat"][0, 0] == (1 - af) * ab
    gt[q] = 1.0
    g[:] = 0
    gb = oracle.blend_backward(L, opa, feat, o["n_blended"], g, gt)
    assert gb["grad_opa"][1] == -(1 - ab)
    assert gb["grad_opa"][0] == -(1 - af)


def test_opaque_front_point_occludes_everything_behind():
    depths = [1.0, 2.0, 3.0, 5.0]
    xyz, feat, opa, cam = _stack((2, 6), depths, [1.0, 0.7, 0.4, 0.9], [[0.3, 0.6], [1, 1], [1, 0], [0, 1]])
    L = oracle.fragments(xyz, cam)
    o = oracle.blend_forward(L, opa, feat, 1e-4)
    q = 6 * 8 + 2
    assert o["image"][q].tolist() == [np.float64(np.float32(0.3)), np.float64(np.float32(0.6))]
    assert o["t_final"][q] == 0.0 and o["n_blended"][q] == 1
    o0 = oracle.blend_forward(L, opa, feat, 0.0)          # no termination: everything blended
    assert o0["n_blended"][q] == 4 and o0["image"][q].tolist() == o["image"][q].tolist()
    rng = np.random.default_rng(0)
    g = rng.normal(size=(64, 2)).astype(np.float32)
    for nb in (o["n_blended"], o0["n_blended"]):
        gb = oracle.blend_backward(L, opa, feat, nb, g, rng.normal(size=64).astype(np.float32))
        assert np.all(gb["grad_feat"][1:] == 0) and np.all(gb["grad_opa"][1:] == 0)


@pytest.mark.parametrize("tau", [1e-4, 0.0])
def test_partition_of_unity(tau):
    s = workloads.config1()
    L = oracle.fragments(s.xyz, s.cam)
    o = oracle.blend_forward(L, s.opa, np.ones((s.n, 1), np.float32), tau)
    assert np.allclose(o["image"][:, 0] + o["t_final"], 1.0, rtol=0, atol=1e-14)


def test_linearity_in_features():
    s = workloads.config1()
    L = oracle.fragments(s.xyz, s.cam)
    rng = np.random.default_rng(1)
    # multiples of 2^-8, so the combination below is exact in float32
    f1 = (rng.integers(0, 256, (s.n, 4)) / 256.0).astype(np.float32)
    f2 = (rng.integers(0, 256, (s.n, 4)) / 256.0).astype(np.float32)
    a, b = 0.25, 2.0
    comb = (a * f1.astype(np.float64) + b * f2.astype(np.float64)).astype(np.float32)
    assert np.array_equal(comb.astype(np.float64), a * f1.astype(np.float64) + b * f2.astype(np.float64))
    o1 = oracle.blend_forward(L, s.opa, f1, 1e-4)["image"]
    o2 = oracle.blend_forward(L, s.opa, f2, 1e-4)["image"]
    oc = oracle.blend_forward(L, s.opa, comb, 1e-4)["image"]
    assert np.allclose(oc, a * o1 + b * o2, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("alpha", [0.1, 0.3, 0.55, 0.8])
def test_equal_splats_terminate_at_first_n_below_tau(alpha):
    tau = 1e-4
    k = 100
    xyz, feat, opa, cam = _stack((0, 0), [1.0 + 0.05 * i for i in range(k)], [alpha] * k, [[1.0]] * k)
    o = oracle.render(xyz, feat, opa, cam, tau)
    a = float(np.float32(alpha))
    n_exp = math.ceil(math.log(tau) / math.log(1 - a))
    assert abs(n_exp - math.log(tau) / math.log(1 - a)) > 1e-6   # not on a rounding boundary
    assert n_exp < k
    assert o["n_blended"][0] == n_exp
    assert o["t_final"].reshape(-1)[0] < tau
    assert o["t_final"].reshape(-1)[0] == pytest.approx((1 - a) ** n_exp, rel=1e-12)


def test_tau_zero_blends_every_splat():
    s = workloads.config1()
    L = oracle.fragments(s.xyz, s.cam)
    o = oracle.blend_forward(L, s.opa, s.feat, 0.0)
    assert np.array_equal(o["n_blended"], np.diff(L.start).astype(np.int32))


def test_bf16_features_are_widened_exactly():
    s = workloads.config1()
    L = oracle.fragments(s.xyz, s.cam)
    bits = (s.feat.view(np.uint32) >> 16).astype(np.uint16)       # truncation: any bf16 pattern
    widened = (bits.astype(np.uint32) << 16).view(np.float32)
    a = oracle.blend_forward(L, s.opa, bits, 1e-4)
    b = oracle.blend_forward(L, s.opa, widened, 1e-4)
    assert np.array_equal(a["image"], b["image"])


# ---------------------------------------------------------- O4/O5: backward
def _loss(L, opa, feat, nb, g, gt):
    o = oracle.blend_forward(L, opa, feat, 0.0, n_override=nb)
    return float(np.sum(o["image"] * g) + np.sum(o["t_final"] * gt))


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_central_differences(seed):
    # L is affine in each point's alpha_h and features when n_blended is held
    # fixed (a point has at most one splat per pixel), so central differences
    # are exact up to rounding.
    xyz, feat, opa, cam = _random_tiny_scene(seed, n=80, W=10, H=9)
    L = oracle.fragments(xyz, cam)
    o = oracle.blend_forward(L, opa, feat, 1e-4)
    rng = np.random.default_rng(seed + 10)
    F = feat.shape[1]
    g = rng.normal(size=(L.P, F)).astype(np.float32)
    gt = rng.normal(size=L.P).astype(np.float32)
    gb = oracle.blend_backward(L, opa, feat, o["n_blended"], g, gt)
    # the oracle takes float32 inputs: perturb by exactly representable steps
    h = 2.0 ** -12
    for p in range(xyz.shape[0]):
        op, om = opa.copy(), opa.copy()
        op[p] += np.float32(h)
        om[p] -= np.float32(h)
        fd = (_loss(L, op, feat, o["n_blended"], g, gt) - _loss(L, om, feat, o["n_blended"], g, gt)) / \
             (float(op[p]) - float(om[p]))
        assert fd == pytest.approx(gb["grad_opa"][p], rel=1e-9, abs=1e-11)
        c = p % F
        fp, fm = feat.copy(), feat.copy()
        fp[p, c] += np.float32(h)
        fm[p, c] -= np.float32(h)
        fd = (_loss(L, opa, fp, o["n_blended"], g, gt) - _loss(L, opa, fm, o["n_blended"], g, gt)) / \
             (float(fp[p, c]) - float(fm[p, c]))
        assert fd == pytest.approx(gb["grad_feat"][p, c], rel=1e-9, abs=1e-11)


def test_backward_dot_product_identity_features():
    # image is jointly linear in all features: <g, J d> = <J^T g, d> exactly
    s = workloads.config1()
    L = oracle.fragments(s.xyz, s.cam)
    o = oracle.blend_forward(L, s.opa, s.feat, 1e-4)
    rng = np.random.default_rng(2)
    g = rng.normal(size=(L.P, 4)).astype(np.float32)
    d = rng.normal(size=(s.n, 4)).astype(np.float32)
    gb = oracle.blend_backward(L, s.opa, s.feat, o["n_blended"], g, None)
    Jd = oracle.blend_forward(L, s.opa, d, 0.0, n_override=o["n_blended"])["image"]
    lhs = float(np.sum(g.astype(np.float64) * Jd))
    rhs = float(np.sum(gb["grad_feat"] * d))
    assert lhs == pytest.approx(rhs, rel=1e-11)


def test_backward_dot_product_identity_opacity():
    s = workloads.config1()
    L = oracle.fragments(s.xyz, s.cam)
    o = oracle.blend_forward(L, s.opa, s.feat, 1e-4)
    rng = np.random.default_rng(3)
    g = rng.normal(size=(L.P, 4)).astype(np.float32)
    gt = rng.normal(size=L.P).astype(np.float32)
    d = rng.normal(size=s.n)
    gb = oracle.blend_backward(L, s.opa, s.feat, o["n_blended"], g, gt)
    h = 2.0 ** -20
    op = (s.opa.astype(np.float64) + h * d).astype(np.float32)
    om = (s.opa.astype(np.float64) - h * d).astype(np.float32)
    dd = (op.astype(np.float64) - om.astype(np.float64)) / 2
    fd = (_loss(L, op, s.feat, o["n_blended"], g, gt) - _loss(L, om, s.feat, o["n_blended"], g, gt)) / 2
    assert fd == pytest.approx(float(np.sum(gb["grad_opa"] * dd)), rel=1e-6)


def test_unsplatted_points_get_exact_zero_gradient():
    xyz, feat, opa, cam = _random_tiny_scene(4)
    xyz[:7, 2] = -5.0                                   # behind the camera
    L = oracle.fragments(xyz, cam)
    o = oracle.blend_forward(L, opa, feat, 1e-4)
    rng = np.random.default_rng(0)
    gb = oracle.blend_backward(L, opa, feat, o["n_blended"], rng.normal(size=(L.P, 3)).astype(np.float32))
    assert np.all(gb["grad_feat"][:7] == 0) and np.all(gb["grad_opa"][:7] == 0)


# ------------------------------------------------ per-point blend weight
def test_blend_weight_single_and_stacked_splats():
    # points on a pixel centre have one splat of weight 1, so b = T alpha
    af, ab = 0.375, 0.625
    xyz, feat, opa, cam = _stack((3, 4), [3.0, 1.5], [ab, af], [[1.0], [1.0]])
    L = oracle.fragments(xyz, cam)
    o = oracle.blend_forward(L, opa, feat, 1e-4)
    b = oracle.blend_weight(L, opa, o["n_blended"])
    assert b[1] == af and b[0] == (1 - af) * ab


def test_blend_weight_bilinear_weighted_closed_form():
    # a lone point at u = 5.75, v = 3.25 (weights 0.1875, 0.0625, 0.5625, 0.1875)
    # is the only splat of its four pixels: b = a * sum_c w_c^2
    xyz = np.asarray([[5.75, 3.25, 1.0]], np.float32)
    cam = ident_cam(16, 16)
    L = oracle.fragments(xyz, cam)
    a = np.float32(0.5)
    o = oracle.blend_forward(L, np.asarray([a]), np.ones((1, 1), np.float32), 1e-4)
    b = oracle.blend_weight(L, np.asarray([a]), o["n_blended"])
    w = np.asarray([0.1875, 0.0625, 0.5625, 0.1875])
    assert b[0] == float(a) * float(np.sum(w * w))


def test_blend_weight_sums_to_coverage_for_centre_points():
    # with every splat at weight 1 the weighted sum is the plain sum, and the
    # blend weights of a pixel add up to 1 - T_final (partition of unity)
    rng = np.random.default_rng(8)
    W = H = 12
    n = 600
    x = rng.integers(0, W, n) + 0.5
    y = rng.integers(0, H, n) + 0.5
    z = 2.0 ** rng.integers(0, 5, n)              # powers of two: x*z/z is exact in float32
    xyz = np.stack([x * z, y * z, z], 1).astype(np.float32)
    cam = ident_cam(W, H)
    L = oracle.fragments(xyz, cam)
    assert np.all(L.w == 1.0)
    opa = rng.uniform(0.05, 0.95, n).astype(np.float32)
    o = oracle.blend_forward(L, opa, np.ones((n, 1), np.float32), 1e-4)
    b = oracle.blend_weight(L, opa, o["n_blended"])
    assert np.sum(b) == pytest.approx(np.sum(1.0 - o["t_final"]), rel=1e-12)


# ------------------------------------------------------------- multisampling
def test_multisample_single_cloud_is_plain_render():
    s = workloads.config1()
    ms = oracle.multisample(s.xyz, s.feat, s.opa, s.cam, [0], [s.n])
    ref = oracle.blend_forward(oracle.fragments(s.xyz, s.cam), s.opa, s.feat, 1e-4)
    assert np.array_equal(ms["image"], ref["image"]) and np.array_equal(ms["t_final"], ref["t_final"])


def test_multisample_two_opaque_clouds_average_not_union():
    # cloud 0: an opaque white point in front; cloud 1: an opaque black point
    # behind it on the same pixel centre.  Each cloud alone covers the pixel,
    # so the mean is 1/2 with T = 0; rendering the union would give 1.
    xyz, feat, opa, cam = _stack((2, 5), [1.0, 2.0], [1.0, 1.0], [[1.0], [0.0]])
    ms = oracle.multisample(xyz, feat, opa, cam, [0, 1], [1, 1])
    q = 5 * 8 + 2
    assert ms["image"][q, 0] == 0.5 and ms["t_final"][q] == 0.0
    other = np.arange(64) != q
    assert np.all(ms["image"][other] == 0) and np.all(ms["t_final"][other] == 1.0)
    union = oracle.blend_forward(oracle.fragments(xyz, cam), opa, feat, 1e-4)
    assert union["image"][q, 0] == 1.0


def test_multisample_closed_form_and_cloud_order():
    a1, a2 = 0.25, 0.75
    c1, c2 = [0.5, 1.0], [1.0, 0.25]
    xyz, feat, opa, cam = _stack((0, 0), [3.0, 1.5], [a1, a2], [c1, c2])
    ms = oracle.multisample(xyz, feat, opa, cam, [0, 1], [1, 1])
    assert np.array_equal(ms["image"][0], [(a1 * c1[0] + a2 * c2[0]) / 2, (a1 * c1[1] + a2 * c2[1]) / 2])
    assert ms["t_final"][0] == ((1 - a1) + (1 - a2)) / 2
    swapped = oracle.multisample(xyz, feat, opa, cam, [1, 0], [1, 1])
    assert np.array_equal(ms["image"], swapped["image"])


def test_multisample_overlapping_clouds_and_repeats():
    # K copies of one cloud average to that cloud's image (up to the rounding
    # of the mean: K * x / K is exact for K a power of two)
    s = workloads.config1()
    one = oracle.multisample(s.xyz, s.feat, s.opa, s.cam, [0], [s.n])
    four = oracle.multisample(s.xyz, s.feat, s.opa, s.cam, [0] * 4, [s.n] * 4)
    assert np.array_equal(one["image"], four["image"]) and np.array_equal(one["t_final"], four["t_final"])


# --------------------------------------------------- appearance (Section 3.3)
from oracle import appearance as A   # noqa: E402


def _unit(rng, n):
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_sh_basis_matches_complex_harmonics_from_scipy():
    # real SH from scipy's complex SH (Condon-Shortley phase included):
    # sqrt(2) Re Y_l^m for m > 0, Y_l^0, sqrt(2) Im Y_l^|m| for m < 0
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(11)
    d = _unit(rng, 500)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    cols = []
    for l in range(3):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            cols.append(np.sqrt(2) * Y.real if m > 0 else (Y.real if m == 0 else np.sqrt(2) * Y.imag))
    ref = np.stack(cols, 1)
    assert np.allclose(A.sh_basis(d), ref, atol=1e-13, rtol=0)


def test_sh_basis_orthonormal_on_the_sphere():
    # Gauss-Legendre in cos(theta) x uniform phi integrates these degree <= 4
    # products exactly
    xg, wg = np.polynomial.legendre.leggauss(8)
    phi = np.arange(16) * (2 * np.pi / 16)
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    w = np.meshgrid(wg, np.full(16, 2 * np.pi / 16), indexing="ij")
    w = (w[0] * w[1]).reshape(-1)
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    Y = A.sh_basis(d)
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(9), atol=1e-13)


def test_sh_addition_theorem_per_band():
    rng = np.random.default_rng(12)
    Y = A.sh_basis(_unit(rng, 100))
    for l, sl in ((0, slice(0, 1)), (1, slice(1, 4)), (2, slice(4, 9))):
        assert np.allclose(np.sum(Y[:, sl] ** 2, 1), (2 * l + 1) / (4 * np.pi), atol=1e-14)


def test_opacity_activation_values_and_slope():
    x = np.array([-40.0, -5.0, np.log(np.log(2.0)), 0.0, 3.0, 40.0])
    a = A.opacity(x)
    assert a[3] == pytest.approx(1 - np.exp(-1), rel=1e-15)
    assert a[2] == pytest.approx(0.5, rel=1e-15)          # exp(x) = ln 2 gives exactly one half
    assert a[0] == pytest.approx(np.exp(-40.0), rel=1e-15)  # tiny opacities keep full precision
    assert a[5] == 1.0 and np.all(np.diff(a) > 0) and np.all((a >= 0) & (a <= 1))
    h = 1e-6
    fd = (A.opacity(x[1:5] + h) - A.opacity(x[1:5] - h)) / (2 * h)
    assert np.allclose(A.opacity_grad(x[1:5]), fd, rtol=1e-8)


def test_appearance_constant_band_and_direction_convention():
    # only the l = 0 coefficients set: the feature is view-independent;
    # only (1,0) set: the feature follows the z component of the direction
    rng = np.random.default_rng(13)
    cam = workloads.canonical_camera(64, 32)
    xyz = (rng.normal(size=(50, 3)) + [0, 0, 5]).astype(np.float32)
    raw = np.zeros((50, A.N_RAW), np.float32)
    raw[:, 1:5] = [1.0, 2.0, -1.0, 0.5]
    _, f = A.forward(xyz, raw, [cam], [0], [50])
    assert np.allclose(f, np.array([1.0, 2.0, -1.0, 0.5]) * 0.5 / np.sqrt(np.pi), rtol=1e-15)
    raw[:] = 0
    raw[:, 1 + 4 * 2] = 1.0                       # basis (1,0), channel 0
    _, f = A.forward(xyz, raw, [cam], [0], [50])
    d = xyz.astype(np.float64) / np.linalg.norm(xyz.astype(np.float64), axis=1, keepdims=True)
    assert np.allclose(f[:, 0], np.sqrt(3 / (4 * np.pi)) * d[:, 2], rtol=1e-14)
    assert np.all(f[:, 1:] == 0)


def test_appearance_backward_is_the_adjoint():
    # <g, J dr> = <J^T g, dr> for random perturbations (J linear in the SH part)
    rng = np.random.default_rng(14)
    cams = [workloads.canonical_camera(64, 32),
            workloads.look_at_camera([0.5, 0.0, -1.0], [0, 0, 5], [0, -1, 0], 64, 32)]
    N = 40
    xyz = (rng.normal(size=(N, 3)) + [0, 0, 5]).astype(np.float32)
    raw = rng.normal(size=(N, A.N_RAW)).astype(np.float32)
    offs, cnts = [0, 10], [30, 30]                 # the views overlap on points 10..29
    go = rng.normal(size=60)
    gf = rng.normal(size=(60, 4))
    g = A.backward(xyz, raw, cams, offs, cnts, go, gf)
    dr = np.zeros((N, A.N_RAW))
    dr[:, 1:] = rng.normal(size=(N, 36)).astype(np.float32)   # the forward reads float32 values
    o0, f0 = A.forward(xyz, raw, cams, offs, cnts)
    # forward is linear in the coefficients: J dr = forward(dr) with zero opacity part
    _, fd = A.forward(xyz, dr.astype(np.float64), cams, offs, cnts)
    lhs = np.sum(gf * fd)
    assert lhs == pytest.approx(np.sum(g[:, 1:] * dr[:, 1:]), rel=1e-12)
    # opacity part by central differences
    h = 1e-3
    rp, rm = raw.astype(np.float64).copy(), raw.astype(np.float64).copy()
    rp[:, 0] += h
    rm[:, 0] -= h
    op = np.concatenate([A.opacity(rp[o:o + c, 0]) for o, c in zip(offs, cnts)])
    om = np.concatenate([A.opacity(rm[o:o + c, 0]) for o, c in zip(offs, cnts)])
    fd_o = np.sum(go * (op - om)) / (2 * h)
    assert fd_o == pytest.approx(np.sum(g[:, 0]), rel=1e-6)


def test_camera_centre_is_the_look_at_eye():
    eye = np.array([0.75, -0.25, -1.5])
    cam = workloads.look_at_camera(eye, [0.0, 0.0, 5.0], [0.0, -1.0, 0.0], 64, 32)
    assert np.allclose(A.camera_centre(cam), eye, atol=1e-6)


# ------------------------------------------- octree sampling (Section 3.2, Eq. 4)
from oracle import sampling as S   # noqa: E402
from workloads.octree import synthetic_octree   # noqa: E402


def test_philox_matches_numpy_bit_generator():
    # numpy's Philox is Philox4x64-10; random_raw() yields the block of counter + 1
    key = (0x243F6A8885A308D3, 0x13198A2E03707344)
    for c0 in (0, 12345, (1 << 64) - 2):
        bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array([c0, 0, 0, 0], np.uint64))
        ref = bg.random_raw(4)
        got = S.philox4x64(np.array([[c0 + 1 & ((1 << 64) - 1), 0, 0, 0]], np.uint64), key)[0]
        assert np.array_equal(got, ref)


def test_mulhi_against_python_integers():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2 ** 63, 1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    for m in (3, 2 ** 40 + 7, 2 ** 64 - 1, S.M0):
        hi, lo = S._mulhilo(a, m)
        for i in range(0, 1000, 97):
            p = int(a[i]) * m
            assert int(hi[i]) == p >> 64 and int(lo[i]) == p & (2 ** 64 - 1)


def test_radical_inverse_matches_scipy_halton():
    from scipy.stats import qmc
    ref = qmc.Halton(d=3, scramble=False).random(200)       # row k is the point of index k
    got = np.stack([S.radical_inverse(np.arange(200), b) for b in (2, 3, 5)], 1)
    assert np.allclose(got, ref, rtol=0, atol=1e-15)
    assert S.radical_inverse(np.array([1, 2, 3, 4]), 2).tolist() == [0.5, 0.25, 0.75, 0.125]


def test_eq4_reweighting_closed_form():
    # one leaf straight ahead of the canonical camera at depth 10.01, level 2:
    # d = |10.01 - 0.01| / 100 = 0.1, factor 2^(2 * 0.5) = 2, p_hat = p / 0.2
    cam = workloads.canonical_camera(64, 64)
    c = np.array([[0.0, 0.0, 10.01]], np.float32)
    ph = S.reweight_view(c, np.array([2]), np.array([0.5], np.float32), 4.0, 0.5, 1e-8, cam)
    d = np.float32(np.abs(np.float32(10.01) - np.float32(0.01)) / np.float32(100.0))
    assert ph[0] == np.float32(np.float32(0.5) / (d * np.float32(2.0)))
    assert abs(float(ph[0]) - 2.5) < 1e-5
    # the global form drops d and visibility: p / 2^(l lambda_l)
    assert S.reweight_global(np.array([2]), np.array([0.5], np.float32), 0.5)[0] == np.float32(0.25)
    # tau_d bounds d from below for a leaf on the near plane
    c2 = np.array([[0.0, 0.0, 0.01]], np.float32)
    ph2 = S.reweight_view(c2, np.array([0]), np.array([1.0], np.float32), 0.5, 0.5, 1e-8, cam)
    assert ph2[0] == np.float32(1.0) / np.float32(1e-8)


def test_leaf_visibility_cases():
    cam = workloads.canonical_camera(64, 32)      # 60 deg horizontal field of view
    cases = {
        (0.0, 0.0, 5.0): True,       # straight ahead
        (0.0, 0.0, -5.0): False,     # behind the camera
        (0.0, 0.0, 0.0): True,       # contains the camera: straddles the near plane
        (40.0, 0.0, 5.0): False,     # far right of the frustum
        (3.5, 0.0, 5.0): True,       # x in [3.0, 4.0] at z = 5.5 reaches inside x < 0.577 z = 3.18
        (3.9, 0.0, 5.0): False,      # x in [3.4, 4.4] stays outside for every z <= 5.5
        (0.0, 0.0, 100.4): True,     # straddles the far plane
        (0.0, 0.0, 101.0): False,    # beyond the far plane
    }
    c = np.array(list(cases), np.float32)
    vis = S.leaf_visible(c, np.zeros(len(cases), np.int32), 1.0, cam)
    assert vis.tolist() == list(cases.values())


def test_integer_cdf_inverse_is_exact():
    ph = np.array([0.0, 1.0, 3.0, 0.0, 4.0], np.float32)
    cdf = S.integer_cdf(ph)
    w = np.diff(np.concatenate([[0], cdf.astype(object)]))
    assert list(w) == [0, 2 ** 35, 3 * 2 ** 35, 0, 2 ** 37]      # max 4 < 2^3: scale 2^(38-3)
    # x spanning [0, 2^64) in equal steps hits each leaf in proportion to its weight
    x = (np.arange(8, dtype=np.uint64) << np.uint64(61))
    assert S.pick_leaves(cdf, x).tolist() == [1, 2, 2, 2, 4, 4, 4, 4]


def test_multinomial_frequencies():
    o = synthetic_octree(seed=3, level0=3, max_level=5, n_surfaces=4, root_size=4.0, origin=(0, 0, 3))
    ph = S.reweight_global(o.level, o.prob, 0.5).astype(np.float64)
    n = 200_000
    blk = S.random_block(np.arange(n), 0, S.STREAM_GLOBAL, (1, 2))
    counts = np.bincount(S.pick_leaves(S.integer_cdf(ph.astype(np.float32)), blk[:, 0]), minlength=o.n)
    expect = n * ph / ph.sum()
    chi2 = np.sum((counts - expect) ** 2 / np.maximum(expect, 1e-9))
    assert chi2 < o.n + 6 * np.sqrt(2 * o.n)          # chi-square with ~L degrees of freedom


def test_view_samples_lie_in_their_leaves_and_the_frustum():
    o = synthetic_octree(seed=4, level0=3, max_level=5, n_surfaces=4, root_size=4.0, origin=(0, 0, 3))
    cam = workloads.look_at_camera([0.3, -0.2, -1.0], [0, 0, 3], [0, -1, 0], 96, 64)
    xyz, leaf, unresolved = S.sample_view(o.centre, o.level, o.prob, o.root_size, 0.5, 1e-8, cam, 20_000,
                                          (5, 6), max_rounds=64)
    assert unresolved == 0 and np.all(S.point_visible(xyz, cam))
    half = S.edge(o.root_size, o.level[leaf]) / 2
    assert np.all(np.abs(xyz - o.centre[leaf]) <= half[:, None] * (1 + 1e-6))
    vis = S.leaf_visible(o.centre, o.level, o.root_size, cam)
    assert np.all(vis[leaf])
    # the index form recomputes the same samples
    sub = np.array([0, 17, 19_999])
    x2, l2, _ = S.sample_view(o.centre, o.level, o.prob, o.root_size, 0.5, 1e-8, cam, 20_000, (5, 6), 64,
                              index=sub)
    assert np.array_equal(x2, xyz[sub]) and np.array_equal(l2, leaf[sub])
    # without re-sampling some samples of partly visible leaves fall outside
    x3, _, _ = S.sample_view(o.centre, o.level, o.prob, o.root_size, 0.5, 1e-8, cam, 20_000, (5, 6), 0)
    assert not np.all(S.point_visible(x3, cam))


def test_global_extraction_counts_and_halton_positions():
    from scipy.stats import qmc
    o = synthetic_octree(seed=5, level0=2, max_level=3, n_surfaces=2, root_size=2.0, origin=(0, 0, 3))
    xyz, leaf, counts = S.sample_global(o.centre, o.level, o.prob, o.root_size, 0.5, 5000, (9, 9))
    assert counts.sum() == 5000 and np.all(np.diff(leaf) >= 0)
    i = int(np.argmax(counts))
    rows = xyz[leaf == i]
    h = qmc.Halton(d=3, scramble=False).random(counts[i] + 1)[1:]
    e = S.edge(o.root_size, o.level[i:i + 1])[0]
    assert np.allclose(rows, o.centre[i] + (h - 0.5) * e, atol=1e-6)


def test_probability_update_eq2_eq3():
    leaf = np.array([0, 0, 2, 0])
    b = np.array([0.25, 0.75, 0.5, 0.125], np.float32)
    p, q = S.update_probabilities(leaf, b, 4, 0.5, np.array([1.0, 0.5, 0.25, 0.125], np.float32),
                                  np.array([0.5, 0.5, 0.5, 1.0], np.float32))
    # leaf 0: max(0.5, 0.75) and max(0.25, 0.75 - 0.125); leaf 1 and 3 decay; leaf 2: max(0.125, 0.5), max(0.25, 0)
    assert p.tolist() == [0.75, 0.25, 0.5, 0.0625]
    assert q.tolist() == [0.625, 0.25, 0.25, 0.5]


# ---- re-sampling predicate (Appendix A.4) and uniform placement in the leaf (Section 3.2)
def _wide_cam(R=None, t=None):
    """W = 64, H = 32 (W != H), f = 32, principal point (32, 16): u = 32 x/z + 32, v = 32 y/z + 16."""
    return workloads.Camera(R=np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32),
                            t=np.zeros(3, np.float32) if t is None else np.asarray(t, np.float32),
                            fx=32.0, fy=32.0, cx=32.0, cy=16.0, width=64, height=32, near=0.01, far=100.0)


def test_point_visible_hand_cases():
    """A sample counts as inside iff near < z < far, 0 <= u < W and 0 <= v < H
    (every u, v below is exact in float32)."""
    from oracle import sampling as S
    f32 = np.float32
    near_up = float(np.nextafter(f32(0.01), f32(1)))
    far_down = float(np.nextafter(f32(100), f32(0)))
    cases = [
        ((0.96875, 0.0, 1.0), True),      # u = 63 = W - 1
        ((1.0, 0.0, 1.0), False),         # u = 64 = W: the right border is outside
        ((-1.0, 0.0, 1.0), True),         # u = 0: the left border is inside
        ((-1.03125, 0.0, 1.0), False),    # u = -1
        ((0.0, 0.46875, 1.0), True),      # v = 31 = H - 1
        ((0.0, 0.5, 1.0), False),         # v = 32 = H (still < W: catches W and H swapped)
        ((0.0, -0.5, 1.0), True),         # v = 0
        ((0.25, -0.1875, 1.0), True),     # u = 40 >= H, v = 10 (catches W and H swapped)
        ((0.0, 0.75, 1.0), False),        # v = 40: H < v < W
        ((0.0, 0.0, 0.01), False),        # z = near exactly
        ((0.0, 0.0, near_up), True),      # just past the near plane
        ((0.0, 0.0, 100.0), False),       # z = far exactly
        ((0.0, 0.0, far_down), True),     # just inside the far plane
        ((1.0, 0.0, -2.0), False),        # behind the camera although u = 16, v = 16 lie in the image
        ((0.0, 0.0, -1.0), False),
        ((float("nan"), 0.0, 1.0), False),
        ((0.0, 0.0, 0.0), False),         # at the camera centre
    ]
    xyz = np.array([c for c, _ in cases], np.float32)
    got = S.point_visible(xyz, _wide_cam())
    assert got.tolist() == [v for _, v in cases]
    # rotation and translation enter as x_c = R x + t (a transposed R or a dropped t fails)
    R = [[0, 0, 1], [0, 1, 0], [-1, 0, 0]]        # x_c = z, z_c = -x
    pts = np.array([[-1.0, 0.0, 0.5], [1.0, 0.0, 0.5], [0.0, 0.0, 0.5]], np.float32)
    assert S.point_visible(pts, _wide_cam(R)).tolist() == [True, False, False]
    assert S.point_visible(pts, _wide_cam(R, t=[0.0, 0.0, 1.0])).tolist() == [True, False, True]


def test_unit24_takes_the_top_24_bits():
    from oracle import sampling as S
    words = np.array([1 << 63, (1 << 64) - 1, (1 << 40) - 1, 1 << 40, 0, 0xABCDEF0000000000,
                      (0x123456 << 40) | 0xFFFFFFFFFF], np.uint64)
    got = S.unit24(words)
    assert got.dtype == np.float32
    assert got.tolist() == [0.5, 1.0 - 2.0 ** -24, 0.0, 2.0 ** -24, 0.0, 0xABCDEF / 2.0 ** 24,
                            0x123456 / 2.0 ** 24]
    rnd = S.random_block(np.arange(50_000), 0, S.STREAM_VIEW, (11, 12))[:, 1]
    u = S.unit24(rnd).astype(np.float64)
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))          # on the 2^-24 grid
    assert u.min() >= 0.0 and u.max() < 1.0 and u.min() < 1e-3 and u.max() > 1 - 1e-3


def test_place_hand_case():
    from oracle import sampling as S
    centre = np.array([[1.0, 2.0, 3.0]], np.float32)
    level = np.array([1], np.int32)                      # edge = 4 * 2^-1 = 2
    frac = np.array([[0.0, 0.5, 0.75]], np.float32)
    assert S._place(centre, level, 4.0, np.array([0]), frac).tolist() == [[0.0, 2.0, 3.5]]


def test_view_samples_are_uniform_inside_the_leaf():
    """Positions fill the leaf uniformly and independently per axis (KS test,
    mean, both halves, no correlation between axes)."""
    from scipy.stats import kstest
    from oracle import sampling as S
    centre = np.array([[0.0, 0.0, 4.0]], np.float32)
    level = np.array([0], np.int32)
    cam = workloads.canonical_camera(64, 64)
    n = 60_000
    xyz, leaf, _ = S.sample_view(centre, level, np.array([1.0], np.float32), 1.0, 0.5, 1e-8, cam, n, (21, 22), 0)
    assert np.all(leaf == 0)
    frac = (xyz.astype(np.float64) - centre[0]) / 1.0 + 0.5
    sd = 1.0 / np.sqrt(12.0 * n)
    for a in range(3):
        f = frac[:, a]
        assert kstest(f, "uniform").pvalue > 1e-4
        assert abs(f.mean() - 0.5) < 5 * sd
        assert abs(np.mean(f < 0.5) - 0.5) < 5 * 0.5 / np.sqrt(n)
        assert f.min() >= 0.0 and f.max() < 1.0
    c = np.corrcoef(frac.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5 / np.sqrt(n))
