"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs (plain single-view calls)."""

import numpy as np
import pytest

import oracle
import workloads
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _scene_case(xyz, feat, opa, cam, tau=1e-4, grads=True, seed=0, mode="save", bf16=False,
                tuning_id=-1, fd=0, g_t=False):
    H.say(f"  case N={xyz.shape[0]} F={feat.shape[1]} {cam.width}x{cam.height} tau={tau} mode={mode} "
          f"bf16={bf16} tuning={tuning_id}")
    lists = oracle.fragments(xyz, cam)
    run = H.gpu_forward(xyz, feat, opa, cam, tau, mode, tuning_id, bf16)
    ofeat = H.bf16_bits(feat) if bf16 else feat
    ref_n = oracle.blend_forward(lists, opa, ofeat, tau, want_t_after=True)
    n_gpu = H.check_fragments(run, lists) if mode == "save" else None
    if n_gpu is None:
        n_gpu = ref_n["n_blended"]
    amb = H.termination_ok(lists, ref_n["t_after"], n_gpu, ref_n["n_blended"], tau)
    H.say(f"    M={lists.m} blended={int(n_gpu.sum())} ambiguous pixels={amb}")
    H.check_image(run, lists, opa, ofeat, tau, n_gpu)
    if not grads:
        return run, lists, n_gpu
    rng = np.random.default_rng(seed + 100)
    P = lists.P
    g_img = rng.normal(size=(P, feat.shape[1])).astype(np.float32)
    gt = rng.normal(size=P).astype(np.float32) if g_t else None
    gf, go = H.gpu_backward(run, g_img, gt)
    ref = oracle.blend_backward(lists, opa, ofeat, n_gpu, g_img, gt)
    H.check_grads(gf, go, ref)
    if fd:
        H.fd_check(lists, opa, ofeat if not bf16 else (ofeat.astype(np.uint32) << 16).view(np.float32),
                   n_gpu, g_img, gt, gf, go, n_check=fd, seed=seed)
    return run, lists, n_gpu


def test_config1_forward():
    s = workloads.config1()
    _scene_case(s.xyz, s.feat, s.opa, s.cam, grads=False)


def test_config1_forward_backward_all_tunings():
    import paper_2403_16862_amd as pr
    s = workloads.config1()
    for tid in range(len(pr.tuning_table())):
        _scene_case(s.xyz, s.feat, s.opa, s.cam, tuning_id=tid)


def test_config2_fwd_bwd_with_fd():
    s = workloads.config2()
    _scene_case(s.xyz, s.feat, s.opa, s.cam, fd=64)


def test_config2_with_transmittance_grad():
    s = workloads.config2(n=200_000, g_t=True)
    _scene_case(s.xyz, s.feat, s.opa, s.cam, g_t=True, fd=16)


@pytest.mark.parametrize("F", [1, 3, 5, 8, 16, 20, 32, 64])
def test_feature_widths(F):
    rng = np.random.default_rng(F)
    s = workloads.config3(n=60_000, width=97, height=61, grads=False)
    feat = rng.uniform(0, 1, (s.n, F)).astype(np.float32)
    _scene_case(s.xyz, feat, s.opa, s.cam, seed=F)


@pytest.mark.parametrize("W,H", [(1, 1), (1, 37), (53, 1), (17, 9), (129, 65), (300, 7)])
def test_ragged_image_sizes(W, H):
    rng = np.random.default_rng(W * 1000 + H)
    cam = workloads.canonical_camera(W, H)
    n = 3000
    s = workloads.scenes.cluster_points(rng, n, 8, cam)
    feat = rng.uniform(0, 1, (n, 4)).astype(np.float32)
    opa = rng.uniform(0.05, 0.95, n).astype(np.float32)
    _scene_case(s.astype(np.float32), feat, opa, cam)


def test_empty_point_cloud():
    cam = workloads.canonical_camera(40, 30)
    z = np.zeros((0, 3), np.float32)
    run = H.gpu_forward(z, np.zeros((0, 4), np.float32), np.zeros(0, np.float32), cam)
    img = run["image"].cpu().numpy()
    assert np.all(img == 0) and np.all(run["t_final"].cpu().numpy() == 1)
    gf, go = H.gpu_backward(run, np.ones((30 * 40, 4), np.float32))
    assert gf.shape == (0, 4) and go.shape == (0,)


def test_everything_culled():
    cam = workloads.canonical_camera(40, 30)
    rng = np.random.default_rng(3)
    xyz = rng.uniform(-1, 1, (5000, 3)).astype(np.float32)
    xyz[:, 2] = -np.abs(xyz[:, 2]) - 0.5      # all behind the camera
    xyz[:100, 2] = 500.0                        # beyond far
    feat = rng.uniform(0, 1, (5000, 4)).astype(np.float32)
    opa = rng.uniform(0, 1, 5000).astype(np.float32)
    run, lists, n = _scene_case(xyz, feat, opa, cam)
    assert lists.m == 0


def test_non_finite_positions_are_culled():
    """Points with NaN or infinite coordinates fail the depth or image test
    of the projection (every comparison with NaN is false) and emit nothing;
    the rest are rasterized as usual."""
    cam = workloads.canonical_camera(40, 30)
    rng = np.random.default_rng(4)
    n = 3000
    xyz = workloads.scenes.cluster_points(rng, n, 4, cam).astype(np.float32)
    xyz[::17, 0] = np.nan
    xyz[5::19, 1] = np.inf
    xyz[7::23, 2] = -np.inf
    xyz[9::29, 2] = np.nan
    feat = rng.uniform(0, 1, (n, 4)).astype(np.float32)
    opa = rng.uniform(0.05, 0.95, n).astype(np.float32)
    run, lists, n_gpu = _scene_case(xyz, feat, opa, cam)
    bad = ~np.isfinite(xyz).all(1)
    assert lists.m > 0 and not np.isin(np.nonzero(bad)[0], lists.ids >> 2).any()


def test_inpc_log_reports_the_choices_of_a_call(capfd, monkeypatch):
    """INPC_LOG set: a forward and its backward each print their tuning, list
    layout and sort passes (here the default tuning: 8x8 tile lists, a 27-bit
    depth key in 3 passes of 9 bits, 2^8 tiles in one pass)."""
    cam = workloads.canonical_camera(128, 128)
    rng = np.random.default_rng(8)
    n = 4000
    xyz = workloads.scenes.cluster_points(rng, n, 4, cam).astype(np.float32)
    feat = rng.uniform(0, 1, (n, 4)).astype(np.float32)
    opa = rng.uniform(0.05, 0.95, n).astype(np.float32)
    monkeypatch.setenv("INPC_LOG", "1")
    capfd.readouterr()
    run = H.gpu_forward(xyz, feat, opa, cam, tuning_id=0)
    H.gpu_backward(run, np.ones((128 * 128, 4), np.float32))
    err = capfd.readouterr().err
    lines = [l for l in err.splitlines() if l.startswith("inpc: ")]
    assert len(lines) == 2 and lines[0].startswith("inpc: forward:") and lines[1].startswith("inpc: backward:")
    for l in lines:
        assert f"{n} view points, 16384 pixels, F=4 float32, save mode; tuning 0" in l
        assert "depth sort 27 bits = 3 pass(es) of 9; tile sort 8 bits = 1 pass(es) of 8" in l


def test_pixel_centres_duplicates_and_opaque_points():
    W, Hh = 32, 24
    cam = workloads.Camera(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), fx=1.0, fy=1.0,
                           cx=0.0, cy=0.0, width=W, height=Hh)
    rng = np.random.default_rng(11)
    n = 4000
    x = rng.integers(0, W, n) + 0.5
    y = rng.integers(0, Hh, n) + 0.5
    frac = rng.random(n) < 0.5                         # half at centres, half anywhere
    x = np.where(frac, x, rng.uniform(-1, W + 1, n))
    y = np.where(frac, y, rng.uniform(-1, Hh + 1, n))
    z = rng.uniform(0.5, 20, n)
    xyz = np.stack([x * z, y * z, z], 1).astype(np.float32)   # projects to about (x, y)
    xyz[200:400] = xyz[:200]                           # exact duplicates: ties broken by index
    feat = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    opa = rng.uniform(0, 1, n).astype(np.float32)
    opa[::7] = 1.0                                     # opaque points
    opa[::11] = 0.0
    for tau in (1e-4, 0.0, 0.5):
        _scene_case(xyz, feat, opa, cam, tau=tau, seed=int(tau * 10))


def test_tau_zero_with_fully_opaque_splats():
    # alpha = 1 splats drive T to exactly 0 while blending continues (tau = 0);
    # the backward must still carry dL/dalpha of the opaque splat.
    W, Hh = 16, 16
    cam = workloads.Camera(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), fx=1.0, fy=1.0,
                           cx=0.0, cy=0.0, width=W, height=Hh)
    rng = np.random.default_rng(5)
    n = 3000
    u = rng.integers(0, W, n) + 0.5
    v = rng.integers(0, Hh, n) + 0.5
    z = rng.uniform(1, 10, n)
    xyz = np.stack([u * z, v * z, z], 1).astype(np.float32)
    opa = rng.uniform(0.2, 0.9, n).astype(np.float32)
    opa[::5] = 1.0
    feat = rng.uniform(0, 1, (n, 4)).astype(np.float32)
    _scene_case(xyz, feat, opa, cam, tau=0.0, g_t=True, fd=32)


def test_bf16_features():
    s = workloads.config2(n=300_000)
    H.say("  bf16 vs oracle on bf16-rounded features")
    run, lists, n_gpu = _scene_case(s.xyz, s.feat, s.opa, s.cam, bf16=True, fd=16)
    ref_unrounded = oracle.blend_forward(lists, s.opa, s.feat, 1e-4, n_override=n_gpu)
    img = run["image"].reshape(-1, s.F).cpu().numpy()
    err = np.abs(img - ref_unrounded["image"])
    H.say(f"    bf16 image abs err vs unrounded features: max {err.max():.3e} "
          f"(bound 2^-9 max|c| = {2.0 ** -9 * float(s.feat.max()):.3e})")
    assert err.max() <= H.BF16_ABS_TOL


def test_recompute_mode_matches_save_mode_bitwise():
    import paper_2403_16862_amd as pr
    s = workloads.config2(n=300_000)
    rng = np.random.default_rng(1)
    g = rng.normal(size=(s.cam.height * s.cam.width, s.F)).astype(np.float32)
    out = []
    for mode in ("save", "recompute"):
        run = H.gpu_forward(s.xyz, s.feat, s.opa, s.cam, mode=mode)
        gf, go = H.gpu_backward(run, g)
        out.append((run["image"].cpu().numpy(), run["t_final"].cpu().numpy(), gf, go))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    _ = pr


def test_deterministic_repeats():
    s = workloads.config2(n=300_000)
    rng = np.random.default_rng(2)
    g = rng.normal(size=(s.cam.height * s.cam.width, s.F)).astype(np.float32)
    outs = []
    for _ in range(2):
        run = H.gpu_forward(s.xyz, s.feat, s.opa, s.cam)
        gf, go = H.gpu_backward(run, g)
        outs.append((run["image"].cpu().numpy(), gf, go))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
