"""Synthetic scenes (points, features, opacities, cameras, upstream grads).

Every array is drawn in float64 from ``numpy.random.Generator(PCG64(seed))``
and cast to float32.  Draw order inside a scene is fixed: clusters, points,
features, opacity, upstream gradients.

Workloads (sizes follow the paper's inference and training workloads: 1-2 MP
images and 4M-33M points per sampled cloud, Table 1 and Section 4.1):

* config 1 -- 4,096 points uniform in [-1,1]^3 shifted to z=+3, 128x128 image,
  f=128, F=4, forward only.
* config 2 -- 1M points, 64 anisotropic Gaussian clusters, 1280x720, F=8.
* config 3 -- 8M points, 256 clusters, 1920x1080, F=16, random look-at camera.
* config 4 -- 16 views, 640x360..1920x1080, 0.5M..8M points each, F=16 (stored
  in bfloat16 by the caller).
* config 5 -- 32M points (95% clusters, 5% background shell at radius 50-200),
  1920x1080, F=16, 8 poses on a circle.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

NEAR = 0.01   # near plane used for every scene (Appendix A.2, Scene Normalization)
FAR = 100.0   # far plane used for every scene (Appendix A.2, Scene Normalization)
TAU = 1e-4    # transmittance threshold for early termination (Appendix A.6)


@dataclass
class Camera:
    """Pinhole camera: x_c = R x + t (R row-major 3x3), u = fx*x_c/z_c + cx.

    Pixel (x, y) covers [x, x+1) x [y, y+1); its centre is (x+0.5, y+0.5).
    """

    R: np.ndarray            # float32 [3,3], world -> camera
    t: np.ndarray            # float32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = NEAR
    far: float = FAR

    def as_dict(self) -> dict:
        return dict(R=np.asarray(self.R, np.float32).reshape(9).tolist(),
                    t=np.asarray(self.t, np.float32).reshape(3).tolist(),
                    fx=float(np.float32(self.fx)), fy=float(np.float32(self.fy)),
                    cx=float(np.float32(self.cx)), cy=float(np.float32(self.cy)),
                    width=int(self.width), height=int(self.height),
                    near=float(np.float32(self.near)), far=float(np.float32(self.far)))


@dataclass
class Scene:
    xyz: np.ndarray                 # float32 [N,3]
    feat: np.ndarray                # float32 [N,F]
    opa: np.ndarray                 # float32 [N], already-activated alpha_h in [0,1]
    cam: Camera
    tau: float = TAU
    g_img: Optional[np.ndarray] = None   # float32 [H,W,F]
    g_t: Optional[np.ndarray] = None     # float32 [H,W]
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def F(self) -> int:
        return int(self.feat.shape[1])


@dataclass
class BatchedScene:
    """Several views; view v renders points [point_offset[v], +point_count[v])."""

    xyz: np.ndarray
    feat: np.ndarray
    opa: np.ndarray
    cams: List[Camera]
    point_offset: List[int]
    point_count: List[int]
    tau: float = TAU
    g_imgs: List[np.ndarray] = field(default_factory=list)
    name: str = ""

    @property
    def F(self) -> int:
        return int(self.feat.shape[1])


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def canonical_camera(width: int, height: int, hfov_deg: float = 60.0) -> Camera:
    """Camera at the origin looking down +z, +y pointing down the image."""
    f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return Camera(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32),
                  fx=float(np.float32(f)), fy=float(np.float32(f)),
                  cx=float(np.float32(width / 2.0)), cy=float(np.float32(height / 2.0)),
                  width=width, height=height)


def look_at_camera(eye, target, up, width: int, height: int, hfov_deg: float = 60.0) -> Camera:
    """Camera at ``eye`` looking at ``target``; ``up`` is the world direction
    that should appear at the top of the image (image +y points the other way).
    """
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    down = -np.asarray(up, np.float64)
    right = np.cross(down, fwd)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ eye
    base = canonical_camera(width, height, hfov_deg)
    return Camera(R=_f32(R), t=_f32(t), fx=base.fx, fy=base.fy, cx=base.cx, cy=base.cy,
                  width=width, height=height)


def cluster_points(rng: np.random.Generator, n: int, n_clusters: int, cam0: Camera) -> np.ndarray:
    """Mixture of anisotropic Gaussian clusters placed inside ``cam0``'s frustum.

    Cluster depth is log-uniform in [0.5, 100] (density proportional to 1/d),
    its screen position uniform over the image; axis standard deviations are
    0.02*d*exp(U(-1.5,1.5)) along a random rotation.
    """
    return sample_mixture(rng, cluster_mixture(rng, n_clusters, cam0), n)


def cluster_mixture(rng: np.random.Generator, n_clusters: int, cam0: Camera):
    """The cluster parameters of ``cluster_points`` (drawn first, in the same order)."""
    d = np.exp(rng.uniform(math.log(0.5), math.log(100.0), n_clusters))
    u = rng.uniform(0.0, cam0.width, n_clusters)
    v = rng.uniform(0.0, cam0.height, n_clusters)
    centres = np.stack([d * (u - cam0.cx) / cam0.fx, d * (v - cam0.cy) / cam0.fy, d], axis=1)
    q = rng.normal(size=(n_clusters, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    rot = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], axis=1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], axis=1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], axis=1),
    ], axis=1)                                           # [K,3,3]
    sigma = 0.02 * d[:, None] * np.exp(rng.uniform(-1.5, 1.5, (n_clusters, 3)))
    return centres, rot, sigma


def sample_mixture(rng: np.random.Generator, mixture, n: int) -> np.ndarray:
    """n points of a cluster mixture: a uniform cluster choice, then a Gaussian draw."""
    centres, rot, sigma = mixture
    n_clusters = centres.shape[0]
    k = rng.integers(0, n_clusters, n)
    nrm = rng.normal(size=(n, 3))
    local = nrm * sigma[k]
    pts = centres[k] + np.einsum("nij,nj->ni", rot[k], local)
    return pts


def _random_look_at(rng: np.random.Generator, width: int, height: int) -> Camera:
    eye = rng.uniform(-0.5, 0.5, 3)
    target = np.array([0.0, 0.0, 5.0]) + rng.uniform(-1.0, 1.0, 3)
    return look_at_camera(eye, target, (0.0, -1.0, 0.0), width, height)


def config1(seed: int = 0) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = rng.uniform(-1.0, 1.0, (4096, 3)) + np.array([0.0, 0.0, 3.0])
    feat = rng.uniform(0.0, 1.0, (4096, 4))
    opa = rng.uniform(0.05, 0.95, 4096)
    cam = Camera(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), fx=128.0, fy=128.0,
                 cx=64.0, cy=64.0, width=128, height=128)
    return Scene(_f32(xyz), _f32(feat), _f32(opa), cam, name="config1")


def _cluster_scene(seed: int, n: int, n_clusters: int, width: int, height: int, F: int,
                   feat_kind: str, look_at: bool, grads: bool, g_t: bool, name: str) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    cam0 = canonical_camera(width, height)
    xyz = cluster_points(rng, n, n_clusters, cam0)
    if feat_kind == "uniform":
        feat = rng.uniform(0.0, 1.0, (n, F))
    else:
        feat = np.clip(rng.normal(0.5, 0.2, (n, F)), 0.0, 1.0)
    opa = rng.uniform(0.01, 0.99, n)
    cam = _random_look_at(rng, width, height) if look_at else cam0
    g_img = _f32(rng.normal(size=(height, width, F))) if grads else None
    gt = _f32(rng.normal(size=(height, width))) if (grads and g_t) else None
    return Scene(_f32(xyz), _f32(feat), _f32(opa), cam, g_img=g_img, g_t=gt, name=name)


def config2(seed: int = 1, n: int = 1_000_000, g_t: bool = False) -> Scene:
    return _cluster_scene(seed, n, 64, 1280, 720, 8, "uniform", False, True, g_t, "config2")


def config3(seed: int = 2, n: int = 8_000_000, width: int = 1920, height: int = 1080,
            grads: bool = True) -> Scene:
    return _cluster_scene(seed, n, 256, width, height, 16, "normal", True, grads, False, "config3")


def config4(seed: int = 3, n_views: int = 16, n_min: float = 0.5e6, n_max: float = 8e6,
            grads: bool = True) -> BatchedScene:
    """Views of uneven size and point count; each view draws its own points.

    View v uses seed 1000*4 + v; the view list itself (sizes, counts) uses ``seed``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.uniform(0.0, 1.0, n_views)
    counts = np.round(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_views))).astype(np.int64)
    xyz_l, feat_l, opa_l, cams, g_l = [], [], [], [], []
    offs = []
    off = 0
    for v in range(n_views):
        W = int(round(640 + 1280 * s[v]))
        H = int(round(360 + 720 * s[v]))
        vr = np.random.Generator(np.random.PCG64(1000 * 4 + v))
        cam0 = canonical_camera(W, H)
        pts = cluster_points(vr, int(counts[v]), 256, cam0)
        feat = np.clip(vr.normal(0.5, 0.2, (int(counts[v]), 16)), 0.0, 1.0)
        opa = vr.uniform(0.01, 0.99, int(counts[v]))
        cams.append(_random_look_at(vr, W, H))
        if grads:
            g_l.append(_f32(vr.normal(size=(H, W, 16))))
        xyz_l.append(pts)
        feat_l.append(feat)
        opa_l.append(opa)
        offs.append(off)
        off += int(counts[v])
    return BatchedScene(_f32(np.concatenate(xyz_l)), _f32(np.concatenate(feat_l)),
                        _f32(np.concatenate(opa_l)), cams, offs, [int(c) for c in counts],
                        g_imgs=g_l, name="config4")


def config5(seed: int = 4, n: int = 32_000_000, n_poses: int = 8, far: float = FAR) -> BatchedScene:
    """32M points seen from 8 poses on a circle; all views alias one point cloud."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W, H = 1920, 1080
    n_shell = n // 20
    n_clu = n - n_shell
    cam0 = canonical_camera(W, H)
    pts = cluster_points(rng, n_clu, 256, cam0)
    dirs = rng.normal(size=(n_shell, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    rad = rng.uniform(50.0, 200.0, n_shell)
    xyz = np.concatenate([pts, dirs * rad[:, None]])
    feat = np.clip(rng.normal(0.5, 0.2, (n, 16)), 0.0, 1.0)
    opa = rng.uniform(0.01, 0.99, n)
    cams = []
    for i in range(n_poses):
        th = 2.0 * math.pi * i / n_poses
        c = look_at_camera((0.5 * math.cos(th), 0.0, 0.5 * math.sin(th)), (0.0, 0.0, 10.0),
                           (0.0, -1.0, 0.0), W, H)
        c.far = far
        cams.append(c)
    return BatchedScene(_f32(xyz), _f32(feat), _f32(opa), cams, [0] * n_poses, [n] * n_poses,
                        name="config5")


def multisample_clouds(seed: int = 6, n_per_cloud: int = 1_000_000, n_clouds: int = 4, width: int = 1280,
                       height: int = 720, F: int = 4) -> BatchedScene:
    """K point clouds drawn independently from one cluster mixture (256
    clusters, as in the full-size scene) and seen by one look-at camera: the
    inference-time multisampling of Section 3.2 (the paper uses 4 clouds and
    4-D features).  Features U(0,1), opacity U(0.01,0.99)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cam0 = canonical_camera(width, height)
    mix = cluster_mixture(rng, 256, cam0)
    xyz = np.concatenate([sample_mixture(rng, mix, n_per_cloud) for _ in range(n_clouds)])
    n = n_per_cloud * n_clouds
    feat = rng.uniform(0.0, 1.0, (n, F))
    opa = rng.uniform(0.01, 0.99, n)
    cam = _random_look_at(rng, width, height)
    return BatchedScene(_f32(xyz), _f32(feat), _f32(opa), [cam], [k * n_per_cloud for k in range(n_clouds)],
                        [n_per_cloud] * n_clouds, name="multisample")


def sh_raw(rng: np.random.Generator, n: int) -> np.ndarray:
    """Raw appearance rows [n, 37] float32 for the appearance step: an opacity
    logit x ~ N(-0.5, 1.5) (so 1 - exp(-exp(x)) covers (0, 1)), then degree-2
    SH coefficients (basis-major, 4 channels): band 0 ~ U(0, 2) (a positive
    base colour after the 0.282 basis value), bands 1 and 2 ~ N(0, 0.3)."""
    logit = rng.normal(-0.5, 1.5, (n, 1))
    dc = rng.uniform(0.0, 2.0, (n, 4))
    hi = rng.normal(0.0, 0.3, (n, 32))
    return _f32(np.concatenate([logit, dc, hi], axis=1))


def make_config(k: int, **kw):
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}[k](**kw)
