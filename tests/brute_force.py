"""Brute-force mini-oracle for tiny scenes (pins the C oracle).

For every pixel it loops over every point, re-derives from scratch whether
the point's 2x2 bilinear footprint (Section 3.4, Eq. 5 and Eq. 6) covers
the pixel and with which weight, orders the covering points by depth, and
blends them with Eq. 1, stopping once T < tau (Appendix A.6).  It shares
no code with oracle.c; only usable for a few hundred points and pixels.
"""

from __future__ import annotations

import numpy as np


def _project_f32(xyz: np.ndarray, cam):
    """float32 projection in the same operation order as the definition."""
    d = cam.as_dict() if hasattr(cam, "as_dict") else dict(cam)
    R = np.asarray(d["R"], np.float32).reshape(3, 3)
    t = np.asarray(d["t"], np.float32)
    f32 = np.float32
    out = []
    for p in range(xyz.shape[0]):
        x, y, z = (f32(xyz[p, 0]), f32(xyz[p, 1]), f32(xyz[p, 2]))
        cam_xyz = []
        for r in range(3):
            acc = f32(R[r, 0] * x)
            acc = f32(acc + f32(R[r, 1] * y))
            acc = f32(acc + f32(R[r, 2] * z))
            acc = f32(acc + t[r])
            cam_xyz.append(acc)
        xc, yc, zc = cam_xyz
        with np.errstate(all="ignore"):
            u = f32(f32(f32(d["fx"]) * f32(xc / zc)) + f32(d["cx"]))
            v = f32(f32(f32(d["fy"]) * f32(yc / zc)) + f32(d["cy"]))
        out.append((xc, yc, zc, u, v))
    return out, d


def covering_points(xyz: np.ndarray, cam):
    """dict pixel -> list of (zbits, id, weight) of every splat landing on it."""
    proj, d = _project_f32(xyz, cam)
    W, H = int(d["width"]), int(d["height"])
    near, far = np.float32(d["near"]), np.float32(d["far"])
    per_pixel = {}
    for py in range(H):
        for px in range(W):
            lst = []
            for p, (xc, yc, zc, u, v) in enumerate(proj):
                if not (zc > near and zc < far):
                    continue
                if not (u > np.float32(-1) and u < np.float32(W + 1)):
                    continue
                if not (v > np.float32(-1) and v < np.float32(H + 1)):
                    continue
                su = np.float32(u - np.float32(0.5))
                sv = np.float32(v - np.float32(0.5))
                x0 = int(np.floor(su))
                y0 = int(np.floor(sv))
                if px not in (x0, x0 + 1) or py not in (y0, y0 + 1):
                    continue
                ax = np.float32(su - np.float32(x0))
                ay = np.float32(sv - np.float32(y0))
                fx_ = ax if px == x0 + 1 else np.float32(np.float32(1) - ax)
                fy_ = ay if py == y0 + 1 else np.float32(np.float32(1) - ay)
                if not (fx_ > 0 and fy_ > 0):
                    continue
                corner = (px - x0) + 2 * (py - y0)
                zbits = int(np.asarray(zc, np.float32).view(np.uint32))
                lst.append((zbits, 4 * p + corner, float(fx_) * float(fy_)))
            if lst:
                per_pixel[py * W + px] = sorted(lst)
    return per_pixel, W, H


def render(xyz, feat, opa, cam, tau):
    """Brute-force image [P,F], t_final [P], n_blended [P] and the sorted (key, id) list."""
    per_pixel, W, H = covering_points(xyz, cam)
    feat = np.asarray(feat, np.float64)
    F = feat.shape[1]
    image = np.zeros((W * H, F))
    t_final = np.ones(W * H)
    n_bl = np.zeros(W * H, np.int64)
    keys, ids = [], []
    for q in sorted(per_pixel):
        T = 1.0
        C = np.zeros(F)
        n = 0
        for zbits, i, w in per_pixel[q]:
            keys.append((q << 32) | zbits)
            ids.append(i)
        for zbits, i, w in per_pixel[q]:
            a = float(opa[i >> 2]) * w
            C += T * a * feat[i >> 2]
            T *= 1.0 - a
            n += 1
            if T < tau:
                break
        image[q] = C
        t_final[q] = T
        n_bl[q] = n
    return dict(image=image, t_final=t_final, n_blended=n_bl,
                keys=np.asarray(keys, np.uint64), ids=np.asarray(ids, np.uint32))
