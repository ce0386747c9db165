"""FP64 oracle of the per-point appearance step (Section 3.3).

TEST INFRASTRUCTURE ONLY: imported by tests/ (and the smoke check); the
product path never imports it.

Each point carries 1 + 36 raw values.  The first is turned into the opacity
alpha_h = 1 - exp(-exp(x)) (the activation of Section 3.3).  The other 36 are
the coefficients of real spherical harmonics of degree 2 (9 basis functions)
for 4 output channels; evaluated at the point's viewing direction they give
the point's 4-D view-dependent feature.

Readings (the paper gives no formulas for these):
* viewing direction: the world-space unit vector from the camera centre
  o = -R^T t to the point (the zero vector for a point at the centre, which
  keeps its gradient finite; such a point is never rendered);
* coefficient layout: raw[1 + 4*j + c] multiplies basis function j for
  channel c (the 4 channels of one basis function are adjacent);
* basis: the real spherical harmonics obtained from the complex ones with the
  Condon-Shortley phase as sqrt(2) Re Y_l^m (m > 0), Y_l^0, sqrt(2) Im Y_l^|m|
  (m < 0), in the order (l, m) = (0,0), (1,-1), (1,0), (1,1), (2,-2), (2,-1),
  (2,0), (2,1), (2,2) -- the convention of common graphics SH code;
* no activation on the SH output.

The gradient with respect to the raw values follows by the chain rule; point
positions get no gradient (positions are sampled, Section 3.2).
"""

from __future__ import annotations

import math

import numpy as np

N_SH = 9          # degree-2 basis functions
N_OUT = 4         # output feature channels
N_RAW = 1 + N_SH * N_OUT


def opacity(x: np.ndarray) -> np.ndarray:
    """alpha_h = 1 - exp(-exp(x)), written as -expm1(-exp(x)) to keep small values exact."""
    return -np.expm1(-np.exp(np.asarray(x, np.float64)))


def opacity_grad(x: np.ndarray) -> np.ndarray:
    """d alpha_h / dx = exp(x) exp(-exp(x))."""
    x = np.asarray(x, np.float64)
    return np.exp(x - np.exp(x))


def sh_basis(d: np.ndarray) -> np.ndarray:
    """Real SH of degree <= 2 at unit directions d [n,3] -> [n,9] (FP64)."""
    d = np.asarray(d, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    k0 = 0.5 * math.sqrt(1.0 / pi)
    k1 = math.sqrt(3.0 / (4.0 * pi))
    k2 = math.sqrt(15.0 / (4.0 * pi))
    k20 = math.sqrt(5.0 / (16.0 * pi))
    k22 = math.sqrt(15.0 / (16.0 * pi))
    return np.stack([
        np.full_like(x, k0),
        -k1 * y,
        k1 * z,
        -k1 * x,
        k2 * x * y,
        -k2 * y * z,
        k20 * (3.0 * z * z - 1.0),
        -k2 * x * z,
        k22 * (x * x - y * y),
    ], axis=1)


def camera_centre(cam) -> np.ndarray:
    d = cam.as_dict() if hasattr(cam, "as_dict") else dict(cam)
    R = np.asarray(d["R"], np.float32).astype(np.float64).reshape(3, 3)
    t = np.asarray(d["t"], np.float32).astype(np.float64).reshape(3)
    return -R.T @ t


def directions(xyz: np.ndarray, cam) -> np.ndarray:
    """Unit vectors from the camera centre to the points (zero for a point at the centre)."""
    v = np.asarray(xyz, np.float32).astype(np.float64) - camera_centre(cam)[None, :]
    n = np.linalg.norm(v, axis=1, keepdims=True)
    return np.divide(v, n, out=np.zeros_like(v), where=n > 0)


def forward(xyz: np.ndarray, raw: np.ndarray, cams, offsets, counts):
    """Per view point (views in order, view v = points [offsets[v], +counts[v])
    seen by cams[v]): opacity [n_vp] and feature [n_vp, 4]."""
    raw = np.asarray(raw, np.float32).astype(np.float64)
    opa, feat = [], []
    for cam, o, c in zip(cams, offsets, counts):
        sl = slice(int(o), int(o) + int(c))
        Y = sh_basis(directions(xyz[sl], cam))                  # [n,9]
        coef = raw[sl, 1:].reshape(-1, N_SH, N_OUT)             # [n,9,4]
        feat.append(np.einsum("nj,njc->nc", Y, coef))
        opa.append(opacity(raw[sl, 0]))
    return np.concatenate(opa), np.concatenate(feat).reshape(-1, N_OUT)


def backward(xyz: np.ndarray, raw: np.ndarray, cams, offsets, counts, g_opa: np.ndarray,
             g_feat: np.ndarray) -> np.ndarray:
    """Gradient of L = <g_opa, opacity> + <g_feat, feature> with respect to
    the raw values [N, 37]; view points of one point add up."""
    raw = np.asarray(raw, np.float32).astype(np.float64)
    N = raw.shape[0]
    g = np.zeros((N, N_RAW))
    vp = 0
    for cam, o, c in zip(cams, offsets, counts):
        o, c = int(o), int(c)
        sl = slice(o, o + c)
        Y = sh_basis(directions(xyz[sl], cam))
        gf = np.asarray(g_feat[vp:vp + c], np.float64)
        g[sl, 0] += np.asarray(g_opa[vp:vp + c], np.float64) * opacity_grad(raw[sl, 0])
        g[sl, 1:] += (Y[:, :, None] * gf[:, None, :]).reshape(c, N_SH * N_OUT)
        vp += c
    return g
