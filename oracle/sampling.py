"""Oracle of point sampling from the probability octree (Section 3.2, Eq. 4;
Appendix A.4) and of the probability updates (Section 3.1, Eq. 2 and Eq. 3).

TEST INFRASTRUCTURE ONLY: imported by tests/; the product path never imports it.

The octree is given by its leaves: centre c_i (float32 x3), subdivision level
l_i and probability p_i; a leaf is the axis-aligned cube of edge
root_size * 2^-l_i around c_i.

Readings (where the paper gives no formula):
* visibility of a leaf (Eq. 4's indicator): its cube is not entirely outside
  any of the six half-spaces of the view frustum (near, far, and the four
  planes through the camera centre and the image borders u = 0, u = W,
  v = 0, v = H), tested on the 8 corners in view space;
* d_i = max(|z_view - near| / far, tau_d) with z_view the view-space depth of
  the leaf centre (Appendix A.4), and the level factor 2^(l_i lambda_l) is
  2.0 ** (l * lambda_l) evaluated in double and rounded to float32;
* multinomial sampling with replacement uses integer weights: with m the
  largest re-weighted probability and m < 2^e, w_i = floor(p_hat_i 2^(38-e))
  (so weights below 2^-38 of the largest one vanish), an exact integer CDF,
  and for a 64-bit random x the leaf is the first i with CDF_i > floor(x W / 2^64);
  this keeps every sampling decision exact (the paper notes the numerical
  limits of multinomial sampling and caps the octree at 256^3 leaves);
* random numbers come from Philox4x64-10 (Salmon et al., SC 2011) with key
  (seed0, seed1) and counter (sample, round, stream, 0): stream 1 for
  viewpoint-specific sampling (word 0 picks the leaf, the top 24 bits of
  words 1-3 give the position fractions), stream 2 for the global
  extraction (word 0 picks the leaf);
* a position is c + (f - 0.5) * edge per axis in float32, f in [0, 1);
* a sample is visible (for the re-sampling of Appendix A.4) when
  near < z < far and 0 <= u < W, 0 <= v < H with the rasterizer's own
  projection; an invisible sample is drawn again (next round) up to
  max_rounds times, then kept as it is and counted as unresolved;
  max_rounds = 0 turns re-sampling off (inference with multisampling);
* global extraction: sample counts per leaf from the multinomial draws,
  outputs ordered by leaf, the j-th sample of a leaf (j = 0, 1, ...) at the
  3D Halton point of index j + 1 (bases 2, 3, 5; radical inverses in double,
  rounded to float32);
* probability updates: for a leaf with points, p = max(lambda_u p, max b) and
  q = max(lambda_u q, max b - min b); a leaf without points decays
  (p = lambda_u p, q = lambda_u q).  float32 arithmetic.
"""

from __future__ import annotations

import numpy as np

M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
_MASK32 = np.uint64(0xFFFFFFFF)
STREAM_VIEW, STREAM_GLOBAL = 1, 2
WEIGHT_BITS = 38
MAX_LEAVES = 1 << 24


def _mulhilo(a: np.ndarray, m: int):
    """(hi, lo) 64-bit halves of a * m for uint64 arrays a (schoolbook on 32-bit limbs)."""
    a = a.astype(np.uint64)
    m_lo, m_hi = np.uint64(m & 0xFFFFFFFF), np.uint64(m >> 32)
    a_lo, a_hi = a & _MASK32, a >> np.uint64(32)
    ll = a_lo * m_lo
    lh = a_lo * m_hi
    hl = a_hi * m_lo
    hh = a_hi * m_hi
    mid = (ll >> np.uint64(32)) + (lh & _MASK32) + (hl & _MASK32)
    lo = (ll & _MASK32) | ((mid & _MASK32) << np.uint64(32))
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    return hi, lo


def philox4x64(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x64-10 block function: ctr [n,4] uint64, key (k0, k1) -> [n,4] uint64."""
    c = [np.asarray(ctr[:, i], np.uint64) for i in range(4)]
    k0, k1 = int(key[0]), int(key[1])
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo(c[0], M0)
            hi1, lo1 = _mulhilo(c[2], M1)
            c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
            k0 = (k0 + W0) & 0xFFFFFFFFFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFFFFFFFFFF
    return np.stack(c, axis=1)


def random_block(index: np.ndarray, rnd: int, stream: int, seed) -> np.ndarray:
    idx = np.asarray(index, np.uint64)
    ctr = np.zeros((idx.shape[0], 4), np.uint64)
    ctr[:, 0] = idx
    ctr[:, 1] = np.uint64(rnd)
    ctr[:, 2] = np.uint64(stream)
    return philox4x64(ctr, seed)


def unit24(x: np.ndarray) -> np.ndarray:
    """float32 in [0, 1) from the top 24 bits of a 64-bit word (exact)."""
    return ((x >> np.uint64(40)).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def level_factors(lambda_l: float, n: int = 32) -> np.ndarray:
    return np.array([np.float32(2.0 ** (l * float(lambda_l))) for l in range(n)], np.float32)


def edge(root_size: float, level: np.ndarray) -> np.ndarray:
    return np.ldexp(np.float32(root_size), -np.asarray(level, np.int32)).astype(np.float32)


def _view(R, t, x, y, z):
    """View-space coordinates in float32 with the rasterizer's operation order."""
    xc = ((R[0] * x + R[1] * y) + R[2] * z) + t[0]
    yc = ((R[3] * x + R[4] * y) + R[5] * z) + t[1]
    zc = ((R[6] * x + R[7] * y) + R[8] * z) + t[2]
    return xc, yc, zc


def _cam(cam):
    d = cam.as_dict() if hasattr(cam, "as_dict") else dict(cam)
    R = np.asarray(d["R"], np.float32).reshape(9)
    t = np.asarray(d["t"], np.float32).reshape(3)
    f32 = np.float32
    return (R, t, f32(d["fx"]), f32(d["fy"]), f32(d["cx"]), f32(d["cy"]), int(d["width"]), int(d["height"]),
            f32(d["near"]), f32(d["far"]))


def leaf_visible(centre: np.ndarray, level: np.ndarray, root_size: float, cam) -> np.ndarray:
    R, t, fx, fy, cx, cy, W, H, near, far = _cam(cam)
    c = np.asarray(centre, np.float32)
    h = (edge(root_size, level) * np.float32(0.5)).astype(np.float32)
    Wf, Hf = np.float32(W), np.float32(H)
    outside = np.ones((c.shape[0], 6), bool)       # all corners outside plane k so far
    for corner in range(8):
        sx = h if corner & 1 else -h
        sy = h if corner & 2 else -h
        sz = h if corner & 4 else -h
        x, y, z = c[:, 0] + sx, c[:, 1] + sy, c[:, 2] + sz
        xc, yc, zc = _view(R, t, x, y, z)
        us = fx * xc + cx * zc
        vs = fy * yc + cy * zc
        f = [zc - near, far - zc, us, Wf * zc - us, vs, Hf * zc - vs]
        for k in range(6):
            outside[:, k] &= ~(f[k] > 0)
    return ~np.any(outside, axis=1)


def reweight_view(centre, level, prob, root_size, lambda_l, tau_d, cam) -> np.ndarray:
    """Eq. 4: p_hat = 1_visible p / (d 2^(l lambda_l)), float32."""
    R, t, fx, fy, cx, cy, W, H, near, far = _cam(cam)
    c = np.asarray(centre, np.float32)
    _, _, zc = _view(R, t, c[:, 0], c[:, 1], c[:, 2])
    d = np.maximum(np.abs(zc - near) / far, np.float32(tau_d)).astype(np.float32)
    fl = level_factors(lambda_l)[np.asarray(level, np.int64)]
    ph = (np.asarray(prob, np.float32) / (d * fl)).astype(np.float32)
    return np.where(leaf_visible(c, level, root_size, cam), ph, np.float32(0)).astype(np.float32)


def reweight_global(level, prob, lambda_l) -> np.ndarray:
    fl = level_factors(lambda_l)[np.asarray(level, np.int64)]
    return (np.asarray(prob, np.float32) / fl).astype(np.float32)


def integer_cdf(p_hat: np.ndarray) -> np.ndarray:
    """Inclusive prefix sums (uint64) of the integer weights of the reading above."""
    m = float(np.max(p_hat)) if p_hat.size else 0.0
    if m <= 0.0:
        return np.zeros(p_hat.shape[0], np.uint64)
    _, e = np.frexp(np.float32(m))
    w = np.floor(np.ldexp(p_hat.astype(np.float64), WEIGHT_BITS - int(e))).astype(np.uint64)
    return np.cumsum(w, dtype=np.uint64)


def pick_leaves(cdf: np.ndarray, x: np.ndarray) -> np.ndarray:
    total = int(cdf[-1]) if cdf.size else 0
    hi, _ = _mulhilo(np.asarray(x, np.uint64), total)       # floor(x * total / 2^64)
    return np.searchsorted(cdf, hi, side="right").astype(np.int64)


def point_visible(xyz: np.ndarray, cam) -> np.ndarray:
    R, t, fx, fy, cx, cy, W, H, near, far = _cam(cam)
    p = np.asarray(xyz, np.float32)
    xc, yc, zc = _view(R, t, p[:, 0], p[:, 1], p[:, 2])
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * (xc / zc) + cx
        v = fy * (yc / zc) + cy
    return (zc > near) & (zc < far) & (u >= 0) & (u < np.float32(W)) & (v >= 0) & (v < np.float32(H))


def _place(centre, level, root_size, leaf, frac):
    e = edge(root_size, level[leaf])
    return (centre[leaf] + (frac - np.float32(0.5)) * e[:, None]).astype(np.float32)


def sample_view(centre, level, prob, root_size, lambda_l, tau_d, cam, n, seed, max_rounds, index=None):
    """Viewpoint-specific samples: (xyz [n,3] f32, leaf [n] i64, unresolved count).
    ``index`` restricts the computation to the given sample indices."""
    centre = np.asarray(centre, np.float32)
    level = np.asarray(level, np.int32)
    cdf = integer_cdf(reweight_view(centre, level, prob, root_size, lambda_l, tau_d, cam))
    idx = np.arange(n, dtype=np.int64) if index is None else np.asarray(index, np.int64)
    xyz = np.zeros((idx.size, 3), np.float32)
    leaf = np.full(idx.size, -1, np.int64)
    if cdf.size == 0 or cdf[-1] == 0:
        xyz[:] = np.nan
        return xyz, leaf, int(idx.size)
    todo = np.arange(idx.size)
    rounds = max(int(max_rounds), 1)
    for r in range(rounds):
        blk = random_block(idx[todo], r, STREAM_VIEW, seed)
        lf = pick_leaves(cdf, blk[:, 0])
        frac = np.stack([unit24(blk[:, 1]), unit24(blk[:, 2]), unit24(blk[:, 3])], 1)
        xyz[todo] = _place(centre, level, root_size, lf, frac)
        leaf[todo] = lf
        if max_rounds <= 0:
            todo = todo[:0]
            break
        todo = todo[~point_visible(xyz[todo], cam)]
        if todo.size == 0:
            break
    return xyz, leaf, int(todo.size)


def radical_inverse(k: np.ndarray, b: int) -> np.ndarray:
    """Van der Corput radical inverse of k in base b, in double, digit by digit."""
    k = np.asarray(k, np.int64).copy()
    inv = 1.0 / b
    f = np.full(k.shape, inv)
    r = np.zeros(k.shape)
    while np.any(k > 0):
        r = r + (k % b).astype(np.float64) * f
        k //= b
        f = f * inv
    return r


def sample_global(centre, level, prob, root_size, lambda_l, n, seed):
    """Global extraction: (xyz [n,3] f32 ordered by leaf, leaf [n] i64, counts [L] i64)."""
    centre = np.asarray(centre, np.float32)
    level = np.asarray(level, np.int32)
    cdf = integer_cdf(reweight_global(level, prob, lambda_l))
    blk = random_block(np.arange(n, dtype=np.int64), 0, STREAM_GLOBAL, seed)
    counts = np.bincount(pick_leaves(cdf, blk[:, 0]), minlength=centre.shape[0]).astype(np.int64)
    leaf = np.repeat(np.arange(centre.shape[0]), counts)
    start = np.concatenate([[0], np.cumsum(counts)[:-1]])
    j = np.arange(n) - start[leaf]
    frac = np.stack([radical_inverse(j + 1, b).astype(np.float32) for b in (2, 3, 5)], 1)
    return _place(centre, level, root_size, leaf, frac), leaf, counts


def update_probabilities(leaf, b, n_leaves, lambda_u, prob, subdiv):
    """Eq. 2 and Eq. 3 for one iteration: returns the new (p, q) float32."""
    leaf = np.asarray(leaf, np.int64)
    b = np.asarray(b, np.float32)
    mx = np.full(n_leaves, -np.inf, np.float32)
    mn = np.full(n_leaves, np.inf, np.float32)
    np.maximum.at(mx, leaf, b)
    np.minimum.at(mn, leaf, b)
    lu = np.float32(lambda_u)
    p = (lu * np.asarray(prob, np.float32)).astype(np.float32)
    q = (lu * np.asarray(subdiv, np.float32)).astype(np.float32)
    has = np.isfinite(mx)
    p = np.where(has, np.maximum(p, mx), p).astype(np.float32)
    q = np.where(has, np.maximum(q, (mx - mn).astype(np.float32)), q).astype(np.float32)
    return p, q
