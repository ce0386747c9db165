"""Shared helpers of the GPU parity tests: run the HIP path through the
binding, run the oracle on the same seeded inputs, and compare them with the
stated rules (bit-exact splat lists; 1e-5 relative on float32 outputs with
the termination-ambiguity band; gradient error relative to the oracle's
adjoint)."""

from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
import paper_2403_16862_amd as pr

DEV = "cuda:0"
REL_TOL = 1e-5          # float32 image / transmittance vs the FP64 oracle
BF16_ABS_TOL = 1e-2     # image with bfloat16 features vs FP64 on unrounded features
GRAD_TOL = 1e-3         # gradients, relative to max(|ref|, 1e-3 rms(ref))
BAND = 1e-4             # relative width of the termination-ambiguity band
# Per-point blend weight: float32 T_k carries at most ~2 roundings per splat in
# front of it (product and compensated 1 - alpha); lists end near 70-150 splats
# at tau = 1e-4, so 2e-5 relative bounds it; values below 1e-7 are compared
# with an absolute floor of 1e-12 (float32 spacing there).
BW_TOL = 2e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return t if dtype is None else t.to(dtype)


def bf16_bits(feat_f32: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns of float32 features, rounded to nearest even (torch's rounding)."""
    t = torch.from_numpy(np.ascontiguousarray(feat_f32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def gpu_forward(xyz, feat, opa, cam, tau=1e-4, mode="save", tuning_id=-1, bf16=False):
    x = to_dev(xyz)
    f = to_dev(feat)
    if bf16:
        f = f.to(torch.bfloat16)
    o = to_dev(opa)
    img, tf, st = pr.rasterize_forward(x, f, o, cam, tau, mode, tuning_id, keep_workspace=True)
    torch.cuda.synchronize()
    return dict(x=x, f=f, o=o, image=img, t_final=tf, state=st)


def gpu_backward(run, g_img, g_t=None):
    gi = to_dev(g_img)
    gt = None if g_t is None else to_dev(g_t)
    gf, go = pr.rasterize_backward(run["x"], run["f"], run["o"], run["state"], gi, gt)
    torch.cuda.synchronize()
    return gf.cpu().numpy(), go.cpu().numpy()


def check_fragments(run, lists: oracle.Lists, pixel_offset=0, vp_offset=0, pix_range=None):
    """GPU sorted splat list == oracle list, bit for bit.  Returns n_blended per pixel."""
    keys, ids, nb = pr.debug_fragments(run["state"])
    if pix_range is not None:
        lo, hi = pix_range
        pix = keys >> np.uint64(32)
        sel = (pix >= lo) & (pix < hi)
        keys, ids = keys[sel], ids[sel]
        nb = nb[lo:hi]
    ref_keys = lists.keys(pixel_offset)
    ref_ids = lists.ids.astype(np.int64) + 4 * vp_offset
    assert keys.shape == ref_keys.shape, (keys.shape, ref_keys.shape)
    assert np.array_equal(keys, ref_keys), "sorted keys differ"
    assert np.array_equal(ids.astype(np.int64), ref_ids), "sorted ids differ"
    return nb.astype(np.int32)


def termination_ok(lists: oracle.Lists, t_after: np.ndarray, n_gpu: np.ndarray, n_ref: np.ndarray,
                   tau: float) -> int:
    """Checks every pixel whose GPU blend count differs from the oracle's lies in
    the ambiguity band of the threshold; returns how many such pixels there are."""
    bad = np.nonzero(n_gpu != n_ref)[0]
    for q in bad:
        s, e = int(lists.start[q]), int(lists.start[q + 1])
        n = int(n_gpu[q])
        assert 1 <= n <= e - s, (q, n, e - s)
        last = t_after[s + n - 1]
        if n < e - s:
            assert last < tau * (1 + BAND), (q, last)
        else:
            assert last >= tau * (1 - BAND) or last < tau * (1 + BAND)
        if n >= 2:
            assert t_after[s + n - 2] >= tau * (1 - BAND), (q, t_after[s + n - 2])
    return int(bad.size)


def rel_err(gpu: np.ndarray, ref: np.ndarray, floor=1e-12) -> np.ndarray:
    return np.abs(gpu.astype(np.float64) - ref) / np.maximum(np.abs(ref), floor)


def check_image(run, lists, opa, feat_for_oracle, tau, n_gpu, img_shape_pf=None, tol=REL_TOL,
                pix_slice=None):
    """Image and t_final vs the oracle rerun with the GPU's blend counts."""
    ref = oracle.blend_forward(lists, opa, feat_for_oracle, tau, n_override=n_gpu)
    img = run["image"].reshape(-1, ref["image"].shape[1]).cpu().numpy()
    tf = run["t_final"].reshape(-1).cpu().numpy()
    if pix_slice is not None:
        img, tf = img[pix_slice], tf[pix_slice]
    e_img = rel_err(img, ref["image"])
    e_t = rel_err(tf, ref["t_final"])
    say(f"    image rel err max {e_img.max():.3e} p99.9 {np.quantile(e_img, 0.999):.3e}; "
        f"t_final rel err max {e_t.max():.3e}")
    assert e_img.max() <= tol, e_img.max()
    assert e_t.max() <= tol, e_t.max()
    return ref


def check_blend_weight(bw_gpu: np.ndarray, lists: oracle.Lists, opa: np.ndarray, n_gpu: np.ndarray,
                       tol=BW_TOL):
    """Per-point blend weights vs the oracle run with the GPU's blend counts."""
    ref = oracle.blend_weight(lists, opa, n_gpu)
    bw = bw_gpu.astype(np.float64)
    err = np.abs(bw - ref)
    rel = err / np.maximum(np.abs(ref), 1e-30)
    ok = (rel <= tol) | (err <= 1e-12)
    say(f"    blend weight: {int((ref > 0).sum())} points > 0, max rel err "
        f"{rel[ref > 1e-7].max() if np.any(ref > 1e-7) else 0.0:.3e}")
    assert np.all(ok), (int(np.argmin(ok)), bw[np.argmin(ok)], ref[np.argmin(ok)])
    assert np.all(bw[ref == 0] == 0)
    return ref


def grad_err(gpu: np.ndarray, ref: np.ndarray):
    rms = float(np.sqrt(np.mean(ref.astype(np.float64) ** 2))) if ref.size else 0.0
    den = np.maximum(np.abs(ref), max(1e-3 * rms, 1e-30))
    e = np.abs(gpu.astype(np.float64) - ref) / den
    return e


def check_grads(gf, go, ref, tol=GRAD_TOL):
    if ref["grad_opa"].size == 0:
        assert gf.size == 0 and go.size == 0
        return
    ef = grad_err(gf, ref["grad_feat"])
    eo = grad_err(go, ref["grad_opa"])
    say(f"    grad_feat err max {ef.max():.3e} p99 {np.quantile(ef, 0.99):.3e}; "
        f"grad_opa err max {eo.max():.3e} p99 {np.quantile(eo, 0.99):.3e}")
    assert ef.max() <= tol, ef.max()
    assert eo.max() <= tol, eo.max()
    # points without any splat get exact zeros (checked where the oracle says so)
    zero = np.all(ref["grad_feat"] == 0, axis=1) & (ref["grad_opa"] == 0)
    assert np.all(gf[zero] == 0) and np.all(go[zero] == 0)


def restrict(lists: oracle.Lists, pixels: np.ndarray) -> oracle.Lists:
    """The lists of a subset of pixels (in the given order), as a compact Lists."""
    starts = lists.start[pixels]
    ends = lists.start[pixels + 1]
    lens = ends - starts
    idx = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)]) if len(pixels) else \
        np.zeros(0, np.int64)
    start = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return oracle.Lists(len(pixels), start, lists.zbits[idx], lists.ids[idx], lists.w[idx], lists.n_points)


def fd_check(lists, opa, feat, n_gpu, g_img, g_t, gf, go, n_check=64, seed=0):
    """Central differences of L = <g, image> + <g_T, t_final> on the FP64 oracle
    (termination counts held at the GPU's) for a seeded subset of points with at
    least one blended splat; L is affine in each point's opacity and features,
    so the difference quotient is exact up to rounding."""
    F = feat.shape[1]
    P = lists.P
    g_img = g_img.reshape(P, F)
    g_t = np.zeros(P, np.float32) if g_t is None else g_t.reshape(P)
    pix_of = np.repeat(np.arange(P), np.diff(lists.start))
    rank = np.arange(lists.m) - lists.start[pix_of]
    blended = rank < n_gpu[pix_of]
    pts = np.unique(lists.ids[blended] >> 2)
    rng = np.random.default_rng(seed)
    chosen = rng.choice(pts, size=min(n_check, pts.size), replace=False)
    worst = 0.0
    for p in chosen:
        mine = np.nonzero((lists.ids >> 2) == p)[0]
        pixels = np.unique(pix_of[mine])
        sub = restrict(lists, pixels)
        nsub = n_gpu[pixels]

        def loss(o, f):
            r = oracle.blend_forward(sub, o, f, 0.0, n_override=nsub)
            return float(np.sum(r["image"] * g_img[pixels]) + np.sum(r["t_final"] * g_t[pixels]))

        h = 1e-4
        op, om = opa.copy(), opa.copy()
        op[p] = np.float32(opa[p] + h)
        om[p] = np.float32(opa[p] - h)
        fd_o = (loss(op, feat) - loss(om, feat)) / (float(op[p]) - float(om[p]))
        c = int(rng.integers(0, F))
        fp, fm = feat.copy(), feat.copy()
        fp[p, c] = np.float32(feat[p, c] + 1e-2)
        fm[p, c] = np.float32(feat[p, c] - 1e-2)
        fd_f = (loss(opa, fp) - loss(opa, fm)) / (float(fp[p, c]) - float(fm[p, c]))
        rms_o = float(np.sqrt(np.mean(go.astype(np.float64) ** 2)))
        rms_f = float(np.sqrt(np.mean(gf.astype(np.float64) ** 2)))
        e_o = abs(go[p] - fd_o) / max(abs(fd_o), 1e-3 * rms_o)
        e_f = abs(gf[p, c] - fd_f) / max(abs(fd_f), 1e-3 * rms_f)
        worst = max(worst, e_o, e_f)
        assert e_o <= GRAD_TOL, (p, go[p], fd_o)
        assert e_f <= GRAD_TOL, (p, c, gf[p, c], fd_f)
    say(f"    finite differences on {len(chosen)} points: worst rel err {worst:.3e}")
    return worst
