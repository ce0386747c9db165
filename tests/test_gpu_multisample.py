"""GPU parity of multisampled inference (Section 3.2: K sampled point clouds
rendered for one camera, per-pixel mean of the feature images): each sample
against the FP64 oracle with the GPU's blend counts, the mean against the
float64 mean of those samples bit for bit, and against the oracle's mean."""

import numpy as np
import pytest
import torch

import oracle
import paper_2403_16862_amd as pr
import workloads
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _case(xyz, feat, opa, cam, offsets, counts, tau=1e-4, bf16=False):
    K = len(offsets)
    H.say(f"  multisample K={K} counts={list(counts)} {cam.width}x{cam.height} F={feat.shape[1]} bf16={bf16}")
    x, o = H.to_dev(xyz), H.to_dev(opa)
    f = H.to_dev(feat)
    if bf16:
        f = f.to(torch.bfloat16)
    ofeat = H.bf16_bits(feat) if bf16 else feat
    img, tf = pr.multisample(x, f, o, cam, offsets, counts, tau)
    # the same K samples through the batched forward, with their splat lists
    views = pr.make_views([cam] * K, offsets, counts)
    s_img, s_tf, st = pr.rasterize_forward_batched(x, f, o, views, tau, keep_workspace=True)
    torch.cuda.synchronize()
    keys, ids, nb = pr.debug_fragments(st)
    P, F = cam.width * cam.height, feat.shape[1]
    s_img = s_img.cpu().numpy().reshape(K, P, F).astype(np.float64)
    s_tf = s_tf.cpu().numpy().reshape(K, P).astype(np.float64)
    img = img.cpu().numpy().reshape(P, F)
    tf = tf.cpu().numpy().reshape(P)
    # 1. the mean is the float64 mean of the samples, rounded once
    assert np.array_equal(img, (np.sum(s_img, 0) / K).astype(np.float32))
    assert np.array_equal(tf, (np.sum(s_tf, 0) / K).astype(np.float32))
    # 2. every sample matches the oracle run with the GPU's blend counts
    means_img = np.zeros((P, F))
    means_tf = np.zeros(P)
    amb = 0
    for k in range(K):
        sl = slice(int(offsets[k]), int(offsets[k]) + int(counts[k]))
        L = oracle.fragments(xyz[sl], cam)
        n_gpu = nb[k * P:(k + 1) * P].astype(np.int32)
        ref_t = oracle.blend_forward(L, opa[sl], ofeat[sl], tau, want_t_after=True)
        amb += H.termination_ok(L, ref_t["t_after"], n_gpu, ref_t["n_blended"], tau)
        ref = oracle.blend_forward(L, opa[sl], ofeat[sl], tau, n_override=n_gpu)
        e = H.rel_err(s_img[k], ref["image"])
        assert e.max() <= H.REL_TOL, (k, e.max())
        assert H.rel_err(s_tf[k], ref["t_final"]).max() <= H.REL_TOL
        means_img += ref["image"]
        means_tf += ref["t_final"]
    # 3. the mean against the oracle's mean (same counts)
    e_img = H.rel_err(img, means_img / K)
    e_tf = H.rel_err(tf, means_tf / K)
    H.say(f"    ambiguous pixels {amb}; mean image rel err {e_img.max():.3e}, t_final {e_tf.max():.3e}")
    assert e_img.max() <= H.REL_TOL and e_tf.max() <= H.REL_TOL
    # 4. with no ambiguous pixel, the oracle's own multisample agrees too
    if amb == 0:
        ms = oracle.multisample(xyz, ofeat, opa, cam, offsets, counts, tau)
        assert H.rel_err(img, ms["image"]).max() <= H.REL_TOL
    return img, tf


def test_multisample_four_clouds():
    b = workloads.multisample_clouds(n_per_cloud=200_000)
    _case(b.xyz, b.feat, b.opa, b.cams[0], b.point_offset, b.point_count)


def test_multisample_odd_count_ragged_image_bf16():
    b = workloads.multisample_clouds(seed=9, n_per_cloud=30_000, n_clouds=3, width=211, height=97, F=5)
    _case(b.xyz, b.feat, b.opa, b.cams[0], b.point_offset, b.point_count, bf16=True)


def test_multisample_one_cloud_is_plain_forward():
    s = workloads.config1()
    img, tf = _case(s.xyz, s.feat, s.opa, s.cam, [0], [s.n])
    p_img, p_tf, _ = pr.rasterize_forward(H.to_dev(s.xyz), H.to_dev(s.feat), H.to_dev(s.opa), s.cam)
    assert np.array_equal(img, p_img.cpu().numpy().reshape(img.shape))


def test_multisample_empty_and_overlapping_clouds():
    s = workloads.config1()
    _case(s.xyz, s.feat, s.opa, s.cam, [0, 1000, 0, 4096], [4096, 2000, 0, 0])
