"""Seeded synthetic probability octrees (leaves only) for the sampling step.

A cube of edge ``root_size`` centred at ``origin`` is split into a regular
grid of 2^level0 cells per axis (the initial leaves, Appendix A.4); leaves
near a set of random "surface" points are subdivided further, up to
``max_level``, the way the octree refines around geometry.  Leaf
probabilities are high near the surfaces and small elsewhere.  This module
draws random numbers and assembles arrays; it holds none of the sampling
arithmetic.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Octree:
    centre: np.ndarray     # float32 [L, 3]
    level: np.ndarray      # int32 [L]
    prob: np.ndarray       # float32 [L]
    subdiv: np.ndarray     # float32 [L]  (q_i of Eq. 3)
    root_size: float

    @property
    def n(self) -> int:
        return int(self.level.shape[0])


def synthetic_octree(seed: int = 7, level0: int = 6, max_level: int = 9, n_surfaces: int = 48,
                     root_size: float = 16.0, origin=(0.0, 0.0, 6.0), refine_radius: float = 0.3) -> Octree:
    rng = np.random.Generator(np.random.PCG64(seed))
    origin = np.asarray(origin, np.float64)
    surf = origin + rng.uniform(-0.4, 0.4, (n_surfaces, 3)) * root_size
    n0 = 1 << level0
    g = (np.arange(n0) + 0.5) / n0 - 0.5
    cx, cy, cz = np.meshgrid(g, g, g, indexing="ij")
    centre = origin + root_size * np.stack([cx.ravel(), cy.ravel(), cz.ravel()], 1)
    level = np.full(centre.shape[0], level0, np.int64)
    for lv in range(level0, max_level):
        edge = root_size / (1 << lv)
        d = np.min(np.linalg.norm(centre[:, None, :] - surf[None, :, :], axis=2), axis=1) \
            if centre.shape[0] * n_surfaces < 60_000_000 else _min_dist_chunked(centre, surf)
        split = (level == lv) & (d < refine_radius * (max_level - lv))
        if not np.any(split):
            continue
        parents = centre[split]
        offs = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], np.float64)
        kids = (parents[:, None, :] + offs[None] * (edge / 4.0)).reshape(-1, 3)
        centre = np.concatenate([centre[~split], kids])
        level = np.concatenate([level[~split], np.full(kids.shape[0], lv + 1)])
    d = _min_dist_chunked(centre, surf)
    near_surf = np.exp(-(d / refine_radius) ** 2)
    prob = np.clip(near_surf * rng.uniform(0.5, 1.0, centre.shape[0]) + rng.uniform(0.0, 0.02, centre.shape[0]),
                   1e-4, 1.0)
    subdiv = rng.uniform(0.0, 0.3, centre.shape[0])
    perm = rng.permutation(centre.shape[0])        # leaves in no spatial order
    return Octree(centre[perm].astype(np.float32), level[perm].astype(np.int32), prob[perm].astype(np.float32),
                  subdiv[perm].astype(np.float32), float(root_size))


def _min_dist_chunked(centre, surf, chunk=1 << 18):
    out = np.empty(centre.shape[0])
    for s in range(0, centre.shape[0], chunk):
        c = centre[s:s + chunk]
        out[s:s + chunk] = np.min(np.linalg.norm(c[:, None, :] - surf[None, :, :], axis=2), axis=1)
    return out
