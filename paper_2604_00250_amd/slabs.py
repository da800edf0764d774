"""Whole-volume fitting as overlapping z-slabs (Sec. 2.5).

The paper fits a whole brain as 30-slice slabs with a 5-slice overlap, each
slab an independent problem with its own calibration, and blends the slab
maps where they overlap.  Here every slab is one group of a single batched
problem, so one launch of the fused pass serves all slabs per iteration, and
the blend runs on the GPU (prism_stitch_maps).

    fit = SlabFit(group, thickness=30, overlap=5)
    fit.run(iterations=100, lr=1e-2)
    maps = fit.maps()          # [P][V] device tensor in the volume's raster order

Layout: slabs start every thickness - overlap slices until one reaches the
end of the volume; the last one stops at the volume's edge and may be
thinner (the paper gives only the thickness and the overlap).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .problem import DeviceState, Problem

CAL_KEYS = ("bias", "alpha", "beta", "sigma_log")


def slab_ranges(nz: int, thickness: int = 30, overlap: int = 5) -> list:
    """[(first slice, slices)] of the slabs along z."""
    if thickness < 1 or overlap < 0 or 2 * overlap > thickness:
        raise ValueError("need thickness >= 1 and 0 <= 2 overlap <= thickness")
    out = [(0, min(thickness, nz))]
    while out[-1][0] + thickness < nz:
        z = out[-1][0] + thickness - overlap
        out.append((z, min(thickness, nz - z)))
    return out


def split_into_slabs(group, ranges) -> list:
    """The group cut into z-slabs: each slab keeps the voxels, measurements and
    micro-structure parameters of its slices and starts from a copy of the
    group's calibration vector (a slab fits its own calibration)."""
    z = group.coords[:, 2]
    out = []
    for a, t in ranges:
        sel = (z >= a) & (z < a + t)
        th = {k: (np.array(v, copy=True) if k in CAL_KEYS else np.asarray(v)[..., sel].copy())
              for k, v in group.theta.items()}
        out.append(dataclasses.replace(group, shape=(group.shape[0], group.shape[1], t),
                                       mask=group.mask[:, :, a:a + t].copy(), y=group.y[:, sel].copy(),
                                       theta=th, truth=None))
    return out


class SlabFit:
    """Fit one large group as z-slabs in one batched problem and stitch the maps."""

    def __init__(self, group, thickness: int = 30, overlap: int = 5, launch: Optional[dict] = None,
                 device: str = "cuda:0"):
        self.volume_shape = tuple(group.shape)
        self.ranges = slab_ranges(group.shape[2], thickness, overlap)
        self.slabs = split_into_slabs(group, self.ranges)
        self.prob = Problem(self.slabs, launch=launch)
        self.n_out = self.prob.stitch_plan(self.volume_shape, [a for a, _ in self.ranges])
        self.state = DeviceState(self.prob, ys=[g.y for g in self.slabs], thetas=[g.theta for g in self.slabs],
                                 device=device)

    def run(self, iterations: int, lr: float = 1e-2, optimizer: str = "adam", graph: bool = True):
        from .fit import fit
        return fit(self.state, iterations, lr=lr, optimizer=optimizer, graph=graph)

    def maps(self):
        return self.state.stitch_maps()
