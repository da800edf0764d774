"""Host logic of the slab pipeline (CPU): the package's slab layout agrees
with the oracle's independent one, and splitting a group into slabs
partitions its voxels with the measurements and parameters that go with
them."""
import numpy as np
import pytest

import oracle as O
from paper_2604_00250_amd import inputs as I
from paper_2604_00250_amd import slabs as S


@pytest.mark.parametrize("nz", [1, 12, 29, 30, 31, 40, 55, 56, 64, 145, 1023])
@pytest.mark.parametrize("T,ov", [(30, 5), (16, 8), (10, 0), (7, 3)])
def test_slab_ranges_agree_with_the_oracle(nz, T, ov):
    assert S.slab_ranges(nz, T, ov) == O.slab_ranges(nz, T, ov)


def test_split_partitions_voxels_and_keeps_calibration_separate():
    g = I.patch16_hcp().groups[0]
    ranges = S.slab_ranges(g.shape[2], 6, 2)
    parts = S.split_into_slabs(g, ranges)
    z = g.coords[:, 2]
    for (a, t), p in zip(ranges, parts):
        sel = (z >= a) & (z < a + t)
        assert p.shape == (g.shape[0], g.shape[1], t)
        assert p.n_vox == int(sel.sum())
        # the slab's voxels, in its own raster order, are the group's voxels of those slices
        c = g.coords[sel].copy()
        c[:, 2] -= a
        assert np.array_equal(p.coords, c)
        assert np.array_equal(p.y, g.y[:, sel])
        assert np.array_equal(p.theta["v"], g.theta["v"][..., sel])
        assert np.array_equal(p.theta["alpha"], g.theta["alpha"])
        assert p.theta["alpha"] is not g.theta["alpha"]
    cover = sum(((z >= a) & (z < a + t)).astype(int) for a, t in ranges)
    assert cover.min() == 1 and cover.max() == 2
