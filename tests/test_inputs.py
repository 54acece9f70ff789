"""The seeded workload generators: shapes, masks, regions and electrode
placement of the benchmark cuboid and of the bidomain-with-bath instance
(no arithmetic of the method here)."""
import numpy as np
import pytest
from scipy import ndimage

import ep_inputs as E


@pytest.mark.parametrize("dx,shape,k", [(0.5, (40, 14, 6), 3), (0.2, (100, 35, 15), 8),
                                        (0.1, (200, 70, 30), 15)])
def test_cuboid_geometry(dx, shape, k):
    inst = E.cuboid(dx, 0.005, t_end=60.0)
    assert inst.n == shape and inst.h == dx and inst.steps == 12000
    assert inst.mask.all() and inst.nt == np.prod(shape)
    assert np.allclose(inst.fibre[..., 0], 1.0) and np.allclose(inst.fibre[..., 1:], 0.0)
    (st,) = inst.stims
    assert tuple(st.lo) == (0, 0, 0) and tuple(st.hi) == (k, k, k)
    # the stimulated cube covers at least 1.5 mm and at most one voxel more
    assert 1.5 - 1e-9 <= k * dx < 1.5 + dx


def test_bidomain_bath_regions():
    inst = E.bidomain_bath(48, steps=0)
    heart, bath = inst.mask.astype(bool), inst.bath.astype(bool)
    assert not (heart & bath).any()
    assert (heart | bath).all()                     # every other voxel conducts
    assert ndimage.label(heart | bath)[1] == 1       # one face-connected domain
    n = inst.n[0]
    for e in inst.electrodes:
        assert all(0 <= c < n for c in e) and bath[tuple(e)]
    ra, la, ll = (np.array(e) for e in inst.electrodes)
    assert np.array_equal(ra + ll, np.full(3, n - 1))   # RA and LL diametrically opposite
    assert inst.sigma_bath > inst.sigma_el              # the bath conducts more
    assert inst.model == "bido" and inst.nt == heart.sum() > 0
