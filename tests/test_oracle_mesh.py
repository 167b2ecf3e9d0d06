"""Mesh pins: counts, Euler characteristic, area, orientation and validity checks."""
import numpy as np
import pytest

import oracle as O
from paper_1708_03183_amd import inputs as I


@pytest.mark.parametrize("n,jit,ren", [(1, 0, None), (4, 0, None), (8, 0.2, 3), (17, 0.2, 5)])
def test_counts_and_euler(n, jit, ren):
    m = I.square_mesh(n, jitter=jit, renumber_seed=ren)
    om = O.OMesh.from_mesh(m)
    assert om.nc == 2 * n * n
    assert om.nf == 3 * n * n - 2 * n
    assert om.nb == 4 * n
    V, E, F = m.nv, om.nf + om.nb, om.nc
    assert V - E + F == 1
    p = m.xy[m.c2v]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    assert np.all(area > 0) and abs(area.sum() - 1.0) < 1e-13
    mp = om.maps()
    # every cell-facet appears exactly once across interior (both sides) and exterior lists
    seen = np.zeros((om.nc, 3), int)
    for (c0, c1), (l0, l1) in zip(mp["f2c"], mp["f2l"]):
        assert c0 < c1
        seen[c0, l0] += 1
        seen[c1, l1] += 1
    for c, l in zip(mp["b2c"], mp["b2l"]):
        seen[c, l] += 1
    assert np.all(seen == 1)
    assert np.all(mp["bside"] >= 0)


def test_periodic_has_no_exterior():
    m = I.square_mesh(6, periodic=3)
    om = O.OMesh.from_mesh(m)
    assert om.nb == 0 and om.nf == 3 * om.nc // 2


def test_invalid_meshes_rejected():
    m = I.square_mesh(2)
    bad = m.c2v.copy()
    bad[0] = bad[0][::-1]  # clockwise
    with pytest.raises(ValueError):
        O.OMesh(m.xy, bad)
    # an edge shared by three cells
    xy = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [0.5, -1]], float)
    c2v = np.array([[0, 1, 2], [1, 3, 2], [0, 4, 1]], np.int32)
    O.OMesh(xy, c2v)  # valid: edge (0,1) shared by two cells
    c2v3 = np.array([[0, 1, 2], [1, 3, 2], [0, 4, 1], [1, 0, 4]], np.int32)
    with pytest.raises(ValueError):
        O.OMesh(xy, c2v3)
