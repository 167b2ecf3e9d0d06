"""Tiles whose working set exceeds the LDS: the generic executor keeps it in a global
scratch region per workgroup (kernel kind 3), and the results match the FP64 oracle
as the in-LDS tiles do; footprints beyond the addressable 16,383 cells are refused.
"""
import numpy as np
import pytest

import oracle as O
from paper_1708_03183_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_03183_amd import dgtile
    dgtile.lib()
    return dgtile


LARGE_CASES = [
    # n, k, order, precision, tile size, splits, kinds expected
    (24, 2, 4, 0, 600, (13,), [3, 3]),
    (20, 2, 4, 0, 100000, (), [3]),
    (16, 4, 4, 0, 300, (4, 8, 13, 17, 21), [3, 2, 3, 2, 3, 3]),  # the matrix-core kernel fits ops 1 and 3
    (40, 1, 2, 1, 100000, (), [3]),  # one tile of 3,200 cells
    (24, 2, 4, 0, 64, (13,), [1, 1]),  # in LDS, for comparison
]


@pytest.mark.parametrize("n,k,order,prec,ts,splits,kinds", LARGE_CASES)
def test_large_tiles_match_oracle(D, n, k, order, prec, ts, splits, kinds):
    m = I.square_mesh(n, jitter=0.2, renumber_seed=8)
    lam, mu, rho = I.layered_material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    od = O.ODG(om, k, lam, mu, rho, flux=1, order=order, dt=dt, free_sides=0x8)
    od.set_source(0.43, 0.52)
    g = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=k, flux=1, time_order=order, precision=prec,
                 free_sides=0x8, dt=dt)
    g.set_source(0.43, 0.52)
    g.inspect(ts, partition=1, splits=splits)
    assert g.kernels() == kinds, g.kernels()
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, 3)
    s[:] = I.random_state(s.shape, 4)
    dtype = torch.float32 if prec else torch.float64
    gv = torch.from_numpy(v).to(dtype).cuda().contiguous()
    gs = torch.from_numpy(s).to(dtype).cuda().contiguous()
    if prec:
        v, s = v.astype(np.float32).astype(np.float64), s.astype(np.float32).astype(np.float64)
    g.upload(gv, gs)
    g.step(3, mode=1, t0=0.1)
    g.download(gv, gs)
    od.step(v, s, 3, t0=0.1)
    torch.cuda.synchronize()
    hv, hs = gv.double().cpu().numpy(), gs.double().cpu().numpy()
    err = max(np.abs(hv - v).max(), np.abs(hs - s).max()) / max(np.abs(v).max(), np.abs(s).max())
    print(f"P{k} order {order} {'FP32' if prec else 'FP64'} ts={ts} kinds {kinds}: max-abs / max {err:.3e}")
    assert err <= (1e-5 if prec else 1e-12)


def test_footprint_beyond_the_slot_limit_is_refused(D):
    m = I.square_mesh(92, jitter=0.2, renumber_seed=8)  # 16,928 cells in one tile
    lam, mu, rho = I.layered_material(m)
    g = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=1, flux=1, time_order=2, precision=1, free_sides=0x8,
                 dt=1e-4)
    g.inspect(100000, partition=1)
    v, s = g.zeros()
    g.upload(v, s)
    with pytest.raises(D.DgtError) as e:
        g.step(1, mode=1)
    assert e.value.status == D.DGT_EUNSUPPORTED
    g.step(1, mode=0)  # the untiled chain still runs
