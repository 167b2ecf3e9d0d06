"""GPU parity of chains fused over several time steps (dgt_solver_fuse_steps).

The chain handed to the inspector repeats the step's loops for F steps, so a
sub-chain can run loops of two steps in one tile pass.  Checked: the GPU schedule
of the fused chain is byte-equal to the oracle's; fused tiled runs (chain kernel
for two whole second-order steps and for a stress half fused with the next
velocity half, the generic kernel for three second-order steps, the matrix-core
kernel at P3/P4 on operators of the second step) match the oracle's untiled steps
within 1e-12 (FP64) and 1e-5 (FP32) under both schedules, with the source in the
mesh so that each step's own source time is exercised; a step count that is not a
multiple of F and a batch of fused solvers are refused.
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


def _pair(D, n, k, order, prec=0):
    m = I.square_mesh(n, jitter=0.2, renumber_seed=6)
    lam, mu, rho = I.lognormal_material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    od = O.ODG(om, k, lam, mu, rho, flux=1, order=order, dt=dt, free_sides=0x8)
    gd = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=k, flux=1, time_order=order, precision=prec,
                  free_sides=0x8, dt=dt)
    return m, om, od, gd


@pytest.mark.parametrize("order,steps,splits,k", [(2, 2, (), 1), (4, 2, (13, 39), 2), (2, 3, (4, 12), 2)])
def test_fused_schedule_matches_oracle(D, order, steps, splits, k):
    m, om, od, gd = _pair(D, 12, k, order)
    gd.fuse_steps(steps)
    gd.inspect(10, partition=1, splits=splits)
    gs = gd.schedule()
    os_ = od.chain(steps).inspect(10, partition=1, seed_xy=m.centroids(), splits=splits)
    assert gs.nsub == os_.nsub == len(splits) + 1
    sizes = {0: om.nc, 1: om.nf, 2: om.nb}
    one = ([0, 1, 2, 0] * 3 + [0]) * 2 if order == 4 else [0, 1, 2, 0] * 2
    pat = one * steps
    for sub in range(gs.nsub):
        gi = gs.sub_info(sub)
        assert gi == os_.sub_info(sub)
        assert np.array_equal(gs.colors(sub), os_.colors(sub))
        for j in range(gi["first"], gi["first"] + gi["nloops"]):
            assert np.array_equal(gs.sigma(j), os_.sigma(j, sizes[pat[j]])), j
        for st in range(3):
            for a, b in zip(gs.footprint(sub, st), os_.footprint(sub, st)):
                assert np.array_equal(a, b)
    assert os_.check() == 0


FUSED_CASES = [
    # n, k, order, steps, splits, tile size, schedule, precision, expected kernels per sub-chain
    (12, 1, 2, 2, (), 12, 1, 0, [1]),
    (12, 2, 2, 2, (), 10, 0, 0, [1]),
    (12, 2, 4, 2, (13, 39), 10, 1, 0, [1, 1, 1]),
    (12, 1, 4, 2, (13, 39), 12, 0, 0, [1, 1, 1]),
    (12, 2, 2, 3, (), 8, 0, 0, [0]),
    (10, 3, 4, 2, (4, 8, 13, 17, 21, 26, 30, 34, 39, 43, 47), 8, 0, 0, [2] * 12),
    (10, 4, 4, 2, (13, 26, 39), 8, 0, 0, [2, 2, 2, 2]),
    (12, 2, 4, 2, (13, 39), 12, 1, 1, [1, 1, 1]),
    # every update a sub-chain of its own (generic kernel), the source update in both steps
    (12, 2, 4, 2, (12, 13, 25, 26, 38, 39, 51), 10, 0, 0, [1, 0, 1, 0, 1, 0, 1, 0]),
]


@pytest.mark.parametrize("n,k,order,steps,splits,ts,schedule,prec,kinds", FUSED_CASES)
def test_fused_steps_match_oracle(D, n, k, order, steps, splits, ts, schedule, prec, kinds):
    m, om, od, gd = _pair(D, n, k, order, prec)
    od.set_source(0.43, 0.52, f0=8.0, t0=0.05)
    gd.set_source(0.43, 0.52, 8.0, 0.05, 1.0)
    gd.fuse_steps(steps)
    gd.inspect(ts, partition=1, splits=splits)
    gd.set_schedule(schedule)
    assert gd.kernels() == kinds, gd.kernels()
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, 13)
    s[:] = I.random_state(s.shape, 14)
    dtype = torch.float32 if prec else torch.float64
    gv = torch.from_numpy(v).to(dtype).cuda().contiguous()
    gs = torch.from_numpy(s).to(dtype).cuda().contiguous()
    if prec:
        v, s = v.astype(np.float32).astype(np.float64), s.astype(np.float32).astype(np.float64)
    gd.upload(gv, gs)
    nsteps = 2 * steps
    gd.step(nsteps, mode=1, t0=0.02)
    gd.download(gv, gs)
    od.step(v, s, nsteps, t0=0.02)
    torch.cuda.synchronize()
    hv, hs = gv.double().cpu().numpy(), gs.double().cpu().numpy()
    ref = max(np.abs(v).max(), np.abs(s).max())
    err = max(np.abs(hv - v).max(), np.abs(hs - s).max()) / ref
    l2 = np.sqrt(((hv - v) ** 2).sum() + ((hs - s) ** 2).sum()) / np.sqrt((v ** 2).sum() + (s ** 2).sum())
    print(f"P{k} order {order}, {steps} steps per chain, splits {splits}, kernels {kinds}: "
          f"max-abs {err:.3e}, rel L2 {l2:.3e}")
    tol = 1e-5 if prec else 1e-12
    assert err <= tol and l2 <= tol


def test_fused_argument_checks(D):
    m, om, od, gd = _pair(D, 8, 1, 2)
    with pytest.raises(D.DgtError):
        gd.fuse_steps(0)
    with pytest.raises(D.DgtError):
        gd.fuse_steps(9)  # 72 loops
    gd.fuse_steps(2)
    v, s = gd.zeros()
    gd.upload(v, s)
    with pytest.raises(D.DgtError):  # the fused chain is not inspected yet
        gd.step(2, mode=1)
    gd.inspect(10, partition=1)
    with pytest.raises(D.DgtError):
        gd.step(3, mode=1)
    gd.step(4, mode=1)
    gd.step(3, mode=0)  # the untiled chain runs any number of steps
    with pytest.raises(D.DgtError):
        D.Batch([gd])
