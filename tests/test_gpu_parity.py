"""GPU parity: libdgtile (HIP, gfx950) against the FP64 CPU oracle.

* the GPU inspector's schedule (colours, tiling functions, iteration lists,
  footprints with loop bits, execution order) is byte-equal to the oracle
  inspector's, for generic chains and for the DG chain;
* the untiled GPU chain and the sparse-tiled fused executor match the oracle
  within 1e-12 (FP64) and 1e-5 (FP32), both in relative L2 and
  in max-abs error relative to the largest reference value; the measured error is
  printed for every case;
* the FP64 energy reduction matches the oracle's energy.
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


def rel_err(a, b):
    """max(relative L2 error, max-abs error relative to max|reference|) over the
    fields: every element is held to the tolerance, not only the global norm."""
    l2 = float(np.sqrt(sum(((x - y) ** 2).sum() for x, y in zip(a, b))) / np.sqrt(sum((y ** 2).sum() for y in b)))
    mx = float(max(np.abs(x - y).max() for x, y in zip(a, b)) / max(np.abs(y).max() for y in b))
    print(f"  [rel L2 {l2:.3e}, rel max-abs {mx:.3e}]")
    return max(l2, mx)


# ------------------------------------------------------------------ inspector

def _compare_schedules(gs, os_, loop_sizes, sets_sizes, nsub):
    assert gs.nsub == os_.nsub == nsub
    for sub in range(nsub):
        gi, oi = gs.sub_info(sub), os_.sub_info(sub)
        assert gi == oi, (gi, oi)
        assert np.array_equal(gs.colors(sub), os_.colors(sub))
        gc, gt = gs.tiles_by_color(sub)
        oc, ot = os_.tiles_by_color(sub)
        assert np.array_equal(gc, oc) and np.array_equal(gt, ot)
        for j in range(gi["first"], gi["first"] + gi["nloops"]):
            assert np.array_equal(gs.sigma(j), os_.sigma(j, loop_sizes[j])), j
            go, git = gs.iters(j, sub)
            oo, oit = os_.iters(j, loop_sizes[j], sub)
            assert np.array_equal(go, oo) and np.array_equal(git, oit), j
        for st in range(len(sets_sizes)):
            g = gs.footprint(sub, st)
            o = os_.footprint(sub, st)
            for a, b in zip(g, o):
                assert np.array_equal(a, b), (sub, st)


def _toy_chain(mod, n=9, seed=3):
    """The vertex/edge/cell program of the paper's running example on a mesh."""
    m = I.square_mesh(n, jitter=0.2, renumber_seed=seed)
    edges = set()
    for c in m.c2v:
        for l in range(3):
            a, b = int(c[l]), int(c[(l + 1) % 3])
            edges.add((min(a, b), max(a, b)))
    e2v = np.array(sorted(edges), np.int32)
    ch = mod()
    E = ch.set(len(e2v))
    Cs = ch.set(m.nc)
    V = ch.set(m.nv)
    em = ch.map(E, V, 2, e2v)
    cm = ch.map(Cs, V, 3, m.c2v)
    ch.loop(E, [(-1, 0, 0), (em, 2, 1)])
    ch.loop(Cs, [(-1, 0, 2), (cm, 2, 1)])
    ch.loop(E, [(-1, 1, 0), (em, 0, 1)])
    xy = 0.5 * (m.xy[e2v[:, 0]] + m.xy[e2v[:, 1]])
    return ch, [len(e2v), m.nc, len(e2v)], [len(e2v), m.nc, m.nv], xy


@pytest.mark.parametrize("ts,part", [(1, 0), (7, 0), (16, 1), (50, 1)])
def test_inspector_toy_chain_matches_oracle(D, ts, part):
    gch, loop_sizes, set_sizes, xy = _toy_chain(D.Chain)
    och, _, _, _ = _toy_chain(O.OChain)
    gs = gch.inspect(ts, partition=part, seed_xy=xy)
    os_ = och.inspect(ts, partition=part, seed_xy=xy)
    _compare_schedules(gs, os_, loop_sizes, set_sizes, 1)
    assert os_.check() == 0


DG_CASES = [
    # n, k, order, flux, free, ts, partition, splits, renumber
    (8, 1, 4, 1, 0x8, 16, 1, (), 7),
    (12, 2, 4, 1, 0x8, 24, 1, (13,), 7),
    (12, 2, 2, 1, 0x0, 10, 0, (), None),
    (16, 1, 4, 0, 0xF, 64, 1, (4, 8, 13, 17, 21), 3),
    (20, 2, 2, 0, 0xF, 32, 1, (), 5),
    (32, 1, 4, 0, 0xF, 256, 0, (), None),
]


def _dg_pair(D, n, k, order, flux, free, ren, prec=0):
    m = I.square_mesh(n, jitter=0.2 if ren is not None else 0.0, renumber_seed=ren)
    lam, mu, rho = I.layered_material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    od = O.ODG(om, k, lam, mu, rho, flux=flux, order=order, dt=dt, free_sides=free)
    gm = D.Mesh.from_mesh(m)
    gd = D.Solver(gm, lam, mu, rho, degree=k, flux=flux, time_order=order, precision=prec, free_sides=free, dt=dt)
    return m, om, od, gm, gd


@pytest.mark.parametrize("n,k,order,flux,free,ts,part,splits,ren", DG_CASES)
def test_dg_schedule_matches_oracle(D, n, k, order, flux, free, ts, part, splits, ren):
    m, om, od, gm, gd = _dg_pair(D, n, k, order, flux, free, ren)
    gd.inspect(ts, partition=part, splits=splits)
    gs = gd.schedule()
    och = od.chain()
    os_ = och.inspect(ts, partition=part, seed_xy=m.centroids(), splits=splits)
    sizes = {0: om.nc, 1: om.nf, 2: om.nb}
    pat = ([0, 1, 2, 0] * 3 + [0]) * 2 if order == 4 else [0, 1, 2, 0] * 2
    _compare_schedules(gs, os_, [sizes[s] for s in pat], [om.nc, om.nf, om.nb], len(splits) + 1)
    assert os_.check() == 0


CAP_CASES = [
    # n, k, order, flux, free, ts, partition, splits, renumber, colour-class cap
    (12, 2, 4, 1, 0x8, 10, 1, (13,), 7, 3),
    (16, 1, 4, 0, 0xF, 16, 1, (), 3, 5),
    (12, 2, 2, 1, 0x8, 8, 0, (), None, 2),
    (20, 2, 4, 1, 0x8, 12, 1, (4, 8, 13, 17, 21), 5, 7),
]


@pytest.mark.parametrize("n,k,order,flux,free,ts,part,splits,ren,cap", CAP_CASES)
def test_dg_schedule_with_colour_cap_matches_oracle(D, n, k, order, flux, free, ts, part, splits, ren, cap):
    m, om, od, gm, gd = _dg_pair(D, n, k, order, flux, free, ren)
    gd.inspect(ts, partition=part, splits=splits, max_colour_tiles=cap)
    gs = gd.schedule()
    os_ = od.chain().inspect(ts, partition=part, seed_xy=m.centroids(), splits=splits, max_colour_tiles=cap)
    sizes = {0: om.nc, 1: om.nf, 2: om.nb}
    pat = ([0, 1, 2, 0] * 3 + [0]) * 2 if order == 4 else [0, 1, 2, 0] * 2
    _compare_schedules(gs, os_, [sizes[s] for s in pat], [om.nc, om.nf, om.nb], len(splits) + 1)
    assert os_.check() == 0
    for sub in range(gs.nsub):
        assert np.diff(gs.tiles_by_color(sub)[0]).max() <= cap


# ------------------------------------------------------------------ executors

def _run_pair(D, n, k, order, flux, free, ren, steps, mode, ts=24, part=1, splits=(), prec=0, seed=1, cap=0,
              schedule=0):
    """Random nodal start state (every cell, boundary and tile border carries
    signal), plus the Ricker source."""
    m, om, od, gm, gd = _dg_pair(D, n, k, order, flux, free, ren, prec)
    od.set_source(0.43, 0.52)
    gd.set_source(0.43, 0.52)
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, seed)
    s[:] = I.random_state(s.shape, seed + 1)
    dtype = torch.float32 if prec else torch.float64
    gv = torch.from_numpy(v).to(dtype).cuda().contiguous()
    gs = torch.from_numpy(s).to(dtype).cuda().contiguous()
    od.step(v, s, steps, t0=0.1)
    if mode == 1:
        gd.inspect(ts, partition=part, splits=splits, max_colour_tiles=cap)
        gd.set_schedule(schedule)
        print(f"  [tile kernels per sub-chain {gd.kernels()}]")
    gd.upload(gv, gs)
    gd.step(steps, mode=mode, t0=0.1)
    gd.download(gv, gs)
    torch.cuda.synchronize()
    return rel_err([gv.double().cpu().numpy(), gs.double().cpu().numpy()], [v, s])


EXEC_CASES = [
    # n, k, order, flux, free, ren, steps
    (32, 1, 4, 0, 0xF, None, 100),   # small P1 workload: central, free surface, 100 steps
    (12, 2, 4, 1, 0x8, 7, 10),
    (12, 2, 2, 1, 0x8, 7, 10),
    (10, 3, 4, 1, 0x8, 5, 30),
    (10, 4, 4, 1, 0x0, 5, 30),
    (9, 2, 4, 0, 0x3, 3, 5),
    (9, 1, 2, 0, 0xF, None, 20),
]


@pytest.mark.parametrize("n,k,order,flux,free,ren,steps", EXEC_CASES)
def test_untiled_fp64_matches_oracle(D, n, k, order, flux, free, ren, steps):
    err = _run_pair(D, n, k, order, flux, free, ren, steps, mode=0)
    print(f"untiled FP64 n={n} k={k} order={order} flux={flux}: err {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("n,k,order,flux,free,ren,steps", EXEC_CASES)
def test_tiled_fp64_matches_oracle(D, n, k, order, flux, free, ren, steps):
    ts = 32 if n == 32 else 16
    splits = ()
    if k == 4:  # the whole 26-loop chain of a P4 FP64 tile does not fit in LDS: one sub-chain per operator
        ts, splits = 8, ((4, 8, 12, 13, 17, 21, 25) if order == 4 else (4,))
    err = _run_pair(D, n, k, order, flux, free, ren, steps, mode=1, ts=ts, splits=splits)
    print(f"tiled FP64 n={n} k={k} order={order} flux={flux} ts={ts} splits={splits}: err {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("ts,part,splits", [(1, 1, ()), (5, 1, ()), (3, 0, (4, 8, 12, 13, 17, 21, 25)), (40, 1, (13,)),
                                           (20, 1, (4, 8, 12, 13, 17, 21, 25))])
def test_tiled_fp64_tile_sizes_and_splits(D, ts, part, splits):
    err = _run_pair(D, 14, 2, 4, 1, 0x8, 9, 4, mode=1, ts=ts, part=part, splits=splits)
    print(f"tiled FP64 ts={ts} part={part} splits={splits}: err {err:.3e}")
    assert err <= 1e-12


DEGENERATE_CASES = [
    # n, k, order, flux, free, ren, steps, ts, splits, schedule
    (1, 2, 4, 1, 0x8, 3, 6, 1, (13,), 1),       # two-cell mesh, one tile per cell, dependence-driven
    (1, 2, 4, 1, 0x8, 3, 6, 8, (), 0),          # two-cell mesh, one tile for the whole step chain
    (2, 1, 2, 0, 0xF, None, 8, 1, (), 1),       # eight cells, order 2, one tile per cell
    (6, 2, 4, 1, 0x8, 3, 5, 1000, (13,), 1),    # one tile holding the whole mesh: no dependences
    (6, 1, 4, 1, 0x8, 3, 5, 1, (13,), 1),       # one tile per cell: 72 tiles, 10 colours per half step
]


@pytest.mark.parametrize("n,k,order,flux,free,ren,steps,ts,splits,schedule", DEGENERATE_CASES)
def test_degenerate_tilings_match_oracle(D, n, k, order, flux, free, ren, steps, ts, splits, schedule):
    """Smallest meshes, tiles of a single seed cell and a single tile for the whole
    mesh, under both schedules."""
    err = _run_pair(D, n, k, order, flux, free, ren, steps, mode=1, ts=ts, splits=splits, schedule=schedule)
    print(f"degenerate tiling n={n} k={k} order={order} ts={ts} splits={splits} schedule={schedule}: "
          f"err {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("mode,schedule", [(0, 0), (1, 0), (1, 1)])
def test_zero_steps_leave_state_unchanged(D, mode, schedule):
    m, om, od, gm, gd = _dg_pair(D, 6, 2, 4, 1, 0x8, 3)
    gd.set_source(0.43, 0.52)
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, 5)
    s[:] = I.random_state(s.shape, 6)
    if mode == 1:
        gd.inspect(10, partition=1, splits=(13,))
        gd.set_schedule(schedule)
    gv, gs = torch.from_numpy(v.copy()).cuda(), torch.from_numpy(s.copy()).cuda()
    gd.upload(gv, gs)
    gd.step(0, mode=mode, t0=0.1)
    gv.zero_()
    gs.zero_()
    gd.download(gv, gs)
    torch.cuda.synchronize()
    assert np.array_equal(gv.cpu().numpy(), v) and np.array_equal(gs.cpu().numpy(), s)
    if mode == 1:  # the dependence counters stay consistent for the next call
        gd.step(2, mode=1, t0=0.1)
        gd.download(gv, gs)
        torch.cuda.synchronize()
        od.set_source(0.43, 0.52)
        od.step(v, s, 2, t0=0.1)
        assert rel_err([gv.cpu().numpy(), gs.cpu().numpy()], [v, s]) <= 1e-12


OP_CASES = [
    # n, k, order, flux, free, ren, steps, ts, splits: one operator application per sub-chain,
    # with the update fused into the operator before it (chain kernel, one operator)
    (12, 2, 4, 1, 0x8, 7, 10, 32, (4, 8, 13, 17, 21)),
    (12, 2, 2, 1, 0x8, 7, 10, 32, (4,)),
    (10, 1, 4, 0, 0xF, 3, 10, 64, (4, 8, 13, 17, 21)),
    (10, 3, 4, 1, 0x8, 5, 20, 32, (4, 8, 13, 17, 21)),
    (10, 4, 4, 1, 0x0, 5, 20, 16, (4, 8, 13, 17, 21)),
    (9, 2, 2, 0, 0x3, 3, 10, 16, (4,)),
    (14, 2, 4, 1, 0x8, 9, 6, 24, (4, 8, 12, 13, 17, 21, 25)),  # updates in sub-chains of their own
]


@pytest.mark.parametrize("n,k,order,flux,free,ren,steps,ts,splits", OP_CASES)
def test_tiled_operator_kernel_fp64_matches_oracle(D, n, k, order, flux, free, ren, steps, ts, splits):
    err = _run_pair(D, n, k, order, flux, free, ren, steps, mode=1, ts=ts, splits=splits)
    print(f"operator-kernel tiled FP64 n={n} k={k} order={order} flux={flux} ts={ts} splits={splits}: "
          f"err {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_tiled_operator_kernel_fp32_matches_oracle(D, k):
    err = _run_pair(D, 10, k, 4, 1, 0x8, 4, 5, mode=1, ts=32, splits=(4, 8, 13, 17, 21), prec=1)
    print(f"operator-kernel tiled FP32 k={k}: err vs FP64 oracle {err:.3e}")
    assert err <= 1e-5


CHAIN_CASES = [
    # n, k, order, flux, free, ren, steps, ts, splits: whole-step and half-step sub-chains
    (12, 2, 4, 1, 0x8, 7, 10, 24, ()),
    (12, 2, 4, 0, 0xF, 7, 10, 24, (13,)),
    (12, 2, 2, 1, 0x8, 7, 10, 24, ()),
    (10, 1, 4, 1, 0x8, 3, 10, 32, ()),
    (10, 3, 4, 1, 0x8, 5, 10, 12, (13,)),
    (10, 4, 4, 1, 0x0, 5, 10, 6, (13,)),
    (16, 2, 4, 1, 0x8, None, 8, 40, (13,)),  # structured mesh in input order
]


@pytest.mark.parametrize("kernel", ["generic", "specialised", "register"])
@pytest.mark.parametrize("n,k,order,flux,free,ren,steps,ts,splits", CHAIN_CASES)
def test_tiled_chain_kernels_fp64_match_oracle(D, monkeypatch, kernel, n, k, order, flux, free, ren, steps, ts,
                                               splits):
    """The same schedule on the generic in-tile executor (every field in LDS),
    on the default specialised kernel (register-resident chain kernel at P1/P2,
    matrix-core kernel at P3/P4), and on the register-resident chain kernel
    where it is built."""
    if kernel == "generic":
        monkeypatch.setenv("DGT_TILE_OP", "0")
    elif kernel == "register":
        monkeypatch.setenv("DGT_TILE_OP", "1")
    err = _run_pair(D, n, k, order, flux, free, ren, steps, mode=1, ts=ts, splits=splits)
    print(f"{kernel} tiled FP64 n={n} k={k} order={order} flux={flux} ts={ts} splits={splits}: err {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("n,k,order,flux,free,ren,steps,ts,splits", CHAIN_CASES)
def test_dependence_driven_schedule_fp64_matches_oracle(D, n, k, order, flux, free, ren, steps, ts, splits):
    """Schedule 1: one launch per sub-chain, tiles started by device-scope
    dependence counters instead of colour launches."""
    err = _run_pair(D, n, k, order, flux, free, ren, steps, mode=1, ts=ts, splits=splits, schedule=1)
    print(f"dependence-driven tiled FP64 n={n} k={k} order={order} flux={flux} ts={ts} splits={splits}: "
          f"err {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_dependence_driven_schedule_fp32_matches_oracle(D, k):
    err = _run_pair(D, 10, k, 4, 1, 0x8, 4, 5, mode=1, ts=8 if k == 4 else 16, splits=(13,), prec=1, schedule=1)
    print(f"dependence-driven tiled FP32 k={k}: err vs FP64 oracle {err:.3e}")
    assert err <= 1e-5


def test_dependence_driven_schedule_repeated_calls(D):
    """Counters carry over between launches: many one-step calls equal one call."""
    m, om, od, gm, gd = _dg_pair(D, 16, 2, 4, 1, 0x8, 5)
    gd.inspect(12, partition=1, splits=(13,))
    gd.set_schedule(1)
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, 11)
    s[:] = I.random_state(s.shape, 12)
    gv = torch.from_numpy(v.copy()).cuda()
    gs = torch.from_numpy(s.copy()).cuda()
    gd.upload(gv, gs)
    for i in range(7):
        gd.step(1, mode=1, t0=0.1 + i * gd.dt)
    gd.download(gv, gs)
    od.step(v, s, 7, t0=0.1)
    err = rel_err([gv.cpu().numpy(), gs.cpu().numpy()], [v, s])
    print(f"dependence-driven, 7 single-step calls: err {err:.3e}")
    assert err <= 1e-12


def test_dependence_wait_timeout_is_reported_and_recovered(D):
    """A poll limit of 1 (set from the host) makes dependence waits give up: the
    kernels exit, the error is reported, the counters are reset, and with the
    default limit the next run is correct again."""
    m, om, od, gm, gd = _dg_pair(D, 16, 2, 4, 1, 0x8, 5)
    gd.inspect(8, partition=1, splits=(13,))
    gd.set_schedule(1)
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, 21)
    s[:] = I.random_state(s.shape, 22)
    gv = torch.from_numpy(v.copy()).cuda()
    gs = torch.from_numpy(s.copy()).cuda()
    gd.set_wait_limit(1)
    gd.upload(gv, gs)
    gd.step(3, mode=1)
    with pytest.raises(D.DgtError):
        gd.download(gv, gs)
    gd.set_wait_limit(1 << 20)
    gv.copy_(torch.from_numpy(v))
    gs.copy_(torch.from_numpy(s))
    gd.upload(gv, gs)
    gd.step(3, mode=1, t0=0.0)
    gd.download(gv, gs)
    od.step(v, s, 3, t0=0.0)
    err = rel_err([gv.cpu().numpy(), gs.cpu().numpy()], [v, s])
    print(f"after a forced timeout and reset: err {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("splits", [(), (13,)])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_tiled_chain_kernel_fp32_matches_oracle(D, k, splits):
    err = _run_pair(D, 10, k, 4, 1, 0x8, 4, 5, mode=1, ts=8 if k == 4 else 16, splits=splits, prec=1)
    print(f"chain-kernel tiled FP32 k={k} splits={splits}: err vs FP64 oracle {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_fp32_matches_oracle(D, mode, k):
    err = _run_pair(D, 10, k, 4, 1, 0x8, 4, 5, mode=mode, ts=16, prec=1)
    print(f"FP32 mode={mode} k={k}: err vs FP64 oracle {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("cap,splits", [(3, (13,)), (5, (4, 8, 13, 17, 21)), (-1, (13,))])
def test_tiled_with_colour_cap_matches_oracle(D, cap, splits):
    """Capped colour classes (and the solver's automatic cap, -1) change the
    schedule, not the result."""
    err = _run_pair(D, 14, 2, 4, 1, 0x8, 9, 6, mode=1, ts=12, splits=splits, cap=cap)
    print(f"tiled FP64 colour cap {cap} splits={splits}: err {err:.3e}")
    assert err <= 1e-12


def test_energy_matches_oracle(D):
    m, om, od, gm, gd = _dg_pair(D, 12, 2, 4, 0, 0xF, 3)
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, 3)
    s[:] = I.random_state(s.shape, 4)
    so = I.random_state(s.shape, 5)
    e_ref = od.energy(v, s, so)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    e = gd.energy(t(v), t(s), t(so))
    print(f"energy GPU {e!r} oracle {e_ref!r} rel {abs(e - e_ref) / abs(e_ref):.3e}")
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref)


def test_energy_conserved_on_gpu_tiled(D):
    m, om, od, gm, gd = _dg_pair(D, 16, 2, 4, 0, 0xF, 3)
    gd.inspect(32, partition=1, splits=(4, 8, 13, 17, 21))
    v, s = gd.zeros()
    v.copy_(torch.from_numpy(I.random_state(v.shape, 3)))
    s.copy_(torch.from_numpy(I.random_state(s.shape, 4)))
    gd.upload(v, s)
    es = []
    for _ in range(50):
        so = s.clone()
        gd.step(1, mode=1)
        gd.download(v, s)
        es.append(gd.energy(v, s, so))
    es = np.array(es)
    drift = np.abs(es - es[0]).max() / es[0]
    print(f"GPU tiled energy drift over 50 steps: {drift:.3e}")
    assert drift < 1e-12


def test_errors_are_reported(D):
    m, om, od, gm, gd = _dg_pair(D, 6, 1, 4, 0, 0xF, None)
    with pytest.raises(D.DgtError):
        gd.step(1, mode=0)  # no state uploaded
    v, s = gd.zeros()
    gd.upload(v, s)
    with pytest.raises(D.DgtError):
        gd.step(1, mode=1)  # not inspected
    with pytest.raises(D.DgtError):
        gd.inspect(0)


@pytest.mark.parametrize("k,sub_ts,schedule", [(2, (12, 30), 1), (1, (40, 9), 0), (3, (6, 10, 7, 12, 8, 9), 0)])
def test_sub_chain_tile_sizes_schedule_and_executor(D, k, sub_ts, schedule):
    """Each sub-chain of a fusion scheme with its own seed tile size: the GPU schedule
    equals the oracle's byte for byte, and the tiled executor matches the oracle."""
    splits = (13,) if len(sub_ts) == 2 else (4, 8, 13, 17, 21)
    n = 12 if k < 3 else 10
    m, om, od, gm, gd = _dg_pair(D, n, k, 4, 1, 0x8, 5)
    gd.inspect(8, partition=1, splits=splits, sub_tile_sizes=sub_ts)
    gs = gd.schedule()
    os_ = od.chain().inspect(8, partition=1, seed_xy=m.centroids(), splits=splits, sub_tile_sizes=sub_ts)
    sizes = {0: om.nc, 1: om.nf, 2: om.nb}
    pat = ([0, 1, 2, 0] * 3 + [0]) * 2
    _compare_schedules(gs, os_, [sizes[s] for s in pat], [om.nc, om.nf, om.nb], len(splits) + 1)
    assert os_.check() == 0
    od.set_source(0.43, 0.52)
    gd.set_source(0.43, 0.52)
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, 3)
    s[:] = I.random_state(s.shape, 4)
    gv, gsg = torch.from_numpy(v.copy()).cuda(), torch.from_numpy(s.copy()).cuda()
    od.step(v, s, 5, t0=0.1)
    gd.set_schedule(schedule)
    gd.upload(gv, gsg)
    gd.step(5, mode=1, t0=0.1)
    gd.download(gv, gsg)
    torch.cuda.synchronize()
    err = rel_err([gv.cpu().numpy(), gsg.cpu().numpy()], [v, s])
    print(f"sub-chain tile sizes {sub_ts} k={k} schedule={schedule}: schedule byte-equal, err {err:.3e}")
    assert err <= 1e-12


MFMA_CASES = [
    # k, prec, splits, schedule, ts: half steps and single operators at P3/P4
    (3, 0, (13,), 0, 12), (3, 0, (13,), 1, 12), (4, 0, (13,), 0, 6), (4, 0, (13,), 1, 6),
    (3, 0, (4, 8, 13, 17, 21), 0, 24), (4, 0, (4, 8, 13, 17, 21), 1, 16),
    (4, 0, (4, 8, 12, 13, 17, 21, 25), 0, 16),
    (3, 1, (13,), 0, 16), (3, 1, (13,), 1, 16), (4, 1, (13,), 1, 8), (4, 1, (4, 8, 13, 17, 21), 0, 24),
]


@pytest.mark.parametrize("k,prec,splits,schedule,ts", MFMA_CASES)
def test_matrix_core_kernel_matches_oracle(D, k, prec, splits, schedule, ts):
    """At P3/P4 the default kernel of whole operator applications is the
    matrix-core one (derivative and lift contractions on MFMA), for half steps
    and single operators, under both schedules; it matches the oracle element by
    element from random states."""
    m, om, od, gm, gd = _dg_pair(D, 12, k, 4, 1, 0x8, 5, prec)
    od.set_source(0.43, 0.52)
    gd.set_source(0.43, 0.52)
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, 31)
    s[:] = I.random_state(s.shape, 32)
    dtype = torch.float32 if prec else torch.float64
    gv = torch.from_numpy(v).to(dtype).cuda().contiguous()
    gs = torch.from_numpy(s).to(dtype).cuda().contiguous()
    od.step(v, s, 6, t0=0.1)
    gd.inspect(ts, partition=1, splits=splits)
    gd.set_schedule(schedule)
    kinds = gd.kernels()
    # every sub-chain of operator applications runs on it (an update alone is no operator)
    whole = [b for b in range(len(splits) + 1) if not (b > 0 and splits[b - 1] in (12, 25))]
    assert [kinds[b] for b in whole] == [2] * len(whole) and set(kinds) <= {0, 2}, kinds
    gd.upload(gv, gs)
    gd.step(6, mode=1, t0=0.1)
    gd.download(gv, gs)
    torch.cuda.synchronize()
    err = rel_err([gv.double().cpu().numpy(), gs.double().cpu().numpy()], [v, s])
    print(f"matrix-core k={k} prec={prec} splits={splits} schedule={schedule} ts={ts}: err {err:.3e}")
    assert err <= (1e-5 if prec else 1e-12)


def test_kernel_selection_follows_environment(D, monkeypatch):
    """DGT_TILE_OP=1 selects the register-resident chain kernel where it is
    built (single operators at P3), 0 the generic kernel; the default is the
    matrix-core kernel, and P2 keeps the register-resident one."""
    m, om, od, gm, gd = _dg_pair(D, 8, 3, 4, 1, 0x8, 5)
    sp = (4, 8, 13, 17, 21)
    gd.inspect(16, partition=1, splits=sp)
    assert gd.kernels() == [2] * 6
    monkeypatch.setenv("DGT_TILE_OP", "1")
    gd.inspect(16, partition=1, splits=sp)
    assert gd.kernels() == [1] * 6
    gd.inspect(16, partition=1, splits=(13,))  # no register chain kernel for P3 half steps
    assert gd.kernels() == [0, 0]
    monkeypatch.setenv("DGT_TILE_OP", "0")
    gd.inspect(16, partition=1, splits=sp)
    assert gd.kernels() == [0] * 6
    monkeypatch.delenv("DGT_TILE_OP")
    m, om, od, gm, gd = _dg_pair(D, 8, 2, 4, 1, 0x8, 5)
    gd.inspect(16, partition=1, splits=(13,))
    assert gd.kernels() == [1, 1]
