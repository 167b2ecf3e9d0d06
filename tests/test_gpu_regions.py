"""GPU parity of the region-aware inspection (Sec. 3.3, Alg. 2, Sec. 5.1.2) and of
one GPU's part of a distributed mesh.

* the GPU inspector with seed regions is byte-equal to the oracle's (tiles,
  colours, tiling functions, iteration lists, footprints, the region ranges and
  the carried seed regions of later sub-chains), on the DG chain of a part mesh and
  on a generic chain with one exchange per sub-chain;
* a solver of the part (owned cells, as many exec halo layers as the step has
  facet loops, one non-exec layer; T_ne never launched) whose halo cells are
  refreshed from the oracle's whole-mesh state before every step matches the
  oracle's whole-mesh run on the owned cells, within 1e-12 (FP64) or 1e-5 (FP32)
  of the largest value, under both executor schedules and every degree; edge
  cases: a part without core cells and a part that is the whole mesh (empty T_ne);
* halo packing and unpacking copy exactly, and a part whose halo is filled on the
  GPU from a whole-mesh solver follows that solver on its owned cells.
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


def _depth(order):
    return 6 if order == 4 else 2  # facet loops of one step


def _setup(D, n, k, order, flux, free, bx, by, part, prec=0, ren=3, depth=None):
    m = I.square_mesh(n, jitter=0.2, renumber_seed=ren)
    lam, mu, rho = I.lognormal_material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    od = O.ODG(om, k, lam, mu, rho, flux=flux, order=order, dt=dt, free_sides=free)
    P = I.mesh_part(m, I.block_parts(m, bx, by), part, _depth(order) if depth is None else depth)
    c = P.cells
    lm = D.Mesh.from_mesh(P.mesh)
    ls = D.Solver(lm, lam[c], mu[c], rho[c], degree=k, flux=flux, time_order=order, precision=prec,
                  free_sides=free, dt=dt)
    lod = O.ODG(O.OMesh.from_mesh(P.mesh), k, lam[c], mu[c], rho[c], flux=flux, order=order, dt=dt, free_sides=free)
    return m, od, P, lm, ls, lod, (lam, mu, rho), dt


def _compare(gs, os_, loop_sizes, set_sizes, nsub, nseed):
    assert gs.nsub == os_.nsub == nsub
    for sub in range(nsub):
        gi, oi = gs.sub_info(sub), os_.sub_info(sub)
        assert gi == oi, (gi, oi)
        ginfo, greg = gs.regions(sub, nseed)
        oinfo, oreg = os_.regions(sub, nseed)
        assert ginfo == oinfo and np.array_equal(greg, oreg), (sub, ginfo, oinfo)
        assert np.array_equal(gs.colors(sub), os_.colors(sub))
        gc, gt = gs.tiles_by_color(sub)
        oc, ot = os_.tiles_by_color(sub)
        assert np.array_equal(gc, oc) and np.array_equal(gt, ot)
        for j in range(gi["first"], gi["first"] + gi["nloops"]):
            assert np.array_equal(gs.sigma(j), os_.sigma(j, loop_sizes[j])), j
            go, git = gs.iters(j, sub)
            oo, oit = os_.iters(j, loop_sizes[j], sub)
            assert np.array_equal(go, oo) and np.array_equal(git, oit), j
        for st in range(len(set_sizes)):
            for a, b in zip(gs.footprint(sub, st), os_.footprint(sub, st)):
                assert np.array_equal(a, b), (sub, st)


INSPECT_CASES = [
    # n, k, order, blocks, part, ts, partition, splits
    (16, 1, 4, (2, 2), 0, 9, 1, (13,)),
    (16, 2, 4, (2, 2), 3, 6, 1, (4, 8, 13, 17, 21)),
    (18, 1, 2, (3, 2), 4, 8, 0, ()),
    (14, 2, 4, (2, 1), 1, 20, 1, ()),
]


@pytest.mark.parametrize("n,k,order,blocks,part,ts,partition,splits", INSPECT_CASES)
def test_region_schedule_matches_oracle(D, n, k, order, blocks, part, ts, partition, splits):
    m, od, P, lm, ls, lod, mat, dt = _setup(D, n, k, order, 1, 0x8, *blocks, part)
    print(f"part {part}: {int(P.owned.sum())} owned, {int(np.sum(P.region == 0))} core, "
          f"{int(np.sum(P.region == 2))} non-exec of {P.cells.size} local cells")
    ls.inspect(ts, partition=partition, splits=splits, seed_region=P.region, region_carry=1)
    gs = ls.schedule()
    os_ = lod.chain().inspect(ts, partition=partition, seed_xy=P.mesh.centroids(), splits=splits,
                              seed_region=P.region, carry=1)
    lom = lod.om
    sizes = {0: lom.nc, 1: lom.nf, 2: lom.nb}
    pat = ([0, 1, 2, 0] * 3 + [0]) * 2 if order == 4 else [0, 1, 2, 0] * 2
    _compare(gs, os_, [sizes[s] for s in pat], [lom.nc, lom.nf, lom.nb], len(splits) + 1, lom.nc)
    assert os_.check() == 0


@pytest.mark.parametrize("carry", [0, 1])
def test_region_schedule_generic_chain(D, carry):
    """Tier-1 chain (cells read/write, facets increment cells) with one exchange per
    sub-chain (carry 0) or per chain (carry 1)."""
    m = I.square_mesh(12, jitter=0.2, renumber_seed=4)
    P = I.mesh_part(m, I.block_parts(m, 2, 2), 2, 3)
    om = O.OMesh.from_mesh(P.mesh)
    mp = om.maps()

    def build(mod):
        ch = mod()
        Cs = ch.set(om.nc)
        F = ch.set(om.nf)
        f2c = ch.map(F, Cs, 2, mp["f2c"])
        for _ in range(2):
            ch.loop(Cs, [(-1, 0, 0), (-1, 1, 1)])
            ch.loop(F, [(f2c, 0, 1), (f2c, 2, 0)])
        return ch

    xy = P.mesh.centroids()
    gs = build(D.Chain).inspect(5, partition=1, seed_xy=xy, splits=(2,), seed_region=P.region, region_carry=carry)
    os_ = build(O.OChain).inspect(5, partition=1, seed_xy=xy, splits=(2,), seed_region=P.region, carry=carry)
    _compare(gs, os_, [om.nc, om.nf, om.nc, om.nf], [om.nc, om.nf], 2, om.nc)


PART_CASES = [
    # n, k, order, flux, free, blocks, part, ts, partition, splits, schedule, precision
    (14, 1, 4, 1, 0x8, (2, 2), 0, 8, 1, (13,), 1, 0),
    (14, 2, 4, 1, 0x8, (2, 2), 3, 12, 1, (13,), 0, 0),
    (14, 2, 4, 0, 0xF, (2, 2), 1, 10, 1, (4, 8, 13, 17, 21), 1, 0),
    (12, 3, 4, 1, 0x8, (2, 2), 2, 8, 1, (4, 8, 13, 17, 21), 0, 0),
    (12, 4, 4, 1, 0x8, (2, 1), 0, 8, 1, (13,), 0, 0),
    (14, 2, 2, 1, 0x8, (3, 2), 4, 10, 0, (), 1, 0),
    (14, 1, 4, 1, 0x8, (2, 2), 1, 10, 1, (), 0, 0),
    (14, 2, 4, 1, 0x8, (2, 2), 0, 12, 1, (13,), 1, 1),
    (12, 3, 4, 1, 0x8, (2, 2), 3, 8, 1, (13,), 0, 1),
    # a part with no core cell (every owned cell touches the halo)
    (12, 2, 4, 1, 0x8, (12, 6), 1, 4, 1, (13,), 1, 0),
    # the whole mesh as one part: every cell core, T_ne empty
    (10, 2, 4, 1, 0x8, (1, 1), 0, 10, 1, (13,), 1, 0),
]


def _refresh_halo(ls, P, v, sg, dtype):
    """The halo exchange of a step, done on the host for the parity test: the local
    state's exec and non-exec cells take the oracle's whole-mesh values."""
    lv, lsg = ls.zeros()
    ls.download(lv, lsg)
    torch.cuda.synchronize()
    hv, hs = lv.cpu().numpy(), lsg.cpu().numpy()
    halo = ~P.owned
    hv[:, :, halo] = v[:, :, P.cells[halo]]
    hs[:, :, halo] = sg[:, :, P.cells[halo]]
    ls.upload(torch.from_numpy(np.ascontiguousarray(hv, dtype)).cuda(),
              torch.from_numpy(np.ascontiguousarray(hs, dtype)).cuda())


@pytest.mark.parametrize("n,k,order,flux,free,blocks,part,ts,partition,splits,schedule,prec", PART_CASES)
def test_part_step_matches_whole_mesh_oracle(D, n, k, order, flux, free, blocks, part, ts, partition, splits,
                                             schedule, prec):
    m, od, P, lm, ls, lod, mat, dt = _setup(D, n, k, order, flux, free, *blocks, part, prec=prec)
    own = np.nonzero(P.owned)[0]
    if blocks == (12, 6):
        assert not np.any(P.region == 0)  # the no-core edge case
    if blocks == (1, 1):
        assert np.all(P.region == 0)  # the whole-mesh edge case
    print(f"P{k} order {order} {'FP32' if prec else 'FP64'} part {part}: {own.size} owned, "
          f"{int(np.sum(P.region == 0))} core, {P.cells.size} local cells; schedule {schedule}")
    # a source in the part: the centroid of its first owned cell
    x, y = P.mesh.centroids()[own[0]]
    od.set_source(x, y)
    ls.set_source(x, y)
    ls.inspect(ts, partition=partition, splits=splits, seed_region=P.region, region_carry=1)
    ls.set_schedule(schedule)
    v, sg = od.zeros()
    v[:] = I.random_state(v.shape, 31)
    sg[:] = I.random_state(sg.shape, 32)
    dtype = np.float32 if prec else np.float64
    c = P.cells
    ls.upload(torch.from_numpy(np.ascontiguousarray(v[:, :, c], dtype)).cuda(),
              torch.from_numpy(np.ascontiguousarray(sg[:, :, c], dtype)).cuda())
    tol = 1e-5 if prec else 1e-12
    worst = 0.0
    for step in range(4):
        t0 = 0.05 + step * dt
        _refresh_halo(ls, P, v, sg, dtype)
        od.step(v, sg, 1, t0=t0)
        ls.step(1, mode=1, t0=t0)
        lv, lsg = ls.zeros()
        ls.download(lv, lsg)
        torch.cuda.synchronize()
        hv, hs = lv.cpu().numpy().astype(np.float64), lsg.cpu().numpy().astype(np.float64)
        ref = max(np.abs(v).max(), np.abs(sg).max())
        err = max(np.abs(hv[:, :, own] - v[:, :, c[own]]).max(), np.abs(hs[:, :, own] - sg[:, :, c[own]]).max()) / ref
        worst = max(worst, err)
    print(f"  owned cells vs whole-mesh oracle over 4 steps: max-abs / max = {worst:.3e} (tolerance {tol:g})")
    assert worst <= tol


@pytest.mark.parametrize("prec", [0, 1])
def test_halo_fill_on_gpu(D, prec):
    """Pack from a whole-mesh solver, unpack into the part's halo, step both: the
    packed values are the whole-mesh state bit for bit and the part follows the
    whole-mesh solver on its owned cells."""
    n, k, order = 16, 2, 4
    m, od, P, lm, ls, lod, (lam, mu, rho), dt = _setup(D, n, k, order, 1, 0x8, 2, 2, 3, prec=prec)
    gm = D.Mesh.from_mesh(m)
    gsol = D.Solver(gm, lam, mu, rho, degree=k, flux=1, time_order=order, precision=prec, free_sides=0x8, dt=dt)
    gsol.inspect(16, partition=1, splits=(13,))
    ls.inspect(12, partition=1, splits=(13,), seed_region=P.region, region_carry=1)
    ls.set_schedule(1)
    dtype = torch.float32 if prec else torch.float64
    gen = torch.Generator(device="cpu").manual_seed(5)
    gv = torch.randn(2, O.np_of(k), m.nc, generator=gen, dtype=torch.float64).to(dtype).cuda()
    gs_ = torch.randn(3, O.np_of(k), m.nc, generator=gen, dtype=torch.float64).to(dtype).cuda()
    cidx = torch.from_numpy(P.cells.astype(np.int64)).cuda()
    gsol.upload(gv.contiguous(), gs_.contiguous())
    ls.upload(gv[:, :, cidx].contiguous(), gs_[:, :, cidx].contiguous())
    halo = np.nonzero(~P.owned)[0]
    send = gsol.cell_list(P.cells[halo])  # the whole mesh's view of the halo cells
    recv = ls.cell_list(halo)  # the part's halo cells
    bv = torch.empty(2, O.np_of(k), halo.size, dtype=dtype, device="cuda")
    bs = torch.empty(3, O.np_of(k), halo.size, dtype=dtype, device="cuda")
    own = torch.from_numpy(np.nonzero(P.owned)[0].astype(np.int64)).cuda()
    gown = cidx[own]
    worst = 0.0
    for step in range(5):
        t0 = step * dt
        gsol.pack(send, bv, bs)
        ls.unpack(recv, bv, bs)
        if step == 0:
            wv, ws = gsol.zeros()
            gsol.download(wv, ws)
            torch.cuda.synchronize()
            hidx = torch.from_numpy(P.cells[halo].astype(np.int64)).cuda()
            assert torch.equal(bv, wv[:, :, hidx]) and torch.equal(bs, ws[:, :, hidx])
        gsol.step(1, mode=1, t0=t0)
        ls.step(1, mode=1, t0=t0)
        wv, ws = gsol.zeros()
        lv, lsg = ls.zeros()
        gsol.download(wv, ws)
        ls.download(lv, lsg)
        torch.cuda.synchronize()
        ref = max(wv.abs().max().item(), ws.abs().max().item())
        err = max((lv[:, :, own] - wv[:, :, gown]).abs().max().item(),
                  (lsg[:, :, own] - ws[:, :, gown]).abs().max().item()) / ref
        worst = max(worst, err)
    print(f"  part vs whole-mesh GPU solver on owned cells, 5 steps: {worst:.3e}")
    assert worst <= (1e-5 if prec else 1e-12)


def test_autotune_keeps_regions(D):
    """The autotuner re-inspects a part with its regions: the chosen schedule still
    has T_ne and the part still follows the whole-mesh oracle on its owned cells."""
    m, od, P, lm, ls, lod, mat, dt = _setup(D, 14, 2, 4, 1, 0x8, 2, 2, 1)
    ls.inspect(10, partition=1, splits=(13,), seed_region=P.region, region_carry=1)
    r = ls.autotune(tile_sizes=(6, 12, 20), splits=(13,), trial_steps=2)
    gs = ls.schedule()
    for sub in range(gs.nsub):
        (ncore, nbnd, tne, tcol), reg = gs.regions(sub, P.cells.size)
        assert tne == gs.sub_info(sub)["ntiles"] - 1
    assert np.array_equal(gs.regions(0, P.cells.size)[1], P.region)
    v, sg = od.zeros()
    v[:] = I.random_state(v.shape, 41)
    sg[:] = I.random_state(sg.shape, 42)
    c = P.cells
    ls.upload(torch.from_numpy(np.ascontiguousarray(v[:, :, c])).cuda(),
              torch.from_numpy(np.ascontiguousarray(sg[:, :, c])).cuda())
    od.step(v, sg, 1, t0=0.0)
    ls.step(1, mode=1, t0=0.0)
    lv, lsg = ls.zeros()
    ls.download(lv, lsg)
    torch.cuda.synchronize()
    own = np.nonzero(P.owned)[0]
    ref = max(np.abs(v).max(), np.abs(sg).max())
    err = max(np.abs(lv.cpu().numpy()[:, :, own] - v[:, :, c[own]]).max(),
              np.abs(lsg.cpu().numpy()[:, :, own] - sg[:, :, c[own]]).max()) / ref
    print(f"  autotuned part ({r}): owned cells vs oracle {err:.3e}")
    assert err <= 1e-12


def test_region_argument_checks(D):
    m, od, P, lm, ls, lod, mat, dt = _setup(D, 10, 1, 4, 1, 0x8, 2, 2, 0)
    with pytest.raises(D.DgtError):  # several sub-chains need one exchange per step
        ls.inspect(8, splits=(13,), seed_region=P.region, region_carry=0)
    with pytest.raises(D.DgtError):
        ls.inspect(8, seed_region=P.region, max_colour_tiles=4)
    bad = P.region.copy()
    bad[3] = 7
    with pytest.raises(D.DgtError):
        ls.inspect(8, seed_region=bad)
    with pytest.raises(D.DgtError):
        ls.cell_list([0, P.cells.size])
    ls.inspect(8, seed_region=P.region)
    with pytest.raises(D.DgtError):  # a part does not join a batch
        D.Batch([ls])
