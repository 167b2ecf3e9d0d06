"""Pins of the oracle's region-aware inspection (Sec. 3.3, Alg. 2, Sec. 5.1.2).

One part of a mesh (owned cells, `depth` exec layers, one non-exec layer) is
inspected with seed regions.  What the paper fixes, checked by brute force:

* tiles never mix regions: core seeds go to core tiles, boundary seeds to
  boundary tiles, in blocks of the seed order; every non-exec seed goes to the
  one tile T_ne (Sec. 5.1.2);
* every boundary tile has a higher colour than every core tile, and T_ne alone
  has the highest colour (Sec. 3.3, Sec. 5.1.2);
* the schedule, T_ne included, is a legal schedule (brute-force dependence
  checker);
* a simulation of stale data: all data is valid after the halo exchange, an
  iteration of T_ne is not executed and makes everything it writes stale; no
  executed iteration ever touches stale data, and with as many exec layers as
  the chain has facet loops every owned cell ends valid, while one layer fewer
  leaves some owned cell stale (the depth requirement of Sec. 4);
* the tiled step of the part (T_ne skipped, halo cells refreshed from the
  whole-mesh run before every step) gives the whole-mesh untiled result on the
  owned cells to rounding.
"""
import numpy as np
import pytest

import oracle as O
from paper_1708_03183_amd import inputs as I


def _part_dg(n, k, order, flux, free, bx, by, part, depth, ren=3, jitter=0.2, seed=11):
    m = I.square_mesh(n, jitter=jitter, jitter_seed=seed, renumber_seed=ren)
    u = I.uniform01(seed + 1, 3 * m.nc).reshape(3, -1)
    lam, mu, rho = 1.0 + u[0], 0.5 + 0.5 * u[1], 1.0 + 0.5 * u[2]
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    g = O.ODG(om, k, lam, mu, rho, flux=flux, order=order, dt=dt, free_sides=free)
    P = I.mesh_part(m, I.block_parts(m, bx, by), part, depth)
    lom = O.OMesh.from_mesh(P.mesh)
    c = P.cells
    loc = O.ODG(lom, k, lam[c], mu[c], rho[c], flux=flux, order=order, dt=dt, free_sides=free)
    return m, g, P, loc


def _facet_loops(order):
    return 6 if order == 4 else 2


def _stale_simulation(ch, sch, nsub, carry, owned_cells):
    """Validity of every element of every set after the chain; returns (violations,
    stale owned cells).  All data is valid at the start (just exchanged); with carry 0
    every sub-chain starts after an exchange of its own."""
    nsets = 3
    sizes = [ch.set_size(s) for s in range(nsets)]
    maps = {}
    viol = 0
    valid = [np.ones(sz, bool) for sz in sizes]
    for sub in range(nsub):
        info = sch.sub_info(sub)
        tne = sch.regions(sub, sizes[0])[0][2]
        if not carry:
            valid = [np.ones(sz, bool) for sz in sizes]
        for j in range(info["first"], info["first"] + info["nloops"]):
            st, descs = ch.loop_info(j)
            sig = sch.sigma(j, sizes[st])
            ex = sig != tne
            targets = []
            for mp, mode in descs:
                if mp < 0:
                    targets.append((st, np.arange(sizes[st])[:, None], mode))
                else:
                    if mp not in maps:
                        maps[mp] = ch.map_info(mp)
                    fr, to, vals = maps[mp]
                    targets.append((to, vals, mode))
            for S, t, mode in targets:
                viol += int(np.sum(ex[:, None] & ~valid[S][t]))
            for S, t, mode in targets:
                if mode != O.R:
                    valid[S][t[~ex].ravel()] = False
    return viol, int(np.sum(~valid[0][owned_cells]))


@pytest.mark.parametrize("splits,ts,part", [((13,), 7, 0), ((4, 8, 13, 17, 21), 5, 3), ((), 9, 1)])
def test_region_tiles_and_colours(splits, ts, part):
    m, g, P, loc = _part_dg(16, 1, 4, 1, 0x8, 2, 2, part, 6)
    ch = loc.chain()
    s = ch.inspect(ts, partition=0, splits=splits, seed_region=P.region, carry=1)
    assert s.check() == 0
    nl = P.cells.size
    for sub in range(s.nsub):
        info = s.sub_info(sub)
        (ncore, nbnd, tne, tcol), reg = s.regions(sub, nl)
        if sub == 0:
            assert np.array_equal(reg, P.region)
        assert info["ntiles"] == ncore + nbnd + 1 and tne == ncore + nbnd
        sig = s.sigma(info["first"], nl)
        # blocks of ts seeds of each region in seed order (partition 0: ascending id)
        expect = np.full(nl, tne, np.int64)
        for r, base in ((0, 0), (1, ncore)):
            ids = np.nonzero(reg == r)[0]
            expect[ids] = base + np.arange(ids.size) // ts
        assert np.array_equal(sig, expect)
        assert ncore == -(-int(np.sum(reg == 0)) // ts) and nbnd == -(-int(np.sum(reg == 1)) // ts)
        col = s.colors(sub)
        assert tcol == info["ncolors"] - 1 and col[tne] == tcol and np.sum(col == tcol) == 1
        if ncore and nbnd:
            assert col[:ncore].max() < col[ncore:tne].min()
        coff, tl = s.tiles_by_color(sub)
        assert tl[-1] == tne


@pytest.mark.parametrize("order,splits,carry", [(4, (13,), 1), (4, (4, 8, 13, 17, 21), 1), (2, (), 1), (4, (), 0),
                                                (2, (4,), 1)])
def test_stale_data_never_read_and_owned_complete(order, splits, carry):
    depth = _facet_loops(order)
    for d, complete in ((depth, True), (depth - 1, False)):
        m, g, P, loc = _part_dg(18, 1, order, 1, 0x8, 2, 2, 2, d)
        ch = loc.chain()
        s = ch.inspect(6, partition=1, seed_xy=P.mesh.centroids(), splits=splits, seed_region=P.region, carry=carry)
        assert s.check() == 0
        viol, stale_owned = _stale_simulation(ch, s, s.nsub, carry, np.nonzero(P.owned)[0])
        print(f"depth {d}: violations {viol}, stale owned cells {stale_owned}")
        assert viol == 0
        if carry or not splits:
            assert (stale_owned == 0) == complete


def test_carry_marks_stale_seeds():
    """With one exchange per chain the second sub-chain's non-exec seeds are the
    first's plus every seed its T_ne wrote, and they grow from the outside in."""
    m, g, P, loc = _part_dg(16, 1, 4, 0, 0xF, 2, 2, 0, 6)
    ch = loc.chain()
    s = ch.inspect(5, partition=0, splits=(13,), seed_region=P.region, carry=1)
    nl = P.cells.size
    r0 = s.regions(0, nl)[1]
    r1 = s.regions(1, nl)[1]
    assert np.all(r1[r0 == 2] == 2)
    newly = (r1 == 2) & (r0 != 2)
    assert newly.any()
    # three facet loops in the first half step: the outer three exec layers turn stale
    assert set(np.unique(P.layer[newly])) == {4, 5, 6}
    s0 = ch.inspect(5, partition=0, splits=(13,), seed_region=P.region, carry=0)
    assert np.array_equal(s0.regions(1, nl)[1], r0)
    # the schedule built for one exchange per sub-chain is wrong with one exchange per
    # chain: the second half step would execute iterations on stale data
    own = np.nonzero(P.owned)[0]
    assert _stale_simulation(ch, s, s.nsub, 1, own)[0] == 0
    assert _stale_simulation(ch, s0, s0.nsub, 1, own)[0] > 0


@pytest.mark.parametrize("k,order,flux,free,splits,part", [(1, 4, 1, 0x8, (13,), 3), (2, 4, 0, 0xF, (4, 8, 13, 17, 21), 0),
                                                            (2, 2, 1, 0x8, (), 1), (1, 2, 0, 0x3, (4,), 2)])
def test_part_step_matches_whole_mesh(k, order, flux, free, splits, part):
    depth = _facet_loops(order)
    m, g, P, loc = _part_dg(14, k, order, flux, free, 2, 2, part, depth)
    npk = O.np_of(k)
    v, sg = g.zeros()
    v[:] = I.random_state(v.shape, 21)
    sg[:] = I.random_state(sg.shape, 22)
    lv, ls = loc.zeros()
    c = P.cells
    lv[:] = v[:, :, c]
    ls[:] = sg[:, :, c]
    ch = loc.chain()
    s = ch.inspect(6, partition=1, seed_xy=P.mesh.centroids(), splits=splits, seed_region=P.region, carry=1)
    halo = ~P.owned
    own = np.nonzero(P.owned)[0]
    worst = 0.0
    for n in range(4):
        t0 = 0.05 + n * g.dt
        # the halo exchange: exec and non-exec cells take the whole-mesh state
        lv[:, :, halo] = v[:, :, c[halo]]
        ls[:, :, halo] = sg[:, :, c[halo]]
        g.step(v, sg, 1, t0=t0)
        loc.step_tiled(s, lv, ls, 1, t0=t0)
        ref = max(np.abs(v).max(), np.abs(sg).max())
        err = max(np.abs(lv[:, :, own] - v[:, :, c[own]]).max(), np.abs(ls[:, :, own] - sg[:, :, c[own]]).max()) / ref
        worst = max(worst, err)
    print(f"P{k} order {order}: owned cells vs whole mesh, max-abs / max {worst:.2e}")
    assert worst <= 1e-13
    assert npk > 0


def test_regions_rejected_combinations():
    m, g, P, loc = _part_dg(10, 1, 4, 1, 0x8, 2, 2, 0, 6)
    ch = loc.chain()
    with pytest.raises(RuntimeError):
        ch.inspect(5, seed_region=P.region, max_colour_tiles=2)
    bad = P.region.copy()
    bad[0] = 3
    with pytest.raises(RuntimeError):
        ch.inspect(5, seed_region=bad)
    with pytest.raises(RuntimeError):  # a sub-chain starting on the facet set
        ch.inspect(5, seed_region=P.region, splits=(1,))
    # a chain writing a set other than the seed set cannot carry stale data
    c2 = O.OChain()
    A = c2.set(4)
    B = c2.set(2)
    mp = c2.map(B, A, 2, [[0, 1], [2, 3]])
    c2.loop(A, [(-1, O.R, 0)])
    c2.loop(B, [(mp, O.R, 0), (-1, O.W, 1)])
    reg = np.array([0, 1, 1, 2], np.uint8)
    with pytest.raises(RuntimeError):
        c2.inspect(1, seed_region=reg, carry=1)
    s = c2.inspect(1, seed_region=reg, carry=0)
    assert s.check() == 0
