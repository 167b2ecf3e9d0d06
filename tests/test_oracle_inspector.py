"""Pins of the oracle inspector (Alg. 1, 3, 4) and executor (Alg. 2).

* the shared-memory worked example of Sec. 3.2 (a vertex with 7 incident
  edges, 2 in the green tile and 5 in the blue one, projects to blue; a cell
  touching blue, green, green vertices goes to blue);
* the conflict scenario of Sec. 3.2 (same-coloured tiles becoming adjacent)
  is resolved by fake connections;
* on random tiny meshes the brute-force dependence checker finds no violation,
  every iteration has exactly one tile, and an integer-instrumented chain gives
  bit-identical data tiled and untiled;
* the checker catches a swapped colour pair and the literal (bottom-reset)
  reading of the projection algorithm;
* the tiled DG chain equals the untiled one to rounding (<= 1e-14 relative).
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1708_03183_amd import inputs as I

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "running_example_sec3.json")))


def _wheel_chain():
    # vertex v0 in the middle of 7 rim vertices v1..v7; spokes e0..e6 = (v0, v_{i+1}),
    # rim edges e7..e13 = (v_{i+1}, v_{(i+1)%7+1}); cells c_i = (v0, v_{i+1}, v_{(i+1)%7+1})
    e2v = [[0, i + 1] for i in range(7)] + [[i + 1, (i + 1) % 7 + 1] for i in range(7)]
    c2v = [[0, i + 1, (i + 1) % 7 + 1] for i in range(7)]
    ch = O.OChain()
    E = ch.set(14)
    Cs = ch.set(7)
    V = ch.set(8)
    e2vm = ch.map(E, V, 2, e2v)
    c2vm = ch.map(Cs, V, 3, c2v)
    # the toy program of Fig. 2: L0 edges inc vertices; L1 cells inc vertices; L2 edges read vertices
    ch.loop(E, [(-1, O.R, 0), (e2vm, O.INC, 1)])
    ch.loop(Cs, [(-1, O.R, 2), (c2vm, O.INC, 1)])
    ch.loop(E, [(-1, O.W, 0), (e2vm, O.R, 1)])
    return ch


def test_worked_example_projection_and_tiling():
    g = GOLDEN
    order = g["colour_order"]
    ch = _wheel_chain()
    # green tile T0 holds spokes e0, e1 and rim edges e7, e8, e13; blue tile T1 the rest
    tile0 = np.ones(14, np.int32)
    tile0[[0, 1, 7, 8, 13]] = 0
    spokes = tile0[:7]
    assert (len(spokes), int((spokes == 0).sum()), int((spokes == 1).sum())) == (
        g["projection"]["incident_edges"], g["projection"]["green_edges"], g["projection"]["blue_edges"])
    color = np.array([order["green"], order["blue"]], np.int32)  # tile 0 green, tile 1 blue
    phi = ch.projection_after(tile0, 2, color, 1, 2, 8)
    assert phi[0] == 1 and color[phi[0]] == order[g["projection"]["phi_v0"]]
    assert phi[1] == 0 and phi[2] == 0   # v1, v2 touch only green edges
    assert [int(color[phi[v]]) for v in (0, 1, 2)] == [order[c] for c in g["cell_tiling"]["vertex_projections"]]
    sig = ch.tile_with_colors(tile0, 2, color, [14, 7, 14])
    # cell c0 = (v0, v1, v2): MAX(B, G, G) = B
    assert sig[1][0] == g["cell_tiling"]["sigma"]


def test_inverse_map_example():
    # Fig. 8: cell 1 -> vertices {3, 7, 9}; the inverse map lists cell 1 under each
    ex = GOLDEN["inverse_map"]
    c2v = np.array([[0, 1, 2], ex["vertices"], [2, 3, 4]], np.int32)
    inv = {}
    for c, vs in enumerate(c2v):
        for v in vs:
            inv.setdefault(int(v), []).append(c)
    assert all(ex["cell"] in inv[v] for v in ex["vertices"])
    # the oracle's projection realises exactly this: a tile written only by cell 1
    ch = O.OChain()
    Cs = ch.set(3)
    V = ch.set(10)
    m = ch.map(Cs, V, 3, c2v)
    ch.loop(Cs, [(m, O.INC, 0)])
    ch.loop(V, [(-1, O.R, 0)])
    phi = ch.projection_after(np.array([0, 1, 2], np.int32), 3, np.array([0, 1, 2], np.int32), 1, V, 10)
    assert phi[7] == 1 and phi[9] == 1 and phi[3] == 2  # vertex 3 also touched by cell 2 (higher colour)


def _strip_chain(n, nloops):
    # 1-D strip of n cells with n-1 interior faces; alternate cell/face loops
    f2c = np.array([[i, i + 1] for i in range(n - 1)], np.int32)
    ch = O.OChain()
    Cs = ch.set(n)
    F = ch.set(n - 1)
    m = ch.map(F, Cs, 2, f2c)
    d = 0
    for j in range(nloops):
        if j % 2 == 0:
            ch.loop(Cs, [(-1, O.R, d), (-1, O.W, d + 1)])
        else:
            ch.loop(F, [(m, O.R, d), (m, O.INC, d + 1)])
        d += 1
    return ch


def test_conflicts_resolved_by_fake_connections():
    # thin middle tiles get swallowed by growth; equal-coloured tiles meet
    ch = _strip_chain(40, 11)
    with pytest.raises(RuntimeError):
        ch.inspect(4, max_rounds=1)   # the first colouring conflicts
    s = ch.inspect(4, max_rounds=64)
    assert s.sub_info(0)["rounds"] >= 2
    assert s.check() == 0
    assert ch.instrumented(None) == ch.instrumented(s)


def _dg(n, k=1, jit=0.2, ren=None, order=4, flux=1, free=0x8):
    m = I.square_mesh(n, jitter=jit, renumber_seed=ren)
    om = O.OMesh.from_mesh(m)
    d = O.ODG(om, k, *I.layered_material(m), flux=flux, order=order, free_sides=free)
    return m, om, d


CASES = [(n, order, flux, ts, part, ren)
         for n in (3, 6, 11)
         for order in (2, 4)
         for flux in (0, 1)
         for ts in (1, 5, 17, 64)
         for part in (0, 1)
         for ren in (None, 7)
         if not (flux == 0 and ren is None and part == 1)]


@pytest.mark.parametrize("n,order,flux,ts,part,ren", CASES[::3])
def test_random_meshes_legal_schedules(n, order, flux, ts, part, ren):
    m, om, d = _dg(n, order=order, flux=flux, ren=ren)
    ch = d.chain()
    s = ch.inspect(ts, partition=part, seed_xy=m.centroids())
    assert s.check() == 0
    info = s.sub_info(0)
    assert ch.instrumented(None) == ch.instrumented(s)
    # tiles of one colour never share an element (the colouring invariant)
    off, el, acc = s.footprint(0, 0)
    col = s.colors(0)
    owner = {}
    for t in range(info["ntiles"]):
        for x in el[off[t]:off[t + 1]]:
            owner.setdefault(int(x), set()).add(t)
    for x, ts_ in owner.items():
        cols = [col[t] for t in ts_]
        assert len(cols) == len(set(cols))
        single = (acc[off[min(ts_)]:off[min(ts_) + 1]][el[off[min(ts_)]:off[min(ts_) + 1]] == x][0] >> 31) & 1
        assert single == (len(ts_) == 1)


def test_every_iteration_once():
    m, om, d = _dg(9, order=4, ren=3)
    ch = d.chain()
    s = ch.inspect(10, partition=1, seed_xy=m.centroids())
    sizes = [om.nc, om.nf, om.nb, om.nc] * 3 + [om.nc]
    sizes = sizes + sizes
    for j in range(ch.nloops):
        off, it = s.iters(j, sizes[j], 0)
        assert off[-1] == sizes[j]
        assert sorted(it.tolist()) == list(range(sizes[j]))
        for t in range(len(off) - 1):
            seg = it[off[t]:off[t + 1]]
            assert np.all(np.diff(seg) > 0)


def test_checker_catches_swapped_colours():
    m, om, d = _dg(8, order=4, ren=3)
    ch = d.chain()
    s = ch.inspect(8, partition=1, seed_xy=m.centroids())
    assert s.check() == 0
    col = s.colors(0)
    a = 0
    b = int(np.nonzero(col != col[a])[0][0])
    s.set_color(0, a, int(col[b]))
    s.set_color(0, b, int(col[a]))
    assert s.check() > 0


def test_checker_catches_literal_projection():
    m, om, d = _dg(8, order=4, ren=3)
    ch = d.chain()
    O.set_literal_projection(True)
    try:
        s = ch.inspect(8, partition=1, seed_xy=m.centroids())
        viol = s.check()
    finally:
        O.set_literal_projection(False)
    assert viol > 0


@pytest.mark.parametrize("order,flux,free,k", [(4, 1, 0x8, 2), (2, 1, 0x8, 1), (4, 0, 0xF, 3), (2, 0, 0x3, 2)])
def test_tiled_equals_untiled_dg(order, flux, free, k):
    m, om, d = _dg(12, k=k, order=order, flux=flux, free=free, ren=5)
    d.set_source(0.43, 0.52)
    ch = d.chain()
    s = ch.inspect(20, partition=1, seed_xy=m.centroids(), splits=(13,) if order == 4 else ())
    v, sg = d.zeros()
    v[:] = I.random_state(v.shape, 1)
    sg[:] = I.random_state(sg.shape, 2)
    v2, s2 = v.copy(), sg.copy()
    d.step(v, sg, 4, t0=0.1)
    d.step_tiled(s, v2, s2, 4, t0=0.1)
    ref = np.sqrt((v ** 2).sum() + (sg ** 2).sum())
    err = np.sqrt(((v - v2) ** 2).sum() + ((sg - s2) ** 2).sum()) / ref
    print("tiled vs untiled relative L2", err)
    assert err <= 1e-14


def test_hilbert_partition_compact():
    # Hilbert chunks of a randomly renumbered mesh cut far fewer facets than
    # chunks of the random numbering
    m, om, d = _dg(32, k=1, ren=9)
    mp = om.maps()
    c = m.centroids()

    def cut(part):
        ch = d.chain()
        s = ch.inspect(64, partition=part, seed_xy=c)
        sig = s.sigma(0, om.nc)
        return int(np.sum(sig[mp["f2c"][:, 0]] != sig[mp["f2c"][:, 1]]))

    assert cut(1) * 4 < cut(0)


@pytest.mark.parametrize("cap", [1, 2, 3, 5, 9])
def test_colour_class_cap(cap):
    """The colour-class cap keeps every class within the cap, the colouring proper
    (the checker finds no violation) and the chain's result unchanged."""
    m, om, d = _dg(11, ren=7)
    base = d.chain().inspect(5, partition=1, seed_xy=m.centroids(), splits=(13,))
    s = d.chain().inspect(5, partition=1, seed_xy=m.centroids(), splits=(13,), max_colour_tiles=cap)
    assert s.check() == 0
    for sub in range(s.nsub):
        co, _ = s.tiles_by_color(sub)
        sizes = np.diff(co)
        assert sizes.max() <= cap and sizes.sum() == s.sub_info(sub)["ntiles"]
    ch = d.chain()
    assert ch.instrumented(None) == ch.instrumented(s)
    # a cap at least as large as every class leaves the schedule as it was
    big = max(int(np.diff(base.tiles_by_color(q)[0]).max()) for q in range(base.nsub))
    same = d.chain().inspect(5, partition=1, seed_xy=m.centroids(), splits=(13,), max_colour_tiles=big)
    for q in range(base.nsub):
        assert np.array_equal(same.colors(q), base.colors(q))


def test_colour_class_cap_greedy_order():
    """On a strip of cells the tiles form a path; cap 1 forces one tile per colour
    and the pass must still give neighbouring tiles different colours."""
    ch = _strip_chain(40, 3)
    s = ch.inspect(10, max_colour_tiles=1)
    co, tl = s.tiles_by_color(0)
    assert np.all(np.diff(co) <= 1)
    col = s.colors(0)
    assert all(col[t] != col[t + 1] for t in range(len(col) - 1))
    assert s.check() == 0


def test_sub_chains_with_their_own_tile_sizes():
    """A fusion scheme gives each sub-chain its own seed tile size: each sub-chain's
    schedule equals that of an inspection with its tile size for all sub-chains, the
    whole schedule is legal, and the tiled chain equals the untiled one."""
    m, om, d = _dg(12, k=2, order=4, flux=1, free=0x8, ren=5)
    d.set_source(0.43, 0.52)
    ch = d.chain()
    xy = m.centroids()
    mixed = ch.inspect(8, partition=1, seed_xy=xy, splits=(13,), sub_tile_sizes=(12, 30))
    assert mixed.check() == 0
    sizes = [om.nc, om.nf, om.nb, om.nc] * 3 + [om.nc]
    sizes = sizes + sizes
    for sub, ts in ((0, 12), (1, 30)):
        ref = ch.inspect(ts, partition=1, seed_xy=xy, splits=(13,))
        assert mixed.sub_info(sub) == ref.sub_info(sub)
        assert np.array_equal(mixed.colors(sub), ref.colors(sub))
        first, n = ref.sub_info(sub)["first"], ref.sub_info(sub)["nloops"]
        for j in range(first, first + n):
            assert np.array_equal(mixed.sigma(j, sizes[j]), ref.sigma(j, sizes[j]))
    assert mixed.sub_info(0)["ntiles"] == -(-om.nc // 12) and mixed.sub_info(1)["ntiles"] == -(-om.nc // 30)
    v, sg = d.zeros()
    v[:] = I.random_state(v.shape, 1)
    sg[:] = I.random_state(sg.shape, 2)
    v2, s2 = v.copy(), sg.copy()
    d.step(v, sg, 3, t0=0.1)
    d.step_tiled(mixed, v2, s2, 3, t0=0.1)
    err = np.sqrt(((v - v2) ** 2).sum() + ((sg - s2) ** 2).sum()) / np.sqrt((v ** 2).sum() + (sg ** 2).sum())
    assert err <= 1e-14


def _hilbert_ranks(xy):
    """Seed ranks of points under the Hilbert partition: one seed per tile, so the
    tile of seed i is its rank along the curve."""
    ch = O.OChain()
    st = ch.set(len(xy))
    ch.loop(st, [(-1, O.R, 0)])
    s = ch.inspect(1, partition=1, seed_xy=np.ascontiguousarray(xy, np.float64))
    return s.sigma(0, len(xy))


# The order-2 Hilbert curve on a 4x4 grid, derived by hand from its construction:
# the top level visits the quadrants (0,0) -> (0,1) -> (1,1) -> (1,0) (x right, y up);
# the lower-left quadrant is the order-1 curve transposed (enter at (0,0), leave
# upwards at (0,1)), the two upper quadrants repeat the order-1 curve unrotated,
# and the lower-right quadrant is the order-1 curve reflected in the anti-diagonal
# (enter at (3,1) from above, leave at (3,0)).
HILBERT_ORDER2 = [(0, 0), (1, 0), (1, 1), (0, 1), (0, 2), (0, 3), (1, 3), (1, 2),
                  (2, 2), (2, 3), (3, 3), (3, 2), (3, 1), (2, 1), (2, 0), (3, 0)]


def test_hilbert_order2_curve_by_hand():
    """Cell centres of a 4x4 grid, plus the two corners that fix the bounding box at
    the unit square, ranked by the seed order: the 16 centres come in the order of
    the hand-derived order-2 curve (the 2^16 curve visits each quarter-of-a-quarter
    whole before the next)."""
    pts = [((x + 0.5) / 4, (y + 0.5) / 4) for (x, y) in HILBERT_ORDER2[::-1]]  # listed backwards on purpose
    xy = np.array(pts + [(0.0, 0.0), (1.0, 1.0)])
    r = _hilbert_ranks(xy)
    order = [int(i) for i in np.argsort(r) if i < 16]
    assert [HILBERT_ORDER2[::-1][i] for i in order] == HILBERT_ORDER2


def test_hilbert_curve_is_continuous_at_order4():
    """On a 16x16 grid of cell centres consecutive seeds along the curve are edge
    neighbours (a property of the Hilbert curve at every level; a wrong rotation
    or reflection in any level breaks it), it starts in the lower-left cell and
    ends in the lower-right one."""
    g = [(x, y) for y in range(16) for x in range(16)]
    xy = np.array([((x + 0.5) / 16, (y + 0.5) / 16) for (x, y) in g] + [(0.0, 0.0), (1.0, 1.0)])
    r = _hilbert_ranks(xy)
    walk = [g[i] for i in np.argsort(r) if i < 256]
    assert walk[0] == (0, 0) and walk[-1] == (15, 0)
    steps = [abs(a[0] - b[0]) + abs(a[1] - b[1]) for a, b in zip(walk, walk[1:])]
    assert steps == [1] * 255


@pytest.mark.parametrize("order,steps,splits,k", [(2, 2, (), 1), (2, 3, (), 2), (2, 2, (4, 12), 1),
                                                  (4, 2, (13, 39), 1), (4, 2, (13, 26, 39), 2)])
def test_chain_fused_over_steps(order, steps, splits, k):
    """A chain of several time steps (the step's loops repeated) tiled in one pass per
    sub-chain: the schedule is legal, the integer-instrumented chain is bit-identical
    tiled and untiled, and the tiled DG run (F steps per pass, each loop at its own
    step's time) equals the untiled one to rounding."""
    m, om, d = _dg(11, k=k, order=order, flux=1, free=0x8, ren=5)
    d.set_source(0.43, 0.52)
    ch = d.chain(steps)
    assert ch.nloops == steps * d.chain().nloops
    s = ch.inspect(9, partition=1, seed_xy=m.centroids(), splits=splits)
    assert s.check() == 0
    assert ch.instrumented(None) == ch.instrumented(s)
    v, sg = d.zeros()
    v[:] = I.random_state(v.shape, 3)
    sg[:] = I.random_state(sg.shape, 4)
    v2, s2 = v.copy(), sg.copy()
    n = 2 * steps
    d.step(v, sg, n, t0=0.1)
    d.step_tiled(s, v2, s2, n, t0=0.1)
    err = max(np.abs(v - v2).max(), np.abs(sg - s2).max()) / max(np.abs(v).max(), np.abs(sg).max())
    print(f"order {order}, {steps} steps per chain, splits {splits}: tiled vs untiled {err:.2e}")
    assert err <= 1e-14
    with pytest.raises(ValueError):  # not a multiple of the fused steps
        d.step_tiled(s, v2, s2, steps + 1, t0=0.0)
