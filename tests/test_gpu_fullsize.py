"""GPU parity at the workloads' full sizes, in the launch configurations bench.py times.

The oracle cannot run a 0.5-2 M cell mesh in seconds, but one step of the chain
only reaches a bounded neighbourhood: every operator application has one facet
loop, so a cell's state after s order-4 steps depends only on cells at most 6 s
facet-neighbour layers away.  For sampled cells (random ones, the source cell, the
free-surface edge and the corners) the oracle runs the same steps on the patch of
cells within 6 s + 1 layers (same geometry, material, state and source, cells kept
in their mesh order so the source lands in the same cell) and the sampled cells'
values are compared with the GPU's full-mesh run.
"""
import numpy as np
import pytest

import oracle as O
from paper_1708_03183_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

OPS = (4, 8, 13, 17, 21)


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_03183_amd import dgtile
    dgtile.lib()
    return dgtile


def _cfl_dt(m, lam, mu, rho, k):
    p = m.xy[m.c2v]
    e = [np.hypot(*(p[:, (i + 1) % 3] - p[:, i]).T) for i in range(3)]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    hmin = float(np.min(4.0 * area / (e[0] + e[1] + e[2])))
    return 0.2 * hmin / ((2 * k + 1) * float(np.max(np.sqrt((lam + 2 * mu) / rho))))


def _adjacency(m):
    f2c = O.OMesh.from_mesh(m).maps()["f2c"].astype(np.int64)
    a = np.concatenate([f2c[:, 0], f2c[:, 1]])
    b = np.concatenate([f2c[:, 1], f2c[:, 0]])
    order = np.argsort(a, kind="stable")
    off = np.zeros(m.nc + 1, np.int64)
    np.add.at(off, a + 1, 1)
    return np.cumsum(off), b[order]


def _patch(off, nb, c, layers):
    seen = {int(c)}
    front = [int(c)]
    for _ in range(layers):
        nxt = []
        for x in front:
            for y in nb[off[x]:off[x + 1]]:
                y = int(y)
                if y not in seen:
                    seen.add(y)
                    nxt.append(y)
        front = nxt
    return np.array(sorted(seen), np.int64)


def _samples(m, rng, nrand, src):
    cen = m.xy[m.c2v].mean(axis=1)
    picks = list(rng.choice(m.nc, nrand, replace=False))
    for target in (src, (0.5, 0.999), (0.001, 0.001), (0.999, 0.999), (0.001, 0.5)):
        picks.append(int(np.argmin(((cen - np.asarray(target)) ** 2).sum(axis=1))))
    return sorted(set(int(x) for x in picks))


def _oracle_on_patch(m, cells, lam, mu, rho, k, order, dt, v, s, steps, src, t0):
    c2v = m.c2v[cells]
    verts, inv = np.unique(c2v.ravel(), return_inverse=True)
    om = O.OMesh(m.xy[verts], inv.reshape(-1, 3).astype(np.int32))
    od = O.ODG(om, k, lam[cells], mu[cells], rho[cells], flux=1, order=order, dt=dt, free_sides=0x8)
    try:
        od.set_source(*src)
    except ValueError:
        pass  # the source lies outside the patch and cannot reach its centre in `steps` steps
    pv = np.ascontiguousarray(v[:, :, cells])
    ps = np.ascontiguousarray(s[:, :, cells])
    od.step(pv, ps, steps, t0=t0)
    return pv, ps


FULL_CASES = [
    # name, n, k, prec, tile size (or one per sub-chain), splits, schedule, steps, shots, DGT_TILE_OP
    ("jitter512_p2_fp64", 512, 2, 0, 256, (13,), 1, 2, 1, None),
    ("jitter512_p2_fp32", 512, 2, 1, (256, 128), (13,), 1, 2, 1, None),
    # P3/P4 on the lognormal material: the matrix-core kernel (default), the register-resident
    # kernel in its own best configuration, and FP64 in the configuration of the FP32-vs-FP64 runs
    ("jitter1024_p3_fp32", 1024, 3, 1, 256, OPS, 0, 1, 1, None),
    ("jitter1024_p4_fp32", 1024, 4, 1, 256, OPS, 0, 1, 1, None),
    ("jitter1024_p3_fp32_register", 1024, 3, 1, 192, OPS, 1, 1, 1, "1"),
    ("jitter1024_p4_fp32_register", 1024, 4, 1, 192, OPS, 0, 1, 1, "1"),
    ("jitter1024_p3_fp64", 1024, 3, 0, 192, OPS, 0, 1, 1, None),
    ("jitter1024_p4_fp64", 1024, 4, 0, 128, OPS, 0, 1, 1, None),
    ("jitter416_p2_fp32_11shots", 416, 2, 1, 256, (13,), 0, 2, 11, None),
]


@pytest.mark.parametrize("name,n,k,prec,ts,splits,schedule,steps,shots,kern", FULL_CASES)
def test_full_size_sampled_cells_match_oracle(D, monkeypatch, name, n, k, prec, ts, splits, schedule, steps, shots,
                                             kern):
    print(f"case {name}: building the mesh", flush=True)
    if kern is not None:
        monkeypatch.setenv("DGT_TILE_OP", kern)
    m = I.square_mesh(n, jitter=0.2, jitter_seed=1, renumber_seed=2)
    lam, mu, rho = I.lognormal_material(m) if k >= 3 else I.layered_material(m)
    dt = _cfl_dt(m, lam, mu, rho, k)
    npk = (k + 1) * (k + 2) // 2
    rng = np.random.default_rng(7)
    srcs = [(0.5, 0.5)] + [tuple(x) for x in rng.uniform(0.1, 0.9, size=(shots - 1, 2))]
    # random start states (FP64 values rounded to the solver precision, used by both sides)
    dtype = torch.float32 if prec else torch.float64
    v = np.stack([I.random_state((2, npk, m.nc), 11 + 2 * q) for q in range(shots)])
    s = np.stack([I.random_state((3, npk, m.nc), 12 + 2 * q) for q in range(shots)])
    if prec:
        v, s = v.astype(np.float32).astype(np.float64), s.astype(np.float32).astype(np.float64)
    gm = D.Mesh.from_mesh(m)
    g = D.Solver(gm, lam, mu, rho, degree=k, flux=1, time_order=4, precision=prec, free_sides=0x8, dt=dt)
    if shots > 1:
        g.set_shots(shots, np.array(srcs))
    else:
        g.set_source(*srcs[0])
    if isinstance(ts, tuple):
        g.inspect(ts[0], partition=1, splits=splits, sub_tile_sizes=ts)
    else:
        g.inspect(ts, partition=1, splits=splits)
    g.set_schedule(schedule)
    kinds = g.kernels()
    assert set(kinds) == ({1} if kern == "1" or k <= 2 else {2}), kinds
    gv = torch.from_numpy(v if shots > 1 else v[0]).to(dtype).cuda().contiguous()
    gs = torch.from_numpy(s if shots > 1 else s[0]).to(dtype).cuda().contiguous()
    g.upload(gv, gs)
    t0 = 0.1
    g.step(steps, mode=1, t0=t0)
    g.download(gv, gs)
    torch.cuda.synchronize()
    rv = gv.double().cpu().numpy().reshape(shots, 2, npk, m.nc)
    rs = gs.double().cpu().numpy().reshape(shots, 3, npk, m.nc)
    off, nb = _adjacency(m)
    num = den = 0.0
    worst = 0.0
    for q in ([0, shots - 1] if shots > 1 else [0]):
        cells = _samples(m, rng, 16, srcs[q])
        for c in cells:
            patch = _patch(off, nb, c, 6 * steps + 1)
            pv, ps = _oracle_on_patch(m, patch, lam, mu, rho, k, 4, dt, v[q], s[q], steps, srcs[q], t0)
            j = int(np.searchsorted(patch, c))
            dv = rv[q][:, :, c] - pv[:, :, j]
            ds = rs[q][:, :, c] - ps[:, :, j]
            e = float((dv ** 2).sum() + (ds ** 2).sum())
            r = float((pv[:, :, j] ** 2).sum() + (ps[:, :, j] ** 2).sum())
            num += e
            den += r
            worst = max(worst, np.sqrt(e / r))
    err = np.sqrt(num / den)
    print(f"{name}: {m.nc} cells, ts={ts}, splits={splits}, schedule={schedule}, {steps} steps, {shots} shot(s): "
          f"sampled cells rel L2 err vs FP64 oracle {err:.3e} (worst cell {worst:.3e})")
    tol = 1e-5 if prec else 1e-12
    assert err <= tol and worst <= 10 * tol


def test_full_size_energy_conserved_over_1000_tiled_steps(D):
    """The discrete energy invariant on the 512x512 bench mesh (524,288 cells, P2,
    FP64, three layers): central flux and free surfaces on every side conserve it
    exactly, so after 1000 tiled steps in the bench's launch configuration (256
    seeds, half steps, dependence-driven) it may move only by rounding."""
    m = I.square_mesh(512, jitter=0.2, jitter_seed=1, renumber_seed=2)
    lam, mu, rho = I.layered_material(m)
    dt = _cfl_dt(m, lam, mu, rho, 2)
    g = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=2, flux=0, time_order=4, precision=0, free_sides=0xF,
                 dt=dt)
    g.inspect(256, partition=1, splits=(13,))
    g.set_schedule(1)
    v, s = g.zeros()
    v.copy_(torch.from_numpy(I.random_state(tuple(v.shape), 41)))
    s.copy_(torch.from_numpy(I.random_state(tuple(s.shape), 42)))
    s_start = s.clone()
    g.upload(v, s)
    energies = []
    done = 0
    for target in (1, 500, 1000):
        if target - 1 > done:
            g.step(target - 1 - done, mode=1, t0=done * dt)
            done = target - 1
        g.download(v, s)
        so = s.clone()
        g.step(1, mode=1, t0=done * dt)
        done = target
        g.download(v, s)
        energies.append(g.energy(v, s, so))
    drift = max(abs(e - energies[0]) for e in energies) / energies[0]
    moved = ((s - s_start).norm() / s_start.norm()).item()
    # (rounding moves a sum of 15.7 M terms by far less than its last bit: the energies may agree exactly)
    print(f"full-size energy over 1000 tiled steps: {energies}, relative drift {drift:.3e}; "
          f"the stress moved by {moved:.3f} of its norm")
    assert drift <= 1e-12
    assert moved > 0.1  # the state did evolve


def test_full_size_part_block_matches_oracle(D):
    """One GPU's share of the 1024x1024 P3 FP32 workload: block 5 of 2 x 4 rectangular
    blocks (262,144 owned cells), 6 exec halo layers and one non-exec layer, inspected
    with regions in the bench's launch configuration; before each of 2 steps the halo
    takes a whole-mesh GPU solver's state by pack / unpack.  Every owned cell follows
    the whole-mesh solver, and sampled owned cells (random ones and ones next to the
    halo) match the FP64 oracle run on their patches of the whole mesh."""
    k, steps, t0 = 3, 2, 0.1
    m = I.square_mesh(1024, jitter=0.2, jitter_seed=1, renumber_seed=2)
    lam, mu, rho = I.lognormal_material(m)
    dt = _cfl_dt(m, lam, mu, rho, k)
    npk = (k + 1) * (k + 2) // 2
    P = I.mesh_part(m, I.block_parts(m, 2, 4), 5, 6)
    c = P.cells
    print(f"part: {int(P.owned.sum())} owned, {int(np.sum(P.region == 0))} core, {c.size} local cells", flush=True)
    v = I.random_state((2, npk, m.nc), 51).astype(np.float32).astype(np.float64)
    s = I.random_state((3, npk, m.nc), 52).astype(np.float32).astype(np.float64)
    src = (0.75, 0.6)
    g = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=k, flux=1, time_order=4, precision=1, free_sides=0x8,
                 dt=dt)
    g.set_source(*src)
    g.inspect(256, partition=1, splits=OPS)
    lp = D.Solver(D.Mesh.from_mesh(P.mesh), lam[c], mu[c], rho[c], degree=k, flux=1, time_order=4, precision=1,
                  free_sides=0x8, dt=dt)
    lp.set_source(*src)
    lp.inspect(256, partition=1, splits=OPS, seed_region=P.region, region_carry=1)
    assert set(lp.kernels()) == {2}
    gv = torch.from_numpy(v).float().cuda().contiguous()
    gs = torch.from_numpy(s).float().cuda().contiguous()
    g.upload(gv, gs)
    ci = torch.from_numpy(c.astype(np.int64)).cuda()
    lp.upload(gv[:, :, ci].contiguous(), gs[:, :, ci].contiguous())
    halo = np.nonzero(~P.owned)[0]
    send, recv = g.cell_list(c[halo]), lp.cell_list(halo)
    bv = torch.empty(2, npk, halo.size, dtype=torch.float32, device="cuda")
    bs = torch.empty(3, npk, halo.size, dtype=torch.float32, device="cuda")
    for i in range(steps):
        g.pack(send, bv, bs)
        lp.unpack(recv, bv, bs)
        g.step(1, mode=1, t0=t0 + i * dt)
        lp.step(1, mode=1, t0=t0 + i * dt)
    lv, ls = lp.zeros()
    lp.download(lv, ls)
    g.download(gv, gs)
    torch.cuda.synchronize()
    own = np.nonzero(P.owned)[0]
    oi = torch.from_numpy(own.astype(np.int64)).cuda()
    ref = max(gv.abs().max().item(), gs.abs().max().item())
    diff = max((lv[:, :, oi] - gv[:, :, ci[oi]]).abs().max().item(),
               (ls[:, :, oi] - gs[:, :, ci[oi]]).abs().max().item()) / ref
    print(f"owned cells vs whole-mesh GPU solver after {steps} steps: max-abs / max = {diff:.3e}")
    assert diff <= 1e-5
    rv, rs = lv.double().cpu().numpy(), ls.double().cpu().numpy()
    rng = np.random.default_rng(9)
    edge = own[np.nonzero(P.region[own] == 1)[0]]
    picks = sorted(set(int(x) for x in np.concatenate([rng.choice(own, 6, replace=False),
                                                       rng.choice(edge, 6, replace=False)])))
    off, nb = _adjacency(m)
    worst = 0.0
    for j in picks:
        cg = int(c[j])
        patch = _patch(off, nb, cg, 6 * steps + 1)
        pv, ps = _oracle_on_patch(m, patch, lam, mu, rho, k, 4, dt, v, s, steps, src, t0)
        q = int(np.searchsorted(patch, cg))
        e = np.sqrt(((rv[:, :, j] - pv[:, :, q]) ** 2).sum() + ((rs[:, :, j] - ps[:, :, q]) ** 2).sum())
        r = np.sqrt((pv[:, :, q] ** 2).sum() + (ps[:, :, q] ** 2).sum())
        worst = max(worst, e / r)
    print(f"sampled owned cells (6 random, 6 next to the halo) vs FP64 oracle: worst cell rel L2 {worst:.3e}")
    assert worst <= 1e-4
