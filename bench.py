"""Benchmark: DG dof-updates/s of the sparse-tiled fused time step vs the
untiled chain on one MI355X.

Workload (default): 512x512 jittered (0.2h) and randomly renumbered unit-square
triangulation, 524288 cells, DG P2 velocity-stress elastic, three-layer
material, upwind flux, free surface on top and absorbing elsewhere, Ricker
source at (0.5, 0.5), 4th-order Taylor leapfrog (26 loops per step), tiles
grown from 256 seed cells in Hilbert order, the chain fused per half step,
tiles of a half step started by dependence counters in one launch.

Prints ONE JSON line.  `value` is the tiled-fused rate in dof-updates/s (5
fields x Np nodes x cells per step, per second) with the state resident in HBM.
Reported beside it: the untiled chain on the same (Hilbert) cell order and on
the mesh's own order, the inspector time and the steps that amortise it, the
measured error against the FP64 oracle, the tile kernel's roofline from HIP
events, and the oracle timed on the host; then, as extra keys, the 1024x1024
P3/P4 FP32 workload, a tile-size sweep, one GPU's part of the 1024x1024 mesh,
the batched shots on six meshes (`config4`, shortened to --config4-steps) and
the FWI gradient (`config5`).  --workload batched / fwi print those two
records alone, at full length.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512, help="squares per side")
    ap.add_argument("--degree", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--tile-size", type=int, default=None)
    ap.add_argument("--splits", type=str, default=None, help="comma-separated loop indices, or 'none'")
    ap.add_argument("--sub-tile-sizes", type=str, default=None,
                    help="comma-separated seed tile size of each sub-chain (one more than the splits)")
    ap.add_argument("--colour-cap", type=int, default=0,
                    help="tiles per colour class: -1 the GPU's resident tile workgroups, 0 uncapped")
    ap.add_argument("--schedule", type=int, default=None,
                    help="tiled executor: 0 one launch per colour, 1 dependence-driven (one launch per sub-chain)")
    ap.add_argument("--partition", type=int, choices=[0, 1], default=1,
                    help="seed partition: 1 Hilbert order of the cell centroids, 0 chunks of the mesh numbering")
    ap.add_argument("--mesh-order", choices=["renumbered", "natural"], default="renumbered",
                    help="cell numbering of the mesh: seeded random renumbering, or the generator's row-major order")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-untiled", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--cpu-cores", type=int, default=0,
                    help="host cores of the multi-core oracle baseline (0: min(16, cpu count); 1: skip it)")
    ap.add_argument("--workload", choices=["single", "batched", "fwi"], default="single",
                    help="batched: 64 Ricker shots on 6 uneven meshes (P2 FP32), the batched form against "
                         "the same shots run one at a time; fwi: misfit gradient of 16 shots on a 256x256 "
                         "mesh (P2, FP32 state, FP64 gradient)")
    ap.add_argument("--fwi-steps", type=int, default=2000)
    ap.add_argument("--fwi-snapshots", type=int, default=32)
    ap.add_argument("--fwi-boundaries", choices=["absorbing", "free"], default="absorbing",
                    help="fwi: upwind flux with a free top and absorbing other sides (closed-form transposed "
                         "step), or central flux with free surfaces everywhere (the reversed chain)")
    ap.add_argument("--shots", type=int, default=64)
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="batched workload: steps per HIP graph of the one-launch batch")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched workload: use the fixed P2 FP32 tile size and schedule instead of the autotuner")
    ap.add_argument("--material", choices=["auto", "layered", "lognormal"], default="auto",
                    help="auto: three layers at P1/P2, the smooth lognormal fields (sigma 0.3) at P3/P4")
    ap.add_argument("--no-horizon", action="store_true",
                    help="skip the FP32-against-GPU-FP64 run over the whole step count")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip the 1024x1024 P3/P4 FP32 extras of the default run")
    ap.add_argument("--config3-steps", type=int, default=100)
    ap.add_argument("--no-sweep", action="store_true", help="skip the tile-size sweep (256-4096 seeds)")
    ap.add_argument("--no-config4", action="store_true",
                    help="skip the batched-shots record (six meshes, 64 shots) in the default line")
    ap.add_argument("--config4-steps", type=int, default=50)
    ap.add_argument("--no-config5", action="store_true",
                    help="skip the FWI-gradient record in the default line")
    ap.add_argument("--sweep-steps", type=int, default=20)
    ap.add_argument("--no-part", action="store_true",
                    help="skip one GPU's region-aware share of the 1024x1024 P3 workload")
    ap.add_argument("--config3-horizon", type=int, default=500)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain elementwise pass over 256 MiB (torch.neg: 256 MiB read, 256 MiB "
                         "written) for scaling HBM byte counters")
    return ap.parse_args()


# tuned defaults per (degree, precision): seed tile size, fusion splits (13: half steps;
# 4,8,13,17,21: one operator per sub-chain), schedule (1: dependence-driven) and,
# optionally, a seed tile size per sub-chain
OPS = (4, 8, 13, 17, 21)
DEFAULTS = {
    (1, "fp64"): (256, (13,), 1),
    (2, "fp64"): (256, (13,), 1),
    (2, "fp32"): (128, (13,), 1, (256, 128)),
    (3, "fp32"): (256, OPS, 0),
    (4, "fp32"): (256, OPS, 0),
    (3, "fp64"): (192, OPS, 0),
    (4, "fp64"): (128, OPS, 0),
}
# the register-resident (VALU) kernel's own best settings at P3/P4, for the A/B
VALU_DEFAULTS = {3: (192, OPS, 1), 4: (192, OPS, 0)}


def host_cpu_model():
    """The host processor's model name (Linux), else the platform's description."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def material(m, k, which):
    from paper_1708_03183_amd import inputs as I
    if which == "auto":
        which = "lognormal" if k >= 3 else "layered"
    return (I.lognormal_material(m) if which == "lognormal" else I.layered_material(m)), which


def rel_errors(a, b):
    """relative L2 and max-abs (over max |b|) errors of state pair a against b (torch tensors)"""
    num = math.sqrt(sum(((x.double() - y.double()) ** 2).sum().item() for x, y in zip(a, b)))
    den = math.sqrt(sum((y.double() ** 2).sum().item() for y in b))
    mx = max((x.double() - y.double()).abs().max().item() for x, y in zip(a, b))
    ref = max(y.double().abs().max().item() for y in b)
    return (num / den if den > 0 else 0.0), (mx / ref if ref > 0 else 0.0)


def horizon(D, make_solver, nsteps, k, ref_state, ref_prec, dt):
    """The other precision's run of the same nsteps from rest (with the source),
    against the reference precision's state: the measured FP32 error against GPU
    FP64 over the whole run."""
    import torch
    other = 1 - ref_prec
    ts, splits, schedule, *rest = DEFAULTS[(k, "fp32" if other else "fp64")]
    s = make_solver(other)
    s.inspect(ts, partition=1, splits=splits, sub_tile_sizes=rest[0] if rest else None)
    s.set_schedule(schedule)
    v, st = s.zeros()
    s.upload(v, st)
    t = time.perf_counter()
    s.step(nsteps, mode=1, t0=0.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    s.download(v, st)
    torch.cuda.synchronize()
    f32, f64 = ((v, st), ref_state) if other else (ref_state, (v, st))
    l2, mx = rel_errors(f32, f64)
    return {"steps": nsteps, "fp32_vs_gpu_fp64_rel_l2": l2, "fp32_vs_gpu_fp64_rel_max_abs": mx,
            "other_precision_ms_per_step": 1e3 * wall / nsteps, "from": "rest, Ricker source at (0.5, 0.5)"}


def oracle_patch(m, npk, cpu_steps, budget, centre):
    """The whole mesh when cpu_steps oracle steps on it fit the budget of
    dof-updates, else the cells within enough facet layers of the cell nearest to
    centre; also the cells deeper than 6 cpu_steps layers inside that patch (a
    cell's state after s steps depends only on cells within 6 s facet layers), and
    the patch as a mesh."""
    import numpy as np
    import oracle as O
    nc = m.c2v.shape[0]
    if 5 * npk * nc * cpu_steps <= budget:
        cells = np.arange(nc)
        return cells, cells, m, f"the same {nc}-cell mesh"
    f2c = O.OMesh.from_mesh(m).maps()["f2c"].astype(np.int64)
    src_, dst_ = np.concatenate([f2c[:, 0], f2c[:, 1]]), np.concatenate([f2c[:, 1], f2c[:, 0]])
    order = np.argsort(src_, kind="stable")
    off = np.concatenate([[0], np.cumsum(np.bincount(src_, minlength=nc))])
    nbr = dst_[order]
    cen = m.xy[m.c2v].mean(axis=1)
    depth = {int(np.argmin(((cen - np.asarray(centre)) ** 2).sum(axis=1))): 0}
    front = list(depth)
    want = budget / (5 * npk * cpu_steps)
    layer = 0
    while len(depth) < want or layer < 6 * cpu_steps + 1:
        layer += 1
        nxt = []
        for x in front:
            for y in nbr[off[x]:off[x + 1]]:
                if int(y) not in depth:
                    depth[int(y)] = layer
                    nxt.append(int(y))
        front = nxt
    cells = np.array(sorted(depth), np.int64)
    core = np.array([c for c in cells if depth[c] <= layer - 6 * cpu_steps - 1], np.int64)
    verts, inv = np.unique(m.c2v[cells].ravel(), return_inverse=True)

    class _Sub:
        pass
    sub = _Sub()
    sub.xy, sub.c2v, sub.periodic = m.xy[verts], inv.reshape(-1, 3).astype(np.int32), 0
    where = (f"a {len(cells)}-cell patch ({layer} facet layers around the centre) of the same "
             f"{nc}-cell mesh, {len(core)} cells compared")
    return cells, core, sub, where


def _oracle_worker(args, barrier, queue):
    """One host core's share of the multi-core oracle baseline: the oracle as it
    stands (single-threaded FP64) on a patch of its own, started together with the
    other workers."""
    n, k, mat_name, cpu_steps, budget, centre, seed = args
    import numpy as np
    import oracle as O
    from paper_1708_03183_amd import inputs as I
    m = I.square_mesh(n, jitter=0.2, jitter_seed=1, renumber_seed=2)
    (lam, mu, rho), _ = material(m, k, mat_name)
    npk = (k + 1) * (k + 2) // 2
    dt = cfl_dt(m, lam, mu, rho, k)
    cells, _, sub, _ = oracle_patch(m, npk, cpu_steps, budget, centre)
    om = O.OMesh(sub.xy, sub.c2v, sub.periodic)
    od = O.ODG(om, k, lam[cells], mu[cells], rho[cells], flux=1, order=4, dt=dt, free_sides=0x8)
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, seed)
    s[:] = I.random_state(s.shape, seed + 1)
    barrier.wait()
    t0 = time.time()
    od.step(v, s, cpu_steps, t0=0.0)
    queue.put((5 * npk * len(cells) * cpu_steps, t0, time.time()))


def oracle_multicore(n, k, mat_name, cpu_steps, budget, cores):
    """Aggregate rate of `cores` concurrent oracle processes, each on its own patch
    (the oracle itself is single-threaded and untuned): total dof-updates over the
    span from the first start to the last finish."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(cores)
    queue = ctx.Queue()
    centres = [(0.2 + 0.6 * ((i * 0.618) % 1.0), 0.2 + 0.6 * ((i * 0.382 + 0.5) % 1.0)) for i in range(cores)]
    procs = [ctx.Process(target=_oracle_worker, args=((n, k, mat_name, cpu_steps, budget, centres[i], 50 + 2 * i),
                                                     barrier, queue)) for i in range(cores)]
    for p in procs:
        p.start()
    res = [queue.get(timeout=600) for _ in procs]
    for p in procs:
        p.join(timeout=60)
    work = sum(r[0] for r in res)
    span = max(r[2] for r in res) - min(r[1] for r in res)
    return work / span, span, work


def config3(a):
    """The 1024x1024 P3/P4 FP32 workload (lognormal material): tiled rates on the
    matrix-core kernel (the default at P3/P4) and on the register-resident kernel,
    the untiled chain, and FP32 against GPU FP64 after the workload's 500 steps."""
    import torch
    from paper_1708_03183_amd import dgtile as D
    from paper_1708_03183_amd import inputs as I
    t0 = time.time()
    m = I.square_mesh(1024, jitter=0.2, jitter_seed=1, renumber_seed=2)
    lam, mu, rho = I.lognormal_material(m)
    mesh = D.Mesh.from_mesh(m)
    out = {"workload": "jitter1024: 1024x1024 jittered renumbered triangulation, 2097152 cells, lognormal "
                       "lambda, mu, rho (sigma 0.3), upwind, order-4 leapfrog, FP32",
           "mesh_gen_s": time.time() - t0}

    def timed(sol, mode, steps, warm, dt):
        v, st = sol.zeros()
        sol.upload(v, st)
        sol.step(warm, mode=mode, t0=0.0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sol.step(steps, mode=mode, t0=warm * dt)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / steps

    for k in (3, 4):
        npk = (k + 1) * (k + 2) // 2
        dofs = 5 * npk * mesh.nc
        dt = cfl_dt(m, lam, mu, rho, k)

        def make(pr):
            s = D.Solver(mesh, lam, mu, rho, degree=k, flux=1, time_order=4, precision=pr, free_sides=0x8, dt=dt)
            s.set_source(0.5, 0.5, 5.0, 0.2, 1.0)
            return s
        r = {}
        ts, splits, sch = DEFAULTS[(k, "fp32")]
        s = make(1)
        s.inspect(ts, partition=1, splits=splits)
        s.set_schedule(sch)
        ms = timed(s, 1, a.config3_steps, 10, dt)
        r["mfma"] = {"value": dofs / ms * 1e3, "ms_per_step": ms, "tile_size": ts, "splits": list(splits),
                     "schedule": sch, "kernels": s.kernels()}
        ms_u = timed(s, 0, min(a.config3_steps, 50), 2, dt)
        r["untiled"] = {"value": dofs / ms_u * 1e3, "ms_per_step": ms_u}
        del s
        ts, splits, sch = VALU_DEFAULTS[k]
        os.environ["DGT_TILE_OP"] = "1"
        try:
            s = make(1)
            s.inspect(ts, partition=1, splits=splits)
        finally:
            del os.environ["DGT_TILE_OP"]
        s.set_schedule(sch)
        ms = timed(s, 1, a.config3_steps, 10, dt)
        r["valu"] = {"value": dofs / ms * 1e3, "ms_per_step": ms, "tile_size": ts, "splits": list(splits),
                     "schedule": sch, "kernels": s.kernels()}
        del s
        if a.config3_horizon > 0:
            ref = make(1)
            ts, splits, sch = DEFAULTS[(k, "fp32")]
            ref.inspect(ts, partition=1, splits=splits)
            ref.set_schedule(sch)
            v, st = ref.zeros()
            ref.upload(v, st)
            ref.step(a.config3_horizon, mode=1, t0=0.0)
            ref.download(v, st)
            torch.cuda.synchronize()
            del ref
            r["horizon"] = horizon(D, make, a.config3_horizon, k, (v, st), 1, dt)
        if not a.no_cpu_baseline:
            # the oracle on the host: 2 steps on a patch around the centre sized to ~10 s of
            # one core, reported per dof-update
            import numpy as np
            import oracle as O
            csteps = 2
            cells, _, sub, where = oracle_patch(m, npk, csteps, 1e7, (0.5, 0.5))
            od = O.ODG(O.OMesh(sub.xy, sub.c2v, sub.periodic), k, lam[cells], mu[cells], rho[cells], flux=1,
                       order=4, dt=dt, free_sides=0x8)
            ov, os_ = od.zeros()
            ov[:] = I.random_state(ov.shape, 41)
            os_[:] = I.random_state(os_.shape, 42)
            tc = time.perf_counter()
            od.step(ov, os_, csteps, t0=0.0)
            tcpu = time.perf_counter() - tc
            r["oracle_on_host"] = {"value": 5 * npk * len(cells) * csteps / tcpu, "unit": "dof-updates/s",
                                   "cores": 1, "kind": "oracle", "cpu_model": host_cpu_model(),
                                   "sample": f"{csteps} steps of {where.rsplit(',', 1)[0]} ({tcpu:.1f} s, FP64, single thread)"}
            del od
        out[f"p{k}"] = r
        print(f"bench: config 3 P{k}: mfma {r['mfma']['ms_per_step']:.3f} ms, valu {r['valu']['ms_per_step']:.3f} "
              f"ms, untiled {r['untiled']['ms_per_step']:.3f} ms", file=sys.stderr, flush=True)
    return out


def part_block(a):
    """One GPU's share of the 1024x1024 P3 FP32 workload: the mesh split into rectangular
    blocks, one block with 6 exec halo layers (the facet loops of a step) and one
    non-exec layer, inspected with regions (core tiles, boundary tiles, T_ne).  Before
    every step the halo cells take a whole-mesh solver's state by a device-to-device
    pack / unpack, the stand-in for the exchange between GPUs; the part's step never
    launches T_ne.  Block 5 of 2 x 4 (262,144 owned cells) is checked against the
    whole-mesh solver after two steps and timed with and without the halo fill; parts
    of 1 x 1 (the whole mesh with regions), 1 x 2, 2 x 2, 2 x 4 and 4 x 4 blocks give
    the owned cells' rate against the whole-mesh rate on the same GPU.  Both run the
    register-resident kernel in its P3 configuration (the faster P3 kernel)."""
    import numpy as np
    import torch
    from paper_1708_03183_amd import dgtile as D
    from paper_1708_03183_amd import inputs as I
    k, depth = 3, 6
    npk = (k + 1) * (k + 2) // 2
    m = I.square_mesh(1024, jitter=0.2, jitter_seed=1, renumber_seed=2)
    lam, mu, rho = I.lognormal_material(m)
    dt = cfl_dt(m, lam, mu, rho, k)
    ts, splits, sch = VALU_DEFAULTS[k]
    os.environ["DGT_TILE_OP"] = "1"
    try:
        g = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=k, flux=1, time_order=4, precision=1, free_sides=0x8,
                     dt=dt)
        g.inspect(ts, partition=1, splits=splits)
    finally:
        del os.environ["DGT_TILE_OP"]
    g.set_schedule(sch)
    gv = torch.from_numpy(I.random_state((2, npk, m.nc), 61)).float().cuda().contiguous()
    gs = torch.from_numpy(I.random_state((3, npk, m.nc), 62)).float().cuda().contiguous()
    g.upload(gv, gs)

    def timed(fn, n):
        fn(3)
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn(n)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / n

    n = a.config3_steps
    ms_whole = timed(lambda q: g.step(q, mode=1, t0=0.0), n)
    whole_rate = 5 * npk * m.nc / ms_whole * 1e3

    def part(blocks, pid, check):
        t0 = time.time()
        P = I.mesh_part(m, I.block_parts(m, *blocks), pid, depth)
        t_part = time.time() - t0
        c = P.cells
        os.environ["DGT_TILE_OP"] = "1"
        try:
            lp = D.Solver(D.Mesh.from_mesh(P.mesh), lam[c], mu[c], rho[c], degree=k, flux=1, time_order=4,
                          precision=1, free_sides=0x8, dt=dt)
            t0 = time.time()
            lp.inspect(ts, partition=1, splits=splits, seed_region=P.region, region_carry=1)
            t_insp = time.time() - t0
        finally:
            del os.environ["DGT_TILE_OP"]
        lp.set_schedule(sch)
        halo = np.nonzero(~P.owned)[0]
        send, recv = g.cell_list(c[halo]), lp.cell_list(halo)
        bv = torch.empty(2, npk, halo.size, dtype=torch.float32, device="cuda")
        bs = torch.empty(3, npk, halo.size, dtype=torch.float32, device="cuda")
        ci = torch.from_numpy(c.astype(np.int64)).cuda()
        g.download(gv, gs)
        lp.upload(gv[:, :, ci].contiguous(), gs[:, :, ci].contiguous())

        def run(q, fill, step, both=False):
            for i in range(q):
                if fill:
                    g.pack(send, bv, bs)
                    lp.unpack(recv, bv, bs)
                if both:
                    g.step(1, mode=1, t0=i * dt)
                if step:
                    lp.step(1, mode=1, t0=i * dt)

        owned = int(P.owned.sum())
        r = {"blocks": f"{blocks[0]}x{blocks[1]}", "part": pid, "owned_cells": owned,
             "core_cells": int(np.sum(P.region == 0)),
             "exec_cells": int(np.sum((P.layer >= 1) & (P.layer <= depth))),
             "nonexec_cells": int(np.sum(P.layer > depth)), "local_cells": int(c.size)}
        if check:  # two steps of both with the halo fill between them
            run(2, True, True, both=True)
            lv, ls = lp.zeros()
            lp.download(lv, ls)
            g.download(gv, gs)
            torch.cuda.synchronize()
            oi = torch.from_numpy(np.nonzero(P.owned)[0].astype(np.int64)).cuda()
            r["owned_vs_whole_mesh_max_rel_after_2_steps"] = max(
                (lv[:, :, oi] - gv[:, :, ci[oi]]).abs().max().item(),
                (ls[:, :, oi] - gs[:, :, ci[oi]]).abs().max().item()) / max(gv.abs().max().item(),
                                                                             gs.abs().max().item())
            sched = lp.schedule()
            r["tiles_core_boundary_per_subchain"] = [sched.regions(b, c.size)[0][:2] for b in range(sched.nsub)]
            r["ms_step_only"] = timed(lambda q: run(q, False, True), n)
            r["ms_halo_fill"] = timed(lambda q: run(q, True, False), n)
            r["halo_bytes_per_step"] = int(halo.size * 5 * npk * 4)
            r["part_build_s"], r["inspect_wall_s"] = t_part, t_insp
        r["ms_per_step"] = timed(lambda q: run(q, True, True), n)
        r["owned_dof_updates_per_s"] = 5 * npk * owned / r["ms_per_step"] * 1e3
        r["rate_vs_whole_mesh"] = r["owned_dof_updates_per_s"] / whole_rate
        return r

    out = {"workload": "jitter1024 P3 FP32 (lognormal, upwind, order 4) split into rectangular blocks; one "
                       "block with 6 exec layers and 1 non-exec layer, halo filled by device-to-device "
                       "pack/unpack from a whole-mesh solver",
           "kernel": "register-resident", "tile_size": ts, "splits": list(splits), "schedule": sch,
           "whole_mesh_ms_per_step": ms_whole, "whole_mesh_dof_updates_per_s": whole_rate}
    out["block_5_of_2x4"] = part((2, 4), 5, True)
    out["by_part_size"] = [part(b, p, False) for b, p in (((1, 1), 0), ((1, 2), 1), ((2, 2), 3), ((2, 4), 5),
                                                          ((4, 4), 9))]
    return out


# the tile kernel and the host code that lays out its data (cell order, footprints)
TILE_SOURCES = ("tile_chain.h", "dg_kernels.h", "tile_args.h", "solver.hip")


def measured_traffic(workload, dtype, ts, splits, schedule):
    """HBM bytes per tile-kernel launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this configuration, scaled by the copy calibration; None
    when there is none or when the kernel's sources changed since it was taken."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in TILE_SOURCES:
        with open(os.path.join(ROOT, "paper_1708_03183_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()[:16]
    want = {"workload": workload, "dtype": dtype, "tile_size": str(ts), "splits": ",".join(map(str, splits)),
            "schedule": str(schedule), "src_sha": sha}
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("traffic: "):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if all(kv.get(key) == val for key, val in want.items()):
                    return float(kv["bytes_per_launch"])
    return None


def cfl_dt(m, lam, mu, rho, k):
    """CFL time step: 0.2 h_min / ((2k+1) c_p,max), h = 4|K| / perimeter."""
    import numpy as np
    p = m.xy[m.c2v]
    e = [np.hypot(*(p[:, (i + 1) % 3] - p[:, i]).T) for i in range(3)]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    hmin = float(np.min(4.0 * area / (e[0] + e[1] + e[2])))
    cmax = float(np.max(np.sqrt((lam + 2 * mu) / rho)))
    return 0.2 * hmin / ((2 * k + 1) * cmax)


BATCH_MESHES = (181, 239, 315, 416, 549, 724)
TUNE_TILE_SIZES = (64, 96, 128, 192, 256, 384, 512)


def batched(a):
    """64 Ricker shots at seeded positions (uniform in [0.1, 0.9]^2), shot i on mesh
    i mod 6 of six jittered renumbered meshes (n = 181 ... 724 squares per side, 65,522
    to 1,048,352 cells), DG P2, FP32, three-layer material, upwind.  Batched form: one
    solver per mesh holding all of its shots, the six advanced on six streams at once.
    Plain form: the same shots one at a time on one-shot solvers.  Every shot of the
    batched run is compared with its plain run: bit-equal when both run the same
    configuration, else (the autotuner may pick different tile sizes, hence tile
    kernels, for the two forms) the relative L2 difference is reported."""
    import numpy as np
    import torch

    from paper_1708_03183_amd import dgtile as D
    from paper_1708_03183_amd import inputs as I

    k, prec = 2, 1
    npk = (k + 1) * (k + 2) // 2
    ts, splits, schedule, *_ = DEFAULTS[(k, "fp32")]
    if a.tile_size:
        ts = a.tile_size
    if a.schedule is not None:
        schedule = a.schedule
    rng = np.random.default_rng(64)
    xy = rng.uniform(0.1, 0.9, size=(a.shots, 2))
    t0 = time.time()
    meshes = []
    for i, n in enumerate(BATCH_MESHES):
        m = I.square_mesh(n, jitter=0.2, jitter_seed=10 + i, renumber_seed=20 + i)
        lam, mu, rho = I.layered_material(m)
        meshes.append((m, lam, mu, rho, cfl_dt(m, lam, mu, rho, k), D.Mesh.from_mesh(m)))
    t_gen = time.time() - t0
    shots_of = [[q for q in range(a.shots) if q % len(meshes) == i] for i in range(len(meshes))]
    streams = [torch.cuda.Stream() for _ in meshes]

    tuned = {"batched": [], "plain": []}

    def make(i, form, stream=None):
        """A solver for mesh i holding its shots (batched) or one shot (plain), tuned by
        the autotuner (tile size and schedule by trial steps) unless --no-autotune."""
        m, lam, mu, rho, dt, gm = meshes[i]
        s = D.Solver(gm, lam, mu, rho, degree=k, flux=1, time_order=4, precision=prec, free_sides=0x8, dt=dt,
                     stream=stream)
        q = shots_of[i]
        if form == "batched":
            s.set_shots(len(q), xy[q])
        else:
            s.set_source(*xy[q[0]])
        if a.no_autotune:
            s.inspect(ts, partition=1, splits=splits)
            s.set_schedule(schedule)
            tuned[form].append({"tile_size": ts, "schedule": schedule})
        else:
            r = s.autotune(TUNE_TILE_SIZES, splits=splits, partition=1, trial_steps=3)
            tuned[form].append({"tile_size": r["tile_size"], "schedule": r["schedule"],
                                "trial_ms_per_step": r["ms_per_step"], "timed": r["timed"]})
        return s

    # batched
    ti = time.time()
    bat = []
    for i in range(len(meshes)):
        if not shots_of[i]:
            continue
        bat.append((i, make(i, "batched", streams[i])))
    torch.cuda.synchronize()
    t_insp = time.time() - ti
    states = {}
    for i, s in bat:
        states[i] = s.zeros()
    torch.cuda.synchronize()  # the zeros come from torch's stream, the solvers run on their own
    for i, s in bat:
        v, st = states[i]
        s.upload(v, st)
        s.step(a.warmup, mode=1, t0=0.0)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for i, s in bat:
        s.step(a.steps, mode=1, t0=a.warmup * meshes[i][4])
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - tb
    for i, s in bat:
        s.download(*states[i])
    torch.cuda.synchronize()
    dofs_step = sum(5 * npk * meshes[i][0].nc * len(shots_of[i]) for i in range(len(meshes)))

    # the same solvers as ONE batch: shared launches for all six meshes (one per colour of a
    # sub-chain, or one per sub-chain under the dependence-driven schedule), launched
    # directly and replayed from a HIP graph of graph_steps steps
    one = None
    try:
        batch = D.Batch([s for _, s in bat])
    except D.DgtError as e:
        one = {"error": str(e)}
    if one is None:
        one = {}
        for mode, sched, g in (("colour_direct", 0, 0), ("colour_graph", 0, a.graph_steps),
                               ("dependence_direct", 1, 0), ("dependence_graph", 1, a.graph_steps)):
            batch.set_schedule(sched)
            batch.set_graph(g)
            for i, s in bat:
                v, st = s.zeros()
                torch.cuda.synchronize()
                s.upload(v, st)
            torch.cuda.synchronize()
            batch.step(a.warmup, [0.0] * len(bat))
            torch.cuda.synchronize()
            tb1 = time.perf_counter()
            batch.step(a.steps, [a.warmup * meshes[i][4] for i, _ in bat])
            torch.cuda.synchronize()
            wall = time.perf_counter() - tb1
            t = batch.timing()
            worst = 0.0
            for i, s in bat:
                v, st = s.zeros()
                torch.cuda.synchronize()
                s.download(v, st)
                torch.cuda.synchronize()
                bv, bs = states[i]
                num = ((v.double() - bv.double()) ** 2).sum() + ((st.double() - bs.double()) ** 2).sum()
                den = (bv.double() ** 2).sum() + (bs.double() ** 2).sum()
                worst = max(worst, math.sqrt(num.item() / den.item()) if den.item() > 0 else 0.0)
            one[mode] = {"value": dofs_step * a.steps / wall, "ms_per_step": 1e3 * wall / a.steps,
                         "event_ms_per_step": t["ms"] / a.steps, "launches_per_step": t["launches"] / a.steps,
                         "graph_replays": t["graph_launches"], "steps_per_graph": g,
                         "rel_l2_vs_six_streams": worst}
            print(f"bench: one batch for all meshes ({mode}): {1e3 * wall / a.steps:.3f} ms/step, "
                  f"{t['launches'] / a.steps:.0f} launches/step", file=sys.stderr, flush=True)
        del batch

    # plain: one shot at a time
    wall_p = 0.0
    equal = True
    diff = 0.0
    for i, _ in bat:
        s = make(i, "plain")
        for j, q in enumerate(shots_of[i]):
            s.set_source(*xy[q])
            v, st = s.zeros()
            s.upload(v, st)
            s.step(a.warmup, mode=1, t0=0.0)
            torch.cuda.synchronize()
            tp = time.perf_counter()
            s.step(a.steps, mode=1, t0=a.warmup * meshes[i][4])
            torch.cuda.synchronize()
            wall_p += time.perf_counter() - tp
            s.download(v, st)
            torch.cuda.synchronize()
            bv, bs = states[i][0][j], states[i][1][j]
            equal &= bool(torch.equal(v, bv) and torch.equal(st, bs))
            num = ((v.double() - bv.double()) ** 2).sum() + ((st.double() - bs.double()) ** 2).sum()
            den = (bv.double() ** 2).sum() + (bs.double() ** 2).sum()
            diff = max(diff, math.sqrt(num.item() / den.item()) if den.item() > 0 else 0.0)
        del s

    # the FP32 batched state of shot 0 (mesh 0), two more steps against the FP64 oracle
    err = None
    if not a.no_cpu_baseline:
        import oracle as O
        m, lam, mu, rho, dt, gm = meshes[0]
        om = O.OMesh.from_mesh(m)
        od = O.ODG(om, k, lam, mu, rho, flux=1, order=4, dt=dt, free_sides=0x8)
        od.set_source(*xy[0], 5.0, 0.2, 1.0)
        v = states[0][0][0].double().cpu().numpy().copy()
        s_ = states[0][1][0].double().cpu().numpy().copy()
        tstart = (a.warmup + a.steps) * dt
        od.step(v, s_, 2, t0=tstart)
        i0, sb = bat[0]
        sb.upload(*states[i0])
        sb.step(2, mode=1, t0=tstart)
        sb.download(*states[i0])
        torch.cuda.synchronize()
        gv = states[i0][0][0].double().cpu().numpy()
        gs = states[i0][1][0].double().cpu().numpy()
        num = math.sqrt(((gv - v) ** 2).sum() + ((gs - s_) ** 2).sum())
        den = math.sqrt((v ** 2).sum() + (s_ ** 2).sum())
        err = num / den if den > 0 else 0.0

    rate_b = dofs_step * a.steps / wall_b
    rate_p = dofs_step * a.steps / wall_p
    out = {
        "metric": "DG dof-updates/s, batched forward shots on uneven meshes, 1 MI355X",
        "value": rate_b,
        "unit": "dof-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall_b / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched: {a.shots} Ricker shots on {len(meshes)} jittered renumbered meshes "
                               f"(n = {', '.join(map(str, BATCH_MESHES))}), DG P2, 3-layer, upwind, order-4 leapfrog",
                   "cells": [mm[0].nc for mm in meshes], "shots_per_mesh": [len(x) for x in shots_of],
                   "dofs_per_step": dofs_step, "splits": list(splits),
                   "tuning": "fixed" if a.no_autotune else "autotuner"},
        "tuned": tuned,
        "one_launch": one,
        "plain": {"value": rate_p, "ms_per_step": 1e3 * wall_p / a.steps,
                  "form": "the same shots one at a time, one-shot solvers"},
        "speedup_batched_vs_plain": rate_b / rate_p,
        "batched_equals_plain_bitwise": equal,
        "max_rel_l2_diff_batched_vs_plain": diff,
        "err_fp32_run_vs_fp64_oracle_rel_l2": err,
        "inspect_and_tune_wall_s": t_insp,
        "mesh_gen_s": t_gen,
    }
    return out


def fwi(a):
    """Full-waveform-inversion gradient: 256x256 jittered renumbered mesh (131,072
    cells), DG P2, 16 Ricker shots at seeded positions just below the top edge, 128
    velocity receivers along the top edge, observed data from the 3-layer true model, gradient at a
    homogeneous starting model (the true model's means), upwind flux with a free top and
    absorbing other sides (the closed-form transposed step; --fwi-boundaries free: the
    central flux with free surfaces everywhere, whose transposed step is the reversed
    chain), order-4 leapfrog, FP32 state, FP64 gradient, 32 checkpoints, tiled forward
    executor (tile size and schedule by the autotuner).  Reports the wall time of one gradient, of one
    forward run of the same shots, and the FP32 gradient's difference from an FP64
    gradient of the first shot alone."""
    import numpy as np
    import torch

    from paper_1708_03183_amd import dgtile as D
    from paper_1708_03183_amd import inputs as I

    k, n, nshots, nrec = 2, 256, 16, 128
    m = I.square_mesh(n, jitter=0.2, jitter_seed=30, renumber_seed=31)
    lam_t, mu_t, rho_t = I.layered_material(m)
    lam0, mu0, rho0 = [np.full(m.nc, float(x.mean())) for x in (lam_t, mu_t, rho_t)]
    dt = min(cfl_dt(m, lam_t, mu_t, rho_t, k), cfl_dt(m, lam0, mu0, rho0, k))
    # a surface survey sized to the window: 2000 steps span 2000 dt = 0.03 time units, in
    # which P waves (c_p = 2) travel 0.06, so the sources sit just below the receivers
    # and the Ricker wavelet (f0 = 100, t0 = 0.012) fits three periods into the window
    rng = np.random.default_rng(16)
    shots = np.stack([rng.uniform(0.1, 0.9, nshots), rng.uniform(0.96, 0.99, nshots)], axis=1)
    recs = np.stack([(np.arange(nrec) + 0.5) / nrec, np.ones(nrec)], axis=1)
    f0, t0 = 100.0, 0.012
    gm = D.Mesh.from_mesh(m)
    npk = (k + 1) * (k + 2) // 2

    absorbing = a.fwi_boundaries == "absorbing"
    flux, free = (1, 0x8) if absorbing else (0, 0xF)

    def make(lam, mu, rho, prec, ns=nshots, tune=True):
        s = D.Solver(gm, lam, mu, rho, degree=k, flux=flux, time_order=4, precision=prec, free_sides=free, dt=dt)
        s.set_shots(ns, shots[:ns], f0, t0, 1.0)
        if tune:
            r = s.autotune((64, 128, 256, 512), splits=(13,), partition=1, trial_steps=3)
        else:
            s.inspect(128, partition=1, splits=(13,))
            r = None
        return s, r

    nsteps, nsnap = a.fwi_steps, a.fwi_snapshots
    true, _ = make(lam_t, mu_t, rho_t, 1, tune=False)
    obs = true.fwi_forward(recs, nsteps, mode=1)
    torch.cuda.synchronize()
    del true
    ti = time.time()
    sol, tuned = make(lam0, mu0, rho0, 1)
    torch.cuda.synchronize()
    t_tune = time.time() - ti
    t = time.perf_counter()
    sol.fwi_forward(recs, nsteps, mode=1)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    t = time.perf_counter()
    J, gl, gm_, gr = sol.fwi_gradient(recs, nsteps, obs, nsnap=nsnap, mode=1)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t
    gnorm = float(torch.sqrt((gl ** 2).sum() + (gm_ ** 2).sum() + (gr ** 2).sum()))

    # FP32 against FP64 on one shot over all steps (the waves reach the receivers late)
    ws, wq = nsteps, 1
    err = None
    if not a.no_cpu_baseline:
        g32, g64 = [], []
        for prec, out in ((1, g32), (0, g64)):
            s_, _ = make(lam0, mu0, rho0, prec, wq, tune=False)
            o = obs[:wq].contiguous()
            _, *g = s_.fwi_gradient(recs, ws, o, nsnap=8, mode=1)
            out.append(torch.stack(g))
            del s_
        err = float((g32[0] - g64[0]).norm() / g64[0].norm())

    out = {
        "metric": "FWI gradient time, 1 MI355X",
        "value": t_grad,
        "unit": "s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": 0,
        "ms_per_step": 1e3 * t_grad / nsteps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state, f64 gradient",
        "data": "synthetic",
        "config": {"workload": f"fwi256_p2: {n}x{n} jittered renumbered triangulation, {m.nc} cells, DG P2, "
                               f"{nshots} shots at y in [0.96, 0.99] (Ricker f0 = {f0}, t0 = {t0}), {nrec} receivers at y = 1, "
                               f"3-layer true model, homogeneous start, "
                               + ("upwind flux, free top, absorbing other sides" if absorbing
                                  else "central flux, free surfaces")
                               + ", order-4 leapfrog",
                   "cells": m.nc, "shots": nshots, "receivers": nrec, "snapshots": nsnap,
                   "dofs_per_step_all_shots": 5 * npk * m.nc * nshots, "tuned": tuned},
        "forward_s": t_fwd,
        "gradient_over_forward": t_grad / t_fwd,
        "misfit": J,
        "gradient_norm": gnorm,
        "err_fp32_vs_fp64_gradient_rel_l2": err,
        "err_window": f"{ws} steps, shot 0 alone",
        "tune_s": t_tune,
    }
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not part of this build",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.workload == "batched":
        print(json.dumps(batched(a)))
        return
    if a.workload == "fwi":
        print(json.dumps(fwi(a)))
        return
    import numpy as np
    import torch

    from paper_1708_03183_amd import dgtile as D
    from paper_1708_03183_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prec = 1 if a.precision == "fp32" else 0
    ts, splits, schedule, *rest = DEFAULTS.get((a.degree, a.precision), (64, OPS, 0))
    default_sub_ts = rest[0] if rest and not (a.tile_size or a.splits) else None
    if a.schedule is not None:
        schedule = a.schedule
    if a.tile_size:
        ts = a.tile_size
    if a.splits is not None:
        splits = () if a.splits in ("", "none") else tuple(int(x) for x in a.splits.split(","))

    t0 = time.time()
    m = I.square_mesh(a.n, jitter=0.2, jitter_seed=1, renumber_seed=2 if a.mesh_order == "renumbered" else None)
    k = a.degree
    (lam, mu, rho), mat_name = material(m, k, a.material)
    t_gen = time.time() - t0
    npk = (k + 1) * (k + 2) // 2
    dt = cfl_dt(m, lam, mu, rho, k)

    mesh = D.Mesh.from_mesh(m)
    dofs = 5 * npk * mesh.nc

    def make(pr):
        s = D.Solver(mesh, lam, mu, rho, degree=k, flux=1, time_order=4, precision=pr, free_sides=0x8, dt=dt)
        s.set_source(0.5, 0.5, 5.0, 0.2, 1.0)
        return s

    if a.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # ---- tiled fused executor
    sol = make(prec)
    torch.cuda.synchronize()
    ti0 = time.time()
    sub_ts = tuple(int(x) for x in a.sub_tile_sizes.split(",")) if a.sub_tile_sizes else default_sub_ts
    sol.inspect(ts, partition=a.partition, splits=splits, max_colour_tiles=a.colour_cap, sub_tile_sizes=sub_ts)
    sol.set_schedule(schedule)
    torch.cuda.synchronize()
    t_insp_wall = time.time() - ti0
    sch_obj = sol.schedule()
    sched = json.loads(sch_obj.summary())
    insp_bytes = 4 * sum(sch_obj.loop_sizes) + 4 * (2 * mesh.nf + mesh.nb)
    del sch_obj
    info = sol.info()

    def run(solver, mode, steps, warm):
        v, s = solver.zeros()
        solver.upload(v, s)
        if warm:
            solver.step(warm, mode=mode, t0=0.0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        solver.step(steps, mode=mode, t0=warm * dt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        tot_ms, ker_ms, launches = solver.last_timing()
        solver.download(v, s)
        torch.cuda.synchronize()
        return wall, tot_ms, ker_ms, launches, v, s

    def progress(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    progress(f"inspected ({t_insp_wall:.2f} s); timing {a.steps} tiled steps")
    wall_t, ev_t, _, launches_t, vt, st_ = run(sol, 1, a.steps, a.warmup)
    progress(f"tiled: {1e3 * wall_t / a.steps:.4f} ms/step; repeats and per-launch timing")
    rate_t = dofs * a.steps / wall_t
    # five more timed repeats of a shorter window, for the spread
    rsteps = min(a.steps, 200)
    reps = sorted(1e3 * run(sol, 1, rsteps, a.warmup)[0] / rsteps for _ in range(5))
    # the same run again with an event pair around every tile-kernel launch
    sol.profile(True)
    psteps = min(a.steps, 200)
    _, _, ker_p, launches_p, _, _ = run(sol, 1, psteps, a.warmup)
    sol.profile(False)

    res = {}
    if not a.no_untiled:
        progress("untiled chain")
        wall_u, _, _, launches_u, vu, su = run(sol, 0, a.steps, a.warmup)
        rate_u = dofs * a.steps / wall_u
        num = torch.sqrt(((vt - vu) ** 2).sum() + ((st_ - su) ** 2).sum()).item()
        den = torch.sqrt((vu ** 2).sum() + (su ** 2).sum()).item()
        res["untiled"] = {"value": rate_u, "ms_per_step": 1e3 * wall_u / a.steps,
                          "launches_per_step": launches_u / a.steps, "cell_order": "hilbert (same as tiled)"}
        res["speedup_tiled_vs_untiled"] = rate_t / rate_u
        res["err_tiled_vs_untiled_rel_l2"] = num / den if den > 0 else 0.0
        # the untiled chain on the mesh's own (randomly renumbered) cell order
        raw = make(prec)
        usteps = min(a.steps, 200)
        wall_r, _, _, _, _, _ = run(raw, 0, usteps, a.warmup)
        res["untiled_mesh_order"] = {"value": dofs * usteps / wall_r, "ms_per_step": 1e3 * wall_r / usteps,
                                     "steps": usteps, "cell_order": "mesh numbering (random renumbering)"}
        del raw

    # roofline of the tile kernel: algorithmic bytes (state read and written once, cell
    # invariants read once per step) per launch over the launch's average duration.  The
    # timed tiled region holds nothing but tile-kernel launches, back to back on the
    # solver stream, so its HIP-event time over its launch count is that average (gaps
    # included); the per-launch event pairs of the second run bound it from above.
    bytes_step = info["bytes_per_step"]
    launches_per_step = launches_t / a.steps
    bytes_launch = bytes_step / launches_per_step
    avg_launch_s = (ev_t / 1e3) / launches_t
    achieved = bytes_launch / avg_launch_s / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": (measured_traffic(f"jitter{a.n}_p{k}", "f32" if prec else "f64", ts, splits, schedule)
                            if a.partition == 1 and a.mesh_order == "renumbered" and not sub_ts else None),
                "kernel": "k_tile_chain",
                "bytes_per_launch": bytes_launch, "avg_launch_us": avg_launch_s * 1e6,
                "avg_launch_us_event_pairs": ker_p / launches_p * 1e3}

    # ---- oracle on the host: a bounded sample of the same workload
    cpu = None
    insp_cpu = None
    err_oracle = None
    err_fp32 = None
    if not a.no_cpu_baseline:
        import oracle as O
        tstart = (a.warmup + a.steps) * dt  # the GPU's state after the timed run
        v0 = vt.double().cpu().numpy()
        s0 = st_.double().cpu().numpy()
        # the whole mesh when a.cpu_steps steps take at most ~30 s on one host core (the
        # oracle runs ~1.4e6 dof-updates/s), else the cells within some facet layers of the
        # centre cell; a cell's state after s steps depends only on cells within 6 s facet
        # layers (one facet loop per operator application), so the cells deeper than that
        # inside the patch are compared
        budget = 4e7
        cells, core, sub, where = oracle_patch(m, npk, a.cpu_steps, budget, (0.5, 0.5))
        print(f"cpu baseline: oracle on {where}, {a.cpu_steps} step(s)", file=sys.stderr, flush=True)
        om = O.OMesh(sub.xy, sub.c2v, sub.periodic)
        od = O.ODG(om, k, lam[cells], mu[cells], rho[cells], flux=1, order=4, dt=dt, free_sides=0x8)
        try:
            od.set_source(0.5, 0.5, 5.0, 0.2, 1.0)
        except ValueError:
            pass  # (the patch is centred on the source; kept for generality)
        v = np.ascontiguousarray(v0[:, :, cells])
        s = np.ascontiguousarray(s0[:, :, cells])
        tc = time.perf_counter()
        od.step(v, s, a.cpu_steps, t0=tstart)
        tcpu = time.perf_counter() - tc
        cpu = {"value": 5 * npk * len(cells) * a.cpu_steps / tcpu, "unit": "dof-updates/s", "cores": 1,
               "kind": "oracle", "cpu_model": host_cpu_model(),
               "sample": f"{a.cpu_steps} step(s) of {where}, from the GPU's final state "
                         f"({tcpu:.1f} s, FP64, single thread)"}
        # the oracle's inspection of the same chain (tile size, partition, splits) on the
        # mesh of half the side from the same generator: a sample of ~10 s on one core
        hn = max(a.n // 2, 8)
        progress(f"oracle inspector on the {hn}x{hn} mesh")
        mi = I.square_mesh(hn, jitter=0.2, jitter_seed=1, renumber_seed=2 if a.mesh_order == "renumbered" else None)
        (li, ui, ri), _ = material(mi, k, a.material)
        odi = O.ODG(O.OMesh.from_mesh(mi), k, li, ui, ri, flux=1, order=4, dt=dt, free_sides=0x8)
        chi = odi.chain(1)
        tc = time.perf_counter()
        chi.inspect(ts, partition=a.partition, seed_xy=mi.centroids() if a.partition else None, splits=splits,
                    max_colour_tiles=a.colour_cap, sub_tile_sizes=sub_ts)
        ti_cpu = time.perf_counter() - tc
        insp_cpu = {"s": ti_cpu, "cells": int(mi.c2v.shape[0]), "cells_per_s": mi.c2v.shape[0] / ti_cpu,
                    "cores": 1, "kind": "oracle",
                    "sample": f"the same chain, tile size and splits on the {hn}x{hn} mesh of the same "
                              f"generator ({mi.c2v.shape[0]} cells), single thread"}
        del chi, odi
        if a.cpu_cores != 1:
            ncores = a.cpu_cores or min(16, os.cpu_count() or 1)
            progress(f"cpu baseline on {ncores} cores")
            rate_mc, span, work = oracle_multicore(a.n, k, mat_name, a.cpu_steps, budget / 2, ncores)
            cpu["all_cores"] = {"value": rate_mc, "unit": "dof-updates/s", "cores": ncores, "kind": "oracle",
                                "sample": f"{ncores} concurrent processes, each the single-threaded oracle on a "
                                          f"patch of its own of the same mesh ({work:.3g} dof-updates in "
                                          f"{span:.1f} s)"}
        pos = np.searchsorted(cells, core)
        vr, sr = v[:, :, pos], s[:, :, pos]
        den = math.sqrt((vr ** 2).sum() + (sr ** 2).sum())
        # GPU FP64 tiled from the same state, compared with the oracle
        chk = make(0)
        chk.inspect(ts, partition=a.partition, splits=splits, max_colour_tiles=a.colour_cap, sub_tile_sizes=sub_ts)
        chk.set_schedule(schedule)
        gv = torch.from_numpy(np.ascontiguousarray(v0)).cuda()
        gs = torch.from_numpy(np.ascontiguousarray(s0)).cuda()
        chk.upload(gv, gs)
        chk.step(a.cpu_steps, mode=1, t0=tstart)
        chk.download(gv, gs)
        torch.cuda.synchronize()
        num = math.sqrt(((gv.cpu().numpy()[:, :, core] - vr) ** 2).sum() + ((gs.cpu().numpy()[:, :, core] - sr) ** 2).sum())
        err_oracle = num / den if den > 0 else 0.0
        if prec:  # the FP32 path itself over the same window, against the FP64 oracle
            fv = vt.clone()
            fs_ = st_.clone()
            sol.upload(fv, fs_)
            sol.step(a.cpu_steps, mode=1, t0=tstart)
            sol.download(fv, fs_)
            torch.cuda.synchronize()
            num = math.sqrt(((fv.double().cpu().numpy()[:, :, core] - vr) ** 2).sum() +
                            ((fs_.double().cpu().numpy()[:, :, core] - sr) ** 2).sum())
            err_fp32 = num / den if den > 0 else 0.0

    out = {
        "metric": "DG dof-updates/s per step, tiled-fused vs untiled, 1 MI355X",
        "value": rate_t,
        "unit": "dof-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall_t / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec else "f64",
        "data": "synthetic",
        "config": {"workload": f"jitter{a.n}_p{k}: {a.n}x{a.n} jittered "
                               f"{'renumbered' if a.mesh_order == 'renumbered' else 'row-major'} triangulation, "
                               f"{mesh.nc} cells, DG P{k}, "
                               f"{'3-layer' if mat_name == 'layered' else 'lognormal (sigma 0.3)'} material, "
                               f"upwind, order-4 leapfrog",
                   "material": mat_name,
                   "cells": mesh.nc, "dofs_per_step": dofs, "tile_size": ts, "splits": list(splits),
                   "sub_tile_sizes": list(sub_ts) if sub_ts else None,
                   "partition": "hilbert" if a.partition == 1 else "chunks of the mesh numbering",
                   "mesh_order": a.mesh_order, "colour_cap": a.colour_cap,
                   "schedule": "dependence-driven" if schedule == 1 else "colour launches"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "err_vs_fp64_oracle_rel_l2": err_oracle,
        "err_fp32_run_vs_fp64_oracle_rel_l2": err_fp32,
        "repeats_ms_per_step": {"steps": rsteps, "median": reps[2], "min": reps[0], "max": reps[-1]},
        "inspector": {"gpu_ms": sched.get("inspector_gpu_ms"), "wall_s": t_insp_wall,
                      "cells_per_s_wall": mesh.nc / t_insp_wall,
                      # the maps read once and every loop's tile assignment written once
                      "bytes_maps_and_sigma": insp_bytes,
                      "effective_gbs": (insp_bytes / (sched["inspector_gpu_ms"] * 1e-3) / 1e9
                                        if sched.get("inspector_gpu_ms") else None),
                      "oracle_on_host": insp_cpu,
                      "subchains": sched.get("subchains"), "lds_bytes": info["lds_bytes"]},
        "launches_per_step": launches_t / a.steps,
        "mesh_gen_s": t_gen,
    }
    out.update(res)
    if not a.no_horizon:
        progress(f"FP32 against GPU FP64 over {a.warmup + a.steps} steps")
        out["precision_horizon"] = horizon(D, make, a.warmup + a.steps, k, (vt, st_), prec, dt)
    if not a.no_config3 and a.n == 512 and k == 2:
        progress("config 3 extras (1024x1024 P3/P4 FP32)")
        out["config3"] = config3(a)
    if not a.no_sweep and a.n == 512 and k == 2:
        progress("tile sizes 256-4096 (working sets beyond the LDS in global memory)")
        sweep = []
        for ts_ in (256, 512, 1024, 2048, 4096):
            s_ = make(prec)
            s_.inspect(ts_, partition=1, splits=splits)
            kinds = s_.kernels()
            s_.set_schedule(1 if all(x in (1, 2) for x in kinds) else 0)
            w_, tot_, _, _, _, _ = run(s_, 1, a.sweep_steps, 2)
            sweep.append({"tile_size": ts_, "kernels": kinds, "ms_per_step": 1e3 * w_ / a.sweep_steps,
                          "value": dofs / (w_ / a.sweep_steps)})
            del s_
        out["tile_size_sweep"] = sweep
    if not a.no_part and a.n == 512 and k == 2:
        progress("one GPU's share of the 1024x1024 P3 workload (regions, halo pack/unpack)")
        out["part_block"] = part_block(a)
    if "untiled" in res:
        gain = (res["untiled"]["ms_per_step"] - out["ms_per_step"]) / 1e3
        out["inspector"]["steps_to_amortise"] = (t_insp_wall / gain) if gain > 0 else None
    if not a.no_config4 and a.n == 512 and k == 2:
        # the batched workload's record, shortened to config4_steps timed steps
        progress(f"config 4 extras (batched shots on six meshes, {a.config4_steps} steps)")
        a4 = argparse.Namespace(**vars(a))
        a4.steps, a4.warmup = a.config4_steps, 5
        r4 = batched(a4)
        out["config4"] = {key: r4[key] for key in ("metric", "value", "unit", "ms_per_step", "steps", "dtype",
                                                    "config", "one_launch", "plain", "speedup_batched_vs_plain",
                                                    "batched_equals_plain_bitwise", "max_rel_l2_diff_batched_vs_plain",
                                                    "err_fp32_run_vs_fp64_oracle_rel_l2")}
    if not a.no_config5 and a.n == 512 and k == 2:
        progress(f"config 5 extras (FWI gradient, {a.fwi_steps} steps)")
        r5 = fwi(a)
        out["config5"] = {key: r5[key] for key in ("metric", "value", "unit", "steps", "ms_per_step", "dtype",
                                                    "config", "forward_s", "gradient_over_forward", "misfit",
                                                    "gradient_norm", "err_fp32_vs_fp64_gradient_rel_l2", "err_window")}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
