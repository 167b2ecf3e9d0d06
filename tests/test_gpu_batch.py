"""GPU: several meshes in one launch per sub-chain (dgt_batch), directly and from
HIP graph replays.

Every (tile, shot) item of a batched launch runs the arithmetic of its member's
own tiled step, so each member's state equals the member stepped alone with the
dependence-driven schedule to rounding (the batched kernel is compiled on its own
and the compiler may contract multiply-adds differently; in most configurations
the two agree bit for bit); graph replays equal direct launches of the same kernel
bit for bit, call after call, with the program's own work and synchronisations
between the replays; one member is also checked against the FP64 oracle.
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


MEMBERS = [  # n, renumber seed, seed tile size, shots, source
    (10, 3, 16, 1, (0.43, 0.52)),
    (14, 5, 24, 2, (0.61, 0.37)),
    (7, 9, 12, 1, (0.25, 0.70)),
]


def _members(D, k, prec, order=4, splits=(13,), flux=1):
    out = []
    for q, (n, ren, ts, shots, src) in enumerate(MEMBERS):
        m = I.square_mesh(n, jitter=0.2, renumber_seed=ren)
        lam, mu, rho = I.layered_material(m)
        om = O.OMesh.from_mesh(m)
        dt = O.cfl_dt(om, k, lam, mu, rho)
        g = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=k, flux=flux, time_order=order, precision=prec,
                     free_sides=0x8, dt=dt)
        if shots > 1:
            g.set_shots(shots, np.array([src, (0.3, 0.3)]))
        else:
            g.set_source(*src)
        g.inspect(ts, partition=1, splits=splits)
        g.set_schedule(1)
        dtype = torch.float32 if prec else torch.float64
        v, s = g.zeros()
        v.copy_(torch.from_numpy(I.random_state(tuple(v.shape), 60 + 2 * q)).to(dtype))
        s.copy_(torch.from_numpy(I.random_state(tuple(s.shape), 61 + 2 * q)).to(dtype))
        out.append(dict(g=g, v0=v.clone(), s0=s.clone(), mesh=m, om=om, mat=(lam, mu, rho), dt=dt, src=src))
    return out


def _same(a, b, prec):
    """rounding-level agreement of two states: max-abs difference within a few units
    in the last place of the largest value"""
    scale = max(b[0].abs().max().item(), b[1].abs().max().item())
    d = max((a[0] - b[0]).abs().max().item(), (a[1] - b[1]).abs().max().item())
    return d <= (8 * 2.0 ** -23 if prec else 8 * 2.0 ** -52) * scale, d


def _alone(mem, steps, t0):
    res = []
    for x in mem:
        v, s = x["v0"].clone(), x["s0"].clone()
        x["g"].upload(v, s)
        x["g"].step(steps, mode=1, t0=t0)
        x["g"].download(v, s)
        res.append((v, s))
    torch.cuda.synchronize()
    return res


def _batched(D, mem, steps, t0, graph=0, calls=1, schedule=0):
    for x in mem:
        x["g"].upload(x["v0"].clone(), x["s0"].clone())
    b = D.Batch([x["g"] for x in mem])
    b.set_schedule(schedule)
    b.set_graph(graph)
    outs = []
    for c in range(calls):
        b.step(steps, [t0 + c * steps * x["dt"] for x in mem])
        t = b.timing()
        res = []
        for x in mem:
            v, s = x["g"].zeros()
            x["g"].download(v, s)
            res.append((v, s))
        torch.cuda.synchronize()
        outs.append((res, t))
    return outs


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("k,prec,order,splits", [(2, 0, 4, (13,)), (2, 1, 4, (13,)), (1, 0, 2, ())])
def test_batch_equals_members_alone(D, k, prec, order, splits, schedule):
    mem = _members(D, k, prec, order, splits)
    ref = _alone(mem, 5, 0.1)
    (res, t), = _batched(D, mem, 5, 0.1, schedule=schedule)
    nsub = len(splits) + 1
    ncol = [max(x["g"].schedule().sub_info(b)["ncolors"] for x in mem) for b in range(nsub)]
    assert t["launches"] == 5 * (nsub if schedule else sum(ncol)) and t["graph_launches"] == 0
    worst = 0.0
    for q, ((v, s), (rv, rs)) in enumerate(zip(res, ref)):
        ok, d = _same((v, s), (rv, rs), prec)
        worst = max(worst, d)
        assert ok, f"member {q} differs from its own run by {d:.3e}"
    # one member against the oracle
    x = mem[0]
    od = O.ODG(x["om"], k, *x["mat"], flux=1, order=order, dt=x["dt"], free_sides=0x8)
    od.set_source(*x["src"])
    v, s = x["v0"].double().cpu().numpy(), x["s0"].double().cpu().numpy()
    od.step(v, s, 5, t0=0.1)
    gv, gs = res[0][0].double().cpu().numpy(), res[0][1].double().cpu().numpy()
    err = np.sqrt(((gv - v) ** 2).sum() + ((gs - s) ** 2).sum()) / np.sqrt((v ** 2).sum() + (s ** 2).sum())
    mx = max(np.abs(gv - v).max(), np.abs(gs - s).max()) / max(np.abs(v).max(), np.abs(s).max())
    print(f"batch k={k} prec={prec} order={order} schedule={schedule}: {len(mem)} members, max-abs difference "
          f"from their own runs "
          f"{worst:.3e}; "
          f"member 0 vs oracle rel L2 {err:.3e}, rel max-abs {mx:.3e}")
    tol = 1e-5 if prec else 1e-12
    assert err <= tol and mx <= tol


@pytest.mark.parametrize("prec,schedule", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_batch_graph_replays_equal_direct_launches(D, prec, schedule):
    """Three calls of 7 steps with 3-step graphs (two replays and one direct step
    per call), each compared with three calls of direct launches."""
    mem = _members(D, 2, prec)
    direct = _batched(D, mem, 7, 0.1, graph=0, calls=3, schedule=schedule)
    graphed = _batched(D, mem, 7, 0.1, graph=3, calls=3, schedule=schedule)
    for c, ((rd, td), (rg, tg)) in enumerate(zip(direct, graphed)):
        assert tg["graph_launches"] == 2 and tg["launches"] == td["launches"]
        for q, ((v, s), (rv, rs)) in enumerate(zip(rg, rd)):
            assert torch.equal(v, rv) and torch.equal(s, rs), f"call {c}, member {q}: graph differs"
        print(f"schedule {schedule} graph call {c}: {tg['ms']:.3f} ms vs direct {td['ms']:.3f} ms "
              f"({td['launches']} launches), bit-equal")
    ref = _alone(mem, 21, 0.1)  # the three calls together equal 21 steps of each member alone
    for q, ((v, s), (rv, rs)) in enumerate(zip(graphed[-1][0], ref)):
        ok, d = _same((v, s), (rv, rs), prec)
        assert ok, f"member {q} differs from 21 steps alone by {d:.3e}"


def test_batch_rejects_bad_members(D):
    mem = _members(D, 2, 0)
    m = I.square_mesh(6, jitter=0.2, renumber_seed=2)
    lam, mu, rho = I.layered_material(m)
    g1 = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=1, flux=1, time_order=4, precision=0, free_sides=0x8,
                  dt=1e-3)
    g1.inspect(8, partition=1, splits=(13,))
    with pytest.raises(D.DgtError) as e:
        D.Batch([mem[0]["g"], g1])  # different degree
    assert e.value.status == D.DGT_EINVAL
    g2 = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=2, flux=1, time_order=4, precision=0, free_sides=0x8,
                  dt=1e-3)
    with pytest.raises(D.DgtError) as e:
        D.Batch([mem[0]["g"], g2])  # not inspected
    assert e.value.status == D.DGT_ESTATE
    with pytest.raises(D.DgtError):
        D.Batch([mem[0]["g"], mem[0]["g"]])  # twice
    for x in mem:
        x["g"].upload(x["v0"].clone(), x["s0"].clone())
    b = D.Batch([x["g"] for x in mem])
    mem[1]["g"].inspect(20, partition=1, splits=(13,))  # a member changes under the batch
    with pytest.raises(D.DgtError) as e:
        b.step(1, 0.0)
    assert e.value.status == D.DGT_ESTATE
