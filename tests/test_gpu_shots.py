"""GPU: batched shots (several independent states on one mesh in the same launches).

Each shot of a batched run equals, bit for bit, a separate single-shot run with the
same source and initial state (the kernels run the same arithmetic on a shot's own
copy of the fields), for the untiled chain, both tile kernels and both schedules;
one shot per case is also checked against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle as O
from paper_1708_03183_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SRC = [(0.43, 0.52), (0.21, 0.74), (0.78, 0.33)]


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_03183_amd import dgtile
    dgtile.lib()
    return dgtile


def _setup(D, n, k, order, prec, ren=7):
    m = I.square_mesh(n, jitter=0.2, renumber_seed=ren)
    lam, mu, rho = I.layered_material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    gm = D.Mesh.from_mesh(m)

    def solver():
        return D.Solver(gm, lam, mu, rho, degree=k, flux=1, time_order=order, precision=prec, free_sides=0x8, dt=dt)

    def oracle():
        return O.ODG(om, k, lam, mu, rho, flux=1, order=order, dt=dt, free_sides=0x8)

    return solver, oracle


def _states(od, k, nshots):
    """Random nodal states, one pair of seeds per shot."""
    out = []
    for q in range(nshots):
        v, s = od.zeros()
        v[:] = I.random_state(v.shape, 100 + 2 * q)
        s[:] = I.random_state(s.shape, 101 + 2 * q)
        out.append((v, s))
    return out


def _prepare(gd, mode, ts, splits, schedule):
    if mode == 1:
        gd.inspect(ts, partition=1, splits=splits)
        gd.set_schedule(schedule)


BATCH_CASES = [
    # k, prec, order, mode, schedule, kernel, ts, splits, steps
    (2, 0, 4, 0, 0, "chain", 0, (), 6),
    (2, 0, 4, 1, 0, "generic", 16, (), 6),
    (2, 0, 4, 1, 0, "chain", 16, (13,), 6),
    (2, 0, 4, 1, 1, "chain", 16, (13,), 6),
    (1, 0, 2, 1, 1, "chain", 12, (), 10),
    (2, 1, 4, 1, 1, "chain", 16, (13,), 6),
    (3, 1, 4, 1, 0, "chain", 16, (4, 8, 12, 13, 17, 21, 25), 8),
    (3, 0, 4, 1, 1, "chain", 16, (4, 8, 12, 13, 17, 21, 25), 8),
]


@pytest.mark.parametrize("k,prec,order,mode,schedule,kernel,ts,splits,steps", BATCH_CASES)
def test_shots_equal_single_shot_runs_and_oracle(D, monkeypatch, k, prec, order, mode, schedule, kernel, ts, splits,
                                                 steps):
    if kernel == "generic":
        monkeypatch.setenv("DGT_TILE_OP", "0")
    solver, oracle = _setup(D, 12, k, order, prec)
    od = oracle()
    states = _states(od, k, len(SRC))
    dtype = torch.float32 if prec else torch.float64
    S = len(SRC)

    gb = solver()
    _prepare(gb, mode, ts, splits, schedule)
    gb.set_shots(S, np.array(SRC))
    bv, bs = gb.zeros()
    assert tuple(bv.shape) == (S, 2, gb.np, gb.mesh.nc)
    for q, (v, s) in enumerate(states):
        bv[q] = torch.from_numpy(v).to(dtype)
        bs[q] = torch.from_numpy(s).to(dtype)
    gb.upload(bv, bs)
    gb.step(steps, mode=mode, t0=0.1)
    gb.download(bv, bs)
    torch.cuda.synchronize()

    for q, (v, s) in enumerate(states):
        g1 = solver()
        _prepare(g1, mode, ts, splits, schedule)
        g1.set_source(*SRC[q])
        sv = torch.from_numpy(v).to(dtype).cuda().contiguous()
        ss = torch.from_numpy(s).to(dtype).cuda().contiguous()
        g1.upload(sv, ss)
        g1.step(steps, mode=mode, t0=0.1)
        g1.download(sv, ss)
        torch.cuda.synchronize()
        assert torch.equal(sv, bv[q]) and torch.equal(ss, bs[q]), f"shot {q} differs from its single-shot run"

    q = 1  # one shot against the oracle
    v, s = states[q][0].copy(), states[q][1].copy()
    od.set_source(*SRC[q])
    od.step(v, s, steps, t0=0.1)
    gv, gs = bv[q].double().cpu().numpy(), bs[q].double().cpu().numpy()
    num = ((gv - v) ** 2).sum() + ((gs - s) ** 2).sum()
    err = float(np.sqrt(num) / np.sqrt((v ** 2).sum() + (s ** 2).sum()))
    emax = float(max(np.abs(gv - v).max(), np.abs(gs - s).max()) / max(np.abs(v).max(), np.abs(s).max()))
    tol = 1e-5 if prec else 1e-12
    print(f"shots={S} k={k} prec={'fp32' if prec else 'fp64'} mode={mode} schedule={schedule} {kernel}: "
          f"bit-equal to single-shot runs; shot {q} vs FP64 oracle: rel L2 {err:.3e}, rel max-abs {emax:.3e}")
    assert err <= tol and emax <= tol


def test_shots_dependence_counters_across_calls(D):
    """Per-shot counters carry over between launches: single-step calls equal one call."""
    solver, oracle = _setup(D, 14, 2, 4, 0, ren=5)
    od = oracle()
    states = _states(od, 2, 2)
    outs = []
    for calls in (1, 5):
        g = solver()
        g.inspect(12, partition=1, splits=(13,))
        g.set_schedule(1)
        g.set_shots(2, np.array(SRC[:2]))
        bv, bs = g.zeros()
        for q in range(2):
            bv[q] = torch.from_numpy(states[q][0])
            bs[q] = torch.from_numpy(states[q][1])
        g.upload(bv, bs)
        if calls == 1:
            g.step(5, mode=1, t0=0.1)
        else:
            for i in range(5):
                g.step(1, mode=1, t0=0.1 + i * g.dt)
        g.download(bv, bs)
        torch.cuda.synchronize()
        outs.append((bv.clone(), bs.clone()))
    # the calls' start times are rounded separately (t0 + i dt), so the source term may
    # differ in its last bits; a counter error would show as a race or a timed-out wait
    num = ((outs[0][0] - outs[1][0]) ** 2).sum() + ((outs[0][1] - outs[1][1]) ** 2).sum()
    den = (outs[0][0] ** 2).sum() + (outs[0][1] ** 2).sum()
    err = float(torch.sqrt(num / den))
    print(f"2 shots, dependence-driven, 5 single-step calls vs one call: rel L2 diff {err:.3e}")
    assert err <= 1e-13


def test_shots_reset_and_errors(D):
    solver, _ = _setup(D, 8, 1, 4, 0)
    g = solver()
    g.inspect(8, partition=1)
    with pytest.raises(D.DgtError) as e:
        g.set_shots(0)
    assert e.value.status == D.DGT_EINVAL
    with pytest.raises(D.DgtError) as e:
        g.set_shots(2, np.array([[0.5, 0.5], [3.0, 0.5]]))
    assert e.value.status == D.DGT_EINVAL
    g.set_shots(2)  # no sources
    with pytest.raises(D.DgtError) as e:  # the state was reset: nothing uploaded yet
        g.step(1, mode=1)
    assert e.value.status == D.DGT_ESTATE
    v, s = g.zeros()
    g.upload(v, s)
    g.step(3, mode=1)
    g.download(v, s)
    torch.cuda.synchronize()
    assert float(v.abs().max()) == 0.0 and float(s.abs().max()) == 0.0  # no sources, zero start
    assert g.info()["bytes_per_step"] == (2 * 5 * g.np * 2 + 9) * 8 * g.mesh.nc


# ------------------------------------------------------------------ autotuner

def test_autotune_picks_a_candidate_keeps_state_and_matches_oracle(D):
    solver, oracle = _setup(D, 16, 2, 4, 0, ren=3)
    od = oracle()
    (v, s), = _states(od, 2, 1)
    g = solver()
    g.set_source(*SRC[0])
    gv = torch.from_numpy(v.copy()).cuda()
    gs = torch.from_numpy(s.copy()).cuda()
    g.upload(gv, gs)
    cands = (8, 16, 24, 40)
    r = g.autotune(cands, splits=(13,), trial_steps=2)
    print(f"autotune: {r}")
    assert r["tile_size"] in cands and r["schedule"] in (0, 1)
    assert r["timed"] >= 4 and r["skipped"] == 0 and r["ms_per_step"] > 0
    sub = g.schedule().sub_info(0)
    assert sub["ntiles"] == -(-g.mesh.nc // r["tile_size"])
    kv, ks = g.zeros()
    g.download(kv, ks)
    torch.cuda.synchronize()
    assert torch.equal(kv, gv) and torch.equal(ks, gs)  # the caller's state survives the trials
    g.step(5, mode=1, t0=0.1)
    g.download(kv, ks)
    torch.cuda.synchronize()
    od.set_source(*SRC[0])
    od.step(v, s, 5, t0=0.1)
    num = ((kv.cpu().numpy() - v) ** 2).sum() + ((ks.cpu().numpy() - s) ** 2).sum()
    err = float(np.sqrt(num / ((v ** 2).sum() + (s ** 2).sum())))
    print(f"after autotune (ts={r['tile_size']}, schedule={r['schedule']}): rel L2 err vs oracle {err:.3e}")
    assert err <= 1e-12


def test_autotune_with_shots_prunes_and_rejects(D):
    solver, _ = _setup(D, 12, 4, 4, 0)
    g = solver()
    g.set_shots(2, np.array(SRC[:2]))
    ops = (4, 8, 12, 13, 17, 21, 25)
    # P4 FP64, one operator per sub-chain: a tile holding the whole mesh exceeds the LDS and
    # would run with its working set in global memory; with candidates that fit the LDS it
    # is not timed
    r = g.autotune((4, 8, 2000), splits=ops, trial_steps=1)
    assert r["tile_size"] in (4, 8) and r["skipped"] == 1
    r = g.autotune((4, 8, 16), splits=ops, trial_steps=1, prune=1.0)
    assert r["timed"] <= 2 and r["skipped"] >= 2  # only the lowest-cost candidate is timed
    with pytest.raises(D.DgtError) as e:
        g.autotune((), splits=(13,))
    assert e.value.status == D.DGT_EINVAL
    with pytest.raises(D.DgtError) as e:
        g.autotune((4,), splits=(13,), trial_steps=0)
    assert e.value.status == D.DGT_EINVAL
    r = g.autotune((5000,), splits=())  # the only candidate: the whole mesh in one tile, from global memory
    assert r["tile_size"] == 5000 and g.kernels() == [3]
