"""GPU: full-waveform-inversion misfit and gradient (dgt_fwi_forward / dgt_fwi_gradient).

The library's receiver traces, misfit and per-cell gradient (lambda, mu, rho)
match the FP64 oracle's traces, misfit and discrete-adjoint gradient (itself
pinned to finite differences on the CPU), for both time orders, untiled and tiled
reversal, both schedules, several checkpoint counts and batched shots.
"""
import numpy as np
import pytest

import oracle as O
from paper_1708_03183_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHOTS = np.array([[0.3, 0.6], [0.7, 0.4]])
RECS = np.array([[0.2, 0.9], [0.5, 0.95], [0.8, 0.7], [0.45, 0.1]])


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_03183_amd import dgtile
    dgtile.lib()
    return dgtile


def _case(D, n, k, order, prec=0, per=0, nsteps=14, shots=SHOTS):
    m = I.square_mesh(n, jitter=0.2, renumber_seed=3, periodic=per)
    lam, mu, rho = I.layered_material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    free = 0x0 if per else 0xF

    def mk(l, u, r, d=dt):
        return O.ODG(om, k, l, u, r, flux=0, order=order, dt=d, free_sides=free)

    obs = O.fwi_traces(mk(lam * 1.1, mu * 0.95, rho * 1.05), RECS, shots, nsteps, f0=8.0, t0=0.05)
    J, g = O.fwi_gradient_adjoint(mk(lam, mu, rho), mk(lam, mu, rho, -dt), order, RECS, shots, nsteps, obs,
                                  f0=8.0, t0=0.05)
    gm = D.Mesh.from_mesh(m)

    def solver(nshots=len(shots), xy=shots):
        s = D.Solver(gm, lam, mu, rho, degree=k, flux=0, time_order=order, precision=prec, free_sides=free, dt=dt)
        s.set_shots(nshots, np.asarray(xy).reshape(-1, 2), 8.0, 0.05, 1.0)
        return s

    return dict(m=m, mk=mk, obs=obs, J=J, g=g, solver=solver, nsteps=nsteps, lam=lam, mu=mu, rho=rho)


def _rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum()) / np.sqrt((b ** 2).sum()))


FWI_CASES = [
    # n, k, order, prec, periodic, mode, schedule, ts, splits, nsnap
    (6, 1, 2, 0, 0, 0, 0, 0, (), 3),
    (6, 1, 4, 0, 0, 1, 0, 10, (13,), 2),
    (6, 2, 4, 0, 0, 1, 1, 10, (13,), 4),
    (6, 2, 2, 0, 3, 1, 1, 12, (), 5),
    (5, 3, 4, 0, 0, 1, 0, 8, (4, 8, 12, 13, 17, 21, 25), 3),
    (6, 2, 4, 1, 0, 1, 1, 10, (13,), 4),
]


@pytest.mark.parametrize("n,k,order,prec,per,mode,schedule,ts,splits,nsnap", FWI_CASES)
def test_fwi_gradient_matches_oracle_adjoint(D, n, k, order, prec, per, mode, schedule, ts, splits, nsnap):
    c = _case(D, n, k, order, prec, per)
    s = c["solver"]()
    if mode == 1:
        s.inspect(ts, partition=1, splits=splits)
        s.set_schedule(schedule)
    tr = s.fwi_forward(RECS, c["nsteps"], mode=mode)
    own = O.fwi_traces(c["mk"](c["lam"], c["mu"], c["rho"]), RECS, SHOTS, c["nsteps"], f0=8.0, t0=0.05)
    err_tr = _rel(tr.cpu().numpy(), own)
    obs = torch.from_numpy(c["obs"]).cuda().contiguous()
    J, gl, gm, gr = s.fwi_gradient(RECS, c["nsteps"], obs, nsnap=nsnap, mode=mode)
    g = np.stack([x.cpu().numpy() for x in (gl, gm, gr)])
    err_J = abs(J - c["J"]) / c["J"]
    err_g = _rel(g, c["g"])
    print(f"FWI n={n} k={k} order={order} {'fp32' if prec else 'fp64'} periodic={per} mode={mode} "
          f"schedule={schedule} nsnap={nsnap}: traces {err_tr:.2e}, misfit {err_J:.2e}, gradient {err_g:.2e} "
          f"(rel L2 vs the FP64 oracle)")
    tol = 1e-4 if prec else 1e-10
    assert err_tr <= (1e-5 if prec else 1e-12)
    assert err_J <= tol and err_g <= tol


def test_fwi_gradient_independent_of_checkpoints_and_shot_batching(D):
    c = _case(D, 6, 2, 4)
    obs = torch.from_numpy(c["obs"]).cuda().contiguous()
    grads = []
    for nsnap in (1, 3, c["nsteps"]):
        s = c["solver"]()
        s.inspect(10, partition=1, splits=(13,))
        s.set_schedule(1)
        J, *g = s.fwi_gradient(RECS, c["nsteps"], obs, nsnap=nsnap, mode=1)
        grads.append((J, torch.stack(g)))
    for J, g in grads[1:]:  # the replays recompute the forward states bit for bit
        assert J == grads[0][0] and torch.equal(g, grads[0][1])
    # two shots in one batch = the sum of the two one-shot gradients
    parts = []
    for q in range(2):
        s = c["solver"](1, SHOTS[q])
        s.inspect(10, partition=1, splits=(13,))
        J, *g = s.fwi_gradient(RECS, c["nsteps"], obs[q:q + 1].contiguous(), nsnap=3, mode=1)
        parts.append((J, torch.stack(g)))
    Jsum = parts[0][0] + parts[1][0]
    gsum = parts[0][1] + parts[1][1]
    assert abs(grads[0][0] - Jsum) <= 1e-13 * Jsum
    assert float((grads[0][1] - gsum).norm() / gsum.norm()) <= 1e-12


def test_fwi_autograd_function(D):
    from paper_1708_03183_amd import fwi as F
    c = _case(D, 6, 1, 4)
    setup = F.FwiSetup(mesh=D.Mesh.from_mesh(c["m"]), degree=1, dt=c["mk"](c["lam"], c["mu"], c["rho"]).dt,
                       shots_xy=SHOTS, rec_xy=RECS, nsteps=c["nsteps"],
                       observed=torch.from_numpy(c["obs"]).cuda().contiguous(), nsnap=4, mode=1, tile_size=10,
                       splits=(13,), f0=8.0, t0=0.05)
    lam, mu, rho = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in (c["lam"], c["mu"], c["rho"])]
    J = F.misfit(lam, mu, rho, setup)
    J.backward()
    g = np.stack([t.grad.numpy() for t in (lam, mu, rho)])
    assert abs(J.detach().item() - c["J"]) <= 1e-10 * c["J"]
    assert _rel(g, c["g"]) <= 1e-10


def test_fwi_errors(D):
    c = _case(D, 5, 1, 2, nsteps=4)
    obs = torch.from_numpy(c["obs"]).cuda().contiguous()
    s = c["solver"]()
    with pytest.raises(D.DgtError) as e:  # tiled mode needs an inspection
        s.fwi_gradient(RECS, 4, obs, mode=1)
    assert e.value.status == D.DGT_ESTATE
    with pytest.raises(D.DgtError) as e:
        s.fwi_gradient(RECS, 4, obs, nsnap=0, mode=0)
    assert e.value.status == D.DGT_EINVAL
    with pytest.raises(D.DgtError) as e:
        s.fwi_gradient(np.array([[0.5, 2.0]] * 4), 4, obs, mode=0)
    assert e.value.status == D.DGT_EINVAL
    m = c["m"]
    gm = D.Mesh.from_mesh(m)
    for flux, free in ((1, 0xF), (0, 0x8)):  # upwind flux; absorbing sides: the closed-form reversal
        u = D.Solver(gm, c["lam"], c["mu"], c["rho"], degree=1, flux=flux, time_order=2, free_sides=free, dt=1e-3)
        u.set_shots(2, SHOTS)
        J, *g = u.fwi_gradient(RECS, 4, obs, mode=0)
        assert np.isfinite(J) and all(bool(torch.isfinite(x).all()) for x in g)


@pytest.mark.parametrize("k,prec,schedule,splits", [(2, 0, 1, (13,)), (2, 1, 0, (13,)), (3, 0, 1, (4, 8, 12, 13, 17, 21, 25))])
def test_fwi_intermediates_from_tiled_steps_match_untiled(D, monkeypatch, k, prec, schedule, splits):
    """Order 4 with a split at the end of the velocity half keeps U, X, Z of recorded
    tiled steps; the untiled operator applications give the same gradient."""
    c = _case(D, 5 if k == 3 else 6, k, 4, prec)
    obs = torch.from_numpy(c["obs"]).cuda().contiguous()
    out = []
    for env in (None, "1"):
        if env:
            monkeypatch.setenv("DGT_FWI_UNTILED_INTERMEDIATES", env)
        s = c["solver"]()
        s.inspect(8 if k == 3 else 10, partition=1, splits=splits)
        s.set_schedule(schedule)
        J, *g = s.fwi_gradient(RECS, c["nsteps"], obs, nsnap=3, mode=1)
        out.append((J, np.stack([x.cpu().numpy() for x in g])))
    err_rec, err_unt = _rel(out[0][1], c["g"]), _rel(out[1][1], c["g"])
    diff = _rel(out[0][1], out[1][1])
    print(f"k={k} {'fp32' if prec else 'fp64'} schedule={schedule}: gradient vs oracle, recorded tiled "
          f"intermediates {err_rec:.2e}, untiled {err_unt:.2e}; between them {diff:.2e}")
    tol = 1e-4 if prec else 1e-10
    assert err_rec <= tol and err_unt <= tol and diff <= tol


def _cfl_dt(m, lam, mu, rho, k):
    p = m.xy[m.c2v]
    e = [np.hypot(*(p[:, (i + 1) % 3] - p[:, i]).T) for i in range(3)]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    hmin = float(np.min(4.0 * area / (e[0] + e[1] + e[2])))
    return 0.2 * hmin / ((2 * k + 1) * float(np.max(np.sqrt((lam + 2 * mu) / rho))))


def test_fwi_gradient_full_size_directional_derivative(D):
    """At the FWI workload's size (256x256 mesh, 131,072 cells, P2, surface survey,
    2000 steps; 4 of its 16 shots, FP64 state, tiled at 256 seeds, dependence-driven)
    the oracle cannot run, but the discrete adjoint gradient is exact for the discrete
    misfit at any size: its inner product with a perturbation of (lambda, mu, rho)
    equals the central difference of the misfit along it, up to O(eps^2)."""
    print("case fwi256 full size: building the mesh and the observed data", flush=True)
    k, n, nrec, nsteps = 2, 256, 128, 2000
    m = I.square_mesh(n, jitter=0.2, jitter_seed=30, renumber_seed=31)
    lam_t, mu_t, rho_t = I.layered_material(m)
    lam0, mu0, rho0 = [np.full(m.nc, float(x.mean())) for x in (lam_t, mu_t, rho_t)]
    dt = min(_cfl_dt(m, lam_t, mu_t, rho_t, k), _cfl_dt(m, lam0, mu0, rho0, k))
    rng = np.random.default_rng(16)
    shots = np.stack([rng.uniform(0.1, 0.9, 16), rng.uniform(0.96, 0.99, 16)], axis=1)[:4]
    recs = np.stack([(np.arange(nrec) + 0.5) / nrec, np.ones(nrec)], axis=1)
    gm = D.Mesh.from_mesh(m)

    def make(lam, mu, rho):
        s = D.Solver(gm, lam, mu, rho, degree=k, flux=0, time_order=4, precision=0, free_sides=0xF, dt=dt)
        s.set_shots(len(shots), shots, 100.0, 0.012, 1.0)
        s.inspect(256, partition=1, splits=(13,))
        s.set_schedule(1)
        return s

    obs = make(lam_t, mu_t, rho_t).fwi_forward(recs, nsteps, mode=1)
    J, gl, gmu, gr = make(lam0, mu0, rho0).fwi_gradient(recs, nsteps, obs, nsnap=32, mode=1)
    g = np.stack([x.cpu().numpy() for x in (gl, gmu, gr)])
    prng = np.random.default_rng(2024)
    dm = np.stack([b * prng.uniform(-1.0, 1.0, m.nc) for b in (lam0, mu0, rho0)])

    def misfit(eps):
        tr = make(*(base + eps * d for base, d in zip((lam0, mu0, rho0), dm))).fwi_forward(recs, nsteps, mode=1)
        return 0.5 * float(((tr - obs) ** 2).sum())

    J0 = misfit(0.0)
    eps = 1e-4
    fd = (misfit(eps) - misfit(-eps)) / (2 * eps)
    ad = float((g * dm).sum())
    err_J, err_d = abs(J0 - J) / J, abs(fd - ad) / abs(ad)
    print(f"fwi256 full size, 4 shots, {nsteps} steps: misfit {J:.6e} (from traces: rel diff {err_J:.1e}); "
          f"directional derivative adjoint {ad:.10e}, central difference {fd:.10e}, rel diff {err_d:.2e}")
    assert err_J <= 1e-12
    assert err_d <= 1e-6


def _case_upw(D, n, k, order, flux, free, prec=0, nsteps=10, shots=SHOTS):
    """Upwind flux and / or absorbing sides on a lognormal material (impedance jumps
    between every pair of cells); the oracle gradient is the Richardson-extrapolated
    difference quotient of the oracle's misfit, parameter by parameter."""
    m = I.square_mesh(n, jitter=0.2, renumber_seed=3)
    lam, mu, rho = I.lognormal_material(m, sigma=0.3, seed=7)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)

    def mk(l, u, r):
        return O.ODG(om, k, l, u, r, flux=flux, order=order, dt=dt, free_sides=free)

    obs = O.fwi_traces(mk(lam * 1.1, mu * 0.95, rho * 1.05), RECS, shots, nsteps, f0=8.0, t0=0.05)
    J = O.fwi_misfit(mk(lam, mu, rho), RECS, shots, nsteps, obs, f0=8.0, t0=0.05)
    g = O.fwi_gradient_fd(mk, lam, mu, rho, RECS, shots, nsteps, obs, f0=8.0, t0=0.05)
    gm = D.Mesh.from_mesh(m)

    def solver():
        s = D.Solver(gm, lam, mu, rho, degree=k, flux=flux, time_order=order, precision=prec, free_sides=free,
                     dt=dt)
        s.set_shots(len(shots), np.asarray(shots).reshape(-1, 2), 8.0, 0.05, 1.0)
        return s

    return dict(obs=obs, J=J, g=g, solver=solver, nsteps=nsteps)


FWI_UPW_CASES = [
    # n, k, order, flux, free sides, precision, mode, schedule, tile size, splits, checkpoints
    (5, 1, 4, 1, 0x8, 0, 0, 0, 0, (), 3),
    (5, 2, 4, 1, 0x8, 0, 1, 1, 10, (13,), 2),
    (5, 1, 2, 1, 0x0, 0, 1, 0, 10, (), 4),
    (5, 2, 2, 1, 0xF, 0, 0, 0, 0, (), 1),
    (5, 1, 4, 0, 0x8, 0, 1, 1, 10, (13,), 3),
    (4, 3, 4, 1, 0x8, 0, 1, 0, 8, (4, 8, 13, 17, 21), 2),
    (5, 2, 4, 1, 0x8, 1, 1, 1, 10, (13,), 3),
]


@pytest.mark.parametrize("n,k,order,flux,free,prec,mode,schedule,ts,splits,nsnap", FWI_UPW_CASES)
def test_fwi_gradient_upwind_absorbing(D, n, k, order, flux, free, prec, mode, schedule, ts, splits, nsnap):
    """The closed-form transposed step with the upwind flux (exact Riemann states at
    impedance jumps) and absorbing sides: misfit and per-cell gradient against the
    oracle's difference quotients (accurate to ~1e-11)."""
    c = _case_upw(D, n, k, order, flux, free, prec)
    s = c["solver"]()
    if mode == 1:
        s.inspect(ts, partition=1, splits=splits)
        s.set_schedule(schedule)
    obs = torch.from_numpy(c["obs"]).cuda().contiguous()
    J, gl, gm, gr = s.fwi_gradient(RECS, c["nsteps"], obs, nsnap=nsnap, mode=mode)
    g = np.stack([x.cpu().numpy() for x in (gl, gm, gr)])
    err_J = abs(J - c["J"]) / c["J"]
    err_g = _rel(g, c["g"])
    mx = float(np.abs(g - c["g"]).max() / np.abs(c["g"]).max())
    print(f"FWI upwind n={n} k={k} order={order} flux={flux} free={free:#x} {'fp32' if prec else 'fp64'} mode={mode} "
          f"nsnap={nsnap}: misfit {err_J:.2e}, gradient rel L2 {err_g:.2e}, max-abs {mx:.2e}")
    tol = 1e-4 if prec else 1e-8
    assert err_J <= (1e-5 if prec else 1e-12)
    assert err_g <= tol and mx <= tol


def test_fwi_closed_form_equals_reversed_chain(D, monkeypatch):
    """In the energy-conserving case both reversals apply: the closed-form transposed
    step gives the reversed chain's gradient (and the oracle adjoint's)."""
    c = _case(D, 6, 2, 4)
    obs = torch.from_numpy(c["obs"]).cuda().contiguous()
    s = c["solver"]()
    J0, *g0 = s.fwi_gradient(RECS, c["nsteps"], obs, nsnap=3, mode=0)
    monkeypatch.setenv("DGT_FWI_CLOSED_FORM", "1")
    s = c["solver"]()
    J1, *g1 = s.fwi_gradient(RECS, c["nsteps"], obs, nsnap=3, mode=0)
    a = np.stack([x.cpu().numpy() for x in g0])
    b = np.stack([x.cpu().numpy() for x in g1])
    err = _rel(b, a)
    print(f"closed form vs reversed chain: misfit {abs(J1 - J0) / J0:.2e}, gradient {err:.2e}; "
          f"vs oracle adjoint {_rel(b, c['g']):.2e}")
    assert abs(J1 - J0) <= 1e-14 * J0 and err <= 1e-12 and _rel(b, c["g"]) <= 1e-10


def test_fwi_upwind_gradient_independent_of_checkpoints(D):
    c = _case_upw(D, 5, 1, 4, 1, 0x8)
    obs = torch.from_numpy(c["obs"]).cuda().contiguous()
    out = []
    for nsnap in (1, 4, 10):
        s = c["solver"]()
        J, *g = s.fwi_gradient(RECS, c["nsteps"], obs, nsnap=nsnap, mode=0)
        out.append(np.stack([x.cpu().numpy() for x in g]))
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
