"""Oracle pins of the FWI adjoint (CPU only).

* The reading the adjoint rests on: with the central flux and free-surface or
  periodic boundaries, the transpose of one time step equals T^-1 Phi(-dt) T with
  T = blockdiag(M_J^-1 / rho, M_J^-1 C) per cell, checked on dense step matrices
  built column by column from the oracle's own time step; with absorbing sides it
  does not hold (the discretisation is then dissipative).
* The oracle's adjoint gradient equals central finite differences of the oracle's
  misfit (error O(h^2)), for time orders 2 and 4.
"""
import numpy as np
import pytest

import oracle as O
from paper_1708_03183_amd import inputs as I


def _material(m, seed=0):
    lam, mu, rho = I.layered_material(m)
    rng = np.random.default_rng(seed)
    return (lam * (1 + 0.3 * rng.random(m.nc)), mu * (1 + 0.3 * rng.random(m.nc)),
            rho * (1 + 0.3 * rng.random(m.nc)))


def _step_matrix(om, k, lam, mu, rho, order, dt, free):
    d = O.ODG(om, k, lam, mu, rho, flux=0, order=order, dt=dt, free_sides=free)
    npk, nc = O.np_of(k), om.nc
    N = 5 * npk * nc
    A = np.zeros((N, N))
    for j in range(N):
        x = np.zeros(N)
        x[j] = 1.0
        v = x[:2 * npk * nc].reshape(2, npk, nc).copy()
        s = x[2 * npk * nc:].reshape(3, npk, nc).copy()
        d.step(v, s, 1, t0=0.0)
        A[:, j] = np.concatenate([v.ravel(), s.ravel()])
    return A


def _T(om, k, lam, mu, rho):
    npk, nc = O.np_of(k), om.nc
    Minv = O.refelem(k)["Minv"]
    p = om.xy[om.c2v]
    det = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    N = 5 * npk * nc
    T = np.zeros((N, N))
    iv = lambda c, i, K: (c * npk + i) * nc + K
    is_ = lambda c, i, K: 2 * npk * nc + (c * npk + i) * nc + K
    for K in range(nc):
        Mi = Minv / det[K]
        Cm = np.array([[lam[K] + 2 * mu[K], lam[K], 0], [lam[K], lam[K] + 2 * mu[K], 0], [0, 0, mu[K]]])
        for i in range(npk):
            for j in range(npk):
                for c in range(2):
                    T[iv(c, i, K), iv(c, j, K)] = Mi[i, j] / rho[K]
                for a in range(3):
                    for b in range(3):
                        T[is_(a, i, K), is_(b, j, K)] = Mi[i, j] * Cm[a, b]
    return T


@pytest.mark.parametrize("k,order,free,per", [(1, 2, 0xF, 0), (1, 4, 0xF, 0), (2, 4, 0xF, 0), (2, 2, 0x0, 3)])
def test_step_transpose_is_the_reversed_transformed_step(k, order, free, per):
    m = I.square_mesh(3, jitter=0.2, renumber_seed=3, periodic=per)
    lam, mu, rho = _material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    F = _step_matrix(om, k, lam, mu, rho, order, dt, free)
    B = _step_matrix(om, k, lam, mu, rho, order, -dt, free)
    T = _T(om, k, lam, mu, rho)
    G = np.linalg.solve(T, B @ T)
    err = np.abs(F.T - G).max() / np.abs(F).max()
    print(f"k={k} order={order} free={free:#x} periodic={per}: max |Phi^T - T^-1 Phi(-dt) T| / max |Phi| = {err:.2e}")
    assert err <= 1e-13


def test_step_transpose_differs_with_absorbing_sides():
    m = I.square_mesh(3, jitter=0.2, renumber_seed=3)
    lam, mu, rho = _material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, 1, lam, mu, rho)
    F = _step_matrix(om, 1, lam, mu, rho, 2, dt, 0x3)
    B = _step_matrix(om, 1, lam, mu, rho, 2, -dt, 0x3)
    T = _T(om, 1, lam, mu, rho)
    err = np.abs(F.T - np.linalg.solve(T, B @ T)).max() / np.abs(F).max()
    assert err > 1e-3


SHOTS = np.array([[0.3, 0.6], [0.7, 0.4]])
RECS = np.array([[0.2, 0.9], [0.5, 0.95], [0.8, 0.7]])


def _fwi_case(n, k, order, per=0, nsteps=12):
    m = I.square_mesh(n, jitter=0.2, renumber_seed=3, periodic=per)
    lam, mu, rho = I.layered_material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    free = 0x0 if per else 0xF

    def mk(l, u, r, d=dt):
        return O.ODG(om, k, l, u, r, flux=0, order=order, dt=d, free_sides=free)

    obs = O.fwi_traces(mk(lam * 1.1, mu * 0.95, rho * 1.05), RECS, SHOTS, nsteps, f0=8.0, t0=0.05)
    return m, lam, mu, rho, dt, mk, obs


@pytest.mark.parametrize("n,k,order,per", [(4, 1, 2, 0), (4, 1, 4, 0), (4, 2, 4, 0), (4, 2, 2, 3)])
def test_oracle_adjoint_gradient_matches_finite_differences(n, k, order, per):
    nsteps = 12
    m, lam, mu, rho, dt, mk, obs = _fwi_case(n, k, order, per, nsteps)
    J, g = O.fwi_gradient_adjoint(mk(lam, mu, rho), mk(lam, mu, rho, -dt), order, RECS, SHOTS, nsteps, obs,
                                  f0=8.0, t0=0.05)
    assert abs(J - O.fwi_misfit(mk(lam, mu, rho), RECS, SHOTS, nsteps, obs, f0=8.0, t0=0.05)) <= 1e-14 * J
    base = np.stack([lam, mu, rho])
    d = np.random.default_rng(5).standard_normal((3, m.nc))
    h = 1e-5
    Jp = O.fwi_misfit(mk(*(base * (1 + h * d))), RECS, SHOTS, nsteps, obs, f0=8.0, t0=0.05)
    Jm = O.fwi_misfit(mk(*(base * (1 - h * d))), RECS, SHOTS, nsteps, obs, f0=8.0, t0=0.05)
    fd = (Jp - Jm) / (2 * h)
    ad = float((g * base * d).sum())
    print(f"n={n} k={k} order={order} periodic={per}: directional derivative fd {fd:.10e} adjoint {ad:.10e}")
    assert abs(fd - ad) <= 1e-7 * abs(ad)


def test_misfit_vanishes_on_its_own_traces():
    m, lam, mu, rho, dt, mk, obs = _fwi_case(4, 1, 2)
    own = O.fwi_traces(mk(lam, mu, rho), RECS, SHOTS, 12, f0=8.0, t0=0.05)
    assert O.fwi_misfit(mk(lam, mu, rho), RECS, SHOTS, 12, own, f0=8.0, t0=0.05) == 0.0
    e = np.random.default_rng(1).standard_normal(own.shape)
    assert abs(O.fwi_misfit(mk(lam, mu, rho), RECS, SHOTS, 12, own + e, f0=8.0, t0=0.05) - 0.5 * (e ** 2).sum()) <= 1e-12
