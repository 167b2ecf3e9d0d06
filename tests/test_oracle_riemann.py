"""Pins of the oracle's facet fluxes against the exact Riemann problem of
isotropic elasticity (the paper's DG solver, Sec. 7.1, prints no flux; the
reading is the exact upwind flux, or the central average).

With a state that is constant in every cell the volume terms vanish and each
facet of a P1 cell contributes a constant jump g_f, lifted onto the cell by a
known vector.  The three P1 lift vectors form a basis, so the rate of one
cell, as the oracle's assembled operator returns it, splits exactly into its
three per-facet jumps; from them the interface traction T* and velocity v*
seen by that cell follow.  Along the facet normal n (Z_p) and tangent t (Z_s)
the exact solution carries the outgoing characteristic of each side:

    T* - Z- v* = T- - Z- v-        (from the inside)
    T* + Z+ v* = T+ + Z+ v+        (from the outside)

with T = sigma n measured with the inside cell's outward normal.  The free
surface is T* = 0 with the inside characteristic (upwind) or v* = v- (central);
the absorbing side lets nothing in: T* + Z v* = 0.  The P1 lift basis and mass
matrix below are the closed forms, not the oracle's tables."""
import numpy as np
import pytest

import oracle as O
from paper_1708_03183_amd import inputs as I

# P1 on the reference triangle: nodes (0,0), (1,0), (0,1); facet l joins local
# vertices l and l+1; the facet mass on [0,1] times (1,1) is (1/2, 1/2)
MHAT = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 24.0
EM1 = np.array([[0.5, 0.0, 0.5],    # column l: facet l's nodes get 1/2 each
                [0.5, 0.5, 0.0],
                [0.0, 0.5, 0.5]])


def _mesh_and_material(n, seed, contrast=True):
    m = I.square_mesh(n, jitter=0.2, jitter_seed=seed)
    u = I.uniform01(seed + 10, 3 * m.nc).reshape(3, m.nc)
    if contrast:  # every cell independently at one of two levels 4x (lam, mu) and 5x (rho) apart
        lam = np.where(u[0] < 0.5, 2.0, 8.0)
        mu = np.where(u[1] < 0.5, 1.0, 4.0)
        rho = np.where(u[2] < 0.5, 1.0, 5.0)
    else:
        lam, mu, rho = I.homogeneous_material(m)
    return m, O.OMesh.from_mesh(m), lam, mu, rho


def _cell_geometry(m, c):
    p = m.xy[m.c2v[c]]
    det = (p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[2, 0] - p[0, 0]) * (p[1, 1] - p[0, 1])
    out = []
    for l in range(3):
        e = p[(l + 1) % 3] - p[l]
        L = float(np.hypot(*e))
        out.append((L, np.array([e[1], -e[0]]) / L))  # counter-clockwise cell: outward normal
    return det, out


def _facet_jumps(rate_cell, det, geo, w):
    """Per-facet constant jumps g_f from a P1 cell's rate (nodes x components):
    rate = (1/(w |J|)) Mhat^-1 sum_f |f| EM1[:, f] g_f."""
    c = np.linalg.solve(EM1, MHAT @ rate_cell)   # row f: |f| g_f / (w |J|)
    return [c[f] * (w * det) / geo[f][0] for f in range(3)]


def _imp(lam, mu, rho):
    return np.sqrt(rho * (lam + 2 * mu)), np.sqrt(rho * mu)


def _interface_states(d, m, om, lam, mu, rho, v, s):
    """For every (cell, local facet): (T-, v-, T*, v*) recovered from the rate."""
    dv, ds = d.rate(v, s)
    out = {}
    for c in range(m.nc):
        det, geo = _cell_geometry(m, c)
        gv = _facet_jumps(dv[:, :, c].T, det, geo, rho[c])         # T* - T-
        gs = _facet_jumps(ds[:, :, c].T, det, geo, 1.0)            # C sym((v* - v-) x n)
        sig = np.array([[s[0, 0, c], s[2, 0, c]], [s[2, 0, c], s[1, 0, c]]])
        vin = v[:, 0, c]
        l2m = lam[c] + 2 * mu[c]
        for f in range(3):
            n = geo[f][1]
            A = np.array([[l2m * n[0], lam[c] * n[1]], [lam[c] * n[0], l2m * n[1]], [mu[c] * n[1], mu[c] * n[0]]])
            e, res, *_ = np.linalg.lstsq(A, gs[f], rcond=None)
            # the stress facet term has the form C sym(e x n): nothing outside that range
            assert np.abs(A @ e - gs[f]).max() <= 1e-12 * max(1.0, np.abs(gs[f]).max())
            Tm = sig @ n
            out[(c, f)] = (Tm, vin.copy(), Tm + gv[f], vin + e, n)
    return out


def _neighbours(om):
    mp = om.maps()
    nb = {}
    for f in range(len(mp["f2c"])):
        a, b = (int(x) for x in mp["f2c"][f])
        la, lb = (int(x) for x in mp["f2l"][f])
        nb[(a, la)] = (b, lb)
        nb[(b, lb)] = (a, la)
    ext = {}
    for b in range(len(mp["b2c"])):
        ext[(int(mp["b2c"][b]), int(mp["b2l"][b]))] = int(mp["bside"][b])
    return nb, ext


def _nt(x, n):
    return np.array([x @ n, x @ np.array([-n[1], n[0]])])


@pytest.mark.parametrize("flux", [1, 0])
@pytest.mark.parametrize("free", [0x8, 0x5, 0xF, 0x0])
def test_facet_fluxes_solve_the_riemann_problem(flux, free):
    """Random constant states, material contrast of 4-5x between neighbours."""
    m, om, lam, mu, rho = _mesh_and_material(3, 7)
    d = O.ODG(om, 1, lam, mu, rho, flux=flux, order=4, dt=1e-3, free_sides=free)
    v, s = d.zeros()
    rv = I.random_state((2, m.nc), 31)
    rs = I.random_state((3, m.nc), 32)
    v[:] = rv[:, None, :]
    s[:] = rs[:, None, :]
    st = _interface_states(d, m, om, lam, mu, rho, v, s)
    nb, ext = _neighbours(om)
    checked = {"int": 0, "free": 0, "abs": 0}
    tol = 1e-14
    for (c, f), (Tm, vm, Ts, vs, n) in st.items():
        zpm, zsm = _imp(lam[c], mu[c], rho[c])
        Zm = np.array([zpm, zsm])
        Tm_, vm_, Ts_, vs_ = _nt(Tm, n), _nt(vm, n), _nt(Ts, n), _nt(vs, n)
        scale = np.abs(np.concatenate([Tm_, Zm * vm_])).max()
        if (c, f) in nb:
            o, lo = nb[(c, f)]
            zpp, zsp = _imp(lam[o], mu[o], rho[o])
            Zp = np.array([zpp, zsp])
            sig_o = np.array([[s[0, 0, o], s[2, 0, o]], [s[2, 0, o], s[1, 0, o]]])
            Tp_, vp_ = _nt(sig_o @ n, n), _nt(v[:, 0, o], n)
            scale = max(scale, np.abs(np.concatenate([Tp_, Zp * vp_])).max())
            if flux == 1:
                assert np.abs((Ts_ - Zm * vs_) - (Tm_ - Zm * vm_)).max() <= tol * scale
                assert np.abs((Ts_ + Zp * vs_) - (Tp_ + Zp * vp_)).max() <= tol * scale
            else:
                assert np.abs(Ts_ - 0.5 * (Tm_ + Tp_)).max() <= tol * scale
                assert np.abs(vs_ - 0.5 * (vm_ + vp_)).max() <= tol * scale
            # the other side sees the same interface state (its normal is -n)
            To, vo, Tso, vso, no = st[(o, lo)]
            assert np.abs(no + n).max() <= 1e-15
            assert np.abs(Tso + Ts).max() <= tol * scale and np.abs(vso - vs).max() <= tol * scale
            checked["int"] += 1
        else:
            side = ext[(c, f)]
            if (free >> side) & 1:
                assert np.abs(Ts_).max() <= tol * scale
                if flux == 1:
                    assert np.abs((Ts_ - Zm * vs_) - (Tm_ - Zm * vm_)).max() <= tol * scale
                else:
                    assert np.abs(vs_ - vm_).max() <= tol * scale
                checked["free"] += 1
            else:
                assert np.abs((Ts_ - Zm * vs_) - (Tm_ - Zm * vm_)).max() <= tol * scale
                assert np.abs(Ts_ + Zm * vs_).max() <= tol * scale
                checked["abs"] += 1
    assert checked["int"] == 2 * len(nb) // 2 and checked["free"] + checked["abs"] == len(ext)
    if free == 0xF:
        assert checked["abs"] == 0
    if free == 0x0:
        assert checked["free"] == 0


@pytest.mark.parametrize("flux", [1, 0])
def test_equal_states_give_the_state_back(flux):
    """Consistency: the same constant state in every cell, whatever the material
    jumps, gives T* = T and v* = v on interior facets, so interior cells do not move."""
    m, om, lam, mu, rho = _mesh_and_material(4, 9)
    d = O.ODG(om, 1, lam, mu, rho, flux=flux, order=4, dt=1e-3, free_sides=0xF)
    v, s = d.zeros()
    v[0], v[1] = 0.7, -1.3
    s[0], s[1], s[2] = 0.4, -0.9, 1.1
    st = _interface_states(d, m, om, lam, mu, rho, v, s)
    nb, ext = _neighbours(om)
    for (c, f), (Tm, vm, Ts, vs, n) in st.items():
        if (c, f) in nb:
            assert np.abs(Ts - Tm).max() <= 1e-14 and np.abs(vs - vm).max() <= 1e-14
    dv, ds = d.rate(v, s)
    inner = [c for c in range(m.nc) if all((c, f) in nb for f in range(3))]
    assert len(inner) > 0
    # scale: the same cell states with random signs, whose facet terms do not cancel
    sg = np.where(I.uniform01(5, m.nc) < 0.5, -1.0, 1.0)
    dvs, dss = d.rate(v * sg, s * sg)
    assert np.abs(dv[:, :, inner]).max() <= 1e-14 * np.abs(dvs).max()
    assert np.abs(ds[:, :, inner]).max() <= 1e-14 * np.abs(dss).max()


def test_upwind_flux_is_not_symmetric_in_the_impedances():
    """A check that would fail for an impedance-swapped flux: with Z- != Z+ the
    interface traction of the upwind flux is the Z-weighted (not the plain)
    average, e.g. v = 0 on both sides, T- = 1, T+ = 0 gives T* = Z+ / (Z- + Z+)."""
    m, om, lam, mu, rho = _mesh_and_material(3, 7)
    d = O.ODG(om, 1, lam, mu, rho, flux=1, order=4, dt=1e-3, free_sides=0xF)
    nb, _ = _neighbours(om)
    (c, f), (o, lo) = next(((a, b) for a, b in nb.items() if (rho[a[0]], lam[a[0]]) != (rho[b[0]], lam[b[0]])))
    det, geo = _cell_geometry(m, c)
    n = geo[f][1]
    v, s = d.zeros()
    # sigma = n n^T in cell c only: T- = n (normal traction 1), no tangential traction
    s[0, :, c], s[1, :, c], s[2, :, c] = n[0] * n[0], n[1] * n[1], n[0] * n[1]
    st = _interface_states(d, m, om, lam, mu, rho, v, s)
    Ts = st[(c, f)][2]
    zpm, _ = _imp(lam[c], mu[c], rho[c])
    zpp, _ = _imp(lam[o], mu[o], rho[o])
    assert abs(Ts @ n - zpp / (zpm + zpp)) <= 1e-14
    assert abs(zpp / (zpm + zpp) - 0.5) > 0.05


def _strip_mesh(n):
    """n x 2 squares of side h = 1/n on [0,1] x [0,2h], periodic in y: a pulse
    travelling along x sees only the two absorbing x sides."""
    h = 1.0 / n
    xy = np.array([(i * h, j * h) for j in range(3) for i in range(n + 1)], np.float64)
    c2v = []
    for j in range(2):
        for i in range(n):
            v00 = j * (n + 1) + i
            c2v.append((v00, v00 + 1, v00 + n + 2))
            c2v.append((v00, v00 + n + 2, v00 + n + 1))
    return xy, np.array(c2v, np.int32)


def _pulse_residual(n, k, T=0.9, width=0.1):
    """Energy left in the strip at time T relative to the start, after a P pulse
    (right-going: v_x = f, sxx = -Z f, syy = -(lam / c) f) has crossed the right
    side and every spurious part of it (left-going P, S) has had time to leave."""
    xy, c2v = _strip_mesh(n)
    om = O.OMesh(xy, c2v, periodic=2)
    nc = len(c2v)
    lam, mu, rho = np.full(nc, 2.0), np.full(nc, 1.0), np.full(nc, 1.0)
    cp = 2.0
    d = O.ODG(om, k, lam, mu, rho, flux=1, order=4, free_sides=0x0)
    steps = int(np.ceil(T / d.dt))
    nodes = np.array([(i / k, j / k) for j in range(k + 1) for i in range(k + 1 - j)])
    p = xy[c2v]
    X = p[:, 0, None, 0] + (p[:, 1, None, 0] - p[:, 0, None, 0]) * nodes[None, :, 0] + \
        (p[:, 2, None, 0] - p[:, 0, None, 0]) * nodes[None, :, 1]
    f = np.exp(-((X - 0.5) / width) ** 2).T          # [node][cell]
    v, s = d.zeros()
    v[0] = f
    s[0] = -rho[0] * cp * f
    s[1] = -(lam[0] / cp) * f
    s_old = s.copy()
    d.step(v, s, 1)
    e0 = d.energy(v, s, s_old)
    s_old = s.copy()
    d.step(v, s, steps - 2)
    s_old = s.copy()
    d.step(v, s, 1)
    return d.energy(v, s, s_old) / e0


@pytest.mark.parametrize("k,ns", [(1, (16, 32, 64)), (2, (16, 32))])
def test_absorbing_sides_let_a_normal_pulse_out(k, ns):
    """At normal incidence the absorbing side (zero exterior state, upwind flux) is
    exactly transparent for the continuous problem, so the energy left behind is the
    discretisation's.  Upwind DG errors are of order h^(k+1/2) in amplitude, so that
    energy must shrink like h^(2k+1) under refinement (measured: P1 x7.0 and x8.8
    per halving, P2 x35); half an order of slack is allowed.  A reflecting side
    would leave energy of order one."""
    res = [_pulse_residual(n, k) for n in ns]
    print(f"P{k} residual energy after the pulse left: {res}")
    assert res[0] < 1e-5
    for a, b in zip(res, res[1:]):
        assert a / b >= 2.0 ** (2 * k + 0.5)
