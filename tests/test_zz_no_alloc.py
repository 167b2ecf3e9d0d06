"""GPU: the allocation-free energy entry point (dgt_energy_noalloc) against
dgt_energy and the FP64 oracle, on two calls in a row (the second on a smaller
mesh, so the shared per-GPU scratch holds the first call's larger contents), and
its size limit."""
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


def _case(D, n, k, prec, seed):
    m = I.square_mesh(n, jitter=0.2, renumber_seed=seed)
    lam, mu, rho = I.layered_material(m)
    om = O.OMesh.from_mesh(m)
    dt = O.cfl_dt(om, k, lam, mu, rho)
    od = O.ODG(om, k, lam, mu, rho, flux=0, order=4, dt=dt, free_sides=0xF)
    gd = D.Solver(D.Mesh.from_mesh(m), lam, mu, rho, degree=k, flux=0, time_order=4, precision=prec,
                  free_sides=0xF, dt=dt)
    v, s = od.zeros()
    v[:] = I.random_state(v.shape, seed)
    s[:] = I.random_state(s.shape, seed + 1)
    so = I.random_state(s.shape, seed + 2)
    return od, gd, v, s, so


@pytest.mark.parametrize("prec", [0, 1])
def test_energy_noalloc_equals_energy_on_two_calls(D, prec):
    dtype = torch.float32 if prec else torch.float64
    for n, k, seed in [(40, 2, 3), (9, 3, 7)]:  # the second call is smaller
        od, gd, v, s, so = _case(D, n, k, prec, seed)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda().contiguous()
        gv, gs, gso = t(v), t(s), t(so)
        e = gd.energy(gv, gs, gso)
        e0 = gd.energy(gv, gs, gso, noalloc=True)
        e_ref = od.energy(*(a.astype(np.float32).astype(np.float64) if prec else a for a in (v, s, so)))
        rel = abs(e0 - e_ref) / abs(e_ref)
        print(f"n={n} k={k} prec={prec}: noalloc {e0!r} alloc {e!r} oracle rel {rel:.3e}")
        assert e0 == e  # same kernels, same order
        assert rel <= (1e-5 if prec else 1e-12)  # an FP32 solver holds its geometry and material in FP32


def test_energy_noalloc_rejects_meshes_beyond_its_limit(D):
    m = I.square_mesh(1449)  # 4,199,202 cells > 2^22
    lam = np.full(m.nc, 2.0)
    one = np.ones(m.nc)
    gd = D.Solver(D.Mesh.from_mesh(m), lam, one, one, degree=1, flux=0, time_order=2, precision=1, free_sides=0xF,
                  dt=1e-4)
    v, s = gd.zeros()
    with pytest.raises(D.DgtError) as e:
        gd.energy(v, s, s, noalloc=True)
    assert e.value.status == D.DGT_EINVAL and "limit" in str(e.value)
