"""FP64 CPU oracle for the sparse-tiled DG elastic loop chain.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (``libdgtile`` and the
``paper_1708_03183_amd`` binding) imports or loads this package; the tests, the
smoke check and the benchmark's CPU-baseline leg do.  The C sources next to this
file hold the arithmetic; this module marshals NumPy arrays to them, apart from
the receiver sampling and misfit of full-waveform inversion (plain NumPy on top
of the C time step, at the end of this file).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRCS = ["refelem.c", "mesh.c", "dg.c", "chain.c", "oracle.h"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C11, -ffp-contract=off)."""
    if force or not os.path.exists(_LIB):
        subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)
    return _LIB


def _stale() -> bool:
    if not os.path.exists(_LIB):
        return True
    t = os.path.getmtime(_LIB)
    return any(os.path.getmtime(os.path.join(_HERE, s)) > t for s in _SRCS)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_p = C.c_void_p
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def _declare(L):
    L.or_np.restype = C.c_int
    L.or_refelem.argtypes = [C.c_int, _p, _p, _p, _p, _p, _p, _p]
    L.or_tri_quad.argtypes = [C.c_int, _f64p, _f64p]
    L.or_basis.argtypes = [C.c_int, C.c_double, C.c_double, _f64p]
    L.or_mesh_build.argtypes = [C.c_int64, _f64p, C.c_int64, _i32p, C.c_int, C.POINTER(_p)]
    L.or_mesh_free.argtypes = [_p]
    L.or_mesh_counts.argtypes = [_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.or_mesh_maps.argtypes = [_p, _i32p, _i8p, _i32p, _i8p, _i8p]
    L.or_dg_create.argtypes = [_p, C.c_int, _f64p, _f64p, _f64p, C.c_int, C.c_int, C.c_double, C.c_int,
                               C.POINTER(_p)]
    L.or_dg_free.argtypes = [_p]
    L.or_dg_set_source.argtypes = [_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]
    L.or_dg_source_cell.argtypes = [_p]
    L.or_dg_step.argtypes = [_p, _f64p, _f64p, C.c_int64, C.c_double]
    L.or_dg_step_tiled.argtypes = [_p, _p, _f64p, _f64p, C.c_int64, C.c_double]
    L.or_dg_energy.argtypes = [_p, _f64p, _f64p, _f64p]
    L.or_dg_energy.restype = C.c_double
    L.or_cfl_dt.argtypes = [_p, C.c_int, _f64p, _f64p, _f64p, C.c_double]
    L.or_cfl_dt.restype = C.c_double
    L.or_ricker.argtypes = [C.c_double] * 4
    L.or_ricker.restype = C.c_double
    L.or_dg_rate.argtypes = [_p, _f64p, _f64p, _f64p, _f64p]
    L.or_dg_chain.argtypes = [_p, C.POINTER(_p)]
    L.or_dg_chain_steps.argtypes = [_p, C.c_int, C.POINTER(_p)]
    L.or_chain_create.argtypes = [C.POINTER(_p)]
    L.or_chain_free.argtypes = [_p]
    L.or_chain_set.argtypes = [_p, C.c_int64]
    L.or_chain_map.argtypes = [_p, C.c_int, C.c_int, C.c_int, _i32p]
    L.or_chain_loop.argtypes = [_p, C.c_int, C.c_int, _i32p, _i32p, _i32p]
    L.or_chain_nloops.argtypes = [_p]
    L.or_chain_set_size.argtypes = [_p, C.c_int]
    L.or_chain_set_size.restype = C.c_int64
    L.or_chain_get_loop.argtypes = [_p, C.c_int, _i32p, _i32p, _i32p, _i32p]
    L.or_chain_get_map.argtypes = [_p, C.c_int, _i32p, _i32p, _i32p, _p]
    L.or_inspect.argtypes = [_p, C.c_int64, C.c_int, _p, C.c_int, C.c_int, _p, C.c_int, _p, C.POINTER(_p)]
    L.or_inspect_regions.argtypes = [_p, C.c_int64, C.c_int, _p, C.c_int, C.c_int, _p, C.c_int, _p, _p, C.c_int,
                                     C.POINTER(_p)]
    L.or_sched_regions.argtypes = [_p, C.c_int, _p, _p]
    L.or_sched_free.argtypes = [_p]
    L.or_sched_nsub.argtypes = [_p]
    L.or_sched_sub_info.argtypes = [_p, C.c_int] + [C.POINTER(C.c_int32)] * 5
    L.or_sched_tile_color.argtypes = [_p, C.c_int, _i32p]
    L.or_sched_sigma.argtypes = [_p, C.c_int, _i32p]
    L.or_sched_iters.argtypes = [_p, C.c_int, _i32p, _i32p]
    L.or_sched_footprint.argtypes = [_p, C.c_int, C.c_int, _p, _p, _p]
    L.or_sched_footprint.restype = C.c_int64
    L.or_sched_tiles_by_color.argtypes = [_p, C.c_int, _i32p, _i32p]
    L.or_sched_set_color.argtypes = [_p, C.c_int, C.c_int, C.c_int]
    L.or_sched_set_sigma.argtypes = [_p, C.c_int, C.c_int64, C.c_int]
    L.or_check.argtypes = [_p, _p]
    L.or_check.restype = C.c_int64
    L.or_tile_with_colors.argtypes = [_p, _i32p, C.c_int, _i32p, _p]
    L.or_projection_after.argtypes = [_p, _i32p, C.c_int, _i32p, C.c_int, C.c_int, _i32p]
    L.or_set_literal_projection.argtypes = [C.c_int]
    L.or_instrumented_run.argtypes = [_p, _p, C.c_int, C.POINTER(C.c_uint64)]


def set_literal_projection(on: bool):
    lib().or_set_literal_projection(1 if on else 0)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ----------------------------------------------------------------- element
def np_of(k: int) -> int:
    return (k + 1) * (k + 2) // 2


def refelem(k: int) -> dict:
    npk, nfp = np_of(k), k + 1
    out = dict(nodes=np.zeros((npk, 2)), M=np.zeros((npk, npk)), Minv=np.zeros((npk, npk)),
               Dr=np.zeros((npk, npk)), Ds=np.zeros((npk, npk)), M1=np.zeros((nfp, nfp)),
               fnodes=np.zeros((3, nfp), np.int32))
    rc = lib().or_refelem(k, *[_ptr(out[n]) for n in ("nodes", "M", "Minv", "Dr", "Ds", "M1", "fnodes")])
    if rc:
        raise ValueError(f"or_refelem({k}) -> {rc}")
    return out


def tri_quad(n: int):
    pts = np.zeros((n * n, 2))
    w = np.zeros(n * n)
    lib().or_tri_quad(n, pts, w)
    return pts, w


def basis(k: int, r: float, s: float) -> np.ndarray:
    phi = np.zeros(np_of(k))
    lib().or_basis(k, r, s, phi)
    return phi


def ricker(t, f0, t0, amp=1.0):
    return lib().or_ricker(t, f0, t0, amp)


# ----------------------------------------------------------------- mesh
class OMesh:
    def __init__(self, xy, c2v, periodic=0):
        self.xy = np.ascontiguousarray(xy, np.float64)
        self.c2v = np.ascontiguousarray(c2v, np.int32)
        h = C.c_void_p()
        rc = lib().or_mesh_build(self.xy.shape[0], self.xy, self.c2v.shape[0], self.c2v, int(periodic), C.byref(h))
        if rc:
            raise ValueError(f"invalid mesh ({rc})")
        self.h = h
        nc, nf, nb = C.c_int64(), C.c_int64(), C.c_int64()
        lib().or_mesh_counts(h, C.byref(nc), C.byref(nf), C.byref(nb))
        self.nc, self.nf, self.nb = nc.value, nf.value, nb.value

    @classmethod
    def from_mesh(cls, m):
        return cls(m.xy, m.c2v, m.periodic)

    def maps(self):
        f2c = np.zeros(2 * self.nf, np.int32)
        f2l = np.zeros(2 * self.nf, np.int8)
        b2c = np.zeros(self.nb, np.int32)
        b2l = np.zeros(self.nb, np.int8)
        bs = np.zeros(self.nb, np.int8)
        lib().or_mesh_maps(self.h, f2c, f2l, b2c, b2l, bs)
        return dict(f2c=f2c.reshape(-1, 2), f2l=f2l.reshape(-1, 2), b2c=b2c, b2l=b2l, bside=bs)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_mesh_free(self.h)
            self.h = None


def cfl_dt(om: OMesh, k, lam, mu, rho, cfl=0.2):
    return lib().or_cfl_dt(om.h, k, *[np.ascontiguousarray(a, np.float64) for a in (lam, mu, rho)], cfl)


# ----------------------------------------------------------------- DG chain
class ODG:
    """Oracle DG solver: state arrays v[2,Np,nc], s[3,Np,nc] (float64)."""

    def __init__(self, om: OMesh, k, lam, mu, rho, flux=0, order=4, dt=None, free_sides=0xF):
        self.om, self.k, self.np = om, k, np_of(k)
        self.lam, self.mu, self.rho = [np.ascontiguousarray(a, np.float64) for a in (lam, mu, rho)]
        if dt is None:
            dt = cfl_dt(om, k, self.lam, self.mu, self.rho)
        self.dt = dt
        h = C.c_void_p()
        rc = lib().or_dg_create(om.h, k, self.lam, self.mu, self.rho, flux, order, dt, free_sides, C.byref(h))
        if rc:
            raise ValueError(f"or_dg_create -> {rc}")
        self.h = h

    def zeros(self):
        return np.zeros((2, self.np, self.om.nc)), np.zeros((3, self.np, self.om.nc))

    def set_source(self, x, y, f0=5.0, t0=0.2, amp=1.0):
        if lib().or_dg_set_source(self.h, x, y, f0, t0, amp):
            raise ValueError("source outside the mesh")
        return lib().or_dg_source_cell(self.h)

    def step(self, v, s, nsteps, t0=0.0):
        lib().or_dg_step(self.h, v, s, nsteps, t0)

    def step_tiled(self, sched, v, s, nsteps, t0=0.0):
        rc = lib().or_dg_step_tiled(self.h, sched.h, v, s, nsteps, t0)
        if rc:
            raise ValueError(f"or_dg_step_tiled -> {rc}")

    def energy(self, v, s_new, s_old):
        return lib().or_dg_energy(self.h, v, s_new, s_old)

    def rate(self, v, s):
        dv, ds = np.zeros_like(v), np.zeros_like(s)
        lib().or_dg_rate(self.h, np.ascontiguousarray(v), np.ascontiguousarray(s), dv, ds)
        return dv, ds

    def chain(self, steps: int = 1) -> "OChain":
        """The loop chain of `steps` consecutive time steps."""
        h = C.c_void_p()
        if lib().or_dg_chain_steps(self.h, int(steps), C.byref(h)):
            raise ValueError("bad number of steps")
        return OChain(handle=h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_dg_free(self.h)
            self.h = None


# ----------------------------------------------------------------- loop chain
R, W, INC = 0, 1, 2


class OChain:
    def __init__(self, handle=None):
        if handle is None:
            handle = C.c_void_p()
            lib().or_chain_create(C.byref(handle))
        self.h = handle

    def set(self, size):
        return lib().or_chain_set(self.h, size)

    def map(self, frm, to, arity, values):
        v = np.ascontiguousarray(values, np.int32).ravel()
        rc = lib().or_chain_map(self.h, frm, to, arity, v)
        if rc < 0:
            raise ValueError("bad map")
        return rc

    def loop(self, set_id, descs):
        """descs: list of (map or -1, mode[, data])"""
        m = np.array([d[0] for d in descs], np.int32)
        mo = np.array([d[1] for d in descs], np.int32)
        da = np.array([d[2] if len(d) > 2 else -1 for d in descs], np.int32)
        rc = lib().or_chain_loop(self.h, set_id, len(descs), m, mo, da)
        if rc < 0:
            raise ValueError("bad loop")
        return rc

    @property
    def nloops(self):
        return lib().or_chain_nloops(self.h)

    def set_size(self, set_id):
        return int(lib().or_chain_set_size(self.h, set_id))

    def loop_info(self, j):
        """(set, [(map, mode), ...]) of loop j"""
        st, nd = np.zeros(1, np.int32), np.zeros(1, np.int32)
        mp, mo = np.zeros(8, np.int32), np.zeros(8, np.int32)
        if lib().or_chain_get_loop(self.h, j, st, nd, mp, mo) < 0:
            raise IndexError(j)
        return int(st[0]), [(int(mp[i]), int(mo[i])) for i in range(int(nd[0]))]

    def map_info(self, m):
        """(from, to, values [size(from), arity]) of map m"""
        fr, to, ar = np.zeros(1, np.int32), np.zeros(1, np.int32), np.zeros(1, np.int32)
        if lib().or_chain_get_map(self.h, m, fr, to, ar, None) < 0:
            raise IndexError(m)
        vals = np.zeros(max(self.set_size(int(fr[0])) * int(ar[0]), 1), np.int32)
        lib().or_chain_get_map(self.h, m, fr, to, ar, _ptr(vals))
        n = self.set_size(int(fr[0]))
        return int(fr[0]), int(to[0]), vals[: n * int(ar[0])].reshape(n, int(ar[0]))

    def inspect(self, ts, partition=0, seed_xy=None, max_rounds=64, splits=(), max_colour_tiles=0,
                sub_tile_sizes=None, seed_region=None, carry=1):
        """sub_tile_sizes: one seed tile size per sub-chain (len(splits) + 1), else ts for all.
        seed_region: per seed iteration 0 core, 1 boundary, 2 non-exec (or None); carry: one
        halo exchange for the whole chain (1) or one per sub-chain (0)."""
        xy = None if seed_xy is None else np.ascontiguousarray(seed_xy, np.float64)
        sp = np.ascontiguousarray(np.array(splits, np.int32))
        st = None
        if sub_tile_sizes is not None:
            st = np.ascontiguousarray(np.array(sub_tile_sizes, np.int32))
            assert st.size == len(sp) + 1
        h = C.c_void_p()
        if seed_region is None:
            rc = lib().or_inspect(self.h, ts, partition, _ptr(xy), max_rounds, max_colour_tiles,
                                  _ptr(sp) if len(sp) else None, len(sp), _ptr(st), C.byref(h))
        else:
            reg = np.ascontiguousarray(seed_region, np.uint8)
            rc = lib().or_inspect_regions(self.h, ts, partition, _ptr(xy), max_rounds, max_colour_tiles,
                                          _ptr(sp) if len(sp) else None, len(sp), _ptr(st), _ptr(reg),
                                          int(carry), C.byref(h))
        if rc:
            raise RuntimeError(f"or_inspect -> {rc}")
        return OSched(h, self)

    def sizes_of_loops(self, set_sizes):
        return [set_sizes[s] for s in self._loop_sets]

    def tile_with_colors(self, tile0, ntiles, color, loop_sizes):
        sig = [np.zeros(n, np.int32) for n in loop_sizes]
        arr = (C.c_void_p * len(sig))(*[a.ctypes.data for a in sig])
        lib().or_tile_with_colors(self.h, np.ascontiguousarray(tile0, np.int32), ntiles,
                                  np.ascontiguousarray(color, np.int32), C.cast(arr, C.c_void_p))
        return sig

    def projection_after(self, tile0, ntiles, color, upto, set_id, set_size):
        out = np.zeros(set_size, np.int32)
        lib().or_projection_after(self.h, np.ascontiguousarray(tile0, np.int32), ntiles,
                                  np.ascontiguousarray(color, np.int32), upto, set_id, out)
        return out

    def instrumented(self, sched=None, nrep=1):
        out = C.c_uint64()
        rc = lib().or_instrumented_run(self.h, None if sched is None else sched.h, nrep, C.byref(out))
        if rc:
            raise RuntimeError("instrumented run failed")
        return out.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_chain_free(self.h)
            self.h = None


class OSched:
    def __init__(self, h, chain):
        self.h, self.chain = h, chain

    @property
    def nsub(self):
        return lib().or_sched_nsub(self.h)

    def sub_info(self, sub):
        v = [C.c_int32() for _ in range(5)]
        lib().or_sched_sub_info(self.h, sub, *[C.byref(x) for x in v])
        return dict(first=v[0].value, nloops=v[1].value, ntiles=v[2].value, ncolors=v[3].value, rounds=v[4].value)

    def colors(self, sub):
        out = np.zeros(self.sub_info(sub)["ntiles"], np.int32)
        lib().or_sched_tile_color(self.h, sub, out)
        return out

    def sigma(self, loop, size):
        out = np.zeros(size, np.int32)
        lib().or_sched_sigma(self.h, loop, out)
        return out

    def iters(self, loop, size, sub):
        nt = self.sub_info(sub)["ntiles"]
        off = np.zeros(nt + 1, np.int32)
        it = np.zeros(size, np.int32)
        lib().or_sched_iters(self.h, loop, off, it)
        return off, it

    def footprint(self, sub, set_id):
        nt = self.sub_info(sub)["ntiles"]
        m = lib().or_sched_footprint(self.h, sub, set_id, None, None, None)
        off = np.zeros(nt + 1, np.int32)
        el = np.zeros(max(m, 0), np.int32)
        acc = np.zeros(max(m, 0), np.uint32)
        lib().or_sched_footprint(self.h, sub, set_id, _ptr(off), _ptr(el), _ptr(acc))
        return off, el, acc

    def tiles_by_color(self, sub):
        info = self.sub_info(sub)
        coff = np.zeros(info["ncolors"] + 1, np.int32)
        tl = np.zeros(info["ntiles"], np.int32)
        lib().or_sched_tiles_by_color(self.h, sub, coff, tl)
        return coff, tl

    def regions(self, sub, seed_size):
        """(core tiles, boundary tiles, T_ne id, T_ne colour), seed regions of the sub-chain;
        None without regions."""
        info = np.zeros(4, np.int32)
        reg = np.zeros(max(seed_size, 1), np.uint8)
        if lib().or_sched_regions(self.h, sub, _ptr(info), _ptr(reg)) < 0:
            return None
        return tuple(int(x) for x in info), reg[:seed_size]

    def set_color(self, sub, tile, color):
        lib().or_sched_set_color(self.h, sub, tile, color)

    def set_sigma(self, loop, it, tile):
        lib().or_sched_set_sigma(self.h, loop, it, tile)

    def check(self):
        return lib().or_check(self.chain.h, self.h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_sched_free(self.h)
            self.h = None


# ----------------------------------------------------------------- FWI misfit
# (the paper runs the forward chain only; these helpers define the receiver
# sampling and the misfit whose gradient the library's adjoint computes)

def locate(om: OMesh, x, y):
    """Lowest-id cell containing (x, y), within 1e-12 in the reference coordinates
    (r, s) of the affine map from the cell's first vertex, and those coordinates."""
    p = om.xy[om.c2v]
    xr, xs = p[:, 1, 0] - p[:, 0, 0], p[:, 2, 0] - p[:, 0, 0]
    yr, ys = p[:, 1, 1] - p[:, 0, 1], p[:, 2, 1] - p[:, 0, 1]
    det = xr * ys - xs * yr
    r = (ys * (x - p[:, 0, 0]) - xs * (y - p[:, 0, 1])) / det
    s = (-yr * (x - p[:, 0, 0]) + xr * (y - p[:, 0, 1])) / det
    inside = np.flatnonzero((r >= -1e-12) & (s >= -1e-12) & (1.0 - r - s >= -1e-12))
    if not len(inside):
        raise ValueError("point outside the mesh")
    c = int(inside[0])
    return c, float(r[c]), float(s[c])


def fwi_traces(od: ODG, rec_xy, shots_xy, nsteps, f0=5.0, t0=0.2, amp=1.0):
    """Velocity traces [nshots, nsteps, nrec, 2]: each shot runs from rest with its
    Ricker source; after step n receiver r reads sum_i phi_i(x_r) v_i of its cell."""
    rec = [locate(od.om, x, y) for x, y in np.asarray(rec_xy, np.float64).reshape(-1, 2)]
    phis = [basis(od.k, r, s) for _, r, s in rec]
    shots = np.asarray(shots_xy, np.float64).reshape(-1, 2)
    out = np.zeros((len(shots), nsteps, len(rec), 2))
    for q, (x, y) in enumerate(shots):
        od.set_source(x, y, f0, t0, amp)
        v, s = od.zeros()
        for n in range(nsteps):
            od.step(v, s, 1, t0=n * od.dt)
            for k, ((c, _, _), phi) in enumerate(zip(rec, phis)):
                out[q, n, k] = v[:, :, c] @ phi
    return out


def fwi_misfit(od: ODG, rec_xy, shots_xy, nsteps, observed, f0=5.0, t0=0.2, amp=1.0):
    """J = 1/2 sum over shots, steps, receivers and components of (r - d)^2."""
    r = fwi_traces(od, rec_xy, shots_xy, nsteps, f0, t0, amp)
    return 0.5 * float(((r - observed) ** 2).sum())



def fwi_gradient_fd(make, lam, mu, rho, rec_xy, shots_xy, nsteps, observed, f0=5.0, t0=0.2, amp=1.0, h=1e-3):
    """The misfit's gradient with respect to each cell's lam, mu, rho by its definition:
    central differences of J in one parameter at a time (relative steps h and h/2),
    Richardson-extrapolated (truncation error O(h^4)).  make(lam, mu, rho) -> ODG with a
    fixed time step.  Any flux and boundaries; slow (4 misfits per parameter)."""
    base = [np.array(lam, np.float64), np.array(mu, np.float64), np.array(rho, np.float64)]
    nc = base[0].size
    g = np.zeros((3, nc))

    def J(p, c, eps):
        m = [x.copy() for x in base]
        m[p][c] *= 1.0 + eps
        return fwi_misfit(make(*m), rec_xy, shots_xy, nsteps, observed, f0, t0, amp)

    for p in range(3):
        for c in range(nc):
            step = h * base[p][c]
            d1 = (J(p, c, h) - J(p, c, -h)) / (2.0 * step)
            d2 = (J(p, c, 0.5 * h) - J(p, c, -0.5 * h)) / step
            g[p, c] = (4.0 * d2 - d1) / 3.0
    return g


def fwi_gradient_adjoint(od: ODG, od_rev: ODG, order, rec_xy, shots_xy, nsteps, observed, f0=5.0, t0=0.2, amp=1.0):
    """Misfit and its gradient (g_lam, g_mu, g_rho per cell) by the discrete adjoint,
    storing every forward state.  Valid for the central flux with free-surface or
    periodic boundaries, where the transpose of a step is T^-1 Phi(-dt) T with
    T = blockdiag(M_J^-1 / rho, M_J^-1 C) per cell; od_rev is the same solver built
    with -dt.  A = velocity operator, B = stress operator (od.rate with the other
    field zero); per step, with alpha the adjoint in T-variables,
      g_rho -= |J| [(dt av + c A B av) . M^ (A s_n) + av . M^ (c A B A s_n)
                    - c (A as) . M^ (A B v')]
      g_lam += |J| [(dt as + c B A as) . (M^ x S_lam) (B v') + as . (M^ x S_lam) (c B A B v')
                    - c (B av) . (M^ x S_lam) (B A s_n)]
    with av the velocity part of alpha after the reversed step, as its stress part
    before it, v' the velocity after the step, c = dt^3/24 (0 at order 2),
    S_m = C^-1 (dC/dm) C^-1."""
    om, k = od.om, od.k
    npk, nc, dt = od.np, om.nc, od.dt
    c3 = dt ** 3 / 24.0 if order == 4 else 0.0
    R = refelem(k)
    M, Minv = R["M"], R["Minv"]
    p = om.xy[om.c2v]
    det = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    lam, mu, rho = od.lam, od.mu, od.rho
    cA, cB, cC = (lam + 2 * mu) / (4 * mu * (lam + mu)), -lam / (4 * mu * (lam + mu)), 1.0 / mu
    rec = [locate(om, x, y) for x, y in np.asarray(rec_xy, np.float64).reshape(-1, 2)]
    phis = [basis(k, r, s) for _, r, s in rec]
    zv, zs = od.zeros()

    def A(s):
        return od.rate(zv, s)[0]

    def B(v):
        return od.rate(v, zs)[1]

    def cinv(x):  # C^-1 on (xx, yy, xy) per node
        return np.stack([cA * x[0] + cB * x[1], cB * x[0] + cA * x[1], cC * x[2]])

    def mdot(a, b):  # per cell: sum_ij a_i M_ij b_j
        return np.einsum("in,ij,jn->n", a, M, b)

    shots = np.asarray(shots_xy, np.float64).reshape(-1, 2)
    g = np.zeros((3, nc))
    J = 0.0
    for q, (x, y) in enumerate(shots):
        od.set_source(x, y, f0, t0, amp)
        v, s = od.zeros()
        states = [(v.copy(), s.copy())]
        for n in range(nsteps):
            od.step(v, s, 1, t0=n * dt)
            states.append((v.copy(), s.copy()))

        def residual(n):  # observation after step n - 1, from state n
            vn = states[n][0]
            return [vn[:, :, c] @ phi - observed[q, n - 1, kk] for kk, ((c, _, _), phi) in enumerate(zip(rec, phis))]

        def inject(av, res):
            for (c, _, _), phi, r in zip(rec, phis, res):
                av[:, :, c] += np.outer(r, Minv @ phi) / (rho[c] * det[c])

        for n in range(1, nsteps + 1):
            J += 0.5 * sum(float(r @ r) for r in residual(n))
        av, as_ = od.zeros()
        inject(av, residual(nsteps))
        for n in range(nsteps - 1, -1, -1):
            v0, s0 = states[n]
            v1 = states[n + 1][0]
            U = A(s0)
            X1 = B(v1)
            Z = c3 * A(B(U)) if order == 4 else None
            V2 = c3 * B(A(X1)) if order == 4 else None
            as_before = as_.copy()
            od_rev.step(av, as_, 1, t0=0.0)
            def lm(b, e):  # (b . (M^ x S_lam) e, b . (M^ x S_mu) e) with b, e already through C^-1
                return (mdot(b[0] + b[1], e[0] + e[1]),
                        2 * (mdot(b[0], e[0]) + mdot(b[1], e[1])) + mdot(b[2], e[2]))

            a = dt * av + (c3 * A(B(av)) if order == 4 else 0.0)
            gr = sum(mdot(a[c], U[c]) for c in range(2))
            P = dt * as_before + (c3 * B(A(as_before)) if order == 4 else 0.0)
            gl, gm = lm(cinv(P), cinv(X1))
            if order == 4:
                # the velocity half's c A B A holds C, the stress half's c B A B holds 1/rho
                gr = gr + sum(mdot(av[c], Z[c]) for c in range(2))
                Ya = A(as_before)
                gr = gr - c3 * sum(mdot(Ya[c], A(X1)[c]) for c in range(2))
                l2, m2 = lm(cinv(as_before), cinv(V2))
                l3, m3 = lm(cinv(B(av)), cinv(B(U)))
                gl, gm = gl + l2 - c3 * l3, gm + m2 - c3 * m3
            g[0] += det * gl
            g[1] += det * gm
            g[2] -= det * gr
            if n >= 1:
                inject(av, residual(n))
    return J, g
