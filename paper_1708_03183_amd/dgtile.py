"""Python binding of libdgtile (ctypes; argument marshalling only).

Every step of the hot path runs in the HIP kernels of ``libdgtile.so``.  PyTorch
is used only for device memory (state tensors) and the current HIP stream.  The
names mirror the C ABI in ``include/dgtile.h``.  Loading fails loudly when the
library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgtile.so")

DGT_OK, DGT_EINVAL, DGT_ENOMEM, DGT_EHIP, DGT_ESTATE, DGT_EUNSUPPORTED = range(6)
R, W, INC = 0, 1, 2


class DgtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libdgtile status {status}: {msg}")
        self.status = status


class _AutotuneParams(C.Structure):
    _fields_ = [("tile_sizes", C.c_void_p), ("ntile_sizes", C.c_int32), ("splits", C.c_void_p),
                ("nsplits", C.c_int32), ("partition", C.c_int32), ("trial_steps", C.c_int32),
                ("prune", C.c_double)]


class _FwiParams(C.Structure):
    _fields_ = [("nrec", C.c_int32), ("rec_xy", C.c_void_p), ("nsteps", C.c_int64), ("nsnap", C.c_int32),
                ("mode", C.c_int32)]


class _AutotuneResult(C.Structure):
    _fields_ = [("tile_size", C.c_int32), ("schedule", C.c_int32), ("ms_per_step", C.c_double),
                ("timed", C.c_int32), ("skipped", C.c_int32)]


class _Desc(C.Structure):
    _fields_ = [("map", C.c_int32), ("mode", C.c_int32), ("data", C.c_int32)]


class _InspectParams(C.Structure):
    _fields_ = [("tile_size", C.c_int64), ("partition", C.c_int32), ("seed_xy", C.c_void_p),
                ("max_conflict_rounds", C.c_int32), ("splits", C.c_void_p), ("nsplits", C.c_int32),
                ("max_colour_tiles", C.c_int32), ("sub_tile_sizes", C.c_void_p), ("seed_region", C.c_void_p),
                ("region_carry", C.c_int32)]


class _SolverParams(C.Structure):
    _fields_ = [("degree", C.c_int32), ("flux", C.c_int32), ("time_order", C.c_int32),
                ("precision", C.c_int32), ("free_sides", C.c_int32), ("dt", C.c_double)]


_lib = None
_p = C.c_void_p
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)

# symbol -> argtypes (every function returns dgt_status unless listed in _VOID)
_SIGS = {
    "dgt_chain_create": [C.POINTER(_p)],
    "dgt_chain_set": [_p, C.c_int64, _i32],
    "dgt_chain_map": [_p, C.c_int32, C.c_int32, C.c_int32, _p, _i32],
    "dgt_chain_loop": [_p, C.c_int32, C.c_int32, C.POINTER(_Desc), _i32],
    "dgt_chain_destroy": [_p],
    "dgt_inspect": [_p, C.POINTER(_InspectParams), _p, C.POINTER(_p)],
    "dgt_schedule_nsub": [_p, _i32],
    "dgt_schedule_sub_info": [_p, C.c_int32, _i32, _i32, _i32, _i32, _i32],
    "dgt_schedule_colors": [_p, C.c_int32, _p],
    "dgt_schedule_sigma": [_p, C.c_int32, _p],
    "dgt_schedule_iters": [_p, C.c_int32, _p, _p],
    "dgt_schedule_footprint": [_p, C.c_int32, C.c_int32, _i64, _p, _p, _p],
    "dgt_schedule_tiles_by_color": [_p, C.c_int32, _p, _p],
    "dgt_schedule_regions": [_p, C.c_int32, _p, _p],
    "dgt_schedule_summary_json": [_p, C.c_char_p, C.c_size_t],
    "dgt_schedule_destroy": [_p],
    "dgt_mesh_create": [C.c_int64, _p, C.c_int64, _p, C.c_int32, C.POINTER(_p)],
    "dgt_mesh_counts": [_p, _i64, _i64, _i64],
    "dgt_mesh_maps": [_p, _p, _p, _p, _p, _p],
    "dgt_mesh_destroy": [_p],
    "dgt_solver_create": [_p, _p, _p, _p, C.POINTER(_SolverParams), _p, C.POINTER(_p)],
    "dgt_solver_inspect": [_p, C.POINTER(_InspectParams)],
    "dgt_solver_fuse_steps": [_p, C.c_int32],
    "dgt_solver_schedule": [_p, C.POINTER(_p)],
    "dgt_set_source": [_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double],
    "dgt_solver_set_shots": [_p, C.c_int32, _p, C.c_double, C.c_double, C.c_double],
    "dgt_solver_autotune": [_p, _p, _p],
    "dgt_fwi_forward": [_p, _p, _p],
    "dgt_fwi_gradient": [_p, _p, _p, _p, _p, _p, _p],
    "dgt_state_upload": [_p, _p, _p],
    "dgt_state_download": [_p, _p, _p],
    "dgt_cell_list_create": [_p, C.c_int64, _p, C.POINTER(_p)],
    "dgt_cell_list_destroy": [_p],
    "dgt_state_pack": [_p, _p, _p, _p],
    "dgt_state_unpack": [_p, _p, _p, _p],
    "dgt_step": [_p, C.c_int64, C.c_int32, C.c_double],
    "dgt_energy": [_p, _p, _p, _p, C.POINTER(C.c_double)],
    "dgt_energy_noalloc": [_p, _p, _p, _p, C.POINTER(C.c_double)],
    "dgt_last_step_timing": [_p, C.POINTER(C.c_double), C.POINTER(C.c_double), _i64],
    "dgt_solver_profile": [_p, C.c_int32],
    "dgt_solver_set_schedule": [_p, C.c_int32],
    "dgt_solver_set_wait_limit": [_p, C.c_int64],
    "dgt_solver_info": [_p, _i64, _i64, _i64],
    "dgt_solver_destroy": [_p],
    "dgt_refelem": [C.c_int32, _p, _p, _p, _p],
    "dgt_solver_kernels": [_p, _i32, _p],
    "dgt_batch_create": [_p, C.c_int32, _p, C.POINTER(_p)],
    "dgt_batch_set_graph": [_p, C.c_int32],
    "dgt_batch_set_schedule": [_p, C.c_int32],
    "dgt_batch_step": [_p, C.c_int64, _p],
    "dgt_batch_timing": [_p, C.POINTER(C.c_double), _i64, _i64],
    "dgt_batch_destroy": [_p],
    "dgt_last_error": [],
    "dgt_version": [],
}
_VOID = {"dgt_chain_destroy", "dgt_schedule_destroy", "dgt_mesh_destroy", "dgt_solver_destroy", "dgt_batch_destroy",
         "dgt_cell_list_destroy"}


def exported_symbols() -> list[str]:
    return sorted(_SIGS)


def lib():
    """Load libdgtile.so (built by ``build()``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1708_03183_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            if name in _VOID:
                f.restype = None
            elif name == "dgt_last_error":
                f.restype = C.c_char_p
            else:
                f.restype = C.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != DGT_OK:
        raise DgtError(st, lib().dgt_last_error().decode())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _inspect_params(tile_size, partition, seed_xy, max_rounds, splits, max_colour_tiles=0, sub_tile_sizes=None,
                    seed_region=None, region_carry=1):
    sp = np.ascontiguousarray(np.array(list(splits), np.int32))
    reg = None if seed_region is None else np.ascontiguousarray(seed_region, np.uint8)
    xy = None if seed_xy is None else np.ascontiguousarray(seed_xy, np.float64)
    st = None
    if sub_tile_sizes is not None:
        st = np.ascontiguousarray(np.array(list(sub_tile_sizes), np.int32))
        if st.size != len(sp) + 1:
            raise ValueError("sub_tile_sizes needs one tile size per sub-chain (len(splits) + 1)")
    p = _InspectParams(int(tile_size), int(partition), _np_ptr(xy), int(max_rounds),
                       _np_ptr(sp) if len(sp) else None, len(sp), int(max_colour_tiles), _np_ptr(st), _np_ptr(reg),
                       int(region_carry))
    return p, (sp, xy, st, reg)


# --------------------------------------------------------------- tier 1
def refelem(degree: int) -> dict:
    """Host copies of the reference-element tables the degree-k kernels use."""
    npn = (degree + 1) * (degree + 2) // 2
    t = {n: np.zeros((npn, npn)) for n in ("Dr", "Ds", "Minv")}
    t["lift"] = np.zeros((3, npn, degree + 1))
    _check(lib().dgt_refelem(degree, _np_ptr(t["Dr"]), _np_ptr(t["Ds"]), _np_ptr(t["Minv"]), _np_ptr(t["lift"])))
    return t


class Chain:
    """Generic loop chain (sets, maps, loops with descriptors)."""

    def __init__(self):
        h = C.c_void_p()
        _check(lib().dgt_chain_create(C.byref(h)))
        self.h = h
        self.sizes = []
        self.loop_sets = []

    def set(self, size: int) -> int:
        out = C.c_int32()
        _check(lib().dgt_chain_set(self.h, int(size), C.byref(out)))
        self.sizes.append(int(size))
        return out.value

    def map(self, frm: int, to: int, arity: int, values) -> int:
        v = np.ascontiguousarray(values, np.int32).ravel()
        out = C.c_int32()
        _check(lib().dgt_chain_map(self.h, frm, to, arity, _np_ptr(v), C.byref(out)))
        return out.value

    def loop(self, set_id: int, descs) -> int:
        arr = (_Desc * max(len(descs), 1))(*[_Desc(d[0], d[1], d[2] if len(d) > 2 else -1) for d in descs])
        out = C.c_int32()
        _check(lib().dgt_chain_loop(self.h, set_id, len(descs), arr, C.byref(out)))
        self.loop_sets.append(set_id)
        return out.value

    def inspect(self, tile_size, partition=0, seed_xy=None, max_rounds=64, splits=(), stream=None,
                max_colour_tiles=0, sub_tile_sizes=None, seed_region=None, region_carry=1) -> "Schedule":
        p, keep = _inspect_params(tile_size, partition, seed_xy, max_rounds, splits, max_colour_tiles, sub_tile_sizes,
                                  seed_region, region_carry)
        h = C.c_void_p()
        _check(lib().dgt_inspect(self.h, C.byref(p), _stream_handle(stream), C.byref(h)))
        return Schedule(h, owner=True, loop_sizes=[self.sizes[s] for s in self.loop_sets])

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dgt_chain_destroy(self.h)
            self.h = None


class Schedule:
    """Read-back view of an inspector schedule (host copies)."""

    def __init__(self, h, owner: bool, loop_sizes):
        self.h, self.owner, self.loop_sizes = h, owner, loop_sizes

    @property
    def nsub(self) -> int:
        n = C.c_int32()
        _check(lib().dgt_schedule_nsub(self.h, C.byref(n)))
        return n.value

    def sub_info(self, sub: int) -> dict:
        v = [C.c_int32() for _ in range(5)]
        _check(lib().dgt_schedule_sub_info(self.h, sub, *[C.byref(x) for x in v]))
        return dict(first=v[0].value, nloops=v[1].value, ntiles=v[2].value, ncolors=v[3].value, rounds=v[4].value)

    def colors(self, sub: int) -> np.ndarray:
        out = np.zeros(self.sub_info(sub)["ntiles"], np.int32)
        _check(lib().dgt_schedule_colors(self.h, sub, _np_ptr(out)))
        return out

    def sigma(self, loop: int) -> np.ndarray:
        out = np.zeros(self.loop_sizes[loop], np.int32)
        _check(lib().dgt_schedule_sigma(self.h, loop, _np_ptr(out)))
        return out

    def iters(self, loop: int, sub: int):
        off = np.zeros(self.sub_info(sub)["ntiles"] + 1, np.int32)
        it = np.zeros(self.loop_sizes[loop], np.int32)
        _check(lib().dgt_schedule_iters(self.h, loop, _np_ptr(off), _np_ptr(it)))
        return off, it

    def footprint(self, sub: int, set_id: int):
        n = C.c_int64()
        _check(lib().dgt_schedule_footprint(self.h, sub, set_id, C.byref(n), None, None, None))
        off = np.zeros(self.sub_info(sub)["ntiles"] + 1, np.int32)
        el = np.zeros(n.value, np.int32)
        acc = np.zeros(n.value, np.uint32)
        _check(lib().dgt_schedule_footprint(self.h, sub, set_id, C.byref(n), _np_ptr(off), _np_ptr(el), _np_ptr(acc)))
        return off, el, acc

    def tiles_by_color(self, sub: int):
        info = self.sub_info(sub)
        coff = np.zeros(info["ncolors"] + 1, np.int32)
        tl = np.zeros(info["ntiles"], np.int32)
        _check(lib().dgt_schedule_tiles_by_color(self.h, sub, _np_ptr(coff), _np_ptr(tl)))
        return coff, tl

    def regions(self, sub: int, seed_size: int):
        """((core tiles, boundary tiles, T_ne id, T_ne colour), seed regions) of a region-aware
        schedule."""
        info = np.zeros(4, np.int32)
        reg = np.zeros(max(seed_size, 1), np.uint8)
        _check(lib().dgt_schedule_regions(self.h, sub, _np_ptr(info), _np_ptr(reg)))
        return tuple(int(x) for x in info), reg[:seed_size]

    def summary(self) -> str:
        buf = C.create_string_buffer(1 << 16)
        _check(lib().dgt_schedule_summary_json(self.h, buf, len(buf)))
        return buf.value.decode()

    def __del__(self):
        if getattr(self, "owner", False) and getattr(self, "h", None) and _lib is not None:
            _lib.dgt_schedule_destroy(self.h)
            self.h = None


# --------------------------------------------------------------- tier 2
class Mesh:
    def __init__(self, xy, c2v, periodic: int = 0):
        self.xy = np.ascontiguousarray(xy, np.float64)
        self.c2v = np.ascontiguousarray(c2v, np.int32)
        h = C.c_void_p()
        _check(lib().dgt_mesh_create(self.xy.shape[0], _np_ptr(self.xy), self.c2v.shape[0], _np_ptr(self.c2v),
                                     int(periodic), C.byref(h)))
        self.h = h
        nc, nf, nb = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().dgt_mesh_counts(h, C.byref(nc), C.byref(nf), C.byref(nb)))
        self.nc, self.nf, self.nb = nc.value, nf.value, nb.value

    @classmethod
    def from_mesh(cls, m):
        return cls(m.xy, m.c2v, m.periodic)

    def maps(self) -> dict:
        f2c = np.zeros(2 * self.nf, np.int32)
        f2l = np.zeros(2 * self.nf, np.int8)
        b2c = np.zeros(self.nb, np.int32)
        b2l = np.zeros(self.nb, np.int8)
        bs = np.zeros(self.nb, np.int8)
        _check(lib().dgt_mesh_maps(self.h, *[_np_ptr(a) for a in (f2c, f2l, b2c, b2l, bs)]))
        return dict(f2c=f2c.reshape(-1, 2), f2l=f2l.reshape(-1, 2), b2c=b2c, b2l=b2l, bside=bs)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dgt_mesh_destroy(self.h)
            self.h = None


class Solver:
    """DG velocity-stress solver; state tensors v[2,Np,nc], s[3,Np,nc] on the GPU
    (v[S,2,Np,nc], s[S,3,Np,nc] with S > 1 shots)."""

    def __init__(self, mesh: Mesh, lam, mu, rho, degree=2, flux=1, time_order=4, precision=0,
                 free_sides=0xF, dt=None, stream=None):
        if dt is None:
            raise ValueError("dt is required")
        self.mesh = mesh
        self.degree, self.precision, self._time_order = degree, precision, time_order
        self.np = (degree + 1) * (degree + 2) // 2
        self._mat = [np.ascontiguousarray(a, np.float64) for a in (lam, mu, rho)]
        prm = _SolverParams(degree, flux, time_order, precision, free_sides, float(dt))
        self.dt = float(dt)
        h = C.c_void_p()
        _check(lib().dgt_solver_create(mesh.h, *[_np_ptr(a) for a in self._mat], C.byref(prm),
                                       _stream_handle(stream), C.byref(h)))
        self.h = h
        self.nshots = 1

    @property
    def dtype(self):
        import torch
        return torch.float32 if self.precision == 1 else torch.float64

    def _shape(self, comps):
        return (comps, self.np, self.mesh.nc) if self.nshots == 1 else (self.nshots, comps, self.np, self.mesh.nc)

    def zeros(self, device="cuda"):
        import torch
        return (torch.zeros(self._shape(2), dtype=self.dtype, device=device),
                torch.zeros(self._shape(3), dtype=self.dtype, device=device))

    def inspect(self, tile_size, partition=1, max_rounds=64, splits=(), max_colour_tiles=0, sub_tile_sizes=None,
                seed_region=None, region_carry=1):
        """max_colour_tiles: 0 none, > 0 cap per colour class, -1 the GPU's resident tile count;
        sub_tile_sizes: one seed tile size per sub-chain (else tile_size for all); seed_region:
        per cell 0 core, 1 boundary, 2 non-exec for one part of a distributed mesh."""
        p, keep = _inspect_params(tile_size, partition, None, max_rounds, splits, max_colour_tiles, sub_tile_sizes,
                                  seed_region, region_carry)
        _check(lib().dgt_solver_inspect(self.h, C.byref(p)))

    def autotune(self, tile_sizes=(64, 96, 128, 192, 256, 384, 512), splits=(), partition=1, trial_steps=5,
                 prune=0.0) -> dict:
        """Pick the seed tile size and schedule by timing trial steps; the solver is left
        inspected and scheduled with the fastest pair."""
        ts = np.ascontiguousarray(tile_sizes, np.int32)
        sp = np.ascontiguousarray(splits, np.int32)
        p = _AutotuneParams(_np_ptr(ts), len(ts), _np_ptr(sp) if len(sp) else None, len(sp), int(partition),
                            int(trial_steps), float(prune))
        r = _AutotuneResult()
        _check(lib().dgt_solver_autotune(self.h, C.byref(p), C.byref(r)))
        return dict(tile_size=r.tile_size, schedule=r.schedule, ms_per_step=r.ms_per_step, timed=r.timed,
                    skipped=r.skipped)

    def _fwi_params(self, rec_xy, nsteps, nsnap, mode):
        xy = np.ascontiguousarray(rec_xy, np.float64).reshape(-1)
        assert xy.size >= 2 and xy.size % 2 == 0
        return _FwiParams(xy.size // 2, _np_ptr(xy), int(nsteps), int(nsnap), int(mode)), xy

    def fwi_forward(self, rec_xy, nsteps: int, mode: int = 1):
        """Receiver traces [nshots, nsteps, nrec, 2] (FP64, on the GPU) of a run from rest."""
        import torch
        p, keep = self._fwi_params(rec_xy, nsteps, 1, mode)
        out = torch.empty((self.nshots, int(nsteps), p.nrec, 2), dtype=torch.float64, device="cuda")
        _check(lib().dgt_fwi_forward(self.h, C.byref(p), C.c_void_p(out.data_ptr())))
        return out

    def fwi_gradient(self, rec_xy, nsteps: int, observed, nsnap: int = 32, mode: int = 1):
        """Misfit 1/2 sum |r - d|^2 and its gradient w.r.t. per-cell lambda, mu, rho
        (FP64 tensors [nc] on the GPU, mesh numbering)."""
        import torch
        p, keep = self._fwi_params(rec_xy, nsteps, nsnap, mode)
        assert observed.dtype == torch.float64 and observed.is_cuda and observed.is_contiguous()
        assert tuple(observed.shape) == (self.nshots, int(nsteps), p.nrec, 2)
        g = torch.zeros((3, self.mesh.nc), dtype=torch.float64, device="cuda")
        J = C.c_double()
        _check(lib().dgt_fwi_gradient(self.h, C.byref(p), C.c_void_p(observed.data_ptr()), C.byref(J),
                                      C.c_void_p(g[0].data_ptr()), C.c_void_p(g[1].data_ptr()),
                                      C.c_void_p(g[2].data_ptr())))
        return J.value, g[0], g[1], g[2]

    def schedule(self) -> Schedule:
        h = C.c_void_p()
        _check(lib().dgt_solver_schedule(self.h, C.byref(h)))
        m = self.mesh
        sizes = {0: m.nc, 1: m.nf, 2: m.nb}
        nl = 26 if self._order() == 4 else 8
        pat = (([0, 1, 2, 0] * 3 + [0]) * 2 if nl == 26 else [0, 1, 2, 0] * 2) * getattr(self, "_fuse", 1)
        return Schedule(h, owner=False, loop_sizes=[sizes[s] for s in pat])

    def _order(self):
        return self._time_order

    def set_source(self, x, y, f0=5.0, t0=0.2, amp=1.0):
        _check(lib().dgt_set_source(self.h, x, y, f0, t0, amp))

    def set_shots(self, nshots: int, xy=None, f0=5.0, t0=0.2, amp=1.0):
        """nshots independent states on this mesh, shot q with a Ricker source at xy[q]
        (or none); the state is reset to zero."""
        keep = None
        if xy is not None:
            keep = np.ascontiguousarray(xy, np.float64).reshape(-1)
            assert keep.size == 2 * nshots
        _check(lib().dgt_solver_set_shots(self.h, int(nshots), None if keep is None else _np_ptr(keep),
                                          float(f0), float(t0), float(amp)))
        self.nshots = int(nshots)

    def upload(self, v, s):
        assert v.dtype == self.dtype and s.dtype == self.dtype and v.is_contiguous() and s.is_contiguous()
        assert tuple(v.shape) == self._shape(2) and tuple(s.shape) == self._shape(3)
        _check(lib().dgt_state_upload(self.h, C.c_void_p(v.data_ptr()), C.c_void_p(s.data_ptr())))

    def download(self, v, s):
        assert v.dtype == self.dtype and s.dtype == self.dtype and v.is_contiguous() and s.is_contiguous()
        assert tuple(v.shape) == self._shape(2) and tuple(s.shape) == self._shape(3)
        _check(lib().dgt_state_download(self.h, C.c_void_p(v.data_ptr()), C.c_void_p(s.data_ptr())))

    def step(self, nsteps: int, mode: int = 1, t0: float = 0.0):
        _check(lib().dgt_step(self.h, int(nsteps), int(mode), float(t0)))

    def fuse_steps(self, steps: int):
        """Hand the inspector a chain of `steps` consecutive time steps (inspect again after)."""
        _check(lib().dgt_solver_fuse_steps(self.h, int(steps)))
        self._fuse = int(steps)

    def cell_list(self, cells) -> "CellList":
        return CellList(self, cells)

    def _halo_shape(self, comps, n):
        return (comps, self.np, n) if self.nshots == 1 else (self.nshots, comps, self.np, n)

    def pack(self, cl: "CellList", v, s):
        """State of the listed cells into packed buffers v[.., 2, Np, n], s[.., 3, Np, n]."""
        assert v.dtype == self.dtype and s.dtype == self.dtype and v.is_contiguous() and s.is_contiguous()
        assert tuple(v.shape) == self._halo_shape(2, cl.n) and tuple(s.shape) == self._halo_shape(3, cl.n)
        _check(lib().dgt_state_pack(self.h, cl.h, C.c_void_p(v.data_ptr()), C.c_void_p(s.data_ptr())))

    def unpack(self, cl: "CellList", v, s):
        """Packed buffers into the state of the listed cells (a halo receive)."""
        assert v.dtype == self.dtype and s.dtype == self.dtype and v.is_contiguous() and s.is_contiguous()
        assert tuple(v.shape) == self._halo_shape(2, cl.n) and tuple(s.shape) == self._halo_shape(3, cl.n)
        _check(lib().dgt_state_unpack(self.h, cl.h, C.c_void_p(v.data_ptr()), C.c_void_p(s.data_ptr())))

    def energy(self, v, s_new, s_old, noalloc: bool = False) -> float:
        """Energy of one shot's state (tensors of one shot, contiguous);
        noalloc selects dgt_energy_noalloc."""
        assert tuple(v.shape) == (2, self.np, self.mesh.nc) and v.is_contiguous()
        assert tuple(s_new.shape) == (3, self.np, self.mesh.nc) and s_new.is_contiguous()
        assert tuple(s_old.shape) == (3, self.np, self.mesh.nc) and s_old.is_contiguous()
        out = C.c_double()
        fn = lib().dgt_energy_noalloc if noalloc else lib().dgt_energy
        _check(fn(self.h, C.c_void_p(v.data_ptr()), C.c_void_p(s_new.data_ptr()), C.c_void_p(s_old.data_ptr()),
                  C.byref(out)))
        return out.value

    def kernels(self) -> list:
        """Tile kernel per sub-chain: 0 generic, 1 register-resident chain, 2 matrix-core,
        3 generic with the working set in global memory."""
        n = C.c_int32()
        _check(lib().dgt_solver_kernels(self.h, C.byref(n), None))
        k = np.zeros(n.value, np.int32)
        _check(lib().dgt_solver_kernels(self.h, C.byref(n), _np_ptr(k)))
        return [int(v) for v in k]

    def set_schedule(self, mode: int):
        """0: one launch per colour; 1: dependence-driven tiles, one launch per sub-chain."""
        _check(lib().dgt_solver_set_schedule(self.h, int(mode)))

    def set_wait_limit(self, polls: int):
        """Polls before a dependence wait of schedule 1 gives up (default 2**20)."""
        _check(lib().dgt_solver_set_wait_limit(self.h, int(polls)))

    def profile(self, on: bool):
        """Per-launch event timing of the tile kernels on (off by default)."""
        _check(lib().dgt_solver_profile(self.h, 1 if on else 0))

    def last_timing(self):
        tot, ker, n = C.c_double(), C.c_double(), C.c_int64()
        _check(lib().dgt_last_step_timing(self.h, C.byref(tot), C.byref(ker), C.byref(n)))
        return tot.value, ker.value, n.value

    def info(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().dgt_solver_info(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(np=a.value, bytes_per_step=b.value, lds_bytes=c.value)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dgt_solver_destroy(self.h)
            self.h = None


class CellList:
    """Cells of a solver's mesh for halo packing and unpacking (ids in the mesh's numbering)."""

    def __init__(self, solver: "Solver", cells):
        c = np.ascontiguousarray(cells, np.int32)
        self.n = int(c.size)
        h = C.c_void_p()
        _check(lib().dgt_cell_list_create(solver.h, self.n, _np_ptr(c), C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dgt_cell_list_destroy(self.h)
            self.h = None


class Batch:
    """Several inspected solvers advanced by one launch per sub-chain (dgt_batch_*)."""

    def __init__(self, solvers, stream=None):
        self.solvers = list(solvers)  # kept alive: members must outlive the batch
        arr = (C.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = C.c_void_p()
        _check(lib().dgt_batch_create(arr, len(self.solvers), _stream_handle(stream), C.byref(h)))
        self.h = h

    def set_graph(self, steps_per_graph: int):
        _check(lib().dgt_batch_set_graph(self.h, int(steps_per_graph)))

    def set_schedule(self, mode: int):
        """0: one launch per colour of a sub-chain; 1: dependence-driven, one per sub-chain."""
        _check(lib().dgt_batch_set_schedule(self.h, int(mode)))

    def step(self, nsteps: int, t0):
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, np.float64), (len(self.solvers),)))
        _check(lib().dgt_batch_step(self.h, int(nsteps), _np_ptr(t)))

    def timing(self):
        ms, n, g = C.c_double(), C.c_int64(), C.c_int64()
        _check(lib().dgt_batch_timing(self.h, C.byref(ms), C.byref(n), C.byref(g)))
        return dict(ms=ms.value, launches=n.value, graph_launches=g.value)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dgt_batch_destroy(self.h)
            self.h = None
