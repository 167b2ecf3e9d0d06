"""Seeded synthetic inputs for the DG elastic loop chain.

This module builds *inputs only*: triangle meshes, per-cell materials and
source positions.  It holds none of the method's arithmetic (no basis, no
flux, no tiling) and imports nothing from the HIP path or from the oracle, so
both sides can draw the same inputs from it.

Randomness comes from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), implemented here from its
published definition so that every stream is reproducible bit for bit.

Shapes follow the paper's workload (Sec. 7.4: 2-D rectangular domain tessellated
with unstructured triangles, polynomial order q = 1..4, explosive point source);
the paper's own meshes are not available, so structured-then-jittered,
optionally renumbered meshes of the unit square stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_MASK64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(seed: int, count: int) -> np.ndarray:
    """Return `count` consecutive SplitMix64 outputs (uint64) of stream `seed`."""
    out = np.empty(count, dtype=np.uint64)
    # vectorised form of the sequential definition: state_i = seed + (i+1)*golden
    idx = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + idx * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    out[:] = z
    return out


def uniform01(seed: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of SplitMix64 outputs."""
    return (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _stream(seed: int, sub: int) -> int:
    """Derive an independent stream seed (hash of (seed, sub))."""
    return int(splitmix64((seed * 0x100000001B3 + sub) & _MASK64, 1)[0])


@dataclass
class Mesh:
    """A CCW triangle mesh: vertex coordinates and cell-to-vertex connectivity."""
    n: int
    xy: np.ndarray          # [nv, 2] float64
    c2v: np.ndarray         # [nc, 3] int32, counter-clockwise
    periodic: int = 0       # bit 0: x-periodic, bit 1: y-periodic
    perm: np.ndarray | None = None   # new cell k = old (structured) cell perm[k]
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return self.xy.shape[0]

    @property
    def nc(self) -> int:
        return self.c2v.shape[0]

    def centroids(self) -> np.ndarray:
        p = self.xy[self.c2v]
        return ((p[:, 0] + p[:, 1]) + p[:, 2]) / 3.0


def square_mesh(n: int, jitter: float = 0.0, jitter_seed: int = 1,
                renumber_seed: int | None = None, periodic: int = 0) -> Mesh:
    """n x n squares on [0,1]^2, each split along its (i,j)-(i+1,j+1) diagonal.

    * vertex (i, j) has id j*(n+1)+i and sits at (i/n, j/n);
    * square (i, j) gives cells 2*(j*n+i) = [(i,j),(i+1,j),(i+1,j+1)] and
      2*(j*n+i)+1 = [(i,j),(i+1,j+1),(i,j+1)], both counter-clockwise;
    * interior vertices move by U(-jitter*h, jitter*h) per coordinate
      (boundary vertices stay put so the domain stays the unit square);
    * if `renumber_seed` is given, cells are shuffled by a seeded Fisher-Yates
      permutation.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    jj, ii = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    xy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)
    if jitter > 0.0:
        interior = ((ii > 0) & (ii < n) & (jj > 0) & (jj < n)).ravel()
        idx = np.nonzero(interior)[0]
        u = uniform01(jitter_seed, 2 * idx.size).reshape(-1, 2)
        xy[idx] += (2.0 * u - 1.0) * (jitter * h)
    sq_j, sq_i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v00 = (sq_j * (n + 1) + sq_i).ravel()
    v10 = v00 + 1
    v11 = v00 + (n + 1) + 1
    v01 = v00 + (n + 1)
    c2v = np.empty((2 * n * n, 3), dtype=np.int32)
    c2v[0::2] = np.stack([v00, v10, v11], axis=1)
    c2v[1::2] = np.stack([v00, v11, v01], axis=1)
    perm = None
    if renumber_seed is not None:
        perm = fisher_yates(c2v.shape[0], renumber_seed)
        c2v = np.ascontiguousarray(c2v[perm])
    m = Mesh(n=n, xy=xy, c2v=c2v, periodic=periodic, perm=perm,
             meta=dict(jitter=jitter, jitter_seed=jitter_seed, renumber_seed=renumber_seed))
    p = xy[c2v]
    det = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - \
          (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    if not np.all(det > 0):
        raise AssertionError("generator produced a non-positive cell orientation")
    return m


def fisher_yates(count: int, seed: int) -> np.ndarray:
    """Seeded Fisher-Yates shuffle of range(count): j = z mod (i+1), i = count-1..1."""
    perm = np.arange(count, dtype=np.int64)
    if count <= 1:
        return perm.astype(np.int32)
    z = splitmix64(seed, count - 1)
    for k, i in enumerate(range(count - 1, 0, -1)):
        j = int(z[k] % np.uint64(i + 1))
        perm[i], perm[j] = perm[j], perm[i]
    return perm.astype(np.int32)


def layered_material(mesh: Mesh) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Three layers by centroid y: (lambda, mu, rho) = m * (2, 1, 1) with
    m = 1 for y >= 2/3, 1.5 for 1/3 <= y < 2/3, 2 for y < 1/3 (impedance
    contrast 2x, wave speeds unchanged)."""
    cy = mesh.centroids()[:, 1]
    m = np.where(cy >= 2.0 / 3.0, 1.0, np.where(cy >= 1.0 / 3.0, 1.5, 2.0))
    return 2.0 * m, 1.0 * m, 1.0 * m


def homogeneous_material(mesh: Mesh, lam: float = 2.0, mu: float = 1.0, rho: float = 1.0):
    nc = mesh.nc
    return np.full(nc, lam), np.full(nc, mu), np.full(nc, rho)


def _gaussian_field(points: np.ndarray, seed: int, modes: int = 64, kscale: float = 4.0) -> np.ndarray:
    """Smooth zero-mean unit-variance random field: sqrt(2/M) sum cos(2 pi k.x + theta)."""
    u = uniform01(seed, 4 * modes).reshape(modes, 4)
    # Box-Muller for the two wave-vector components
    r = np.sqrt(-2.0 * np.log(1.0 - u[:, 0]))
    kx = kscale * r * np.cos(2.0 * math.pi * u[:, 1])
    ky = kscale * r * np.sin(2.0 * math.pi * u[:, 1])
    theta = 2.0 * math.pi * u[:, 2]
    ph = 2.0 * math.pi * (points[:, :1] * kx[None, :] + points[:, 1:2] * ky[None, :]) + theta[None, :]
    return math.sqrt(2.0 / modes) * np.cos(ph).sum(axis=1)


def lognormal_material(mesh: Mesh, sigma: float = 0.3, seed: int = 3):
    """lambda = 2 exp(sigma g1), mu = exp(sigma g2), rho = exp(sigma g3), each g an
    independent smooth field sampled at cell centroids."""
    c = mesh.centroids()
    g = [_gaussian_field(c, _stream(seed, s)) for s in (1, 2, 3)]
    return 2.0 * np.exp(sigma * g[0]), np.exp(sigma * g[1]), np.exp(sigma * g[2])


def shot_positions(count: int, seed: int = 4) -> np.ndarray:
    """Source positions uniform in [0.1, 0.9]^2."""
    u = uniform01(seed, 2 * count).reshape(count, 2)
    return 0.1 + 0.8 * u


def random_state(shape, seed: int) -> np.ndarray:
    """Uniform(-1, 1) doubles, for parity tests that start from a non-zero state."""
    n = int(np.prod(shape))
    return (2.0 * uniform01(seed, n) - 1.0).reshape(shape)


# -- one GPU's share of a distributed mesh ----------------------------------
# A mesh distributor (DMPlex in the paper's Firedrake setting, Sec. 5.2) hands each
# process a contiguous block of cells plus layers of halo cells, with every cell
# labelled by region (Sec. 3.3).  These helpers build that input for one part.

CORE, BOUNDARY, NON_EXEC = 0, 1, 2


@dataclass
class MeshPart:
    """Cells of one part: owned cells, `depth` layers of exec halo, one non-exec layer."""
    cells: np.ndarray       # [nl] global cell ids of the local cells, ascending
    layer: np.ndarray       # [nl] 0 owned, 1..depth exec halo, depth+1 non-exec
    region: np.ndarray      # [nl] uint8: CORE, BOUNDARY (owned next to the halo, or exec), NON_EXEC
    mesh: Mesh              # the local mesh (vertices of the local cells, ascending global id)
    vertices: np.ndarray    # [nv_local] global vertex ids

    @property
    def owned(self) -> np.ndarray:
        return self.layer == 0


def cell_neighbours(mesh: Mesh) -> np.ndarray:
    """[nc, 3] the cell across each edge (vertices l, l+1 mod 3), -1 on the boundary."""
    if mesh.periodic:
        raise ValueError("cell_neighbours takes non-periodic meshes")
    nc = mesh.nc
    a = mesh.c2v
    ev = np.stack([a, np.roll(a, -1, axis=1)], axis=2).reshape(-1, 2).astype(np.int64)
    key = np.minimum(ev[:, 0], ev[:, 1]) * (mesh.nv + 1) + np.maximum(ev[:, 0], ev[:, 1])
    order = np.argsort(key, kind="stable")
    ks = key[order]
    nb = np.full(3 * nc, -1, np.int64)
    same = np.nonzero(ks[1:] == ks[:-1])[0]
    h0, h1 = order[same], order[same + 1]
    nb[h0] = h1 // 3
    nb[h1] = h0 // 3
    return nb.reshape(nc, 3).astype(np.int32)


def block_parts(mesh: Mesh, bx: int, by: int) -> np.ndarray:
    """Part of each cell for bx x by rectangular blocks of the bounding box (by centroid)."""
    c = mesh.centroids()
    lo, hi = mesh.xy.min(axis=0), mesh.xy.max(axis=0)
    ix = np.clip(np.floor((c[:, 0] - lo[0]) / (hi[0] - lo[0]) * bx), 0, bx - 1).astype(np.int32)
    iy = np.clip(np.floor((c[:, 1] - lo[1]) / (hi[1] - lo[1]) * by), 0, by - 1).astype(np.int32)
    return iy * bx + ix


def mesh_part(mesh: Mesh, parts: np.ndarray, part: int, depth: int) -> MeshPart:
    """Owned cells of `part`, `depth` exec layers around them (cells sharing an edge with
    the previous layer), one non-exec layer beyond; regions: owned cells with a neighbour
    outside the part are BOUNDARY (owned sub-region), the other owned cells CORE, exec
    cells BOUNDARY, the last layer NON_EXEC."""
    if depth < 0:
        raise ValueError("depth must be >= 0")
    nb = cell_neighbours(mesh)
    layer = np.full(mesh.nc, -1, np.int32)
    owned = np.asarray(parts) == part
    layer[owned] = 0
    front = np.nonzero(owned)[0]
    for d in range(1, depth + 2):
        cand = nb[front].ravel()
        cand = np.unique(cand[cand >= 0])
        cand = cand[layer[cand] < 0]
        layer[cand] = d
        front = cand
    cells = np.nonzero(layer >= 0)[0].astype(np.int32)
    lay = layer[cells]
    region = np.where(lay == 0, CORE, np.where(lay <= depth, BOUNDARY, NON_EXEC)).astype(np.uint8)
    nbo = nb[cells[lay == 0]]
    touches = ((nbo >= 0) & (~owned[np.maximum(nbo, 0)])).any(axis=1)
    r0 = region[lay == 0]
    r0[touches] = BOUNDARY
    region[lay == 0] = r0
    verts = np.unique(mesh.c2v[cells].ravel())
    remap = np.full(mesh.nv, -1, np.int64)
    remap[verts] = np.arange(verts.size)
    local = Mesh(n=mesh.n, xy=np.ascontiguousarray(mesh.xy[verts]),
                 c2v=np.ascontiguousarray(remap[mesh.c2v[cells]].astype(np.int32)),
                 meta=dict(part=part, depth=depth))
    return MeshPart(cells=cells, layer=lay, region=region, mesh=local, vertices=verts.astype(np.int32))


# -- named workloads ---------------------------------------------------------

def workload(name: str):
    """Return (mesh, (lam, mu, rho), params) for a named synthetic workload.

    `small_p1`: 32x32 structured (2048 cells), P1, homogeneous (2,1,1), central
    flux, free surface all round, Ricker f=5 at (0.5,0.5), FP64, 100 steps.
    `jitter512_p2`: 512x512 jittered (0.2h) and randomly renumbered mesh
    (524288 cells), P2, three layers, upwind flux, free top / absorbing
    elsewhere.
    `jitter1024_p3`/`_p4`: 1024x1024 jittered and renumbered, lognormal
    sigma 0.3 material, P3 / P4, upwind.
    """
    if name == "small_p1":
        m = square_mesh(32)
        mat = homogeneous_material(m)
        prm = dict(degree=1, flux=0, time_order=4, free_sides=0xF, steps=100,
                   source=(0.5, 0.5, 5.0, 0.2, 1.0))
    elif name == "jitter512_p2":
        m = square_mesh(512, jitter=0.2, jitter_seed=1, renumber_seed=2)
        mat = layered_material(m)
        prm = dict(degree=2, flux=1, time_order=4, free_sides=0x8, steps=1000,
                   source=(0.5, 0.5, 5.0, 0.2, 1.0))
    elif name in ("jitter1024_p3", "jitter1024_p4"):
        m = square_mesh(1024, jitter=0.2, jitter_seed=1, renumber_seed=2)
        mat = lognormal_material(m)
        prm = dict(degree=3 if name.endswith("p3") else 4, flux=1, time_order=4,
                   free_sides=0x8, steps=500, source=(0.5, 0.5, 5.0, 0.2, 1.0))
    else:
        raise KeyError(name)
    return m, mat, prm
