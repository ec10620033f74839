"""Seeded mesh and grid generators (numpy only).

These stand in for the real meshes the paper evaluates on (its Experiments
section: 828 to 268 686 faces, some not watertight, normalised into a cube),
which are not available here.  Every routine is deterministic given its
``numpy.random.Generator``.

Conventions
-----------
* Vertices ``V``: float64 ``[nV, 3]``; faces ``F``: int64 ``[nF, 3]``.  Callers
  cast to float32 / int32 for the GPU library.
* Faces of closed generators are wound counter-clockwise seen from outside, so
  ``(v1 - v0) x (v2 - v0)`` points out of the solid.
* A voxel grid is described by ``Grid(lo, hi, n)``; voxel centres are computed
  by the consumers, never here (except :func:`ellipsoid_target_on_grid`, which
  only builds a loss target and is not a checked output).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Grid:
    """Axis-aligned voxel grid: ``n[d]`` cells per axis spanning ``[lo[d], hi[d]]``.

    Flat voxel index is C order with x slowest and z fastest:
    ``idx = (i * n[1] + j) * n[2] + k``.
    """

    lo: tuple = (-0.5, -0.5, -0.5)
    hi: tuple = (0.5, 0.5, 0.5)
    n: tuple = (32, 32, 32)

    @staticmethod
    def cube(res: int, lo: float = -0.5, hi: float = 0.5) -> "Grid":
        return Grid((lo, lo, lo), (hi, hi, hi), (res, res, res))

    @property
    def size(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


def grid_flat_index(grid: Grid, i: int, j: int, k: int) -> int:
    return (int(i) * int(grid.n[1]) + int(j)) * int(grid.n[2]) + int(k)


# ----------------------------------------------------------------------------
# basic solids
# ----------------------------------------------------------------------------

def _orient_outward(V: np.ndarray, F: np.ndarray, centre=None) -> np.ndarray:
    """Flip faces of a star-shaped closed mesh so normals point away from ``centre``."""
    c = V.mean(axis=0) if centre is None else np.asarray(centre, dtype=np.float64)
    a, b, d = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, d - a)
    s = np.einsum("ij,ij->i", n, (a + b + d) / 3.0 - c)
    F = F.copy()
    flip = s < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return F


def octahedron_mesh(scale: float = 1.0):
    """Regular octahedron with vertices at +-scale on each axis (8 faces, outward)."""
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64) * scale
    F = []
    for x in (0, 1):
        for y in (2, 3):
            for z in (4, 5):
                F.append([x, y, z])
    F = _orient_outward(V, np.array(F, dtype=np.int64), centre=(0, 0, 0))
    return V, F


def cube_mesh(lo: float = 0.0, hi: float = 1.0):
    """Axis-aligned cube ``[lo, hi]^3`` as 12 outward triangles.

    Each square face is split along the diagonal from its lowest-index corner.
    """
    V = np.array([[x, y, z] for x in (lo, hi) for y in (lo, hi) for z in (lo, hi)], dtype=np.float64)
    # corner index = 4*ix + 2*iy + iz
    quads = [
        (0, 1, 3, 2),  # x = lo
        (4, 6, 7, 5),  # x = hi
        (0, 4, 5, 1),  # y = lo
        (2, 3, 7, 6),  # y = hi
        (0, 2, 6, 4),  # z = lo
        (1, 5, 7, 3),  # z = hi
    ]
    F = []
    for a, b, c, d in quads:
        F.append([a, b, c])
        F.append([a, c, d])
    mid = 0.5 * (lo + hi)
    F = _orient_outward(V, np.array(F, dtype=np.int64), centre=(mid, mid, mid))
    return V, F


def icosphere(subdiv: int):
    """Unit icosphere: regular icosahedron, each level splits every edge at its
    midpoint and projects onto the unit sphere.  ``s=3`` gives 642 vertices /
    1280 faces, ``s=4`` gives 2562 / 5120."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = [
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ]
    F = [
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        nf = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        F = nf
    V = np.array(V, dtype=np.float64)
    F = _orient_outward(V, np.array(F, dtype=np.int64), centre=(0, 0, 0))
    return V, F


def uv_ellipsoid(m: int, n: int, semi_axes=(1.0, 1.0, 1.0), rotation=None, centre=(0.0, 0.0, 0.0)):
    """UV sphere with ``m`` longitudes and ``n`` latitude bands, mapped to an ellipsoid.

    ``2 + m (n - 1)`` vertices and exactly ``2 m (n - 1)`` triangles, wound outward.
    A point ``u`` of the unit sphere maps to ``centre + R (semi_axes * u)``.
    """
    if m < 3 or n < 2:
        raise ValueError("uv_ellipsoid needs m >= 3 and n >= 2")
    th = math.pi * np.arange(1, n) / n
    ph = 2.0 * math.pi * np.arange(m) / m
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    ringv = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1).reshape(-1, 3)
    U = np.concatenate([[[0.0, 0.0, 1.0]], ringv, [[0.0, 0.0, -1.0]]], axis=0)
    south = len(U) - 1

    j = np.arange(m)
    jn = (j + 1) % m

    def ring(i, jj):  # i in 1..n-1
        return 1 + (i - 1) * m + jj

    parts = [np.stack([np.zeros(m, np.int64), ring(1, j), ring(1, jn)], -1)]
    if n > 2:
        i = np.arange(1, n - 1)[:, None]
        a, b = ring(i, j[None, :]), ring(i, jn[None, :])
        c, d = ring(i + 1, j[None, :]), ring(i + 1, jn[None, :])
        quad = np.stack([np.stack([a, c, d], -1), np.stack([a, d, b], -1)], axis=2)  # [n-2, m, 2, 3]
        parts.append(quad.reshape(-1, 3))
    parts.append(np.stack([np.full(m, south, np.int64), ring(n - 1, jn), ring(n - 1, j)], -1))
    F = np.concatenate(parts, axis=0).astype(np.int64)
    F = _orient_outward(U, F, centre=(0, 0, 0))
    R = np.eye(3) if rotation is None else np.asarray(rotation, dtype=np.float64)
    V = (U * np.asarray(semi_axes, dtype=np.float64)) @ R.T + np.asarray(centre, dtype=np.float64)
    if np.linalg.det(R) < 0:  # a mirror would turn the winding inside out
        F = F[:, [0, 2, 1]]
    return V, F


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation: QR of a Gaussian 3x3, column signs fixed, det +1."""
    A = rng.normal(size=(3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def uv_resolution_for_faces(target_faces: int):
    """(m, n) with m ~ 2(n-1) so that 2 m (n-1) is close to ``target_faces``."""
    k = max(2, int(round(math.sqrt(max(target_faces, 16) / 4.0))))
    return 2 * k, k + 1


@dataclass
class Ellipsoid:
    centre: np.ndarray
    rotation: np.ndarray
    semi_axes: np.ndarray

    def mesh(self, m: int, n: int):
        return uv_ellipsoid(m, n, self.semi_axes, self.rotation, self.centre)


def random_ellipsoid(rng, axes_lo, axes_hi, centre_lo, centre_hi) -> Ellipsoid:
    a = rng.uniform(axes_lo, axes_hi, size=3)
    c = rng.uniform(centre_lo, centre_hi, size=3)
    R = random_rotation(rng)
    return Ellipsoid(c, R, a)


def concat_meshes(meshes):
    Vs, Fs, off = [], [], 0
    for V, F in meshes:
        Vs.append(np.asarray(V, dtype=np.float64))
        Fs.append(np.asarray(F, dtype=np.int64) + off)
        off += len(V)
    return np.concatenate(Vs, axis=0), np.concatenate(Fs, axis=0)


def ellipsoid_union(rng, n_ellipsoids: int, faces_each: int, axes=(0.05, 0.3), centres=(-0.3, 0.3)):
    """Concatenation (not a boolean union: shells may overlap) of seeded ellipsoids."""
    m, n = uv_resolution_for_faces(faces_each)
    parts, ells = [], []
    for _ in range(n_ellipsoids):
        e = random_ellipsoid(rng, axes[0], axes[1], centres[0], centres[1])
        ells.append(e)
        parts.append(e.mesh(m, n))
    V, F = concat_meshes(parts)
    return V, F, ells


def delete_faces(F: np.ndarray, count: int, rng: np.random.Generator) -> np.ndarray:
    """Remove exactly ``count`` faces chosen uniformly without replacement (order kept)."""
    count = int(count)
    if count <= 0:
        return np.asarray(F).copy()
    drop = rng.choice(len(F), size=count, replace=False)
    keep = np.ones(len(F), dtype=bool)
    keep[drop] = False
    return np.asarray(F)[keep].copy()


def jitter(V: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Add i.i.d. N(0, sigma^2) to every vertex coordinate (sigma is a standard deviation)."""
    return np.asarray(V, dtype=np.float64) + rng.normal(0.0, sigma, size=np.shape(V))


def reverse_faces(F: np.ndarray) -> np.ndarray:
    return np.asarray(F)[:, [0, 2, 1]].copy()


def ellipsoid_inside(points: np.ndarray, e: Ellipsoid) -> np.ndarray:
    """Analytic inside test of a solid ellipsoid (used only to build loss targets)."""
    p = (np.asarray(points, dtype=np.float64) - e.centre) @ e.rotation
    return (np.sum((p / e.semi_axes) ** 2, axis=-1) < 1.0)


def ellipsoid_target_on_grid(grid: Grid, e: Ellipsoid) -> np.ndarray:
    """{0,1} float32 target of a solid ellipsoid sampled at the grid's cell centres.

    It is an input of the sigmoid-MSE loss, never compared with a winding number.
    Evaluated separably per axis so that 256^3 grids stay cheap."""
    axes = [np.asarray(grid.lo[d], np.float64) + (np.arange(grid.n[d]) + 0.5) *
            ((grid.hi[d] - grid.lo[d]) / grid.n[d]) - e.centre[d] for d in range(3)]
    acc = np.zeros(tuple(int(x) for x in grid.n), dtype=np.float64)
    for c in range(3):
        u = (axes[0][:, None, None] * e.rotation[0, c] + axes[1][None, :, None] * e.rotation[1, c]
             + axes[2][None, None, :] * e.rotation[2, c]) / e.semi_axes[c]
        acc += u * u
    return (acc < 1.0).astype(np.float32).reshape(-1)


def signed_volume(V: np.ndarray, F: np.ndarray) -> float:
    """Divergence-theorem volume; positive for an outward-wound closed mesh."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)
