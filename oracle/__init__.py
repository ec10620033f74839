"""FP64 CPU oracle for the generalized winding number (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never touches it and the
two share no code.  The arithmetic lives in ``wn_oracle.c`` (plain C, FP64,
OpenMP over independent outputs); this module loads it with ``ctypes`` and adds
the trivial element-wise maps (occupancy, sigmoid-MSE loss) in numpy FP64.

Paper sections followed (arXiv 2407.11272):
  * Section 2.2, Eq. 5: W(q) = (1/4 pi) sum_f Omega_f(q);
  * Section 2.2, Eq. 7 with the half-angle factor 2, and Eq. 8 (ATAN2 cases);
  * Algorithm 1 (per-face normalise, alpha, beta, ATAN2, accumulate);
  * Section 2.1, Eq. 3: for a closed surface W is the occupancy; the map to a hard
    or soft occupancy uses a threshold or a sigmoid around 0.5;
  * Section 2.4 (mesh morphing): the voxel loss drives the vertices through Adam
    (Kingma and Ba, 2015, Algorithm 1), written out in numpy FP64;
  * Section 3 (evaluation): occupancy -> cube surface ("cubified"), or marching cubes
    of the field -> Laplacian smoothing (10 iterations, lambda = 0.15) -> 20 000
    surface samples -> Chamfer and Hausdorff distances to the original mesh.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wn_oracle.c")
_LIB = os.path.join(_HERE, "libwn_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    lib.wno_atan2_eq8.restype = ctypes.c_double
    lib.wno_atan2_eq8.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.wno_solid_angle.restype = ctypes.c_double
    lib.wno_solid_angle.argtypes = [_dp, _dp, _dp, _dp]
    lib.wno_alpha_beta.restype = None
    lib.wno_alpha_beta.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp]
    lib.wno_solid_angle_grad.restype = None
    lib.wno_solid_angle_grad.argtypes = [_dp, _dp, _dp, _dp, _dp]
    lib.wno_winding.restype = ctypes.c_int
    lib.wno_winding.argtypes = [_dp, ctypes.c_int64, _lp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, ctypes.c_int]
    lib.wno_grad.restype = ctypes.c_int
    lib.wno_grad.argtypes = [_dp, ctypes.c_int64, _lp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _dp, _dp,
                             ctypes.c_int]
    lib.wno_min_dist.restype = ctypes.c_int
    lib.wno_min_dist.argtypes = [_dp, ctypes.c_int64, _lp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _dp,
                                 ctypes.c_int]
    lib.wno_grid_points.restype = None
    lib.wno_grid_points.argtypes = [_dp, _dp, _lp, _dp]
    lib.wno_max_threads.restype = ctypes.c_int
    lib.wno_max_threads.argtypes = []
    lib.wno_winding_naive.restype = ctypes.c_int
    lib.wno_winding_naive.argtypes = [_dp, ctypes.c_int64, _lp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _dp,
                                      ctypes.c_int]
    lib.wno_naive_term_grad.restype = None
    lib.wno_naive_term_grad.argtypes = [_dp, _dp, _dp, _dp, _dp]
    lib.wno_grad_naive.restype = ctypes.c_int
    lib.wno_grad_naive.argtypes = [_dp, ctypes.c_int64, _lp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _dp, _dp,
                                   ctypes.c_int]
    lib.wno_nn_dist.restype = ctypes.c_int
    lib.wno_nn_dist.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, ctypes.c_int]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


class use_library:
    """Context manager that routes every oracle call to another build of the same
    source (the mutation tests load deliberately broken copies this way)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _bind(ctypes.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_lp)


def max_threads() -> int:
    return int(_load().wno_max_threads())


def atan2_eq8(y: float, x: float) -> float:
    """Section 2.2, Eq. 8 case table (ATAN2(0, 0) = 0; y = -0 counts as y >= 0)."""
    return float(_load().wno_atan2_eq8(float(y), float(x)))


def alpha_beta(v0, v1, v2, q):
    """Section 2.2, Eq. 7 numerator det(e0,e1,e2) and denominator 1 + sum of dots."""
    a = ctypes.c_double()
    b = ctypes.c_double()
    args = [_d(x) for x in (v0, v1, v2, q)]
    _load().wno_alpha_beta(*(p for _, p in args), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def solid_angle(v0, v1, v2, q) -> float:
    """Omega = 2 ATAN2(alpha, beta) of one triangle at q (Eq. 7 with the factor 2)."""
    args = [_d(x) for x in (v0, v1, v2, q)]
    return float(_load().wno_solid_angle(*(p for _, p in args)))


def solid_angle_grad(v0, v1, v2, q) -> np.ndarray:
    """dOmega/dv_j as a [3, 3] array (row j = vertex j)."""
    out = np.zeros(9, dtype=np.float64)
    args = [_d(x) for x in (v0, v1, v2, q)]
    _load().wno_solid_angle_grad(*(p for _, p in args), out.ctypes.data_as(_dp))
    return out.reshape(3, 3)


def grid_points(grid) -> np.ndarray:
    """Voxel centres ``lo + (idx + 1/2)(hi - lo)/n`` in FP64, C order (z fastest)."""
    lo, plo = _d(np.asarray(grid.lo, dtype=np.float64))
    hi, phi = _d(np.asarray(grid.hi, dtype=np.float64))
    n, pn = _i(np.asarray(grid.n, dtype=np.int64))
    Q = np.empty((int(np.prod(n)), 3), dtype=np.float64)
    _load().wno_grid_points(plo, phi, pn, Q.ctypes.data_as(_dp))
    return Q


def winding(V, F, Q, threads: int = 0) -> np.ndarray:
    """W(q) for every row of Q by brute force over all faces (Eq. 5, 7, 8), FP64."""
    V, pv = _d(np.asarray(V).reshape(-1, 3))
    F, pf = _i(np.asarray(F).reshape(-1, 3))
    Q, pq = _d(np.asarray(Q).reshape(-1, 3))
    W = np.empty(len(Q), dtype=np.float64)
    rc = _load().wno_winding(pv, len(V), pf, len(F), pq, len(Q), W.ctypes.data_as(_dp), int(threads))
    if rc != 0:
        raise ValueError("oracle: face index out of range")
    return W


def winding_grid(V, F, grid, threads: int = 0) -> np.ndarray:
    return winding(V, F, grid_points(grid), threads)


def grad(V, F, Q, dLdW, threads: int = 0):
    """(dL/dT [nF, 3, 3], dL/dV [nV, 3]) for the given dL/dW at the rows of Q."""
    V, pv = _d(np.asarray(V).reshape(-1, 3))
    F, pf = _i(np.asarray(F).reshape(-1, 3))
    Q, pq = _d(np.asarray(Q).reshape(-1, 3))
    g, pg = _d(np.asarray(dLdW).reshape(-1))
    if len(g) != len(Q):
        raise ValueError("dLdW must have one entry per query point")
    T = np.zeros((len(F), 9), dtype=np.float64)
    D = np.zeros((len(V), 3), dtype=np.float64)
    rc = _load().wno_grad(pv, len(V), pf, len(F), pq, len(Q), pg, T.ctypes.data_as(_dp), D.ctypes.data_as(_dp),
                          int(threads))
    if rc != 0:
        raise ValueError("oracle: face index out of range")
    return T.reshape(-1, 3, 3), D


def winding_naive(V, F, Q, threads: int = 0, with_scale: bool = False):
    """Section 2.1, Eq. 4: one centroid sample per face, 1/(8 pi) sum <N, c - q>/|c - q|^3.
    With ``with_scale`` also returns 1/(8 pi) sum |term| per point (the rounding scale)."""
    V, pv = _d(np.asarray(V).reshape(-1, 3))
    F, pf = _i(np.asarray(F).reshape(-1, 3))
    Q, pq = _d(np.asarray(Q).reshape(-1, 3))
    W = np.empty(len(Q))
    S = np.empty(len(Q))
    rc = _load().wno_winding_naive(pv, len(V), pf, len(F), pq, len(Q), W.ctypes.data_as(_dp), S.ctypes.data_as(_dp),
                                   int(threads))
    if rc != 0:
        raise ValueError("oracle: face index out of range")
    return (W, S) if with_scale else W


def naive_term_grad(v0, v1, v2, q) -> np.ndarray:
    out = np.zeros(9, dtype=np.float64)
    args = [_d(x) for x in (v0, v1, v2, q)]
    _load().wno_naive_term_grad(*(p for _, p in args), out.ctypes.data_as(_dp))
    return out.reshape(3, 3)


def grad_naive(V, F, Q, dLdW, threads: int = 0):
    """(dL/dT [nF, 3, 3], dL/dV [nV, 3]) of the Eq. 4 sum for the given dL/dW."""
    V, pv = _d(np.asarray(V).reshape(-1, 3))
    F, pf = _i(np.asarray(F).reshape(-1, 3))
    Q, pq = _d(np.asarray(Q).reshape(-1, 3))
    g, pg = _d(np.asarray(dLdW).reshape(-1))
    T = np.zeros((len(F), 9))
    D = np.zeros((len(V), 3))
    rc = _load().wno_grad_naive(pv, len(V), pf, len(F), pq, len(Q), pg, T.ctypes.data_as(_dp),
                                D.ctypes.data_as(_dp), int(threads))
    if rc != 0:
        raise ValueError("oracle: face index out of range")
    return T.reshape(-1, 3, 3), D


def min_dist(V, F, Q, threads: int = 0):
    """(distance to nearest edge or vertex, distance to nearest face) per query point."""
    V, pv = _d(np.asarray(V).reshape(-1, 3))
    F, pf = _i(np.asarray(F).reshape(-1, 3))
    Q, pq = _d(np.asarray(Q).reshape(-1, 3))
    de = np.empty(len(Q))
    df = np.empty(len(Q))
    rc = _load().wno_min_dist(pv, len(V), pf, len(F), pq, len(Q), de.ctypes.data_as(_dp), df.ctypes.data_as(_dp),
                              int(threads))
    if rc != 0:
        raise ValueError("oracle: face index out of range")
    return de, df


def guard_mask(V, F, Q, edge_tol: float = 1e-4, face_tol: float = 1e-6, threads: int = 0) -> np.ndarray:
    """True where a point is too close to the surface for an FP32 result to be held
    to the FP64 one: within ``edge_tol`` of an edge or vertex, or ``face_tol`` of a face.
    Section 2.2 notes the field is binary except at points on the surface."""
    de, df = min_dist(V, F, Q, threads)
    return (de < edge_tol) | (df < face_tol)


# ------------------------------------------------------- flipping duplication ---

def vertex_normals(V, F) -> np.ndarray:
    """Unit vertex normals: the sum of the (area-weighted) face normals
    (v1 - v0) x (v2 - v0) of the faces using the vertex, normalised; 0 for a vertex
    no face uses or whose sum vanishes.  (Algorithm 2 asks for per-vertex normals
    without fixing their weighting; area weighting is the reading taken.)"""
    V = np.asarray(V, dtype=np.float64).reshape(-1, 3)
    F = np.asarray(F, dtype=np.int64).reshape(-1, 3)
    acc = np.zeros_like(V)
    for f in F:  # in face order
        n = np.cross(V[f[1]] - V[f[0]], V[f[2]] - V[f[0]])
        for j in range(3):
            acc[f[j]] += n
    norm = np.linalg.norm(acc, axis=1, keepdims=True)
    out = np.zeros_like(V)
    ok = norm[:, 0] > 0
    out[ok] = acc[ok] / norm[ok]
    return out


def flip_duplicate(V, F, eps: float = 0.01):
    """Algorithm 2 (flipping duplication): V' = V - eps N (vertex normals), faces copied
    onto V' with their orientation reversed, returned as (V | V', F | F')."""
    V = np.asarray(V, dtype=np.float64).reshape(-1, 3)
    F = np.asarray(F, dtype=np.int64).reshape(-1, 3)
    N = vertex_normals(V, F)
    V2 = np.concatenate([V, V - eps * N], axis=0)
    Fp = F[:, [0, 2, 1]] + len(V)
    return V2, np.concatenate([F, Fp], axis=0)


# ------------------------------------------------------------ occupancy maps ---

def occupancy_threshold(W, tau: float = 0.5) -> np.ndarray:
    """Hard occupancy 1[W > tau] as uint8 (Eq. 3: W is the occupancy of a closed surface)."""
    return (np.asarray(W, dtype=np.float64) > tau).astype(np.uint8)


def occupancy_sigmoid(W, tau: float = 0.5, k: float = 50.0) -> np.ndarray:
    """Soft occupancy 1 / (1 + exp(-k (W - tau)))."""
    W = np.asarray(W, dtype=np.float64)
    return 1.0 / (1.0 + np.exp(-k * (W - tau)))


def sigmoid_mse(W, target, tau: float = 0.5, k: float = 50.0):
    """Loss L = mean_q (sigmoid(k (W_q - tau)) - target_q)^2 and dL/dW_q."""
    W = np.asarray(W, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    s = occupancy_sigmoid(W, tau, k)
    n = max(len(W), 1)
    L = float(np.sum((s - t) ** 2) / n)
    dLdW = 2.0 * (s - t) / n * k * s * (1.0 - s)
    return L, dLdW


def adam(x, g, m, v, t: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma and Ba, 2015, Algorithm 1), FP64: the moment estimates
    m, v are exponential averages of g and g^2, divided by (1 - beta^t) to remove
    their bias towards the zero start, and x moves by lr m_hat / (sqrt(v_hat) + eps).
    Returns the new (x, m, v)."""
    x, g, m, v = (np.asarray(a, dtype=np.float64) for a in (x, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return x - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def morph(V, F, grid, target, iters: int, integral: str = "naive", tau: float = 0.5, k: float = 50.0,
          lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, t0: int = 0,
          m=None, v=None, threads: int = 0):
    """Mesh morphing by voxel supervision (Section 2.4): repeat {W at the voxel centres
    (Eq. 4 naive sum, or Eq. 5/7), the soft-occupancy MSE against the target, its
    gradient with respect to the vertices, one Adam step}.  FP64 throughout.
    Returns (V, m, v, losses) with losses[i] evaluated before update i."""
    V = np.array(V, dtype=np.float64)
    m = np.zeros_like(V) if m is None else np.array(m, dtype=np.float64)
    v = np.zeros_like(V) if v is None else np.array(v, dtype=np.float64)
    Q = grid_points(grid)
    fwd = winding_naive if integral == "naive" else winding
    bwd = grad_naive if integral == "naive" else grad
    losses = []
    for i in range(iters):
        W = fwd(V, F, Q, threads=threads)
        L, dLdW = sigmoid_mse(W, target, tau, k)
        _, dLdV = bwd(V, F, Q, dLdW, threads=threads)
        V, m, v = adam(V, dLdV, m, v, t0 + 1 + i, lr, beta1, beta2, eps)
        losses.append(L)
    return V, m, v, np.array(losses)


# ------------------------------------------------------------ evaluation chain (Section 3)

# Faces of the unit cube [0,1]^3 around a voxel, in the order -x, +x, -y, +y, -z, +z.
# Each entry: (axis, side, the two in-plane axes (u, w) with u x w = +axis).  A face's
# corners p0..p3 walk (0,0), (1,0), (1,1), (0,1) in (u, w); triangles (p0,p1,p2),
# (p0,p2,p3) face +axis, and their reversal faces -axis.
_CUBE_DIRS = [(0, 0, 1, 2), (0, 1, 1, 2), (1, 0, 2, 0), (1, 1, 2, 0), (2, 0, 0, 1), (2, 1, 0, 1)]


def _quad_corners(ijk, d):
    axis, side, u, w = _CUBE_DIRS[d]
    base = list(ijk)
    base[axis] += side
    out = []
    for du, dw in ((0, 0), (1, 0), (1, 1), (0, 1)):
        c = list(base)
        c[u] += du
        c[w] += dw
        out.append(tuple(c))
    if side == 0:
        tris = [(out[0], out[2], out[1]), (out[0], out[3], out[2])]
    else:
        tris = [(out[0], out[1], out[2]), (out[0], out[2], out[3])]
    return tris


def cubify(occ, grid):
    """Cube surface of an occupancy grid (the 'cubified' occupancy of Section 3): every
    face of an occupied voxel whose neighbour is empty or outside the grid becomes two
    outward triangles.  Faces in voxel C order, then -x, +x, -y, +y, -z, +z; vertices
    are the lattice corners used, numbered in lattice C order, at lo + corner * h (FP64).
    Returns (V [nV, 3] float64, F [nF, 3] int64)."""
    occ = np.asarray(occ).reshape(tuple(int(x) for x in grid.n)).astype(bool)
    n = occ.shape
    pad = np.pad(occ, 1)
    keys, tris = [], []
    idx = np.argwhere(occ)  # C order
    lin = (idx[:, 0] * n[1] + idx[:, 1]) * n[2] + idx[:, 2]
    for d in range(6):
        axis, side = _CUBE_DIRS[d][0], _CUBE_DIRS[d][1]
        nb = idx + 1
        nb[:, axis] += 1 if side else -1
        bnd = ~pad[nb[:, 0], nb[:, 1], nb[:, 2]]
        for t in range(2):
            corners = np.stack([np.array(_quad_corners((0, 0, 0), d)[t][j]) for j in range(3)])  # [3, 3]
            tris.append(idx[bnd][:, None, :] + corners[None])
            keys.append(lin[bnd] * 12 + 2 * d + t)
    if not idx.size or not np.concatenate(keys).size:
        return np.zeros((0, 3)), np.zeros((0, 3), np.int64)
    order = np.argsort(np.concatenate(keys), kind="stable")
    T = np.concatenate(tris)[order]  # [nF, 3 corners, 3 coords]
    clin = (T[..., 0] * (n[1] + 1) + T[..., 1]) * (n[2] + 1) + T[..., 2]
    used, F = np.unique(clin.reshape(-1), return_inverse=True)
    F = F.reshape(-1, 3)
    ci = np.stack([used // ((n[1] + 1) * (n[2] + 1)), (used // (n[2] + 1)) % (n[1] + 1), used % (n[2] + 1)], 1)
    lo = np.asarray(grid.lo, np.float64)
    h = (np.asarray(grid.hi, np.float64) - lo) / np.asarray(grid.n, np.float64)
    return lo + ci * h, F


# ---------------------------------------------------------------- marching cubes
#
# The reconstruction the paper names when it motivates its metric (Section 3): the
# surface between field values above a level (inside) and at or below it (outside).
# Derived here from a rule on the cell faces rather than from a printed case table:
#   * on every face of a cell, walking its corners counter-clockwise as seen from outside
#     the cell, the face's crossed edges alternate between entries (outside -> inside)
#     and exits; each entry is joined to the next exit, so where two diagonal corners are
#     inside, the segments cut each inside corner off on its own (both cells sharing the
#     face see the same segments, so the surface is closed);
#   * every crossed cell edge ends one segment and starts one, so the segments close into
#     loops, each started at its lowest local edge number and split into a fan;
#   * the direction of the segments is fixed once so that faces point outward.

def _mc_cell():
    corners = [np.array((a, b, c), np.float64) for c in (0, 1) for b in (0, 1) for a in (0, 1)]  # a + 2b + 4c
    edges = []                                   # local edge -> (corner, corner)
    for axis in range(3):
        o1, o2 = [d for d in range(3) if d != axis]
        for hi2 in (0, 1):
            for hi1 in (0, 1):
                lo_c = [0, 0, 0]
                lo_c[o1], lo_c[o2] = hi1, hi2
                hi_c = list(lo_c)
                hi_c[axis] = 1
                edges.append((lo_c[0] + 2 * lo_c[1] + 4 * lo_c[2], hi_c[0] + 2 * hi_c[1] + 4 * hi_c[2]))
    faces = []                                   # corner lists, counter-clockwise from outside
    for axis in range(3):
        for side in (0, 1):
            n = np.zeros(3)
            n[axis] = 1.0 if side else -1.0
            cs = [i for i in range(8) if corners[i][axis] == side]
            cen = sum(corners[i] for i in cs) / 4
            u = np.zeros(3)
            u[(axis + 1) % 3] = 1.0
            v = np.cross(n, u)
            cs.sort(key=lambda i: np.arctan2((corners[i] - cen) @ v, (corners[i] - cen) @ u))
            faces.append(cs)
    return corners, edges, faces


def _mc_loops(case):
    """Loops of crossed local edges of one inside/outside pattern of the 8 corners,
    each starting at its lowest edge number and following the segments' direction."""
    corners, edges, faces = _mc_cell()
    inside = [(case >> i) & 1 == 1 for i in range(8)]
    edge_of = {frozenset(e): k for k, e in enumerate(edges)}
    succ = {}
    for cs in faces:
        walk = []
        for t in range(4):
            a, b = cs[t], cs[(t + 1) % 4]
            if inside[a] != inside[b]:
                walk.append((edge_of[frozenset((a, b))], inside[b]))   # True: entry
        for t, (e, entry) in enumerate(walk):
            if entry:
                succ[e] = next(walk[(t + s) % len(walk)][0] for s in range(1, len(walk) + 1)
                               if not walk[(t + s) % len(walk)][1])
    loops, seen = [], set()
    for start in sorted(succ):
        if start in seen:
            continue
        loop = [start]
        seen.add(start)
        while succ[loop[-1]] != start:
            loop.append(succ[loop[-1]])
            seen.add(loop[-1])
        loops.append(loop)
    return loops


def _mc_fan(loop):
    """A loop split into a fan from its first vertex whose diagonals all join crossings
    lying on no common cell face (a diagonal inside a face could coincide with the
    neighbouring cell's triangles); one exists for every loop of every pattern."""
    _, edges, faces = _mc_cell()
    on = [{f for f, cs in enumerate(faces) if edges[e][0] in cs and edges[e][1] in cs} for e in loop]
    m = len(loop)
    for s in range(m):
        if all(not (on[s] & on[j]) for j in range(m) if (j - s) % m not in (0, 1, m - 1)):
            r = loop[s:] + loop[:s]
            return [(r[0], r[i], r[i + 1]) for i in range(1, m - 1)]
    raise AssertionError("no valid fan")


_MC_TRIS = {}


def _mc_case(case):
    """Triangles (local edge triples) of one pattern, facing outward."""
    if case not in _MC_TRIS:
        tris = [t for loop in _mc_loops(case) for t in _mc_fan(loop)]
        _MC_TRIS[case] = [(t[0], t[2], t[1]) for t in tris] if _MC_FLIP else tris
    return _MC_TRIS[case]


def _mc_needs_flip():
    """Whether the segment direction gives inward faces: test one corner inside."""
    corners, edges, _ = _mc_cell()
    t = _mc_fan(_mc_loops(1)[0])[0]
    mid = [0.5 * (corners[edges[e][0]] + corners[edges[e][1]]) for e in t]
    return bool(np.cross(mid[1] - mid[0], mid[2] - mid[0]) @ (mid[0] - corners[0]) < 0)


_MC_FLIP = _mc_needs_flip()


def marching_cubes(values, grid, iso: float = 0.5):
    """Marching cubes of a field sampled at the grid's voxel centres (C order), at level
    ``iso`` > 0: the surface between values > iso and values <= iso, the grid surrounded
    by one layer of zeros so that the surface is closed.  Vertices: one per crossed edge
    between neighbouring centres of the padded lattice, at the linear interpolation of
    the two values, numbered by edge (3 * padded lattice index + axis).  Faces: cell by
    cell in padded C order, each cell's triangles in case order, facing outward.
    Returns (V [nV, 3] float64, F [nF, 3] int64)."""
    if not iso > 0:
        raise ValueError("iso must be > 0 (the padding is 0)")
    n = tuple(int(x) for x in grid.n)
    f = np.pad(np.asarray(values, np.float64).reshape(n), 1)
    ins = f > iso
    N = f.shape
    lo = np.asarray(grid.lo, np.float64)
    h = (np.asarray(grid.hi, np.float64) - lo) / np.asarray(n, np.float64)
    flags = np.zeros(N + (3,), bool)
    for axis in range(3):
        sl = [slice(None)] * 3
        sl2 = [slice(None)] * 3
        sl[axis] = slice(0, N[axis] - 1)
        sl2[axis] = slice(1, N[axis])
        fl = [slice(None)] * 3 + [axis]
        fl[axis] = slice(0, N[axis] - 1)
        flags[tuple(fl)] = ins[tuple(sl)] != ins[tuple(sl2)]
    vid = np.cumsum(flags.reshape(-1)) - 1            # vertex id of each crossed edge
    eid = np.flatnonzero(flags.reshape(-1))
    p = eid // 3
    axis = eid % 3
    P = np.stack(np.unravel_index(p, N), 1)
    Q = P.copy()
    Q[np.arange(len(Q)), axis] += 1
    fa, fb = f[tuple(P.T)], f[tuple(Q.T)]
    t = (iso - fa) / (fb - fa)
    V = lo + (P - 1 + 0.5) * h
    V[np.arange(len(V)), axis] += t * h[axis]
    # cells
    C = tuple(x - 1 for x in N)
    case = np.zeros(C, np.int64)
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                case |= ins[a:a + C[0], b:b + C[1], c:c + C[2]].astype(np.int64) << (a + 2 * b + 4 * c)
    _, edges, _ = _mc_cell()
    keys, tris = [], []
    cell_lin = np.arange(case.size).reshape(C)
    for k in np.unique(case):
        tl = _mc_case(int(k))
        if not tl:
            continue
        cells = np.argwhere(case == k)               # C order
        for ti, tri in enumerate(tl):
            g = []
            for e in tri:
                c0, c1 = edges[e]
                off = np.array((c0 & 1, (c0 >> 1) & 1, (c0 >> 2) & 1))
                ax = int(np.flatnonzero(np.array((c1 & 1, (c1 >> 1) & 1, (c1 >> 2) & 1)) - off)[0])
                pt = cells + off
                lin = (pt[:, 0] * N[1] + pt[:, 1]) * N[2] + pt[:, 2]
                g.append(vid[3 * lin + ax])
            tris.append(np.stack(g, 1))
            keys.append(cell_lin[tuple(cells.T)] * 16 + ti)
    if not tris:
        return V, np.zeros((0, 3), np.int64)
    order = np.argsort(np.concatenate(keys), kind="stable")
    return V, np.concatenate(tris)[order].astype(np.int64)


def vertex_neighbours(nV, F):
    """Sorted unique neighbour lists (vertices joined by a face edge), as CSR arrays."""
    F = np.asarray(F, np.int64)
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 0]], F[:, [1, 2]], F[:, [2, 1]], F[:, [2, 0]], F[:, [0, 2]]])
    e = np.unique(e, axis=0)
    e = e[e[:, 0] != e[:, 1]]
    off = np.zeros(nV + 1, np.int64)
    np.add.at(off, e[:, 0] + 1, 1)
    return np.cumsum(off), e[:, 1]


def enclosed_volume(V, F) -> float:
    """Signed volume enclosed by a closed, outward-wound surface: the sum over faces of
    the signed tetrahedra (origin, v0, v1, v2), v0 . (v1 x v2) / 6 (divergence theorem)."""
    V = np.asarray(V, np.float64)
    F = np.asarray(F, np.int64).reshape(-1, 3)
    if len(F) == 0:
        return 0.0
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return float(np.sum(np.einsum("ij,ij->i", a, np.cross(b, c)))) / 6.0


def laplacian_smooth(V, F, lam: float = 0.15, iters: int = 10, keep_volume: bool = True):
    """Laplacian filter of Section 3 (the smoothing applied to each cubified occupancy):
    umbrella operator in Jacobi form, every iteration moving each vertex by lam times
    (mean of its edge neighbours - itself), isolated vertices staying.  With keep_volume
    (the filter's default in the tool the paper names) every iteration is followed by a
    uniform scaling about the origin by (V0 / V)^(1/3), V0 the volume enclosed before the
    first iteration and V the volume after this one, so the enclosed volume stays V0; the
    scaling is skipped when V0 / V is not positive and finite (no enclosed volume)."""
    V = np.array(V, dtype=np.float64)
    off, nbr = vertex_neighbours(len(V), F)
    deg = np.diff(off)
    vol0 = enclosed_volume(V, F) if keep_volume else 0.0
    for _ in range(iters):
        S = np.zeros_like(V)
        for c in range(3):
            S[:, c] = np.add.reduceat(np.concatenate([V[nbr, c], [0.0]]), off[:-1]) if len(nbr) else 0.0
        has = deg > 0
        mean = np.zeros_like(V)
        mean[has] = S[has] / deg[has, None]
        V = np.where(has[:, None], V + lam * (mean - V), V)
        if keep_volume:
            vol = enclosed_volume(V, F)
            ratio = vol0 / vol if vol != 0.0 else 0.0
            if ratio > 0.0 and np.isfinite(ratio):
                V = V * np.cbrt(ratio)
    return V


def face_area_weights(V, F):
    """Integer sampling weights w_f = floor(area_f * 2^32 / max area) (uint64): areas in
    FP64 from the given coordinates, so that face choice is exact integer arithmetic."""
    V = np.asarray(V, np.float64)
    F = np.asarray(F, np.int64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    e1, e2 = b - a, c - a
    cx = e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1]
    cy = e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2]
    cz = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    area = 0.5 * np.sqrt((cx * cx + cy * cy) + cz * cz)
    amax = area.max() if len(area) else 0.0
    if amax <= 0:
        return np.zeros(len(F), np.uint64)
    return np.floor(area * (4294967296.0 / amax)).astype(np.uint64)


def sample_surface(V, F, u):
    """Area-uniform surface samples from uniform numbers u [n, 3] in [0, 1): u0 picks the
    face by inverse CDF of the integer area weights, (u1, u2) the barycentric point
    (reflected into the triangle when u1 + u2 > 1).  Returns (points [n, 3], face ids)."""
    V = np.asarray(V, np.float64)
    F = np.asarray(F, np.int64)
    u = np.asarray(u, np.float64)
    w = face_area_weights(V, F)
    cdf = np.cumsum(w, dtype=np.uint64)
    total = int(cdf[-1])
    t = np.minimum(np.floor(u[:, 0] * float(total)), float(total - 1)).astype(np.uint64)
    f = np.minimum(np.searchsorted(cdf, t, side="right"), len(F) - 1)
    r1, r2 = u[:, 1].copy(), u[:, 2].copy()
    flip = r1 + r2 > 1.0
    r1[flip], r2[flip] = 1.0 - r1[flip], 1.0 - r2[flip]
    a, b, c = V[F[f, 0]], V[F[f, 1]], V[F[f, 2]]
    return a + r1[:, None] * (b - a) + r2[:, None] * (c - a), f


def nn_distances(A, B, threads: int = 0):
    """d[i] = min_j |A_i - B_j| (FP64 brute force)."""
    A, pa = _d(np.asarray(A, np.float64).reshape(-1, 3))
    B, pb = _d(np.asarray(B, np.float64).reshape(-1, 3))
    d = np.empty(len(A))
    if _load().wno_nn_dist(pa, len(A), pb, len(B), d.ctypes.data_as(_dp), threads) != 0:
        raise ValueError("empty point set")
    return d


def chamfer_hausdorff(A, B, threads: int = 0):
    """Chamfer distance mean_a min_b |a-b| + mean_b min_a |a-b| and Hausdorff distance
    max(max_a min_b, max_b min_a) between two point sets."""
    dab, dba = nn_distances(A, B, threads), nn_distances(B, A, threads)
    return float(dab.mean() + dba.mean()), float(max(dab.max(), dba.max()))
