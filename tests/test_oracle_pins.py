"""Pins of the FP64 oracle against results the paper and mathematics fix, not against itself.

Each test names the passage of arXiv 2407.11272 it follows.  Independent formulas
(L'Huilier's spherical excess, quadrature of the flux integral, the Biot-Savart edge
sum, half-space and ray-parity inside tests, finite differences) are written here in
numpy and share nothing with the oracle's C code.
"""
import math

import numpy as np
import pytest

import wn_inputs as wi
from wn_inputs.meshgen import signed_volume

PI = math.pi


# ------------------------------------------------------------ independent refs

def lhuilier_signed(v, q):
    """Signed solid angle of the spherical triangle (L'Huilier), sign from det(e0,e1,e2)."""
    e = [(np.asarray(x, float) - q) / np.linalg.norm(np.asarray(x, float) - q) for x in v]

    def ang(a, b):
        return math.atan2(np.linalg.norm(np.cross(a, b)), float(a @ b))

    a, b, c = ang(e[1], e[2]), ang(e[2], e[0]), ang(e[0], e[1])
    s = 0.5 * (a + b + c)
    t = math.tan(s / 2) * math.tan((s - a) / 2) * math.tan((s - b) / 2) * math.tan((s - c) / 2)
    E = 4.0 * math.atan(math.sqrt(max(t, 0.0)))
    return math.copysign(E, np.linalg.det(np.array(e)))


def flux_quadrature(v, q, n=48):
    """Section 2.1, Eq. 2 on one triangle: integral of <n, (x-q)/|x-q|^3> ds by a
    Duffy-collapsed Gauss-Legendre product rule (returns the solid angle, 4 pi W)."""
    v0, v1, v2 = (np.asarray(x, float) for x in v)
    N = np.cross(v1 - v0, v2 - v0)  # n ds = N du dv
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    S, T = np.meshgrid(g, g, indexing="ij")
    WS, WT = np.meshgrid(w, w, indexing="ij")
    u = S * (1 - T)
    vv = S * T
    X = v0 + u[..., None] * (v1 - v0) + vv[..., None] * (v2 - v0)
    D = X - q
    r3 = np.linalg.norm(D, axis=-1) ** 3
    f = (D @ N) / r3
    return float(np.sum(f * S * WS * WT))


def biot_savart_grad_q(v, q):
    """Gradient of the signed solid angle with respect to the observation point: the
    Biot-Savart sum over the directed boundary edges a -> b with A = a - q, B = b - q."""
    g = np.zeros(3)
    for i in range(3):
        A = np.asarray(v[i], float) - q
        B = np.asarray(v[(i + 1) % 3], float) - q
        a, b = np.linalg.norm(A), np.linalg.norm(B)
        g += np.cross(A, B) * (a + b) / (a * b * (a * b + A @ B))
    return g


def convex_inside(V, F, Q, eps=0.0):
    """Half-space test for a convex outward-wound mesh: inside iff behind every face plane."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, c - a)
    s = np.einsum("qfd,fd->qf", Q[:, None, :] - a[None], n)
    return np.all(s < -eps, axis=1), np.any(s > eps, axis=1)


def ray_parity(V, F, Q, direction=(0.5773502691896258, 0.5773502691896257, 0.5773502691896259)):
    """Crossing count of the ray q + t d (t > 0) with every face (Moller-Trumbore), mod 2."""
    d = np.asarray(direction, float)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    e1, e2 = b - a, c - a
    p = np.cross(d, e2)
    det = np.einsum("fd,fd->f", e1, p)
    out = []
    for q in Q:
        s = q - a
        u = np.einsum("fd,fd->f", s, p) / det
        qq = np.cross(s, e1)
        v = (qq @ d) / det
        t = np.einsum("fd,fd->f", e2, qq) / det
        hit = (u > 0) & (v > 0) & (u + v < 1) & (t > 0)
        out.append(int(hit.sum()) % 2)
    return np.array(out)


# ------------------------------------------------------------------- Eq. 8

def test_atan2_eq8_case_table(orc):
    """Section 2.2, Eq. 8: every branch of the case table at points with known angles."""
    assert orc.atan2_eq8(1.0, 1.0) == pytest.approx(PI / 4, abs=1e-15)
    assert orc.atan2_eq8(1.0, -1.0) == pytest.approx(3 * PI / 4, abs=1e-15)
    assert orc.atan2_eq8(-1.0, -1.0) == pytest.approx(-3 * PI / 4, abs=1e-15)
    assert orc.atan2_eq8(-1.0, 1.0) == pytest.approx(-PI / 4, abs=1e-15)
    assert orc.atan2_eq8(2.0, 0.0) == PI / 2
    assert orc.atan2_eq8(-2.0, 0.0) == -PI / 2
    assert orc.atan2_eq8(2.0, -0.0) == PI / 2
    # x = 0, y = 0 gives 0 whatever the signs of the zeros
    for y in (0.0, -0.0):
        for x in (0.0, -0.0):
            assert orc.atan2_eq8(y, x) == 0.0
    # x < 0 and y = 0: the y >= 0 branch, +pi, also for y = -0 (-0 >= 0 holds)
    assert orc.atan2_eq8(0.0, -3.0) == pytest.approx(PI, abs=1e-15)
    assert orc.atan2_eq8(-0.0, -3.0) == pytest.approx(PI, abs=1e-15)
    # agrees with the library atan2 away from the zero cases
    rng = np.random.default_rng(11)
    for y, x in rng.normal(size=(200, 2)):
        assert orc.atan2_eq8(y, x) == pytest.approx(math.atan2(y, x), abs=1e-15)


# ------------------------------------------------------------- closed forms

def test_octant_triangle_is_one_eighth(orc):
    """Eq. 7 with the half-angle factor 2: the triangle (e_x, e_y, e_z) seen from the
    origin subtends one octant, Omega = 4 pi / 8, so W = 1/8."""
    v = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
    q = [0, 0, 0]
    a, b = orc.alpha_beta(*v, q)
    assert a == pytest.approx(1.0, abs=1e-15) and b == pytest.approx(1.0, abs=1e-15)
    assert orc.solid_angle(*v, q) == pytest.approx(4 * PI / 8, abs=1e-15)
    assert orc.winding(np.array(v, float), np.array([[0, 1, 2]]), [q])[0] == pytest.approx(1 / 8, abs=1e-15)
    # scaled vertices, same directions: same solid angle
    assert orc.solid_angle([3, 0, 0], [0, 0.5, 0], [0, 0, 7], q) == pytest.approx(PI / 2, abs=1e-14)
    # cyclic relabelling keeps it, a swap flips it
    assert orc.solid_angle(v[1], v[2], v[0], q) == pytest.approx(PI / 2, abs=1e-15)
    assert orc.solid_angle(v[0], v[2], v[1], q) == pytest.approx(-PI / 2, abs=1e-15)


def test_regular_solids_from_centre(orc):
    """Eq. 3: a closed surface has W = 1 at interior points; each octahedron face is an octant."""
    V, F = wi.octahedron_mesh(1.0)
    assert signed_volume(V, F) > 0
    for f in F:
        assert orc.solid_angle(*V[f], [0, 0, 0]) == pytest.approx(PI / 2, abs=1e-14)
    W = orc.winding(V, F, [[0, 0, 0], [0.2, -0.1, 0.3], [1.5, 0, 0], [0.0, 0.0, -4.0]])
    np.testing.assert_allclose(W, [1, 1, 0, 0], atol=1e-14)


def test_cube_special_positions(orc):
    """Eq. 8 zeros and the vertex reading: on the closed unit cube,
    centre -> 1; a vertex -> 1/8 (octant, the incident faces give 0);
    an edge midpoint -> 1/4 (dihedral angle pi/2, the two incident faces give 0);
    a face centre, which lies on that face's diagonal -> 1/2 (half-space)."""
    V, F = wi.cube_mesh(0.0, 1.0)
    assert signed_volume(V, F) == pytest.approx(1.0)
    Q = [[0.5, 0.5, 0.5], [0, 0, 0], [1, 1, 1], [0.5, 0, 0], [0, 1, 0.5], [0.5, 0.5, 0], [1, 0.5, 0.5],
         [3, 3, 3]]
    W = orc.winding(V, F, Q)
    np.testing.assert_allclose(W, [1, 1 / 8, 1 / 8, 1 / 4, 1 / 4, 1 / 2, 1 / 2, 0], atol=1e-14)


def test_vertex_and_edge_faces_contribute_zero(orc):
    """A face with q at one of its vertices gives 0 (unit vector of a zero vector taken
    as 0, then ATAN2(0, beta >= 0) = 0); q on an edge gives alpha = beta = 0 -> 0."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        v = rng.normal(size=(3, 3))
        for j in range(3):
            assert orc.solid_angle(*v, v[j]) == 0.0
        # midpoint of an edge with exactly representable coordinates
        a = np.round(rng.normal(size=3) * 8) / 8
        b = a + np.array([0.5, 0.0, 0.0])
        c = rng.normal(size=3)
        assert orc.solid_angle(a, b, c, (a + b) / 2) == 0.0


def test_degenerate_face_contributes_nothing(orc):
    """A collinear (zero-area) face subtends no solid angle from any point."""
    rng = np.random.default_rng(6)
    for _ in range(50):
        a = rng.normal(size=3)
        d = rng.normal(size=3)
        v = [a, a + 0.3 * d, a + 1.1 * d]
        q = rng.normal(size=3) * 2
        assert abs(orc.solid_angle(*v, q)) < 1e-12


# ------------------------------------------------------- independent formulas

def test_lhuilier_spherical_excess(orc):
    """Per-triangle Omega equals L'Huilier's spherical excess of the projected triangle,
    signed by det(e0, e1, e2)."""
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(300):
        v = rng.normal(size=(3, 3))
        q = rng.normal(size=3) * 1.5
        worst = max(worst, abs(orc.solid_angle(*v, q) - lhuilier_signed(v, q)))
    assert worst < 1e-10


def test_flux_quadrature_eq2(orc):
    """Section 2.1, Eq. 2: the flux integral over a triangle, computed by quadrature,
    converges to the closed-form solid angle for points not close to the triangle."""
    rng = np.random.default_rng(8)
    for _ in range(40):
        v = rng.normal(size=(3, 3)) * 0.3
        dirn = rng.normal(size=3)
        q = v.mean(0) + dirn / np.linalg.norm(dirn) * rng.uniform(1.0, 3.0)
        assert orc.solid_angle(*v, q) == pytest.approx(flux_quadrature(v, q), abs=1e-10)


# ------------------------------------------------------------- Eq. 3 pins

def test_closed_icosphere_is_occupancy(orc):
    """Eq. 3: W of a closed surface is 1 inside and 0 outside.  The inside set comes
    from an independent half-space test (the icosphere is convex)."""
    V, F = wi.icosphere(2)
    rng = np.random.default_rng(9)
    Q = rng.uniform(-1.3, 1.3, size=(600, 3))
    inside, outside = convex_inside(V, F, Q, eps=1e-6)
    W = orc.winding(V, F, Q)
    assert inside.sum() > 50 and outside.sum() > 50
    np.testing.assert_allclose(W[inside], 1.0, atol=1e-12)
    np.testing.assert_allclose(W[outside], 0.0, atol=1e-12)


def test_nonconvex_closed_mesh_matches_ray_parity(orc):
    """Eq. 3 on a non-convex closed mesh (heavily jittered icosphere): W equals the
    crossing parity of a ray, an independent inside test."""
    rng = np.random.default_rng(10)
    V, F = wi.icosphere(2)
    V = V * (1.0 + 0.25 * rng.uniform(-1, 1, size=(len(V), 1)))
    Q = rng.uniform(-1.2, 1.2, size=(400, 3))
    W = orc.winding(V, F, Q)
    par = ray_parity(V, F, Q)
    np.testing.assert_allclose(W, par, atol=1e-10)


def test_overlapping_shells_count(orc):
    """Overlapping closed shells (the union workload before face deletion): W counts
    how many shells contain the point; each shell is convex, so a half-space test per
    shell gives the count independently."""
    rng = np.random.default_rng(12)
    V, F, ells = wi.ellipsoid_union(rng, 4, 200, axes=(0.15, 0.4), centres=(-0.15, 0.15))
    Q = rng.uniform(-0.5, 0.5, size=(500, 3))
    W = orc.winding(V, F, Q)
    faces_per = len(F) // 4
    count = np.zeros(len(Q))
    sure = np.ones(len(Q), dtype=bool)
    for s in range(4):
        Fs = F[s * faces_per:(s + 1) * faces_per]
        ins, outs = convex_inside(V, Fs, Q, eps=1e-9)
        count += ins
        sure &= ins | outs
    assert W.max() > 1.5  # some points really are inside several shells
    np.testing.assert_allclose(W[sure], count[sure], atol=1e-10)


def test_orientation_flip_negates(orc):
    """Reversing every face reverses the normal in Eq. 2, so W -> -W."""
    c1 = wi.config1_icosphere()
    rng = np.random.default_rng(13)
    Q = rng.uniform(-0.5, 0.5, size=(300, 3))
    W = orc.winding(c1.V, c1.F, Q)
    Wr = orc.winding(c1.V, wi.reverse_faces(c1.F), Q)
    np.testing.assert_allclose(Wr, -W, atol=1e-12)


def test_rigid_and_scale_invariance_and_mirror(orc):
    """W is invariant under a joint rotation, translation and positive scaling of mesh
    and points; a mirror reverses orientation, so W -> -W."""
    rng = np.random.default_rng(14)
    V, F, _ = wi.ellipsoid_union(rng, 3, 300)
    Q = rng.uniform(-0.5, 0.5, size=(200, 3))
    W = orc.winding(V, F, Q)
    R = wi.random_rotation(rng)
    t = rng.normal(size=3)
    s = 2.7
    W2 = orc.winding(s * V @ R.T + t, F, s * Q @ R.T + t)
    np.testing.assert_allclose(W2, W, atol=1e-11)
    M = np.diag([-1.0, 1.0, 1.0])
    W3 = orc.winding(V @ M, F, Q @ M)
    np.testing.assert_allclose(W3, -W, atol=1e-11)


def test_open_mesh_is_fractional(orc):
    """A single hemisphere shell: points on the axis see the fraction of the sphere it
    covers; far below the opening W -> 0; at the centre exactly 1/2 (half of the sphere)."""
    V, F = wi.uv_ellipsoid(64, 32)
    cen = (V[F].mean(1))
    Fh = F[cen[:, 2] > 0]  # upper hemisphere (latitude bands split evenly at the equator)
    W = orc.winding(V, Fh, [[0, 0, 0]])
    assert W[0] == pytest.approx(0.5, abs=1e-12)


def test_grid_point_layout(orc):
    """Voxel centres lo + (idx + 1/2)(hi - lo)/n in C order (z fastest)."""
    g = wi.Grid((-1.0, 0.0, 2.0), (1.0, 4.0, 3.0), (4, 2, 8))
    Q = orc.grid_points(g)
    assert Q.shape == (64, 3)
    idx = wi.grid_flat_index(g, 3, 1, 5)
    np.testing.assert_allclose(Q[idx], [-1 + 3.5 * 0.5, 0 + 1.5 * 2.0, 2 + 5.5 / 8])
    np.testing.assert_allclose(Q[1] - Q[0], [0, 0, 1 / 8])


# ------------------------------------------------------------------ gradient

def test_gradient_vs_central_differences(orc):
    """Analytic dOmega/dv_j against FP64 central differences of the oracle's Omega
    and of L'Huilier's (independent) Omega."""
    rng = np.random.default_rng(15)
    h = 1e-6
    for _ in range(60):
        v = rng.normal(size=(3, 3))
        q = rng.normal(size=3)
        G = orc.solid_angle_grad(*v, q)
        fd = np.zeros((3, 3))
        fd2 = np.zeros((3, 3))
        for j in range(3):
            for c in range(3):
                vp, vm = v.copy(), v.copy()
                vp[j, c] += h
                vm[j, c] -= h
                fd[j, c] = (orc.solid_angle(*vp, q) - orc.solid_angle(*vm, q)) / (2 * h)
                fd2[j, c] = (lhuilier_signed(vp, q) - lhuilier_signed(vm, q)) / (2 * h)
        scale = max(1.0, np.abs(fd).max())
        assert np.abs(G - fd).max() < 1e-6 * scale
        assert np.abs(G - fd2).max() < 1e-6 * scale


def test_gradient_translation_identity_biot_savart(orc):
    """Moving all three vertices by d equals moving q by -d, so sum_j dOmega/dv_j =
    -grad_q Omega, and grad_q Omega is the Biot-Savart sum over the boundary edges."""
    rng = np.random.default_rng(16)
    for _ in range(100):
        v = rng.normal(size=(3, 3))
        q = rng.normal(size=3)
        G = orc.solid_angle_grad(*v, q)
        np.testing.assert_allclose(G.sum(0), -biot_savart_grad_q(v, q), atol=1e-11, rtol=1e-9)


def test_gradient_special_cases_zero(orc):
    """q at a vertex or on an edge: the face contributes 0 to the gradient."""
    rng = np.random.default_rng(17)
    v = rng.normal(size=(3, 3))
    assert np.all(orc.solid_angle_grad(*v, v[1]) == 0.0)
    a = np.array([0.25, 0.5, -0.75])
    b = a + np.array([0.0, 0.5, 0.0])
    assert np.all(orc.solid_angle_grad(a, b, rng.normal(size=3), (a + b) / 2) == 0.0)


def test_closed_mesh_vertex_gradient_vanishes(orc):
    """W of a surface depends only on its boundary curve, so for a closed mesh every
    vertex gradient is 0 (the paper notes the vanishing gradients of the binary field,
    Section 2.4), while per-corner terms are not."""
    c = wi.config1_icosphere()
    rng = np.random.default_rng(18)
    Q = rng.uniform(-0.5, 0.5, size=(64, 3))
    g = rng.normal(size=64)
    T, D = orc.grad(c.V, c.F, Q, g)
    corner_scale = np.zeros((len(c.V), 3))
    np.add.at(corner_scale, c.F.reshape(-1), np.abs(T.reshape(-1, 3)))
    assert np.abs(T).max() > 1e-3
    assert np.all(np.abs(D) <= 1e-9 * corner_scale + 1e-14)


def test_open_mesh_gradient_vs_finite_differences(orc):
    """Open mesh: dL/dV of L = sum_q g_q W_q matches central differences of the oracle's
    W, and only vertices on the hole rims carry gradient."""
    rng = np.random.default_rng(19)
    V, F = wi.icosphere(1)
    F = wi.delete_faces(F, 6, rng)
    Q = rng.uniform(-1.2, 1.2, size=(40, 3))
    g = rng.normal(size=40)
    _, D = orc.grad(V, F, Q, g)
    h = 1e-6
    fd = np.zeros_like(V)
    for i in range(len(V)):
        for c in range(3):
            Vp, Vm = V.copy(), V.copy()
            Vp[i, c] += h
            Vm[i, c] -= h
            fd[i, c] = (g @ orc.winding(Vp, F, Q) - g @ orc.winding(Vm, F, Q)) / (2 * h)
    np.testing.assert_allclose(D, fd, atol=1e-6)
    # boundary (rim) vertices: those on an edge used by exactly one face
    from collections import Counter
    cnt = Counter()
    for f in F:
        for j in range(3):
            a, b = f[j], f[(j + 1) % 3]
            cnt[(min(a, b), max(a, b))] += 1
    rim = set()
    for (a, b), n in cnt.items():
        if n == 1:
            rim |= {a, b}
    interior = np.array([i for i in range(len(V)) if i not in rim and i in set(F.reshape(-1))])
    assert np.abs(D[interior]).max() < 1e-9
    assert np.abs(D[sorted(rim)]).max() > 1e-3


# ------------------------------------------------------------ guard distances

def test_distance_functions(orc):
    """Point-to-edge and point-to-face distances against closed forms and dense sampling."""
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    F = np.array([[0, 1, 2]])
    de, df = orc.min_dist(V, F, [[0.2, 0.2, 0.5], [2, 0, 0], [0.5, 0.5, 0.0], [-1, -1, 0]])
    np.testing.assert_allclose(df, [0.5, 1.0, 0.0, math.sqrt(2)], atol=1e-15)
    np.testing.assert_allclose(de, [math.sqrt(0.04 + 0.25), 1.0, 0.0, math.sqrt(2)], atol=1e-15)
    rng = np.random.default_rng(20)
    v = rng.normal(size=(3, 3))
    u = rng.uniform(size=(200000, 2))
    u = np.where(u.sum(1, keepdims=True) > 1, 1 - u, u)
    S = v[0] + u[:, :1] * (v[1] - v[0]) + u[:, 1:] * (v[2] - v[0])
    for q in rng.normal(size=(10, 3)):
        _, d = orc.min_dist(v, F, [q])
        ds = np.linalg.norm(S - q, axis=1).min()
        assert d[0] <= ds + 1e-12 and ds - d[0] < 5e-3


# ---------------------------------------------------------------- occupancy

def test_occupancy_maps(orc):
    """Hard map is strict (W = tau -> 0); the soft map is 1/2 at tau; sigmoid-MSE
    gradient against central differences."""
    W = np.array([0.0, 0.5, 0.5000001, 1.0, 2.0, -1.0])
    np.testing.assert_array_equal(orc.occupancy_threshold(W), [0, 0, 1, 1, 1, 0])
    assert orc.occupancy_sigmoid([0.5])[0] == 0.5
    rng = np.random.default_rng(21)
    W = rng.uniform(0.3, 0.7, 50)
    t = (rng.uniform(size=50) > 0.5).astype(float)
    _, g = orc.sigmoid_mse(W, t, 0.5, 50.0)
    h = 1e-6
    for i in range(0, 50, 7):
        Wp, Wm = W.copy(), W.copy()
        Wp[i] += h
        Wm[i] -= h
        fd = (orc.sigmoid_mse(Wp, t)[0] - orc.sigmoid_mse(Wm, t)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=5e-3, abs=1e-12)


def test_thread_count_does_not_change_results(orc):
    c = wi.config1_icosphere()
    rng = np.random.default_rng(22)
    Q = rng.uniform(-0.5, 0.5, size=(100, 3))
    a = orc.winding(c.V, c.F, Q, threads=1)
    b = orc.winding(c.V, c.F, Q, threads=4)
    np.testing.assert_array_equal(a, b)


# ---------------------------------------------------- flipping duplication

def test_vertex_normals_closed_forms(orc):
    """Regular octahedron: each vertex's four faces have equal area, so its normal is
    the axis direction; icosphere normals converge to the radial direction."""
    V, F = wi.octahedron_mesh(1.0)
    np.testing.assert_allclose(orc.vertex_normals(V, F), V, atol=1e-15)
    errs = []
    for s in (2, 3, 4):
        V, F = wi.icosphere(s)
        N = orc.vertex_normals(V, F)
        assert np.abs(np.linalg.norm(N, axis=1) - 1).max() < 1e-14
        errs.append(np.abs(N - V).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-2


def test_vertex_normals_are_area_weighted(orc):
    """A vertex shared by two faces of unequal area: the right-angled faces
    (0, e_x, e_y) (normal e_z, |N| = 1) and (0, 3 e_y, e_z) (normal e_x, |N| = 3) give
    vertex 0 the normal (3, 0, 1) / sqrt(10); uniform or angle weights (both corner
    angles are right angles) would give (1, 0, 1) / sqrt(2).  Algorithm 2 moves the copy
    of vertex 0 by -eps times that normal and reverses the copied faces."""
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 3, 0], [0, 0, 1]], float)
    F = np.array([[0, 1, 2], [0, 3, 4]])
    N = orc.vertex_normals(V, F)
    np.testing.assert_allclose(N[0], np.array([3.0, 0.0, 1.0]) / math.sqrt(10), atol=1e-15)
    np.testing.assert_allclose(N[1], [0, 0, 1], atol=1e-15)
    np.testing.assert_allclose(N[3], [1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(N[2], [0, 0, 1], atol=1e-15)
    V2, F2 = orc.flip_duplicate(V, F, 0.05)
    np.testing.assert_allclose(V2[5], -0.05 * np.array([3.0, 0.0, 1.0]) / math.sqrt(10), atol=1e-15)
    np.testing.assert_array_equal(V2[:5], V)
    np.testing.assert_array_equal(F2, [[0, 1, 2], [0, 3, 4], [5, 7, 6], [5, 9, 8]])


def test_flip_duplicate_of_octahedron_is_a_shell(orc):
    """Algorithm 2 on the closed octahedron: V' = (1 - eps) V exactly, so Sigma^-2 is the
    octahedron minus a concentric one: W = 1 in the slab between them, 0 inside the
    inner one and outside (the octahedron is |x|+|y|+|z| <= 1)."""
    V, F = wi.octahedron_mesh(1.0)
    eps = 0.1
    V2, F2 = orc.flip_duplicate(V, F, eps)
    np.testing.assert_allclose(V2[6:], (1 - eps) * V, atol=1e-15)
    assert np.array_equal(F2[8:], F[:, [0, 2, 1]] + 6)
    rng = np.random.default_rng(30)
    Q = rng.uniform(-1.1, 1.1, size=(2000, 3))
    l1 = np.abs(Q).sum(1)
    sure = (np.abs(l1 - 1) > 1e-6) & (np.abs(l1 - (1 - eps)) > 1e-6)
    expect = ((l1 < 1) & (l1 > 1 - eps)).astype(float)
    W = orc.winding(V2, F2, Q)
    np.testing.assert_allclose(W[sure], expect[sure], atol=1e-10)


def test_flip_duplicate_closes_an_open_hemisphere(orc):
    """An open hemisphere shell: alone it gives fractional W; after flipping duplication
    W is ~1 inside the eps-thin slit under the shell and ~0 away from it (Algorithm 2)."""
    V, F = wi.uv_ellipsoid(64, 32, semi_axes=(0.4, 0.4, 0.4))
    cen = V[F].mean(1)
    F = F[cen[:, 2] > 0]
    V2, F2 = orc.flip_duplicate(V, F, 0.02)
    # on the pole axis: inside the slit (radius 0.39), below it (0.3), above (0.45)
    W = orc.winding(V2, F2, [[0, 0, 0.39], [0, 0, 0.3], [0, 0, 0.45], [0, 0, -0.2]])
    assert W[0] == pytest.approx(1.0, abs=2e-2)
    assert abs(W[1]) < 2e-2 and abs(W[2]) < 2e-2 and abs(W[3]) < 2e-2
    Wopen = orc.winding(V, F, [[0, 0, 0.3]])
    assert 0.1 < Wopen[0] < 0.9


# ---------------------------------------------------- naive integral (Eq. 4)

def test_naive_integral_far_field_is_the_solid_angle(orc):
    """Eq. 4 far from a triangle: the centroid sample of the flux integral is the dipole
    limit of the solid angle; the relative error falls like (size / distance)^2."""
    rng = np.random.default_rng(40)
    for _ in range(10):
        v = rng.normal(size=(3, 3)) * 0.1
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        errs = []
        for dist in (2.0, 4.0, 8.0):
            q = v.mean(0) + dist * d
            wn_ = orc.winding_naive(v, [[0, 1, 2]], [q])[0]
            ex = orc.solid_angle(*v, q) / (4 * PI)
            errs.append(abs(wn_ / ex - 1))
        assert errs[2] < 1e-3
        assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_naive_integral_converges_under_refinement(orc):
    """Eq. 4 is accurate for well-shaped meshes away from the surface (Section 2.1): on
    icospheres of increasing subdivision the error against the exact W shrinks about
    4x per level at interior and exterior points."""
    Q = np.array([[0, 0, 0], [0.3, 0.2, -0.1], [0.0, 0.55, 0.1], [1.6, 0, 0], [0.7, 0.8, 0.6]])
    errs = []
    for s in (2, 3, 4):
        V, F = wi.icosphere(s)
        errs.append(np.abs(orc.winding_naive(V, F, Q) - orc.winding(V, F, Q)).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0 and errs[2] < 2e-3


def test_naive_integral_orientation_and_scale(orc):
    """The sum is linear in the normals (reversal negates it) and invariant under a joint
    scaling of mesh and points; a point at a centroid contributes 0 for that face."""
    V, F = wi.icosphere(2)
    rng = np.random.default_rng(41)
    Q = rng.uniform(-1.2, 1.2, size=(50, 3))
    W = orc.winding_naive(V, F, Q)
    np.testing.assert_allclose(orc.winding_naive(V, wi.reverse_faces(F), Q), -W, atol=1e-12)
    np.testing.assert_allclose(orc.winding_naive(3 * V, F, 3 * Q), W, atol=1e-12)
    c = V[F[0]].mean(0)
    single = orc.winding_naive(V, F[:1], [c])
    assert single[0] == 0.0
    W, S = orc.winding_naive(V, F, Q, with_scale=True)
    assert np.all(S >= np.abs(W) - 1e-15)


def test_naive_gradient_vs_finite_differences(orc):
    """Analytic gradient of one Eq. 4 term and of the summed field against FP64 central
    differences."""
    rng = np.random.default_rng(42)
    h = 1e-6
    for _ in range(30):
        v = rng.normal(size=(3, 3))
        q = rng.normal(size=3) * 2
        G = orc.naive_term_grad(*v, q)
        fd = np.zeros((3, 3))
        for j in range(3):
            for c in range(3):
                vp, vm = v.copy(), v.copy()
                vp[j, c] += h
                vm[j, c] -= h
                fp = orc.winding_naive(vp, [[0, 1, 2]], [q])[0] * 8 * PI
                fm = orc.winding_naive(vm, [[0, 1, 2]], [q])[0] * 8 * PI
                fd[j, c] = (fp - fm) / (2 * h)
        assert np.abs(G - fd).max() < 1e-6 * max(1.0, np.abs(fd).max())
    V, F = wi.icosphere(1)
    Q = rng.uniform(-1.0, 1.0, size=(20, 3))
    g = rng.normal(size=20)
    T, D = orc.grad_naive(V, F, Q, g)
    fdV = np.zeros_like(V)
    for i in range(len(V)):
        for c in range(3):
            Vp, Vm = V.copy(), V.copy()
            Vp[i, c] += h
            Vm[i, c] -= h
            fdV[i, c] = (g @ orc.winding_naive(Vp, F, Q) - g @ orc.winding_naive(Vm, F, Q)) / (2 * h)
    np.testing.assert_allclose(D, fdV, atol=1e-6 * np.abs(fdV).max())
    # unlike the exact field, the naive field has non-zero vertex gradients on a closed mesh
    assert np.abs(D).max() > 1e-3


# ------------------------------------------------ morphing loop (Section 2.4)

def test_adam_first_and_constant_gradient_steps(orc):
    """Adam's bias correction makes the first step, and every step under a constant
    gradient, exactly lr g / (|g| + eps) (m_hat = g, v_hat = g^2 at every t)."""
    rng = np.random.default_rng(31)
    g = rng.normal(size=50) * 10.0 ** rng.uniform(-3, 3, size=50)
    x = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 0.01, 1e-8
    for t in range(1, 8):
        x2, m, v = orc.adam(x, g, m, v, t, lr, 0.9, 0.999, eps)
        np.testing.assert_allclose(x - x2, lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15)
        x = x2


def test_adam_alternating_gradient_closed_form(orc):
    """g = +1 then -1 from a zero state: m_hat_2 = -(1 - b1)/(1 + b1) and v_hat_2 = 1,
    so the second step moves x by +lr (1 - b1) / ((1 + b1)(1 + eps))."""
    for b1, b2 in ((0.9, 0.999), (0.5, 0.9), (0.0, 0.99)):
        x1, m, v = orc.adam([0.0], [1.0], [0.0], [0.0], 1, 0.1, b1, b2, 1e-3)
        x2, _, _ = orc.adam(x1, [-1.0], m, v, 2, 0.1, b1, b2, 1e-3)
        assert abs((x2[0] - x1[0]) - 0.1 * (1 - b1) / ((1 + b1) * (1 + 1e-3))) < 1e-12


def test_adam_eps_outside_the_root(orc):
    """eps is added to sqrt(v_hat), not under it: for |g| << eps the step is lr g / eps."""
    x, _, _ = orc.adam([0.0], [1e-12], [0.0], [0.0], 1, 1.0, 0.9, 0.999, 1e-6)
    assert abs(-x[0] - 1e-12 / (1e-12 + 1e-6)) < 1e-15


def test_adam_minimises_a_quadratic(orc):
    """On f(x) = sum a_i x_i^2, Adam with a decaying step reaches the minimum."""
    rng = np.random.default_rng(32)
    a = 10.0 ** rng.uniform(-2, 2, size=20)
    x = rng.normal(size=20)
    m = np.zeros(20)
    v = np.zeros(20)
    for t in range(1, 3001):
        x, m, v = orc.adam(x, 2 * a * x, m, v, t, 0.1 / math.sqrt(t))
    assert np.abs(x).max() < 1e-2


def _recover_gradient(dx, lr, eps):
    """Invert the first Adam step with beta1 = beta2 = 0 (m_hat = g, v_hat = g^2):
    dx = -lr g / (|g| + eps)  =>  g = -eps (dx/lr) / (1 - |dx/lr|)."""
    u = dx / lr
    return -eps * u / (1.0 - np.abs(u))


@pytest.mark.parametrize("integral", ["naive", "gwn"])
def test_morph_step_follows_the_loss_gradient(orc, integral):
    """One morphing iteration moves the vertices by Adam's step on dL/dV, where L is the
    soft-occupancy MSE of the voxelized mesh: the gradient recovered from the step agrees
    with central differences of L.  The exact (GWN) field needs an open mesh: on a closed
    mesh its vertex gradient vanishes (the paper's reason to morph with Eq. 4)."""
    V, F = wi.octahedron_mesh(1.0)
    V = V + np.random.default_rng(33).normal(scale=0.05, size=V.shape)
    if integral == "gwn":
        F = F[1:]
    grid = wi.Grid.cube(6, -1.6, 1.6)
    Q = orc.grid_points(grid)
    target = (np.linalg.norm(Q, axis=1) < 0.8).astype(np.float64)
    k, lr, eps = 4.0, 1e-3, 1.0
    fwd = orc.winding_naive if integral == "naive" else orc.winding
    V1, _, _, losses = orc.morph(V, F, grid, target, 1, integral=integral, k=k, lr=lr, beta1=0.0, beta2=0.0, eps=eps)
    L0, _ = orc.sigmoid_mse(fwd(V, F, Q), target, 0.5, k)
    assert abs(losses[0] - L0) < 1e-15
    g = _recover_gradient(V1 - V, lr, eps)
    h = 1e-6
    fd = np.zeros_like(V)
    for i in range(len(V)):
        for c in range(3):
            Vp, Vm = V.copy(), V.copy()
            Vp[i, c] += h
            Vm[i, c] -= h
            fd[i, c] = (orc.sigmoid_mse(fwd(Vp, F, Q), target, 0.5, k)[0]
                        - orc.sigmoid_mse(fwd(Vm, F, Q), target, 0.5, k)[0]) / (2 * h)
    assert np.abs(fd).max() > 1e-4
    np.testing.assert_allclose(g, fd, atol=1e-6 * np.abs(fd).max() + 1e-9)


def test_morph_first_step_is_a_sign_step(orc):
    """From zero moments, the first iteration is Adam step t = 1: with the default betas
    every coordinate whose gradient exceeds eps moves by lr (m_hat = g, v_hat = g^2)."""
    V, F = wi.octahedron_mesh(1.0)
    V = V + np.random.default_rng(34).normal(scale=0.05, size=V.shape)
    grid = wi.Grid.cube(6, -1.6, 1.6)
    target = (np.linalg.norm(orc.grid_points(grid), axis=1) < 0.8).astype(np.float64)
    V1, _, _, _ = orc.morph(V, F, grid, target, 1, integral="naive", k=4.0, lr=1e-3, eps=1e-14)
    np.testing.assert_allclose(np.abs(V1 - V), 1e-3, rtol=1e-6)


def test_morph_lowers_the_loss(orc):
    """Small steps along the naive-integral gradient lower the voxel loss: a sphere
    morphing towards an ellipsoid target."""
    c = wi.config3_differentiable(res=12)
    _, _, _, losses = orc.morph(c.V, c.F, c.grid, c.target, 6, integral="naive", lr=2e-3)
    assert np.all(np.diff(losses) < 0)


# ------------------------------------------------ evaluation chain (Section 3)

def _edge_use_counts(F):
    e = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    return cnt


def test_cubify_single_voxel_and_block(orc):
    """One voxel gives the 8-corner, 12-triangle cube; an a x b x c block gives a closed
    box of area 2(ab + bc + ca) h^2 and volume abc h^3."""
    g = wi.Grid((0.0, 0.0, 0.0), (2.0, 3.0, 4.0), (4, 6, 8))  # h = 0.5 on every axis
    occ = np.zeros((4, 6, 8), np.uint8)
    occ[0, 0, 0] = 1
    V, F = orc.cubify(occ, g)
    assert V.shape == (8, 3) and F.shape == (12, 3)
    assert abs(signed_volume(V, F) - 0.125) < 1e-15
    assert np.all(_edge_use_counts(F) == 2)
    occ[:] = 0
    occ[1:3, 2:5, 3:7] = 1  # 2 x 3 x 4 voxels
    V, F = orc.cubify(occ, g)
    a, b, c = 2, 3, 4
    area = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1).sum()
    assert abs(area - 2 * (a * b + b * c + c * a) * 0.25) < 1e-12
    assert abs(signed_volume(V, F) - a * b * c * 0.125) < 1e-12
    assert np.all(_edge_use_counts(F) == 2)
    assert len(F) == 2 * 2 * (a * b + b * c + c * a)


def test_cubify_winding_number_is_the_occupancy(orc):
    """Eq. 3 applied to the cube surface: its winding number at every voxel centre is
    exactly that voxel's occupancy, for random occupancy (non-manifold contacts and
    grid-boundary voxels included).  Fixes orientation, completeness and placement."""
    rng = np.random.default_rng(51)
    for shape, p in (((6, 5, 4), 0.5), ((7, 3, 9), 0.3), ((5, 5, 5), 0.9)):
        g = wi.Grid((-1.0, -0.5, 0.0), (1.0, 0.5, 2.0), shape)
        occ = (rng.random(shape) < p).astype(np.uint8)
        V, F = orc.cubify(occ, g)
        W = orc.winding(V, F, orc.grid_points(g))
        assert np.abs(W - occ.reshape(-1)).max() < 1e-12
        # one quad (two triangles) per occupied voxel face next to empty or outside
        pad = np.pad(occ.astype(bool), 1)
        inner = pad[1:-1, 1:-1, 1:-1]
        n_quads = sum(int(np.sum(inner & ~np.roll(pad, s, ax)[1:-1, 1:-1, 1:-1]))
                      for ax in range(3) for s in (1, -1))
        assert len(F) == 2 * n_quads
    V, F = orc.cubify(np.zeros((3, 3, 3), np.uint8), wi.Grid.cube(3))
    assert V.shape == (0, 3) and F.shape == (0, 3)


def _directed_edges_pair_up(F):
    """Every directed edge is used once and its reverse once: a closed, consistently
    oriented 2-manifold (no edge shared by more than two faces)."""
    d = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    u, cnt = np.unique(d, axis=0, return_counts=True)
    rev = set(map(tuple, u[:, ::-1]))
    return bool(np.all(cnt == 1)) and all(tuple(x) in rev for x in u)


def _components(nV, F):
    parent = list(range(nV))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for a, b, c in F:
        for u, v in ((a, b), (b, c)):
            ru, rv = find(int(u)), find(int(v))
            if ru != rv:
                parent[ru] = rv
    return len({find(int(x)) for x in np.unique(F)})


def test_marching_cubes_separates_inside_from_outside(orc):
    """For random fields the surface is a closed oriented 2-manifold, and its winding
    number at every voxel centre is exactly [value > iso] (Eq. 3): it separates the
    centres and faces outward, grid-boundary voxels included."""
    orc._MC_TRIS.clear()
    rng = np.random.default_rng(52)
    for shape, iso in (((6, 5, 4), 0.5), ((3, 7, 5), 0.3), ((5, 5, 5), 0.8), ((2, 2, 2), 0.5)):
        g = wi.Grid((-1.0, -0.5, 0.0), (1.0, 0.5, 2.0), shape)
        f = rng.random(shape)
        V, F = orc.marching_cubes(f, g, iso)
        assert _directed_edges_pair_up(F)
        W = orc.winding(V, F, orc.grid_points(g))
        assert np.abs(W - (f.reshape(-1) > iso)).max() < 1e-9
    V, F = orc.marching_cubes(np.zeros((3, 3, 3)), wi.Grid.cube(3), 0.5)
    assert V.shape == (0, 3) and F.shape == (0, 3)
    with pytest.raises(ValueError):
        orc.marching_cubes(np.zeros((3, 3, 3)), wi.Grid.cube(3), 0.0)


def test_marching_cubes_single_voxel_diagonal_pair_and_strict_level(orc):
    """One voxel above the level gives an octahedron with its 6 vertices halfway to the
    neighbouring centres; two voxels touching only along an edge stay two separate
    closed surfaces (inside corners are cut off on their own on an ambiguous face); a
    value exactly at the level counts as outside, so the crossing lands on its centre."""
    orc._MC_TRIS.clear()
    g = wi.Grid((0.0, 0.0, 0.0), (3.0, 3.0, 3.0), (3, 3, 3))  # centres at 0.5, 1.5, 2.5
    f = np.zeros((3, 3, 3))
    f[1, 1, 1] = 1.0
    V, F = orc.marching_cubes(f, g, 0.5)
    assert V.shape == (6, 3) and F.shape == (8, 3)
    d = np.sort(np.abs(V - 1.5), axis=1)
    np.testing.assert_allclose(d, np.tile([0.0, 0.0, 0.5], (6, 1)), atol=1e-15)
    assert abs(signed_volume(V, F) - 4 / 3 * 0.5 ** 3) < 1e-15
    f[:] = 0.0
    f[0, 0, 1] = f[1, 1, 1] = 1.0
    V, F = orc.marching_cubes(f, g, 0.5)
    assert _directed_edges_pair_up(F) and _components(len(V), F) == 2
    f[:] = 0.0
    f[1, 1, 1], f[1, 1, 2] = 1.0, 0.5
    V, F = orc.marching_cubes(f, g, 0.5)
    assert V.shape == (6, 3) and F.shape == (8, 3)
    assert np.any(np.all(V == [1.5, 1.5, 2.5], axis=1))


def test_marching_cubes_every_corner_pattern(orc):
    """Each of the 256 inside/outside patterns of one cell (a 2 x 2 x 2 grid of 0/1
    values), and a dense random pattern: closed oriented 2-manifolds whose winding
    number is 1 at the inside centres and 0 at the others."""
    orc._MC_TRIS.clear()
    g = wi.Grid.cube(2)
    Q = orc.grid_points(g)
    for case in range(256):
        f = np.array([(case >> (a + 2 * b + 4 * c)) & 1 for a in (0, 1) for b in (0, 1) for c in (0, 1)], float)
        V, F = orc.marching_cubes(f.reshape(2, 2, 2), g, 0.5)
        assert _directed_edges_pair_up(F), case
        assert np.abs(orc.winding(V, F, Q) - f).max() < 1e-9, case
    rng = np.random.default_rng(53)
    g = wi.Grid.cube(9)
    f = (rng.random((9, 9, 9)) < 0.5).astype(float)
    V, F = orc.marching_cubes(f, g, 0.5)
    assert _directed_edges_pair_up(F)
    assert np.abs(orc.winding(V, F, orc.grid_points(g)) - f.reshape(-1)).max() < 1e-9


def test_marching_cubes_sphere(orc):
    """A sphere's distance field: vertices within 1e-3 of the radius at h = 1/24 (linear
    interpolation of a smooth field, error O(h^2)), area within 1 % of 4 pi r^2, and the
    enclosed volume within 2 % of 4/3 pi r^3."""
    orc._MC_TRIS.clear()
    g = wi.Grid.cube(24)
    Q = orc.grid_points(g)
    r = 0.3
    V, F = orc.marching_cubes(0.5 + (r - np.linalg.norm(Q, axis=1)), g, 0.5)
    assert _directed_edges_pair_up(F)
    assert np.abs(np.linalg.norm(V, axis=1) - r).max() < 1e-3
    area = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1).sum()
    assert abs(area / (4 * math.pi * r * r) - 1) < 0.01
    assert abs(signed_volume(V, F) / (4 / 3 * math.pi * r ** 3) - 1) < 0.02


def test_laplacian_smoothing_closed_forms(orc):
    """Umbrella smoothing of regular solids (without the volume rescale) shrinks them
    radially by a known factor per iteration: octahedron 1 - lam (neighbour mean is the
    centre), icosahedron 1 - lam + lam / sqrt(5) (neighbours at cos = 1/sqrt 5).
    lam = 0 is the identity."""
    V, F = wi.octahedron_mesh(1.0)
    S = orc.laplacian_smooth(V, F, 0.15, 10, keep_volume=False)
    np.testing.assert_allclose(S, V * (1 - 0.15) ** 10, atol=1e-15)
    V, F = wi.icosphere(0)
    S = orc.laplacian_smooth(V, F, 0.15, 10, keep_volume=False)
    np.testing.assert_allclose(S, V * (1 - 0.15 + 0.15 / math.sqrt(5)) ** 10, atol=1e-14)
    np.testing.assert_array_equal(orc.laplacian_smooth(V, F, 0.0, 10, keep_volume=False), V)
    np.testing.assert_allclose(orc.laplacian_smooth(V, F, 0.0, 10), V, atol=1e-15)


def test_enclosed_volume_closed_forms(orc):
    """Divergence-theorem volume: unit cube 1, regular octahedron |x|+|y|+|z| <= r
    (4/3) r^3, independent of a translation of a closed surface, negative when the faces
    are reversed, and 0 for an open flat patch."""
    V, F = wi.cube_mesh(0.0, 1.0)
    assert orc.enclosed_volume(V, F) == pytest.approx(1.0, abs=1e-15)
    assert orc.enclosed_volume(V + [3.0, -2.0, 5.0], F) == pytest.approx(1.0, abs=1e-13)
    assert orc.enclosed_volume(V, F[:, ::-1]) == pytest.approx(-1.0, abs=1e-15)
    V, F = wi.octahedron_mesh(0.7)
    assert orc.enclosed_volume(V, F) == pytest.approx(4 / 3 * 0.7 ** 3, rel=1e-14)
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float)
    assert orc.enclosed_volume(P, np.array([[0, 1, 2], [1, 3, 2]])) == 0.0


def test_laplacian_smoothing_keeps_enclosed_volume(orc):
    """With the volume rescale (the default), each Jacobi step is followed by a uniform
    scaling about the origin back to the starting volume:
      * a regular octahedron or icosahedron centred at the origin only shrinks radially,
        so the rescale undoes the step exactly: they are fixed points;
      * an octahedron centred at c shrinks about c by 1 - lam, then is scaled about the
        origin by 1 / (1 - lam): its shape is kept and its centre moves to c / (1 - lam)
        each step (scaling about the centroid would leave it in place);
      * the cube surface of a random voxel set keeps its volume while its vertices move."""
    lam = 0.15
    for V, F in (wi.octahedron_mesh(1.0), wi.icosphere(0)):
        np.testing.assert_allclose(orc.laplacian_smooth(V, F, lam, 10), V, atol=1e-14)
    V, F = wi.octahedron_mesh(0.2)
    c = np.array([0.3, -0.1, 0.05])
    S = orc.laplacian_smooth(V + c, F, lam, 4)
    np.testing.assert_allclose(S, V + c / (1 - lam) ** 4, atol=1e-14)
    rng = np.random.default_rng(61)
    occ = (rng.random((6, 5, 7)) < 0.45).astype(np.uint8)
    grid = wi.Grid((-0.5, -0.4, -0.6), (0.5, 0.6, 0.4), (6, 5, 7))
    Vc, Fc = orc.cubify(occ, grid)
    vol0 = orc.enclosed_volume(Vc, Fc)
    assert vol0 == pytest.approx(occ.sum() * (1 / 6) * (1 / 5) * (1 / 7), rel=1e-12)
    S = orc.laplacian_smooth(Vc, Fc, lam, 10)
    assert orc.enclosed_volume(S, Fc) == pytest.approx(vol0, rel=1e-12)
    assert np.abs(S - Vc).max() > 1e-3
    S0 = orc.laplacian_smooth(Vc, Fc, lam, 10, keep_volume=False)
    assert orc.enclosed_volume(S0, Fc) < 0.9 * vol0


def test_laplacian_smoothing_keeps_planar_grid_interior(orc):
    """On a flat triangulated grid (diagonals all one way) interior vertices are the mean
    of their six neighbours, so they do not move; boundary vertices do."""
    n = 6
    x, y = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    V = np.stack([x.ravel(), y.ravel(), np.zeros(n * n)], 1)
    F = []
    for i in range(n - 1):
        for j in range(n - 1):
            a, b, c, d = i * n + j, (i + 1) * n + j, (i + 1) * n + j + 1, i * n + j + 1
            F += [[a, b, c], [a, c, d]]
    S = orc.laplacian_smooth(V, np.array(F), 0.3, 1, keep_volume=False)
    np.testing.assert_array_equal(orc.laplacian_smooth(V, np.array(F), 0.3, 1), S)  # no volume: no rescale
    inner = (x.ravel() > 0) & (x.ravel() < n - 1) & (y.ravel() > 0) & (y.ravel() < n - 1)
    np.testing.assert_allclose(S[inner], V[inner], atol=1e-15)
    assert np.abs(S[~inner] - V[~inner]).max() > 0.05
    # two triangles sharing edge (1, 2): each neighbour counts once however many faces share it
    K = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [2, 2, 1]], float)
    S = orc.laplacian_smooth(K, np.array([[0, 1, 2], [1, 3, 2]]), 0.3, 1, keep_volume=False)
    np.testing.assert_allclose(S[1], K[1] + 0.3 * ((K[0] + K[2] + K[3]) / 3 - K[1]), atol=1e-15)
    np.testing.assert_allclose(S[0], K[0] + 0.3 * ((K[1] + K[2]) / 2 - K[0]), atol=1e-15)


def test_surface_sampling_exact_face_choice_and_placement(orc):
    """Face choice is integer inverse-CDF sampling of w_f = floor(area_f 2^32 / max):
    two triangles of areas 1 and 3 split u0 at w_0 / (w_0 + w_1) = floor(2^32/3) /
    (floor(2^32/3) + 2^32).  Points lie in their face, and their mean over one triangle
    approaches its centroid."""
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 1], [3, 0, 1], [0, 2, 1]], float)
    F = np.array([[0, 1, 2], [3, 4, 5]])
    w0, w1 = math.floor(2 ** 32 / 3), 2 ** 32
    np.testing.assert_array_equal(orc.face_area_weights(V, F), [w0, w1])
    split = w0 / (w0 + w1)
    u = np.array([[np.nextafter(split, 0), 0.2, 0.3], [split + 1e-12, 0.2, 0.3], [0.0, 0.9, 0.8],
                  [np.nextafter(1.0, 0), 0.5, 0.5]])
    P, f = orc.sample_surface(V, F, u)
    np.testing.assert_array_equal(f, [0, 1, 0, 1])
    np.testing.assert_allclose(P[2], V[0] + 0.1 * (V[1] - V[0]) + 0.2 * (V[2] - V[0]), atol=1e-15)
    u = np.random.default_rng(52).random((200000, 3))
    P, f = orc.sample_surface(V[:3], F[:1], u)
    bary = np.linalg.lstsq(np.stack([V[1] - V[0], V[2] - V[0]], 1)[:2], (P - V[0])[:, :2].T, rcond=None)[0]
    assert np.all(bary >= -1e-12) and np.all(bary.sum(0) <= 1 + 1e-12) and np.all(P[:, 2] == 0)
    assert np.abs(P.mean(0) - V[:3].mean(0)).max() < 5e-3


def test_nn_distances_and_chamfer_hausdorff(orc):
    """Brute-force nearest neighbours against a k-d tree (scipy), and the metrics on
    point sets with known answers."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(53)
    A, B = rng.normal(size=(3000, 3)), rng.normal(size=(2000, 3)) * 1.5
    np.testing.assert_allclose(orc.nn_distances(A, B), cKDTree(B).query(A)[0], rtol=1e-12)
    cd, hd = orc.chamfer_hausdorff(A, A)
    assert cd == 0.0 and hd == 0.0
    cd, hd = orc.chamfer_hausdorff([[0, 0, 0]], [[3, 4, 0]])
    assert cd == 10.0 and hd == 5.0
    # a set against itself plus one outlier at distance 2 from its nearest point
    B = np.concatenate([A, [[100.0, 0, 0]]])
    dmin = np.min(np.linalg.norm(A - [100.0, 0, 0], axis=1))
    cd, hd = orc.chamfer_hausdorff(A, B)
    assert abs(hd - dmin) < 1e-12 and abs(cd - dmin / len(B)) < 1e-12
