"""GPU forward parity: the HIP library through its C ABI against the FP64 oracle.

Tolerances (stated by the method's target): |W_gpu - W_ref| <= 1e-4 at every point
outside the guard band E (within 1e-4 of an edge or vertex, or 1e-6 of a face, where
FP32 cannot resolve the field; Section 2.2 notes the field is binary except on the
surface), and hard occupancy bit-identical where additionally |W_ref - 0.5| > 1e-3.
Sigmoid occupancy (k = 50): |docc| <= (k/4) 1e-4 + 1e-6 = 1.25e-3.
"""
import numpy as np
import pytest

import wn_inputs as wi

pytestmark = pytest.mark.gpu

TOL_W = 1e-4
BAND = 1e-3


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_11272_amd as wn
    wn.wn_version()  # loads libwn.so or raises
    return torch.device("cuda", 0)


def _gpu_w(V, F, grid=None, Q=None, occupancy=None, **kw):
    import torch
    import paper_2407_11272_amd as wn
    Vt = torch.as_tensor(np.asarray(V, np.float32)).cuda()
    Ft = torch.as_tensor(np.asarray(F, np.int32)).cuda()
    Qt = None if Q is None else torch.as_tensor(np.asarray(Q, np.float32)).cuda()
    g = None if grid is None else wn.Grid.of(grid)
    out = wn.wn_voxelize(Vt, Ft, grid=g, Q=Qt, occupancy=occupancy, **kw)
    torch.cuda.synchronize()
    if occupancy is None:
        return out.cpu().numpy().reshape(-1)
    return out[0].cpu().numpy().reshape(-1), out[1].cpu().numpy().reshape(-1)


def _f32(V):
    """The GPU sees float32 vertices; the oracle is given the same rounded values."""
    return np.asarray(V, np.float32).astype(np.float64)


def _compare(orc, V, F, Q, Wg, label, occ_g=None, tau=0.5):
    V64 = _f32(V)
    Wr = orc.winding(V64, F, Q)
    guard = orc.guard_mask(V64, F, Q)
    err = np.abs(Wg.astype(np.float64) - Wr)
    ok = ~guard
    print(f"[{label}] points={len(Q)} guard={int(guard.sum())} max|dW| off-guard={err[ok].max() if ok.any() else 0:.3e}"
          f" on-guard={err[guard].max() if guard.any() else 0:.3e}", flush=True)
    assert guard.sum() <= max(2, 1e-3 * len(Q)), "guard band unexpectedly large"
    assert np.all(err[ok] <= TOL_W), f"{label}: max |dW| {err[ok].max():.3e}"
    if occ_g is not None:
        m = ok & (np.abs(Wr - tau) > BAND)
        ref = orc.occupancy_threshold(Wr, tau)
        np.testing.assert_array_equal(occ_g[m], ref[m])
    return Wr, guard


def test_config1_full_grid(dev, orc):
    """Plain forward on the 1280-face jittered icosphere at 32^3: every voxel."""
    c = wi.config1_icosphere()
    Q = orc.grid_points(c.grid)
    Wg, occ = _gpu_w(c.V, c.F, grid=c.grid, occupancy="threshold")
    Wr, _ = _compare(orc, c.V, c.F, Q, Wg, "C1", occ_g=occ)
    assert 0.05 < (Wr > 0.5).mean() < 0.5


def test_config2_full_grid(dev, orc):
    """Non-watertight union (19 000 faces) at 128^3 on the path the benchmark times: the
    triangle-strip order, after the autotuner has picked the launch configuration.  Every
    one of the 2 097 152 voxels is held to the oracle (4e10 FP64 point-face pairs, about
    a minute on 16 host threads): W within 1e-4 wherever a point is not in the guard band
    (the guard band is evaluated for the points that miss the bar, which must all be in
    it, at most 1e-4 of the grid), and the occupancy bit-identical to the oracle's
    wherever |W - 0.5| > 1e-3 off those points."""
    import time
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config2_ellipsoid_union()
    V, F = wn.as_mesh(torch.as_tensor(np.asarray(c.V, np.float32)), torch.as_tensor(c.F))
    R = _strips_dev(c.F, len(c.V))
    grid = wn.Grid.of(c.grid)
    W = torch.empty(tuple(grid.n), dtype=torch.float32, device="cuda")
    occ = torch.empty(tuple(grid.n), dtype=torch.uint8, device="cuda")
    wn.wn_autotune("voxelize", [wn.MeshJob(V, F, grid, "threshold", W=W, occ=occ, strips=R)])
    W, occ = wn.wn_voxelize_strips(V, F, R, grid=grid, occupancy="threshold")
    Wg, og = W.cpu().numpy().reshape(-1), occ.cpu().numpy().reshape(-1)
    assert Wg.shape == (128 ** 3,) and np.isfinite(Wg).all()
    t0 = time.perf_counter()
    V64 = np.asarray(c.V, np.float32).astype(np.float64)
    Wr = orc.winding_grid(V64, c.F, c.grid)
    miss = np.abs(Wg - Wr) > TOL_W
    Q = orc.grid_points(c.grid)
    guard = orc.guard_mask(V64, c.F, Q[miss]) if miss.any() else np.zeros(0, bool)
    print(f"[C2 full grid, strips] oracle {time.perf_counter() - t0:.0f} s; max |dW| = "
          f"{np.abs(Wg - Wr)[~miss].max():.2e} on {int((~miss).sum())} points, {int(miss.sum())} beyond 1e-4 "
          f"(all in the guard band: {bool(guard.all())})", flush=True)
    assert guard.all() and miss.sum() <= 1e-4 * len(Wg)
    off = (np.abs(Wr - 0.5) > BAND) & ~miss
    np.testing.assert_array_equal(og[off], orc.occupancy_threshold(Wr, 0.5)[off])
    assert off.mean() > 0.99


def test_largest_served_request_sampled(dev, orc):
    """The largest request shape of the served workload (100 000 faces at 256^3,
    1.7e12 pairs), in strip order and in three records per face; the oracle checks
    1500 seeded voxels plus the first and last."""
    import torch
    import paper_2407_11272_amd as wn
    req = wi.configs.Request(0, 0.0, 100_000, 256, False, 12345)
    w = req.build()
    V, F = wn.as_mesh(torch.as_tensor(w.V), torch.as_tensor(w.F))
    R = torch.as_tensor(wn.wn_build_strips(np.asarray(w.F, np.int32), len(w.V))).cuda()
    grid = wn.Grid.of(w.grid)
    Ws = wn.wn_voxelize_strips(V, F, R, grid=grid).cpu().numpy().reshape(-1)
    Wp = wn.wn_voxelize(V, F, grid=grid).cpu().numpy().reshape(-1)
    assert Ws.shape == (256 ** 3,)
    rng = np.random.default_rng(102)
    idx = np.unique(np.concatenate([rng.integers(0, len(Ws), 1500), [0, len(Ws) - 1]]))
    Q = orc.grid_points(w.grid)[idx]
    _compare(orc, w.V, w.F, Q, Ws[idx], "served-max strips")
    _compare(orc, w.V, w.F, Q, Wp[idx], "served-max plain")
    assert np.isfinite(Ws).all() and np.isfinite(Wp).all()


def test_convenience_voxelize_uses_strips_for_host_faces(dev, orc):
    """voxelize() with host faces runs the strip order, with device faces the default
    order; both match the oracle and each other to rounding."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config1_icosphere()
    Wh = wn.voxelize(np.asarray(c.V, np.float32), c.F, grid=c.grid).cpu().numpy().reshape(-1)
    Wd = wn.voxelize(torch.as_tensor(np.asarray(c.V, np.float32)).cuda(),
                     torch.as_tensor(c.F, dtype=torch.int32).cuda(), grid=c.grid).cpu().numpy().reshape(-1)
    _compare(orc, c.V, c.F, orc.grid_points(c.grid), Wh, "voxelize host faces")
    assert np.abs(Wh - Wd).max() <= 1e-5


def test_config3_mesh_full_grid(dev, orc):
    """The 5120-face icosphere of the differentiable workload at 64^3 (forward)."""
    c = wi.config3_differentiable()
    Q = orc.grid_points(c.grid)
    rng = np.random.default_rng(101)
    idx = rng.choice(len(Q), 20000, replace=False)
    Wg = _gpu_w(c.V, c.F, grid=c.grid)
    _compare(orc, c.V, c.F, Q[idx], Wg[idx], "C3")


@pytest.mark.parametrize("nF", [1, 2, 5, 16, 63, 64, 65, 129, 300])
def test_random_small_meshes_point_list(dev, orc, nF):
    """Random triangles (tile boundaries at 64 faces) and random points in list mode,
    a ragged point count, and the face-split path (few points)."""
    rng = np.random.default_rng(1000 + nF)
    V = rng.uniform(-0.6, 0.6, size=(3 * nF, 3))
    F = rng.permutation(3 * nF).reshape(nF, 3)
    Q = rng.uniform(-0.7, 0.7, size=(1000 + nF, 3)).astype(np.float32).astype(np.float64)
    Wg = _gpu_w(V, F, Q=Q)
    _compare(orc, V, F, Q, Wg, f"random nF={nF}")


@pytest.mark.parametrize("shape", [(7, 9, 11), (1, 1, 1), (3, 64, 5), (33, 17, 2)])
def test_ragged_grids(dev, orc, shape):
    """Non-cubic grids with odd sizes and a non-symmetric extent."""
    c = wi.config1_icosphere()
    g = wi.Grid((-0.45, -0.5, -0.41), (0.47, 0.43, 0.5), shape)
    Q = orc.grid_points(g)
    Wg = _gpu_w(c.V, c.F, grid=g)
    assert Wg.shape == (int(np.prod(shape)),)
    # the fp32 voxel centres differ from the fp64 ones by rounding only
    _compare(orc, c.V, c.F, Q, Wg, f"grid {shape}")


def test_orientation_flip_and_determinism(dev, orc):
    c = wi.config1_icosphere()
    W1 = _gpu_w(c.V, c.F, grid=c.grid)
    W2 = _gpu_w(c.V, c.F, grid=c.grid)
    np.testing.assert_array_equal(W1, W2)  # bit-identical reruns
    Wr = _gpu_w(c.V, wi.reverse_faces(c.F), grid=c.grid)
    np.testing.assert_allclose(Wr, -W1, atol=2e-6)


@pytest.mark.parametrize("scale", [1e-3, 1e4, 1e7, 1e11])
def test_scale_invariance_across_the_pair_range(dev, scale):
    """W is invariant under a common scaling of mesh and points.  Scaled by 1e7 and 1e11
    the two-face products leave the normal FP32 range, so the per-face fallback of the
    paired ATAN2 runs; 1e-3 and 1e4 stay on the fast path."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config1_icosphere()
    V = np.asarray(c.V, np.float64)
    R = torch.as_tensor(wn.wn_build_strips(c.F, len(V))).cuda()
    F = torch.as_tensor(c.F, dtype=torch.int32).cuda()
    g = c.grid
    W1 = wn.wn_voxelize_strips(torch.as_tensor(V, dtype=torch.float32).cuda(), F, R, grid=g).cpu().numpy()
    gs = wn.Grid(tuple(np.float32(x * scale) for x in g.lo), tuple(np.float32(x * scale) for x in g.hi), g.n)
    Ws = wn.wn_voxelize_strips(torch.as_tensor(V * scale, dtype=torch.float32).cuda(), F, R,
                               grid=gs).cpu().numpy()
    err = np.abs(Ws - W1)
    print(f"[scale {scale:g}] max|W(scaled) - W| = {err.max():.2e}", flush=True)
    assert np.isfinite(Ws).all() and err.max() <= 1e-4


def test_cube_closed_forms(dev, orc):
    """Closed unit cube: centre 1, vertices 1/8 (the faces at the vertex give 0), far 0."""
    V, F = wi.cube_mesh(0.0, 1.0)
    Q = np.array([[0.5, 0.5, 0.5], [0, 0, 0], [1, 1, 1], [1, 0, 1], [3, 3, 3], [-1, 0.5, 0.5], [0.25, 0.75, 0.5]])
    Wg = _gpu_w(V, F, Q=Q)
    np.testing.assert_allclose(Wg, [1, 1 / 8, 1 / 8, 1 / 8, 0, 0, 1], atol=1e-6)


def test_empty_inputs(dev):
    import torch
    import paper_2407_11272_amd as wn
    V = torch.zeros((4, 3), device="cuda")
    F = torch.zeros((0, 3), dtype=torch.int32, device="cuda")
    W = wn.wn_voxelize(V, F, grid=wn.Grid.cube(8))
    torch.cuda.synchronize()
    assert torch.all(W == 0)
    W, occ = wn.wn_voxelize(V, F, grid=wn.Grid.cube(4), occupancy="sigmoid", k=10.0)
    torch.cuda.synchronize()
    assert torch.allclose(occ, torch.full_like(occ, 1.0 / (1.0 + np.exp(5.0))), atol=1e-6)
    Q = torch.zeros((0, 3), device="cuda")
    W = wn.wn_voxelize(V, torch.zeros((2, 3), dtype=torch.int32, device="cuda"), Q=Q)
    assert W.numel() == 0
    W = wn.wn_voxelize(V, F, grid=wn.Grid((0, 0, 0), (1, 1, 1), (0, 4, 4)))
    assert W.numel() == 0


def test_bad_face_index_is_reported_not_read(dev, orc):
    """Out-of-range indices are replaced by 0 on the device and reported."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config1_icosphere()
    F = c.F.copy()
    F[5, 1] = 10 ** 6
    F[9, 0] = -3
    Vt = torch.as_tensor(c.V, dtype=torch.float32).cuda()
    Ft = torch.as_tensor(F, dtype=torch.int32).cuda()
    W = wn.wn_voxelize(Vt, Ft, grid=c.grid)
    assert wn.wn_get_device_error() == wn._lib.WN_ERR_BAD_INDEX
    assert wn.wn_get_device_error() == 0  # cleared by the read
    F2 = F.copy()
    F2[5, 1] = 0
    F2[9, 0] = 0
    W2 = wn.wn_voxelize(Vt, torch.as_tensor(F2, dtype=torch.int32).cuda(), grid=c.grid)
    assert wn.wn_get_device_error() == 0
    torch.testing.assert_close(W, W2, rtol=0, atol=0)


def test_argument_errors(dev):
    import ctypes
    import torch
    import paper_2407_11272_amd as wn
    from paper_2407_11272_amd import _lib as L
    lib = L.load()
    V = torch.zeros((3, 3), device="cuda")
    F = torch.tensor([[0, 1, 2]], dtype=torch.int32, device="cuda")
    W = torch.empty(8, device="cuda")
    g = wn.Grid.cube(2).to_c()
    ws = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    base = ws.data_ptr() + ((-ws.data_ptr()) % 256)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = ctypes.c_void_p
    ok = lib.wn_voxelize(p(V.data_ptr()), 3, p(F.data_ptr()), 1, ctypes.byref(g), None, 0, p(W.data_ptr()), 0, 0.5,
                         50.0, None, p(base), 1 << 19, s)
    assert ok == L.WN_OK
    # both grid and Q
    assert lib.wn_voxelize(p(V.data_ptr()), 3, p(F.data_ptr()), 1, ctypes.byref(g), p(V.data_ptr()), 3,
                           p(W.data_ptr()), 0, 0.5, 50.0, None, p(base), 1 << 19, s) == L.WN_ERR_INVALID_ARG
    # negative count, null mesh with faces, bad occupancy mode, nQ inconsistent with the grid
    assert lib.wn_voxelize(p(V.data_ptr()), -1, p(F.data_ptr()), 1, ctypes.byref(g), None, 0, p(W.data_ptr()), 0,
                           0.5, 50.0, None, p(base), 1 << 19, s) == L.WN_ERR_INVALID_ARG
    assert lib.wn_voxelize(None, 3, p(F.data_ptr()), 1, ctypes.byref(g), None, 0, p(W.data_ptr()), 0, 0.5, 50.0,
                           None, p(base), 1 << 19, s) == L.WN_ERR_INVALID_ARG
    assert lib.wn_voxelize(p(V.data_ptr()), 3, p(F.data_ptr()), 1, ctypes.byref(g), None, 0, p(W.data_ptr()), 7, 0.5,
                           50.0, None, p(base), 1 << 19, s) == L.WN_ERR_INVALID_ARG
    assert lib.wn_voxelize(p(V.data_ptr()), 3, p(F.data_ptr()), 1, ctypes.byref(g), None, 5, p(W.data_ptr()), 0, 0.5,
                           50.0, None, p(base), 1 << 19, s) == L.WN_ERR_INVALID_ARG
    # workspace: missing, misaligned, too small
    assert lib.wn_voxelize(p(V.data_ptr()), 3, p(F.data_ptr()), 1, ctypes.byref(g), None, 0, p(W.data_ptr()), 0, 0.5,
                           50.0, None, None, 0, s) == L.WN_ERR_WORKSPACE
    assert lib.wn_voxelize(p(V.data_ptr()), 3, p(F.data_ptr()), 1, ctypes.byref(g), None, 0, p(W.data_ptr()), 0, 0.5,
                           50.0, None, p(base + 4), 1 << 19, s) == L.WN_ERR_WORKSPACE
    assert lib.wn_voxelize(p(V.data_ptr()), 3, p(F.data_ptr()), 1, ctypes.byref(g), None, 0, p(W.data_ptr()), 0, 0.5,
                           50.0, None, p(base), 16, s) == L.WN_ERR_WORKSPACE
    assert lib.wn_occupancy(p(W.data_ptr()), 8, 9, 0.5, 1.0, p(W.data_ptr()), s) == L.WN_ERR_INVALID_ARG
    with pytest.raises(wn.WnError):
        L.check("wn_occupancy", lib.wn_occupancy(p(W.data_ptr()), -2, 1, 0.5, 1.0, p(W.data_ptr()), s))
    torch.cuda.synchronize()


def test_occupancy_maps_and_loss(dev, orc):
    """Occupancy maps, the sigmoid-MSE loss and its gradient, and the soft occupancy's
    adjoint, all applied on the GPU to the oracle's W (rounded to FP32): the same input
    on both sides.  The fused occupancy of the forward equals the separate map."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config3_differentiable(res=32)
    Vt, Ft = wn.as_mesh(torch.as_tensor(c.V), torch.as_tensor(c.F))
    Wf, occf = wn.wn_voxelize(Vt, Ft, grid=c.grid, occupancy="sigmoid", k=50.0)
    torch.testing.assert_close(occf, wn.wn_occupancy(Wf, "sigmoid", 0.5, 50.0), rtol=0, atol=0)
    W32 = orc.winding(np.asarray(c.V, np.float32).astype(np.float64), c.F, orc.grid_points(c.grid)).astype(np.float32)
    Wn = W32.astype(np.float64)
    W = torch.as_tensor(W32).cuda()
    occ = wn.wn_occupancy(W, "sigmoid", 0.5, 50.0)
    thr = wn.wn_occupancy(W, "threshold", 0.5)
    c_t = torch.as_tensor(c.target).cuda()
    loss, g = wn.wn_sigmoid_mse(W, c_t)
    # soft-occupancy adjoint: with g_occ = 2 (occ - target) / P it is the loss gradient
    s_ref = orc.occupancy_sigmoid(Wn, 0.5, 50.0)
    g_occ = torch.as_tensor((2.0 * (s_ref - c.target) / len(Wn)).astype(np.float32)).cuda()
    dW = wn.wn_occupancy_backward(W, g_occ, 0.5, 50.0)
    torch.cuda.synchronize()
    np.testing.assert_allclose(occ.cpu().numpy(), s_ref, atol=1e-6)
    np.testing.assert_array_equal(thr.cpu().numpy(), orc.occupancy_threshold(Wn))
    Lr, gr = orc.sigmoid_mse(Wn, c.target, 0.5, 50.0)
    assert float(loss.item()) == pytest.approx(Lr, rel=1e-5)
    np.testing.assert_allclose(g.cpu().numpy(), gr, rtol=1e-4, atol=1e-12)
    np.testing.assert_allclose(dW.cpu().numpy(), gr, rtol=1e-4, atol=1e-12)


def _strips_dev(F, nV):
    import torch
    import paper_2407_11272_amd as wn
    return torch.as_tensor(wn.wn_build_strips(F, nV)).cuda()


@pytest.mark.parametrize("cfg", ["c1", "c3", "open", "c2"])
def test_strip_order_parity(dev, orc, cfg):
    """Triangle-strip record streams give the same field (to rounding) as three records
    per face, agree with the oracle, and are bit-reproducible."""
    import torch
    import paper_2407_11272_amd as wn
    c = {"c1": wi.config1_icosphere, "c3": wi.config3_differentiable,
         "open": lambda: wi.config3_differentiable(open_variant=True), "c2": wi.config2_ellipsoid_union}[cfg]()
    Vt, Ft = wn.as_mesh(torch.as_tensor(np.asarray(c.V, np.float32)), torch.as_tensor(c.F))
    R = _strips_dev(c.F, len(c.V))
    Ws, occ = wn.wn_voxelize_strips(Vt, Ft, R, grid=c.grid, occupancy="threshold")
    Ws2 = wn.wn_voxelize_strips(Vt, Ft, R, grid=c.grid)
    Wp = wn.wn_voxelize(Vt, Ft, grid=c.grid)
    torch.cuda.synchronize()
    assert wn.wn_get_device_error() == 0
    torch.testing.assert_close(Ws, Ws2, rtol=0, atol=0)
    diff = (Ws - Wp).abs().cpu().numpy().reshape(-1)
    Q = orc.grid_points(c.grid)
    # the two face orders round differently; where they differ by more than 2e-6 the
    # voxel must lie in the guard band, or both must hold the oracle's 1e-4
    far = np.nonzero(diff > 2e-6)[0]
    print(f"[strips {cfg}] records/face={R.shape[0] / len(c.F):.3f} max|strips - plain|={diff.max():.2e} "
          f"voxels > 2e-6: {len(far)}", flush=True)
    assert len(far) <= 1e-3 * len(diff)
    if len(far):
        V64 = np.asarray(c.V, np.float32).astype(np.float64)
        g = orc.guard_mask(V64, c.F, Q[far])
        Wr = orc.winding(V64, c.F, Q[far])
        Wsn = Ws.cpu().numpy().reshape(-1)[far]
        Wpn = Wp.cpu().numpy().reshape(-1)[far]
        assert np.all(g | ((np.abs(Wsn - Wr) <= 1e-4) & (np.abs(Wpn - Wr) <= 1e-4)))
    Wn = Ws.cpu().numpy().reshape(-1)
    idx = np.random.default_rng(9).choice(len(Q), 3000, replace=False)
    _compare(orc, c.V, c.F, Q[idx], Wn[idx], f"strips {cfg}", occ_g=occ.cpu().numpy().reshape(-1)[idx])


def test_strips_split_path_primes_windows(dev, orc):
    """Few query points and many faces: the record stream is split over workgroups at
    arbitrary records, so each split primes its vertex window from the two records
    before it."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config2_ellipsoid_union()
    Vt, Ft = wn.as_mesh(torch.as_tensor(np.asarray(c.V, np.float32)), torch.as_tensor(c.F))
    R = _strips_dev(c.F, len(c.V))
    rng = np.random.default_rng(11)
    Q = rng.uniform(-0.5, 0.5, size=(333, 3)).astype(np.float32).astype(np.float64)
    Qt = torch.as_tensor(Q, dtype=torch.float32).cuda()
    Ws = wn.wn_voxelize_strips(Vt, Ft, R, Q=Qt).cpu().numpy()
    _compare(orc, c.V, c.F, Q, Ws, "strips split")


def test_bad_strip_records_are_reported(dev):
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config1_icosphere()
    Vt, Ft = wn.as_mesh(torch.as_tensor(c.V), torch.as_tensor(c.F))
    R = wn.wn_build_strips(c.F, len(c.V))
    R[5, 0] = 10 ** 7
    R[9, 1] = len(c.F) + 3
    R[12, 1] = -7
    W = wn.wn_voxelize_strips(Vt, Ft, torch.as_tensor(R).cuda(), grid=c.grid)
    assert wn.wn_get_device_error() == wn._lib.WN_ERR_BAD_INDEX
    assert torch.isfinite(W).all()


def test_forged_strip_windows_are_reported(dev):
    """A strip record that claims face f must complete F[f]: its vertex id and those of
    the two records before it are F[f]'s ids in some order.  A window with an in-range
    but wrong vertex id (a stale strip order, a hand-built stream) and a face flag on
    record 0 are reported as bad indices, by the single-mesh and the batched packs; the
    valid stream is not."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config1_icosphere(res=16)
    Vt, Ft = wn.as_mesh(torch.as_tensor(c.V), torch.as_tensor(c.F))
    R = wn.wn_build_strips(c.F, len(c.V))
    face_rows = np.nonzero(R[:, 1] >= 0)[0]
    i = int(face_rows[len(face_rows) // 2])
    wrong = next(v for v in range(len(c.V)) if v not in set(c.F[R[i, 1]].tolist()))
    bad_window = R.copy()
    bad_window[i, 0] = wrong            # in range, but not a vertex of face R[i, 1]
    bad_first = R.copy()
    bad_first[0, 1] = R[i, 1]           # a face flag on record 0 (no window)
    for name, stream, expect in (("valid", R, 0), ("wrong vertex", bad_window, wn._lib.WN_ERR_BAD_INDEX),
                                 ("flag on record 0", bad_first, wn._lib.WN_ERR_BAD_INDEX)):
        Rt = torch.as_tensor(stream).cuda()
        W = wn.wn_voxelize_strips(Vt, Ft, Rt, grid=c.grid)
        assert wn.wn_get_device_error() == expect, name
        assert torch.isfinite(W).all()
        job = wn.MeshJob(Vt, Ft, c.grid, strips=Rt).prepare()
        wn.wn_voxelize_batched([job], graph=False)
        assert wn.wn_get_device_error() == expect, name + " (batched)"
        assert torch.isfinite(job.W).all()


def test_adversarial_points_on_vertices_and_edges(dev, orc):
    """Query points exactly at mesh vertices (a face with q at its vertex contributes 0,
    as in the oracle) and on edges (inside the guard band: any value, but finite), for
    both record orders; far-from-surface points of the same call keep 1e-4 parity."""
    import torch
    import paper_2407_11272_amd as wn
    rng = np.random.default_rng(77)
    for seed in range(3):
        V = np.round(rng.uniform(-0.5, 0.5, (12, 3)) * 64) / 64  # exactly representable
        F = rng.permutation(12).reshape(4, 3)
        mids = [(V[a] + V[b]) / 2 for a, b in ((F[0, 0], F[0, 1]), (F[2, 1], F[2, 2]))]
        far = rng.uniform(-0.5, 0.5, (50, 3)).astype(np.float32).astype(np.float64)
        Q = np.concatenate([V, np.array(mids), far])
        Vt, Ft = wn.as_mesh(torch.as_tensor(V), torch.as_tensor(F))
        Qt = torch.as_tensor(Q, dtype=torch.float32).cuda()
        R = torch.as_tensor(wn.wn_build_strips(F, len(V))).cuda()
        for W in (wn.wn_voxelize(Vt, Ft, Q=Qt), wn.wn_voxelize_strips(Vt, Ft, R, Q=Qt)):
            Wn = W.cpu().numpy()
            assert np.isfinite(Wn).all()
            # each vertex belongs to exactly one face of this soup: that face gives 0
            Wr = orc.winding(V, F, Q)
            np.testing.assert_allclose(Wn[:12], Wr[:12], atol=1e-4)
            guard = orc.guard_mask(V, F, far)
            assert np.abs(Wn[14:] - Wr[14:])[~guard].max() <= 1e-4
