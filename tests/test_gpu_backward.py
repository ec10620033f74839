"""GPU adjoint parity: wn_backward / the autograd Function against the FP64 oracle.

For the closed icosphere of the differentiable workload the vertex gradient is zero
analytically (W depends only on a surface's boundary), so the check is split:
  (i)   per-corner dL/dT against the oracle's analytic gradient:
        |d|_inf <= 1e-3 |ref|_inf and elementwise 1e-3 relative where |ref| > 1e-2 |ref|_inf;
  (ii)  dL/dV against the oracle, cancellation-aware: |d_v| <= 1e-3 sum over v's corners |dL/dT|;
  (iii) on an open variant (5 % of faces removed) dL/dV of the sigmoid-MSE loss against
        FP64 central differences of the oracle's loss on hole-rim vertices (1e-3 relative).
"""
import numpy as np
import pytest

import wn_inputs as wi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_11272_amd as wn
    wn.wn_version()
    return torch.device("cuda", 0)


def _to_dev(c):
    import torch
    import paper_2407_11272_amd as wn
    return wn.as_mesh(torch.as_tensor(np.asarray(c.V, np.float32)), torch.as_tensor(c.F))


def _f32(V):
    return np.asarray(V, np.float32).astype(np.float64)


def _oracle_dLdW(orc, c, Q=None):
    """The oracle's W, loss and dL/dW of the sigmoid-MSE loss (FP64); the GPU adjoint is
    then given the same dL/dW (rounded to FP32), so both sides differentiate the same
    loss at the same point and no input of the oracle comes from the GPU."""
    V64 = _f32(c.V)
    Q = orc.grid_points(c.grid) if Q is None else Q
    W = orc.winding(V64, c.F, Q)
    L, g = orc.sigmoid_mse(W, c.target, c.tau, c.k)
    g32 = np.asarray(g, np.float32)
    return W, L, g32, Q


def _gpu_adjoint(c, g32):
    import torch
    import paper_2407_11272_amd as wn
    Vt, Ft = _to_dev(c)
    dLdV, dLdT = wn.wn_backward(Vt, Ft, torch.as_tensor(g32).cuda(), grid=c.grid, want_dLdT=True)
    torch.cuda.synchronize()
    return dLdV.cpu().numpy().astype(np.float64), dLdT.cpu().numpy().astype(np.float64)


def _check_T(Tg, Tr, label):
    scale = np.abs(Tr).max()
    d = np.abs(Tg - Tr)
    big = np.abs(Tr) > 1e-2 * scale
    rel = d[big] / np.abs(Tr[big])
    print(f"[{label}] |dL/dT|inf={scale:.3e} max abs err={d.max():.3e} max rel (big)={rel.max():.3e} "
          f"({int(big.sum())} of {big.size} entries big)", flush=True)
    assert d.max() <= 1e-3 * scale
    assert rel.max() <= 1e-3


def _check_V(Dg, Dr, Tr, F, label):
    """dL/dV is a sum of corner gradients that cancel (exactly, for a closed mesh): each
    vertex is held to 1e-3 of the sum of the magnitudes of its corners' terms."""
    corner_abs = np.zeros_like(Dr)
    np.add.at(corner_abs, np.asarray(F).reshape(-1), np.abs(Tr.reshape(-1, 3)))
    err = np.abs(Dg - Dr)
    print(f"[{label}] max |d dL/dV| / corner scale = {(err / (corner_abs + 1e-300)).max():.3e}", flush=True)
    assert np.all(err <= 1e-3 * corner_abs + 1e-12)


def test_corner_and_vertex_gradients_32(dev, orc):
    """(i) + (ii) on the differentiable workload's mesh at 32^3, every face and vertex;
    the loss of the GPU's own forward against the oracle's."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config3_differentiable(res=32)
    Wr, Lr, g32, Q = _oracle_dLdW(orc, c)
    Dg, Tg = _gpu_adjoint(c, g32)
    Tr, Dr = orc.grad(_f32(c.V), c.F, Q, g32.astype(np.float64))
    _check_T(Tg.reshape(-1), Tr.reshape(-1), "C3@32 dL/dT")
    _check_V(Dg, Dr, Tr, c.F, "C3@32 dL/dV")
    Vt, Ft = _to_dev(c)
    W = wn.wn_voxelize(Vt, Ft, grid=c.grid).reshape(-1)
    loss, _ = wn.wn_sigmoid_mse(W, torch.as_tensor(c.target).cuda(), c.tau, c.k)
    assert float(loss.item()) == pytest.approx(Lr, rel=1e-4)


def test_corner_and_vertex_gradients_full_size(dev, orc):
    """(i) + (ii) on the differentiable workload at its full size (5120 faces, 64^3):
    all 46 080 corner components and all 2562 vertices against the oracle."""
    c = wi.config3_differentiable(res=64)
    Wr, Lr, g32, Q = _oracle_dLdW(orc, c)
    Dg, Tg = _gpu_adjoint(c, g32)
    Tr, Dr = orc.grad(_f32(c.V), c.F, Q, g32.astype(np.float64))
    _check_T(Tg.reshape(-1), Tr.reshape(-1), "C3@64 dL/dT all faces")
    _check_V(Dg, Dr, Tr, c.F, "C3@64 dL/dV all vertices")


def _rim_vertices(F):
    from collections import Counter
    cnt = Counter()
    for f in F:
        for j in range(3):
            a, b = sorted((int(f[j]), int(f[(j + 1) % 3])))
            cnt[(a, b)] += 1
    return {x for (a, b), n in cnt.items() if n == 1 for x in (a, b)}


def test_open_mesh_vertex_gradient_vs_finite_differences_full_size(dev, orc):
    """(iii) The open variant of the differentiable workload at its full 64^3 grid: dL/dV
    of the sigmoid-MSE loss against FP64 central differences (h = 1e-6) of the oracle's
    loss, on the 8 rim vertices with the largest gradient (1e-3 relative).
    Moving vertex v changes only the faces that use it, so the perturbed field is
    W - W_adj(V) + W_adj(V +- h e_d), with W_adj the oracle's sum over v's faces: the
    same FP64 loss as a full re-evaluation, at a few faces' cost per difference.
    Interior vertices carry no gradient (W depends only on the boundary)."""
    c = wi.config3_differentiable(res=64, open_variant=True)
    Wr, Lr, g32, Q = _oracle_dLdW(orc, c)
    Dg, Tg = _gpu_adjoint(c, g32)
    V64 = _f32(c.V)
    _, Dr = orc.grad(V64, c.F, Q, g32.astype(np.float64))
    rim = _rim_vertices(c.F)
    mag = np.linalg.norm(Dr, axis=1)
    picks = [v for v in np.argsort(-mag) if v in rim][:8]
    assert len(picks) == 8
    h = 1e-6
    compared = 0
    for v in picks:
        adj = np.nonzero((c.F == v).any(axis=1))[0]
        Fa = c.F[adj]
        W_rest = Wr - orc.winding(V64, Fa, Q)
        for d in range(3):
            Vp, Vm = V64.copy(), V64.copy()
            Vp[v, d] += h
            Vm[v, d] -= h
            Lp = orc.sigmoid_mse(W_rest + orc.winding(Vp, Fa, Q), c.target, c.tau, c.k)[0]
            Lm = orc.sigmoid_mse(W_rest + orc.winding(Vm, Fa, Q), c.target, c.tau, c.k)[0]
            fd = (Lp - Lm) / (2 * h)
            if abs(fd) > 1e-2 * mag[picks[0]]:
                print(f"v={v} d={d} gpu={Dg[v, d]:.6e} fd={fd:.6e} rel={abs(Dg[v, d] - fd) / abs(fd):.2e}",
                      flush=True)
                assert Dg[v, d] == pytest.approx(fd, rel=1e-3)
                compared += 1
    assert compared >= 12
    interior = np.array(sorted(set(range(len(c.V))) - rim))
    assert np.abs(Dg[interior]).max() <= 1e-3 * np.abs(Dg).max()


def test_autograd_function_matches_direct_calls(dev):
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config3_differentiable(res=16, open_variant=True)
    Vt, Ft = _to_dev(c)
    V = Vt.clone().requires_grad_(True)
    occ = wn.soft_occupancy(V, Ft, grid=c.grid, tau=0.5, k=50.0)
    T = torch.as_tensor(c.target).cuda().reshape(occ.shape)
    loss = ((occ - T) ** 2).mean()
    loss.backward()
    W = wn.wn_voxelize(Vt, Ft, grid=c.grid).reshape(-1)
    _, dLdW = wn.wn_sigmoid_mse(W, T.reshape(-1), 0.5, 50.0)
    dLdV = wn.wn_backward(Vt, Ft, dLdW, grid=c.grid)
    torch.cuda.synchronize()
    torch.testing.assert_close(V.grad, dLdV, rtol=1e-4, atol=1e-7 * float(dLdV.abs().max()))
    # the strip-order forward and the face-pair adjoint through the same Function
    R = torch.as_tensor(wn.wn_build_strips(c.F, len(c.V))).cuda()
    P = torch.as_tensor(wn.wn_build_face_pairs(c.F, len(c.V))).cuda()
    V2 = Vt.clone().requires_grad_(True)
    occ2 = wn.soft_occupancy(V2, Ft, grid=c.grid, tau=0.5, k=50.0, strips=R, pairs=P)
    ((occ2 - T) ** 2).mean().backward()
    W2 = wn.wn_voxelize_strips(Vt, Ft, R, grid=c.grid).reshape(-1)
    _, dLdW2 = wn.wn_sigmoid_mse(W2, T.reshape(-1), 0.5, 50.0)
    dLdV2 = wn.wn_backward(Vt, Ft, dLdW2, grid=c.grid, pairs=P)
    torch.cuda.synchronize()
    torch.testing.assert_close(occ2, occ, rtol=0, atol=1e-4)
    torch.testing.assert_close(V2.grad, dLdV2, rtol=1e-4, atol=1e-7 * float(dLdV2.abs().max()))
    torch.testing.assert_close(V2.grad, V.grad, rtol=0, atol=1e-3 * float(V.grad.abs().max()))


def test_backward_edge_cases(dev, orc):
    import torch
    import paper_2407_11272_amd as wn
    V = torch.rand((5, 3), device="cuda")
    F0 = torch.zeros((0, 3), dtype=torch.int32, device="cuda")
    g = torch.ones(8, device="cuda")
    d = wn.wn_backward(V, F0, g, grid=wn.Grid.cube(2))
    torch.cuda.synchronize()
    assert torch.all(d == 0)
    # an unreferenced vertex gets exactly 0; two runs are bit-identical
    c = wi.config1_icosphere()
    Vn = np.concatenate([c.V, [[0.9, 0.9, 0.9]]])
    Vt, Ft = wn.as_mesh(torch.as_tensor(Vn), torch.as_tensor(c.F))
    gg = torch.randn(16 ** 3, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    d1, t1 = wn.wn_backward(Vt, Ft, gg, grid=wn.Grid.cube(16), want_dLdT=True)
    d2, t2 = wn.wn_backward(Vt, Ft, gg, grid=wn.Grid.cube(16), want_dLdT=True)
    torch.cuda.synchronize()
    assert float(d1[-1].abs().max()) == 0.0
    torch.testing.assert_close(d1, d2, rtol=0, atol=0)
    torch.testing.assert_close(t1, t2, rtol=0, atol=0)
    # point-list mode against the oracle on a tiny mesh, ragged point count
    rng = np.random.default_rng(7)
    Vs = rng.uniform(-0.5, 0.5, (9, 3))
    Fs = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8], [0, 4, 8]])
    Q = rng.uniform(-0.6, 0.6, (777, 3)).astype(np.float32).astype(np.float64)
    gq = rng.normal(size=777)
    Vt, Ft = wn.as_mesh(torch.as_tensor(Vs), torch.as_tensor(Fs))
    dg, tg = wn.wn_backward(Vt, Ft, torch.as_tensor(gq, dtype=torch.float32).cuda(),
                            Q=torch.as_tensor(Q, dtype=torch.float32).cuda(), want_dLdT=True)
    torch.cuda.synchronize()
    Tr, Dr = orc.grad(_f32(Vs), Fs, Q, np.asarray(gq, np.float32).astype(np.float64))
    guard = orc.guard_mask(_f32(Vs), Fs, Q)
    assert guard.sum() == 0
    np.testing.assert_allclose(tg.cpu().numpy(), Tr, rtol=1e-3, atol=1e-4 * np.abs(Tr).max())
    np.testing.assert_allclose(dg.cpu().numpy(), Dr, rtol=1e-3, atol=1e-4 * np.abs(Dr).max())


def test_sliced_adjoint_equals_one_call_and_the_oracle(dev, orc):
    """wn_backward_range: consecutive ranges of whole 256-point tiles in increasing order
    (shorter and longer than one round over the splits, the last reaching the final
    point) give the same bits as wn_backward, and hold the oracle's bar (i)."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config3_differentiable(res=64, open_variant=True)
    Vt, Ft = _to_dev(c)
    P = c.grid.size
    g = torch.randn(P, device="cuda", generator=torch.Generator("cuda").manual_seed(11))
    Dw, Tw = wn.wn_backward(Vt, Ft, g, grid=c.grid, want_dLdT=True)
    one = wn.SlicedBackward(Vt, Ft, grid=c.grid)
    tiles = -(-P // one.tile)
    print(f"[sliced] {P} points, {tiles} tiles, {one.splits} splits", flush=True)
    assert 1 < one.splits < tiles   # so that ranges can be shorter and longer than a round
    one.begin()
    one.points(0, P, g)
    T0 = torch.empty((len(c.F), 3, 3), device="cuda")
    D0 = one.end(dLdT=T0)
    torch.cuda.synchronize()
    assert torch.equal(D0, Dw) and torch.equal(T0, Tw)
    rng = np.random.default_rng(5)
    for trial in range(4):
        cuts = np.sort(rng.choice(np.arange(1, tiles), size=7 if trial < 3 else tiles - 1, replace=False))
        bounds = [0] + [int(x) * one.tile for x in cuts] + [P]
        sb = wn.SlicedBackward(Vt, Ft, grid=c.grid)
        sb.begin()
        for a, b in zip(bounds[:-1], bounds[1:]):
            sb.points(a, b - a, g)
        T2 = torch.empty_like(T0)
        D2 = sb.end(dLdT=T2)
        torch.cuda.synchronize()
        print(f"[sliced] trial {trial}: {len(bounds) - 1} ranges, tiles per range "
              f"{sorted(set(np.diff(bounds) // one.tile))[:8]}", flush=True)
        assert torch.equal(D2, Dw) and torch.equal(T2, Tw)
    Tr, _ = orc.grad(_f32(c.V), c.F, orc.grid_points(c.grid), g.cpu().numpy().astype(np.float64))
    _check_T(T0.cpu().numpy().astype(np.float64).reshape(-1), Tr.reshape(-1), "sliced")
    # ranges out of order are refused by the binding before anything is launched
    sb = wn.SlicedBackward(Vt, Ft, grid=c.grid)
    sb.begin()
    with pytest.raises(ValueError):
        sb.points(one.tile, P - one.tile, g)
    with pytest.raises(ValueError):
        sb.end()


def test_sliced_adjoint_point_list_and_argument_errors(dev, orc):
    import ctypes
    import torch
    import paper_2407_11272_amd as wn
    from paper_2407_11272_amd import _lib as L
    rng = np.random.default_rng(9)
    Vs = rng.uniform(-0.5, 0.5, (9, 3))
    Fs = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8], [0, 4, 8]])
    Q = rng.uniform(-0.6, 0.6, (1000, 3)).astype(np.float32)
    gq = rng.normal(size=1000).astype(np.float32)
    Vt, Ft = wn.as_mesh(torch.as_tensor(Vs), torch.as_tensor(Fs))
    Qt, gt = torch.as_tensor(Q).cuda(), torch.as_tensor(gq).cuda()
    sb = wn.SlicedBackward(Vt, Ft, Q=Qt)
    sb.begin()
    sb.points(0, 256, gt)
    sb.points(256, 512, gt)
    sb.points(768, 232, gt)   # the ragged last tile
    D = sb.end()
    Dw = wn.wn_backward(Vt, Ft, gt, Q=Qt)
    torch.cuda.synchronize()
    assert torch.equal(D, Dw)
    _, Dr = orc.grad(_f32(Vs), Fs, Q.astype(np.float64), gq.astype(np.float64))
    np.testing.assert_allclose(D.cpu().numpy(), Dr, rtol=1e-3, atol=1e-4 * np.abs(Dr).max())
    # argument errors, before any launch
    lib = L.load()
    p = ctypes.c_void_p
    s = p(torch.cuda.current_stream().cuda_stream)
    need = wn.wn_workspace_size(L.WN_OP_BACKWARD, 9, 4, 1000)
    ws = torch.zeros(need + 256, dtype=torch.uint8, device="cuda")
    base = p(ws.data_ptr() + (-ws.data_ptr()) % 256)
    dV = torch.empty_like(Vt)

    dT = torch.empty((4, 3, 3), dtype=torch.float32, device="cuda")

    def call(p0, n, flags=0, wsb=need, dLdV=dV, pairs=None, n_pairs=0, dLdT=None):
        return lib.wn_backward_range(p(Vt.data_ptr()), 9, p(Ft.data_ptr()), 4, pairs, n_pairs, None,
                                     p(Qt.data_ptr()), 1000, p(gt.data_ptr()), p0, n, flags,
                                     p(dLdV.data_ptr()) if dLdV is not None else None,
                                     p(dLdT.data_ptr()) if dLdT is not None else None, base, wsb, s)

    assert call(0, 0, L.WN_BWD_BEGIN) == L.WN_OK
    assert call(100, 256) == L.WN_ERR_INVALID_ARG          # p0 not on a tile boundary
    assert call(0, 300) == L.WN_ERR_INVALID_ARG            # n not whole tiles and not the end
    assert call(768, 233) == L.WN_ERR_INVALID_ARG          # past the last point
    assert call(-256, 256) == L.WN_ERR_INVALID_ARG
    assert call(0, 256, 8) == L.WN_ERR_INVALID_ARG         # unknown flag
    # per-vertex sums only: no dL/dT at the end
    assert call(0, 0, L.WN_BWD_END | L.WN_BWD_VERTEX_SUMS, dLdT=dT) == L.WN_ERR_INVALID_ARG
    assert call(0, 0, L.WN_BWD_END, dLdV=None) == L.WN_ERR_INVALID_ARG
    assert call(0, 256, wsb=need - 1) == L.WN_ERR_WORKSPACE
    pr = torch.tensor([[0, 3], [1, 2]], dtype=torch.int32, device="cuda")
    assert call(0, 256, pairs=p(pr.data_ptr()), n_pairs=1) == L.WN_ERR_INVALID_ARG   # fewer than nF / 2 entries
    assert call(0, 256, pairs=p(pr.data_ptr()), n_pairs=5) == L.WN_ERR_INVALID_ARG   # more than nF
    assert call(0, 256, pairs=None, n_pairs=2) == L.WN_ERR_INVALID_ARG
    torch.cuda.synchronize()


@pytest.mark.parametrize("case", ["closed", "open"])
def test_face_pair_adjoint_matches_one_face_per_lane_and_the_oracle(dev, orc, case):
    """Two faces per lane (wn_build_face_pairs): the same per-face arithmetic as one face
    per lane, so dL/dT within 5e-4 of its scale of that kernel's; both against the oracle
    (bars (i) and (ii)) on the differentiable workload at 64^3 (the open variant has
    unpaired faces at its holes); consecutive ranges give the same bits as one call."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config3_differentiable(res=64, open_variant=(case == "open"))
    Wr, Lr, g32, Q = _oracle_dLdW(orc, c)
    Vt, Ft = _to_dev(c)
    g = torch.as_tensor(g32).cuda()
    pairs_h = wn.wn_build_face_pairs(c.F, len(c.V))
    pairs = torch.as_tensor(pairs_h).cuda()
    print(f"[pairs {case}] {len(c.F)} faces -> {len(pairs_h)} lanes, {(pairs_h[:, 1] < 0).sum()} unpaired", flush=True)
    D1, T1 = wn.wn_backward(Vt, Ft, g, grid=c.grid, want_dLdT=True)
    D2, T2 = wn.wn_backward(Vt, Ft, g, grid=c.grid, want_dLdT=True, pairs=pairs)
    assert wn.wn_get_device_error() == 0
    sb = wn.SlicedBackward(Vt, Ft, grid=c.grid, pairs=pairs)
    sb.begin()
    P = c.grid.size
    cut = [0, 256 * 7, 256 * 400, 256 * 401, P]
    for a, b in zip(cut[:-1], cut[1:]):
        sb.points(a, b - a, g)
    T3 = torch.empty_like(T2)
    D3 = sb.end(dLdT=T3)
    torch.cuda.synchronize()
    assert torch.equal(D3, D2) and torch.equal(T3, T2)
    T1n, T2n = T1.cpu().numpy().astype(np.float64), T2.cpu().numpy().astype(np.float64)
    scale = np.abs(T1n).max()
    print(f"[pairs {case}] |pairs - one face per lane| / scale = {np.abs(T2n - T1n).max() / scale:.2e}", flush=True)
    # the same per-face formula, rounded differently (E's sum order, contractions); the
    # sums over 262 144 points cancel, which amplifies the difference
    assert np.abs(T2n - T1n).max() <= 5e-4 * scale
    Tr, Dr = orc.grad(_f32(c.V), c.F, Q, g32.astype(np.float64))
    _check_T(T2n.reshape(-1), Tr.reshape(-1), f"pairs {case} dL/dT")
    _check_V(D2.cpu().numpy().astype(np.float64), Dr, Tr, c.F, f"pairs {case} dL/dV")
    # the two faces of a pair sharing their sums at the shared edge (dL/dV only): the
    # same vertex sums in another grouping, against the oracle; ranges give the same bits
    D4 = wn.wn_backward(Vt, Ft, g, grid=c.grid, pairs=pairs)
    sb = wn.SlicedBackward(Vt, Ft, grid=c.grid, pairs=pairs, vertex_sums=True)
    sb.begin()
    for a, b in zip(cut[:-1], cut[1:]):
        sb.points(a, b - a, g)
    with pytest.raises(ValueError):
        sb.end(dLdT=T3)
    D5 = sb.end()
    torch.cuda.synchronize()
    assert wn.wn_get_device_error() == 0
    assert torch.equal(D5, D4)
    D2n, D4n = D2.cpu().numpy().astype(np.float64), D4.cpu().numpy().astype(np.float64)
    print(f"[pairs {case}] |merged - per corner| / scale = {np.abs(D4n - D2n).max() / np.abs(D2n).max():.2e}",
          flush=True)
    _check_V(D4n, Dr, Tr, c.F, f"pairs {case} merged dL/dV")


def test_vertex_sums_with_unpaired_faces(dev, orc):
    """Shared vertex sums with lanes that hold one face, on the open variant of the
    differentiable mesh at 32^3: every face alone (no lane has a second face; the same
    arithmetic as the per-corner sums, up to the compiler's contractions), and a list in
    which every third pair is split into two single faces, so that waves mix lanes with
    and without a second face; both against the oracle."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config3_differentiable(res=32, open_variant=True)
    Wr, Lr, g32, Q = _oracle_dLdW(orc, c)
    Vt, Ft = _to_dev(c)
    g = torch.as_tensor(g32).cuda()
    nF = len(c.F)
    alone = torch.as_tensor(np.stack([np.arange(nF), np.full(nF, -1)], 1).astype(np.int32)).cuda()
    Tr, Dr = orc.grad(_f32(c.V), c.F, Q, g32.astype(np.float64))
    Da = wn.wn_backward(Vt, Ft, g, grid=c.grid, pairs=alone, vertex_sums=False)
    Db = wn.wn_backward(Vt, Ft, g, grid=c.grid, pairs=alone, vertex_sums=True)
    torch.cuda.synchronize()
    assert wn.wn_get_device_error() == 0
    Dan, Dbn = Da.cpu().numpy().astype(np.float64), Db.cpu().numpy().astype(np.float64)
    print(f"[vertex sums] singles: |merged - per corner|_inf = {np.abs(Dbn - Dan).max():.3e} "
          f"of {np.abs(Dan).max():.3e}", flush=True)
    _check_V(Dbn, Dr, Tr, c.F, "single lanes merged dL/dV")
    P = wn.wn_build_face_pairs(c.F, len(c.V))
    mixed = []
    for i, (f, h) in enumerate(P.tolist()):
        if h >= 0 and i % 3 == 0:
            mixed += [[f, -1], [h, -1]]
        else:
            mixed.append([f, h])
    mixed = np.asarray(mixed, np.int32)
    print(f"[vertex sums] {nF} faces, {len(P)} pairs -> {len(mixed)} lanes, {(mixed[:, 1] < 0).sum()} single",
          flush=True)
    Dm = wn.wn_backward(Vt, Ft, g, grid=c.grid, pairs=torch.as_tensor(mixed).cuda())
    torch.cuda.synchronize()
    assert wn.wn_get_device_error() == 0
    _check_V(Dm.cpu().numpy().astype(np.float64), Dr, Tr, c.F, "mixed lanes merged dL/dV")
    with pytest.raises(ValueError):
        wn.wn_backward(Vt, Ft, g, grid=c.grid, pairs=alone, want_dLdT=True, vertex_sums=True)


def test_merged_adjoint_with_wide_splits_at_128(dev, orc):
    """At 128^3 (8192 tiles, at least 12 per split) the merged pair adjoint takes twice its
    splits in a doubled running-sum space: point ranges give the same bits as one call,
    and dL/dV at 8 rim and 8 interior vertices of the open differentiable mesh (seeded
    choices, with every face around them) holds to the oracle for a seeded dL/dW."""
    import torch
    import paper_2407_11272_amd as wn
    L = wn._lib
    c = wi.config3_differentiable(res=128, open_variant=True)
    Vt, Ft = _to_dev(c)
    P, nF = c.grid.size, len(c.F)
    splits = int(L.load().wn_backward_splits(nF, P))
    assert P // 256 >= 12 * splits
    assert wn.wn_workspace_size(L.WN_OP_BACKWARD, len(c.V), nF, P) >= 2 * 72 * splits * nF
    rng = np.random.default_rng(11)
    g32 = rng.standard_normal(P).astype(np.float32)
    g = torch.as_tensor(g32).cuda()
    pairs = torch.as_tensor(wn.wn_build_face_pairs(c.F, len(c.V))).cuda()
    D = wn.wn_backward(Vt, Ft, g, grid=c.grid, pairs=pairs)
    sb = wn.SlicedBackward(Vt, Ft, grid=c.grid, pairs=pairs, vertex_sums=True)
    sb.begin()
    cut = [0, 256 * 5, 256 * 3000, 256 * 3001, P]
    for a, b in zip(cut[:-1], cut[1:]):
        sb.points(a, b - a, g)
    D2 = sb.end()
    torch.cuda.synchronize()
    assert wn.wn_get_device_error() == 0
    assert torch.equal(D, D2)
    F = np.asarray(c.F)
    edges = np.sort(F[:, [[0, 1], [1, 2], [2, 0]]].reshape(-1, 2), axis=1)
    uniq, cnt = np.unique(edges, axis=0, return_counts=True)
    rim = np.unique(uniq[cnt == 1])
    interior = np.setdiff1d(np.arange(len(c.V)), rim)
    vs = np.concatenate([rng.choice(rim, 8, replace=False), rng.choice(interior, 8, replace=False)])
    faces = np.nonzero(np.isin(F, vs).any(axis=1))[0]
    Tr, Dr = orc.grad(_f32(c.V), F[faces], orc.grid_points(c.grid), g32.astype(np.float64))
    Dg = Dr.copy()
    Dg[vs] = D.cpu().numpy().astype(np.float64)[vs]
    print(f"[wide splits] {splits} base splits, {len(faces)} faces around {len(vs)} vertices; "
          f"|dL/dV| at the rim up to {np.abs(Dr[vs[:8]]).max():.3e}", flush=True)
    _check_V(Dg, Dr, Tr, F[faces], "128^3 merged, wide splits, sampled dL/dV")


def test_face_pairs_that_break_the_rules_are_reported(dev):
    """A face left out of the pairs, a face given twice, and a pair without a shared edge
    are recorded as bad indices; a valid list is not."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config1_icosphere(res=8)
    Vt, Ft = wn.as_mesh(torch.as_tensor(c.V), torch.as_tensor(c.F))
    g = torch.ones(c.grid.size, device="cuda")
    P = wn.wn_build_face_pairs(c.F, len(c.V))
    missing = P.copy()
    i = int(np.nonzero(missing[:, 1] >= 0)[0][0])
    missing[i, 1] = -1                                  # face g of pair i appears nowhere
    twice = P.copy()
    twice[i, 1] = twice[i + 1, 0]                       # a face in two pairs
    for name, pp, expect in (("valid", P, 0), ("missing", missing, wn._lib.WN_ERR_BAD_INDEX),
                             ("twice", twice, wn._lib.WN_ERR_BAD_INDEX)):
        d = wn.wn_backward(Vt, Ft, g, grid=c.grid, pairs=torch.as_tensor(pp).cuda())
        assert wn.wn_get_device_error() == expect, name
        assert torch.isfinite(d).all() or expect != 0
    # a pair of two faces that share no edge keeps only its first face: reported
    bad = P.copy()
    a0 = int(bad[i, 0])
    b0 = next(k for k in range(len(c.F)) if not (set(c.F[k].tolist()) & set(c.F[a0].tolist())))
    rows = np.nonzero((bad == b0).any(axis=1))[0]
    r = int(rows[0])
    partner = bad[r, 1] if bad[r, 0] == b0 else bad[r, 0]
    other = bad[i, 1]
    bad[i] = [a0, b0]
    bad[r] = [partner, other] if partner >= 0 else [other, -1]
    d = wn.wn_backward(Vt, Ft, g, grid=c.grid, pairs=torch.as_tensor(bad).cuda())
    assert wn.wn_get_device_error() == wn._lib.WN_ERR_BAD_INDEX
