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


def _gpu_loss_grad(c):
    """Forward, sigmoid-MSE loss and its gradient, adjoint: all in the HIP library."""
    import torch
    import paper_2407_11272_amd as wn
    Vt, Ft = _to_dev(c)
    W = wn.wn_voxelize(Vt, Ft, grid=c.grid).reshape(-1)
    T = torch.as_tensor(c.target).cuda()
    loss, dLdW = wn.wn_sigmoid_mse(W, T, c.tau, c.k)
    dLdV, dLdT = wn.wn_backward(Vt, Ft, dLdW, grid=c.grid, want_dLdT=True)
    torch.cuda.synchronize()
    return (W.cpu().numpy().astype(np.float64), float(loss.item()), dLdW.cpu().numpy().astype(np.float64),
            dLdV.cpu().numpy().astype(np.float64), dLdT.cpu().numpy().astype(np.float64))


def _f32(V):
    return np.asarray(V, np.float32).astype(np.float64)


def _check_T(Tg, Tr, label):
    scale = np.abs(Tr).max()
    d = np.abs(Tg - Tr)
    big = np.abs(Tr) > 1e-2 * scale
    rel = d[big] / np.abs(Tr[big])
    print(f"[{label}] |dL/dT|inf={scale:.3e} max abs err={d.max():.3e} max rel (big)={rel.max():.3e}", flush=True)
    assert d.max() <= 1e-3 * scale
    assert rel.max() <= 1e-3


def test_corner_and_vertex_gradients_32(dev, orc):
    """(i) + (ii) on the differentiable workload's mesh at 32^3, every face."""
    c = wi.config3_differentiable(res=32)
    Wg, Lg, gg, Dg, Tg = _gpu_loss_grad(c)
    V64 = _f32(c.V)
    Q = orc.grid_points(c.grid)
    # the gradient is taken at the GPU's dL/dW so only the adjoint is compared here
    Tr, Dr = orc.grad(V64, c.F, Q, gg)
    _check_T(Tg.reshape(-1), Tr.reshape(-1), "C3@32 dL/dT")
    corner_abs = np.zeros_like(Dr)
    np.add.at(corner_abs, c.F.reshape(-1), np.abs(Tr.reshape(-1, 3)))
    assert np.all(np.abs(Dg - Dr) <= 1e-3 * corner_abs + 1e-12)
    # the loss itself against the oracle's forward
    Lr, gr = orc.sigmoid_mse(orc.winding(V64, c.F, Q), c.target, c.tau, c.k)
    assert Lg == pytest.approx(Lr, rel=1e-4)


def test_corner_gradients_full_size_sampled_faces(dev, orc):
    """(i) at the full 64^3 grid for 96 seeded faces (the oracle's cost is per face)."""
    c = wi.config3_differentiable(res=64)
    Wg, Lg, gg, Dg, Tg = _gpu_loss_grad(c)
    rng = np.random.default_rng(200)
    fs = np.sort(rng.choice(len(c.F), 96, replace=False))
    Tr, _ = orc.grad(_f32(c.V), c.F[fs], orc.grid_points(c.grid), gg)
    _check_T(Tg[fs].reshape(-1), Tr.reshape(-1), "C3@64 dL/dT sampled")


def test_open_mesh_vertex_gradient_vs_finite_differences(dev, orc):
    """(iii) Open variant at 24^3: the full sigmoid-MSE loss differentiated by FP64
    central differences of the oracle (h = 1e-6) on the rim vertices with the largest
    gradient; interior vertices carry no gradient."""
    c = wi.config3_differentiable(res=24, open_variant=True)
    Wg, Lg, gg, Dg, Tg = _gpu_loss_grad(c)
    V64 = _f32(c.V)
    Q = orc.grid_points(c.grid)
    _, Dr = orc.grad(V64, c.F, Q, orc.sigmoid_mse(orc.winding(V64, c.F, Q), c.target, c.tau, c.k)[1])
    mag = np.linalg.norm(Dr, axis=1)
    picks = np.argsort(-mag)[:4]
    h = 1e-6
    for v in picks:
        for d in range(3):
            Vp, Vm = V64.copy(), V64.copy()
            Vp[v, d] += h
            Vm[v, d] -= h
            Lp = orc.sigmoid_mse(orc.winding(Vp, c.F, Q), c.target, c.tau, c.k)[0]
            Lm = orc.sigmoid_mse(orc.winding(Vm, c.F, Q), c.target, c.tau, c.k)[0]
            fd = (Lp - Lm) / (2 * h)
            if abs(fd) > 1e-2 * mag[picks[0]]:
                print(f"v={v} d={d} gpu={Dg[v, d]:.6e} fd={fd:.6e}", flush=True)
                assert Dg[v, d] == pytest.approx(fd, rel=1e-3)
    # interior (not on a hole rim) vertices: zero up to FP32 cancellation
    from collections import Counter
    cnt = Counter()
    for f in c.F:
        for j in range(3):
            a, b = sorted((f[j], f[(j + 1) % 3]))
            cnt[(a, b)] += 1
    rim = {x for (a, b), n in cnt.items() if n == 1 for x in (a, b)}
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
    """wn_backward_range: ranges of whole splits in any order and grouping give the same
    bits as one call with the same split size; split size 0 is wn_backward bit for bit;
    and the sliced result holds the oracle's bar (i)."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config3_differentiable(res=32, open_variant=True)
    Vt, Ft = _to_dev(c)
    P = c.grid.size
    g = torch.randn(P, device="cuda", generator=torch.Generator("cuda").manual_seed(11))
    # chunk 0: the same as wn_backward
    sb0 = wn.SlicedBackward(Vt, Ft, grid=c.grid)
    sb0.begin()
    sb0.points(0, P, g)
    T0 = torch.empty((len(c.F), 3, 3), device="cuda")
    D0 = sb0.end(dLdT=T0)
    Dw, Tw = wn.wn_backward(Vt, Ft, g, grid=c.grid, want_dLdT=True)
    torch.cuda.synchronize()
    assert torch.equal(D0, Dw) and torch.equal(T0, Tw)
    # chunk 1280 (not a multiple of the 256-point tile): 26 splits, the last ragged
    chunk = 1280
    one = wn.SlicedBackward(Vt, Ft, grid=c.grid, chunk=chunk)
    assert one.chunk == chunk and one.splits == -(-P // chunk)
    one.begin()
    one.points(0, P, g)
    T1 = torch.empty_like(T0)
    D1 = one.end(dLdT=T1)
    rng = np.random.default_rng(5)
    for trial in range(3):
        cuts = np.sort(rng.choice(np.arange(1, one.splits), size=6, replace=False))
        bounds = [0] + [int(x) * chunk for x in cuts] + [P]
        ranges = [(bounds[i], bounds[i + 1] - bounds[i]) for i in range(len(bounds) - 1)]
        rng.shuffle(ranges)
        sb = wn.SlicedBackward(Vt, Ft, grid=c.grid, chunk=chunk)
        sb.begin()
        for p0, n in ranges:
            sb.points(p0, n, g)
        T2 = torch.empty_like(T0)
        D2 = sb.end(dLdT=T2)
        torch.cuda.synchronize()
        print(f"[sliced] trial {trial}: {len(ranges)} ranges, order {[p0 // chunk for p0, _ in ranges]}", flush=True)
        assert torch.equal(D1, D2) and torch.equal(T1, T2)
    # the split size changes only the summation order: the oracle's bar (i)
    Tr, _ = orc.grad(_f32(c.V), c.F, orc.grid_points(c.grid), g.cpu().numpy().astype(np.float64))
    _check_T(T1.cpu().numpy().astype(np.float64).reshape(-1), Tr.reshape(-1), "sliced chunk 1280")


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
    sb = wn.SlicedBackward(Vt, Ft, Q=Qt, chunk=256)
    sb.begin()
    sb.points(768, 232, gt)   # the ragged last split first
    sb.points(0, 768, gt)
    D = sb.end()
    Dw = wn.wn_backward(Vt, Ft, gt, Q=Qt)
    torch.cuda.synchronize()
    _, Dr = orc.grad(_f32(Vs), Fs, Q.astype(np.float64), gq.astype(np.float64))
    np.testing.assert_allclose(D.cpu().numpy(), Dr, rtol=1e-3, atol=1e-4 * np.abs(Dr).max())
    np.testing.assert_allclose(D.cpu().numpy(), Dw.cpu().numpy(), rtol=1e-4, atol=1e-5 * np.abs(Dr).max())
    # argument errors, before any launch
    lib = L.load()
    p = ctypes.c_void_p
    s = p(torch.cuda.current_stream().cuda_stream)
    need = lib.wn_workspace_size_backward(9, 4, 1000, 256)
    ws = torch.zeros(need + 256, dtype=torch.uint8, device="cuda")
    base = p(ws.data_ptr() + (-ws.data_ptr()) % 256)
    dV = torch.empty_like(Vt)

    def call(p0, n, flags=0, chunk=256, wsb=need, dLdV=dV):
        return lib.wn_backward_range(p(Vt.data_ptr()), 9, p(Ft.data_ptr()), 4, None, p(Qt.data_ptr()), 1000,
                                     p(gt.data_ptr()), chunk, p0, n, flags, p(dLdV.data_ptr()) if dLdV is not None
                                     else None, None, base, wsb, s)

    assert call(0, 0, L.WN_BWD_BEGIN) == L.WN_OK
    assert call(100, 256) == L.WN_ERR_INVALID_ARG          # p0 not on a split boundary
    assert call(0, 300) == L.WN_ERR_INVALID_ARG            # n not whole splits and not the end
    assert call(768, 233) == L.WN_ERR_INVALID_ARG          # past the last point
    assert call(0, 256, 4) == L.WN_ERR_INVALID_ARG         # unknown flag
    assert call(0, 0, L.WN_BWD_END, dLdV=None) == L.WN_ERR_INVALID_ARG
    assert call(0, 256, chunk=-1) == L.WN_ERR_INVALID_ARG
    assert call(0, 256, wsb=need - 1) == L.WN_ERR_WORKSPACE
    Q2 = torch.zeros((70000, 3), device="cuda")
    g2 = torch.zeros(70000, device="cuda")
    assert lib.wn_backward_range(p(Vt.data_ptr()), 9, p(Ft.data_ptr()), 4, None, p(Q2.data_ptr()), 70000,
                                 p(g2.data_ptr()), 1, 0, 1, 0, None, None, base, need, s) == L.WN_ERR_INVALID_ARG
    torch.cuda.synchronize()
