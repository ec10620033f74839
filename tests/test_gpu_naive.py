"""GPU parity of the naive flux integral (Eq. 4) and its adjoint against the FP64 oracle.

The sum has no bounded condition number near the surface (terms grow like 1/|c - q|^2),
so the forward tolerance follows the FP32 error model: arithmetic rounding relative to
the sum of absolute terms S(q) that the oracle returns, plus the rounding of the inputs
(voxel centres and centroids, about 6e-8 relative) amplified by 3/|c - q| per term:
|W_gpu - W_ref| <= 1e-5 S + 5e-7 S2 + 2e-6 with S2 = 1/(8 pi) sum |term| / |c - q|.  Gradients: dL/dT elementwise 1e-3 relative
where |ref| > 1e-2 |ref|_inf, and dL/dV (not vanishing here) to 1e-3 |ref|_inf.
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


def _mesh(c):
    import torch
    import paper_2407_11272_amd as wn
    return wn.as_mesh(torch.as_tensor(np.asarray(c.V, np.float32)), torch.as_tensor(c.F))


def _input_scale(V, F, Q):
    """S2(q) = 1/(8 pi) sum_f |<N_f, c_f - q>| / |c_f - q|^4 (FP64, numpy)."""
    V = np.asarray(V, np.float64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    N = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0
    out = np.empty(len(Q))
    for i0 in range(0, len(Q), 256):
        r = cen[None, :, :] - Q[i0:i0 + 256, None, :]
        d = np.linalg.norm(r, axis=-1)
        t = np.abs(np.einsum("qfd,fd->qf", r, N)) / np.maximum(d, 1e-300) ** 4
        out[i0:i0 + 256] = t.sum(1) / (8 * np.pi)
    return out


@pytest.mark.parametrize("cfg", ["c1", "c3", "c2"])
def test_naive_forward_matches_oracle(dev, orc, cfg):
    import paper_2407_11272_amd as wn
    c = {"c1": wi.config1_icosphere, "c3": wi.config3_differentiable, "c2": wi.config2_ellipsoid_union}[cfg]()
    Vt, Ft = _mesh(c)
    W = wn.wn_voxelize_naive(Vt, Ft, grid=c.grid).cpu().numpy().reshape(-1)
    Q = orc.grid_points(c.grid)
    idx = np.random.default_rng(21).choice(len(Q), 2000, replace=False)
    V64 = np.asarray(c.V, np.float32).astype(np.float64)
    Wr, S = orc.winding_naive(V64, c.F, Q[idx], with_scale=True)
    S2 = _input_scale(V64, c.F, Q[idx])
    err = np.abs(W[idx] - Wr)
    print(f"[naive {cfg}] max|dW|={err.max():.2e} max err/(1e-5 S + 5e-7 S2 + 2e-6)="
          f"{np.max(err / (1e-5 * S + 5e-7 * S2 + 2e-6)):.2f}", flush=True)
    assert np.all(err <= 1e-5 * S + 5e-7 * S2 + 2e-6)


def test_naive_split_path(dev, orc):
    """Few points, many faces: face splits and the fixed-order reduction."""
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config2_ellipsoid_union()
    Vt, Ft = _mesh(c)
    Q = np.random.default_rng(22).uniform(-0.5, 0.5, (257, 3)).astype(np.float32).astype(np.float64)
    W = wn.wn_voxelize_naive(Vt, Ft, Q=torch.as_tensor(Q, dtype=torch.float32).cuda()).cpu().numpy()
    V64 = np.asarray(c.V, np.float32).astype(np.float64)
    Wr, S = orc.winding_naive(V64, c.F, Q, with_scale=True)
    assert np.all(np.abs(W - Wr) <= 1e-5 * S + 5e-7 * _input_scale(V64, c.F, Q) + 2e-6)


def test_naive_adjoint_matches_oracle(dev, orc):
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config3_differentiable(res=24)
    Vt, Ft = _mesh(c)
    rng = np.random.default_rng(23)
    g = rng.normal(size=c.grid.size).astype(np.float32)
    dLdV, dLdT = wn.wn_backward_naive(Vt, Ft, torch.as_tensor(g).cuda(), grid=c.grid, want_dLdT=True)
    Tg, Dg = dLdT.cpu().numpy().reshape(-1), dLdV.cpu().numpy()
    Tr, Dr = orc.grad_naive(np.asarray(c.V, np.float32).astype(np.float64), c.F, orc.grid_points(c.grid),
                            g.astype(np.float64))
    Tr = Tr.reshape(-1)
    big = np.abs(Tr) > 1e-2 * np.abs(Tr).max()
    rel = np.abs(Tg - Tr)[big] / np.abs(Tr[big])
    print(f"[naive adjoint] dL/dT max rel={rel.max():.2e}  dL/dV max abs err / max={np.abs(Dg - Dr).max() / np.abs(Dr).max():.2e}",
          flush=True)
    assert rel.max() <= 1e-3
    assert np.abs(Dg - Dr).max() <= 1e-3 * np.abs(Dr).max()
    assert np.abs(Dr).max() > 0


def test_naive_autograd(dev):
    import torch
    import paper_2407_11272_amd as wn
    c = wi.config3_differentiable(res=16)
    Vt, Ft = _mesh(c)
    V = Vt.clone().requires_grad_(True)
    W = wn.naive_winding_number(V, Ft, grid=c.grid)
    T = torch.as_tensor(c.target).cuda().reshape(W.shape)
    loss = ((torch.sigmoid(20.0 * (W - 0.5)) - T) ** 2).mean()
    loss.backward()
    with torch.no_grad():
        W2 = wn.wn_voxelize_naive(Vt, Ft, grid=c.grid)
        s = torch.sigmoid(20.0 * (W2 - 0.5))
        gW = (2.0 * (s - T) * 20.0 * s * (1 - s) / W2.numel()).reshape(-1)
        d = wn.wn_backward_naive(Vt, Ft, gW, grid=c.grid)
    torch.testing.assert_close(V.grad, d, rtol=1e-4, atol=1e-6 * float(d.abs().max()))
    assert float(V.grad.abs().max()) > 0
