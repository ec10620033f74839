"""GPU parity of flipping duplication (Algorithm 2) and of voxelizing its result.

V2 is compared with the oracle's FP64 construction from the same float32 vertices
(|dV| <= 1e-6 absolute), F2 bit for bit; the winding number of the duplicated mesh
(computed on the GPU from the GPU's V2, F2) against the oracle's on its own
construction, |dW| <= 1e-4 off the guard band.
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


def _hemisphere():
    V, F = wi.uv_ellipsoid(48, 24, semi_axes=(0.4, 0.35, 0.3))
    cen = V[F].mean(1)
    return V, F[cen[:, 2] > 0]


@pytest.mark.parametrize("case", ["hemisphere", "open_icosphere", "octahedron"])
def test_flip_duplicate_matches_oracle(dev, orc, case):
    import torch
    import paper_2407_11272_amd as wn
    if case == "hemisphere":
        V, F = _hemisphere()
        eps = 0.02
    elif case == "open_icosphere":
        c = wi.config3_differentiable(open_variant=True)
        V, F, eps = c.V, c.F, 0.01
    else:
        V, F = wi.octahedron_mesh(0.45)
        eps = 0.05
    V32 = np.asarray(V, np.float32)
    Vt, Ft = wn.as_mesh(torch.as_tensor(V32), torch.as_tensor(F))
    V2, F2 = wn.wn_flip_duplicate(Vt, Ft, eps)
    torch.cuda.synchronize()
    assert wn.wn_get_device_error() == 0
    V2r, F2r = orc.flip_duplicate(V32.astype(np.float64), F, eps)
    np.testing.assert_array_equal(F2.cpu().numpy(), F2r)
    assert np.abs(V2.cpu().numpy() - V2r).max() <= 1e-6
    # the duplicate voxelizes like a closed mesh: the oracle's duplicate (rounded to FP32)
    # is the input of both sides
    grid = wi.Grid.cube(40)
    V2in = np.asarray(V2r, np.float32)
    V2d, F2d = wn.as_mesh(torch.as_tensor(V2in), torch.as_tensor(F2r))
    R = torch.as_tensor(wn.wn_build_strips(F2r, len(V2in))).cuda()
    W = wn.wn_voxelize_strips(V2d, F2d, R, grid=grid).cpu().numpy().reshape(-1)
    Q = orc.grid_points(grid)
    idx = np.random.default_rng(3).choice(len(Q), 4000, replace=False)
    V2g = V2in.astype(np.float64)
    Wr = orc.winding(V2g, F2r, Q[idx])
    guard = orc.guard_mask(V2g, F2r, Q[idx])
    err = np.abs(W[idx] - Wr)[~guard]
    print(f"[flip {case}] guard={guard.sum()} max|dW|={err.max():.2e} W in [{W.min():.3f}, {W.max():.3f}]", flush=True)
    assert err.max() <= 1e-4
    if case == "octahedron":
        l1 = np.abs(Q[idx]).sum(1)
        sure = ~guard & (np.abs(l1 - 0.45) > 1e-3) & (np.abs(l1 - 0.45 * (1 - eps / 0.45)) > 1e-3)
        inner = 0.45 - eps  # vertex normals of the octahedron are the axes: V' = V - eps * V/|V|
        expect = ((l1 < 0.45) & (l1 > inner)).astype(float)
        np.testing.assert_allclose(W[idx][sure], expect[sure], atol=1e-4)


def test_flip_duplicate_edge_cases(dev):
    import torch
    import paper_2407_11272_amd as wn
    V = torch.rand((7, 3), device="cuda")
    F = torch.zeros((0, 3), dtype=torch.int32, device="cuda")
    V2, F2 = wn.wn_flip_duplicate(V, F, 0.01)
    torch.cuda.synchronize()
    assert torch.equal(V2[:7], V) and torch.equal(V2[7:], V) and F2.numel() == 0
    Fb = torch.tensor([[0, 1, 9]], dtype=torch.int32, device="cuda")
    V2, F2 = wn.wn_flip_duplicate(V, Fb, 0.01)
    assert wn.wn_get_device_error() == wn._lib.WN_ERR_BAD_INDEX
    assert F2.cpu().tolist() == [[0, 1, 0], [7, 7, 8]]
