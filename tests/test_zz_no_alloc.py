"""The allocation-free forward (wn_voxelize_strips_noalloc) against wn_voxelize_strips,
both called through the C ABI: the same inputs must give bit-identical W and occupancy,
on two calls in a row (the second smaller, so that it runs over what the first left in
the shared device array), a request beyond the array's size is refused before anything
is enqueued, and the array's error record is read with wn_get_device_error(NULL)."""
import ctypes

import numpy as np
import pytest

import wn_inputs as wi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_11272_amd import _lib as L
    return L.load()


def _grid(g):
    from paper_2407_11272_amd import _lib as L
    c = L.WnGrid()
    for d in range(3):
        c.lo[d], c.hi[d], c.n[d] = float(g.lo[d]), float(g.hi[d]), int(g.n[d])
    return c


def _mesh(w):
    import torch
    import paper_2407_11272_amd as wn
    V = torch.as_tensor(np.asarray(w.V, np.float32)).cuda().contiguous()
    F = torch.as_tensor(np.asarray(w.F, np.int32)).cuda().contiguous()
    R = torch.as_tensor(wn.wn_build_strips(w.F, len(w.V))).cuda().contiguous()
    return V, F, R


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(lib, w, occ_mode):
    """W and occupancy from the workspace entry point and from the allocation-free one."""
    import torch
    from paper_2407_11272_amd import _lib as L
    V, F, R = _mesh(w)
    P = w.grid.size
    g = _grid(w.grid)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ws_bytes = lib.wn_workspace_size(L.WN_OP_VOXELIZE, len(w.V), len(w.F), P)
    ws = torch.zeros(ws_bytes + 256, dtype=torch.uint8, device="cuda")
    wsp = ctypes.c_void_p(ws.data_ptr() + (-ws.data_ptr()) % 256)
    odt = torch.uint8 if occ_mode == L.WN_OCC_THRESHOLD else torch.float32
    W1 = torch.full((P,), np.nan, dtype=torch.float32, device="cuda")
    O1 = torch.zeros(P, dtype=odt, device="cuda")
    W2 = torch.full((P,), np.nan, dtype=torch.float32, device="cuda")
    O2 = torch.zeros(P, dtype=odt, device="cuda")
    print(f"[no-alloc] {w.name}: faces={len(w.F)} records={R.shape[0]} points={P}", flush=True)
    st = lib.wn_voxelize_strips(_p(V), len(w.V), _p(F), len(w.F), _p(R), R.shape[0], ctypes.byref(g), None, 0,
                                _p(W1), occ_mode, 0.5, 50.0, _p(O1), wsp, ws_bytes - 0, s)
    assert st == L.WN_OK
    st = lib.wn_voxelize_strips_noalloc(_p(V), len(w.V), _p(F), len(w.F), _p(R), R.shape[0], ctypes.byref(g), None,
                                        0, _p(W2), occ_mode, 0.5, 50.0, _p(O2), s)
    assert st == L.WN_OK
    assert lib.wn_get_device_error(None, s) == L.WN_OK
    torch.cuda.synchronize()
    return W1.cpu().numpy(), O1.cpu().numpy(), W2.cpu().numpy(), O2.cpu().numpy()


def test_noalloc_matches_workspace_entry_point_twice(lib):
    from paper_2407_11272_amd import _lib as L
    # first call: 19 000 faces at 128^3 (vertex records and split partial sums in the array)
    W1, O1, W2, O2 = _both(lib, wi.config2_ellipsoid_union(), L.WN_OCC_THRESHOLD)
    assert np.all(np.isfinite(W2))
    assert np.array_equal(W1.view(np.uint32), W2.view(np.uint32))
    assert np.array_equal(O1, O2)
    # second call, smaller, over what the first left in the array: 1280 faces at 32^3,
    # sigmoid occupancy
    W1, O1, W2, O2 = _both(lib, wi.config1_icosphere(), L.WN_OCC_SIGMOID)
    assert np.all(np.isfinite(W2))
    assert np.array_equal(W1.view(np.uint32), W2.view(np.uint32))
    assert np.array_equal(O1.view(np.uint32), O2.view(np.uint32))


def test_noalloc_refuses_requests_beyond_the_array(lib):
    import torch
    from paper_2407_11272_amd import _lib as L
    w = wi.config1_icosphere()
    V, F, R = _mesh(w)
    W = torch.zeros(w.grid.size, dtype=torch.float32, device="cuda")
    g = _grid(w.grid)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # a claimed stream of 4 million records needs 128 MB of vertex records: refused on the
    # host, before anything is enqueued (the buffers are never read)
    big_r, big_f = 4_000_000, 2_000_000
    assert 32 * big_r > L.WN_NOALLOC_SCRATCH_BYTES
    st = lib.wn_voxelize_strips_noalloc(_p(V), len(w.V), _p(F), big_f, _p(R), big_r, ctypes.byref(g), None, 0,
                                        _p(W), L.WN_OCC_NONE, 0.5, 50.0, None, s)
    assert st == L.WN_ERR_WORKSPACE
    # no strip stream is an argument error, as for wn_voxelize_strips
    st = lib.wn_voxelize_strips_noalloc(_p(V), len(w.V), _p(F), len(w.F), None, 0, ctypes.byref(g), None, 0, _p(W),
                                        L.WN_OCC_NONE, 0.5, 50.0, None, s)
    assert st == L.WN_ERR_INVALID_ARG
    torch.cuda.synchronize()


def test_noalloc_error_record(lib):
    import torch
    from paper_2407_11272_amd import _lib as L
    w = wi.config1_icosphere(res=8)
    V, F, R = _mesh(w)
    Rbad = R.clone()
    Rbad[5, 0] = len(w.V) + 7   # an out-of-range vertex id: replaced by 0 on the device and recorded
    W = torch.zeros(w.grid.size, dtype=torch.float32, device="cuda")
    g = _grid(w.grid)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.wn_voxelize_strips_noalloc(_p(V), len(w.V), _p(F), len(w.F), _p(Rbad), Rbad.shape[0], ctypes.byref(g),
                                        None, 0, _p(W), L.WN_OCC_NONE, 0.5, 50.0, None, s)
    assert st == L.WN_OK
    assert lib.wn_get_device_error(None, s) == L.WN_ERR_BAD_INDEX
    assert lib.wn_get_device_error(None, s) == L.WN_OK   # cleared by the read
    st = lib.wn_voxelize_strips_noalloc(_p(V), len(w.V), _p(F), len(w.F), _p(R), R.shape[0], ctypes.byref(g), None,
                                        0, _p(W), L.WN_OCC_NONE, 0.5, 50.0, None, s)
    assert st == L.WN_OK
    assert lib.wn_get_device_error(None, s) == L.WN_OK
    torch.cuda.synchronize()
