"""GPU parity of the batched persistent launch (many meshes, one graph-captured launch).

Each mesh's W is held to the FP64 oracle (|dW| <= 1e-4 off the guard band), to the
plain one-mesh launch (|dW| <= 2e-6; bit-identical when both sum the faces in the same
tiles), and to itself alone vs in the mix (bit-identical: its chunking depends only on
its own size).  Graph replays with changing batches are compared with eager launches.
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


def _job(V, F, grid, occupancy="threshold"):
    import torch
    import paper_2407_11272_amd as wn
    Vt, Ft = wn.as_mesh(torch.as_tensor(np.asarray(V, np.float32)), torch.as_tensor(F))
    return wn.MeshJob(Vt, Ft, wn.Grid.of(grid), occupancy)


def _small_batch(seed=0):
    """Uneven meshes: single-chunk, multi-chunk (> 4096 faces), tiny, empty, odd grids."""
    rng = np.random.default_rng(seed)
    out = []
    V, F, _ = wi.ellipsoid_union(rng, 3, 1800)  # 5400 faces -> 2 chunks
    out.append((V, F, wi.Grid.cube(24)))
    V, F = wi.icosphere(2)
    out.append((0.3 * V, F, wi.Grid((-0.4, -0.5, -0.3), (0.45, 0.5, 0.3), (9, 13, 7))))
    V, F, _ = wi.ellipsoid_union(rng, 2, 4500)  # ~9000 faces -> 3 chunks
    F = wi.delete_faces(F, 300, rng)
    out.append((V, F, wi.Grid.cube(16)))
    out.append((np.zeros((3, 3)), np.zeros((0, 3), np.int64), wi.Grid.cube(5)))  # no faces -> W = 0
    V = rng.uniform(-0.5, 0.5, (30, 3))
    out.append((V, rng.integers(0, 30, (10, 3)), wi.Grid.cube(11)))
    return out


def _run(jobs, graph=True):
    import torch
    import paper_2407_11272_amd as wn
    wn.wn_voxelize_batched(jobs, graph=graph)
    torch.cuda.synchronize()
    return [j.W.cpu().numpy().reshape(-1).copy() for j in jobs]


def test_small_batch_vs_oracle_and_plain(dev, orc):
    import torch
    import paper_2407_11272_amd as wn
    meshes = _small_batch()
    jobs = [_job(V, F, g) for V, F, g in meshes]
    Ws = _run(jobs)
    for (V, F, g), Wb, j in zip(meshes, Ws, jobs):
        Q = orc.grid_points(g)
        if len(F) == 0:
            assert np.all(Wb == 0)
            continue
        V64 = np.asarray(V, np.float32).astype(np.float64)
        Wr = orc.winding(V64, F, Q)
        guard = orc.guard_mask(V64, F, Q)
        err = np.abs(Wb - Wr)[~guard]
        print(f"[batched faces={len(F)} grid={g.n}] guard={guard.sum()} max|dW|={err.max():.2e}", flush=True)
        assert err.max() <= 1e-4
        occ = j.occ.cpu().numpy().reshape(-1)
        m = ~guard & (np.abs(Wr - 0.5) > 1e-3)
        np.testing.assert_array_equal(occ[m], orc.occupancy_threshold(Wr)[m])
        Wp = wn.wn_voxelize(j.V, j.F, grid=j.grid).cpu().numpy().reshape(-1)
        assert np.abs(Wp - Wb).max() <= 2e-6


def test_single_chunk_mesh_matches_plain_bitwise(dev):
    """A mesh of at most one chunk (<= 4096 faces) on a grid large enough that the plain
    launch does not split the faces (at least 131072 point waves: 256^3): both sum the
    same tiles in the same order."""
    import paper_2407_11272_amd as wn
    from paper_2407_11272_amd import _lib as L
    c = wi.config1_icosphere()
    j = _job(c.V, c.F, wi.Grid.cube(256))
    # no split: the plain workspace holds no per-split partials
    assert wn.wn_workspace_size(L.WN_OP_VOXELIZE, len(c.V), len(c.F), 256 ** 3) < 256 ** 3 * 4
    Wb = _run([j])[0]
    Wp = wn.wn_voxelize(j.V, j.F, grid=j.grid).cpu().numpy().reshape(-1)
    np.testing.assert_array_equal(Wp, Wb)


def test_alone_equals_in_mix_bitwise(dev):
    meshes = _small_batch(1)
    mix = _run([_job(V, F, g) for V, F, g in meshes])
    for i, (V, F, g) in enumerate(meshes):
        alone = _run([_job(V, F, g)])[0]
        np.testing.assert_array_equal(alone, mix[i])
    # a different mix (reversed order, extra meshes) gives the same bits again
    extra = _small_batch(7)[:2]
    mix2 = _run([_job(V, F, g) for V, F, g in (extra + meshes[::-1])])
    for i in range(len(meshes)):
        np.testing.assert_array_equal(mix2[len(extra) + len(meshes) - 1 - i], mix[i])


def test_graph_replays_match_eager(dev):
    """The captured graph is replayed for changing batches on one workspace, with eager
    work in between; every replay must match an eager (no-graph) launch bit for bit."""
    import torch
    base = _small_batch(2)
    batches = [base, base[::-1], base[1:3], base]
    for b in batches:
        g = _run([_job(V, F, gr) for V, F, gr in b], graph=True)
        torch.ones(1000, device="cuda").sum().item()  # unrelated eager work
        e = _run([_job(V, F, gr) for V, F, gr in b], graph=False)
        for x, y in zip(g, e):
            np.testing.assert_array_equal(x, y)


def test_autotune_does_not_change_results(dev, tmp_path, monkeypatch):
    import paper_2407_11272_amd as wn
    meshes = _small_batch(3)
    ref = _run([_job(V, F, g) for V, F, g in meshes])
    rep = wn.wn_autotune("batched", [_job(V, F, g) for V, F, g in meshes])
    print("autotune report", rep, flush=True)
    # points per lane x record tiles per barrier, then the winner with fewer workgroups
    assert rep["chosen"]["ppl"] in (1, 2, 4) and rep["chosen"]["depth"] in (1, 2, 4)
    assert len(rep["candidates"]) == 10
    assert rep["identical"] and len({c["checksum"] for c in rep["candidates"]}) == 1
    again = _run([_job(V, F, g) for V, F, g in meshes])
    for x, y in zip(ref, again):
        np.testing.assert_array_equal(x, y)
    rep = wn.wn_autotune("voxelize", [_job(*meshes[0])])
    assert len(rep["candidates"]) == 9
    assert rep["identical"] and len({c["checksum"] for c in rep["candidates"]}) == 1


def test_full_batch_64_meshes(dev, orc):
    """64 meshes of 500-50k faces at 32^3/64^3/128^3 in one launch: every mesh against the
    plain launch, and every mesh against the oracle on 1024 seeded voxels (65 536 voxels,
    about 6e8 point-face pairs), W within 1e-4 outside the guard band."""
    import torch
    import paper_2407_11272_amd as wn
    ws = wi.config4_batch()
    jobs = [_job(w.V, w.F, w.grid) for w in ws]
    Wb = _run(jobs)
    rng = np.random.default_rng(5)
    worst = 0.0
    for i, (w, j) in enumerate(zip(ws, jobs)):
        Wp = wn.wn_voxelize(j.V, j.F, grid=j.grid).cpu().numpy().reshape(-1)
        worst = max(worst, float(np.abs(Wp - Wb[i]).max()))
    print(f"[C4] max |batched - plain| = {worst:.2e}", flush=True)
    assert worst <= 2e-6
    worst, guarded = 0.0, 0
    for i, w in enumerate(ws):
        Q = orc.grid_points(w.grid)
        idx = rng.choice(len(Q), 1024, replace=False)
        V64 = np.asarray(w.V, np.float32).astype(np.float64)
        Wr = orc.winding(V64, w.F, Q[idx])
        guard = orc.guard_mask(V64, w.F, Q[idx])
        guarded += int(guard.sum())
        worst = max(worst, float(np.abs(Wb[i][idx] - Wr)[~guard].max()))
    print(f"[C4 vs oracle] 64 meshes x 1024 voxels: max |dW| = {worst:.2e} off the guard band "
          f"({guarded} guarded)", flush=True)
    assert worst <= 1e-4 and guarded <= 1e-3 * 64 * 1024
    torch.cuda.synchronize()


def test_batched_argument_errors(dev):
    import torch
    import paper_2407_11272_amd as wn
    from paper_2407_11272_amd import _lib as L
    lib = L.load()
    j = _job(*_small_batch()[1])
    arr = (L.WnMeshDesc * 1)()
    arr[0] = j.prepare().desc()
    need = lib.wn_workspace_size_batched(arr, 1)
    assert need > 256
    buf = torch.zeros(need + 512, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr() + ((-buf.data_ptr()) % 256)
    import ctypes
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.wn_voxelize_batched(arr, 1, 0, ctypes.c_void_p(base), 64, s) == L.WN_ERR_WORKSPACE
    assert lib.wn_voxelize_batched(arr, 1, 8, ctypes.c_void_p(base), need, s) == L.WN_ERR_INVALID_ARG
    bad = (L.WnMeshDesc * 1)()
    bad[0] = j.desc()
    bad[0].W = None
    assert lib.wn_voxelize_batched(bad, 1, 0, ctypes.c_void_p(base), need, s) == L.WN_ERR_INVALID_ARG
    assert lib.wn_workspace_size_batched(bad, 1) == 0
    bad[0] = j.desc()
    bad[0].grid.n[1] = 0
    assert lib.wn_voxelize_batched(bad, 1, 0, ctypes.c_void_p(base), need, s) == L.WN_ERR_INVALID_ARG
    assert lib.wn_voxelize_batched(arr, 1, 0, ctypes.c_void_p(base), need, s) == L.WN_OK
    torch.cuda.synchronize()


def test_batched_strips_alone_mix_and_plain(dev):
    """Strip streams in a batch: bit-identical alone and in the mix; single-chunk meshes
    bit-identical to the plain strip launch; within 2e-6 of three records per face."""
    import torch
    import paper_2407_11272_amd as wn
    meshes = [m for m in _small_batch(4) if len(m[1])]

    def jobs():
        out = []
        for V, F, g in meshes:
            j = _job(V, F, g)
            j.strips = torch.as_tensor(wn.wn_build_strips(F, len(V))).cuda()
            out.append(j)
        return out

    mix = _run(jobs())
    for i, j in enumerate(jobs()):
        alone = _run([j])[0]
        np.testing.assert_array_equal(alone, mix[i])
        plain_trivial = wn.wn_voxelize(j.V, j.F, grid=j.grid).cpu().numpy().reshape(-1)
        assert np.abs(plain_trivial - mix[i]).max() <= 2e-6
    V, F = wi.icosphere(3)
    j = _job(0.4 * V, F, wi.Grid.cube(256))   # enough point waves for an unsplit plain launch
    j.strips = torch.as_tensor(wn.wn_build_strips(F, len(V))).cuda()
    b = _run([j])[0]
    p = wn.wn_voxelize_strips(j.V, j.F, j.strips, grid=j.grid).cpu().numpy().reshape(-1)
    np.testing.assert_array_equal(b, p)


def test_back_to_back_batches_without_host_waits_and_release(dev):
    """Several different batches enqueued on one workspace with no synchronisation in
    between (each call stages its table in its own pinned buffer of the workspace's ring
    instead of waiting for the previous copy), each into its own outputs: every mesh
    equals its eager result.  wn_release_workspace then frees the graphs and buffers, and
    the next call rebuilds them."""
    import ctypes
    import torch
    import paper_2407_11272_amd as wn
    from paper_2407_11272_amd import _lib as L
    base = _small_batch(3)
    batches = [base, base[::-1], base[1:4], base[:2], base]
    ref = [_run([_job(V, F, gr) for V, F, gr in b], graph=False) for b in batches]
    lib = L.load()
    jobs_all = [[_job(V, F, gr).prepare() for V, F, gr in b] for b in batches]
    need = max(int(lib.wn_workspace_size_batched(wn.api._descs(js), len(js))) for js in jobs_all)
    buf = torch.zeros(need + 256, dtype=torch.uint8, device="cuda")
    ws = ctypes.c_void_p(buf.data_ptr() + (-buf.data_ptr()) % 256)
    for rnd in range(2):
        for js in jobs_all:   # no synchronisation between the calls
            wn.wn_voxelize_batched(js, graph=True, workspace=(ws, need))
        torch.cuda.synchronize()
        for js, r in zip(jobs_all, ref):
            for j, x in zip(js, r):
                np.testing.assert_array_equal(j.W.cpu().numpy().reshape(-1), x)
        for js in jobs_all:
            for j in js:
                j.W.fill_(float("nan"))
        assert lib.wn_release_workspace(ws) == L.WN_OK
    assert lib.wn_release_workspace(ws) == L.WN_OK    # nothing held: a no-op
    assert lib.wn_release_workspace(None) == L.WN_ERR_INVALID_ARG
