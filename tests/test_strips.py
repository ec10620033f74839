"""CPU tests of the host triangle-strip builder (wn_build_strips): every face exactly
once, each face record's vertices are the face's vertices, at most 3 records per face,
deterministic, and long strips on regular meshes."""
import numpy as np
import pytest

import paper_2407_11272_amd as wn
import wn_inputs as wi
from paper_2407_11272_amd import _lib as L


def _check_stream(F, R):
    F = np.asarray(F)
    faces = R[:, 1]
    assert sorted(faces[faces >= 0].tolist()) == list(range(len(F)))
    for i in np.nonzero(faces >= 0)[0]:
        assert i >= 2
        assert sorted(R[i - 2:i + 1, 0].tolist()) == sorted(F[faces[i]].tolist())
    assert len(R) <= 3 * len(F)
    # every strip opens with two vertex-only records
    assert len(R) == 0 or (R[0, 1] == -1 and R[1, 1] == -1)


@pytest.mark.parametrize("mesh", ["ico3", "ico4", "c2", "open", "soup", "degenerate", "dense", "fan"])
def test_strip_stream_is_valid(mesh):
    rng = np.random.default_rng(3)
    if mesh == "ico3":
        V, F = wi.icosphere(3)
    elif mesh == "ico4":
        V, F = wi.icosphere(4)
    elif mesh == "c2":
        c = wi.config2_ellipsoid_union()
        V, F = c.V, c.F
    elif mesh == "open":
        c = wi.config3_differentiable(open_variant=True)
        V, F = c.V, c.F
    elif mesh == "soup":
        V = rng.normal(size=(90, 3))
        F = rng.permutation(90).reshape(30, 3)
    elif mesh == "dense":   # 300 random faces on 12 vertices: repeated, degenerate, non-manifold
        V = rng.normal(size=(12, 3))
        F = rng.integers(0, 12, size=(300, 3))
    elif mesh == "fan":     # 50 faces around one edge
        V = rng.normal(size=(52, 3))
        F = np.array([[0, 1, 2 + k] for k in range(50)])
    else:
        V = rng.normal(size=(10, 3))
        F = np.array([[0, 1, 2], [1, 1, 3], [2, 3, 3], [4, 5, 6], [5, 4, 7], [0, 0, 0]])
    R = wn.wn_build_strips(F, len(V))
    _check_stream(F, R)
    R2 = wn.wn_build_strips(F, len(V))
    np.testing.assert_array_equal(R, R2)


def test_strips_are_long_on_regular_meshes():
    V, F = wi.icosphere(4)
    assert len(wn.wn_build_strips(F, len(V))) / len(F) < 1.1
    c = wi.config2_ellipsoid_union()
    assert len(wn.wn_build_strips(c.F, len(c.V))) / len(c.F) < 1.25


def test_strip_builder_errors():
    import ctypes
    lib = L.load()
    n = ctypes.c_int64(-1)
    F = np.array([[0, 1, 5]], dtype=np.int32)
    assert lib.wn_build_strips(F.ctypes.data, 1, 3, None, 0, ctypes.byref(n)) == L.WN_ERR_INVALID_ARG
    F = np.array([[0, 1, 2]], dtype=np.int32)
    assert lib.wn_build_strips(F.ctypes.data, 1, 3, None, 0, ctypes.byref(n)) == L.WN_OK and n.value == 3
    out = np.zeros((2, 2), dtype=np.int32)
    assert lib.wn_build_strips(F.ctypes.data, 1, 3, out.ctypes.data, 2, ctypes.byref(n)) == L.WN_ERR_WORKSPACE
    assert lib.wn_build_strips(None, 0, 0, None, 0, ctypes.byref(n)) == L.WN_OK and n.value == 0
    assert lib.wn_build_strips(F.ctypes.data, 1, 3, None, 0, None) == L.WN_ERR_INVALID_ARG


@pytest.mark.parametrize("mesh", ["ico4", "c2", "open", "soup", "degenerate", "dense", "fan"])
def test_face_pairs_are_valid(mesh):
    """wn_build_face_pairs: every face exactly once; a pair's faces have three distinct
    vertex ids each and share exactly two; pairs come before the unpaired faces;
    deterministic; and few faces stay unpaired on manifold meshes."""
    rng = np.random.default_rng(4)
    if mesh == "ico4":
        V, F = wi.icosphere(4)
    elif mesh == "c2":
        c = wi.config2_ellipsoid_union()
        V, F = c.V, c.F
    elif mesh == "open":
        c = wi.config3_differentiable(open_variant=True)
        V, F = c.V, c.F
    elif mesh == "soup":
        V = rng.normal(size=(90, 3))
        F = rng.permutation(90).reshape(30, 3)
    elif mesh == "dense":   # 300 random faces on 12 vertices: repeated, degenerate, non-manifold
        V = rng.normal(size=(12, 3))
        F = rng.integers(0, 12, size=(300, 3))
    elif mesh == "fan":     # 50 faces around one edge: at most 25 pairs
        V = rng.normal(size=(52, 3))
        F = np.array([[0, 1, 2 + k] for k in range(50)])
    else:
        V = rng.normal(size=(10, 3))
        F = np.array([[0, 1, 2], [1, 1, 3], [2, 3, 3], [4, 5, 6], [5, 4, 7], [0, 0, 0], [1, 2, 3], [2, 1, 8]])
    F = np.asarray(F)
    P = wn.wn_build_face_pairs(F, len(V))
    assert P.dtype == np.int32 and P.shape[1] == 2
    ids = np.concatenate([P[:, 0], P[P[:, 1] >= 0, 1]])
    assert sorted(ids.tolist()) == list(range(len(F)))
    single = P[:, 1] < 0
    if single.any():
        assert np.all(single[np.argmax(single):])   # the unpaired faces come last
    for f, g in P[~single]:
        a, b = F[f].tolist(), F[g].tolist()
        assert len(set(a)) == 3 and len(set(b)) == 3 and len(set(a) & set(b)) == 2
    np.testing.assert_array_equal(P, wn.wn_build_face_pairs(F, len(V)))
    if mesh == "ico4":
        assert single.sum() <= 0.02 * len(F)
    if mesh == "soup":
        assert single.all()
    if mesh == "c2":
        assert single.sum() <= 0.06 * len(F)


def test_face_pair_builder_errors():
    lib = L.load()
    import ctypes
    F = np.array([[0, 1, 2], [0, 2, 5]], np.int32)
    n = ctypes.c_int64(0)
    assert lib.wn_build_face_pairs(F.ctypes.data, 2, 4, None, 0, ctypes.byref(n)) == L.WN_ERR_INVALID_ARG
    assert lib.wn_build_face_pairs(F.ctypes.data, 2, 6, None, 0, ctypes.byref(n)) == L.WN_OK and n.value == 1
    out = np.zeros((1, 2), np.int32)
    assert lib.wn_build_face_pairs(F.ctypes.data, 2, 6, out.ctypes.data, 0, ctypes.byref(n)) == L.WN_ERR_WORKSPACE
    assert lib.wn_build_face_pairs(F.ctypes.data, 2, 6, out.ctypes.data, 1, ctypes.byref(n)) == L.WN_OK
    assert sorted(out[0].tolist()) == [0, 1]
