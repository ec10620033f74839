"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/wn.h declares, and answers the host-only queries (no GPU calls)."""
import os
import re

import pytest

import paper_2407_11272_amd as wn
from paper_2407_11272_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "wn.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"WN_API\s+[\w\s\*]*?\b(wn_\w+)\s*\(", text)))


def test_header_declares_the_expected_entry_points():
    assert declared_symbols() == sorted(L.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    out = os.popen(f"nm -D --defined-only {L.LIB_PATH}").read()
    exported = set(re.findall(r" T (wn_\w+)", out))
    assert set(declared_symbols()) <= exported
    # nothing else leaks out of the library under the wn_ prefix
    assert exported == set(declared_symbols())


def test_status_strings_and_version():
    for s in (L.WN_OK, L.WN_ERR_INVALID_ARG, L.WN_ERR_HIP, L.WN_ERR_WORKSPACE, L.WN_ERR_BAD_INDEX,
              L.WN_ERR_UNSUPPORTED):
        assert L.status_string(s) and L.status_string(s) != "unknown status"
    assert L.status_string(12345) == "unknown status"
    assert "gfx950" in wn.wn_version()


def test_workspace_sizes_are_host_only_and_monotone():
    s1 = wn.wn_workspace_size(L.WN_OP_VOXELIZE, 642, 1280, 32 ** 3)
    s2 = wn.wn_workspace_size(L.WN_OP_VOXELIZE, 10016, 19000, 128 ** 3)
    assert s1 >= 256 + 48 * 1280 and s2 >= 256 + 48 * 19000
    assert wn.wn_workspace_size(L.WN_OP_VOXELIZE, 0, 0, 0) == 256
    b = wn.wn_workspace_size(L.WN_OP_BACKWARD, 2562, 5120, 64 ** 3)
    assert b >= 256 + 48 * 5120 + 9 * 4 * 5120
    assert wn.wn_workspace_size(L.WN_OP_LOSS, 0, 0, 1000) >= 256 + 4
    assert wn.wn_workspace_size(99, 1, 1, 1) == 0
    assert wn.wn_workspace_size(L.WN_OP_VOXELIZE, -1, 1, 1) == 0


def test_no_cpu_fallback_on_host_tensors():
    import torch
    with pytest.raises(ValueError):
        wn.wn_voxelize(torch.zeros((3, 3)), torch.zeros((1, 3), dtype=torch.int32), grid=wn.Grid.cube(2))


def test_backward_splits_are_host_only():
    lib = L.load()
    # a pure function of the sizes: at most one split per 256-point tile, at most 4096,
    # and at most 256 MiB of running sums (72 bytes per face per split)
    assert lib.wn_backward_splits(5120, 64 ** 3) == lib.wn_backward_splits(5120, 64 ** 3)
    assert 1 <= lib.wn_backward_splits(5120, 64 ** 3) <= 1024
    assert lib.wn_backward_splits(10, 300) == 2
    assert lib.wn_backward_splits(10, 0) == 1
    assert lib.wn_backward_splits(100000, 256 ** 3) * 72 * 100000 <= 256 << 20
    assert lib.wn_backward_splits(-1, 10) == -1 and lib.wn_backward_splits(1, -5) == -1
    # the adjoint workspace grows with the split count's running sums
    b = wn.wn_workspace_size(L.WN_OP_BACKWARD, 2562, 5120, 64 ** 3)
    assert b >= 256 + 48 * 5120 + 72 * 5120 * lib.wn_backward_splits(5120, 64 ** 3)


def test_backward_workspace_doubles_its_running_sums_with_many_tiles_per_split():
    """With at least 12 point tiles per split the adjoint workspace holds twice the running
    sums (room for three times the merged face-pair splits); below that it does not."""
    lib = L.load()
    for nV, nF, P in ((2562, 5120, 64 ** 3), (2562, 5120, 96 ** 3), (2562, 5120, 128 ** 3),
                      (642, 1280, 128 ** 3), (50000, 100000, 256 ** 3)):
        S = lib.wn_backward_splits(nF, P)
        wide = P // 256 >= 12 * S
        # the running sums, then records, corner sort buffers and the rest (under 300 B
        # per face and 32 B per vertex, plus alignment and the sort's scratch)
        b = wn.wn_workspace_size(L.WN_OP_BACKWARD, nV, nF, P)
        base = 72 * nF * S
        assert b >= base * (2 if wide else 1)
        assert b < base * (2 if wide else 1) + 256 * 16 + 300 * nF + 32 * nV + (1 << 20)
