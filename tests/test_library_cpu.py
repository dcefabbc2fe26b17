"""Host-only checks of libgapd.so: it loads, exports every entry point that
include/gapd.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2007_16076_amd import gapd
    return gapd.load_library()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gapd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gapd_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_2007_16076_amd import gapd
    assert sorted(gapd.EXPORTED) == names


def test_strerror(lib):
    assert lib.gapd_strerror(0) == b"ok"
    assert lib.gapd_strerror(-5) == b"propagation did not converge"


@pytest.mark.parametrize("H,W,C,conn,wmode", [(0, 4, 1, 4, 0), (4, 0, 1, 4, 0), (513, 4, 1, 4, 0),
                                              (4, 4, 1, 6, 0), (4, 4, 3, 4, 0), (4, 4, 1, 4, 7),
                                              (4, 4, 300, 4, 1)])
def test_create_rejects_bad_arguments(lib, H, W, C, conn, wmode):
    img = np.ones(max(H, 1) * max(W, 1) * C, dtype=np.uint8)
    h = ctypes.c_void_p()
    st = lib.gapd_create(img.ctypes.data, H, W, C, conn, wmode, ctypes.byref(h))
    assert st == -1 and not h.value
    assert lib.gapd_last_error(None)


def test_create_rejects_zero_weight_edges(lib):
    img = np.ones((3, 3), dtype=np.uint8)
    img[1, 1] = img[1, 2] = 0
    h = ctypes.c_void_p()
    assert lib.gapd_create(img.ctypes.data, 3, 3, 1, 4, 0, ctypes.byref(h)) == -1
    assert b"weighs 0" in lib.gapd_last_error(None)
    img = np.ones((3, 3), dtype=np.uint8)
    img[0, 0] = img[1, 1] = 0       # diagonal neighbours: only an edge under 8-connectivity
    # 4-connectivity: no zero edge, accepted by validation (then needs a device)
    assert lib.gapd_create(img.ctypes.data, 3, 3, 1, 8, 0, ctypes.byref(h)) == -1


def test_batched_workspace_size(lib):
    from paper_2007_16076_amd import gapd
    n_naive = gapd.batched_workspace_size([(10, 12), (5, 7)], mode=gapd.MODE_NAIVE)
    n_fr = gapd.batched_workspace_size([(10, 12), (5, 7)], mode=gapd.MODE_TREE_FILL_FR)
    assert 0 < n_naive < n_fr
    with pytest.raises(gapd.GapdError):
        gapd.batched_workspace_size([(0, 12)])


def test_null_arguments(lib):
    assert lib.gapd_create(None, 4, 4, 1, 4, 0, None) == -1
    assert lib.gapd_sssp(None, None, 1, None) == -1
    assert lib.gapd_all_pairs(None, 0, None, None) == -1
    assert lib.gapd_serve_submit(None, None, None) == -1
    lib.gapd_destroy(None)
    lib.gapd_server_destroy(None)
