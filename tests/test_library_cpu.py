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


def _csr(n, edges):
    adj = [[] for _ in range(n)]
    for u, v, w in edges:
        adj[u].append((v, w))
        adj[v].append((u, w))
    rp = np.zeros(n + 1, np.int64)
    ci, cw = [], []
    for u in range(n):
        for v, w in sorted(adj[u]):
            ci.append(v)
            cw.append(w)
        rp[u + 1] = len(ci)
    return rp, np.array(ci, np.int32), np.array(cw, np.int32)


@pytest.mark.parametrize("case", ["asymmetric", "missing_reverse", "self_loop", "zero_weight", "duplicate",
                                  "disconnected", "out_of_range", "too_many", "empty", "no_boundary", "range",
                                  "heavy_edge"])
def test_graph_create_rejects_bad_graphs(lib, case):
    """gapd_graph_create checks the CSR graph on the host before any device
    call: these all fail with GAPD_EINVAL (or GAPD_ERANGE) and a message."""
    rp, ci, cw = _csr(4, [(0, 1, 2), (1, 2, 3), (2, 3, 4)])
    ci, cw, bnd, want = ci.copy(), cw.copy(), None, -1
    if case == "asymmetric":
        cw[0] += 1
    elif case == "missing_reverse":
        rp, ci, cw = np.array([0, 1, 1, 1, 1], np.int64), np.array([1], np.int32), np.array([1], np.int32)
    elif case == "self_loop":
        ci[0] = 0
    elif case == "zero_weight":
        rp, ci, cw = _csr(4, [(0, 1, 0), (1, 2, 3), (2, 3, 4)])
    elif case == "duplicate":
        rp, ci, cw = _csr(4, [(0, 1, 2), (0, 1, 2), (1, 2, 3), (2, 3, 4)])
    elif case == "disconnected":
        rp, ci, cw = _csr(4, [(0, 1, 2), (2, 3, 4)])
    elif case == "out_of_range":
        ci[0] = 7
    elif case == "too_many":
        rp, ci, cw = _csr(32769, [(i, i + 1, 1) for i in range(32768)])
    elif case == "empty":
        rp = np.zeros(1, np.int64)
    elif case == "no_boundary":
        bnd = np.zeros(4, np.uint8)
    elif case == "heavy_edge":
        # triangle 0-1 (1), 1-2 (1), 0-2 (2^31 - 1): the breadth-first tree from 0
        # takes 0-1 and 0-2, so only a per-edge bound catches the heavy edge,
        # whose weight added to a distance would wrap in int32
        rp, ci, cw = _csr(3, [(0, 1, 1), (1, 2, 1), (0, 2, 2**31 - 1)])
        want = -4
    else:
        rp, ci, cw = _csr(3, [(0, 1, 1 << 26), (1, 2, 1 << 26)])
        want = -4
    n = rp.size - 1
    h = ctypes.c_void_p()
    st = lib.gapd_graph_create(n, rp.ctypes.data, ci.ctypes.data if ci.size else None,
                               cw.ctypes.data if cw.size else None,
                               None if bnd is None else bnd.ctypes.data, ctypes.byref(h))
    assert st == want
    assert not h.value
    assert lib.gapd_graph_last_error(None)
