"""GPU parity on general graphs (CSR, Section 5) against the CPU oracle.

Distances are integers: D, the source sequences, a(t) and n_prop must be
identical (tolerance 0).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def G(torch_mod):
    from paper_2007_16076_amd import gapd
    gapd.load_library()
    return gapd


def edges_csr(n, edges):
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


def geo(n, seed):
    import synth
    return synth.geometric_graph(np.random.default_rng(seed), n)


def run_tree(G, torch, graph, mode, boundary=None):
    rp, ci, cw = graph
    g = G.Graph(rp, ci, cw, boundary=boundary)
    n = g.n
    seq = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    fil = torch.zeros((n,), dtype=torch.int64, device="cuda")
    D, st = g.all_pairs(mode, out=torch.full((n, n), -7, dtype=torch.int32, device="cuda"), sources_out=seq,
                        filled_out=fil)
    torch.cuda.synchronize()
    k = st.n_prop
    return D.cpu().numpy(), seq.cpu().numpy()[:k], fil.cpu().numpy()[:k], st


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (40, 2), (300, 3), (2000, 4)])
def test_graph_naive_matches_oracle(G, torch_mod, oracle_lib, n, seed):
    graph = geo(n, seed)
    say("graph naive", n)
    g = G.Graph(*graph)
    D, st = g.all_pairs(G.MODE_NAIVE, out=torch_mod.full((g.n, g.n), -7, dtype=torch_mod.int32, device="cuda"))
    assert np.array_equal(D.cpu().numpy(), oracle_lib.graph_naive(*graph))
    assert st.n_prop == n


def test_graph_sssp_matches_oracle(G, torch_mod, oracle_lib):
    graph = geo(5000, 5)
    src = np.array([0, 17, 4999, 2500, 17], np.int32)
    say("graph sssp")
    got = G.Graph(*graph).sssp(src).cpu().numpy()
    assert np.array_equal(got, oracle_lib.graph_rows(*graph, src))


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (60, 3), (150, 4), (700, 6)])
def test_graph_tree_methods_match_oracle(G, torch_mod, oracle_lib, n, seed, mode):
    graph = geo(n, seed)
    say("graph tree", n, mode)
    D, seq, fil, st = run_tree(G, torch_mod, graph, mode)
    ref = oracle_lib.graph_tree_method(*graph, rule=0 if mode == G.MODE_TREE_FILL_FR else 1)
    assert st.n_prop == ref.n_prop
    assert np.array_equal(seq, ref.sequence)
    assert np.array_equal(fil, ref.filled)
    assert np.array_equal(D, ref.D)
    if n > 1:
        assert st.centroid == ref.centroid and st.n_prop_setup == 2


@pytest.mark.parametrize("name", ["path", "star", "lollipop", "cycle"])
def test_graph_small_shapes(G, torch_mod, oracle_lib, name):
    graphs = {"path": edges_csr(5, [(0, 1, 1), (1, 2, 2), (2, 3, 3), (3, 4, 4)]),
              "star": edges_csr(5, [(0, 1, 1), (0, 2, 2), (0, 3, 3), (0, 4, 4)]),
              "lollipop": edges_csr(4, [(0, 1, 1), (1, 2, 1), (0, 2, 1), (2, 3, 1)]),
              "cycle": edges_csr(6, [(i, (i + 1) % 6, 1 + i) for i in range(6)])}
    graph = graphs[name]
    say("graph shape", name)
    for mode, rule in ((G.MODE_TREE_FILL_FR, 0), (G.MODE_TREE_FILL_EXTREMA, 1)):
        D, seq, fil, st = run_tree(G, torch_mod, graph, mode)
        ref = oracle_lib.graph_tree_method(*graph, rule=rule)
        assert np.array_equal(seq, ref.sequence) and np.array_equal(D, ref.D)


def test_grid_as_graph_matches_grid_path(G, torch_mod):
    """The same image through the grid kernels and through the graph kernels
    (with the border as the boundary): identical D and sequence."""
    rng = np.random.default_rng(9)
    img = rng.integers(1, 256, (23, 29)).astype(np.uint8)
    H, W = img.shape
    f = img.astype(np.int64).reshape(-1)
    edges = []
    for p in range(H * W):
        y, x = divmod(p, W)
        if x + 1 < W:
            edges.append((p, p + 1, int(f[p] + f[p + 1])))
        if y + 1 < H:
            edges.append((p, p + W, int(f[p] + f[p + W])))
    graph = edges_csr(H * W, edges)
    yy, xx = np.mgrid[0:H, 0:W]
    bnd = ((yy == 0) | (yy == H - 1) | (xx == 0) | (xx == W - 1)).reshape(-1).astype(np.uint8)
    say("grid as graph")
    Dg, seqg, filg, _ = run_tree(G, torch_mod, graph, G.MODE_TREE_FILL_FR, boundary=bnd)
    ctx = G.Context(img, conn=4)
    seq = torch_mod.full((H * W,), -1, dtype=torch_mod.int32, device="cuda")
    D, st = ctx.all_pairs(G.MODE_TREE_FILL_FR, sources_out=seq)
    assert np.array_equal(Dg, D.cpu().numpy())
    assert np.array_equal(seqg, seq.cpu().numpy()[:st.n_prop])


def two_level_graph(n, seed):
    """A hub joined to about sqrt(n) sub-hubs, each with its share of leaves,
    consecutive sub-hubs joined, and one extra edge between leaves of a
    sub-hub per 16 leaves; random weights 1..50.  Shallow trees keep each
    propagation short, so large n stays cheap."""
    rng = np.random.default_rng(seed)
    k = max(1, int(np.sqrt(n - 1)))
    edges = []
    hubs = list(range(1, k + 1))
    for h in hubs:
        edges.append((0, h, int(rng.integers(1, 51))))
    for a, b in zip(hubs[:-1], hubs[1:]):
        edges.append((a, b, int(rng.integers(1, 51))))
    leaves = np.arange(k + 1, n)
    owner = leaves % k + 1
    for v, h in zip(leaves, owner):
        edges.append((int(h), int(v), int(rng.integers(1, 51))))
    for h in hubs:
        mine = leaves[owner == h]
        for _ in range(len(mine) // 16):
            a, b = rng.choice(mine, 2, replace=False)
            edges.append((int(a), int(b), int(rng.integers(1, 51))))
    seen, uniq = set(), []
    for u, v, w in edges:
        key = (min(u, v), max(u, v))
        if key not in seen:
            seen.add(key)
            uniq.append((u, v, w))
    return edges_csr(n, uniq)


@pytest.mark.parametrize("n", [14000, 21000])
def test_graph_large_fill_paths(G, torch_mod, oracle_lib, n):
    """Graphs whose tree entries fit LDS without the counts (14000) or do not
    fit at all (21000): the filling-rate D equals the naive D everywhere, the
    naive D equals the oracle on sampled rows, and the run ends complete."""
    graph = two_level_graph(n, 7)
    say("graph large", n)
    g = G.Graph(*graph)
    Dn, _ = g.all_pairs(G.MODE_NAIVE, out=torch_mod.full((n, n), -7, dtype=torch_mod.int32, device="cuda"))
    rows = np.array([0, 1, n // 3, n // 2, n - 1], np.int32)
    assert np.array_equal(Dn[torch_mod.from_numpy(rows).long().cuda()].cpu().numpy(),
                          oracle_lib.graph_rows(*graph, rows))
    fil = torch_mod.zeros((n,), dtype=torch_mod.int64, device="cuda")
    Df, st = g.all_pairs(G.MODE_TREE_FILL_FR, out=torch_mod.full((n, n), -7, dtype=torch_mod.int32, device="cuda"), filled_out=fil)
    assert torch_mod.equal(Df, Dn)
    assert int(fil[st.n_prop - 1]) == n * (n - 1) // 2
    del Df, Dn
    torch_mod.cuda.empty_cache()


@pytest.mark.parametrize("case", ["asymmetric", "disconnected", "self_loop", "too_big"])
def test_graph_invalid_inputs(G, torch_mod, case):
    rp, ci, cw = edges_csr(4, [(0, 1, 2), (1, 2, 3), (2, 3, 4)])
    if case == "asymmetric":
        cw = cw.copy()
        cw[0] += 1
    elif case == "disconnected":
        rp, ci, cw = edges_csr(4, [(0, 1, 2), (2, 3, 4)])
    elif case == "self_loop":
        ci = ci.copy()
        ci[0] = 0
    else:
        rp, ci, cw = edges_csr(32769, [(i, i + 1, 1) for i in range(32768)])
    with pytest.raises(G.GapdError) as e:
        G.Graph(rp, ci, cw)
    assert e.value.status == G.EINVAL


def test_graph_rejects_spiral_mode(G, torch_mod):
    import ctypes
    g = G.Graph(*geo(30, 1))
    lib = G.load_library()
    n = ctypes.c_size_t()
    assert lib.gapd_graph_workspace_size(g._h, G.MODE_TREE_FILL_SPIRAL, ctypes.byref(n)) == G.EINVAL
    out = torch_mod.empty((30, 30), dtype=torch_mod.int32, device="cuda")
    st = G.Stats()
    assert lib.gapd_graph_all_pairs(g._h, G.MODE_TREE_FILL_SPIRAL, out.data_ptr(), ctypes.byref(st)) == G.EINVAL
