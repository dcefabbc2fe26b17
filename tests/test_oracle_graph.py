"""Pins of the oracle on general graphs (CSR), the generalisation of Section 5.

* A pixel grid written as a CSR graph must give exactly what the grid oracle
  gives (itself pinned in ``test_oracle.py``): rows, parents, centroid, ranks,
  and the sequences of the filling-rate and extrema methods.  With the degree
  rule, a 4-neighbour grid's boundary vertices are its border pixels.
* Distances equal scipy's Dijkstra (an independent library routine).
* Hand-derived runs on a path, a star, a lollipop and a cycle.
* Every selection satisfies its rule's defining property on a replay of the
  fills, and invalid graphs are refused.
"""
import numpy as np
import pytest


def grid_csr(img, conn=4):
    """The grid graph of a one-band image with w = f(p) + f(q), as CSR."""
    H, W = img.shape
    f = img.astype(np.int64).reshape(-1)
    rp, ci, cw = [0], [], []
    for p in range(H * W):
        y, x = divmod(p, W)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dy, dx) == (0, 0) or (conn == 4 and dy and dx):
                    continue
                yy, xx = y + dy, x + dx
                if 0 <= yy < H and 0 <= xx < W:
                    q = yy * W + xx
                    ci.append(q)
                    cw.append(f[p] + f[q])
        rp.append(len(ci))
    return np.array(rp, np.int64), np.array(ci, np.int32), np.array(cw, np.int32)


def border_mask(H, W):
    y, x = np.mgrid[0:H, 0:W]
    return ((y == 0) | (y == H - 1) | (x == 0) | (x == W - 1)).reshape(-1).astype(np.uint8)


def edges_csr(n, edges):
    """CSR of an undirected graph given as (u, v, w) triples."""
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


@pytest.mark.parametrize("shape,conn", [((5, 7), 4), ((6, 6), 8), ((1, 6), 4), ((4, 9), 4), ((3, 3), 8)])
def test_grid_as_graph_equals_grid(oracle_lib, shape, conn):
    rng = np.random.default_rng(sum(shape) + conn)
    img = rng.integers(1, 256, shape).astype(np.uint8)
    rp, ci, cw = grid_csr(img, conn)
    H, W = shape
    assert np.array_equal(oracle_lib.graph_naive(rp, ci, cw), oracle_lib.naive(img, conn=conn))
    d = oracle_lib.dijkstra(img, [3 % img.size], conn=conn)
    assert np.array_equal(oracle_lib.graph_parents(rp, ci, cw, d), oracle_lib.parents(img, d, conn=conn))
    bnd = border_mask(H, W)
    ge = oracle_lib.graph_extrema(rp, ci, cw, boundary=bnd)
    ex = oracle_lib.extrema(img, conn=conn)
    assert ge.centroid == ex.centroid and np.array_equal(ge.rank, ex.rank)
    for rule, ref in ((0, oracle_lib.filling_rate(img, conn=conn)), (1, oracle_lib.extrema_method(img, conn=conn))):
        g = oracle_lib.graph_tree_method(rp, ci, cw, rule=rule, boundary=bnd)
        assert np.array_equal(g.sequence, ref.sequence) and np.array_equal(g.filled, ref.filled)
        assert np.array_equal(g.D, ref.D)


@pytest.mark.parametrize("H,W", [(5, 5), (5, 7), (8, 4), (3, 3)])
def test_degree_rule_on_a_4_grid(oracle_lib, H, W):
    """The average degree of a 4-neighbour grid is 4 - 2/W - 2/H: above 3 when
    2/H + 2/W < 1, and then exactly the border pixels (degrees 2 and 3) are
    below it; otherwise only the corners are."""
    rp, _, _ = grid_csr(np.ones((H, W), np.uint8), 4)
    if 2 / H + 2 / W < 1:
        assert np.array_equal(oracle_lib.graph_boundary(rp), border_mask(H, W))
    else:
        corners = np.zeros((H, W), np.uint8)
        corners[[0, 0, -1, -1], [0, -1, 0, -1]] = 1
        assert np.array_equal(oracle_lib.graph_boundary(rp), corners.reshape(-1))


@pytest.mark.parametrize("n,seed", [(40, 0), (200, 1), (501, 2)])
def test_distances_equal_scipy(oracle_lib, n, seed):
    import synth
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    rp, ci, cw = synth.geometric_graph(np.random.default_rng(seed), n)
    S = shortest_path(csr_matrix((cw.astype(np.float64), ci, rp), shape=(n, n)), method="D")
    assert np.array_equal(oracle_lib.graph_naive(rp, ci, cw), S.astype(np.int64))


def test_path_graph_hand_derived(oracle_lib):
    # 0 -1- 1 -2- 2 -3- 3 -4- 4: degrees 1,2,2,2,1, average 1.6, so the ends are
    # the boundary; distance to the nearest end [0,1,3,4,0]: the centre is 3;
    # from 3: [6,5,3,0,4], ranks by (-d, index): 0,1,4,2,3 -> rank [0,1,3,4,2].
    # The tree from vertex 0 (rank 0) is the whole path: one propagation.
    rp, ci, cw = edges_csr(5, [(0, 1, 1), (1, 2, 2), (2, 3, 3), (3, 4, 4)])
    assert oracle_lib.graph_boundary(rp).tolist() == [1, 0, 0, 0, 1]
    ex = oracle_lib.graph_extrema(rp, ci, cw)
    assert ex.centroid == 3 and ex.d_c.tolist() == [6, 5, 3, 0, 4] and ex.rank.tolist() == [0, 1, 3, 4, 2]
    for rule in (0, 1):
        r = oracle_lib.graph_tree_method(rp, ci, cw, rule=rule)
        assert r.sequence.tolist() == [0] and r.filled.tolist() == [10]


def test_star_graph_hand_derived(oracle_lib):
    # centre 0, leaves 1..4 at weights 1..4: the leaves are the boundary, the
    # centre is the centroid, d_c = [0,1,2,3,4], ranks 4,3,2,1,0.  Step 1: s=4,
    # tree 4->0->{1,2,3} leaves {1,2},{1,3},{2,3}; counts [5,3,3,3,5].  Step 2:
    # the least filled of 1,2,3 with the best rank is 3, leaving {1,2}.  Step 3:
    # 2 (rank 2 beats 1's rank 3).  The extrema rule picks the same: the
    # farthest unfilled point each time.
    rp, ci, cw = edges_csr(5, [(0, 1, 1), (0, 2, 2), (0, 3, 3), (0, 4, 4)])
    ex = oracle_lib.graph_extrema(rp, ci, cw)
    assert ex.centroid == 0 and ex.rank.tolist() == [4, 3, 2, 1, 0]
    for rule in (0, 1):
        r = oracle_lib.graph_tree_method(rp, ci, cw, rule=rule)
        assert r.sequence.tolist() == [4, 3, 2] and r.filled.tolist() == [7, 9, 10]
        assert r.D[1, 2] == 3 and r.D[3, 4] == 7


def test_lollipop_degree_equal_to_average_is_not_boundary(oracle_lib):
    # triangle 0-1-2 plus tail 2-3, unit weights: degrees 2,2,3,1, average 2;
    # only vertex 3 has fewer neighbours than the average.  Distances to it:
    # [2,2,1,0], so the centroid is 0 (the first of the two farthest).
    rp, ci, cw = edges_csr(4, [(0, 1, 1), (1, 2, 1), (0, 2, 1), (2, 3, 1)])
    assert oracle_lib.graph_boundary(rp).tolist() == [0, 0, 0, 1]
    ex = oracle_lib.graph_extrema(rp, ci, cw)
    assert ex.centroid == 0 and ex.d_edge.tolist() == [2, 2, 1, 0]


def test_regular_graph_all_boundary(oracle_lib):
    rp, ci, cw = edges_csr(6, [(i, (i + 1) % 6, 1 + i) for i in range(6)])
    assert oracle_lib.graph_boundary(rp).tolist() == [1] * 6
    ex = oracle_lib.graph_extrema(rp, ci, cw)
    assert ex.centroid == 0 and np.all(ex.d_edge == 0)


@pytest.mark.parametrize("n,seed", [(60, 3), (150, 4)])
def test_selection_rules_on_graphs(oracle_lib, n, seed):
    import synth
    rp, ci, cw = synth.geometric_graph(np.random.default_rng(seed), n)
    ex0 = oracle_lib.graph_extrema(rp, ci, cw)
    naive = oracle_lib.graph_naive(rp, ci, cw)
    for rule in (0, 1):
        r = oracle_lib.graph_tree_method(rp, ci, cw, rule=rule)
        assert np.array_equal(r.D, naive)
        mask = np.eye(n, dtype=bool)
        for s in r.sequence:
            c = mask.sum(1)
            unfilled = np.nonzero(c < n)[0]
            if rule == 0:
                least = unfilled[c[unfilled] == c[unfilled].min()]
                assert s == least[np.argmin(ex0.rank[least])]
            else:
                far = unfilled[ex0.d_c[unfilled] == ex0.d_c[unfilled].max()]
                least = far[c[far] == c[far].min()]
                assert s == least.min()
            par = oracle_lib.graph_parents(rp, ci, cw, oracle_lib.graph_dijkstra(rp, ci, cw, [int(s)]))
            for v in range(n):
                u = par[v]
                while u >= 0:
                    mask[u, v] = mask[v, u] = True
                    u = par[u]
        assert mask.all()


@pytest.mark.parametrize("case", ["asymmetric_weight", "missing_reverse", "self_loop", "zero_weight",
                                  "duplicate", "disconnected", "out_of_range"])
def test_invalid_graphs_refused(oracle_lib, case):
    rp, ci, cw = edges_csr(4, [(0, 1, 2), (1, 2, 3), (2, 3, 4)])
    ci, cw = ci.copy(), cw.copy()
    if case == "asymmetric_weight":
        cw[0] += 1
    elif case == "missing_reverse":
        rp, ci, cw = np.array([0, 1, 1, 1, 1], np.int64), np.array([1], np.int32), np.array([1], np.int32)
    elif case == "self_loop":
        ci[0] = 0
    elif case == "zero_weight":
        rp, ci, cw = edges_csr(4, [(0, 1, 0), (1, 2, 3), (2, 3, 4)])
    elif case == "duplicate":
        rp, ci, cw = edges_csr(4, [(0, 1, 2), (0, 1, 2), (1, 2, 3), (2, 3, 4)])
    elif case == "disconnected":
        rp, ci, cw = edges_csr(4, [(0, 1, 2), (2, 3, 4)])
    else:
        ci[0] = 9
    with pytest.raises(RuntimeError):
        oracle_lib.graph_naive(rp, ci, cw)
