"""Pins of the oracle's other tree-based methods: the geodesic extrema method
(Section 3.3, algorithm extrema) and the spiral methods without and with
repulsion (Sections 3.1 and 3.2).

They share the filling-rate method's propagation and redundancy fill, which
``test_oracle.py`` pins; what is new here is the choice of the sources.  The
pins are hand-derived sequences (``golden/ext_2x3_const.json``,
``golden/spiral_2x3_const.json``), the spiral turns' geometry, and, on random
images, the defining property of every selection checked against a replay of
the fills (the replay only tracks which pairs are filled; it never chooses a
source).
"""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def border_distance(H, W):
    y, x = np.mgrid[0:H, 0:W]
    return np.minimum(np.minimum(y, x), np.minimum(H - 1 - y, W - 1 - x)).reshape(-1)


def replay_counts(oracle_lib, img, seq, conn):
    """counts[t] = per-point filled-entry counts before step t (and after the last)."""
    N = img.shape[0] * img.shape[1]
    mask = np.eye(N, dtype=bool)
    out = [mask.sum(1)]
    for s in seq:
        d = oracle_lib.dijkstra(img, [int(s)], conn=conn)
        par = oracle_lib.parents(img, d, conn=conn)
        for v in range(N):
            u = par[v]
            while u >= 0:
                mask[u, v] = mask[v, u] = True
                u = par[u]
        out.append(mask.sum(1))
    return out


# ---- spiral turns ------------------------------------------------------------------------

@pytest.mark.parametrize("H,W", [(1, 1), (1, 7), (6, 1), (2, 2), (2, 3), (4, 4), (5, 5), (5, 8), (9, 4)])
def test_spiral_turns_partition_the_image(oracle_lib, H, W):
    bd = border_distance(H, W)
    seen = []
    for k in range(max(H, W)):
        pix, cyc = oracle_lib.spiral_turn(H, W, k)
        if pix.size == 0:
            assert k > bd.max()
            continue
        assert np.all(bd[pix] == k)                                # the frame at distance k
        assert set(pix.tolist()) == set(np.nonzero(bd == k)[0].tolist())
        assert pix[0] == k * W + k                                 # starts at the top-left corner
        y, x = pix // W, pix % W
        steps = np.abs(np.diff(y)) + np.abs(np.diff(x))
        assert np.all(steps == 1)                                  # consecutive pixels are neighbours
        if pix.size > 1 and H - 2 * k > 1 and W - 2 * k > 1:
            assert cyc and abs(y[-1] - y[0]) + abs(x[-1] - x[0]) == 1   # a closed frame
            assert (y[1], x[1]) == (k, k + 1)                          # clockwise
        else:
            assert not cyc
        seen += pix.tolist()
    assert sorted(seen) == list(range(H * W))


def test_spiral_turn_golden(oracle_lib):
    g = gold("spiral_2x3_const.json")
    pix, cyc = oracle_lib.spiral_turn(2, 3, 0)
    assert pix.tolist() == g["turn0"] and cyc


# ---- hand-derived sequences --------------------------------------------------------------

def test_extrema_method_golden(oracle_lib):
    g = gold("ext_2x3_const.json")
    img = np.array(g["image"], np.uint8)
    ex = oracle_lib.extrema_method(img, conn=g["conn"])
    fr = oracle_lib.filling_rate(img, conn=g["conn"])
    assert ex.sequence.tolist() == g["sequence_extrema"]
    assert fr.sequence.tolist() == g["sequence_filling"]
    assert ex.centroid == g["centroid"]
    assert np.array_equal(ex.D, oracle_lib.naive(img, conn=g["conn"]))


@pytest.mark.parametrize("draws", ["draws_first", "draws_last"])
def test_spiral_golden(oracle_lib, draws):
    g = gold("spiral_2x3_const.json")
    img = np.array(g["image"], np.uint8)
    r = np.full(6, 0 if draws == "draws_first" else 0xFFFFFFFF, np.uint32)
    assert oracle_lib.spiral(img, r, h=0).sequence.tolist() == g[draws]["spiral"]
    assert oracle_lib.spiral(img, r, h=1).sequence.tolist() == g[draws]["spiral"]   # h <= 1: no repulsion
    assert oracle_lib.spiral(img, r, h=3).sequence.tolist() == g[draws]["repulsion3"]


@pytest.mark.parametrize("W", [1, 2, 5, 9])
def test_strip_special_cases(oracle_lib, W):
    """On a 1xW strip every pixel is a border pixel (centroid 0) and the tree
    from an end pixel is the whole strip: one propagation fills D."""
    rng = np.random.default_rng(W)
    img = rng.integers(1, 256, (1, W)).astype(np.uint8)
    ex = oracle_lib.extrema_method(img)
    assert ex.sequence.tolist() == ([W - 1] if W > 1 else [])
    # spiral: the single turn is the row; the first draw picks pixel 0, an end
    sp = oracle_lib.spiral(img, np.zeros(W, np.uint32), h=3)
    assert sp.sequence.tolist() == ([0] if W > 1 else [])
    # from an interior pixel the two branches leave their cross pairs
    if W >= 3:
        mid = np.full(W, (1 << 32) // W + 1, np.uint32)     # picks member 1 of S
        sp = oracle_lib.spiral(img, mid, h=0)
        assert sp.sequence[0] == 1 and sp.n_prop == 2


# ---- invariants and selection properties on random images --------------------------------

def methods(oracle_lib, img, conn, rnd):
    return {"extrema": oracle_lib.extrema_method(img, conn=conn),
            "spiral": oracle_lib.spiral(img, rnd, h=0, conn=conn),
            "repulsion3": oracle_lib.spiral(img, rnd, h=3, conn=conn)}


@pytest.mark.parametrize("shape,conn,seed", [((7, 9), 4, 0), ((8, 8), 8, 1), ((5, 11), 4, 2), ((6, 6, 3), 4, 3)])
def test_methods_fill_exactly_and_select_by_their_rule(oracle_lib, shape, conn, seed):
    rng = np.random.default_rng(seed)
    img = rng.integers(1, 256, shape).astype(np.uint8)
    H, W = shape[:2]
    N = H * W
    rnd = rng.integers(0, 1 << 32, N, dtype=np.uint64).astype(np.uint32)
    naive = oracle_lib.naive(img, conn=conn)
    ex0 = oracle_lib.extrema(img, conn=conn)
    bd = border_distance(H, W)
    for name, res in methods(oracle_lib, img, conn, rnd).items():
        seq = res.sequence
        assert np.array_equal(res.D, naive), name                 # Property 1: every entry exact
        assert len(set(seq.tolist())) == len(seq) <= N              # distinct sources
        assert np.all(np.diff(res.filled) > 0)                      # every step fills a new pair
        assert res.filled[-1] == N * (N - 1) // 2
        counts = replay_counts(oracle_lib, img, seq, conn)
        assert np.all(counts[-1] == N)
        for t, s in enumerate(seq):
            c = counts[t]
            unfilled = np.nonzero(c < N)[0]
            assert c[s] < N, name                                   # sources are unfilled points
            if name == "extrema":
                far = unfilled[ex0.d_c[unfilled] == ex0.d_c[unfilled].max()]
                least = far[c[far] == c[far].min()]
                assert s == least.min()
            else:
                assert bd[s] == bd[unfilled].min()                  # the most exterior unfilled turn
        # the selection rule stops exactly when D is filled
        assert np.any(counts[-2] < N)


def test_repulsion_keeps_draws_apart(oracle_lib):
    """With h = 3, the first two draws of a turn are at least 3 turn positions
    apart while the turn's S lasts (a 12x12 image: the outer frame has 44
    pixels, far more than its first two sources fill)."""
    rng = np.random.default_rng(9)
    img = rng.integers(1, 256, (12, 12)).astype(np.uint8)
    pix, _ = oracle_lib.spiral_turn(12, 12, 0)
    pos = {int(p): i for i, p in enumerate(pix)}
    L = len(pix)
    for trial in range(20):
        rnd = rng.integers(0, 1 << 32, 144, dtype=np.uint64).astype(np.uint32)
        seq = oracle_lib.spiral(img, rnd, h=3, max_steps=2).sequence
        a, b = pos[int(seq[0])], pos[int(seq[1])]
        gap = min((a - b) % L, (b - a) % L)
        assert gap >= 3


def test_spiral_draws_exhausted_is_an_error(oracle_lib):
    img = np.random.default_rng(0).integers(1, 256, (6, 6)).astype(np.uint8)
    with pytest.raises(RuntimeError):
        oracle_lib.spiral(img, np.zeros(1, np.uint32))
