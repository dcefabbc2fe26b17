"""GPU parity of the geodesic extrema method and the spiral methods.

Each run is compared with the CPU oracle on the same seeded input: D bit for
bit, and the whole source sequence, the filled-pair counts a(t) and the number
of propagations exactly (integer work, tolerance 0).  The spiral methods take
their random draws as an input, so both sides see the same draws.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


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


def rand_img(seed, h, w, c=1):
    rng = np.random.default_rng(seed)
    shape = (h, w) if c == 1 else (h, w, c)
    return rng.integers(1, 256, size=shape, dtype=np.uint8)


def draws_for(seed, n):
    return np.random.default_rng(1000 + seed).integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)


def run_method(G, torch, img, conn, mode=None, draws=None, h=0):
    ctx = G.Context(img, conn=conn)
    N = ctx.N
    seq = torch.full((N,), -1, dtype=torch.int32, device="cuda")
    fil = torch.zeros((N,), dtype=torch.int64, device="cuda")
    if draws is None:
        D, st = ctx.all_pairs(mode, out=torch.full((N, N), -7, dtype=torch.int32, device="cuda"),
                              sources_out=seq, filled_out=fil)
    else:
        D, st = ctx.all_pairs_spiral(draws, h=h, out=torch.full((N, N), -7, dtype=torch.int32, device="cuda"),
                                     sources_out=seq, filled_out=fil)
    torch.cuda.synchronize()
    k = st.n_prop
    return D.cpu().numpy(), seq.cpu().numpy()[:k], fil.cpu().numpy()[:k], st


def check_same(res, ref, N):
    D, seq, fil, st = res
    assert st.n_prop == ref.n_prop
    assert np.array_equal(seq, ref.sequence)
    assert np.array_equal(fil, ref.filled)
    assert np.array_equal(D, ref.D.reshape(N, N))


SHAPES = [((1, 1), 1), ((1, 9), 1), ((9, 1), 1), ((2, 3), 1), ((6, 7), 1), ((11, 13), 1), ((16, 16), 1),
          ((7, 9), 3)]


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("shape,bands", SHAPES)
def test_extrema_method_matches_oracle(G, torch_mod, oracle_lib, shape, bands, conn):
    img = rand_img(sum(shape) + bands + conn, *shape, c=bands)
    say("extrema", shape, bands, conn)
    res = run_method(G, torch_mod, img, conn, mode=G.MODE_TREE_FILL_EXTREMA)
    ref = oracle_lib.extrema_method(img, conn=conn)
    check_same(res, ref, shape[0] * shape[1])
    N = shape[0] * shape[1]
    if N > 1:
        assert res[3].centroid == ref.centroid and res[3].n_prop_setup == 2


def test_extrema_golden(G, torch_mod):
    g = json.load(open(os.path.join(GOLD, "ext_2x3_const.json")))
    img = np.array(g["image"], np.uint8)
    say("extrema golden")
    D, seq, fil, st = run_method(G, torch_mod, img, g["conn"], mode=G.MODE_TREE_FILL_EXTREMA)
    assert seq.tolist() == g["sequence_extrema"]
    D, seq, fil, st = run_method(G, torch_mod, img, g["conn"], mode=G.MODE_TREE_FILL_FR)
    assert seq.tolist() == g["sequence_filling"]


def test_extrema_blob_speculative_cache(G, torch_mod, oracle_lib):
    """A 48x48 blob image: the speculative tree cache is in use and the
    sequence is still the oracle's, step for step."""
    import synth
    img = synth.blob_image(np.random.default_rng(3), 48, 48)
    say("extrema blob48")
    res = run_method(G, torch_mod, img, 4, mode=G.MODE_TREE_FILL_EXTREMA)
    ref = oracle_lib.extrema_method(img, conn=4)
    check_same(res, ref, 48 * 48)
    assert res[3].n_cache_hits > 0


@pytest.mark.parametrize("h", [0, 3, 5])
@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("shape,bands", SHAPES)
def test_spiral_matches_oracle(G, torch_mod, oracle_lib, shape, bands, conn, h):
    img = rand_img(3 * sum(shape) + bands + conn, *shape, c=bands)
    N = shape[0] * shape[1]
    r = draws_for(N + h + conn, N)
    say("spiral", shape, bands, conn, h)
    res = run_method(G, torch_mod, img, conn, draws=r, h=h)
    ref = oracle_lib.spiral(img, r, h=h, conn=conn)
    check_same(res, ref, N)
    assert res[3].n_prop_setup == 0 and res[3].centroid == -1


@pytest.mark.parametrize("which", ["draws_first", "draws_last"])
def test_spiral_golden(G, torch_mod, which):
    g = json.load(open(os.path.join(GOLD, "spiral_2x3_const.json")))
    img = np.array(g["image"], np.uint8)
    r = np.full(6, 0 if which == "draws_first" else 0xFFFFFFFF, np.uint32)
    say("spiral golden", which)
    assert run_method(G, torch_mod, img, g["conn"], draws=r, h=0)[1].tolist() == g[which]["spiral"]
    assert run_method(G, torch_mod, img, g["conn"], draws=r, h=3)[1].tolist() == g[which]["repulsion3"]


@pytest.mark.parametrize("h", [0, 3])
def test_spiral_blob_40(G, torch_mod, oracle_lib, h):
    """Several turns, long turns (156 pixels for the outer frame of 40x40),
    ragged block counts in the member search."""
    import synth
    img = synth.blob_image(np.random.default_rng(11), 40, 40)
    r = draws_for(40 + h, 1600)
    say("spiral blob40", h)
    res = run_method(G, torch_mod, img, 4, draws=r, h=h)
    ref = oracle_lib.spiral(img, r, h=h, conn=4)
    check_same(res, ref, 1600)


def test_spiral_argument_errors(G, torch_mod):
    import ctypes
    import torch
    ctx = G.Context(rand_img(1, 5, 5), conn=4)
    lib = G.load_library()
    ctx._ensure_workspace(G.MODE_TREE_FILL_SPIRAL)
    out = torch.empty((25, 25), dtype=torch.int32, device="cuda")
    d = torch.zeros(25, dtype=torch.int32, device="cuda")
    st = G.Stats()
    assert lib.gapd_all_pairs_spiral(ctx._h, -1, d.data_ptr(), out.data_ptr(), ctypes.byref(st)) == G.EINVAL
    assert lib.gapd_all_pairs_spiral(ctx._h, 65537, d.data_ptr(), out.data_ptr(), ctypes.byref(st)) == G.EINVAL
    assert lib.gapd_all_pairs_spiral(ctx._h, 3, None, out.data_ptr(), ctypes.byref(st)) == G.EINVAL
    assert lib.gapd_all_pairs(ctx._h, G.MODE_TREE_FILL_SPIRAL, out.data_ptr(), ctypes.byref(st)) == G.EINVAL
    # the context still works afterwards
    D, st2 = ctx.all_pairs_spiral(np.zeros(25, np.uint32), h=3)
    assert st2.n_prop > 0


def test_batched_extrema_matches_oracle(G, torch_mod, oracle_lib):
    import torch
    rng = np.random.default_rng(21)
    shapes = [(int(rng.integers(3, 20)), int(rng.integers(3, 20))) for _ in range(7)] + [(1, 1), (1, 6)]
    imgs = [rand_img(100 + i, h, w) for i, (h, w) in enumerate(shapes)]
    say("batched extrema", shapes)
    offs = G.pack_offsets(shapes)
    out = torch.full((int(offs[-1]),), -7, dtype=torch.int32, device="cuda")
    out, offs, nprop = G.all_pairs_batched(imgs, mode=G.MODE_TREE_FILL_EXTREMA, conn=4, out=out, offsets=offs)
    o = out.cpu().numpy()
    for b, img in enumerate(imgs):
        ref = oracle_lib.extrema_method(img, conn=4)
        N = img.size
        assert np.array_equal(o[offs[b]:offs[b] + N * N].reshape(N, N), ref.D)
        assert int(nprop[b]) == ref.n_prop


def test_server_extrema_job(G, torch_mod, oracle_lib):
    img = rand_img(5, 14, 17)
    say("server extrema")
    srv = G.Server(1 << 28, max_slots=2)
    t = srv.submit_all_pairs(img, mode=G.MODE_TREE_FILL_EXTREMA)
    r = srv.wait(t)
    got = srv.result_tensor(r).cpu().numpy()
    ref = oracle_lib.extrema_method(img, conn=4)
    assert np.array_equal(got.reshape(ref.D.shape), ref.D)
    assert r.n_prop == ref.n_prop
    srv.release(t)
    srv.close()


@pytest.mark.parametrize("name", ["random", "bumps", "hairpin"])
def test_comparison_images_all_methods(G, torch_mod, oracle_lib, name):
    """The 25x25 stand-ins of the method comparison, 8-neighbours: every tree
    method on the GPU gives the oracle's sequence and D."""
    import synth
    img = synth.deltar_images()[name]
    N = img.size
    say("comparison image", name)
    check_same(run_method(G, torch_mod, img, 8, mode=G.MODE_TREE_FILL_FR), oracle_lib.filling_rate(img, conn=8), N)
    check_same(run_method(G, torch_mod, img, 8, mode=G.MODE_TREE_FILL_EXTREMA),
               oracle_lib.extrema_method(img, conn=8), N)
    r = synth.spiral_draws(0, N)
    for h in (0, 3):
        check_same(run_method(G, torch_mod, img, 8, draws=r, h=h), oracle_lib.spiral(img, r, h=h, conn=8), N)
