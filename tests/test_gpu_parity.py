"""GPU parity: the HIP library against the CPU oracle, element by element.

Distances are integers, so every comparison is exact (bit-exact int32).
For the filling-rate method the source sequence, the number of propagations,
the geodesic centroid and the filled-pairs trajectory a(t) must equal the
oracle's as well (they are unique given the tie rules both sides follow).
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    return torch


@pytest.fixture(scope="module")
def G(torch_mod):
    from paper_2007_16076_amd import gapd
    gapd.load_library()
    return gapd


def poisoned(torch, *shape):
    """An int32 output pre-filled with -7, so a skipped write cannot pass as an old result."""
    return torch.full(shape, -7, dtype=torch.int32, device="cuda")


def rand_img(seed, h, w, c=1, lo=1, hi=255):
    rng = np.random.default_rng(seed)
    shape = (h, w) if c == 1 else (h, w, c)
    return rng.integers(lo, hi + 1, size=shape, dtype=np.uint8)


def run_fr(G, torch, img, conn):
    ctx = G.Context(img, conn=conn)
    N = ctx.N
    seq = torch.full((N,), -1, dtype=torch.int32, device="cuda")
    fil = torch.zeros((N,), dtype=torch.int64, device="cuda")
    D, st = ctx.all_pairs(G.MODE_TREE_FILL_FR, out=poisoned(torch, N, N), sources_out=seq, filled_out=fil)
    torch.cuda.synchronize()
    k = st.n_prop
    return D.cpu().numpy(), seq.cpu().numpy()[:k], fil.cpu().numpy()[:k], st


# ------------------------------------------------------------------------------------- naive

# (40, 64), (64, 40), (50, 128), (128, 50): one side fills every lane slot of its
# size class, so the sweeps along it take the full-line variant and the others not.
SHAPES = [(1, 1), (1, 7), (7, 1), (2, 2), (5, 9), (32, 32), (33, 65), (70, 3), (3, 70), (64, 64), (65, 64),
          (17, 130), (40, 64), (64, 40), (50, 128), (128, 50)]


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("shape", SHAPES)
def test_naive_matches_oracle(G, torch_mod, oracle_lib, shape, conn):
    say("naive", shape, conn)
    img = rand_img(sum(shape) + conn, *shape)
    D, st = G.Context(img, conn=conn).all_pairs(G.MODE_NAIVE, out=poisoned(torch_mod, img.size, img.size))
    ref = oracle_lib.naive(img, conn=conn)
    assert np.array_equal(D.cpu().numpy(), ref)
    assert st.n_prop == img.size


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("bands", [3, 8])
def test_naive_multiband_matches_oracle(G, torch_mod, oracle_lib, conn, bands):
    say("naive multiband", bands, conn)
    img = rand_img(bands * 10 + conn, 21, 27, c=bands, lo=0)
    N = img.shape[0] * img.shape[1]
    D, _ = G.Context(img, conn=conn).all_pairs(G.MODE_NAIVE, out=poisoned(torch_mod, N, N))
    assert np.array_equal(D.cpu().numpy(), oracle_lib.naive(img, conn=conn))


def test_naive_constant_and_plateau_images(G, torch_mod, oracle_lib):
    say("ties")
    for img in (np.full((9, 14), 3, np.uint8), np.kron(rand_img(4, 4, 5), np.ones((5, 5), np.uint8))):
        for conn in (4, 8):
            D, _ = G.Context(img, conn=conn).all_pairs(G.MODE_NAIVE, out=poisoned(torch_mod, img.size, img.size))
            assert np.array_equal(D.cpu().numpy(), oracle_lib.naive(img, conn=conn))


# ------------------------------------------------------------------------------------- filling rate

@pytest.mark.parametrize("name", ["fr_2x2.json", "fr_3x3_const.json", "fr_strip5.json",
                                  "worked_example_chasles.json"])
def test_filling_rate_golden(G, torch_mod, name):
    g = json.load(open(os.path.join(GOLD, name)))
    say("fr golden", name)
    img = np.array(g["image"], dtype=np.uint8)
    D, seq, fil, st = run_fr(G, torch_mod, img, g["conn"])
    assert seq.tolist() == g["sequence"]
    if "filled" in g:
        assert fil.tolist() == g["filled"]
    if "centroid" in g:
        assert st.centroid == g["centroid"]
    if "D" in g:
        assert D.tolist() == g["D"]
    assert st.n_prop_setup == 2


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("shape,bands", [((1, 1), 1), ((1, 9), 1), ((9, 1), 1), ((6, 7), 1), ((11, 13), 1),
                                         ((16, 16), 1), ((25, 25), 1), ((9, 12), 3), ((20, 7), 8),
                                         ((32, 32), 1), ((40, 64), 1), ((64, 40), 1)])
def test_filling_rate_matches_oracle(G, torch_mod, oracle_lib, shape, bands, conn):
    say("fr", shape, bands, conn)
    img = rand_img(shape[0] * 31 + shape[1] + bands + conn, *shape, c=bands, lo=0 if bands > 1 else 1)
    D, seq, fil, st = run_fr(G, torch_mod, img, conn)
    ref = oracle_lib.filling_rate(img, conn=conn)
    assert st.centroid == ref.centroid
    assert st.n_prop == ref.n_prop
    assert np.array_equal(seq, ref.sequence)
    assert np.array_equal(fil, ref.filled)
    assert np.array_equal(D, ref.D)


def test_filling_rate_blob_128_sampled(G, torch_mod, oracle_lib):
    """Config-2 size (128x128 blobs, N = 16384, D = 1 GiB): the sequence
    equals the oracle's recorded one (tests/golden/fr_blob128.json, written by
    tests/golden/make_golden.py from the oracle only) and sampled rows of D
    equal the oracle's propagations from those sources."""
    import synth
    path = os.path.join(GOLD, "fr_blob128.json")
    img = synth.config2()
    say("fr blob128")
    ctx = G.Context(img)
    torch = torch_mod
    seq = torch.full((ctx.N,), -1, dtype=torch.int32, device="cuda")
    D, st = ctx.all_pairs(G.MODE_TREE_FILL_FR, out=poisoned(torch, ctx.N, ctx.N), sources_out=seq)
    torch.cuda.synchronize()
    say("fr blob128 done", st.n_prop, st.ms_total)
    rng = np.random.default_rng(7)
    rows = rng.choice(ctx.N, size=24, replace=False)
    ref = oracle_lib.rows(img, rows)
    assert np.array_equal(D[torch.as_tensor(rows, device="cuda")].cpu().numpy(), ref)
    if os.path.exists(path):
        g = json.load(open(path))
        assert g["sha256"] == synth.sha256(img)
        assert st.n_prop == g["n_prop"]
        assert st.centroid == g["centroid"]
        assert seq[: st.n_prop].cpu().numpy().tolist() == g["sequence"]


def test_filling_rate_voronoi_192_sampled(G, torch_mod, oracle_lib):
    """Config-3 size (192x192x8 Voronoi, w = 1 + L1, N = 36864, D = 5.4 GB):
    the filling-rate D equals the naive D everywhere (tree words fit LDS, the
    counts do not: the other fill variant with the tree cache), sampled rows
    equal the oracle's propagations, and a(t) ends at N(N-1)/2."""
    import synth
    img = synth.config3()
    say("fr voronoi192")
    ctx = G.Context(img)
    torch = torch_mod
    N = ctx.N
    fil = torch.zeros((N,), dtype=torch.int64, device="cuda")
    D, st = ctx.all_pairs(G.MODE_TREE_FILL_FR, out=poisoned(torch, N, N), filled_out=fil)
    torch.cuda.synchronize()
    say("fr voronoi192 done", st.n_prop, st.ms_total, st.n_cache_hits)
    assert int(fil[st.n_prop - 1]) == N * (N - 1) // 2
    assert st.n_cache_hits > 0
    rows = np.random.default_rng(8).choice(N, size=8, replace=False)
    ref = oracle_lib.rows(img, rows)
    assert np.array_equal(D[torch.as_tensor(rows, device="cuda")].cpu().numpy(), ref)
    Dn, _ = ctx.all_pairs(G.MODE_NAIVE, out=poisoned(torch, N, N))
    assert torch.equal(D, Dn)
    del D, Dn
    torch.cuda.empty_cache()


# ------------------------------------------------------------------------------------- sssp

def test_sssp_matches_oracle(G, torch_mod, oracle_lib):
    say("sssp small")
    img = rand_img(3, 40, 50)
    ctx = G.Context(img)
    src = np.array([0, 1999, 777, 1000, 1000], dtype=np.int32)
    out = ctx.sssp(src, out=poisoned(torch_mod, src.size, ctx.N)).cpu().numpy()
    assert np.array_equal(out, oracle_lib.rows(img, src))


def test_sssp_large_image_global_field(G, torch_mod, oracle_lib):
    """512x512 blob image: the distance field does not fit in LDS and lives in
    the output rows."""
    import synth
    say("sssp 512")
    img = synth.blob_image(np.random.default_rng(12), 512, 512)
    ctx = G.Context(img)
    src = np.array([0, 512 * 512 - 1, 123456, 77], dtype=np.int32)
    out = ctx.sssp(src, out=poisoned(torch_mod, src.size, ctx.N)).cpu().numpy()
    assert np.array_equal(out, oracle_lib.rows(img, src))


def test_sssp_rejects_out_of_range(G, torch_mod):
    ctx = G.Context(rand_img(1, 4, 4))
    with pytest.raises(G.GapdError) as e:
        ctx.sssp(np.array([0, 16], dtype=np.int32))
    assert e.value.status == G.EINVAL


# ------------------------------------------------------------------------------------- batched

@pytest.mark.parametrize("mode", [0, 1])
def test_batched_matches_solo(G, torch_mod, oracle_lib, mode):
    say("batched", mode)
    rng = np.random.default_rng(99)
    imgs = [rng.integers(1, 256, size=(int(rng.integers(1, 30)), int(rng.integers(1, 30))), dtype=np.uint8)
            for _ in range(12)]
    offs = G.pack_offsets([im.shape for im in imgs])
    out, offs, nprop = G.all_pairs_batched(imgs, mode=mode, out=poisoned(torch_mod, int(offs[-1])), offsets=offs)
    o = out.cpu().numpy()
    for b, im in enumerate(imgs):
        N = im.size
        Db = o[offs[b]: offs[b] + N * N].reshape(N, N)
        if mode == 0:
            assert np.array_equal(Db, oracle_lib.naive(im))
        else:
            ref = oracle_lib.filling_rate(im)
            assert np.array_equal(Db, ref.D)
            assert nprop[b] == ref.n_prop


@pytest.mark.parametrize("chunk", ["3", "64"])
def test_step_graph_replay_equals_direct(G, torch_mod, monkeypatch, chunk):
    """Chunks of loop steps replayed as a HIP graph give the run of direct
    launches: the same D, source sequence and a(t) after every step, that is
    after every replay (eager polls and synchronisations between replays),
    for one image and for a batch."""
    import synth
    torch = torch_mod
    monkeypatch.setenv("GAPD_FR_CHUNK", chunk)
    img = synth.blob_image(np.random.default_rng(21), 40, 44)
    res = {}
    for on in ("0", "1"):
        monkeypatch.setenv("GAPD_FR_GRAPH", on)
        res[on] = run_fr(G, torch, img, 4)
    say("graph replays", chunk, res["1"][3].graph_replays)
    assert res["0"][3].graph_replays == 0 and res["1"][3].graph_replays > 0
    for k in range(3):
        assert np.array_equal(res["0"][k], res["1"][k])
    rng = np.random.default_rng(22)
    imgs = [rng.integers(1, 256, size=(int(rng.integers(8, 40)), int(rng.integers(8, 40))), dtype=np.uint8)
            for _ in range(6)]
    offs = G.pack_offsets([im.shape for im in imgs])
    nseq = sum(im.size for im in imgs)
    outs = {}
    for on in ("0", "1"):
        monkeypatch.setenv("GAPD_FR_GRAPH", on)
        seq = torch.full((nseq,), -7, dtype=torch.int32, device="cuda")
        out, _, nprop = G.all_pairs_batched(imgs, mode=G.MODE_TREE_FILL_FR, out=poisoned(torch, int(offs[-1])),
                                            offsets=offs, sources_out=seq)
        outs[on] = (out.cpu().numpy(), nprop.copy(), seq.cpu().numpy())
    for k in range(3):
        assert np.array_equal(outs["0"][k], outs["1"][k])


# ------------------------------------------------------------------------------------- errors, determinism

def test_round_cap_reports_no_convergence(G, torch_mod, monkeypatch):
    say("enoconv")
    monkeypatch.setenv("GAPD_MAX_ROUNDS", "1")
    ctx = G.Context(rand_img(5, 30, 30))
    with pytest.raises(G.GapdError) as e:
        ctx.all_pairs(G.MODE_NAIVE)
    assert e.value.status == G.ENOCONV


def test_filling_rate_deterministic(G, torch_mod):
    say("determinism")
    img = rand_img(6, 24, 31)
    a = run_fr(G, torch_mod, img, 4)
    b = run_fr(G, torch_mod, img, 4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
