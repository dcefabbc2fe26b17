"""Launch-shape tuning: every shape the tuner can pick gives the same results.

D is unique (the minimum over paths), and the filling-rate source sequence is
unique under the tie rules of Section 3.4, so each pinned shape must give
exactly the naive D and the same sequence; gapd_autotune must time every
candidate, write its choice to the JSON cache and leave a correct D in out.
"""
import itertools
import json
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
    assert torch.cuda.is_available(), "needs a GPU"
    return torch


@pytest.fixture(scope="module")
def G(torch_mod):
    from paper_2007_16076_amd import gapd
    gapd.load_library()
    return gapd


def poisoned(torch, *shape):
    return torch.full(shape, -7, dtype=torch.int32, device="cuda")


@pytest.mark.parametrize("mode_name", ["MODE_TREE_FILL_FR", "MODE_TREE_FILL_EXTREMA"])
def test_every_tree_shape_gives_the_same_result(G, torch_mod, oracle_lib, mode_name):
    import synth
    torch = torch_mod
    rng = np.random.default_rng(77)
    img = synth.blob_image(rng, 72, 61)
    ctx = G.Context(img)
    N = ctx.N
    ref = oracle_lib.naive(img)
    mode = getattr(G, mode_name)
    first = None
    for lanes, pf, cap in itertools.product([128, 256], [16, 8], [32, 16, 5]):
        say(mode_name, "lanes", lanes, "pf", pf, "cap", cap)
        ctx.set_tuning(mode, fill_lanes=lanes, walk_pf=pf, spec_cap=cap)
        seq = torch.full((N,), -1, dtype=torch.int32, device="cuda")
        D, st = ctx.all_pairs(mode, out=poisoned(torch, N, N), sources_out=seq)
        torch.cuda.synchronize()
        assert np.array_equal(D.cpu().numpy(), ref), (lanes, pf, cap)
        got = (st.n_prop, seq[: st.n_prop].cpu().numpy().tolist())
        first = first or got
        assert got == first, (lanes, pf, cap)
    ctx.set_tuning(mode)


def test_every_naive_shape_gives_the_same_result(G, torch_mod, oracle_lib):
    torch = torch_mod
    rng = np.random.default_rng(78)
    img = rng.integers(1, 256, size=(40, 97), dtype=np.uint8)
    ctx = G.Context(img, conn=8)
    ref = oracle_lib.naive(img, conn=8)
    for pfw, c1 in itertools.product((4, 8), (0, 1)):
        say("naive pfw", pfw, "check1", c1)
        ctx.set_tuning(G.MODE_NAIVE, naive_pfw=pfw, naive_check1=c1)
        D, _ = ctx.all_pairs(G.MODE_NAIVE, out=poisoned(torch, ctx.N, ctx.N))
        torch.cuda.synchronize()
        assert np.array_equal(D.cpu().numpy(), ref), (pfw, c1)
    ctx.set_tuning(G.MODE_NAIVE)


def test_set_tuning_rejects_unsupported_shapes(G, torch_mod):
    ctx = G.Context(np.full((8, 8), 3, dtype=np.uint8))
    for bad in ({"fill_lanes": 64}, {"walk_pf": 4}, {"spec_cap": 0}, {"spec_cap": 33}, {"naive_pfw": 2},
                {"naive_check1": 2}):
        with pytest.raises(G.GapdError):
            ctx.set_tuning(G.MODE_TREE_FILL_FR, **bad)
    with pytest.raises(G.GapdError):
        ctx.set_tuning(G.MODE_TREE_FILL_SPIRAL)


def test_autotune_writes_the_cache_and_a_correct_D(G, torch_mod, oracle_lib, tmp_path, monkeypatch):
    import synth
    torch = torch_mod
    path = tmp_path / "tune.json"
    monkeypatch.setenv("GAPD_TUNE_FILE", str(path))
    rng = np.random.default_rng(79)
    img = synth.blob_image(rng, 50, 50)
    ctx = G.Context(img)
    N = ctx.N
    ref = oracle_lib.naive(img)
    for mode, ncand in ((G.MODE_NAIVE, 4), (G.MODE_TREE_FILL_FR, 8)):
        say("autotune mode", mode)
        out = poisoned(torch, N, N)
        best = ctx.autotune(mode, out=out)
        torch.cuda.synchronize()
        assert best["candidates"] == ncand and 0 < best["ms"] <= best["ms_default"]
        assert np.array_equal(out.cpu().numpy(), ref)
        D, _ = ctx.all_pairs(mode, out=poisoned(torch, N, N))
        torch.cuda.synchronize()
        assert np.array_equal(D.cpu().numpy(), ref)
    cache = json.loads(path.read_text())
    keys = [k for k in cache if k.endswith("/50x50x1/c4/m0") or k.endswith("/50x50x1/c4/m1")]
    assert len(keys) == 2, cache
