"""gapd_all_pairs_noalloc (fixed device scratch, no allocation) against
gapd_all_pairs (caller's workspace), through the C ABI.

Two calls in a row, the second on a smaller image, so anything the first call
left in the shared scratch would show up in the second; both must equal the
workspace entry point bit for bit (D, source sequence, a(t), counts).
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
    assert torch.cuda.is_available(), "needs a GPU"
    return torch


@pytest.fixture(scope="module")
def G(torch_mod):
    from paper_2007_16076_amd import gapd
    gapd.load_library()
    return gapd


def run(G, torch, ctx, mode, noalloc):
    N = ctx.N
    out = torch.full((N, N), -7, dtype=torch.int32, device="cuda")
    seq = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    fil = torch.full((N,), -7, dtype=torch.int64, device="cuda")
    if noalloc:
        D, st = ctx.all_pairs_noalloc(mode, out, sources_out=seq, filled_out=fil)
    else:
        D, st = ctx.all_pairs(mode, out=out, sources_out=seq, filled_out=fil)
    torch.cuda.synchronize()
    return D.cpu().numpy(), seq.cpu().numpy(), fil.cpu().numpy(), st


@pytest.mark.parametrize("mode", [1, 2, 0])
def test_noalloc_equals_workspace_entry_point(G, torch_mod, mode):
    import synth
    rng = np.random.default_rng(31 + mode)
    for shape in [(48, 52), (20, 25)]:  # the second call is smaller
        img = synth.blob_image(rng, *shape)
        ctx = G.Context(img)
        say("noalloc", mode, shape)
        a = run(G, torch_mod, ctx, mode, noalloc=False)
        b = run(G, torch_mod, ctx, mode, noalloc=True)
        assert np.array_equal(a[0], b[0]), "D differs"
        assert (a[0] >= 0).all()
        assert np.array_equal(a[1], b[1]), "source sequence differs"
        assert np.array_equal(a[2], b[2]), "a(t) differs"
        assert a[3].n_prop == b[3].n_prop and a[3].centroid == b[3].centroid
        assert a[3].n_prop_setup == b[3].n_prop_setup
        ctx.close()


def test_noalloc_refuses_workspace_beyond_scratch(G, torch_mod):
    import synth
    img = synth.blob_image(np.random.default_rng(5), 150, 150)  # tree workspace ~75 MB > 64 MiB
    ctx = G.Context(img)
    out = torch_mod.empty((ctx.N, ctx.N), dtype=torch_mod.int32, device="cuda")
    with pytest.raises(G.GapdError) as e:
        ctx.all_pairs_noalloc(G.MODE_TREE_FILL_FR, out)
    assert e.value.status == G.ENOMEM
    # the context is still usable afterwards
    D, st = ctx.all_pairs_noalloc(G.MODE_NAIVE, out)
    assert st.n_prop == ctx.N
    ctx.close()
