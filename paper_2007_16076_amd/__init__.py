"""gapd: all pairs of geodesic distances on a pixel grid, on AMD MI355X (gfx950).

The computation runs in libgapd.so (hand-written HIP kernels, C ABI in
include/gapd.h); :mod:`paper_2007_16076_amd.gapd` is its ctypes binding.
"""
from .gapd import (  # noqa: F401
    CONN4, CONN8, W_SUM, W_1PL1, MODE_NAIVE, MODE_TREE_FILL_FR, Context, Server, GapdError,
    all_pairs_batched, batched_workspace_size, load_library, pack_offsets,
)
