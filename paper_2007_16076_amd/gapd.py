"""ctypes binding of libgapd.so (include/gapd.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  torch tensors provide device memory and the HIP
stream (``torch.cuda.current_stream().cuda_stream`` on ROCm).  If the built
library is missing, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgapd.so")

OK, PENDING, EINVAL, ENOMEM, EDEVICE, ERANGE, ENOCONV, EBUSY, ENOTFOUND = 0, 1, -1, -2, -3, -4, -5, -6, -7
CONN4, CONN8 = 4, 8
W_SUM, W_1PL1 = 0, 1
MODE_NAIVE, MODE_TREE_FILL_FR, MODE_TREE_FILL_EXTREMA, MODE_TREE_FILL_SPIRAL = 0, 1, 2, 3
JOB_ALL_PAIRS, JOB_MULTI_SOURCE = 0, 1

EXPORTED = [
    "gapd_create", "gapd_set_stream", "gapd_workspace_size", "gapd_set_workspace", "gapd_sssp",
    "gapd_all_pairs", "gapd_all_pairs_spiral", "gapd_all_pairs_noalloc", "gapd_autotune", "gapd_set_tuning", "gapd_destroy", "gapd_strerror", "gapd_last_error", "gapd_batched_workspace_size",
    "gapd_all_pairs_batched", "gapd_server_create", "gapd_serve_submit", "gapd_serve_poll", "gapd_serve_wait",
    "gapd_serve_release", "gapd_server_destroy", "gapd_graph_create", "gapd_graph_set_stream",
    "gapd_graph_workspace_size", "gapd_graph_set_workspace", "gapd_graph_sssp", "gapd_graph_all_pairs",
    "gapd_graph_last_error", "gapd_graph_destroy",
]


class GapdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gapd status {status}: {msg}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("n_prop", ctypes.c_int64), ("n_prop_setup", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("centroid", ctypes.c_int32), ("_pad", ctypes.c_int32),
                ("sources_out", ctypes.c_void_p), ("filled_out", ctypes.c_void_p),
                ("ms_total", ctypes.c_float), ("ms_setup", ctypes.c_float), ("ms_kernel", ctypes.c_float),
                ("time_kernels", ctypes.c_int32), ("ms_step_kernels", ctypes.c_float),
                ("ms_fill_kernels", ctypes.c_float), ("graph_replays", ctypes.c_int32),
                ("n_prop_speculative", ctypes.c_int64), ("n_cache_hits", ctypes.c_int64),
                ("step_trace", ctypes.c_void_p), ("rounds_speculative", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("fill_lanes", ctypes.c_int32), ("walk_pf", ctypes.c_int32), ("spec_cap", ctypes.c_int32),
                ("naive_pfw", ctypes.c_int32), ("ms", ctypes.c_float), ("ms_default", ctypes.c_float),
                ("candidates", ctypes.c_int32), ("naive_check1", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("H", ctypes.c_int), ("W", ctypes.c_int), ("C", ctypes.c_int),
                ("conn", ctypes.c_int), ("weight_mode", ctypes.c_int), ("mode", ctypes.c_int),
                ("image", ctypes.c_void_p), ("sources", ctypes.c_void_p), ("K", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("dev_out", ctypes.c_void_p), ("elems", ctypes.c_size_t), ("n_prop", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgapd.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2007_16076_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    P, I, I64, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "gapd_create": ([P, I, I, I, I, I, ctypes.POINTER(P)], I),
        "gapd_set_stream": ([P, P], I),
        "gapd_workspace_size": ([P, I, ctypes.POINTER(SZ)], I),
        "gapd_set_workspace": ([P, P, SZ], I),
        "gapd_sssp": ([P, P, I, P], I),
        "gapd_all_pairs": ([P, I, P, ctypes.POINTER(Stats)], I),
        "gapd_all_pairs_spiral": ([P, I, P, P, ctypes.POINTER(Stats)], I),
        "gapd_destroy": ([P], None),
        "gapd_strerror": ([I], ctypes.c_char_p),
        "gapd_last_error": ([P], ctypes.c_char_p),
        "gapd_batched_workspace_size": ([P, P, I, I, I, I, ctypes.POINTER(SZ)], I),
        "gapd_all_pairs_noalloc": ([P, I, P, ctypes.POINTER(Stats)], I),
        "gapd_autotune": ([P, I, P, ctypes.POINTER(Tuning)], I),
        "gapd_set_tuning": ([P, I, ctypes.POINTER(Tuning)], I),
        "gapd_all_pairs_batched": ([P, P, P, I, I, I, I, I, P, P, P, P, P, SZ, P], I),
        "gapd_server_create": ([P, SZ, I, ctypes.POINTER(P)], I),
        "gapd_serve_submit": ([P, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)], I),
        "gapd_serve_poll": ([P, ctypes.c_uint64, ctypes.POINTER(Result)], I),
        "gapd_serve_wait": ([P, ctypes.c_uint64, ctypes.POINTER(Result)], I),
        "gapd_serve_release": ([P, ctypes.c_uint64], I),
        "gapd_server_destroy": ([P], None),
        "gapd_graph_create": ([ctypes.c_int64, P, P, P, P, ctypes.POINTER(P)], I),
        "gapd_graph_set_stream": ([P, P], I),
        "gapd_graph_workspace_size": ([P, I, ctypes.POINTER(SZ)], I),
        "gapd_graph_set_workspace": ([P, P, SZ], I),
        "gapd_graph_sssp": ([P, P, I, P], I),
        "gapd_graph_all_pairs": ([P, I, P, ctypes.POINTER(Stats)], I),
        "gapd_graph_last_error": ([P], ctypes.c_char_p),
        "gapd_graph_destroy": ([P], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load_library().gapd_strerror(status).decode()


def _check(status: int, ctx=None):
    if status not in (OK, PENDING):
        lib = load_library()
        msg = lib.gapd_last_error(ctx).decode() if ctx is not None else lib.gapd_last_error(None).decode()
        raise GapdError(status, f"{strerror(status)}: {msg}")
    return status


def _img_arr(image):
    image = np.ascontiguousarray(image, dtype=np.uint8)
    if image.ndim == 2:
        return image, image.shape[0], image.shape[1], 1
    if image.ndim == 3:
        return image, image.shape[0], image.shape[1], image.shape[2]
    raise ValueError("image must be (H, W) or (H, W, C)")


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dptr(t) -> int:
    return t.data_ptr()


@dataclass
class AllPairsStats:
    n_prop: int
    n_prop_setup: int
    rounds: int
    centroid: int
    ms_total: float
    ms_setup: float
    ms_kernel: float
    ms_step_kernels: float
    ms_fill_kernels: float
    n_prop_speculative: int = 0
    n_cache_hits: int = 0
    graph_replays: int = 0
    rounds_speculative: int = 0


class Context:
    """One image on the device (gapd_create)."""

    def __init__(self, image, conn: int = CONN4, weight_mode: int | None = None, stream=None):
        lib = load_library()
        self._img, self.H, self.W, self.C = _img_arr(image)
        self.N = self.H * self.W
        self.conn = conn
        self.wmode = (W_SUM if self.C == 1 else W_1PL1) if weight_mode is None else weight_mode
        h = ctypes.c_void_p()
        _check(lib.gapd_create(self._img.ctypes.data, self.H, self.W, self.C, conn, self.wmode, ctypes.byref(h)))
        self._h = h
        self._ws = None
        self.set_stream(stream)

    def set_stream(self, stream=None):
        _check(load_library().gapd_set_stream(self._h, _stream_ptr(stream)), self._h)

    def close(self):
        if getattr(self, "_h", None):
            load_library().gapd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_size(self, mode: int) -> int:
        n = ctypes.c_size_t()
        _check(load_library().gapd_workspace_size(self._h, mode, ctypes.byref(n)), self._h)
        return n.value

    def _ensure_workspace(self, mode: int):
        import torch
        need = self.workspace_size(mode)
        if need == 0:
            return
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        _check(load_library().gapd_set_workspace(self._h, _dptr(self._ws), self._ws.numel()), self._h)

    def sssp(self, sources, out=None):
        """K propagations: returns a (K, N) int32 device tensor."""
        import torch
        src = sources if isinstance(sources, torch.Tensor) else torch.as_tensor(np.asarray(sources, np.int32))
        src = src.to(device="cuda", dtype=torch.int32).contiguous()
        K = src.numel()
        if out is None:
            out = torch.empty((K, self.N), dtype=torch.int32, device="cuda")
        _check(load_library().gapd_sssp(self._h, _dptr(src), K, _dptr(out)), self._h)
        return out

    def all_pairs(self, mode: int = MODE_NAIVE, out=None, sources_out=None, filled_out=None,
                  time_kernels: bool = False, step_trace=None):
        """The N x N distances array (device int32) and the call's statistics.
        step_trace: optional device int64 tensor of 32 * N entries (per-step
        counters of the tree modes, see gapd_stats.step_trace)."""
        import torch
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.int32, device="cuda")
        self._ensure_workspace(mode)
        st = Stats()
        st.sources_out = _dptr(sources_out) if sources_out is not None else None
        st.filled_out = _dptr(filled_out) if filled_out is not None else None
        st.step_trace = _dptr(step_trace) if step_trace is not None else None
        st.time_kernels = 1 if time_kernels else 0
        _check(load_library().gapd_all_pairs(self._h, mode, _dptr(out), ctypes.byref(st)), self._h)
        return out, _stats(st)

    def autotune(self, mode: int, out=None) -> dict:
        """gapd_autotune: time the candidate launch shapes of `mode` on this image
        and keep the fastest (JSON cache); returns the choice and both timings."""
        import torch
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.int32, device="cuda")
        self._ensure_workspace(mode)
        t = Tuning()
        _check(load_library().gapd_autotune(self._h, mode, _dptr(out), ctypes.byref(t)), self._h)
        return {k: getattr(t, k) for k, _ in Tuning._fields_ if not k.startswith("_")}

    def set_tuning(self, mode: int, fill_lanes=128, walk_pf=16, spec_cap=32, naive_pfw=4, naive_check1=0) -> None:
        """gapd_set_tuning: pin the launch shapes of `mode` on images of this key."""
        t = Tuning(fill_lanes, walk_pf, spec_cap, naive_pfw, 0.0, 0.0, 0, naive_check1)
        _check(load_library().gapd_set_tuning(self._h, mode, ctypes.byref(t)), self._h)

    def all_pairs_noalloc(self, mode: int, out, sources_out=None, filled_out=None):
        """gapd_all_pairs_noalloc: the library allocates nothing (the tree modes use
        its fixed 64 MiB device scratch); out is the caller's (N, N) int32 tensor."""
        st = Stats()
        st.sources_out = _dptr(sources_out) if sources_out is not None else None
        st.filled_out = _dptr(filled_out) if filled_out is not None else None
        _check(load_library().gapd_all_pairs_noalloc(self._h, mode, _dptr(out), ctypes.byref(st)), self._h)
        return out, _stats(st)

    def all_pairs_spiral(self, draws, h: int = 0, out=None, sources_out=None, filled_out=None,
                         time_kernels: bool = False):
        """The spiral method (h <= 1) or the spiral method with repulsion h (the
        paper's is 3).  draws: N uniform uint32 (any array; copied to the device)."""
        import torch
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.int32, device="cuda")
        d = draws if isinstance(draws, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(draws, dtype=np.uint32).view(np.int32))
        d = d.to(device="cuda").contiguous()
        if d.numel() < self.N or d.element_size() != 4:
            raise ValueError("draws must hold N 32-bit values")
        self._ensure_workspace(MODE_TREE_FILL_SPIRAL)
        st = Stats()
        st.sources_out = _dptr(sources_out) if sources_out is not None else None
        st.filled_out = _dptr(filled_out) if filled_out is not None else None
        st.time_kernels = 1 if time_kernels else 0
        _check(load_library().gapd_all_pairs_spiral(self._h, int(h), _dptr(d), _dptr(out), ctypes.byref(st)),
               self._h)
        return out, _stats(st)


def _stats(st) -> "AllPairsStats":
    return AllPairsStats(st.n_prop, st.n_prop_setup, st.rounds, st.centroid, st.ms_total, st.ms_setup,
                         st.ms_kernel, st.ms_step_kernels, st.ms_fill_kernels, st.n_prop_speculative,
                         st.n_cache_hits, st.graph_replays, st.rounds_speculative)


def batched_workspace_size(shapes, C: int = 1, conn: int = CONN4, mode: int = MODE_NAIVE) -> int:
    H = np.ascontiguousarray([s[0] for s in shapes], dtype=np.int32)
    W = np.ascontiguousarray([s[1] for s in shapes], dtype=np.int32)
    n = ctypes.c_size_t()
    _check(load_library().gapd_batched_workspace_size(H.ctypes.data, W.ctypes.data, len(shapes), C, conn, mode,
                                                      ctypes.byref(n)))
    return n.value


def pack_offsets(shapes):
    """int64 element offsets of each image's N x N block in one packed output."""
    sizes = [int(h) * int(w) for h, w in shapes]
    return np.concatenate([[0], np.cumsum([n * n for n in sizes])]).astype(np.int64)


def all_pairs_batched(images, mode: int = MODE_NAIVE, conn: int = CONN4, weight_mode: int | None = None,
                      out=None, offsets=None, workspace=None, stream=None, sources_out=None):
    """All-pairs arrays of many images in one call.  Returns (out, offsets, n_prop).
    sources_out (tree modes, optional): a device int32 tensor of sum(N_b)
    elements that receives image b's source sequence from sum(N_0..N_b-1) on."""
    import torch
    imgs = [_img_arr(im) for im in images]
    C = imgs[0][3]
    if any(c != C for _, _, _, c in imgs):
        raise ValueError("all images of a batch must have the same number of bands")
    wmode = (W_SUM if C == 1 else W_1PL1) if weight_mode is None else weight_mode
    shapes = [(h, w) for _, h, w, _ in imgs]
    B = len(imgs)
    H = np.ascontiguousarray([s[0] for s in shapes], dtype=np.int32)
    W = np.ascontiguousarray([s[1] for s in shapes], dtype=np.int32)
    packed = np.ascontiguousarray(np.concatenate([a.reshape(-1) for a, _, _, _ in imgs]))
    if offsets is None:
        offsets = pack_offsets(shapes)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    if out is None:
        out = torch.empty(int(offsets[-1]), dtype=torch.int32, device="cuda")
    need = batched_workspace_size(shapes, C, conn, mode)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    nprop = np.zeros(B, dtype=np.int64)
    _check(load_library().gapd_all_pairs_batched(packed.ctypes.data, H.ctypes.data, W.ctypes.data, B, C, conn, wmode,
                                                 mode, _dptr(out), offsets.ctypes.data, nprop.ctypes.data,
                                                 _dptr(sources_out) if sources_out is not None else None,
                                                 _dptr(workspace), workspace.numel(), _stream_ptr(stream)))
    return out, offsets, nprop


class Server:
    """Continuous-batching server over a caller-owned device arena."""

    def __init__(self, arena_bytes: int, max_slots: int = 4, arena=None):
        import torch
        self.arena = arena if arena is not None else torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
        # the server's streams do not wait for work queued on the arena
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(load_library().gapd_server_create(_dptr(self.arena), self.arena.numel(), max_slots, ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit_all_pairs(self, image, mode: int = MODE_NAIVE, conn: int = CONN4, weight_mode: int | None = None) -> int:
        img, H, W, C = _img_arr(image)
        wmode = (W_SUM if C == 1 else W_1PL1) if weight_mode is None else weight_mode
        job = Job(JOB_ALL_PAIRS, H, W, C, conn, wmode, mode, img.ctypes.data, None, 0)
        t = ctypes.c_uint64()
        _check(load_library().gapd_serve_submit(self._h, ctypes.byref(job), ctypes.byref(t)))
        return t.value

    def submit_multi_source(self, image, sources, conn: int = CONN4, weight_mode: int | None = None) -> int:
        img, H, W, C = _img_arr(image)
        wmode = (W_SUM if C == 1 else W_1PL1) if weight_mode is None else weight_mode
        src = np.ascontiguousarray(sources, dtype=np.int32)
        job = Job(JOB_MULTI_SOURCE, H, W, C, conn, wmode, MODE_NAIVE, img.ctypes.data, src.ctypes.data, src.size)
        t = ctypes.c_uint64()
        _check(load_library().gapd_serve_submit(self._h, ctypes.byref(job), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        r = Result()
        st = load_library().gapd_serve_poll(self._h, ticket, ctypes.byref(r))
        if st == PENDING:
            return None
        _check(st)
        return r

    def wait(self, ticket: int):
        r = Result()
        _check(load_library().gapd_serve_wait(self._h, ticket, ctypes.byref(r)))
        return r

    def result_tensor(self, res: Result):
        """A torch view of a finished job's result inside the arena (valid until release)."""
        import torch
        base = _dptr(self.arena)
        off = (res.dev_out - base) // 4
        return self.arena.view(torch.int32)[off: off + res.elems]

    def release(self, ticket: int):
        _check(load_library().gapd_serve_release(self._h, ticket))

    def close(self):
        if getattr(self, "_h", None):
            load_library().gapd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A general undirected graph in CSR form on the device (gapd_graph_create).

    row_ptr (n+1 int64), col_idx and weight (int32) describe both directions of
    every edge; boundary (n flags) is optional (default: degree below the
    average)."""

    def __init__(self, row_ptr, col_idx, weight, boundary=None, stream=None):
        lib = load_library()
        self._rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self._ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        self._cw = np.ascontiguousarray(weight, dtype=np.int32)
        self._bnd = None if boundary is None else np.ascontiguousarray(boundary, dtype=np.uint8)
        self.n = self._rp.size - 1
        h = ctypes.c_void_p()
        st = lib.gapd_graph_create(self.n, self._rp.ctypes.data, self._ci.ctypes.data, self._cw.ctypes.data,
                                   None if self._bnd is None else self._bnd.ctypes.data, ctypes.byref(h))
        if st != OK:
            raise GapdError(st, f"{strerror(st)}: {lib.gapd_graph_last_error(None).decode()}")
        self._h = h
        self._ws = None
        _gcheck(lib.gapd_graph_set_stream(self._h, _stream_ptr(stream)), self._h)

    def close(self):
        if getattr(self, "_h", None):
            load_library().gapd_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ensure_workspace(self, mode: int):
        import torch
        n = ctypes.c_size_t()
        _gcheck(load_library().gapd_graph_workspace_size(self._h, mode, ctypes.byref(n)), self._h)
        if n.value == 0:
            return
        if self._ws is None or self._ws.numel() < n.value:
            self._ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        _gcheck(load_library().gapd_graph_set_workspace(self._h, _dptr(self._ws), self._ws.numel()), self._h)

    def sssp(self, sources, out=None):
        import torch
        src = sources if isinstance(sources, torch.Tensor) else torch.as_tensor(np.asarray(sources, np.int32))
        src = src.to(device="cuda", dtype=torch.int32).contiguous()
        K = src.numel()
        if out is None:
            out = torch.empty((K, self.n), dtype=torch.int32, device="cuda")
        _gcheck(load_library().gapd_graph_sssp(self._h, _dptr(src), K, _dptr(out)), self._h)
        return out

    def all_pairs(self, mode: int = MODE_NAIVE, out=None, sources_out=None, filled_out=None,
                  time_kernels: bool = False):
        import torch
        if out is None:
            out = torch.empty((self.n, self.n), dtype=torch.int32, device="cuda")
        self._ensure_workspace(mode)
        st = Stats()
        st.sources_out = _dptr(sources_out) if sources_out is not None else None
        st.filled_out = _dptr(filled_out) if filled_out is not None else None
        st.time_kernels = 1 if time_kernels else 0
        _gcheck(load_library().gapd_graph_all_pairs(self._h, mode, _dptr(out), ctypes.byref(st)), self._h)
        return out, _stats(st)


def _gcheck(status: int, h):
    if status not in (OK, PENDING):
        raise GapdError(status, f"{strerror(status)}: {load_library().gapd_graph_last_error(h).decode()}")
