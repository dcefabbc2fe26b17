"""CPU oracle for all pairs of geodesic distances -- TEST INFRASTRUCTURE ONLY.

This package wraps ``gapd_oracle.c``, a plain C implementation of what the
GPU library computes, written from the paper (Noyel, Angulo, Jeulin, "Fast
computation of all pairs of geodesic distances"): Dijkstra propagations,
Floyd-Warshall for tiny images, the naive method, the geodesic centroid and
extrema list, the filling-rate method with its redundancy fill, and with the
same fill the geodesic extrema method and the spiral methods (with their
random draws passed in), and the propagation, fill and deterministic
selection rules on general graphs in CSR form.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import it.  It shares no code with the GPU library and never imports it;
the GPU library never imports this package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gapd_oracle.c")
_LIB = os.environ.get("GAPD_ORACLE_LIB") or os.path.join(_HERE, "libgapd_oracle.so")

W_SUM = 0
W_1PL1 = 1
TRUNCATED = 2

_lib = None


def build(force: bool = True, out: str = None, mutant: int = 0) -> str:
    """Compile the oracle with gcc (plain -O3, portable code, OpenMP).

    ``mutant`` > 0 plants one of the deliberate mistakes of ``gapd_oracle.c``
    (used only by the test that checks the pins reject them)."""
    out = out or _LIB
    if force or not os.path.exists(out):
        cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               f"-DORACLE_MUTANT={int(mutant)}", "-o", out + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        sigs = {
            "gapd_oracle_dijkstra": [P, i32, i32, i32, i32, i32, P, i64, P],
            "gapd_oracle_floyd": [P, i32, i32, i32, i32, i32, P],
            "gapd_oracle_rows": [P, i32, i32, i32, i32, i32, P, i64, P, i32],
            "gapd_oracle_naive": [P, i32, i32, i32, i32, i32, P, i32],
            "gapd_oracle_parents": [P, i32, i32, i32, i32, i32, P, P],
            "gapd_oracle_extrema": [P, i32, i32, i32, i32, i32, P, P, P, P],
            "gapd_oracle_filling_rate": [P, i32, i32, i32, i32, i32, P, P, P, P, P, P, i64],
            "gapd_oracle_extrema_method": [P, i32, i32, i32, i32, i32, P, P, P, P, P, i64],
            "gapd_oracle_spiral": [P, i32, i32, i32, i32, i32, i32, P, i64, P, P, P, P, i64],
            "gapd_oracle_spiral_turn": [i32, i32, i32, P, P],
            "gapd_oracle_graph_boundary": [i64, P, P],
            "gapd_oracle_graph_dijkstra": [i64, P, P, P, P, i64, P],
            "gapd_oracle_graph_parents": [i64, P, P, P, P, P],
            "gapd_oracle_graph_rows": [i64, P, P, P, P, i64, P, i32],
            "gapd_oracle_graph_extrema": [i64, P, P, P, P, P, P, P, P],
            "gapd_oracle_graph_tree_method": [i64, P, P, P, P, i32, P, P, P, P, P, P, i64],
        }
        for name, args in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _img(image: np.ndarray):
    image = np.ascontiguousarray(image, dtype=np.uint8)
    if image.ndim == 2:
        H, W = image.shape
        C = 1
    elif image.ndim == 3:
        H, W, C = image.shape
    else:
        raise ValueError("image must be (H, W) or (H, W, C)")
    return image, H, W, C


def _check(st: int, name: str):
    if st not in (0, TRUNCATED):
        raise RuntimeError(f"{name} failed with status {st}")
    return st


def default_wmode(image: np.ndarray) -> int:
    return W_SUM if (image.ndim == 2 or image.shape[2] == 1) else W_1PL1


def dijkstra(image, seeds, conn=4, wmode=None) -> np.ndarray:
    """Distances (int64, length N) from the seed pixels (all at distance 0)."""
    image, H, W, C = _img(image)
    wmode = default_wmode(image) if wmode is None else wmode
    seeds = np.ascontiguousarray(np.atleast_1d(seeds), dtype=np.int64)
    out = np.empty(H * W, dtype=np.int64)
    _check(_load().gapd_oracle_dijkstra(_ptr(image), H, W, C, conn, wmode, _ptr(seeds), seeds.size,
                                        _ptr(out)), "dijkstra")
    return out


def floyd(image, conn=4, wmode=None) -> np.ndarray:
    """All-pairs distances (int64 N x N) by Floyd-Warshall; N <= 1024."""
    image, H, W, C = _img(image)
    wmode = default_wmode(image) if wmode is None else wmode
    out = np.empty((H * W, H * W), dtype=np.int64)
    _check(_load().gapd_oracle_floyd(_ptr(image), H, W, C, conn, wmode, _ptr(out)), "floyd")
    return out


def rows(image, sources, conn=4, wmode=None, threads=None) -> np.ndarray:
    """Distance rows (int32, K x N) for the given sources."""
    image, H, W, C = _img(image)
    wmode = default_wmode(image) if wmode is None else wmode
    src = np.ascontiguousarray(np.atleast_1d(sources), dtype=np.int32)
    out = np.empty((src.size, H * W), dtype=np.int32)
    threads = threads or os.cpu_count() or 1
    _check(_load().gapd_oracle_rows(_ptr(image), H, W, C, conn, wmode, _ptr(src), src.size, _ptr(out),
                                    threads), "rows")
    return out


def naive(image, conn=4, wmode=None, threads=None) -> np.ndarray:
    """The naive method: the full N x N int32 distances array."""
    image, H, W, C = _img(image)
    wmode = default_wmode(image) if wmode is None else wmode
    out = np.empty((H * W, H * W), dtype=np.int32)
    threads = threads or os.cpu_count() or 1
    _check(_load().gapd_oracle_naive(_ptr(image), H, W, C, conn, wmode, _ptr(out), threads), "naive")
    return out


def parents(image, dist, conn=4, wmode=None) -> np.ndarray:
    """Canonical geodesic-tree parents (int32, -1 at the root) from final distances."""
    image, H, W, C = _img(image)
    wmode = default_wmode(image) if wmode is None else wmode
    dist = np.ascontiguousarray(dist, dtype=np.int64)
    out = np.empty(H * W, dtype=np.int32)
    _check(_load().gapd_oracle_parents(_ptr(image), H, W, C, conn, wmode, _ptr(dist), _ptr(out)), "parents")
    return out


@dataclass
class Extrema:
    centroid: int
    d_edge: np.ndarray
    d_c: np.ndarray
    rank: np.ndarray


def extrema(image, conn=4, wmode=None) -> Extrema:
    """Geodesic centroid, the two setup propagations and the extrema ranks."""
    image, H, W, C = _img(image)
    wmode = default_wmode(image) if wmode is None else wmode
    N = H * W
    c = np.zeros(1, dtype=np.int32)
    de = np.empty(N, dtype=np.int64)
    dc = np.empty(N, dtype=np.int64)
    rk = np.empty(N, dtype=np.int32)
    _check(_load().gapd_oracle_extrema(_ptr(image), H, W, C, conn, wmode, _ptr(c), _ptr(de), _ptr(dc),
                                       _ptr(rk)), "extrema")
    return Extrema(int(c[0]), de, dc, rk)


@dataclass
class FillingRate:
    D: np.ndarray            # N x N int32 (partly written if truncated)
    sequence: np.ndarray     # sources, one per propagation
    filled: np.ndarray       # a(t): filled pairs after each propagation
    n_prop: int              # propagations in the loop (setup's 2 not included)
    centroid: int
    rank: np.ndarray
    truncated: bool


def filling_rate(image, conn=4, wmode=None, max_steps: int = -1) -> FillingRate:
    """The filling-rate method; ``max_steps`` bounds the loop (for timing samples)."""
    image, H, W, C = _img(image)
    wmode = default_wmode(image) if wmode is None else wmode
    N = H * W
    D = np.full((N, N), -1, dtype=np.int32)
    seq = np.full(N, -1, dtype=np.int32)
    a = np.zeros(N, dtype=np.int64)
    n = np.zeros(1, dtype=np.int64)
    c = np.zeros(1, dtype=np.int32)
    rk = np.empty(N, dtype=np.int32)
    st = _check(_load().gapd_oracle_filling_rate(_ptr(image), H, W, C, conn, wmode, _ptr(D), _ptr(seq), _ptr(a),
                                                 _ptr(n), _ptr(c), _ptr(rk), int(max_steps)), "filling_rate")
    k = int(n[0])
    return FillingRate(D, seq[:k].copy(), a[:k].copy(), k, int(c[0]), rk, st == TRUNCATED)


@dataclass
class TreeMethod:
    D: np.ndarray            # N x N int32 (partly written if truncated)
    sequence: np.ndarray     # sources, one per propagation
    filled: np.ndarray       # a(t): filled pairs after each propagation
    n_prop: int              # propagations in the loop (setup not included)
    centroid: int            # -1 for the spiral methods
    truncated: bool


def extrema_method(image, conn=4, wmode=None, max_steps: int = -1) -> TreeMethod:
    """The geodesic extrema method (two setup propagations, then the farthest
    unfilled point from the centroid, least filled among ties)."""
    image, H, W, C = _img(image)
    wmode = default_wmode(image) if wmode is None else wmode
    N = H * W
    D = np.full((N, N), -1, dtype=np.int32)
    seq = np.full(N, -1, dtype=np.int32)
    a = np.zeros(N, dtype=np.int64)
    n = np.zeros(1, dtype=np.int64)
    c = np.zeros(1, dtype=np.int32)
    st = _check(_load().gapd_oracle_extrema_method(_ptr(image), H, W, C, conn, wmode, _ptr(D), _ptr(seq), _ptr(a),
                                                   _ptr(n), _ptr(c), int(max_steps)), "extrema_method")
    k = int(n[0])
    return TreeMethod(D, seq[:k].copy(), a[:k].copy(), k, int(c[0]), st == TRUNCATED)


def spiral(image, rnd, h: int = 0, conn=4, wmode=None, max_steps: int = -1) -> TreeMethod:
    """The spiral method (h <= 1) or the spiral method with repulsion h (the
    paper's is 3); ``rnd`` holds the uniform uint32 draws, one per propagation."""
    image, H, W, C = _img(image)
    wmode = default_wmode(image) if wmode is None else wmode
    N = H * W
    rnd = np.ascontiguousarray(rnd, dtype=np.uint32)
    D = np.full((N, N), -1, dtype=np.int32)
    seq = np.full(N, -1, dtype=np.int32)
    a = np.zeros(N, dtype=np.int64)
    n = np.zeros(1, dtype=np.int64)
    st = _check(_load().gapd_oracle_spiral(_ptr(image), H, W, C, conn, wmode, int(h), _ptr(rnd), rnd.size,
                                           _ptr(D), _ptr(seq), _ptr(a), _ptr(n), int(max_steps)), "spiral")
    k = int(n[0])
    return TreeMethod(D, seq[:k].copy(), a[:k].copy(), k, -1, st == TRUNCATED)


def spiral_turn(H: int, W: int, k: int):
    """Pixels of spiral turn k in turn order, and whether the turn is a closed frame."""
    out = np.empty(2 * (H + W) + 4, dtype=np.int32)
    cyc = np.zeros(1, dtype=np.int32)
    n = _load().gapd_oracle_spiral_turn(H, W, k, _ptr(out), _ptr(cyc))
    return out[:n].copy(), bool(cyc[0])


# ---- general graphs (CSR) ------------------------------------------------------------------

def _csr(rp, ci, cw):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    cw = np.ascontiguousarray(cw, dtype=np.int32)
    return rp.size - 1, rp, ci, cw


def _bnd(b):
    return None if b is None else np.ascontiguousarray(b, dtype=np.uint8)


def graph_boundary(rp) -> np.ndarray:
    """Boundary flags by the degree rule (degree below the average; all if none)."""
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    out = np.zeros(rp.size - 1, dtype=np.uint8)
    _check(_load().gapd_oracle_graph_boundary(rp.size - 1, _ptr(rp), _ptr(out)), "graph_boundary")
    return out


def graph_dijkstra(rp, ci, cw, seeds) -> np.ndarray:
    n, rp, ci, cw = _csr(rp, ci, cw)
    seeds = np.ascontiguousarray(np.atleast_1d(seeds), dtype=np.int64)
    out = np.empty(n, dtype=np.int64)
    _check(_load().gapd_oracle_graph_dijkstra(n, _ptr(rp), _ptr(ci), _ptr(cw), _ptr(seeds), seeds.size, _ptr(out)),
           "graph_dijkstra")
    return out


def graph_parents(rp, ci, cw, dist) -> np.ndarray:
    n, rp, ci, cw = _csr(rp, ci, cw)
    dist = np.ascontiguousarray(dist, dtype=np.int64)
    out = np.empty(n, dtype=np.int32)
    _check(_load().gapd_oracle_graph_parents(n, _ptr(rp), _ptr(ci), _ptr(cw), _ptr(dist), _ptr(out)),
           "graph_parents")
    return out


def graph_rows(rp, ci, cw, sources, threads=None) -> np.ndarray:
    n, rp, ci, cw = _csr(rp, ci, cw)
    src = np.ascontiguousarray(np.atleast_1d(sources), dtype=np.int32)
    out = np.empty((src.size, n), dtype=np.int32)
    _check(_load().gapd_oracle_graph_rows(n, _ptr(rp), _ptr(ci), _ptr(cw), _ptr(src), src.size, _ptr(out),
                                          threads or os.cpu_count() or 1), "graph_rows")
    return out


def graph_naive(rp, ci, cw, threads=None) -> np.ndarray:
    n = np.asarray(rp).size - 1
    return graph_rows(rp, ci, cw, np.arange(n, dtype=np.int32), threads)


def graph_extrema(rp, ci, cw, boundary=None) -> Extrema:
    n, rp, ci, cw = _csr(rp, ci, cw)
    b = _bnd(boundary)
    c = np.zeros(1, dtype=np.int32)
    de = np.empty(n, dtype=np.int64)
    dc = np.empty(n, dtype=np.int64)
    rk = np.empty(n, dtype=np.int32)
    _check(_load().gapd_oracle_graph_extrema(n, _ptr(rp), _ptr(ci), _ptr(cw), None if b is None else _ptr(b),
                                             _ptr(c), _ptr(de), _ptr(dc), _ptr(rk)), "graph_extrema")
    return Extrema(int(c[0]), de, dc, rk)


def graph_tree_method(rp, ci, cw, rule: int = 0, boundary=None, max_steps: int = -1) -> FillingRate:
    """rule 0: filling rate; rule 1: geodesic extrema method."""
    n, rp, ci, cw = _csr(rp, ci, cw)
    b = _bnd(boundary)
    D = np.full((n, n), -1, dtype=np.int32)
    seq = np.full(n, -1, dtype=np.int32)
    a = np.zeros(n, dtype=np.int64)
    k = np.zeros(1, dtype=np.int64)
    c = np.zeros(1, dtype=np.int32)
    rk = np.empty(n, dtype=np.int32)
    st = _check(_load().gapd_oracle_graph_tree_method(n, _ptr(rp), _ptr(ci), _ptr(cw),
                                                      None if b is None else _ptr(b), int(rule), _ptr(D),
                                                      _ptr(seq), _ptr(a), _ptr(k), _ptr(c), _ptr(rk),
                                                      int(max_steps)), "graph_tree_method")
    m = int(k[0])
    return FillingRate(D, seq[:m].copy(), a[:m].copy(), m, int(c[0]), rk, st == TRUNCATED)
