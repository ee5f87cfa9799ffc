"""CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product code never does.

Thin ctypes wrapper around ``liboracle.so`` (built from ``oracle.c`` with gcc
and OpenMP).  Inputs are canonical CSR graphs (see ``graphgen``) and plain
per-vertex numpy vectors; nothing here knows about B2SR tiles except
``b2sr_build``, which writes the format out from its definition (Sec. III).

Parity status: every function here is pinned by ``tests/test_oracle.py``
(brute force on dense adjacency, closed forms, the paper's worked example of
Sec. III-C, and independent scipy routines).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# B2SR_ORACLE_LIB names another build of oracle.c (the sanitizer test's)
_LIB = os.environ.get("B2SR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
UNREACHED = 0xFFFFFFFF

_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                        "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("B2SR_ORACLE_LIB") and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_b2sr_count_tiles.restype = ctypes.c_uint64
        L.orc_b2sr_count_tiles.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_uint32, ctypes.c_int]
        L.orc_b2sr_build.restype = ctypes.c_int
        L.orc_b2sr_build.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_uint32, ctypes.c_int,
                                     _u32p, _u32p, _vp]
        L.orc_spmv_or.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u8p, _vp, ctypes.c_int, _u8p]
        L.orc_spmv_count.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u8p, _vp, ctypes.c_int, _u32p]
        L.orc_spmv_plus.argtypes = [ctypes.c_uint32, _u32p, _u32p, _f64p, _vp, _vp, ctypes.c_int, _f64p]
        L.orc_spmv_min_plus.argtypes = [ctypes.c_uint32, _u32p, _u32p, _f64p, ctypes.c_double,
                                        ctypes.c_int, _vp, ctypes.c_int, _f64p]
        L.orc_spmv_or64.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u64p, _vp, _u64p]
        L.orc_masked_sum.restype = ctypes.c_uint64
        L.orc_masked_sum.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u32p, _u32p, _vp, _vp]
        L.orc_bfs.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_uint32, _u32p]
        L.orc_bfs_multi.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_uint32, _u32p, _u32p]
        L.orc_sssp_unit.restype = ctypes.c_uint32
        L.orc_sssp_unit.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_uint32, _u32p]
        L.orc_cc.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u32p]
        L.orc_pagerank.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_double, ctypes.c_uint32, _f64p]
        L.orc_pagerank_directed.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_double, ctypes.c_uint32, _f64p]
        L.orc_spmv_max.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u64p, _u64p]
        L.orc_eccentricity.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u32p, ctypes.c_uint32, _u32p]
        L.orc_mis.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u64p, _u8p]
        L.orc_mis.restype = ctypes.c_uint32
        L.orc_mis_greedy.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u64p, _u8p]
        L.orc_color.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u64p, _u32p]
        L.orc_color.restype = ctypes.c_uint32
        L.orc_ppr.argtypes = [ctypes.c_uint32, _u32p, _u32p, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint32,
                              _f64p]
        L.orc_sweep_cut.argtypes = [ctypes.c_uint32, _u32p, _u32p, _f32p, _u32p, _u64p]
        L.orc_tc.restype = ctypes.c_uint64
        L.orc_tc.argtypes = [ctypes.c_uint32, _u32p, _u32p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _mask(mask):
    return None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(t: int) -> None:
    lib().orc_set_num_threads(int(t))


# ---- B2SR from its definition -------------------------------------------------

def row_bytes(T: int) -> int:
    """Bytes per bit-row (Table II; T=4 uses half of an unsigned char; T=64
    the unsigned long long packing type of Sec. III-A)."""
    return {4: 1, 8: 1, 16: 2, 32: 4, 64: 8}[T]


def b2sr_count_tiles(g, T: int, lower_only: bool = False) -> int:
    return int(lib().orc_b2sr_count_tiles(g.n, g.rowptr, g.colind, T, int(lower_only)))


def b2sr_build(g, T: int, lower_only: bool = False):
    """Returns (tile_rowptr u32[nTR+1], tile_colind u32[nT], bits) with bits as
    u8/u8/u16/u32/u64 words for T = 4/8/16/32/64, T words per tile."""
    ntr = (g.n + T - 1) // T
    nt = b2sr_count_tiles(g, T, lower_only)
    trp = np.zeros(ntr + 1, dtype=np.uint32)
    tci = np.zeros(max(nt, 1), dtype=np.uint32)
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}[row_bytes(T)]
    bits = np.zeros(max(nt * T, 1), dtype=dt)
    rc = lib().orc_b2sr_build(g.n, g.rowptr, g.colind, T, int(lower_only), trp, tci, _ptr(bits))
    if rc != 0:
        raise ValueError("bad tile size")
    return trp, tci[:nt], bits[:nt * T]


def b2sr_bytes(ntiles: int, n: int, T: int) -> int:
    """Storage of the three B2SR arrays with 4-byte indices (Sec. III-A/B)."""
    ntr = (n + T - 1) // T
    return 4 * (ntr + 1) + 4 * ntiles + ntiles * T * row_bytes(T)


def csr_bytes(nnz: int, n: int) -> int:
    """Float CSR: 4-byte value + 4-byte column per nonzero, 4-byte row pointer."""
    return 8 * nnz + 4 * (n + 1)


# ---- products -------------------------------------------------------------------

def spmv_or(g, x, mask=None, complement=False):
    y = np.zeros(g.n, dtype=np.uint8)
    lib().orc_spmv_or(g.n, g.rowptr, g.colind, np.ascontiguousarray(x, dtype=np.uint8),
                      _ptr(_mask(mask)), int(complement), y)
    return y.astype(bool)


def spmv_count(g, x, mask=None, complement=False):
    y = np.zeros(g.n, dtype=np.uint32)
    m = _mask(mask)
    lib().orc_spmv_count(g.n, g.rowptr, g.colind, np.ascontiguousarray(x, dtype=np.uint8),
                         _ptr(m), int(complement), y)
    return y


def spmv_plus(g, x, s=None, mask=None, complement=False):
    y = np.zeros(g.n, dtype=np.float64)
    s = None if s is None else np.ascontiguousarray(s, dtype=np.float64)
    m = _mask(mask)
    lib().orc_spmv_plus(g.n, g.rowptr, g.colind, np.ascontiguousarray(x, dtype=np.float64),
                        _ptr(s), _ptr(m), int(complement), y)
    return y


def spmv_min_plus(g, x, w=1.0, self_loop=False, mask=None, complement=False):
    y = np.zeros(g.n, dtype=np.float64)
    m = _mask(mask)
    lib().orc_spmv_min_plus(g.n, g.rowptr, g.colind, np.ascontiguousarray(x, dtype=np.float64),
                            float(w), int(self_loop), _ptr(m), int(complement), y)
    return y


def spmv_or64(g, x, visited=None):
    y = np.zeros(g.n, dtype=np.uint64)
    v = None if visited is None else np.ascontiguousarray(visited, dtype=np.uint64)
    lib().orc_spmv_or64(g.n, g.rowptr, g.colind, np.ascontiguousarray(x, dtype=np.uint64), _ptr(v), y)
    return y


def masked_sum(a, bt, m=None) -> int:
    """sum_{(i,j) in M} (A B)_ij with B given as its transpose Bt."""
    if m is None:
        return int(lib().orc_masked_sum(a.n, a.rowptr, a.colind, bt.rowptr, bt.colind, None, None))
    return int(lib().orc_masked_sum(a.n, a.rowptr, a.colind, bt.rowptr, bt.colind,
                                    _ptr(m.rowptr), _ptr(m.colind)))


# ---- algorithms -------------------------------------------------------------

def bfs(g, src: int):
    lv = np.zeros(g.n, dtype=np.uint32)
    lib().orc_bfs(g.n, g.rowptr, g.colind, int(src), lv)
    return lv


def bfs_multi(g, srcs):
    srcs = np.ascontiguousarray(srcs, dtype=np.uint32)
    out = np.zeros((srcs.size, g.n), dtype=np.uint32)
    lib().orc_bfs_multi(g.n, g.rowptr, g.colind, srcs.size, srcs, out)
    return out


def sssp_unit(g, src: int):
    d = np.zeros(g.n, dtype=np.uint32)
    lib().orc_sssp_unit(g.n, g.rowptr, g.colind, int(src), d)
    return d


def cc(g):
    lab = np.zeros(g.n, dtype=np.uint32)
    lib().orc_cc(g.n, g.rowptr, g.colind, lab)
    return lab


def pagerank(g, d: float = 0.85, iters: int = 20):
    r = np.zeros(g.n, dtype=np.float64)
    lib().orc_pagerank(g.n, g.rowptr, g.colind, float(d), int(iters), r)
    return r


def pagerank_directed(g, d: float = 0.85, iters: int = 20):
    """PageRank of the directed graph whose CSR row u lists the heads of u's arcs."""
    r = np.zeros(g.n, dtype=np.float64)
    lib().orc_pagerank_directed(g.n, g.rowptr, g.colind, float(d), int(iters), r)
    return r


def spmv_max(g, x):
    y = np.zeros(g.n, dtype=np.uint64)
    lib().orc_spmv_max(g.n, g.rowptr, g.colind, np.ascontiguousarray(x, dtype=np.uint64), y)
    return y


def mis(g, key):
    """(membership bool array, rounds) of the local-maxima independent set."""
    out = np.zeros(g.n, dtype=np.uint8)
    r = lib().orc_mis(g.n, g.rowptr, g.colind, np.ascontiguousarray(key, dtype=np.uint64), out)
    return out.astype(bool), int(r)


def mis_greedy(g, key):
    out = np.zeros(g.n, dtype=np.uint8)
    lib().orc_mis_greedy(g.n, g.rowptr, g.colind, np.ascontiguousarray(key, dtype=np.uint64), out)
    return out.astype(bool)


def color(g, key):
    """(colour per vertex, number of colours) by successive independent sets."""
    out = np.zeros(g.n, dtype=np.uint32)
    c = lib().orc_color(g.n, g.rowptr, g.colind, np.ascontiguousarray(key, dtype=np.uint64), out)
    return out, int(c)


def eccentricity(g, srcs):
    srcs = np.ascontiguousarray(srcs, dtype=np.uint32)
    out = np.zeros(srcs.size, dtype=np.uint32)
    lib().orc_eccentricity(g.n, g.rowptr, g.colind, srcs, srcs.size, out)
    return out


def diameter(g) -> int:
    """The largest finite distance: the largest eccentricity over every vertex."""
    return int(eccentricity(g, np.arange(g.n)).max(initial=0))


def ppr(g, seed: int, a: float = 0.85, iters: int = 20):
    """Personalised PageRank from one seed (float64), see orc_ppr."""
    p = np.zeros(g.n, dtype=np.float64)
    lib().orc_ppr(g.n, g.rowptr, g.colind, int(seed), float(a), int(iters), p)
    return p


def sweep_cut(g, score):
    """Sweep cut of a score vector (single-precision quotients), see
    orc_sweep_cut.  Returns (order u32[n], stats dict)."""
    score = np.ascontiguousarray(score, dtype=np.float32)
    order = np.zeros(g.n, dtype=np.uint32)
    st = np.zeros(5, dtype=np.uint64)
    lib().orc_sweep_cut(g.n, g.rowptr, g.colind, score, order, st)
    return order, sweep_stats(st)


def sweep_stats(st) -> dict:
    k, cut, vol, vol_all, taken = (int(v) for v in st)
    den = min(vol, vol_all - vol)
    return {"size": k, "cut": cut, "vol": vol, "vol_all": vol_all, "taken": taken,
            "conductance": cut / den if den else None}


def lgc(g, seed: int, a: float = 0.85, iters: int = 20):
    """Local clustering around seed: personalised PageRank, then the sweep cut
    of its single-precision rounding.  Returns (p float64, cluster bool[n],
    stats)."""
    p = ppr(g, seed, a, iters)
    order, st = sweep_cut(g, p.astype(np.float32))
    cluster = np.zeros(g.n, dtype=bool)
    cluster[order[:st["size"]]] = True
    return p, cluster, st


def tc(g) -> int:
    return int(lib().orc_tc(g.n, g.rowptr, g.colind))


def tril(g):
    """Strictly lower triangle L of a CSR (j < i) as a CSR-like object."""
    from graphgen import Csr
    rows = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    keep = g.colind.astype(np.int64) < rows
    counts = np.bincount(rows[keep], minlength=g.n)
    rp = np.zeros(g.n + 1, dtype=np.uint32)
    np.cumsum(counts, out=rp[1:])
    return Csr(g.n, rp, g.colind[keep].copy(), name=g.name + "_L")
