"""Python binding of libb2sr.so: B2SR bit-tiled graphs and bit-level GraphBLAS
kernels on AMD Instinct MI355X (gfx950).

This module only marshals arguments: every step runs in the HIP kernels of
``libb2sr.so`` (declared in ``include/b2sr.h``).  PyTorch provides device
memory and the current stream.  The functions carry the C ABI's names.

Integer vectors cross the boundary as int32/int64 tensors whose bits are the
ABI's uint32/uint64 values (``as_u32``/``as_u64`` reinterpret them on the host).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

__all__ = [
    "B2SRError", "B2SR", "lib", "b2sr_count_tiles", "b2sr_from_csr", "b2sr_pack_bits", "spmv_bin_bin",
    "spmv_bin_full", "spmv_bin_full_workspace_bytes", "spmv_bin_full_noalloc", "spgemm_masked", "spgemm_masked_workspace_bytes",
    "spgemm_masked_profile", "spgemm_masked_rows", "b2sr_pagerank_directed", "b2sr_csr_transpose", "b2sr_mis", "b2sr_color",
    "mis_keys", "b2sr_eccentricity", "b2sr_diameter",
    "b2sr_algo_workspace_bytes", "b2sr_bfs", "b2sr_msbfs", "b2sr_sssp", "b2sr_cc", "b2sr_pagerank",
    "triangle_count", "b2sr_strerror", "as_u32", "as_u64", "header_functions", "FLAGS", "SEMIRINGS",
    "b2sr_msbfs_batch", "b2sr_msbfs_batch_workspace_bytes", "b2sr_msbfs_batch_timed", "MsbfsPlan", "BfsSession",
    "b2sr_bfs_session_bytes", "b2sr_lgc", "b2sr_sweep_cut",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
# B2SR_LIB names another build of the same sources (the sanitizer test's host-instrumented one)
LIB_PATH = os.environ.get("B2SR_LIB") or os.path.join(_HERE, "libb2sr.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "b2sr.h")

# flags and semirings (values from include/b2sr.h)
BUILD_LOWER = 0x1
MASK_COMPLEMENT = 0x1
OUT_COUNT = 0x2
ACCUMULATE = 0x4
SELF = 0x8
SPARSE_X = 0x10
PLUS_TIMES_F32, MIN_PLUS_F32, MIN_PLUS_U32, OR_U64, MAX_TIMES_U64 = 1, 2, 3, 4, 5
ALGO_BFS, ALGO_SSSP, ALGO_CC, ALGO_PAGERANK, ALGO_MSBFS, ALGO_MIS, ALGO_COLOR, ALGO_ECC = 1, 2, 3, 4, 5, 6, 7, 8
ALGO_LGC = 9
BATCH_LEVELS, BATCH_PERSISTENT = 0, 1
FLAGS = {"BUILD_LOWER": BUILD_LOWER, "MASK_COMPLEMENT": MASK_COMPLEMENT, "OUT_COUNT": OUT_COUNT,
         "ACCUMULATE": ACCUMULATE, "SELF": SELF, "SPARSE_X": SPARSE_X}
SEMIRINGS = {"plus_times_f32": PLUS_TIMES_F32, "min_plus_f32": MIN_PLUS_F32, "min_plus_u32": MIN_PLUS_U32,
             "or_u64": OR_U64, "max_times_u64": MAX_TIMES_U64}
UNREACHED = 0xFFFFFFFF


class B2SRError(RuntimeError):
    def __init__(self, status: int, where: str):
        text = _lib.b2sr_strerror(status).decode() if _lib is not None else str(status)
        extra = _lib.b2sr_last_hip_error().decode() if (_lib is not None and status == -4) else ""
        super().__init__(f"{where}: {text} ({status}){': ' + extra if extra else ''}")
        self.status = status


class b2sr_matrix(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("tile", ctypes.c_uint32), ("ntiles", ctypes.c_uint32),
                ("chunk_blocks", ctypes.c_uint32), ("tile_rowptr", ctypes.c_void_p),
                ("tile_colind", ctypes.c_void_p), ("bits", ctypes.c_void_p)]


_lib = None
_P = ctypes.c_void_p
_MP = ctypes.POINTER(b2sr_matrix)
_U32, _U64, _I, _D, _SZ = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t

_SIGS = {
    "b2sr_strerror": (ctypes.c_char_p, [_I]),
    "b2sr_last_hip_error": (ctypes.c_char_p, []),
    "b2sr_version": (_I, []),
    "b2sr_count_tiles": (_I, [_U32, _U64, _P, _P, _U32, ctypes.c_uint, _P, ctypes.POINTER(_U64), _P]),
    "b2sr_from_csr": (_I, [_U32, _U64, _P, _P, _U32, ctypes.c_uint, _P, _U64, _P, _P, _P]),
    "b2sr_pack_bits": (_I, [_U32, _P, _P, _P]),
    "spmv_bin_bin": (_I, [_MP, _P, _P, ctypes.c_uint, _P, _P]),
    "spmv_bin_full_workspace_bytes": (_SZ, [_MP, _I]),
    "spmv_bin_full": (_I, [_MP, _I, _P, _P, _P, _P, ctypes.c_uint, _D, _D, _P, _P, _SZ, _P]),
    "spmv_bin_full_noalloc": (_I, [_MP, _I, _P, _P, _P, _P, ctypes.c_uint, _D, _D, _P, _P]),
    "spgemm_masked_workspace_bytes": (_SZ, [_MP, _MP]),
    "spgemm_masked": (_I, [_MP, _MP, _MP, ctypes.c_uint, _P, _P, _SZ, _P]),
    "spgemm_masked_profile": (_I, [_MP, _MP, _MP, _P, _P]),
    "spgemm_masked_rows": (_I, [_MP, _MP, _MP, _U32, _U32, ctypes.c_uint, _P, _P]),
    "b2sr_algo_workspace_bytes": (_SZ, [_MP, _I]),
    "b2sr_bfs": (_I, [_MP, _U32, _P, _P, _SZ, ctypes.POINTER(_U32), _P]),
    "b2sr_msbfs": (_I, [_MP, ctypes.POINTER(_U32), _U32, _P, _P, _SZ, ctypes.POINTER(_U32), _P]),
    "b2sr_sssp": (_I, [_MP, _U32, _P, _P, _SZ, ctypes.POINTER(_U32), _P]),
    "b2sr_cc": (_I, [_MP, _P, _P, _SZ, ctypes.POINTER(_U32), _P]),
    "b2sr_pagerank": (_I, [_MP, ctypes.c_float, _U32, _P, _P, _SZ, _P]),
    "b2sr_pagerank_directed": (_I, [_MP, ctypes.c_float, _U32, _P, _P, _SZ, _P]),
    "b2sr_mis": (_I, [_MP, _P, _P, _P, _SZ, ctypes.POINTER(_U32), _P]),
    "b2sr_stream_read": (_I, [_P, _SZ, _P, _P]),
    "b2sr_eccentricity": (_I, [_MP, _P, _U32, _P, _P, _SZ, _P]),
    "b2sr_diameter": (_I, [_MP, ctypes.POINTER(_U32), _P, _SZ, _P]),
    "b2sr_color": (_I, [_MP, _P, _P, _P, _SZ, ctypes.POINTER(_U32), _P]),
    "b2sr_lgc": (_I, [_MP, _U32, ctypes.c_float, _U32, _P, _P, _P, _P, _SZ, _P]),
    "b2sr_sweep_cut": (_I, [_MP, _P, _P, _P, _P, _P, _SZ, _P]),
    "b2sr_csr_transpose_workspace_bytes": (_SZ, [_U32]),
    "b2sr_csr_transpose": (_I, [_U32, _U64, _P, _P, _P, _P, _P, _SZ, _P]),
    "b2sr_msbfs_batch_workspace_bytes": (_SZ, [_U32]),
    "b2sr_msbfs_batch": (_I, [_U32, _U32, _MP, _U32, _P, _P, _P, ctypes.c_uint, _P, _SZ, ctypes.POINTER(_U32), _P]),
    "b2sr_msbfs_batch_timed": (_I, [_U32, _U32, _MP, _U32, _P, _P, _P, _P, _SZ, _P, _U32, _U32,
                                    ctypes.POINTER(_U32), ctypes.POINTER(_U32), ctypes.POINTER(_U32), _P]),
    "b2sr_msbfs_batch_plan_create": (_I, [_U32, _U32, _MP, _U32, _P, _P, _P, ctypes.c_uint, _P, _SZ,
                                          ctypes.POINTER(_P)]),
    "b2sr_msbfs_batch_plan_launch": (_I, [_P, ctypes.POINTER(_U32), _P]),
    "b2sr_msbfs_batch_plan_status": (_I, [_P, ctypes.POINTER(_U32), _P]),
    "b2sr_msbfs_batch_plan_destroy": (_I, [_P]),
    "b2sr_bfs_session_bytes": (_SZ, [_U32]),
    "b2sr_bfs_session_create": (_I, [_MP, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "b2sr_bfs_session_join": (_I, [_P, _U32, _U32, _P]),
    "b2sr_bfs_session_step": (_I, [_P, _P, _P]),
    "b2sr_bfs_session_extract": (_I, [_P, _U32, _P, _P]),
    "b2sr_bfs_session_info": (_I, [_P, ctypes.POINTER(_U32), ctypes.POINTER(_U64)]),
    "b2sr_bfs_session_destroy": (_I, [_P]),
}


def lib():
    """Loads libb2sr.so; raises when it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(or python paper_2201_08560_amd/build_lib.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of every function declared in include/b2sr.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z][a-z0-9_]*)\s*\(", text)) - {"defined", "sizeof"})


def b2sr_strerror(status: int) -> str:
    return lib().b2sr_strerror(status).decode()


def _check(rc: int, where: str):
    if rc != 0:
        raise B2SRError(rc, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def as_u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def as_u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def _i32(a, device="cuda"):
    """uint32 data (numpy or tensor) as an int32 device tensor with the same bits."""
    if isinstance(a, torch.Tensor):
        return a.to(device)
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(device)


def _words(n: int) -> int:
    return (n + 31) // 32


_ROW_BYTES = {4: 1, 8: 1, 16: 2, 32: 4, 64: 8}


class B2SR:
    """A device-resident B2SR matrix; owns the three arrays as torch tensors."""

    def __init__(self, n: int, tile: int, tile_rowptr, tile_colind, bits, ntiles: int):
        self.n, self.tile, self.ntiles = int(n), int(tile), int(ntiles)
        self.tile_rowptr, self.tile_colind, self.bits = tile_rowptr, tile_colind, bits
        self._view = b2sr_matrix(self.n, self.tile, self.ntiles, 0, tile_rowptr.data_ptr(),
                                 tile_colind.data_ptr(), bits.data_ptr())

    @property
    def view(self):
        return ctypes.byref(self._view)

    @property
    def chunk_blocks(self) -> int:
        """The products' work split (b2sr.h: 0 = the library's choice, else
        1..64 blocks of tiles per wave)."""
        return int(self._view.chunk_blocks)

    @chunk_blocks.setter
    def chunk_blocks(self, k: int):
        if not 0 <= int(k) <= 64:
            raise ValueError("chunk_blocks must be in 0..64")
        self._view.chunk_blocks = int(k)

    def with_split(self, chunk_blocks: int) -> "B2SR":
        """The same arrays (shared, not copied) under another work split."""
        other = B2SR(self.n, self.tile, self.tile_rowptr, self.tile_colind, self.bits, self.ntiles)
        other.chunk_blocks = chunk_blocks
        return other

    @property
    def ntile_rows(self) -> int:
        return (self.n + self.tile - 1) // self.tile

    @property
    def nbytes(self) -> int:
        """Storage of the three arrays with 4-byte indices (Sec. III)."""
        return 4 * (self.ntile_rows + 1) + 4 * self.ntiles + self.ntiles * self.tile * _ROW_BYTES[self.tile]

    @classmethod
    def from_csr(cls, rowptr, colind, n: int, tile: int, lower: bool = False, transpose: bool = False):
        """Builds B2SR on the device from CSR (uint32 numpy arrays or int32 device
        tensors); ``transpose`` builds the transposed matrix (a directed graph's
        pull matrix)."""
        if transpose:
            rowptr, colind = b2sr_csr_transpose(n, rowptr, colind)
        rp, ci = _i32(rowptr), _i32(colind)
        nnz = int(ci.numel())
        flags = BUILD_LOWER if lower else 0
        trp = torch.empty((n + tile - 1) // tile + 1, dtype=torch.int32, device="cuda")
        nt = b2sr_count_tiles(n, nnz, rp, ci, tile, flags, trp)
        tci = torch.empty(max(nt, 1), dtype=torch.int32, device="cuda")
        bits = torch.empty(max(nt * tile * _ROW_BYTES[tile], 16), dtype=torch.uint8, device="cuda")
        b2sr_from_csr(n, nnz, rp, ci, tile, flags, trp, nt, tci, bits)
        return cls(n, tile, trp, tci, bits, nt)

    @classmethod
    def from_graph(cls, g, tile: int, lower: bool = False, transpose: bool = False):
        return cls.from_csr(g.rowptr, g.colind, g.n, tile, lower, transpose)

    def to_host(self):
        """(tile_rowptr u32, tile_colind u32, bits as u8/u8/u16/u32/u64 words)."""
        trp = as_u32(self.tile_rowptr)
        tci = as_u32(self.tile_colind)[: self.ntiles]
        raw = self.bits.cpu().numpy()[: self.ntiles * self.tile * _ROW_BYTES[self.tile]]
        dt = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}[_ROW_BYTES[self.tile]]
        return trp, tci, raw.view(dt)


# ---- format ------------------------------------------------------------------

def b2sr_count_tiles(n, nnz, rowptr, colind, tile, flags, tile_rowptr) -> int:
    out = _U64(0)
    _check(lib().b2sr_count_tiles(n, nnz, _ptr(rowptr), _ptr(colind), tile, flags, _ptr(tile_rowptr),
                                  ctypes.byref(out), _stream()), "b2sr_count_tiles")
    return int(out.value)


def b2sr_from_csr(n, nnz, rowptr, colind, tile, flags, tile_rowptr, ntiles, tile_colind, bits):
    _check(lib().b2sr_from_csr(n, nnz, _ptr(rowptr), _ptr(colind), tile, flags, _ptr(tile_rowptr), ntiles,
                               _ptr(tile_colind), _ptr(bits), _stream()), "b2sr_from_csr")


def b2sr_pack_bits(pred: torch.Tensor, out=None) -> torch.Tensor:
    """Bool/uint8 device vector -> bit vector (int32 words)."""
    n = pred.numel()
    p = pred.to(torch.uint8).contiguous()
    out = torch.empty(max(_words(n), 1), dtype=torch.int32, device="cuda") if out is None else out
    _check(lib().b2sr_pack_bits(n, _ptr(p), _ptr(out), _stream()), "b2sr_pack_bits")
    return out


# ---- products -------------------------------------------------------------------

def spmv_bin_bin(A: B2SR, x, mask=None, complement=False, count=False, accumulate=False, out=None,
                 sparse_x=False):
    flags = (MASK_COMPLEMENT if complement else 0) | (OUT_COUNT if count else 0) | (ACCUMULATE if accumulate else 0)
    flags |= SPARSE_X if sparse_x else 0
    if out is None:
        out = torch.empty(A.n if count else max(_words(A.n), 1), dtype=torch.int32, device="cuda")
    _check(lib().spmv_bin_bin(A.view, _ptr(x), _ptr(mask), flags, _ptr(out), _stream()), "spmv_bin_bin")
    return out


def spmv_bin_full_workspace_bytes(A: B2SR, semiring: int) -> int:
    return int(lib().spmv_bin_full_workspace_bytes(A.view, semiring))


_FULL_DTYPE = {PLUS_TIMES_F32: torch.float32, MIN_PLUS_F32: torch.float32, MIN_PLUS_U32: torch.int32,
               OR_U64: torch.int64, MAX_TIMES_U64: torch.int64}


def spmv_bin_full(A: B2SR, semiring: int, x, col_scale=None, mask=None, complement=False, self_loop=False,
                  accumulate=False, alpha=1.0, beta=0.0, out=None, ws=None, x_active=None):
    flags = (MASK_COMPLEMENT if complement else 0) | (SELF if self_loop else 0) | (ACCUMULATE if accumulate else 0)
    if out is None:
        out = torch.empty(A.n, dtype=_FULL_DTYPE[semiring], device="cuda")
    need = spmv_bin_full_workspace_bytes(A, semiring)
    if ws is None and need:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    _check(lib().spmv_bin_full(A.view, semiring, _ptr(x), _ptr(col_scale), _ptr(x_active), _ptr(mask), flags, float(alpha),
                               float(beta), _ptr(out), _ptr(ws), need if ws is not None else 0, _stream()),
           "spmv_bin_full")
    return out


def spmv_bin_full_noalloc(A: B2SR, semiring: int, x, col_scale=None, mask=None, complement=False,
                          self_loop=False, accumulate=False, alpha=1.0, beta=0.0, out=None, x_active=None):
    """spmv_bin_full with the library's own scratch array as its workspace (no
    device allocation inside the call; ``out`` must be given for that)."""
    flags = (MASK_COMPLEMENT if complement else 0) | (SELF if self_loop else 0) | (ACCUMULATE if accumulate else 0)
    if out is None:
        out = torch.empty(A.n, dtype=_FULL_DTYPE[semiring], device="cuda")
    _check(lib().spmv_bin_full_noalloc(A.view, semiring, _ptr(x), _ptr(col_scale), _ptr(x_active), _ptr(mask), flags,
                                       float(alpha), float(beta), _ptr(out), _stream()), "spmv_bin_full_noalloc")
    return out


def spgemm_masked_workspace_bytes(A: B2SR, M: B2SR | None) -> int:
    return int(lib().spgemm_masked_workspace_bytes(A.view, None if M is None else M.view))


def spgemm_masked(A: B2SR, Bt: B2SR, M: B2SR | None = None, accumulate=False, out=None, ws=None):
    """Device int64 scalar (uint64 bits) = sum over M's ones of (A B)_ij, B = Bt^T."""
    out = torch.zeros(1, dtype=torch.int64, device="cuda") if out is None else out
    need = spgemm_masked_workspace_bytes(A, M)
    if ws is None and need:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    _check(lib().spgemm_masked(A.view, Bt.view, None if M is None else M.view, ACCUMULATE if accumulate else 0,
                               _ptr(out), _ptr(ws), need, _stream()), "spgemm_masked")
    return out


# ---- algorithms -------------------------------------------------------------

def spgemm_masked_rows(A: B2SR, Bt: B2SR, M: B2SR, row_begin: int, row_end: int, accumulate=False, out=None):
    """spgemm_masked over the mask tile-rows [row_begin, row_end) only."""
    out = torch.zeros(1, dtype=torch.int64, device="cuda") if out is None else out
    _check(lib().spgemm_masked_rows(A.view, Bt.view, M.view, int(row_begin), int(row_end),
                                    ACCUMULATE if accumulate else 0, _ptr(out), _stream()), "spgemm_masked_rows")
    return out


def spgemm_masked_profile(A: B2SR, Bt: B2SR, M: B2SR, out=None) -> dict:
    """Work counts of spgemm_masked(A, Bt, M) (b2sr.h): mask tiles, lookups,
    matched tile pairs, bit-row pair operations."""
    out = torch.empty(4, dtype=torch.int64, device="cuda") if out is None else out
    _check(lib().spgemm_masked_profile(A.view, Bt.view, M.view, _ptr(out), _stream()), "spgemm_masked_profile")
    c = as_u64(out)
    return {"mask_tiles": int(c[0]), "lookups": int(c[1]), "tile_pairs": int(c[2]), "row_pairs": int(c[3])}


def b2sr_algo_workspace_bytes(A: B2SR, algo: int) -> int:
    return int(lib().b2sr_algo_workspace_bytes(A.view, algo))


def _ws(A, algo, ws):
    need = b2sr_algo_workspace_bytes(A, algo)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    return ws, need


def b2sr_bfs(A: B2SR, src: int, out=None, ws=None):
    """Returns (levels int32 tensor with uint32 bits, levels run)."""
    out = torch.empty(A.n, dtype=torch.int32, device="cuda") if out is None else out
    ws, need = _ws(A, ALGO_BFS, ws)
    it = _U32(0)
    _check(lib().b2sr_bfs(A.view, src, _ptr(out), _ptr(ws), need, ctypes.byref(it), _stream()), "b2sr_bfs")
    return out, it.value


def b2sr_msbfs(A: B2SR, srcs, out=None, ws=None):
    srcs = np.ascontiguousarray(srcs, dtype=np.uint32)
    out = torch.empty((srcs.size, A.n), dtype=torch.int32, device="cuda") if out is None else out
    ws, need = _ws(A, ALGO_MSBFS, ws)
    it = _U32(0)
    arr = (_U32 * srcs.size)(*srcs.tolist())
    _check(lib().b2sr_msbfs(A.view, arr, srcs.size, _ptr(out), _ptr(ws), need, ctypes.byref(it), _stream()),
           "b2sr_msbfs")
    return out, it.value


def b2sr_sssp(A: B2SR, src: int, out=None, ws=None):
    out = torch.empty(A.n, dtype=torch.int32, device="cuda") if out is None else out
    ws, need = _ws(A, ALGO_SSSP, ws)
    it = _U32(0)
    _check(lib().b2sr_sssp(A.view, src, _ptr(out), _ptr(ws), need, ctypes.byref(it), _stream()), "b2sr_sssp")
    return out, it.value


def b2sr_cc(A: B2SR, out=None, ws=None):
    out = torch.empty(A.n, dtype=torch.int32, device="cuda") if out is None else out
    ws, need = _ws(A, ALGO_CC, ws)
    it = _U32(0)
    _check(lib().b2sr_cc(A.view, _ptr(out), _ptr(ws), need, ctypes.byref(it), _stream()), "b2sr_cc")
    return out, it.value


def b2sr_pagerank(A: B2SR, damping=0.85, iterations=20, out=None, ws=None):
    out = torch.empty(A.n, dtype=torch.float32, device="cuda") if out is None else out
    ws, need = _ws(A, ALGO_PAGERANK, ws)
    _check(lib().b2sr_pagerank(A.view, float(damping), int(iterations), _ptr(out), _ptr(ws), need, _stream()),
           "b2sr_pagerank")
    return out


def b2sr_pagerank_directed(At: B2SR, damping=0.85, iterations=20, out=None, ws=None):
    """PageRank of a directed graph given its pull matrix At (B2SR.from_csr(..., transpose=True))."""
    out = torch.empty(At.n, dtype=torch.float32, device="cuda") if out is None else out
    ws, need = _ws(At, ALGO_PAGERANK, ws)
    _check(lib().b2sr_pagerank_directed(At.view, float(damping), int(iterations), _ptr(out), _ptr(ws), need,
                                        _stream()), "b2sr_pagerank_directed")
    return out


STREAM_READ_BLOCKS = 8192


def b2sr_stream_read(t: torch.Tensor, nbytes: int | None = None, out=None):
    """Streams the bytes of device tensor t once (roofline calibration)."""
    nbytes = t.numel() * t.element_size() if nbytes is None else nbytes
    out = torch.empty(STREAM_READ_BLOCKS, dtype=torch.int32, device="cuda") if out is None else out
    _check(lib().b2sr_stream_read(_ptr(t), nbytes, _ptr(out), _stream()), "b2sr_stream_read")
    return out


def b2sr_eccentricity(A: B2SR, srcs, ws=None) -> np.ndarray:
    """Eccentricities (largest finite BFS level) of the given sources, host uint32."""
    srcs = np.ascontiguousarray(srcs, dtype=np.uint32)
    ecc = np.zeros(srcs.size, dtype=np.uint32)
    ws, need = _ws(A, ALGO_ECC, ws)
    _check(lib().b2sr_eccentricity(A.view, srcs.ctypes.data_as(_P), srcs.size, ecc.ctypes.data_as(_P), _ptr(ws),
                                   need, _stream()), "b2sr_eccentricity")
    return ecc


def b2sr_diameter(A: B2SR, ws=None) -> int:
    d = _U32(0)
    ws, need = _ws(A, ALGO_ECC, ws)
    _check(lib().b2sr_diameter(A.view, ctypes.byref(d), _ptr(ws), need, _stream()), "b2sr_diameter")
    return d.value


def sweep_stats(st) -> dict:
    """The five stats words of a sweep cut as a dict (conductance as a float)."""
    k, cut, vol, vol_all, taken = (int(v) for v in np.asarray(st, dtype=np.uint64))
    den = min(vol, vol_all - vol)
    return {"size": k, "cut": cut, "vol": vol, "vol_all": vol_all, "taken": taken,
            "conductance": cut / den if den else None}


def b2sr_sweep_cut(A: B2SR, score: torch.Tensor, order: bool = True, ws=None):
    """Sweep cut of a float32 score vector: (order u32 tensor or None, cluster
    bit words, stats dict)."""
    n = A.n
    o = torch.empty(n, dtype=torch.int32, device="cuda") if order else None
    bits = torch.empty(max(1, (n + 31) // 32), dtype=torch.int32, device="cuda")
    st = torch.empty(5, dtype=torch.int64, device="cuda")
    ws, need = _ws(A, ALGO_LGC, ws)
    _check(lib().b2sr_sweep_cut(A.view, _ptr(score), _ptr(o), _ptr(bits), _ptr(st), _ptr(ws), need, _stream()),
           "b2sr_sweep_cut")
    return o, bits, sweep_stats(st.cpu().numpy().view(np.uint64))


def b2sr_lgc(A: B2SR, seed: int, alpha: float = 0.85, iterations: int = 20, ws=None):
    """Local clustering around `seed`: (personalised PageRank float32 tensor,
    cluster bit words, stats dict)."""
    p = torch.empty(A.n, dtype=torch.float32, device="cuda")
    bits = torch.empty(max(1, (A.n + 31) // 32), dtype=torch.int32, device="cuda")
    st = torch.empty(5, dtype=torch.int64, device="cuda")
    ws, need = _ws(A, ALGO_LGC, ws)
    _check(lib().b2sr_lgc(A.view, int(seed), float(alpha), int(iterations), _ptr(p), _ptr(bits), _ptr(st), _ptr(ws),
                          need, _stream()), "b2sr_lgc")
    return p, bits, sweep_stats(st.cpu().numpy().view(np.uint64))


def mis_keys(n: int, seed: int) -> torch.Tensor:
    """Distinct nonzero keys for b2sr_mis / b2sr_color: a random 32-bit
    priority above the vertex id + 1 (so ties are impossible), as an int64
    device tensor holding the uint64 bits."""
    r = np.random.Generator(np.random.PCG64(seed)).integers(0, 1 << 31, size=n, dtype=np.uint64)
    k = (r << np.uint64(32)) | (np.arange(n, dtype=np.uint64) + np.uint64(1))
    return torch.from_numpy(k.view(np.int64)).cuda()


def b2sr_mis(A: B2SR, key, out=None, ws=None):
    """(membership bit vector int32 tensor, rounds) of the max-times independent set."""
    out = torch.empty(max(_words(A.n), 1), dtype=torch.int32, device="cuda") if out is None else out
    ws, need = _ws(A, ALGO_MIS, ws)
    it = _U32(0)
    _check(lib().b2sr_mis(A.view, _ptr(key), _ptr(out), _ptr(ws), need, ctypes.byref(it), _stream()), "b2sr_mis")
    return out, it.value


def b2sr_color(A: B2SR, key, out=None, ws=None):
    """(colour per vertex int32 tensor with uint32 bits, colours used)."""
    out = torch.empty(A.n, dtype=torch.int32, device="cuda") if out is None else out
    ws, need = _ws(A, ALGO_COLOR, ws)
    nc = _U32(0)
    _check(lib().b2sr_color(A.view, _ptr(key), _ptr(out), _ptr(ws), need, ctypes.byref(nc), _stream()),
           "b2sr_color")
    return out, nc.value


def b2sr_csr_transpose(n: int, rowptr, colind):
    """(t_rowptr, t_colind) int32 device tensors of the transposed CSR; the
    columns within a row are in no particular order."""
    rp, ci = _i32(rowptr), _i32(colind)
    nnz = int(ci.numel())
    trp = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    tci = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    need = int(lib().b2sr_csr_transpose_workspace_bytes(n))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    _check(lib().b2sr_csr_transpose(n, nnz, _ptr(rp), _ptr(ci), _ptr(trp), _ptr(tci), _ptr(ws), need, _stream()),
           "b2sr_csr_transpose")
    return trp, tci[:nnz]


def triangle_count(rowptr, colind, n: int, tile: int) -> int:
    """Triangles of an undirected graph (Sec. V): L = strict lower triangle in
    B2SR, then the sum of (L L^T) masked by L."""
    L = B2SR.from_csr(rowptr, colind, n, tile, lower=True)
    s = spgemm_masked(L, L, L)
    return int(as_u64(s)[0])


# ---- batched multi-source BFS -----------------------------------------------

def _views(groups):
    arr = (b2sr_matrix * len(groups))()
    for k, A in enumerate(groups):
        arr[k] = A._view
    return arr


def b2sr_msbfs_batch_workspace_bytes(n: int) -> int:
    return int(lib().b2sr_msbfs_batch_workspace_bytes(n))


def b2sr_msbfs_batch(n: int, groups, seed_vertex, seed_bit, mode=BATCH_LEVELS, out=None, ws=None):
    """Batched 64-wide BFS over block-diagonal groups sharing an n-vertex space.
    Returns (levels int32 tensor [n, 64] with uint32 bits, levels run)."""
    out = torch.empty((n, 64), dtype=torch.int32, device="cuda") if out is None else out
    need = b2sr_msbfs_batch_workspace_bytes(n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda") if ws is None else ws
    it = _U32(0)
    views = _views(groups)
    _check(lib().b2sr_msbfs_batch(n, len(groups), views, seed_vertex.numel(), _ptr(seed_vertex), _ptr(seed_bit),
                                  _ptr(out), mode, _ptr(ws), need, ctypes.byref(it), _stream()), "b2sr_msbfs_batch")
    return out, it.value


def b2sr_msbfs_batch_timed(n: int, groups, seed_vertex, seed_bit, out=None, ws=None, stamp_levels: int = 64,
                           stamp_blocks: int = 4096):
    """The persistent batched BFS with its phase timestamps (b2sr.h).  Returns
    (levels, levels run, per-level phase times in microseconds: a dict of
    arrays over the levels run, each the median over blocks except `product`,
    the span from the earliest start to the last block's product end)."""
    out = torch.empty((n, 64), dtype=torch.int32, device="cuda") if out is None else out
    need = b2sr_msbfs_batch_workspace_bytes(n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda") if ws is None else ws
    stamps = torch.zeros(stamp_levels * stamp_blocks * 5, dtype=torch.int64, device="cuda")
    it, grid, khz = _U32(0), _U32(0), _U32(0)
    _check(lib().b2sr_msbfs_batch_timed(n, len(groups), _views(groups), seed_vertex.numel(), _ptr(seed_vertex),
                                        _ptr(seed_bit), _ptr(out), _ptr(ws), need, _ptr(stamps), stamp_levels,
                                        stamp_blocks, ctypes.byref(grid), ctypes.byref(khz), ctypes.byref(it),
                                        _stream()), "b2sr_msbfs_batch_timed")
    nb = min(grid.value, stamp_blocks)
    lv = min(it.value, stamp_levels)
    a = stamps.view(stamp_levels, stamp_blocks, 5)[:lv, :nb].cpu().numpy().astype(np.float64) * (1e3 / khz.value)
    start = a[:, :, 0].min(axis=1, keepdims=True)
    phases = {"product": a[:, :, 1].max(axis=1) - start[:, 0],
              "product_median_block": np.median(a[:, :, 1] - start, axis=1),
              "barrier1_wait": np.median(a[:, :, 2] - a[:, :, 1], axis=1),
              "update": np.median(a[:, :, 3] - a[:, :, 2], axis=1),
              "barrier2_wait": np.median(a[:, :, 4] - a[:, :, 3], axis=1)}
    return out, it.value, phases


class MsbfsPlan:
    """The batched BFS instantiated once as hipGraphs and replayed (b2sr.h):
    per-level kernels (BATCH_LEVELS) or the persistent kernel (BATCH_PERSISTENT)."""

    def __init__(self, n: int, groups, seed_vertex, seed_bit, mode=BATCH_LEVELS, out=None, ws=None):
        self.n = n
        self.mode = mode
        self.groups = list(groups)
        self.seed_vertex, self.seed_bit = seed_vertex, seed_bit
        self.out = torch.empty((n, 64), dtype=torch.int32, device="cuda") if out is None else out
        need = b2sr_msbfs_batch_workspace_bytes(n)
        self.ws = torch.empty(need, dtype=torch.uint8, device="cuda") if ws is None else ws
        self._views = _views(self.groups)
        h = _P()
        _check(lib().b2sr_msbfs_batch_plan_create(n, len(self.groups), self._views, seed_vertex.numel(),
                                                  _ptr(seed_vertex), _ptr(seed_bit), _ptr(self.out), mode,
                                                  _ptr(self.ws), need, ctypes.byref(h)), "b2sr_msbfs_batch_plan_create")
        self._h = h

    def launch(self, want_iters: bool = False, check: bool = True):
        """Replays the plan.  With ``check`` (the default) the call waits for the
        replay and raises if a grid barrier timed out; ``check=False`` only
        enqueues it (call ``status`` later)."""
        it = _U32(0)
        sync = want_iters or check
        _check(lib().b2sr_msbfs_batch_plan_launch(self._h, ctypes.byref(it) if sync else None, _stream()),
               "b2sr_msbfs_batch_plan_launch")
        return it.value if want_iters else None

    def status(self) -> int:
        """Waits for the enqueued replays; raises if a barrier timed out since the
        last status read; returns the levels run by the last replay."""
        it = _U32(0)
        _check(lib().b2sr_msbfs_batch_plan_status(self._h, ctypes.byref(it), _stream()),
               "b2sr_msbfs_batch_plan_status")
        return it.value

    def close(self):
        if self._h is not None and _lib is not None:
            _check(lib().b2sr_msbfs_batch_plan_destroy(self._h), "b2sr_msbfs_batch_plan_destroy")
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving: continuous multi-source BFS sessions ---------------------------

def b2sr_bfs_session_bytes(n: int) -> int:
    return int(lib().b2sr_bfs_session_bytes(n))


class BfsSession:
    """Up to 64 BFS queries on one graph sharing 64-bit frontier words; queries
    join and leave between levels (b2sr.h).  Every call is issued on
    ``stream`` (a torch.cuda.Stream; the current stream when None).  One step
    is in flight at a time: ``step()`` copies the step's alive word to pinned
    host memory and records an event; ``ready()`` polls it."""

    SLOTS = 64

    def __init__(self, A: B2SR, ws=None, stream=None):
        self.A = A
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._s = ctypes.c_void_p(self.stream.cuda_stream)
        need = b2sr_bfs_session_bytes(A.n)
        if ws is None:
            with torch.cuda.stream(self.stream):  # the allocator then orders reuse after this stream's work
                ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        self.ws = ws
        if self.ws.numel() < need:
            raise ValueError("session workspace too small")
        self._alive = torch.zeros(1, dtype=torch.int64).pin_memory()
        self._event = torch.cuda.Event()
        self._pending = False
        h = _P()
        _check(lib().b2sr_bfs_session_create(A.view, _ptr(self.ws), need, self._s, ctypes.byref(h)),
               "b2sr_bfs_session_create")
        self._h = h

    def join(self, slot: int, source: int):
        _check(lib().b2sr_bfs_session_join(self._h, slot, source, self._s), "b2sr_bfs_session_join")

    def step(self):
        _check(lib().b2sr_bfs_session_step(self._h, ctypes.c_void_p(self._alive.data_ptr()), self._s),
               "b2sr_bfs_session_step")
        self._event.record(self.stream)
        self._pending = True

    def ready(self) -> bool:
        return not self._pending or self._event.query()

    def alive(self) -> int:
        """The alive word of the last step (waits for it)."""
        if self._pending:
            self._event.synchronize()
            self._pending = False
        return int(self._alive.numpy().view(np.uint64)[0])

    def extract(self, slot: int, out=None):
        """Levels of the finished query in ``slot`` (int32 tensor with uint32
        bits, 0xFFFFFFFF = unreached); frees the slot."""
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty(self.A.n, dtype=torch.int32, device="cuda")
        _check(lib().b2sr_bfs_session_extract(self._h, slot, _ptr(out), self._s), "b2sr_bfs_session_extract")
        return out

    def cancel(self, slot: int):
        _check(lib().b2sr_bfs_session_extract(self._h, slot, None, self._s), "b2sr_bfs_session_extract")

    def info(self):
        st, busy = _U32(0), _U64(0)
        _check(lib().b2sr_bfs_session_info(self._h, ctypes.byref(st), ctypes.byref(busy)), "b2sr_bfs_session_info")
        return st.value, busy.value

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _check(lib().b2sr_bfs_session_destroy(self._h), "b2sr_bfs_session_destroy")
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
