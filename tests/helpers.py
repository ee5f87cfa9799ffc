"""Shared test utilities (no product arithmetic; vectors are packed with numpy)."""
import numpy as np

import graphgen as gg

UNR = 0xFFFFFFFF
TILES = (4, 8, 16, 32, 64)
EPS32 = 2.0 ** -24


def pack_bits(b: np.ndarray) -> np.ndarray:
    """Bool vector -> LSB-first uint32 words (padding bits zero)."""
    b = np.asarray(b, dtype=bool)
    nw = max((b.size + 31) // 32, 1)
    pad = np.zeros(nw * 32, dtype=np.uint8)
    pad[: b.size] = b
    return np.packbits(pad, bitorder="little").view(np.uint32).copy()


def unpack_bits(w: np.ndarray, n: int) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.uint32)
    return np.unpackbits(w.view(np.uint8), bitorder="little")[:n].astype(bool)


def padding_zero(w: np.ndarray, n: int) -> bool:
    w = np.ascontiguousarray(w, dtype=np.uint32)
    allbits = np.unpackbits(w.view(np.uint8), bitorder="little")
    return not allbits[n:].any()


def small_graphs():
    """Small graphs spanning several tiles, ragged tails and the degenerate cases."""
    gs = [
        gg.er_gnm(4096, 16384, seed=1),           # the correctness-scale ER workload
        gg.er_gnm(4099, 12000, seed=2),           # ragged last tile-row
        gg.er_gnm(2049, 6000, seed=7),            # one vertex alone in the last tile column
        gg.rmat(13, 16, seed=13),                 # power-law rows crossing wave chunks
        gg.star(20000),                           # one tile-row far longer than a chunk
        gg.king_grid(61, 67),                     # banded
        gg.mycielski(10),
        gg.path(1000),
        gg.disjoint_union(gg.complete(40), gg.path(1), gg.cycle(37), gg.path(1)),
        gg.canonical_csr(100, [], [], name="empty100"),
        gg.canonical_csr(1, [], [], name="single"),
        gg.complete(33),
    ]
    for s in range(6):
        r = gg.rng(700 + s)
        gs.append(gg.random_graph_tiny(int(r.integers(2, 200)), float(r.choice([0.01, 0.05, 0.3])), 700 + s))
    return gs


def rel_l1(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))
