"""Tile-width choice per graph.

Step 1, a sampling profile (Sec. III-C, Algorithm 1): for N sampled rows and
each k in {4, 8, 16, 32}, count the distinct k-wide column chunks the row
touches (its bit-rows in B2SR-k).  Algorithm 1 as printed is garbled (it
indexes the counter with a nonzero's position and divides a count by itself);
the reading used here: for a sampled row with e nonzeros and c_k distinct
chunks, B2SR-k stores c_k bit-rows of w_k bytes plus its share of each tile's
index and other bit-rows, estimated as c_k * (w_k + (4 + (k - 1) * w_k) / k)
bytes, against 8 * e bytes of float CSR; the estimate is the mean ratio.

Step 2, exact: the tile count for every k, from b2sr_count_tiles on the
device (one call per tile width).

Step 3, the choice: the tile width with the smallest modelled per-product cost
ntiles * (k * w_k + 4 + beta * k * V) bytes, where V is the width of a vector
value the product stages per tile column (8 for the 64-wide BFS frontier) and
beta discounts those re-reads, which mostly hit L2.
"""
from __future__ import annotations

import numpy as np
import torch

from . import BUILD_LOWER, _i32, b2sr_count_tiles  # noqa: F401

TILES = (4, 8, 16, 32)
ROW_BYTES = {4: 1, 8: 1, 16: 2, 32: 4}


def sampling_profile(rowptr: np.ndarray, colind: np.ndarray, n: int, nsample: int = 1024, seed: int = 0) -> dict:
    """Estimated B2SR/CSR storage ratio per tile width from sampled rows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = rng.choice(n, size=min(nsample, n), replace=False) if n else np.zeros(0, dtype=np.int64)
    est = {}
    for k in TILES:
        w = ROW_BYTES[k]
        ratios = []
        for i in rows:
            a, b = int(rowptr[i]), int(rowptr[i + 1])
            if a == b:
                continue
            c = np.unique(colind[a:b] // k).size
            ratios.append(c * (w + (4 + (k - 1) * w) / k) / (8.0 * (b - a)))
        est[k] = float(np.mean(ratios)) if ratios else 0.0
    return est


def exact_tiles(rowptr, colind, n: int) -> dict:
    """Exact non-empty tile count for every tile width (device counting)."""
    rp, ci = _i32(rowptr), _i32(colind)
    out = {}
    for k in TILES:
        trp = torch.empty((n + k - 1) // k + 1, dtype=torch.int32, device="cuda")
        out[k] = b2sr_count_tiles(n, int(ci.numel()), rp, ci, k, 0, trp)
    return out


def product_cost(ntiles: dict, value_bytes: int = 8, beta: float = 0.25) -> dict:
    return {k: ntiles[k] * (k * ROW_BYTES[k] + 4 + beta * k * value_bytes) for k in ntiles}


def choose_tile(g, value_bytes: int = 8, beta: float = 0.25, nsample: int = 1024) -> tuple[int, dict]:
    """(tile width, report) for graph g (a canonical CSR)."""
    prof = sampling_profile(g.rowptr, g.colind, g.n, nsample)
    tiles = exact_tiles(g.rowptr, g.colind, g.n)
    cost = product_cost(tiles, value_bytes, beta)
    best = min(cost, key=lambda k: (cost[k], k))
    return best, {"sampling_estimate": prof, "ntiles": tiles, "cost": cost}
