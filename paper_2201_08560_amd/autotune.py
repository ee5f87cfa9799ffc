"""Tile-width choice per graph.

Step 1, a sampling profile (Sec. III-C, Algorithm 1): for N sampled rows and
each k in {4, 8, 16, 32, 64}, count the distinct k-wide column chunks the row
touches (its bit-rows in B2SR-k).  Algorithm 1 as printed is garbled (it
indexes the counter with a nonzero's position and divides a count by itself);
the reading used here: for a sampled row with e nonzeros and c_k distinct
chunks, B2SR-k stores c_k bit-rows of w_k bytes plus its share of each tile's
index and other bit-rows, estimated as c_k * (w_k + (4 + (k - 1) * w_k) / k)
bytes, against 8 * e bytes of float CSR; the estimate is the mean ratio.

Step 2, exact: the tile count for every k, from b2sr_count_tiles on the
device (one call per tile width).

Step 3, the modelled choice (choose_tile): the tile width with the smallest
modelled per-product cost ntiles * (k * w_k + 4 + beta * k * V) bytes, where V
is the width of a vector value the product stages per tile column (8 for the
64-wide BFS frontier) and beta discounts those re-reads, which mostly hit L2.

The measured choice (tune): the Algorithm 1 estimate prunes the tile widths
(those within a factor of the best estimate, at most a few), then every
surviving tile width is built on the device and the products are timed with
HIP events under each work split (the matrix view's chunk_blocks: blocks of
tiles per wave); the (tile width, split) with the least measured time wins,
and the report holds every candidate's time.
"""
from __future__ import annotations

import numpy as np
import torch

from . import BUILD_LOWER, _i32, b2sr_count_tiles  # noqa: F401

TILES = (4, 8, 16, 32, 64)
ROW_BYTES = {4: 1, 8: 1, 16: 2, 32: 4, 64: 8}


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


def choose_batch_tile(graphs, value_bytes: int = 8, beta: float = 0.25) -> tuple[int, dict]:
    """One tile width for a whole batch: the T with the least modelled product
    cost summed over the graphs.  A batch holds one block-diagonal matrix per
    tile width present, each a product launch per level, and on the benchmark
    batch a separate group for a few small graphs whose own best width differs
    by a few percent costs more than it saves."""
    total = {T: 0.0 for T in TILES}
    for g in graphs:
        cost = product_cost(exact_tiles(g.rowptr, g.colind, g.n), value_bytes, beta)
        for T in TILES:
            total[T] += cost[T]
    best = min(total, key=lambda k: (total[k], k))
    return best, {"cost": total}


def prune(estimate: dict, slack: float = 1.5, keep: int = 3) -> list[int]:
    """Tile widths whose Algorithm 1 storage estimate is within `slack` of the
    smallest, the `keep` smallest of them (every width when none is > 0)."""
    pos = {k: v for k, v in estimate.items() if v > 0}
    if not pos:
        return list(TILES)
    best = min(pos.values())
    cands = sorted((k for k, v in pos.items() if v <= slack * best), key=lambda k: (pos[k], k))
    return sorted(cands[:keep])


SPLITS = (0, 1, 2, 4, 8, 16)


def _time_ms(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def _product_fns(A, kinds, seed: int = 0):
    """One callable per product kind on matrix A (full frontier / random x)."""
    from . import OR_U64, PLUS_TIMES_F32, spmv_bin_bin, spmv_bin_full, spmv_bin_full_workspace_bytes
    n = A.n
    r = np.random.default_rng(seed)
    fns = {}
    if "bits" in kinds:
        x = torch.full((max((n + 31) // 32, 1),), -1, dtype=torch.int32, device="cuda")
        if n % 32:
            x[-1] = (1 << (n % 32)) - 1
        y = torch.empty_like(x)
        fns["bits"] = lambda: spmv_bin_bin(A, x, out=y)
    if "plus" in kinds:
        xf = torch.from_numpy(r.random(n).astype(np.float32)).cuda()
        yf = torch.empty(n, dtype=torch.float32, device="cuda")
        ws = torch.empty(max(spmv_bin_full_workspace_bytes(A, PLUS_TIMES_F32), 1), dtype=torch.uint8, device="cuda")
        fns["plus"] = lambda: spmv_bin_full(A, PLUS_TIMES_F32, xf, out=yf, ws=ws)
    if "or64" in kinds:
        xu = torch.from_numpy(r.integers(0, 2**63, n, dtype=np.int64)).cuda()
        yu = torch.empty(n, dtype=torch.int64, device="cuda")
        fns["or64"] = lambda: spmv_bin_full(A, OR_U64, xu, out=yu)
    return fns


def tune(g, kinds=("bits", "plus"), splits=SPLITS, slack: float = 1.5, keep: int = 3, nsample: int = 1024,
         reps: int = 5, tiles=None) -> tuple[int, int, dict]:
    """(tile width, chunk_blocks, report) for graph g: candidates pruned by the
    Algorithm 1 estimate (or the given `tiles`), each timed on the device for
    every work split in `splits`; the least summed time over `kinds` wins."""
    import time
    from . import B2SR
    t0 = time.perf_counter()
    est = sampling_profile(g.rowptr, g.colind, g.n, nsample)
    cands = list(tiles) if tiles is not None else prune(est, slack, keep)
    times = {}
    for T in cands:
        A = B2SR.from_graph(g, T)
        for k in splits:
            Ak = A.with_split(k)
            fns = _product_fns(Ak, kinds)
            times[(T, k)] = sum(_time_ms(f, reps) for f in fns.values())
        del A
    best = min(times, key=lambda tk: (times[tk], tk))
    report = {"sampling_estimate": est, "candidates": cands, "splits": list(splits), "kinds": list(kinds),
              "times_ms": {f"T{T}/k{k}": v for (T, k), v in times.items()},
              "choice": {"tile": best[0], "chunk_blocks": best[1]}, "seconds": time.perf_counter() - t0}
    return best[0], best[1], report


def tune_batch(graphs, sources, candidates=None, keep: int = 2, reps: int = 3) -> tuple[int, dict]:
    """(tile width, report) for a batch: the `keep` widths with the least
    modelled summed cost (or the given candidates), each built as the batch's
    one group and timed as a per-level batched BFS with these sources; the
    least measured time wins."""
    import time
    from . import BATCH_LEVELS
    from .batch import GraphBatch
    t0 = time.perf_counter()
    modelled = choose_batch_tile(graphs)[1]["cost"]
    cands = list(candidates) if candidates is not None else sorted(sorted(modelled, key=lambda k: (modelled[k], k))[:keep])
    times = {}
    for T in cands:
        B = GraphBatch(graphs, [T] * len(graphs))
        B.set_sources(sources)
        times[T] = _time_ms(lambda: B.run(BATCH_LEVELS), reps)
        del B
    best = min(times, key=lambda k: (times[k], k))
    return best, {"modelled_cost": {str(k): v for k, v in modelled.items()}, "candidates": cands,
                  "times_ms": {str(k): v for k, v in times.items()}, "choice": best,
                  "seconds": time.perf_counter() - t0}


def _load_graph(spec: str):
    """A graph from a generator spec (rmat:SCALE:EF[:SEED], rmat_dir:SCALE:EF[:SEED],
    er:N:M[:SEED], king:R:C) or an .npz file holding n, rowptr and colind."""
    import graphgen as gg
    if spec.endswith(".npz"):
        z = np.load(spec, allow_pickle=False)
        return gg.Csr(int(z["n"]), z["rowptr"].astype(np.uint32), z["colind"].astype(np.uint32), spec)
    kind, *args = spec.split(":")
    a = [int(v) for v in args]
    if kind == "rmat":
        return gg.rmat(a[0], a[1], seed=a[2] if len(a) > 2 else 0)
    if kind == "rmat_dir":
        return gg.rmat_directed(a[0], a[1], seed=a[2] if len(a) > 2 else 0)
    if kind == "er":
        return gg.er_gnm(a[0], a[1], seed=a[2] if len(a) > 2 else 0)
    if kind == "king":
        return gg.king_grid(a[0], a[1])
    raise ValueError(f"unknown graph spec {spec!r}")


def main(argv=None) -> int:
    """Command line: the sampling profile of Algorithm 1 for a graph, and with
    a GPU the exact tile counts, the modelled product costs and the choice."""
    import argparse
    import json
    ap = argparse.ArgumentParser(prog="python -m paper_2201_08560_amd.autotune", description=main.__doc__)
    ap.add_argument("graph", help="rmat:S:EF[:SEED] | rmat_dir:S:EF[:SEED] | er:N:M[:SEED] | king:R:C | file.npz")
    ap.add_argument("--sample", type=int, default=1024, help="rows sampled for the profile")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--value-bytes", type=int, default=8, help="bytes of a vector value staged per tile column")
    ap.add_argument("--no-exact", action="store_true", help="only the sampling profile (no GPU needed)")
    ap.add_argument("--measure", action="store_true",
                    help="also time the pruned tile widths under every work split on the GPU (tune)")
    args = ap.parse_args(argv)
    g = _load_graph(args.graph)
    out = {"graph": g.name, "n": g.n, "nnz": g.nnz,
           "sampling_estimate_b2sr_over_csr": sampling_profile(g.rowptr, g.colind, g.n, args.sample, args.seed)}
    if not args.no_exact:
        tiles = exact_tiles(g.rowptr, g.colind, g.n)
        cost = product_cost(tiles, args.value_bytes)
        out.update({"ntiles": tiles, "exact_b2sr_over_csr": {
            k: (4 * ((g.n + k - 1) // k + 1) + tiles[k] * (4 + k * ROW_BYTES[k])) / (8.0 * g.nnz + 4.0 * (g.n + 1))
            for k in TILES} if g.nnz else {}, "product_cost_bytes": cost,
            "choice": min(cost, key=lambda k: (cost[k], k))})
    if args.measure:
        T, k, rep = tune(g, nsample=args.sample)
        out["measured"] = rep
    print(json.dumps(out, indent=1))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
