"""Benchmark of the B2SR hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (timed step): R-MAT scale 20, edge factor 16 (a, b, c = 0.57, 0.19,
0.19; symmetrised, self-loops removed, seed 20), B2SR tile 32x32, resident in
HBM.  One step runs every product of the path once over it:
  * vector binarisation of a predicate vector;
  * one masked bin x bin SpMV with a full frontier (mask: 1 % visited);
  * one bin x bin count SpMV (popcount dot products);
  * one plus-times and one min-plus bin x full SpMV;
  * BFS from 64 seeded sources as one 64-wide bit-frontier BFS;
  * SSSP (unit weights) from the first source; CC by min-label propagation;
  * 50 PageRank iterations (d = 0.85) in float32.
value = edges evaluated per second over the step: a product over the whole
matrix counts nnz(A); a product that reads only the tiles of its active
columns (the BFS levels, SSSP and CC iterations) counts the nonzeros inside
the tiles it reads, which the bench derives exactly from the step's own
outputs (the tile bytes read per product are reported too).

Also reported (same process, outside the timed step): the roofline of the
step's dominant kernel (the plus-times product) and of the headline masked
bin x bin product, both measured with HIP events on their stream; the CSR ->
B2SR conversion time; single-source BFS GTEPS (Graph500 style); the
correctness-scale workload (ER n = 4096, B2SR-8); B2SR storage and product
times at every tile width (4 .. 64) on R-MAT s20, the king grid and a
Mycielski graph; the measured autotuner's choice; triangle counting (masked
SpGEMM) on R-MAT scale 18 and a 2048 x 2048 king grid for every tile width;
batched against per-graph BFS; serving at several offered rates; and the CPU
oracle timed on the host (whose results also verify the step's outputs).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import paper_2201_08560_amd as b2  # noqa: E402

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pack(b: np.ndarray) -> torch.Tensor:
    nw = max((b.size + 31) // 32, 1)
    pad = np.zeros(nw * 32, dtype=np.uint8)
    pad[: b.size] = b
    return torch.from_numpy(np.packbits(pad, bitorder="little").view(np.int32).copy()).cuda()


def spmv_bytes(A: b2.B2SR, with_mask: bool) -> int:
    """Compulsory HBM bytes of one full-frontier bin x bin SpMV: the three B2SR
    arrays once, the x bit vector, the y bit vector and the mask."""
    vec = ((A.n + 31) // 32) * 4
    return A.nbytes + vec * (3 if with_mask else 2)


def source_digest() -> str:
    h = hashlib.sha256()
    for f in ("common.h", "spmv_core.h", "spmv.hip"):
        with open(os.path.join(ROOT, "paper_2201_08560_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(digest: str, name: str):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it was
    taken on the current kernel source."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_digest") != digest:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Workload:
    def __init__(self, g: gg.Csr, tile: int):
        self.g = g
        small = gg.er_gnm(1024, 4096, seed=3)  # first launches load the code objects: keep them out of the timing
        b2.B2SR.from_graph(small, tile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.A = b2.B2SR.from_graph(g, tile)
        torch.cuda.synchronize()
        self.convert_s = time.perf_counter() - t0   # from host CSR: includes its copy to the device
        rp = torch.from_numpy(g.rowptr.view(np.int32)).cuda()
        ci = torch.from_numpy(g.colind.view(np.int32)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b2.B2SR.from_csr(rp, ci, g.n, tile)
        torch.cuda.synchronize()
        self.convert_device_s = time.perf_counter() - t0   # CSR already in device memory
        del rp, ci
        n = g.n
        r = gg.rng(2020)
        self.sources = gg.sample_sources(g, 64, seed=64)
        self.pred = torch.from_numpy((r.random(n) < 0.5).astype(np.uint8)).cuda()
        self.x_full = pack(np.ones(n, bool))
        self.mask = pack(r.random(n) < 0.01)
        self.xf = torch.from_numpy(r.random(n).astype(np.float32)).cuda()
        self.xd = torch.from_numpy(np.where(r.random(n) < 0.5, r.integers(0, 20, n), np.inf).astype(np.float32)).cuda()
        self.bits_out = torch.empty(max((n + 31) // 32, 1), dtype=torch.int32, device="cuda")
        self.y_bits = torch.zeros_like(self.bits_out)
        self.y_cnt = torch.empty(n, dtype=torch.int32, device="cuda")
        self.y_f = torch.empty(n, dtype=torch.float32, device="cuda")
        self.y_f2 = torch.empty(n, dtype=torch.float32, device="cuda")
        self.ws_plus = torch.empty(max(b2.spmv_bin_full_workspace_bytes(self.A, b2.PLUS_TIMES_F32), 1),
                                   dtype=torch.uint8, device="cuda")
        self.ws = {a: torch.empty(b2.b2sr_algo_workspace_bytes(self.A, a), dtype=torch.uint8, device="cuda")
                   for a in (b2.ALGO_MSBFS, b2.ALGO_SSSP, b2.ALGO_CC, b2.ALGO_PAGERANK, b2.ALGO_BFS)}
        self.lv_multi = torch.empty((64, n), dtype=torch.int32, device="cuda")
        self.dist = torch.empty(n, dtype=torch.int32, device="cuda")
        self.labels = torch.empty(n, dtype=torch.int32, device="cuda")
        self.rank = torch.empty(n, dtype=torch.float32, device="cuda")
        self.ev = []
        self.ev_plus = []
        self.products = 0
        self.it_msbfs = self.it_sssp = self.it_cc = 0

    def step(self, record: bool):
        A = self.A
        prods = 0
        b2.b2sr_pack_bits(self.pred, out=self.bits_out)
        # headline kernel: masked bin x bin SpMV, bracketed by events on its stream
        self.y_bits.zero_()
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
        b2.spmv_bin_bin(A, self.x_full, self.mask, complement=True, accumulate=True, out=self.y_bits)
        if record:
            e1.record()
            self.ev.append((e0, e1))
        b2.spmv_bin_bin(A, self.x_full, None, count=True, out=self.y_cnt)
        # the step's dominant kernel: the plus-times product (PageRank's), bracketed the same way
        if record:
            p0 = torch.cuda.Event(enable_timing=True)
            p1 = torch.cuda.Event(enable_timing=True)
            p0.record()
        b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, self.xf, out=self.y_f, ws=self.ws_plus)
        if record:
            p1.record()
            self.ev_plus.append((p0, p1))
        b2.spmv_bin_full(A, b2.MIN_PLUS_F32, self.xd, self_loop=True, alpha=1.0, out=self.y_f2)
        prods += 4
        _, self.it_msbfs = b2.b2sr_msbfs(A, self.sources, out=self.lv_multi, ws=self.ws[b2.ALGO_MSBFS])
        _, self.it_sssp = b2.b2sr_sssp(A, int(self.sources[0]), out=self.dist, ws=self.ws[b2.ALGO_SSSP])
        _, self.it_cc = b2.b2sr_cc(A, out=self.labels, ws=self.ws[b2.ALGO_CC])
        prods += self.it_msbfs + self.it_sssp + self.it_cc
        b2.b2sr_pagerank(A, 0.85, 50, out=self.rank, ws=self.ws[b2.ALGO_PAGERANK])
        prods += 51  # 50 iterations + the degree count
        self.products = prods


ROW_BYTES = {4: 1, 8: 1, 16: 2, 32: 4, 64: 8}


def tile_nnz(g: gg.Csr, T: int) -> np.ndarray:
    """Nonzeros of every non-empty T x T tile, in B2SR tile order (tile-rows
    in order, tile columns ascending within a row)."""
    ntc = (g.n + T - 1) // T
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.rowptr.astype(np.int64)))
    key = (rows // T) * ntc + g.colind.astype(np.int64) // T
    return np.unique(key, return_counts=True)[1]


def _cc_changed_sets(g: gg.Csr, max_iter: int):
    """The vertices whose label changes in each round of min-label
    propagation from x_i = i (bookkeeping of the step's CC product reads)."""
    x = np.arange(g.n, dtype=np.int64)
    rp = g.rowptr.astype(np.int64)
    nonempty = np.diff(rp) > 0
    ci = g.colind.astype(np.int64)
    out = []
    for _ in range(max_iter):
        m = x.copy()
        m[nonempty] = np.minimum(x[nonempty], np.minimum.reduceat(x[ci], rp[:-1][nonempty]))
        changed = m != x
        out.append(changed)
        x = m
        if not changed.any():
            break
    return out


def tile_reads(w: "Workload") -> dict:
    """Edges (nonzeros of the tiles read) and tile bytes read by each product of
    the step.  A product over the whole matrix reads every tile.  The products
    with x_active read only tiles whose column segment holds an active entry:
    the 64-source BFS at level k the vertices with a source at level k - 1,
    SSSP at iteration i the vertices at distance i - 1 (unit weights), CC the
    vertices whose label changed in the round before (all at first); the sets
    come from the step's outputs (CC's from its propagation rounds)."""
    g, A = w.g, w.A
    T = A.tile
    nnz_t = tile_nnz(g, T)
    tci = b2.as_u32(A.tile_colind)[: A.ntiles].astype(np.int64)
    assert nnz_t.size == A.ntiles
    ntc = (g.n + T - 1) // T
    per_tile = T * ROW_BYTES[T] + 4  # bit-rows and the tile's column index

    def read(active: np.ndarray):
        cols = np.zeros(ntc, bool)
        cols[np.flatnonzero(active) // T] = True
        sel = cols[tci]
        return int(nnz_t[sel].sum()), int(sel.sum()) * per_tile

    lv = b2.as_u32(w.lv_multi)
    msbfs = [read((lv == k - 1).any(axis=0)) for k in range(1, w.it_msbfs + 1)]
    dist = b2.as_u32(w.dist)
    sssp = [read(dist == i - 1) for i in range(1, w.it_sssp + 1)]
    cc_sets = [np.ones(g.n, bool)] + _cc_changed_sets(g, w.it_cc)
    cc = [read(a) for a in cc_sets[: w.it_cc]]
    full_products = 4 + 51
    edges = full_products * g.nnz + sum(e for e, _ in msbfs + sssp + cc)
    full_bytes = A.ntiles * per_tile
    return {"edges_per_step": edges, "full_products": full_products,
            "tile_bytes_full_product": full_bytes,
            "msbfs_levels": [{"edges": e, "tile_bytes": b, "frac_of_full": b / full_bytes} for e, b in msbfs],
            "sssp_iterations": [{"edges": e, "tile_bytes": b, "frac_of_full": b / full_bytes} for e, b in sssp],
            "cc_iterations": [{"edges": e, "tile_bytes": b, "frac_of_full": b / full_bytes} for e, b in cc],
            "blended_edges_per_step": w.products * g.nnz}


def _median_ms(fn, reps: int = 5) -> float:
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


def c1_section(reps: int = 20) -> dict:
    """The correctness-scale workload: ER G(n, m), n = 4096, m = 16384, seed 1,
    B2SR-8: one bin x bin SpMV (the BFS step from vertex 0), 20 PageRank
    iterations, and the masked triangle count; launch-bound at this size."""
    g = gg.er_gnm(4096, 16384, seed=1)
    A = b2.B2SR.from_graph(g, 8)
    L = b2.B2SR.from_graph(g, 8, lower=True)
    x = np.zeros(g.n, bool)
    x[0] = True
    xb, visited = pack(x), pack(x)
    y = torch.empty_like(xb)
    ws = torch.empty(b2.b2sr_algo_workspace_bytes(A, b2.ALGO_PAGERANK), dtype=torch.uint8, device="cuda")
    r = torch.empty(g.n, dtype=torch.float32, device="cuda")
    s = b2.spgemm_masked(L, L, L)
    t_spmv = _median_ms(lambda: b2.spmv_bin_bin(A, xb, visited, complement=True, out=y), reps)
    t_pr = _median_ms(lambda: b2.b2sr_pagerank(A, 0.85, 20, out=r, ws=ws), reps)
    t_tc = _median_ms(lambda: b2.spgemm_masked(L, L, L, out=s), reps)
    return {"workload": "ER n=4096 m=16384 seed 1, B2SR-8", "nnz": g.nnz, "ntiles": A.ntiles,
            "spmv_bfs_step_ms": t_spmv, "spmv_gteps": g.nnz / t_spmv / 1e6,
            "pagerank20_ms": t_pr, "pagerank_gteps": 21 * g.nnz / t_pr / 1e6,
            "tc_ms": t_tc, "triangles": int(b2.as_u64(s)[0]), "tc_edges_per_s": g.edges / t_tc * 1e3}


def tiles_section(step_graph: gg.Csr, reps: int = 5) -> dict:
    """B2SR storage and product times at every tile width on three patterns
    (Table VI classes): the step's R-MAT s20 (hybrid power law), the 2048^2 king
    grid (banded) and the Mycielski graph M15 (block: dense, triangle-free).
    Products: the full-frontier bin x bin SpMV and the plus-times bin x full SpMV."""
    out = {}
    for name, g in (("rmat20_ef16", step_graph), ("king2048", gg.king_grid(2048, 2048)),
                    ("mycielski15", gg.mycielski(15))):
        log(f"tile widths: {name}")
        res = {"n": g.n, "nnz": g.nnz, "csr_bytes": 4 * (g.n + 1) + 4 * g.nnz}
        x = torch.from_numpy(gg.rng(7).random(g.n).astype(np.float32)).cuda()
        ones = pack(np.ones(g.n, bool))
        yb = torch.empty_like(ones)
        yf = torch.empty(g.n, dtype=torch.float32, device="cuda")
        for T in (4, 8, 16, 32, 64):
            A = b2.B2SR.from_graph(g, T)
            ws = torch.empty(max(b2.spmv_bin_full_workspace_bytes(A, b2.PLUS_TIMES_F32), 1), dtype=torch.uint8,
                             device="cuda")
            tb = _median_ms(lambda: b2.spmv_bin_bin(A, ones, out=yb), reps)
            tp = _median_ms(lambda: b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, x, out=yf, ws=ws), reps)
            res[f"T{T}"] = {"ntiles": A.ntiles, "bytes": A.nbytes, "bits_ms": tb, "plus_ms": tp,
                            "bits_gteps": g.nnz / tb / 1e6, "plus_gteps": g.nnz / tp / 1e6,
                            "bits_GB_per_s": (A.nbytes + g.n // 4) / tb / 1e6}
            del A, ws
        out[name] = res
    return out


def autotune_section(g: gg.Csr) -> dict:
    """The measured autotuner on the step's graph: tile widths pruned by the
    Algorithm 1 estimate, each timed under every work split (bin x bin and
    plus-times products); the choice and every candidate's time."""
    from paper_2201_08560_amd import autotune
    T, k, rep = autotune.tune(g, kinds=("bits", "plus"), reps=5)
    rep["sampling_estimate"] = {str(a): v for a, v in rep["sampling_estimate"].items()}
    return rep


def bfs_gteps(w: Workload, nsrc: int = 8) -> dict:
    """Single-source BFS, Graph500 style: undirected edges of the source's
    component over the BFS time, harmonic mean over sources."""
    g = w.g
    rates, times = [], []
    for s in w.sources[:nsrc]:
        lv, _ = b2.b2sr_bfs(w.A, int(s), ws=w.ws[b2.ALGO_BFS])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lv, _ = b2.b2sr_bfs(w.A, int(s), ws=w.ws[b2.ALGO_BFS])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        reached = b2.as_u32(lv) != b2.UNREACHED
        edges = int(g.degrees()[reached].sum()) // 2
        rates.append(edges / dt / 1e9)
        times.append(dt)
    return {"gteps_hmean": len(rates) / sum(1.0 / r for r in rates), "ms_mean": 1e3 * float(np.mean(times)),
            "sources": nsrc}


def lgc_section(w: Workload, nsrc: int = 4, iters: int = 20) -> dict:
    """Local clustering from benchmark sources: personalised PageRank
    (`iters` plus-times products) then the sweep cut; and the sweep alone."""
    ws = torch.empty(b2.b2sr_algo_workspace_bytes(w.A, b2.ALGO_LGC), dtype=torch.uint8, device="cuda")
    total, sweep, clusters = [], [], []
    for s in w.sources[:nsrc]:
        b2.b2sr_lgc(w.A, int(s), 0.85, iters, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p, _, st = b2.b2sr_lgc(w.A, int(s), 0.85, iters, ws=ws)   # stats are read back: synchronises
        total.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        _, _, st2 = b2.b2sr_sweep_cut(w.A, p, order=False, ws=ws)
        sweep.append(time.perf_counter() - t0)
        assert st2 == st
        clusters.append({"seed": int(s), "size": st["size"], "conductance": st["conductance"], "taken": st["taken"]})
    return {"iterations": iters, "ms_median": 1e3 * float(np.median(total)),
            "sweep_ms_median": 1e3 * float(np.median(sweep)), "clusters": clusters}


VALU_OPS_PER_S = 256 * 4 * 16 * 2.4e9  # 32-bit integer VALU operations per second, one per lane-cycle


def tc_section(reps: int = 3) -> dict:
    out = {}
    for name, g in (("rmat18_ef16", gg.rmat(18, 16, seed=18)), ("king2048", gg.king_grid(2048, 2048))):
        log(f"tc {name}: n={g.n} nnz={g.nnz}")
        res = {"edges": g.edges}
        for T in (4, 8, 16, 32, 64):
            L = b2.B2SR.from_graph(g, T, lower=True)
            s = b2.spgemm_masked(L, L, L)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                b2.spgemm_masked(L, L, L, out=s)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) / 1e3)
            t = float(np.median(ts))
            # work counts of the plain orientation (every mask tile scanning Bt's
            # row); matched pairs and bit-row pairs are the same in the oriented
            # product the timing ran, its lookups are fewer
            work = b2.spgemm_masked_profile(L, L, L)
            res[f"T{T}"] = {"triangles": int(b2.as_u64(s)[0]), "ms": 1e3 * t, "edges_per_s": g.edges / t,
                            "plain_work": work, "row_pairs_per_s": work["row_pairs"] / t,
                            # one AND + popcount per bit-row pair against the integer VALU
                            # rate (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz): far below it, the
                            # product is bound by the latency of its lookups and gathers
                            "row_pairs_frac_of_valu_peak": work["row_pairs"] / t / VALU_OPS_PER_S}
            del L
        out[name] = res
    return out


def batched_section(graphs, reps: int = 3) -> dict:
    """256 Chung-Lu graphs (n log-uniform in 1K..256K, mean degree 4..32,
    exponent 2.1), 64 sources each; a query is one graph's 64-source BFS.
    Per-graph launches (b2sr_msbfs per graph) against the batched forms; every
    graph's levels must be identical between them."""
    from paper_2201_08560_amd import autotune
    from paper_2201_08560_amd.batch import GraphBatch
    count = len(graphs)
    t0 = time.perf_counter()
    tiles = [autotune.choose_tile(g, nsample=256)[0] for g in graphs]   # per-graph launches
    tune_s = time.perf_counter() - t0
    sources = [gg.sample_sources(g, 64, seed=1000 + i) for i, g in enumerate(graphs)]
    batch_tile, batch_tune = autotune.tune_batch(graphs, sources)      # the batched forms: measured
    B = GraphBatch(graphs, [batch_tile] * count)
    B.set_sources(sources)
    # the other layout: each graph at its own autotuned width (one group per width)
    Bw = GraphBatch(graphs, tiles)
    Bw.set_sources(sources)
    lv_w = torch.empty((Bw.n, 64), dtype=torch.int32, device="cuda")
    ws_w = torch.empty(b2.b2sr_msbfs_batch_workspace_bytes(Bw.n), dtype=torch.uint8, device="cuda")
    singles = [b2.B2SR.from_graph(g, t) for g, t in zip(graphs, tiles)]
    ws_single = torch.empty(max(b2.b2sr_algo_workspace_bytes(A, b2.ALGO_MSBFS) for A in singles),
                            dtype=torch.uint8, device="cuda")
    outs = [torch.empty((64, g.n), dtype=torch.int32, device="cuda") for g in graphs]
    torch.cuda.synchronize()

    def per_graph():
        for A, src, o in zip(singles, sources, outs):
            b2.b2sr_msbfs(A, src, out=o, ws=ws_single)

    lv = torch.empty((B.n, 64), dtype=torch.int32, device="cuda")
    ws_b = torch.empty(b2.b2sr_msbfs_batch_workspace_bytes(B.n), dtype=torch.uint8, device="cuda")
    plan = B.plan(b2.BATCH_LEVELS, out=torch.empty_like(lv), ws=torch.empty_like(ws_b))
    plan_p = B.plan(b2.BATCH_PERSISTENT, out=torch.empty_like(lv), ws=torch.empty_like(ws_b))
    modes = {"per_graph": per_graph,
             "batched_levels": lambda: B.run(b2.BATCH_LEVELS, out=lv, ws=ws_b),
             "batched_persistent": lambda: B.run(b2.BATCH_PERSISTENT, out=lv, ws=ws_b),
             "batched_hipgraph_levels": lambda: plan.launch(want_iters=True),
             "batched_hipgraph_persistent": lambda: plan_p.launch(want_iters=True),
             "batched_levels_per_graph_width": lambda: Bw.run(b2.BATCH_LEVELS, out=lv_w, ws=ws_w),
             "batched_persistent_per_graph_width": lambda: Bw.run(b2.BATCH_PERSISTENT, out=lv_w, ws=ws_w)}
    res = {}
    for name, fn in modes.items():
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        t = float(np.median(ts))
        res[name] = {"ms": 1e3 * t, "graphs_per_s": count / t, "bfs_per_s": 64 * count / t}
        log(f"batched {name}: {1e3 * t:.2f} ms")
    same = all(torch.equal(outs[i], B.levels_of(lv, i)) and torch.equal(outs[i], B.levels_of(plan.out, i))
               and torch.equal(outs[i], B.levels_of(plan_p.out, i)) and torch.equal(outs[i], Bw.levels_of(lv_w, i))
               for i in range(count))
    # where the persistent kernel's time goes: device wall-clock stamps per level and block
    lvt, _, ph = b2.b2sr_msbfs_batch_timed(B.n, B.groups, B.seed_vertex, B.seed_bit, ws=ws_b)
    same = same and all(torch.equal(outs[i], B.levels_of(lvt, i)) for i in range(count))
    phases = {k: {"total_ms": float(v.sum()) / 1e3, "per_level_us": [round(float(x), 1) for x in v]}
              for k, v in ph.items()}
    plan.close()
    plan_p.close()
    hist = {str(T): tiles.count(T) for T in (4, 8, 16, 32, 64)}
    best = min((k for k in res if k != "per_graph"), key=lambda k: res[k]["ms"])
    return {"graphs": count, "n_total": B.n, "nnz_total": int(sum(g.nnz for g in graphs)),
            "sources_per_graph": 64, "tile_histogram": hist, "batch_tile": batch_tile, "autotune_s": tune_s,
            "batch_tile_tuning": batch_tune, "persistent_phases": phases,
            "modes": res,
            "identical_results": bool(same),
            "speedup_best_batched_vs_per_graph": res["per_graph"]["ms"] / res[best]["ms"]}


def stream_read_ceiling(w: "Workload", reps: int = 7) -> dict:
    """The read-only bandwidth of a plain stream over the same number of bytes
    as the headline product (its matrix's tile bits plus a tail of indices):
    the practical ceiling the product is compared with."""
    nbytes = spmv_bytes(w.A, True) & ~15
    buf = w.A.bits if w.A.bits.numel() >= nbytes else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    if buf.numel() < nbytes:
        nbytes = buf.numel() & ~15
    out = b2.b2sr_stream_read(buf, nbytes)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b2.b2sr_stream_read(buf, nbytes, out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    t = float(np.median(ts))
    return {"bytes": nbytes, "ms": 1e3 * t, "GB_per_s": nbytes / t / 1e9, "frac_of_peak": nbytes / t / 1e9 / HBM_PEAK_GBS}


def cold_warm(w: "Workload", reps: int = 5) -> dict:
    """The headline product timed warm (back to back) and cold (a 1 GiB read of
    an unrelated buffer between launches evicts the 256 MB Infinity Cache and
    the L2s without leaving dirty lines to write back)."""
    scrub = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda")
    scrub_out = b2.b2sr_stream_read(scrub)

    def one():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b2.spmv_bin_bin(w.A, w.x_full, w.mask, complement=True, accumulate=True, out=w.y_bits)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    one()
    warm = float(np.median([one() for _ in range(reps)]))
    cold = []
    for _ in range(reps):
        b2.b2sr_stream_read(scrub, out=scrub_out)
        torch.cuda.synchronize()
        cold.append(one())
    cold = float(np.median(cold))
    alg = spmv_bytes(w.A, True)
    return {"warm_ms": 1e3 * warm, "cold_ms": 1e3 * cold, "warm_frac": alg / warm / 1e9 / HBM_PEAK_GBS,
            "cold_frac": alg / cold / 1e9 / HBM_PEAK_GBS, "scrub_bytes_read": scrub.numel()}


def cpu_baseline(w: Workload, edges_per_step: float, threads: int | None = None, min_s: float = 10.0,
                 check: bool = False) -> dict:
    """The oracle on the host: the same step's results (the four single
    products, 64 BFS, SSSP, CC, PageRank x 50), timed over whole steps.  With
    `check`, the last step's GPU outputs are compared with these results."""
    import oracle as orc
    g = w.g
    n = g.n
    r = gg.rng(2020)
    pred = r.random(n) < 0.5  # noqa: F841  (same draws as the GPU inputs)
    ones = np.ones(n, bool)
    mask = r.random(n) < 0.01
    xf = r.random(n).astype(np.float32).astype(np.float64)
    xd = np.where(r.random(n) < 0.5, r.integers(0, 20, n), np.inf).astype(np.float32).astype(np.float64)
    orc.lib()
    saved = orc.num_threads()
    if threads is not None:
        orc.set_num_threads(threads)
    reps = 0
    t0 = time.perf_counter()
    while True:  # whole steps until at least min_s of host work
        y_or = orc.spmv_or(g, ones, mask, True)
        y_cnt = orc.spmv_count(g, ones)
        y_plus = orc.spmv_plus(g, xf)
        y_min = orc.spmv_min_plus(g, xd, 1.0, True)
        lv = orc.bfs_multi(g, w.sources)
        dist = orc.sssp_unit(g, int(w.sources[0]))
        labels = orc.cc(g)
        pr = orc.pagerank(g, 0.85, 50)
        reps += 1
        if time.perf_counter() - t0 >= min_s:
            break
    dt = (time.perf_counter() - t0) / reps
    cores = orc.num_threads()
    orc.set_num_threads(saved)
    out = {"value": edges_per_step / dt / 1e9, "unit": "GTEPS", "cores": cores, "kind": "oracle",
           "sample": f"{reps} full steps of the same workload (R-MAT s20: 4 single products, 64 BFS, SSSP, CC, "
                     f"PageRank x 50), {dt:.2f} s wall each"}
    if check:
        yb = b2.as_u32(w.y_bits)
        got_or = np.unpackbits(yb.view(np.uint8), bitorder="little")[:n].astype(bool)
        gp = w.y_f.cpu().numpy().astype(np.float64)
        gpr = w.rank.cpu().numpy().astype(np.float64)
        bound = (g.degrees() + 2) * 2.0 ** -24 * y_plus + 1e-30
        out["verify_step_outputs"] = {
            "spmv_bits_masked": bool(np.array_equal(got_or, y_or)),
            "spmv_count": bool(np.array_equal(b2.as_u32(w.y_cnt), y_cnt)),
            "spmv_plus_within_bound": bool(np.all(np.abs(gp - y_plus) <= bound)),
            "spmv_min_plus": bool(np.array_equal(w.y_f2.cpu().numpy(), y_min.astype(np.float32))),
            "bfs_64_sources": bool(np.array_equal(b2.as_u32(w.lv_multi), lv)),
            "sssp": bool(np.array_equal(b2.as_u32(w.dist), dist)),
            "cc": bool(np.array_equal(b2.as_u32(w.labels), labels)),
            "pagerank_rel_l1": float(np.abs(gpr - pr).sum() / pr.sum())}
    return out


def profile_mode(args):
    """A short fixed program for rocprofv3 counter runs: a 1 GiB device-to-device
    copy (the known-size reference for FETCH_SIZE / WRITE_SIZE), then --steps
    launches each of the headline masked bin x bin SpMV and of the plus-times
    bin x full SpMV on the R-MAT s20 B2SR-32 workload."""
    g = gg.rmat(20, 16, seed=20)
    w = Workload(g, 32)
    src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        w.y_bits.zero_()
        b2.spmv_bin_bin(w.A, w.x_full, w.mask, complement=True, accumulate=True, out=w.y_bits)
    for _ in range(args.steps):
        b2.spmv_bin_full(w.A, b2.PLUS_TIMES_F32, w.xf, out=w.y_f, ws=w.ws_plus)
    torch.cuda.synchronize()
    log(json.dumps({"profile_mode": True, "spmv_bits_alg_bytes": spmv_bytes(w.A, True),
                    "spmv_plus_alg_bytes": w.A.nbytes + 8 * g.n,
                    "copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                    "kernel_source_digest": source_digest()}))


def serving_section(pool, rates, seconds: float, budget_bytes: int, seed: int = 77, mix=(0.6, 0.15, 0.15, 0.1),
                    workers: int = 2, streams: int = 4):
    """Poisson streams of BFS/SSSP/CC/TC queries over a resident pool of R-MAT
    graphs, continuous batching with admission by a device-memory budget, at
    increasing offered rates: each rate runs for `seconds`; the sweep stops
    after the first rate whose answered rate (queries done or rejected per
    second) falls below 90 % of the offered one (the knee).  The budget is
    below a scale-20 graph's BFS session (its 64 level arrays), so those
    queries are rejected, and sessions of the next scales contend for it.  A
    sample of each rate's answers is compared with the single-query drivers
    run alone."""
    from paper_2201_08560_amd import autotune
    from paper_2201_08560_amd.serve import GpuExecutor, Query, Server
    t0 = time.perf_counter()
    tiles = [autotune.choose_tile(g, nsample=256)[0] for g in pool]
    mats = [(b2.B2SR.from_graph(g, t), b2.B2SR.from_graph(g, GpuExecutor.tc_tile(t), lower=True))
            for g, t in zip(pool, tiles)]
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    pool_bytes = sum(A.nbytes + L.nbytes for A, L in mats)
    log(f"serving pool: {len(pool)} graphs resident, {pool_bytes / 2**30:.2f} GiB B2SR, {load_s:.1f} s")
    cand = [np.flatnonzero(g.degrees() > 0) for g in pool]
    # warm-up: one query of each kind on a small graph (first launches of each kernel)
    ex = GpuExecutor(mats, pool, streams=streams, workers=workers)
    small = int(np.argmin([g.n for g in pool]))
    Server(ex, budget_bytes, cache=False).run(
        [Query(-1 - k, kind, small, int(cand[small][0]), 0.0) for k, kind in enumerate(("bfs", "sssp", "cc", "tc"))])
    torch.cuda.synchronize()
    ex.shutdown()
    per_rate = []
    for qps in rates:
        ex = GpuExecutor(mats, pool, streams=streams, workers=workers)
        r = np.random.default_rng(seed)
        nq = int(qps * seconds)
        arrivals = np.cumsum(r.exponential(1.0 / qps, nq))
        kinds = r.choice(np.array(["bfs", "sssp", "cc", "tc"]), p=list(mix), size=nq)
        gidx = r.integers(len(pool), size=nq)
        queries = [Query(i, str(kinds[i]), int(gidx[i]), int(r.choice(cand[gidx[i]])), float(arrivals[i]))
                   for i in range(nq)]
        sample = {}

        def on_done(q, sample=sample):
            if q.status == "done" and q.qid % 40 == 0:
                sample[q.qid] = (q, q.result)

        srv = Server(ex, budget_bytes, on_done=on_done, keep_results=False)
        t1 = time.perf_counter()
        srv.run(queries)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        ex.shutdown()
        st = srv.stats()
        same = True
        for qid, (q, res) in sorted(sample.items()):
            A = mats[q.graph][0]
            if q.kind == "bfs":
                ref = b2.b2sr_bfs(A, q.source)[0]
            elif q.kind == "sssp":
                ref = b2.b2sr_sssp(A, q.source)[0]
            elif q.kind == "cc":
                ref = b2.b2sr_cc(A)[0]
            else:
                L = mats[q.graph][1]
                same &= int(b2.as_u64(res)[0]) == int(b2.as_u64(b2.spgemm_masked(L, L, L))[0])
                continue
            same &= bool(torch.equal(res, ref))
        st["job_count"] = dict(ex.job_count)
        answered = [q for q in srv.done if q.status in ("done", "rejected")]
        span = max(q.finished for q in answered) - min(q.arrival for q in answered) if answered else 0.0
        st["answered_qps"] = len(answered) / span if span > 0 else 0.0
        st.update({"offered_qps": qps, "window_s": seconds, "wall_s": wall,
                   "session_queries": sum(1 for q in srv.done if q.kind in ("bfs", "sssp") and q.joined_step),
                   "sampled": len(sample), "sample_identical_alone": bool(same)})
        per_rate.append(st)
        log(f"serving {qps:.0f} q/s offered: {st['answered_qps']:.0f} answered, "
            f"{st.get('queries_per_s', 0):.0f} done per s, p50 {st.get('p50_ms', 0):.2f} ms, "
            f"p99 {st.get('p99_ms', 0):.2f} ms, waited {st['waited_for_memory']}, rejected {st['rejected']}")
        if st["answered_qps"] < 0.9 * qps:
            break
    return {"pool_graphs": len(pool), "pool_scales": sorted({int(np.log2(g.n)) for g in pool}),
            "pool_bytes": pool_bytes, "pool_load_s": load_s, "budget_bytes": budget_bytes,
            "tile_histogram": {str(T): tiles.count(T) for T in (4, 8, 16, 32, 64)}, "rates": per_rate}


def profile_tc(args):
    """A short fixed program for rocprofv3: --steps masked SpGEMM triangle counts
    each on R-MAT s18 ef16 at T = 8 and on the 2048 x 2048 king grid at T = 32
    (the best tile width of each)."""
    for name, g, T in (("rmat18_ef16", gg.rmat(18, 16, seed=18), 8), ("king2048", gg.king_grid(2048, 2048), 32)):
        L = b2.B2SR.from_graph(g, T, lower=True)
        s = b2.spgemm_masked(L, L, L)
        for _ in range(args.steps):
            b2.spgemm_masked(L, L, L, out=s)
        torch.cuda.synchronize()
        log(json.dumps({"profile_tc": name, "tile": T, "triangles": int(b2.as_u64(s)[0])}))


def profile_batch(args, graphs):
    """A short fixed program for rocprofv3: the batched 64-source BFS over the
    256-graph Chung-Lu batch at B2SR-4 (the width the batch tuning picks), --steps
    runs in the per-level mode, then --steps in the persistent mode, then one
    persistent run with its phase timestamps (printed per level, microseconds)."""
    from paper_2201_08560_amd.batch import GraphBatch
    sources = [gg.sample_sources(g, 64, seed=1000 + i) for i, g in enumerate(graphs)]
    B = GraphBatch(graphs, [4] * len(graphs))
    B.set_sources(sources)
    lv = torch.empty((B.n, 64), dtype=torch.int32, device="cuda")
    ws = torch.empty(b2.b2sr_msbfs_batch_workspace_bytes(B.n), dtype=torch.uint8, device="cuda")
    for mode, name in ((b2.BATCH_LEVELS, "levels"), (b2.BATCH_PERSISTENT, "persistent")):
        for _ in range(args.steps):
            _, it = B.run(mode, out=lv, ws=ws)
        torch.cuda.synchronize()
        log(json.dumps({"profile_batch": name, "levels": it}))
    _, it, ph = b2.b2sr_msbfs_batch_timed(B.n, B.groups, B.seed_vertex, B.seed_bit, ws=ws)
    log(json.dumps({"profile_batch": "persistent_phases_us",
                    **{k: [round(float(x), 1) for x in v] for k, v in ph.items()}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--profile-mode", action="store_true")
    ap.add_argument("--profile-tc", action="store_true")
    ap.add_argument("--profile-batch", action="store_true")
    ap.add_argument("--serve-qps", default="250,500,1000,2000,4000,8000,16000",
                    help="offered rates of the serving sweep (comma-separated, increasing)")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-budget-gib", type=float, default=0.25)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    batch_graphs = pool_graphs = None
    if args.profile_batch and args.gpus == 1 and world == 1:
        batch_graphs = gg.chung_lu_batch(256, 2.1, seed=1000, workers=min(8, os.cpu_count() or 1))
    profiling = args.profile_mode or args.profile_tc or args.profile_batch
    if not args.no_extras and not profiling and args.gpus == 1 and world == 1:
        # generated in worker processes before this process touches the GPU
        t0 = time.perf_counter()
        batch_graphs = gg.chung_lu_batch(256, 2.1, seed=1000, workers=min(8, os.cpu_count() or 1))
        log(f"batched workload: {len(batch_graphs)} graphs in {time.perf_counter() - t0:.1f} s, "
            f"n={sum(g.n for g in batch_graphs)} nnz={sum(g.nnz for g in batch_graphs)}")
        t0 = time.perf_counter()
        pool_graphs = gg.rmat_pool(64, seed=2000, workers=min(8, os.cpu_count() or 1))
        log(f"serving pool: {len(pool_graphs)} R-MAT graphs in {time.perf_counter() - t0:.1f} s, "
            f"nnz={sum(g.nnz for g in pool_graphs)}")
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} (WORLD_SIZE={world}) is not supported: the B2SR "
              "path runs on a single MI355X (the design notes describe how it would shard).", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.profile_mode:
        profile_mode(args)
        return
    if args.profile_tc:
        profile_tc(args)
        return
    if args.profile_batch:
        profile_batch(args, batch_graphs)
        return

    log("generating R-MAT s20 ef16 ...")
    g = gg.rmat(20, 16, seed=20)
    w = Workload(g, 32)
    log(f"B2SR-32: ntiles={w.A.ntiles} bytes={w.A.nbytes} convert={w.convert_s * 1e3:.1f} ms")

    for _ in range(args.warmup):
        w.step(record=False)
    torch.cuda.synchronize()
    w.ev.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        w.step(record=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    reads = tile_reads(w)
    edges_per_step = reads["edges_per_step"]
    value = edges_per_step * args.steps / t / 1e9
    kt = float(np.mean([a.elapsed_time(b) for a, b in w.ev])) / 1e3
    kp = float(np.mean([a.elapsed_time(b) for a, b in w.ev_plus])) / 1e3
    alg = spmv_bytes(w.A, True)
    alg_plus = w.A.nbytes + 8 * g.n  # the B2SR arrays once, x and y (float32) once
    digest = source_digest()
    traffic = read_traffic(digest, "spmv_plus_t32_rmat20_pmc.txt")
    traffic_bits = read_traffic(digest, "spmv_bits_t32_rmat20_pmc.txt")
    out = {
        "metric": "B2SR SpMV GTEPS + masked-SpGEMM TC edges/s; batched vs per-graph launches",
        "value": value, "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * t / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 bit tiles; f32 PageRank/SSSP; u32 CC", "data": "synthetic",
        "config": {"workload": "R-MAT scale 20, edge factor 16 (0.57/0.19/0.19), symmetrised, B2SR-32: "
                               "4 single products + 64-source BFS + SSSP + CC + 50 PageRank iterations",
                   "n": g.n, "nnz": g.nnz, "tile": 32, "ntiles": w.A.ntiles, "products_per_step": w.products,
                   "edges_per_step": edges_per_step, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm",
                     "kernel": "spmv_bin_full plus-times (spmv_kernel<32, 2, false, false> with its output "
                               "initialisation and split-row fixup kernels), the step's dominant kernel",
                     "achieved": alg_plus / kp / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg_plus / kp / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_plus, "ms_per_launch": kp * 1e3, "gteps": g.nnz / kp / 1e9,
                     "kernel_source_digest": digest},
        "roofline_headline_bits": {"bound": "hbm",
                                   "kernel": "spmv_kernel<32, 0, false, false> (masked bin x bin SpMV, full frontier)",
                                   "achieved": alg / kt / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": alg / kt / 1e9 / HBM_PEAK_GBS, "traffic": traffic_bits,
                                   "alg_bytes_per_launch": alg, "ms_per_launch": kt * 1e3,
                                   "gteps": g.nnz / kt / 1e9},
        "spmv_gteps": g.nnz / kt / 1e9,
        "step_reads": reads,
        "step_rate_blended_gteps": reads["blended_edges_per_step"] * args.steps / t / 1e9,
        "convert_ms": w.convert_s * 1e3,
        "convert_device_csr_ms": w.convert_device_s * 1e3,
    }
    ceiling = stream_read_ceiling(w)
    out["roofline_headline_bits"]["stream_read_ceiling"] = ceiling
    out["roofline_headline_bits"]["frac_of_stream_read"] = (alg / kt / 1e9) / ceiling["GB_per_s"]
    out["roofline"]["frac_of_stream_read"] = (alg_plus / kp / 1e9) / ceiling["GB_per_s"]
    if not args.no_extras:
        out["bfs_single_source"] = bfs_gteps(w)
        out["c1_er4096"] = c1_section()
        out["autotune"] = autotune_section(g)
        out["tile_widths"] = tiles_section(g)
        out["lgc"] = lgc_section(w)
        out["tc"] = tc_section()
        out["batched"] = batched_section(batch_graphs)
        out["serving"] = serving_section(pool_graphs, [float(v) for v in str(args.serve_qps).split(",")],
                                         args.serve_seconds, int(args.serve_budget_gib * 2**30))
        out["headline_cold_warm"] = cold_warm(w)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, edges_per_step, check=True)
        if not args.no_extras:
            log("cpu baseline on one thread ...")
            out["cpu_baseline_1thread"] = cpu_baseline(w, edges_per_step, threads=1, min_s=1.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
