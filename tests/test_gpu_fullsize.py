"""Parity at the benchmark's full size and launch configuration: R-MAT scale
20, edge factor 16, B2SR-32, the same inputs and flags as the timed step; every
output is compared with the oracle (which runs these sizes in seconds), and
triangle counting on R-MAT scale 18 at every tile width."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as orc
from helpers import EPS32, TILES, pack_bits, padding_zero, rel_l1, unpack_bits

pytestmark = pytest.mark.gpu
b2 = pytest.importorskip("paper_2201_08560_amd")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


@pytest.fixture(scope="module")
def big():
    print("generating R-MAT s20 ef16", flush=True)
    g = gg.rmat(20, 16, seed=20)
    A = b2.B2SR.from_graph(g, 32)
    r = gg.rng(2020)
    n = g.n
    pred = r.random(n) < 0.5
    mask = r.random(n) < 0.01
    xf = r.random(n).astype(np.float32)
    xd = np.where(r.random(n) < 0.5, r.integers(0, 20, n), np.inf).astype(np.float32)
    return {"g": g, "A": A, "pred": pred, "mask": mask, "xf": xf, "xd": xd,
            "sources": gg.sample_sources(g, 64, seed=64)}


def dev_bits(b):
    return torch.from_numpy(pack_bits(b).view(np.int32)).cuda()


def test_headline_products(big):
    g, A, n = big["g"], big["A"], big["g"].n
    ones, mask = np.ones(n, bool), big["mask"]
    # the headline product: full frontier, 1 % visited mask, complemented, accumulated into zeros
    y = torch.zeros((n + 31) // 32, dtype=torch.int32, device="cuda")
    b2.spmv_bin_bin(A, dev_bits(ones), dev_bits(mask), complement=True, accumulate=True, out=y)
    yb = b2.as_u32(y)
    assert padding_zero(yb, n)
    assert np.array_equal(unpack_bits(yb, n), orc.spmv_or(g, ones, mask, True))
    # the same with the random half frontier the step packs, and under the sparse-frontier hint
    half = big["pred"]
    assert np.array_equal(unpack_bits(b2.as_u32(b2.spmv_bin_bin(A, dev_bits(half))), n), orc.spmv_or(g, half))
    sparse = gg.rng(5).random(n) < 0.001
    assert np.array_equal(unpack_bits(b2.as_u32(b2.spmv_bin_bin(A, dev_bits(sparse), sparse_x=True)), n),
                          orc.spmv_or(g, sparse))
    assert np.array_equal(b2.as_u32(b2.spmv_bin_bin(A, dev_bits(ones), count=True)), orc.spmv_count(g, ones))


def test_value_products(big):
    g, A = big["g"], big["A"]
    xf, xd = big["xf"], big["xd"]
    y = b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, torch.from_numpy(xf).cuda()).cpu().numpy()
    ref = orc.spmv_plus(g, xf.astype(np.float64))
    bound = (g.degrees() + 2) * EPS32 * ref + 1e-30  # x >= 0: sum |terms| = the sum
    assert np.all(np.abs(y - ref) <= bound)
    ym = b2.spmv_bin_full(A, b2.MIN_PLUS_F32, torch.from_numpy(xd).cuda(), self_loop=True, alpha=1.0).cpu().numpy()
    assert np.array_equal(ym, orc.spmv_min_plus(g, xd.astype(np.float64), 1.0, True).astype(np.float32))


def test_algorithms(big):
    g, A, src = big["g"], big["A"], big["sources"]
    print("bfs / msbfs", flush=True)
    assert np.array_equal(b2.as_u32(b2.b2sr_bfs(A, int(src[0]))[0]), orc.bfs(g, int(src[0])))
    lvm, _ = b2.b2sr_msbfs(A, src)  # all 64 sources of the step: every bit lane of the frontier word
    assert np.array_equal(b2.as_u32(lvm), orc.bfs_multi(g, src))
    print("sssp / cc", flush=True)
    assert np.array_equal(b2.as_u32(b2.b2sr_sssp(A, int(src[0]))[0]), orc.sssp_unit(g, int(src[0])))
    assert np.array_equal(b2.as_u32(b2.b2sr_cc(A)[0]), orc.cc(g))
    print("pagerank x 50", flush=True)
    pr = b2.b2sr_pagerank(A, 0.85, 50).cpu().numpy()
    assert rel_l1(pr, orc.pagerank(g, 0.85, 50)) <= 1e-5


@pytest.mark.parametrize("T", TILES)
def test_triangle_count_king2048(T):
    """The 2048 x 2048 king grid of the triangle-counting workload at every tile
    width: 4 (R - 1)(C - 1) triangles, and the oracle's count."""
    g = gg.king_grid(2048, 2048)
    print(f"tc king2048 T={T}", flush=True)
    assert b2.triangle_count(g.rowptr, g.colind, g.n, T) == orc.tc(g) == 4 * 2047 * 2047


def test_triangle_count_unmapped_rows():
    """A wheel on 2^19 + 2^12 vertices at T = 4 has 132096 tile columns, more
    than the product's LDS bitmap covers (131072): the hub's tile-row, and in A
    every rim tile-row far from the hub, look tile columns up by binary search
    in global memory instead.  Every triangle holds the hub, the largest id, so
    all n - 1 lie in L's last tile-row and none before it; the A.A masked sum is
    6 (n - 1).  (Closed forms: the oracle's merge over the hub's row of n - 1
    entries per edge takes minutes here; the same forms are pinned against the
    oracle on small wheels.)"""
    n = (1 << 19) + (1 << 12)
    g = gg.wheel(n)
    print(f"tc wheel n={n} T=4", flush=True)
    ntr = (n + 3) // 4
    assert ntr > 131072
    Ld = b2.B2SR.from_graph(g, 4, lower=True)
    A = b2.B2SR.from_graph(g, 4)
    assert int(b2.as_u64(b2.spgemm_masked(Ld, Ld, Ld))[0]) == n - 1
    assert int(b2.as_u64(b2.spgemm_masked(A, A, A))[0]) == 6 * (n - 1)
    # without the orientation workspace every mask tile scans Bt's row
    for X, ref in ((Ld, n - 1), (A, 6 * (n - 1))):
        plain = torch.zeros(1, dtype=torch.int64, device="cuda")
        assert b2.lib().spgemm_masked(X.view, X.view, X.view, 0, b2._ptr(plain), None, 0, b2._stream()) == 0
        assert int(b2.as_u64(plain)[0]) == ref
    assert int(b2.as_u64(b2.spgemm_masked_rows(Ld, Ld, Ld, ntr - 1, ntr))[0]) == n - 1
    assert int(b2.as_u64(b2.spgemm_masked_rows(Ld, Ld, Ld, 0, ntr - 1))[0]) == 0


@pytest.mark.parametrize("T", TILES)
def test_triangle_count_rmat18(T):
    g = gg.rmat(18, 16, seed=18)
    print(f"tc rmat18 T={T}", flush=True)
    assert b2.triangle_count(g.rowptr, g.colind, g.n, T) == orc.tc(g) == 82552366


def test_batched_full_config():
    """The 256-graph batch, 64 sources per graph, as the benchmark times it (one
    tile width for the batch, per-level and persistent launches) and with each
    graph's own autotuned width (several groups): sampled graphs' levels against
    the oracle; padding vertices stay unreached; both layouts give the same levels."""
    from paper_2201_08560_amd import autotune
    from paper_2201_08560_amd.batch import GraphBatch
    graphs = gg.chung_lu_batch(256, 2.1, seed=1000, workers=1)  # no fork of a process using the GPU
    sources = [gg.sample_sources(g, 64, seed=1000 + i) for i, g in enumerate(graphs)]
    sizes = np.array([g.n for g in graphs])
    sample = sorted({int(np.argmax(sizes)), int(np.argmin(sizes))} | set(gg.rng(9).choice(256, 6, replace=False).tolist()))
    per_graph = [autotune.choose_tile(g, nsample=256)[0] for g in graphs]
    batch_tile = autotune.choose_batch_tile(graphs)[0]
    ref = None  # (batch, levels) of the first run: every later run must agree graph by graph
    for tiles in ([batch_tile] * len(graphs), per_graph):
        B = GraphBatch(graphs, tiles)
        B.set_sources(sources)
        for mode in (b2.BATCH_LEVELS, b2.BATCH_PERSISTENT):
            lv, _ = B.run(mode)
            for i in sample:
                print(f"batch graph {i} n={graphs[i].n} T={tiles[i]} mode={mode}", flush=True)
                assert np.array_equal(B.levels_of_host(lv, i), orc.bfs_multi(graphs[i], B.sources[i]))
            pad = torch.cat([lv[int(B.offsets[i]) + g.n:int(B.offsets[i + 1])].reshape(-1)
                             for i, g in enumerate(graphs)])
            assert bool((pad == -1).all())  # 0xFFFFFFFF: unreached
            if ref is None:
                ref = (B, lv)
            else:
                assert all(torch.equal(B.levels_of(lv, i), ref[0].levels_of(ref[1], i)) for i in range(len(graphs)))


def test_local_clustering_full_size(big):
    """Sweep cut of a seeded score vector over all 2^20 vertices, bit-exact, and
    local clustering from the first benchmark source: personalised PageRank
    within 1e-5 relative L1 and a consistent cluster."""
    g, A = big["g"], big["A"]
    s = (gg.rng(4040).random(g.n) ** 4 * (gg.rng(4041).random(g.n) < 0.6)).astype(np.float32)
    print("sweep cut s20", flush=True)
    order, st = orc.sweep_cut(g, s)
    go, gbits, gst = b2.b2sr_sweep_cut(A, torch.from_numpy(s).cuda())
    assert gst == st and np.array_equal(b2.as_u32(go), order)
    c = np.zeros(g.n, bool)
    c[order[:st["size"]]] = True
    assert np.array_equal(unpack_bits(b2.as_u32(gbits), g.n), c)
    seed = int(big["sources"][0])
    print("lgc s20", flush=True)
    p, bits, st = b2.b2sr_lgc(A, seed, 0.85, 20)
    assert rel_l1(p.cpu().numpy(), orc.ppr(g, seed, 0.85, 20)) <= 1e-5
    cluster = unpack_bits(b2.as_u32(bits), g.n)
    deg = g.degrees().astype(np.int64)
    M = g.to_scipy().tocsr()
    cut = int((M[cluster] @ (~cluster).astype(np.int64)).sum())
    assert (st["size"], st["cut"], st["vol"], st["vol_all"]) == (int(cluster.sum()), cut, int(deg[cluster].sum()),
                                                                  int(deg.sum()))
