"""Directed graphs on the GPU: the CSR transpose, and BFS, multi-source BFS,
SSSP and PageRank on the pull matrix (the transposed arc matrix) against the
oracle's directed answers; products on unsymmetric matrices."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as orc
from helpers import EPS32, TILES, pack_bits, rel_l1

pytestmark = pytest.mark.gpu
b2 = pytest.importorskip("paper_2201_08560_amd")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def digraphs():
    n = 1000
    return [
        gg.random_digraph(300, 0.02, 1),
        gg.rmat_directed(12, 8, seed=3),
        gg.directed_csr(n, np.arange(n - 1), np.arange(1, n), name="dir_path"),
        gg.directed_csr(5000, np.arange(1, 5000), np.zeros(4999, dtype=np.int64), name="in_star"),
        gg.directed_csr(4099, np.zeros(4098, dtype=np.int64), np.arange(1, 4099), name="out_star"),
        gg.directed_csr(10, [], [], name="empty10"),
    ]


GRAPHS = digraphs()
IDS = [g.name for g in GRAPHS]


@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_csr_transpose(gi):
    g = GRAPHS[gi]
    trp, tci = b2.b2sr_csr_transpose(g.n, g.rowptr, g.colind)
    trp, tci = b2.as_u32(trp), b2.as_u32(tci)
    t = gg.transpose(g)
    assert np.array_equal(trp, t.rowptr)
    for v in range(t.n):  # the order within a row is free
        assert np.array_equal(np.sort(tci[trp[v]:trp[v + 1]]), t.colind[t.rowptr[v]:t.rowptr[v + 1]]), v


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_directed_algorithms(gi, T):
    g = GRAPHS[gi]
    gt = gg.transpose(g)
    At = b2.B2SR.from_graph(g, T, transpose=True)
    srcs = np.unique(np.r_[0, gg.rng(gi).integers(0, g.n, 3), g.n - 1]).astype(np.uint32)
    for s in srcs:
        print(f"directed {g.name} T={T} src={s}", flush=True)
        assert np.array_equal(b2.as_u32(b2.b2sr_bfs(At, int(s))[0]), orc.bfs(g, int(s)))
        assert np.array_equal(b2.as_u32(b2.b2sr_sssp(At, int(s))[0]), orc.sssp_unit(gt, int(s)))
    lvm, _ = b2.b2sr_msbfs(At, srcs)
    assert np.array_equal(b2.as_u32(lvm), orc.bfs_multi(g, srcs))
    for iters in (1, 20):
        pr = b2.b2sr_pagerank_directed(At, 0.85, iters).cpu().numpy()
        assert rel_l1(pr, orc.pagerank_directed(g, 0.85, iters)) <= 1e-5


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_products_on_unsymmetric_matrices(gi, T):
    """y = A x on the arc matrix itself (not symmetric): bits, counts, plus-times, min-plus."""
    g = GRAPHS[gi]
    A = b2.B2SR.from_graph(g, T)
    r = gg.rng(300 + gi)
    x = r.random(g.n) < 0.3
    xd = torch.from_numpy(pack_bits(x).view(np.int32)).cuda()
    assert np.array_equal(b2.as_u32(b2.spmv_bin_bin(A, xd))[: (g.n + 31) // 32],
                          pack_bits(orc.spmv_or(g, x))[: (g.n + 31) // 32])
    assert np.array_equal(b2.as_u32(b2.spmv_bin_bin(A, xd, count=True)), orc.spmv_count(g, x))
    xf = r.random(g.n).astype(np.float32)
    y = b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, torch.from_numpy(xf).cuda()).cpu().numpy()
    ref = orc.spmv_plus(g, xf.astype(np.float64))
    bound = (g.degrees() + 2) * EPS32 * orc.spmv_plus(g, np.abs(xf).astype(np.float64)) + 1e-30
    assert np.all(np.abs(y - ref) <= bound)
    xm = np.where(r.random(g.n) < 0.5, r.integers(0, 50, g.n), np.inf).astype(np.float32)
    ym = b2.spmv_bin_full(A, b2.MIN_PLUS_F32, torch.from_numpy(xm).cuda(), alpha=1.0).cpu().numpy()
    assert np.array_equal(ym, orc.spmv_min_plus(g, xm.astype(np.float64), 1.0).astype(np.float32))
