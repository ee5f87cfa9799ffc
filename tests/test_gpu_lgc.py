"""Local graph clustering on the GPU against the oracle, through the C ABI.

The sweep cut takes the same seeded float32 score vector on both sides and so
the same single-precision decisions: its order, statistics and cluster must be
bit-exact.  Personalised PageRank is a float32 sum against the float64 oracle:
relative L1 within 1e-5, as for PageRank.  Whole clusterings are compared
exactly where the answer is fixed by the graph (barbells, disjoint cliques, an
isolated seed) and otherwise checked for consistency: the returned cluster's
cut and volume, recomputed from the graph, match the reported ones."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as orc
from helpers import TILES, padding_zero, rel_l1, small_graphs, unpack_bits

pytestmark = pytest.mark.gpu
b2 = pytest.importorskip("paper_2201_08560_amd")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

GRAPHS = small_graphs() + [gg.king_grid(37, 41), gg.rmat(14, 8, seed=14)]
IDS = [g.name for g in GRAPHS]


def barbell(m: int):
    i, j = np.triu_indices(m, 1)
    return gg.canonical_csr(2 * m, np.concatenate([i, i + m, [m - 1]]), np.concatenate([j, j + m, [m]]),
                            name=f"barbell{m}")


def scores(n: int, kind: str, seed: int) -> np.ndarray:
    r = gg.rng(seed)
    if kind == "uniform":
        return (r.random(n) - 0.2).astype(np.float32)        # about a fifth not taken
    if kind == "ties":
        return r.integers(-1, 3, n).astype(np.float32)       # many equal quotients
    if kind == "sparse":
        return (r.random(n) ** 8 * (r.random(n) < 0.3)).astype(np.float32)
    s = r.random(n).astype(np.float32)                       # special values
    s[r.random(n) < 0.05] = np.inf
    s[r.random(n) < 0.05] = np.nan
    s[r.random(n) < 0.05] = -np.inf
    return s


def cluster_of(order, st, n):
    c = np.zeros(n, dtype=bool)
    c[order[:st["size"]]] = True
    return c


def cut_vol(g, cluster):
    A = g.to_scipy().tocsr()
    deg = g.degrees().astype(np.int64)
    inside = cluster.astype(np.int64)
    cut = int((A[cluster] @ (1 - inside)).sum()) if cluster.any() else 0
    return cut, int(deg[cluster].sum())


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_sweep_cut_bit_exact(gi, T):
    g = GRAPHS[gi]
    A = b2.B2SR.from_graph(g, T)
    for k, kind in enumerate(("uniform", "ties", "sparse", "special")):
        print(f"sweep {g.name} T={T} {kind}", flush=True)
        s = scores(g.n, kind, 5000 + 10 * gi + k)
        order, st = orc.sweep_cut(g, s)
        go, gbits, gst = b2.b2sr_sweep_cut(A, torch.from_numpy(s).cuda())
        assert gst == st
        assert np.array_equal(b2.as_u32(go), order)
        words = b2.as_u32(gbits)
        assert padding_zero(words, g.n)
        assert np.array_equal(unpack_bits(words, g.n), cluster_of(order, st, g.n))


@pytest.mark.parametrize("T", TILES)
def test_ppr_and_clusters_on_fixed_answers(T):
    for m in (5, 21, 40):
        g = barbell(m)
        A = b2.B2SR.from_graph(g, T)
        for seed in (0, m - 1):
            print(f"lgc barbell{m} T={T} seed={seed}", flush=True)
            p, bits, st = b2.b2sr_lgc(A, seed, 0.85, 30)
            assert rel_l1(p.cpu().numpy(), orc.ppr(g, seed, 0.85, 30)) <= 1e-5
            assert np.array_equal(unpack_bits(b2.as_u32(bits), g.n), np.arange(2 * m) < m)
            assert (st["size"], st["cut"], st["vol"], st["vol_all"]) == (m, 1, m * (m - 1) + 1, 2 * (m * (m - 1) + 1))
    u = gg.disjoint_union(gg.complete(6), gg.path(1), gg.complete(9))
    A = b2.B2SR.from_graph(u, T)
    _, bits, st = b2.b2sr_lgc(A, 8, 0.85, 10)
    assert np.array_equal(unpack_bits(b2.as_u32(bits), u.n), np.arange(u.n) >= 7) and st["cut"] == 0
    p, bits, st = b2.b2sr_lgc(A, 6, 0.85, 10)                # the isolated vertex
    assert st["size"] == 0 and st["taken"] == 0 and not unpack_bits(b2.as_u32(bits), u.n).any()
    restart = np.float32(1.0 - float(np.float32(0.85)))    # 1 - alpha, alpha taken as a float
    assert p.cpu().numpy()[6] == restart and np.count_nonzero(p.cpu().numpy()) == 1


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_lgc_ppr_and_consistency(gi, T):
    g = GRAPHS[gi]
    deg = g.degrees()
    if not (deg > 0).any():
        return
    A = b2.B2SR.from_graph(g, T)
    seed = int(np.flatnonzero(deg > 0)[len(np.flatnonzero(deg > 0)) // 3])
    for iters in (0, 1, 20):
        print(f"lgc {g.name} T={T} seed={seed} iters={iters}", flush=True)
        p, bits, st = b2.b2sr_lgc(A, seed, 0.85, iters)
        ph = p.cpu().numpy()
        assert rel_l1(ph, orc.ppr(g, seed, 0.85, iters)) <= 1e-5
        cluster = unpack_bits(b2.as_u32(bits), g.n)
        assert padding_zero(b2.as_u32(bits), g.n)
        assert cluster.sum() == st["size"] and st["vol_all"] == int(deg.sum())
        assert (st["cut"], st["vol"]) == cut_vol(g, cluster)
        if iters == 0:   # p = e_seed: the seed alone
            assert cluster.tolist() == (np.arange(g.n) == seed).tolist()


def test_sweep_without_order_output():
    g = gg.rmat(12, 8, seed=3)
    A = b2.B2SR.from_graph(g, 16)
    s = scores(g.n, "uniform", 77)
    order, st = orc.sweep_cut(g, s)
    go, gbits, gst = b2.b2sr_sweep_cut(A, torch.from_numpy(s).cuda(), order=False)
    assert go is None and gst == st
    assert np.array_equal(unpack_bits(b2.as_u32(gbits), g.n), cluster_of(order, st, g.n))
