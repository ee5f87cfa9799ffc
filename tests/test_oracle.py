"""Pins for the CPU oracle: brute force, closed forms, the paper's worked example
and independent library routines.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen as gg
import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TILES = (4, 8, 16, 32)
TILES64 = TILES + (64,)  # B2SR-64: the 64-bit packing type of Sec. III-A
UNR = orc.UNREACHED


def tiny_graphs(count=60, seed0=0):
    out = []
    for s in range(count):
        r = gg.rng(10_000 + s)
        n = int(r.integers(1, 65))
        p = float(r.choice([0.02, 0.08, 0.2, 0.5, 0.9]))
        out.append(gg.random_graph_tiny(n, p, seed0 + s))
    return out


TINY = tiny_graphs()


# ---------------------------------------------------------------- B2SR by definition

def decode_b2sr(n, T, trp, tci, bits):
    """Independent decode of B2SR arrays into a dense 0/1 matrix."""
    a = np.zeros((len(trp) - 1) * T, dtype=np.uint8)
    a = np.zeros((a.size, a.size if a.size else 0), dtype=np.uint8)
    for I in range(len(trp) - 1):
        for t in range(int(trp[I]), int(trp[I + 1])):
            J = int(tci[t])
            for r in range(T):
                w = int(bits[t * T + r])
                for c in range(T):
                    if (w >> c) & 1:
                        a[I * T + r, J * T + c] = 1
    return a[:n, :n]


# graphs spanning several 64-row tile-rows, with a ragged last one
SMALL = [gg.random_graph_tiny(int(gg.rng(20_000 + s).integers(65, 300)), p, 300 + s)
         for s, p in enumerate([0.01, 0.03, 0.1, 0.3, 0.6, 0.02, 0.05, 0.2])]


@pytest.mark.parametrize("T", TILES64)
def test_b2sr_build_brute_force(T):
    for g in TINY[:40] + SMALL:
        for lower in (False, True):
            trp, tci, bits = orc.b2sr_build(g, T, lower_only=lower)
            dense = g.dense()
            if lower:
                dense = np.tril(dense, -1)
            ii, jj = np.nonzero(dense)
            pairs = np.unique(np.stack([ii // T, jj // T], 1), axis=0) if ii.size else np.zeros((0, 2))
            assert len(tci) == len(pairs) == orc.b2sr_count_tiles(g, T, lower)
            assert trp[0] == 0 and np.all(np.diff(trp.astype(np.int64)) >= 0)
            ntr = (g.n + T - 1) // T
            assert len(trp) == ntr + 1
            # tile columns strictly ascending inside each tile-row, and equal to the pair set
            got = []
            for I in range(ntr):
                cols = tci[trp[I]:trp[I + 1]]
                assert np.all(np.diff(cols.astype(np.int64)) > 0)
                got += [(I, int(c)) for c in cols]
            assert got == [tuple(map(int, p)) for p in pairs]
            assert np.array_equal(decode_b2sr(g.n, T, trp, tci, bits), dense)
            # padding bits beyond n are zero (decode above cut them; check directly)
            if T == 4:
                assert np.all(bits < 16)


def test_mycielskian12_storage_matches_paper():
    """Sec. III-C worked example: CSR and B2SR-4/8/16/32 byte sizes of mycielskian12."""
    with open(os.path.join(GOLDEN, "mycielskian12_storage.json")) as f:
        gold = json.load(f)
    g = gg.mycielski(12)
    assert g.n == 3071 and g.edges == 203600
    assert round(orc.csr_bytes(g.nnz, g.n) / 2**20, 2) == gold["csr_MB"]
    for T in TILES:
        nt = orc.b2sr_count_tiles(g, T)
        kib = orc.b2sr_bytes(nt, g.n, T) / 1024
        assert round(kib, 2) == pytest.approx(gold["b2sr_KB"][str(T)], abs=1e-9), T


def test_b2sr64_closed_forms():
    """B2SR-64 (no printed number pins T = 64): tile words written out by hand
    for graphs whose bit patterns are known, and the byte formula of the three
    arrays (4-byte indices, 8-byte bit-rows)."""
    full = (1 << 64) - 1
    # K_64: one tile, bit-row r is every column but the diagonal
    trp, tci, bits = orc.b2sr_build(gg.complete(64), 64)
    assert trp.tolist() == [0, 1] and tci.tolist() == [0]
    assert bits.dtype == np.uint64 and [int(w) for w in bits] == [full ^ (1 << r) for r in range(64)]
    # K_130: 3 x 3 tiles; the last tile-row and column hold 2 vertices
    g = gg.complete(130)
    trp, tci, bits = orc.b2sr_build(g, 64)
    assert trp.tolist() == [0, 3, 6, 9] and tci.tolist() == [0, 1, 2] * 3
    w = [int(v) for v in bits]
    assert w[2 * 64 + 5] == 0b11 and w[8 * 64 + 1] == 0b01 and w[8 * 64 + 2] == 0  # padding rows are zero
    assert w[4 * 64 + 7] == full ^ (1 << 7) and w[1 * 64 + 0] == full
    assert orc.b2sr_bytes(9, 130, 64) == 4 * 4 + 4 * 9 + 9 * 64 * 8
    # path on 200 vertices: 4 diagonal tiles and 3 pairs of corner tiles
    trp, tci, bits = orc.b2sr_build(gg.path(200), 64)
    assert trp.tolist() == [0, 2, 5, 8, 10] and tci.tolist() == [0, 1, 0, 1, 2, 1, 2, 3, 2, 3]
    w = [int(v) for v in bits]
    assert w[0 * 64 + 0] == 0b10 and w[0 * 64 + 5] == (1 << 4) | (1 << 6) and w[0 * 64 + 63] == 1 << 62
    assert w[1 * 64 + 63] == 1 and sum(w[64:128]) == 1  # (63, 64) in tile (0, 1)
    assert w[2 * 64 + 0] == 1 << 63  # (64, 63) in tile (1, 0)
    # the lower triangle of K_64 keeps bits below the diagonal only
    _, _, bits = orc.b2sr_build(gg.complete(64), 64, lower_only=True)
    assert [int(v) for v in bits] == [(1 << r) - 1 for r in range(64)]


def test_mycielski_edge_recurrence_and_triangle_free():
    e, n = 1, 2
    for k in range(2, 11):
        g = gg.mycielski(k)
        assert (g.n, g.edges) == (n, e)
        e, n = 3 * e + n, 2 * n + 1
    for k in (4, 6, 9):
        g = gg.mycielski(k)
        assert orc.tc(g) == 0
        assert orc.masked_sum(orc.tril(g), orc.tril(g), orc.tril(g)) == 0
        assert np.all(orc.cc(g) == 0)


def test_tile_count_against_numpy_pairs_medium():
    g = gg.er_gnm(3000, 9000, seed=5)
    rows = np.repeat(np.arange(g.n), g.degrees())
    for T in TILES64:
        key = (rows // T) * ((g.n + T - 1) // T) + g.colind // T
        assert orc.b2sr_count_tiles(g, T) == np.unique(key).size


# ---------------------------------------------------------------- products vs brute force

@pytest.mark.parametrize("complement", [False, True])
def test_spmv_or_count_brute_force(complement):
    for s, g in enumerate(TINY):
        r = gg.rng(s)
        x = r.random(g.n) < 0.3
        m = r.random(g.n) < 0.5
        A = g.dense().astype(np.int64)
        keep = ~m if complement else m
        cnt = A @ x.astype(np.int64)
        assert np.array_equal(orc.spmv_or(g, x, m, complement), (cnt > 0) & keep)
        assert np.array_equal(orc.spmv_count(g, x, m, complement), np.where(keep, cnt, 0))
        assert np.array_equal(orc.spmv_or(g, x), cnt > 0)
        assert np.array_equal(orc.spmv_count(g, x), cnt)


def test_spmv_invariants_all_ones():
    g = gg.er_gnm(2000, 5000, seed=3)
    ones = np.ones(g.n, dtype=bool)
    assert np.array_equal(orc.spmv_count(g, ones), g.degrees())
    assert np.array_equal(orc.spmv_or(g, ones), g.degrees() > 0)


def test_spmv_plus_brute_force():
    for s, g in enumerate(TINY):
        r = gg.rng(100 + s)
        # integer-valued inputs make every sum exact, so the comparison is exact
        x = r.integers(-50, 50, g.n).astype(np.float64)
        sc = r.integers(1, 5, g.n).astype(np.float64)
        A = g.dense().astype(np.float64)
        assert np.array_equal(orc.spmv_plus(g, x), A @ x)
        assert np.array_equal(orc.spmv_plus(g, x, sc), A @ (x * sc))
        m = r.random(g.n) < 0.5
        assert np.array_equal(orc.spmv_plus(g, x, None, m, True), np.where(~m, A @ x, 0.0))


def test_spmv_plus_scipy_medium():
    g = gg.er_gnm(4096, 16384, seed=1)
    x = gg.rng(7).random(g.n)
    ref = g.to_scipy().astype(np.float64) @ x
    np.testing.assert_allclose(orc.spmv_plus(g, x), ref, rtol=1e-13, atol=0)


def test_spmv_min_plus_brute_force():
    for s, g in enumerate(TINY):
        r = gg.rng(200 + s)
        x = r.integers(0, 20, g.n).astype(np.float64)
        x[r.random(g.n) < 0.2] = np.inf
        A = g.dense().astype(bool)
        for w in (0.0, 1.0, 2.5):
            cand = np.where(A, x[None, :] + w, np.inf)
            best = cand.min(axis=1) if g.n else cand.sum(axis=1)
            assert np.array_equal(orc.spmv_min_plus(g, x, w, False), best)
            assert np.array_equal(orc.spmv_min_plus(g, x, w, True), np.minimum(best, x))
        m = r.random(g.n) < 0.5
        got = orc.spmv_min_plus(g, x, 1.0, True, m, False)
        ref = np.where(m, np.minimum(np.where(A, x[None, :] + 1, np.inf).min(axis=1, initial=np.inf), x), np.inf)
        assert np.array_equal(got, ref)


def test_spmv_or64_brute_force():
    for s, g in enumerate(TINY[:30]):
        r = gg.rng(300 + s)
        x = r.integers(0, 2**63, g.n, dtype=np.uint64) & r.integers(0, 2**63, g.n, dtype=np.uint64)
        v = r.integers(0, 2**63, g.n, dtype=np.uint64)
        A = g.dense().astype(bool)
        ref = np.array([np.bitwise_or.reduce(x[A[i]]) if A[i].any() else 0 for i in range(g.n)],
                       dtype=np.uint64)
        assert np.array_equal(orc.spmv_or64(g, x), ref)
        assert np.array_equal(orc.spmv_or64(g, x, v), ref & ~v)
        # bit b of the 64-wide product equals the Boolean product of bit b
        for b in (0, 17, 63):
            xb = ((x >> np.uint64(b)) & np.uint64(1)).astype(bool)
            yb = ((ref >> np.uint64(b)) & np.uint64(1)).astype(bool)
            assert np.array_equal(orc.spmv_or(g, xb), yb)


def directed_csr(dense):
    """CSR of an arbitrary (non-symmetric) 0/1 matrix, columns ascending."""
    n = dense.shape[0]
    rows, cols = np.nonzero(dense)
    rp = np.zeros(n + 1, dtype=np.uint32)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return gg.Csr(n, rp, cols.astype(np.uint32), "directed")


def test_masked_sum_brute_force():
    for s in range(40):
        r = gg.rng(900 + s)
        n = int(r.integers(1, 50))
        A, B, M = ((r.random((n, n)) < p).astype(np.int64) for p in (0.3, 0.25, 0.4))
        a, bt, m = directed_csr(A), directed_csr(B.T), directed_csr(M)
        P = A @ B
        assert orc.masked_sum(a, bt, m) == int((P * M).sum())
        assert orc.masked_sum(a, bt) == int(P.sum())
    for g in TINY[:30]:
        A = g.dense().astype(np.int64)
        assert orc.masked_sum(g, g, g) == int(np.trace(A @ A @ A))


def test_masked_sum_closed_forms():
    for n in (3, 5, 12, 33):
        K = gg.complete(n)
        L = orc.tril(K)
        assert orc.masked_sum(L, L, L) == math.comb(n, 3)
        assert orc.masked_sum(K, K, K) == 6 * math.comb(n, 3)
        assert orc.masked_sum(K, K) == n * (n - 1) ** 2
    g = gg.mycielski(8)
    deg = g.degrees().astype(np.int64)
    assert orc.masked_sum(g, g) == int((deg ** 2).sum())


def test_tc_closed_forms_and_brute_force():
    for n in (3, 4, 10, 40):
        assert orc.tc(gg.complete(n)) == math.comb(n, 3)
    for R, C in ((2, 2), (3, 7), (20, 31)):
        assert orc.tc(gg.king_grid(R, C)) == 4 * (R - 1) * (C - 1)
    for g in (gg.path(50), gg.star(40), gg.grid4(9, 11), gg.cycle(30)):
        assert orc.tc(g) == 0
    assert orc.tc(gg.cycle(3)) == 1
    # wheels (rim cycle 0..n-2, hub n-1): n - 1 triangles, all holding the hub,
    # the largest id; the A.A masked sum counts each of them 6 times
    for n in (5, 9, 64, 300):
        w = gg.wheel(n)
        A = w.dense().astype(np.int64)
        assert orc.tc(w) == n - 1 == int(np.trace(A @ A @ A)) // 6
        assert orc.masked_sum(w, w, w) == 6 * (n - 1)
        L = orc.tril(w)
        hub_rows = gg.directed_csr(n, np.full(n - 1, n - 1), np.arange(n - 1))  # L's hub row alone
        assert orc.masked_sum(L, L, hub_rows) == n - 1
    for g in TINY:
        A = g.dense().astype(np.int64)
        assert orc.tc(g) == int(np.trace(A @ A @ A)) // 6
        L = orc.tril(g)
        assert orc.masked_sum(L, L, L) == orc.tc(g)


# ---------------------------------------------------------------- algorithms

def bfs_dense(g, src):
    A = g.dense().astype(bool)
    lv = np.full(g.n, UNR, dtype=np.uint32)
    lv[src] = 0
    front = np.zeros(g.n, dtype=bool)
    front[src] = True
    seen = front.copy()
    k = 0
    while front.any():
        k += 1
        nxt = (A[:, front].any(axis=1)) & ~seen
        lv[nxt] = k
        seen |= nxt
        front = nxt
    return lv


def test_bfs_brute_force_and_sssp_equals_bfs():
    for s, g in enumerate(TINY):
        if g.n == 0:
            continue
        src = int(gg.rng(s).integers(0, g.n))
        lv = orc.bfs(g, src)
        assert np.array_equal(lv, bfs_dense(g, src))
        assert np.array_equal(orc.sssp_unit(g, src), lv)


def test_bfs_closed_forms():
    n = 57
    assert np.array_equal(orc.bfs(gg.path(n), 13), np.abs(np.arange(n) - 13).astype(np.uint32))
    st = gg.star(20)
    assert np.array_equal(orc.bfs(st, 0), np.r_[0, np.ones(19)].astype(np.uint32))
    lv = orc.bfs(st, 5)
    assert lv[5] == 0 and lv[0] == 1 and np.all(np.delete(lv, [0, 5]) == 2)
    R, C = 13, 17
    r, c = np.divmod(np.arange(R * C), C)
    s = 4 * C + 9
    assert np.array_equal(orc.bfs(gg.grid4(R, C), s), (np.abs(r - 4) + np.abs(c - 9)).astype(np.uint32))
    assert np.array_equal(orc.bfs(gg.king_grid(R, C), s),
                          np.maximum(np.abs(r - 4), np.abs(c - 9)).astype(np.uint32))
    assert np.array_equal(orc.sssp_unit(gg.king_grid(R, C), s),
                          np.maximum(np.abs(r - 4), np.abs(c - 9)).astype(np.uint32))
    K = orc.bfs(gg.complete(9), 3)
    assert K[3] == 0 and np.all(np.delete(K, 3) == 1)
    u = gg.disjoint_union(gg.path(5), gg.path(4))
    assert np.all(orc.bfs(u, 0)[5:] == UNR)


def test_bfs_scipy_medium():
    g = gg.er_gnm(4096, 16384, seed=1)
    d = csg.shortest_path(g.to_scipy(), unweighted=True, indices=[0, 77])
    for k, src in enumerate((0, 77)):
        ref = np.where(np.isinf(d[k]), UNR, d[k]).astype(np.uint32)
        assert np.array_equal(orc.bfs(g, src), ref)
    multi = orc.bfs_multi(g, np.array([0, 77], dtype=np.uint32))
    assert np.array_equal(multi[1], orc.bfs(g, 77))


def cc_dense(g):
    A = g.dense().astype(bool) | np.eye(g.n, dtype=bool)
    R = A.copy()
    while True:
        R2 = (R.astype(np.int64) @ R.astype(np.int64)) > 0
        if np.array_equal(R2, R):
            break
        R = R2
    return np.array([np.flatnonzero(R[i]).min() for i in range(g.n)], dtype=np.uint32)


def test_cc_brute_force_and_unions():
    for g in TINY:
        assert np.array_equal(orc.cc(g), cc_dense(g))
    u = gg.disjoint_union(gg.path(5), gg.complete(4), gg.star(3), gg.cycle(6))
    lab = orc.cc(u)
    assert np.array_equal(lab, np.r_[[0] * 5, [5] * 4, [9] * 3, [12] * 6].astype(np.uint32))


def test_cc_scipy_medium():
    g = gg.rmat(12, 4, seed=3)
    ncomp, lab = csg.connected_components(g.to_scipy(), directed=False)
    mins = np.full(ncomp, g.n, dtype=np.int64)
    np.minimum.at(mins, lab, np.arange(g.n))
    assert np.array_equal(orc.cc(g), mins[lab].astype(np.uint32))


def pagerank_dense(g, d, iters):
    A = g.dense().astype(np.float64)
    deg = A.sum(axis=1)
    inv = np.divide(1.0, deg, out=np.zeros_like(deg), where=deg > 0)
    r = np.full(g.n, 1.0 / g.n)
    for _ in range(iters):
        r = (1 - d) / g.n + d * (A @ (r * inv))
    return r


def test_pagerank_brute_force():
    for g in TINY:
        if g.n == 0:
            continue
        np.testing.assert_allclose(orc.pagerank(g, 0.85, 20), pagerank_dense(g, 0.85, 20),
                                   rtol=1e-12, atol=1e-15)


def test_pagerank_regular_graphs_stay_uniform():
    for g in (gg.cycle(100), gg.complete(31), gg.torus(8, 12)):
        for k in (1, 7, 20):
            np.testing.assert_allclose(orc.pagerank(g, 0.85, k), 1.0 / g.n, rtol=1e-13)


def test_pagerank_mass_invariant_with_dangling():
    g = gg.disjoint_union(gg.rmat(10, 4, seed=2), gg.path(1), gg.path(1))
    deg = g.degrees()
    d = 0.85
    for k in (1, 2, 5):
        r_prev = orc.pagerank(g, d, k - 1)
        r = orc.pagerank(g, d, k)
        np.testing.assert_allclose(r.sum(), (1 - d) + d * r_prev[deg > 0].sum(), rtol=1e-13)


def test_thread_count_independence():
    g = gg.rmat(13, 8, seed=4)
    t0 = orc.num_threads()
    try:
        orc.set_num_threads(1)
        a = (orc.pagerank(g, 0.85, 5), orc.tc(g), orc.spmv_count(g, np.ones(g.n, bool)))
        orc.set_num_threads(max(2, t0))
        b = (orc.pagerank(g, 0.85, 5), orc.tc(g), orc.spmv_count(g, np.ones(g.n, bool)))
    finally:
        orc.set_num_threads(t0)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[2], b[2])


# ---------------------------------------------------------------- planted mistakes fail the pins

def test_pins_catch_planted_mistakes():
    """Each pin above is sensitive: a plausibly wrong variant of the definition,
    planted here on the CPU, disagrees with it."""
    g = gg.complete(10)
    # dropping the self term in min-plus changes SSSP fixpoints on a path
    p = gg.path(6)
    x = np.array([0, np.inf, np.inf, np.inf, np.inf, np.inf])
    assert not np.array_equal(orc.spmv_min_plus(p, x, 1.0, False), orc.spmv_min_plus(p, x, 1.0, True))
    # counting nonzero output entries instead of summing products breaks K_n
    A = g.dense().astype(np.int64)
    L = np.tril(A, -1)
    boolean_count = int(((L @ L.T) > 0).astype(np.int64)[L > 0].sum())
    assert boolean_count != math.comb(10, 3) == orc.tc(g)
    # passing B instead of its transpose changes a non-symmetric product
    r = gg.rng(5)
    A = (r.random((30, 30)) < 0.3).astype(np.int64)
    B = (r.random((30, 30)) < 0.3).astype(np.int64)
    M = (r.random((30, 30)) < 0.5).astype(np.int64)
    right = orc.masked_sum(directed_csr(A), directed_csr(B.T), directed_csr(M))
    wrong = orc.masked_sum(directed_csr(A), directed_csr(B), directed_csr(M))
    assert right == int(((A @ B) * M).sum()) != wrong


# ---- directed graphs -----------------------------------------------------------

def test_transpose_generator():
    for g in (gg.random_digraph(40, 0.1, 3), gg.rmat_directed(8, 8, seed=2), gg.path(30)):
        t = gg.transpose(g)
        assert np.array_equal(t.dense(), g.dense().T)
        tt = gg.transpose(t)
        assert np.array_equal(tt.rowptr, g.rowptr) and np.array_equal(tt.colind, g.colind)


def test_directed_bfs_pins():
    """BFS along arcs: a directed path reaches forward only; BFS (push along the
    arc rows) equals unit-weight Bellman-Ford pulled over the reversed rows."""
    n = 50
    p = gg.directed_csr(n, np.arange(n - 1), np.arange(1, n))
    assert np.array_equal(orc.bfs(p, 0), np.arange(n, dtype=np.uint32))
    lv = orc.bfs(p, 20)
    assert np.all(lv[:20] == UNR) and np.array_equal(lv[20:], np.arange(n - 20, dtype=np.uint32))
    for seed in range(4):
        g = gg.random_digraph(60, 0.04, 100 + seed)
        gt = gg.transpose(g)
        for s in (0, 7, 59):
            assert np.array_equal(orc.bfs(g, s), orc.sssp_unit(gt, s))


def test_directed_pagerank_pins():
    d = 0.85
    # an undirected graph given as both arcs of every edge: the undirected PageRank
    g = gg.er_gnm(200, 700, seed=5)
    assert np.allclose(orc.pagerank_directed(g, d, 15), orc.pagerank(g, d, 15), rtol=1e-13, atol=0)
    # a directed cycle keeps the uniform vector
    n = 17
    cyc = gg.directed_csr(n, np.arange(n), (np.arange(n) + 1) % n)
    assert np.allclose(orc.pagerank_directed(cyc, d, 9), np.full(n, 1.0 / n), rtol=1e-14, atol=0)
    # an inward star: leaves keep (1-d)/n; the centre, a sink, gets d (n-1)/n, then d (n-1)(1-d)/n
    n = 9
    star = gg.directed_csr(n, np.arange(1, n), np.zeros(n - 1, dtype=np.int64))
    r1, r2 = orc.pagerank_directed(star, d, 1), orc.pagerank_directed(star, d, 2)
    assert np.allclose(r1[1:], (1 - d) / n) and np.isclose(r1[0], (1 - d) / n + d * (n - 1) / n)
    assert np.allclose(r2[1:], (1 - d) / n) and np.isclose(r2[0], (1 - d) / n + d * (n - 1) * (1 - d) / n)
    # small random digraphs: the matrix form r' = (1-d)/n + d P (r / o), P = A^T
    for seed in range(3):
        g = gg.random_digraph(30, 0.1, 40 + seed)
        A = g.dense().astype(np.float64)
        o = A.sum(1)
        r = np.full(g.n, 1.0 / g.n)
        for _ in range(6):
            r = (1 - d) / g.n + d * A.T @ np.divide(r, o, out=np.zeros_like(r), where=o > 0)
        assert np.allclose(orc.pagerank_directed(g, d, 6), r, rtol=1e-12, atol=0)


# ---- max-times: MIS and colouring (Table V) ------------------------------------

def _keys(n, seed):
    r = np.random.default_rng(seed).integers(0, 1 << 31, size=n, dtype=np.uint64)
    return (r << np.uint64(32)) | (np.arange(n, dtype=np.uint64) + np.uint64(1))


def test_spmv_max_brute_force():
    for seed in range(3):
        g = gg.random_graph_tiny(40, 0.15, 900 + seed)
        x = np.random.default_rng(seed).integers(0, 1 << 62, size=g.n, dtype=np.uint64)
        x[::3] = 0
        A = g.dense().astype(bool)
        exp = np.array([x[A[i]].max() if A[i].any() else 0 for i in range(g.n)], dtype=np.uint64)
        assert np.array_equal(orc.spmv_max(g, x), exp)


def _independent_and_maximal(g, inset, among=None):
    A = g.dense().astype(bool)
    among = np.ones(g.n, bool) if among is None else among
    assert not (A & np.outer(inset, inset)).any()                       # independent
    covered = inset | (A[:, inset].any(1) if inset.any() else np.zeros(g.n, bool))
    assert np.all(covered[among])                                       # maximal among the candidates


def test_mis_pins():
    for seed in range(6):
        g = gg.random_graph_tiny(60, 0.08, 950 + seed)
        k = _keys(g.n, seed)
        m, rounds = orc.mis(g, k)
        assert np.array_equal(m, orc.mis_greedy(g, k))   # rounds of local maxima == sequential greedy
        _independent_and_maximal(g, m)
        assert rounds >= 1
    n = 30
    K = gg.complete(n)
    k = _keys(n, 1)
    assert np.flatnonzero(orc.mis(K, k)[0]).tolist() == [int(np.argmax(k))]
    p = gg.path(n)
    up = np.arange(1, n + 1, dtype=np.uint64)           # keys increase along the path
    assert np.flatnonzero(orc.mis(p, up)[0]).tolist() == list(range(n - 1, -1, -2))[::-1]
    s = gg.star(10)                                      # vertex 0 is the centre
    hi = np.r_[100, np.arange(1, 10)].astype(np.uint64)
    lo = np.r_[1, np.arange(2, 11)].astype(np.uint64)
    assert np.flatnonzero(orc.mis(s, hi)[0]).tolist() == [0]
    assert np.flatnonzero(orc.mis(s, lo)[0]).tolist() == list(range(1, 10))
    e = gg.canonical_csr(5, [], [])
    assert orc.mis(e, _keys(5, 2))[0].all()
    z = _keys(5, 3)
    z[2] = 0                                             # key 0: never a candidate
    assert not orc.mis(e, z)[0][2]


def test_color_pins():
    for seed in range(5):
        g = gg.random_graph_tiny(50, 0.1, 970 + seed)
        k = _keys(g.n, seed)
        col, nc = orc.color(g, k)
        A = g.dense().astype(bool)
        assert np.all(col < nc)
        assert not (A & (col[:, None] == col[None, :])).any()          # proper
        for c in range(nc):                                             # class c: MIS of what was left
            _independent_and_maximal(g, col == c, among=col >= c)
        assert nc <= int(g.degrees().max(initial=0)) + 1
    K = gg.complete(12)
    col, nc = orc.color(K, _keys(12, 4))
    assert nc == 12 and sorted(col.tolist()) == list(range(12))
    e = gg.canonical_csr(7, [], [])
    col, nc = orc.color(e, _keys(7, 5))
    assert nc == 1 and not col.any()


def test_eccentricity_closed_forms():
    n = 41
    p = gg.path(n)
    assert np.array_equal(orc.eccentricity(p, np.arange(n)), np.maximum(np.arange(n), n - 1 - np.arange(n)))
    c = gg.cycle(n)
    assert np.all(orc.eccentricity(c, np.arange(n)) == n // 2)
    s = gg.star(12)                                  # vertex 0 is the centre
    assert orc.eccentricity(s, [0, 1, 5]).tolist() == [1, 2, 2]
    assert np.all(orc.eccentricity(gg.complete(9), np.arange(9)) == 1)
    k = gg.king_grid(7, 11)                          # Chebyshev distance from a corner
    assert orc.eccentricity(k, [0])[0] == 10 and orc.diameter(k) == 10
    u = gg.disjoint_union(gg.path(5), gg.path(1), gg.cycle(8))
    assert orc.eccentricity(u, [0, 5, 6]).tolist() == [4, 0, 4]
    assert orc.diameter(u) == 4
    # brute force on small random graphs: all-pairs BFS distances
    for seed in range(3):
        g = gg.random_graph_tiny(40, 0.08, 990 + seed)
        D = csg.shortest_path(g.to_scipy(), unweighted=True, directed=False)
        D[np.isinf(D)] = -1
        assert np.array_equal(orc.eccentricity(g, np.arange(g.n)), D.max(1).astype(np.uint32))


# ---- local graph clustering: personalised PageRank and the sweep cut ------------

def barbell(m: int):
    """Two copies of K_m (vertices 0..m-1 and m..2m-1) joined by the edge (m-1, m)."""
    i, j = np.triu_indices(m, 1)
    src = np.concatenate([i, i + m, [m - 1]])
    dst = np.concatenate([j, j + m, [m]])
    return gg.canonical_csr(2 * m, src, dst, name=f"barbell{m}")


def walk_matrix(g):
    """P = A D^-1 as a dense matrix (zero columns at degree-0 vertices)."""
    A = g.dense().astype(np.float64)
    deg = A.sum(0)
    return A / np.where(deg > 0, deg, 1.0)


def test_ppr_matches_the_matrix_power_series():
    """K steps from e_s give (aP)^K e_s + (1-a) sum_{k<K} (aP)^k e_s."""
    a = 0.85
    for g in TINY[:30]:
        if g.n == 0:
            continue
        s = g.n // 2
        aP = a * walk_matrix(g)
        e = np.zeros(g.n)
        e[s] = 1.0
        for K in (0, 1, 6):
            want = np.linalg.matrix_power(aP, K) @ e
            want += (1 - a) * sum(np.linalg.matrix_power(aP, k) @ e for k in range(K))
            np.testing.assert_allclose(orc.ppr(g, s, a, K), want, rtol=1e-12, atol=1e-15)


def test_ppr_fixed_point_and_mass():
    a = 0.7
    g = gg.random_graph_tiny(50, 0.15, 4242)
    s = 3
    # far enough out, the iteration sits on the solution of (I - aP) p = (1 - a) e_s
    e = np.zeros(g.n)
    e[s] = 1.0
    want = np.linalg.solve(np.eye(g.n) - a * walk_matrix(g), (1 - a) * e)
    np.testing.assert_allclose(orc.ppr(g, s, a, 300), want, rtol=1e-10, atol=1e-14)
    # without degree-0 vertices the walk keeps all of the mass
    k = gg.king_grid(9, 13)
    for K in (1, 5, 40):
        assert abs(orc.ppr(k, 17, 0.85, K).sum() - 1.0) < 1e-12
    # an isolated seed keeps 1 - a after the first step and nothing else moves
    u = gg.disjoint_union(gg.path(1), gg.cycle(6))
    p = orc.ppr(u, 0, 0.85, 4)
    assert p[0] == pytest.approx(0.15, abs=1e-15) and np.all(p[1:] == 0)


def sweep_brute_force(g, score):
    """Every prefix's conductance from the set itself, compared as exact fractions."""
    from fractions import Fraction
    A = g.dense().astype(np.int64)
    deg = A.sum(1)
    q = np.where(deg > 0, score.astype(np.float32) / np.maximum(deg, 1).astype(np.float32), np.float32(0))
    taken = [v for v in range(g.n) if deg[v] > 0 and q[v] > 0]
    taken.sort(key=lambda v: (-float(q[v]), v))
    vol_all = int(deg.sum())
    best = None
    for k in range(1, len(taken) + 1):
        S = np.zeros(g.n, bool)
        S[taken[:k]] = True
        cut = int(A[S][:, ~S].sum())
        vol = int(deg[S].sum())
        den = min(vol, vol_all - vol)
        if den and (best is None or Fraction(cut, den) < best[0]):
            best = (Fraction(cut, den), k, cut, vol)
    return taken, best


def test_sweep_cut_brute_force():
    r = gg.rng(777)
    for g in TINY[:40]:
        for kind in ("continuous", "ties"):
            if kind == "continuous":
                score = r.random(g.n).astype(np.float32) - np.float32(0.2)   # some negative: not taken
            else:
                score = r.integers(-1, 3, g.n).astype(np.float32)          # many equal quotients
            order, st = orc.sweep_cut(g, score)
            taken, best = sweep_brute_force(g, score)
            assert order[:len(taken)].tolist() == taken and st["taken"] == len(taken)
            rest = sorted(set(range(g.n)) - set(taken))
            assert order[len(taken):].tolist() == rest
            assert st["vol_all"] == int(g.degrees().sum())
            if best is None:
                assert (st["size"], st["cut"], st["vol"]) == (0, 0, 0)
            else:
                assert (st["size"], st["cut"], st["vol"]) == best[1:]


def test_lgc_closed_forms():
    for m in (5, 12):
        g = barbell(m)
        for seed in (0, m - 1):                       # inside clique 1, and its bridge end
            _, cluster, st = orc.lgc(g, seed, 0.85, 30)
            assert cluster.tolist() == [True] * m + [False] * m
            assert (st["cut"], st["vol"]) == (1, m * (m - 1) + 1)
            assert st["conductance"] == 1 / (m * (m - 1) + 1)
    # a seed's own component is a cluster of conductance 0
    u = gg.disjoint_union(gg.complete(6), gg.complete(9))
    _, cluster, st = orc.lgc(u, 8, 0.85, 10)
    assert cluster.tolist() == [False] * 6 + [True] * 9 and st["cut"] == 0 and st["conductance"] == 0
    # an isolated seed gives no candidate prefix
    _, cluster, st = orc.lgc(gg.disjoint_union(gg.path(1), gg.cycle(5)), 0, 0.85, 10)
    assert st["size"] == 0 and st["taken"] == 0 and not cluster.any()


def test_sweep_pins_catch_planted_mistakes():
    """A sweep that orders by the raw score, not score / degree, or that counts an
    edge into S as crossing, disagrees with the brute force."""
    g = barbell(6)
    score = np.ones(g.n, np.float32)
    score[[0, 1]] = 2.0
    score[5] = 1.1                                  # the bridge end: degree 6, the others 5
    taken, best = sweep_brute_force(g, score)
    assert taken[:3] == [0, 1, 2]                   # 1.1 / 6 < 1 / 5: vertex 5 comes after the unit scores
    assert orc.sweep_cut(g, score)[0][:len(taken)].tolist() == taken
    raw = sorted((v for v in range(g.n)), key=lambda v: (-float(score[v]), v))
    assert raw[:3] == [0, 1, 5]
    # counting every edge of the joining vertex as crossing overstates the cut
    A = g.dense().astype(np.int64)
    S = np.zeros(g.n, bool)
    S[:6] = True
    assert int(A[S][:, ~S].sum()) == 1 != int(A[S].sum())
