"""GPU parity: the HIP path through the C ABI against the CPU oracle, on seeded
inputs of several tiles with ragged tails and the degenerate cases.

Integer, bit and min-plus results must be bit-exact.  Float sums follow the
bound of a float32 sum of m non-negative-magnitude terms (each term rounded once
and every partial sum rounded once): |y - y_exact| <= (m + 2) * 2^-24 * sum|terms|,
plus one rounding each for the alpha and beta terms.  PageRank must match the
float64 oracle within 1e-5 relative L1.
"""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle as orc
from helpers import EPS32, TILES, UNR, pack_bits, padding_zero, rel_l1, small_graphs, unpack_bits

pytestmark = pytest.mark.gpu

b2 = pytest.importorskip("paper_2201_08560_amd")

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

GRAPHS = small_graphs()
IDS = [g.name for g in GRAPHS]


def dev_u32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


_cache = {}


def b2sr(g, T, lower=False):
    key = (g.name, g.n, g.nnz, T, lower)
    if key not in _cache:
        _cache[key] = b2.B2SR.from_graph(g, T, lower)
    return _cache[key]


# ------------------------------------------------------------------ format

@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_b2sr_build_bit_exact(gi, T):
    g = GRAPHS[gi]
    for lower in (False, True):
        print(f"build {g.name} T={T} lower={lower}", flush=True)
        A = b2sr(g, T, lower)
        trp, tci, bits = orc.b2sr_build(g, T, lower_only=lower)
        assert A.ntiles == len(tci)
        gtrp, gtci, gbits = A.to_host()
        assert np.array_equal(gtrp, trp)
        assert np.array_equal(gtci, tci)
        assert np.array_equal(gbits, bits)
        assert A.nbytes == orc.b2sr_bytes(A.ntiles, g.n, T)


def test_build_unsorted_and_repeated_columns():
    g = gg.rmat(11, 8, seed=4)
    r = gg.rng(5)
    rows = np.repeat(np.arange(g.n), g.degrees())
    # shuffle columns inside each row and repeat a third of the entries
    perm = np.lexsort((r.random(g.nnz), rows))
    ci = g.colind[perm]
    dup = r.random(g.nnz) < 0.33
    rows2 = np.concatenate([rows, rows[dup]])
    ci2 = np.concatenate([ci, ci[dup]])
    order = np.argsort(rows2, kind="stable")
    ci2 = ci2[order]
    rp2 = np.zeros(g.n + 1, dtype=np.uint32)
    np.cumsum(np.bincount(rows2, minlength=g.n), out=rp2[1:])
    for T in TILES:
        A = b2.B2SR.from_csr(rp2, ci2.astype(np.uint32), g.n, T)
        trp, tci, bits = orc.b2sr_build(g, T)
        gtrp, gtci, gbits = A.to_host()
        assert np.array_equal(gtrp, trp) and np.array_equal(gtci, tci) and np.array_equal(gbits, bits)


def test_pack_bits():
    for n in (1, 31, 32, 33, 64, 65, 1000, 4099):
        p = gg.rng(n).random(n) < 0.4
        got = b2.as_u32(b2.b2sr_pack_bits(torch.from_numpy(p).cuda()))
        assert np.array_equal(got, pack_bits(p)), n


# ------------------------------------------------------------------ bin x bin

def masks_for(n, seed):
    r = gg.rng(seed)
    return [(None, False), (r.random(n) < 0.5, False), (r.random(n) < 0.5, True), (r.random(n) < 0.97, True)]


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_spmv_bin_bin(gi, T):
    g = GRAPHS[gi]
    A = b2sr(g, T)
    r = gg.rng(31 * gi + T)
    for density in (0.0, 0.002, 0.3, 1.0):
        x = r.random(g.n) < density
        if density == 0.002 and g.n:
            x[0] = True
        xd = dev_u32(pack_bits(x))
        for (mask, comp), sparse in zip(masks_for(g.n, gi + T), (False, True, False, True)):
            print(f"spmv_bin_bin {g.name} T={T} density={density} mask={mask is not None} comp={comp} "
                  f"sparse={sparse}", flush=True)
            md = None if mask is None else dev_u32(pack_bits(mask))
            ref = orc.spmv_or(g, x, mask, comp)
            refc = orc.spmv_count(g, x, mask, comp)
            for sp in (sparse, not sparse):
                yb = b2.as_u32(b2.spmv_bin_bin(A, xd, md, comp, sparse_x=sp))
                assert padding_zero(yb, g.n)
                assert np.array_equal(unpack_bits(yb, g.n), ref)
                yc = b2.as_u32(b2.spmv_bin_bin(A, xd, md, comp, count=True, sparse_x=sp))
                assert np.array_equal(yc, refc)
    # accumulate: y |= A x (bits), y += A x (counts); masked rows keep their old value
    x = r.random(g.n) < 0.2
    mask = r.random(g.n) < 0.6
    old = r.random(g.n) < 0.5
    y = dev_u32(pack_bits(old))
    b2.spmv_bin_bin(A, dev_u32(pack_bits(x)), dev_u32(pack_bits(mask)), False, accumulate=True, out=y)
    assert np.array_equal(unpack_bits(b2.as_u32(y), g.n), old | orc.spmv_or(g, x, mask, False))
    oldc = r.integers(0, 1000, g.n).astype(np.uint32)
    yc = dev_u32(oldc)
    b2.spmv_bin_bin(A, dev_u32(pack_bits(x)), None, False, count=True, accumulate=True, out=yc)
    assert np.array_equal(b2.as_u32(yc), oldc + orc.spmv_count(g, x))


# ------------------------------------------------------------------ bin x full

def plus_bound(g, x, s, alpha, beta, mask, comp):
    deg = g.degrees().astype(np.float64)
    mag = orc.spmv_plus(g, np.abs(x), None if s is None else np.abs(s), mask, comp)
    return abs(alpha) * (deg + 2) * EPS32 * mag * 1.0001 + EPS32 * (abs(alpha) * mag + abs(beta)) * 2 + 1e-30


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_spmv_plus_times_f32(gi, T):
    g = GRAPHS[gi]
    A = b2sr(g, T)
    r = gg.rng(97 * gi + T)
    x = r.random(g.n).astype(np.float32)
    x[r.random(g.n) < 0.3] *= -1
    s = (1.0 / np.maximum(g.degrees(), 1)).astype(np.float32)
    for use_s, alpha, beta, (mask, comp) in [(False, 1.0, 0.0, (None, False)), (True, 0.85, 0.15 / max(g.n, 1), (None, False)),
                                             (False, -2.0, 0.5, (r.random(g.n) < 0.5, True))]:
        print(f"plus {g.name} T={T} s={use_s} a={alpha} mask={mask is not None}", flush=True)
        sd = dev(s, torch.float32) if use_s else None
        md = None if mask is None else dev_u32(pack_bits(mask))
        y = b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, dev(x, torch.float32), sd, md, comp, alpha=alpha, beta=beta)
        y = y.cpu().numpy().astype(np.float64)
        t = orc.spmv_plus(g, x.astype(np.float64), s.astype(np.float64) if use_s else None, mask, comp)
        keep = np.ones(g.n, bool) if mask is None else (~mask if comp else mask)
        ref = np.where(keep, alpha * t + beta, 0.0)
        bound = plus_bound(g, x.astype(np.float64), s if use_s else None, alpha, beta, mask, comp)
        assert np.all(np.abs(y - ref) <= bound), np.max(np.abs(y - ref) - bound)
        assert np.all(y[~keep] == 0.0)
    # accumulate
    old = r.random(g.n).astype(np.float32)
    yd = dev(old, torch.float32)
    b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, dev(x, torch.float32), alpha=0.5, beta=1.0, accumulate=True, out=yd)
    ref = old + 0.5 * orc.spmv_plus(g, x.astype(np.float64)) + 1.0
    bound = plus_bound(g, x.astype(np.float64), None, 0.5, 1.0, None, False) + 4 * EPS32 * np.abs(ref)
    assert np.all(np.abs(yd.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_spmv_full_x_active(gi, T):
    """Inactive x entries count as the identity; inactive tiles are skipped."""
    g = GRAPHS[gi]
    A = b2sr(g, T)
    r = gg.rng(991 * gi + T)
    for density in (0.0, 0.001, 0.05, 0.6):
        act = r.random(g.n) < density
        ad = dev_u32(pack_bits(act))
        print(f"x_active {g.name} T={T} density={density}", flush=True)
        # plus-times (integer-valued, so the sum is exact)
        x = r.integers(-8, 9, g.n).astype(np.float32)
        y = b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, dev(x, torch.float32), x_active=ad).cpu().numpy()
        assert np.array_equal(y, orc.spmv_plus(g, np.where(act, x, 0.0)).astype(np.float32))
        # min-plus with the diagonal term, which reads every x_i
        xf = r.integers(0, 40, g.n).astype(np.float32)
        yf = b2.spmv_bin_full(A, b2.MIN_PLUS_F32, dev(xf, torch.float32), self_loop=True, alpha=1.0, x_active=ad)
        ref = np.minimum(orc.spmv_min_plus(g, np.where(act, xf, np.inf), 1.0, False), xf).astype(np.float32)
        assert np.array_equal(yf.cpu().numpy(), ref)
        xu = r.integers(0, 1000, g.n).astype(np.uint32)
        yu = b2.as_u32(b2.spmv_bin_full(A, b2.MIN_PLUS_U32, dev_u32(xu), self_loop=True, alpha=0, x_active=ad))
        refu = np.minimum(orc.spmv_min_plus(g, np.where(act, xu.astype(np.float64), np.inf), 0.0, False), xu)
        assert np.array_equal(yu, refu.astype(np.uint32))
        x64 = r.integers(0, 2**63, g.n, dtype=np.uint64)
        y64 = b2.as_u64(b2.spmv_bin_full(A, b2.OR_U64, torch.from_numpy(x64.view(np.int64)).cuda(), x_active=ad))
        assert np.array_equal(y64, orc.spmv_or64(g, np.where(act, x64, np.uint64(0))))


def test_plus_times_deterministic():
    g = gg.rmat(14, 16, seed=3)
    x = gg.rng(1).random(g.n).astype(np.float32)
    for T in TILES:
        A = b2sr(g, T)
        xd = dev(x, torch.float32)
        ys = [b2.spmv_bin_full(A, b2.PLUS_TIMES_F32, xd).cpu().numpy() for _ in range(3)]
        assert all(np.array_equal(ys[0].view(np.uint32), y.view(np.uint32)) for y in ys[1:])


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_spmv_min_plus(gi, T):
    g = GRAPHS[gi]
    A = b2sr(g, T)
    r = gg.rng(13 * gi + T)
    xf = r.integers(0, 50, g.n).astype(np.float32) + r.random(g.n).astype(np.float32)
    xf[r.random(g.n) < 0.3] = np.inf
    xu = r.integers(0, 2**32 - 1, g.n, dtype=np.uint64).astype(np.uint32)
    xu[r.random(g.n) < 0.3] = UNR
    xu[r.random(g.n) < 0.1] = 2**32 - 3  # saturates with weight >= 2
    for w, self_loop, (mask, comp) in [(1.0, True, (None, False)), (0.0, True, (None, False)),
                                       (2.0, False, (r.random(g.n) < 0.5, False)), (3.0, True, (r.random(g.n) < 0.5, True))]:
        print(f"minplus {g.name} T={T} w={w} self={self_loop} mask={mask is not None}", flush=True)
        md = None if mask is None else dev_u32(pack_bits(mask))
        yf = b2.spmv_bin_full(A, b2.MIN_PLUS_F32, dev(xf, torch.float32), None, md, comp, self_loop, alpha=w)
        ref = orc.spmv_min_plus(g, xf.astype(np.float64), w, self_loop, mask, comp).astype(np.float32)
        assert np.array_equal(yf.cpu().numpy(), ref)
        yu = b2.as_u32(b2.spmv_bin_full(A, b2.MIN_PLUS_U32, dev_u32(xu), None, md, comp, self_loop, alpha=w))
        xd = np.where(xu == UNR, np.inf, xu.astype(np.float64))
        refu = orc.spmv_min_plus(g, xd, w, self_loop, mask, comp)
        refu = np.where(refu >= UNR, UNR, refu).astype(np.uint32)
        assert np.array_equal(yu, refu)
    # accumulate: y = min(y, t)
    old = r.integers(0, 60, g.n).astype(np.float32)
    yd = dev(old, torch.float32)
    b2.spmv_bin_full(A, b2.MIN_PLUS_F32, dev(xf, torch.float32), alpha=1.0, accumulate=True, out=yd)
    ref = np.minimum(old, orc.spmv_min_plus(g, xf.astype(np.float64), 1.0, False).astype(np.float32))
    assert np.array_equal(yd.cpu().numpy(), ref)


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_spmv_or_u64(gi, T):
    g = GRAPHS[gi]
    A = b2sr(g, T)
    r = gg.rng(7 * gi + T)
    x = r.integers(0, 2**63, g.n, dtype=np.uint64) & r.integers(0, 2**63, g.n, dtype=np.uint64)
    x[r.random(g.n) < 0.5] = 0
    x[r.random(g.n) < 0.1] |= np.uint64(1 << 63)
    xd = torch.from_numpy(x.view(np.int64)).cuda()
    for mask, comp in masks_for(g.n, 5 + gi):
        md = None if mask is None else dev_u32(pack_bits(mask))
        y = b2.as_u64(b2.spmv_bin_full(A, b2.OR_U64, xd, None, md, comp))
        keep = np.ones(g.n, bool) if mask is None else (~mask if comp else mask)
        assert np.array_equal(y, np.where(keep, orc.spmv_or64(g, x), np.uint64(0)))


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_spmv_max_times(gi, T):
    g = GRAPHS[gi]
    A = b2sr(g, T)
    r = gg.rng(600 + gi)
    x = r.integers(0, 1 << 63, size=g.n, dtype=np.uint64) * (r.random(g.n) < 0.4)
    xd = torch.from_numpy(x.view(np.int64)).cuda()
    ref = orc.spmv_max(g, x)
    assert np.array_equal(b2.as_u64(b2.spmv_bin_full(A, b2.MAX_TIMES_U64, xd)), ref)
    act = dev_u32(pack_bits(x != 0))  # only the non-zero entries: the same maximum
    assert np.array_equal(b2.as_u64(b2.spmv_bin_full(A, b2.MAX_TIMES_U64, xd, x_active=act)), ref)
    for mask, comp in masks_for(g.n, 9 + gi):
        md = None if mask is None else dev_u32(pack_bits(mask))
        keep = np.ones(g.n, bool) if mask is None else (~mask if comp else mask)
        y = b2.as_u64(b2.spmv_bin_full(A, b2.MAX_TIMES_U64, xd, None, md, comp))
        assert np.array_equal(y, np.where(keep, ref, np.uint64(0)))


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_mis_and_color(gi, T):
    g = GRAPHS[gi]
    A = b2sr(g, T)
    key = b2.mis_keys(g.n, 40 + gi)
    k = b2.as_u64(key)
    m, rounds = b2.b2sr_mis(A, key)
    exp, exp_rounds = orc.mis(g, k)
    assert np.array_equal(unpack_bits(b2.as_u32(m), g.n), exp) and rounds == exp_rounds
    assert padding_zero(b2.as_u32(m), g.n)
    col, nc = b2.b2sr_color(A, key)
    exp_col, exp_nc = orc.color(g, k)
    assert nc == exp_nc and np.array_equal(b2.as_u32(col), exp_col)


@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_mis_and_color_with_keyless_vertices(gi):
    """Vertices whose key is 0 are never candidates: they stay out of the set and
    uncoloured, and colouring still ends (a pass starts only while keyed
    vertices are uncoloured).  All keys 0: no round, no colour."""
    g = GRAPHS[gi]
    A = b2sr(g, 16)
    key = b2.mis_keys(g.n, 90 + gi).clone()
    key[::7] = 0
    k = b2.as_u64(key)
    m, rounds = b2.b2sr_mis(A, key)
    exp, exp_rounds = orc.mis(g, k)
    assert np.array_equal(unpack_bits(b2.as_u32(m), g.n), exp) and rounds == exp_rounds
    col, nc = b2.b2sr_color(A, key)
    exp_col, exp_nc = orc.color(g, k)
    assert nc == exp_nc and np.array_equal(b2.as_u32(col), exp_col)
    zero = torch.zeros_like(key)
    m0, r0 = b2.b2sr_mis(A, zero)
    c0, n0 = b2.b2sr_color(A, zero)
    assert r0 == 0 and n0 == 0 and not b2.as_u32(m0).any() and np.all(b2.as_u32(c0) == b2.UNREACHED)


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_eccentricity_and_diameter(gi, T):
    g = GRAPHS[gi]
    A = b2sr(g, T)
    # more than one batch of 64, with a repeated source
    srcs = np.r_[gg.rng(800 + gi).integers(0, g.n, 70), 0].astype(np.uint32)
    assert np.array_equal(b2.b2sr_eccentricity(A, srcs), orc.eccentricity(g, srcs))
    if g.n <= 5000:
        assert b2.b2sr_diameter(A) == orc.diameter(g)


# ------------------------------------------------------------------ masked SpGEMM

@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_spgemm_masked(gi, T):
    g = GRAPHS[gi]
    print(f"spgemm {g.name} T={T}", flush=True)
    L = orc.tril(g)
    Ld = b2sr(g, T, lower=True)
    assert int(b2.as_u64(b2.spgemm_masked(Ld, Ld, Ld))[0]) == orc.tc(g) == orc.masked_sum(L, L, L)
    A = b2sr(g, T)
    assert int(b2.as_u64(b2.spgemm_masked(A, A, A))[0]) == orc.masked_sum(g, g, g)
    # a different mask and second operand, and the unmasked sum
    h = gg.random_graph_tiny(g.n, min(1.0, 8.0 / max(g.n, 1)), 55 + gi) if g.n <= 5000 else g
    M = gg.random_graph_tiny(g.n, min(1.0, 5.0 / max(g.n, 1)), 77 + gi) if g.n <= 5000 else g
    Hd, Md = b2sr(h, T), b2sr(M, T)
    assert int(b2.as_u64(b2.spgemm_masked(A, Hd, Md))[0]) == orc.masked_sum(g, h, M)
    if g.n <= 5000:
        assert int(b2.as_u64(b2.spgemm_masked(A, Hd))[0]) == orc.masked_sum(g, h)
    acc = b2.spgemm_masked(A, A, A)
    b2.spgemm_masked(A, A, A, accumulate=True, out=acc)
    assert int(b2.as_u64(acc)[0]) == 2 * orc.masked_sum(g, g, g)
    # A = Bt (oriented) under masks unrelated to A: a symmetric one and a directed one
    if g.n <= 5000:
        assert int(b2.as_u64(b2.spgemm_masked(A, A, Md))[0]) == orc.masked_sum(g, g, M)
        r = gg.rng(990 + gi)
        k = 4 * g.n
        D = gg.directed_csr(g.n, r.integers(0, g.n, k), r.integers(0, g.n, k))
        Dd = b2.B2SR.from_csr(D.rowptr, D.colind, D.n, T)
        assert int(b2.as_u64(b2.spgemm_masked(A, A, Dd))[0]) == orc.masked_sum(g, g, D)
        assert int(b2.as_u64(b2.spgemm_masked(Ld, Ld, Dd))[0]) == orc.masked_sum(L, L, D)
    # with A = Bt the binding passes the orientation workspace; without it every
    # mask tile scans Bt's row: the same sums
    for X in (Ld, A):
        plain = torch.zeros(1, dtype=torch.int64, device="cuda")
        assert b2.lib().spgemm_masked(X.view, X.view, X.view, 0, b2._ptr(plain), None, 0, b2._stream()) == 0
        assert int(b2.as_u64(plain)[0]) == int(b2.as_u64(b2.spgemm_masked(X, X, X))[0])


def _rows_only(c, r0, r1):
    """CSR c with every row outside [r0, r1) emptied (a mask restricted to rows)."""
    rows = np.repeat(np.arange(c.n, dtype=np.int64), np.diff(c.rowptr.astype(np.int64)))
    keep = (rows >= r0) & (rows < r1)
    return gg.directed_csr(c.n, rows[keep], c.colind.astype(np.int64)[keep])


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_spgemm_masked_rows(gi, T):
    """The product over consecutive ranges of mask tile-rows: each range equals
    the oracle's sum with the mask restricted to those rows, and the ranges add
    up to the whole product (triangle counting and the A.A mask)."""
    g = GRAPHS[gi]
    ntr = (g.n + T - 1) // T
    cuts = sorted({0, ntr, *gg.rng(900 + gi).integers(0, ntr + 1, 3).tolist()})
    L = orc.tril(g)
    Ld, A = b2sr(g, T, lower=True), b2sr(g, T)
    for X, Xd in ((L, Ld), (g, A)):
        total = b2.spgemm_masked_rows(Xd, Xd, Xd, 0, 0)          # an empty range gives 0
        assert int(b2.as_u64(total)[0]) == 0
        for r0, r1 in zip(cuts[:-1], cuts[1:]):
            print(f"spgemm rows {g.name} T={T} [{r0}, {r1})", flush=True)
            part = b2.spgemm_masked_rows(Xd, Xd, Xd, r0, r1)
            assert int(b2.as_u64(part)[0]) == orc.masked_sum(X, X, _rows_only(X, r0 * T, r1 * T))
            b2.spgemm_masked_rows(Xd, Xd, Xd, r0, r1, accumulate=True, out=total)
        assert int(b2.as_u64(total)[0]) == int(b2.as_u64(b2.spgemm_masked(Xd, Xd, Xd))[0])


def _tiles(c, T):
    """(tile-row, tile-column, set bits) of every non-empty T x T tile of CSR c."""
    rows = np.repeat(np.arange(c.n, dtype=np.int64), np.diff(c.rowptr.astype(np.int64)))
    key, cnt = np.unique((rows // T) * (1 << 32) + c.colind.astype(np.int64) // T, return_counts=True)
    return key >> 32, key & 0xFFFFFFFF, cnt


def _profile_expected(a, bt, m, T):
    import scipy.sparse as sp
    ntr = (a.n + T - 1) // T
    ai, ak, _ = _tiles(a, T)
    bj, bk, _ = _tiles(bt, T)
    mi, mj, mc = _tiles(m, T)
    At = sp.csr_matrix((np.ones(ai.size, np.int64), (ai, ak)), shape=(ntr, ntr))
    Bt = sp.csr_matrix((np.ones(bj.size, np.int64), (bj, bk)), shape=(ntr, ntr))
    common = np.asarray((At @ Bt.T).tocsr()[mi, mj]).ravel() if mi.size else np.zeros(0, np.int64)
    visit = np.bincount(ai, minlength=ntr)[mi] > 0
    brow = np.bincount(bj, minlength=ntr)
    return {"mask_tiles": int(visit.sum()), "lookups": int(brow[mj][visit].sum()),
            "tile_pairs": int(common[visit].sum()), "row_pairs": int((common * mc)[visit].sum())}


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", [i for i, g in enumerate(GRAPHS) if 0 < g.n <= 5000], ids=lambda i: IDS[i])
def test_spgemm_profile_counts(gi, T):
    """The work counts of the masked product equal those read off the tile
    structure on the host: for triangle counting and for unrelated operands."""
    g = GRAPHS[gi]
    L = orc.tril(g)
    Ld = b2sr(g, T, lower=True)
    assert b2.spgemm_masked_profile(Ld, Ld, Ld) == _profile_expected(L, L, L, T)
    h = gg.random_graph_tiny(g.n, min(1.0, 8.0 / g.n), 55 + gi)
    M = gg.random_graph_tiny(g.n, min(1.0, 5.0 / g.n), 77 + gi)
    A = b2sr(g, T)
    assert b2.spgemm_masked_profile(A, b2sr(h, T), b2sr(M, T)) == _profile_expected(g, h, M, T)


def test_triangle_count_closed_forms():
    for T in TILES:
        for R, C in ((2, 2), (17, 90), (64, 64)):
            k = gg.king_grid(R, C)
            assert b2.triangle_count(k.rowptr, k.colind, k.n, T) == 4 * (R - 1) * (C - 1)
        for n in (3, 33, 100):
            K = gg.complete(n)
            assert b2.triangle_count(K.rowptr, K.colind, n, T) == n * (n - 1) * (n - 2) // 6
        M = gg.mycielski(11)
        assert b2.triangle_count(M.rowptr, M.colind, M.n, T) == 0


# ------------------------------------------------------------------ algorithms

def last_level(levels):
    """The largest finite level (hop distance) in an oracle result, -1 if none."""
    fin = levels[levels != UNR]
    return int(fin.max()) if fin.size else -1


@pytest.mark.parametrize("T", TILES)
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_algorithms(gi, T):
    g = GRAPHS[gi]
    A = b2sr(g, T)
    srcs = np.unique(np.r_[0, gg.rng(gi).integers(0, g.n, 3)]).astype(np.uint32)
    for s in srcs[:3]:
        print(f"bfs/sssp {g.name} T={T} src={s}", flush=True)
        lv, it = b2.b2sr_bfs(A, int(s))
        ref = orc.bfs(g, int(s))
        assert np.array_equal(b2.as_u32(lv), ref)
        assert it == last_level(ref) + 1  # every level that found vertices, then one that found none
        d, it = b2.b2sr_sssp(A, int(s))
        assert np.array_equal(b2.as_u32(d), orc.sssp_unit(g, int(s)))
        assert it == last_level(ref) + 1
    ms = srcs if g.n < 64 else np.unique(gg.rng(gi + 1).choice(g.n, 64, replace=False)).astype(np.uint32)
    lvm, it = b2.b2sr_msbfs(A, ms)
    refm = orc.bfs_multi(g, ms)
    assert np.array_equal(b2.as_u32(lvm), refm)
    assert it == last_level(refm) + 1
    lab, it = b2.b2sr_cc(A)
    refc = orc.cc(g)
    assert np.array_equal(b2.as_u32(lab), refc)
    # a label moves one hop per iteration from each component's least vertex
    assert it == max((last_level(orc.bfs(g, int(r))) for r in np.unique(refc)), default=-1) + 1
    if g.n:
        for iters in (1, 20):
            pr = b2.b2sr_pagerank(A, 0.85, iters).cpu().numpy()
            assert rel_l1(pr, orc.pagerank(g, 0.85, iters)) <= 1e-5


def test_pagerank_deterministic_and_mass():
    g = gg.rmat(14, 16, seed=9)
    for T in TILES:
        A = b2sr(g, T)
        a = b2.b2sr_pagerank(A, 0.85, 20).cpu().numpy()
        b = b2.b2sr_pagerank(A, 0.85, 20).cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert rel_l1(a, orc.pagerank(g, 0.85, 20)) <= 1e-5


def test_stream_read_reads_every_word():
    r = gg.rng(77)
    for nbytes in (16, 16 * 1000, 16 * 8192 * 256 * 3 + 16 * 5):
        h = r.integers(0, 2**32, size=nbytes // 4, dtype=np.uint64).astype(np.uint32)
        t = torch.from_numpy(h.view(np.int32)).cuda()
        out = b2.as_u32(b2.b2sr_stream_read(t, nbytes))
        assert np.bitwise_xor.reduce(out) == np.bitwise_xor.reduce(h)


@pytest.mark.parametrize("T", TILES)
def test_long_runs_reuse_the_workspace(T):
    """Hundreds of iterations (many batches of enqueued, device-gated
    iterations, most of the last batch returning at once), the same workspace
    reused across sources and drivers' runs: every run matches the oracle."""
    g = gg.path(700)
    A = b2sr(g, T)
    ws = {algo: torch.empty(b2.b2sr_algo_workspace_bytes(A, algo), dtype=torch.uint8, device="cuda")
          for algo in (b2.ALGO_BFS, b2.ALGO_SSSP, b2.ALGO_CC, b2.ALGO_MSBFS)}
    for s in (0, 350, 699, 1):
        print(f"path700 T={T} src={s}", flush=True)
        ref = orc.bfs(g, s)
        lv, it = b2.b2sr_bfs(A, s, ws=ws[b2.ALGO_BFS])
        assert np.array_equal(b2.as_u32(lv), ref) and it == last_level(ref) + 1
        d, it = b2.b2sr_sssp(A, s, ws=ws[b2.ALGO_SSSP])
        assert np.array_equal(b2.as_u32(d), ref) and it == last_level(ref) + 1
        lvm, it = b2.b2sr_msbfs(A, [s, (s + 3) % 700], ws=ws[b2.ALGO_MSBFS])
        assert np.array_equal(b2.as_u32(lvm), orc.bfs_multi(g, np.array([s, (s + 3) % 700], dtype=np.uint32)))
        lab, it = b2.b2sr_cc(A, ws=ws[b2.ALGO_CC])
        assert np.all(b2.as_u32(lab) == 0) and it == 700
