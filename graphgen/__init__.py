"""Seeded synthetic graph and vector generators.

This module only builds inputs.  It holds none of the B2SR method's arithmetic
(no tiling, no bit packing, no semiring products) and it imports neither the
HIP product package nor the CPU oracle, so both sides can be fed the same data.

Every generator returns a *canonical* CSR of a simple undirected graph:
symmetric, no self-loops, no duplicate entries, column indices ascending within
each row, ``rowptr`` and ``colind`` as ``numpy.uint32``.  The paper evaluates on
binary square adjacency matrices (Sec. VI-A), which is exactly this shape.

Families (the paper's SuiteSparse set is not available; these stand in for its
pattern classes of Table VI):

* ``er_gnm``      Erdos-Renyi G(n, m)             ("dot" pattern)
* ``rmat``        R-MAT / Kronecker quadrant walk ("hybrid"/"block" pattern)
* ``king_grid``   2D grid with diagonals          ("diagonal"/banded pattern)
* ``grid4``       4-neighbour 2D grid
* ``mycielski``   textbook Mycielski construction ("block"; the paper's worked
                  storage example in Sec. III-C is mycielskian12)
* ``chung_lu``    power-law expected-degree graph
* ``path``, ``star``, ``complete``, ``cycle``, ``torus``, ``disjoint_union``
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Csr", "canonical_csr", "er_gnm", "rmat", "king_grid", "grid4", "mycielski",
    "chung_lu", "chung_lu_batch", "batch_params", "path", "star", "complete", "cycle", "torus", "disjoint_union",
    "random_graph_tiny", "sample_sources", "random_mask", "rng",
]


def rng(seed: int) -> np.random.Generator:
    """numpy PCG64 generator; every input in this repository is drawn from one."""
    return np.random.Generator(np.random.PCG64(seed))


class Csr:
    """A canonical CSR adjacency (uint32 arrays)."""

    __slots__ = ("n", "rowptr", "colind", "name")

    def __init__(self, n: int, rowptr: np.ndarray, colind: np.ndarray, name: str = ""):
        self.n = int(n)
        self.rowptr = rowptr
        self.colind = colind
        self.name = name

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    @property
    def edges(self) -> int:
        """Undirected edge count (each stored twice)."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def to_scipy(self):
        import scipy.sparse as sp
        data = np.ones(self.nnz, dtype=np.int8)
        return sp.csr_matrix((data, self.colind.astype(np.int64), self.rowptr.astype(np.int64)),
                             shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n), dtype=np.uint8)
        rows = np.repeat(np.arange(self.n), self.degrees())
        a[rows, self.colind.astype(np.int64)] = 1
        return a

    def __repr__(self):
        return f"Csr({self.name!r}, n={self.n}, nnz={self.nnz})"


def canonical_csr(n: int, src, dst, name: str = "") -> Csr:
    """Symmetrise, drop self-loops, de-duplicate and sort an edge list into CSR."""
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    if src.size:
        if src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n:
            raise ValueError("edge endpoint out of range")
    keep = src != dst
    src, dst = src[keep], dst[keep]
    rows = np.concatenate([src, dst])
    cols = np.concatenate([dst, src])
    key = np.unique(rows * np.int64(n) + cols)
    rows = key // n
    cols = key - rows * n
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**32:
        raise ValueError("nnz does not fit uint32")
    return Csr(n, rowptr.astype(np.uint32), cols.astype(np.uint32), name)


def directed_csr(n: int, src, dst, name: str = "") -> Csr:
    """A directed graph: row u lists v for every arc u -> v; self-loops are
    dropped, repeated arcs kept once, rows sorted."""
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("arc endpoint out of range")
    keep = src != dst
    key = np.unique(src[keep] * np.int64(n) + dst[keep])
    rows = key // n
    cols = key - rows * n
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    if rowptr[-1] >= 2**32:
        raise ValueError("nnz does not fit uint32")
    return Csr(n, rowptr.astype(np.uint32), cols.astype(np.uint32), name)


def transpose(g: Csr) -> Csr:
    """The reversed graph (CSR of the transposed adjacency)."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    return directed_csr(g.n, g.colind.astype(np.int64), rows, name=g.name + "_T")


def rmat_directed(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                  seed: int = 0) -> Csr:
    """R-MAT arcs as drawn (tuple (i, j) is the arc i -> j), no symmetrisation."""
    n = 1 << scale
    m = edge_factor * n
    g = rng(seed)
    i = np.zeros(m, dtype=np.int64)
    j = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for level in range(scale):
        r = g.random(m)
        bit = np.int64(1) << np.int64(scale - 1 - level)
        i |= np.where(r >= ab, bit, 0)
        j |= np.where(((r >= a) & (r < ab)) | (r >= abc), bit, 0)
    return directed_csr(n, i, j, name=f"rmat_dir_s{scale}_ef{edge_factor}_s{seed}")


def random_digraph(n: int, p: float, seed: int) -> Csr:
    """Each ordered pair (u, v), u != v, is an arc with probability p."""
    g = rng(seed)
    u, v = np.nonzero(g.random((n, n)) < p)
    return directed_csr(n, u, v, name=f"digraph_n{n}_p{p:g}_s{seed}")


def er_gnm(n: int, m: int, seed: int) -> Csr:
    """Erdos-Renyi G(n, m): exactly ``m`` distinct undirected edges, uniform."""
    if m > n * (n - 1) // 2:
        raise ValueError("m too large")
    g = rng(seed)
    chosen = np.empty(0, dtype=np.int64)
    while chosen.size < m:
        need = m - chosen.size
        a = g.integers(0, n, size=2 * need + 16, dtype=np.int64)
        b = g.integers(0, n, size=2 * need + 16, dtype=np.int64)
        ok = a != b
        lo, hi = np.minimum(a[ok], b[ok]), np.maximum(a[ok], b[ok])
        cand = np.concatenate([chosen, lo * n + hi])
        # keep first occurrences in draw order so the result does not depend on sorting
        _, first = np.unique(cand, return_index=True)
        chosen = cand[np.sort(first)][:m]
    lo, hi = chosen // n, chosen % n
    return canonical_csr(n, lo, hi, name=f"er_n{n}_m{m}_s{seed}")


def rmat(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 0, permute: bool = False, chunk: int = 1 << 22) -> Csr:
    """R-MAT: each of ``edge_factor * 2**scale`` tuples picks a quadrant ``scale``
    times with probabilities (a, b, c, d=1-a-b-c); no noise.  Then symmetrise,
    drop self-loops and de-duplicate.  ``permute`` relabels vertices randomly."""
    n = 1 << scale
    m = edge_factor * n
    g = rng(seed)
    src = np.empty(m, dtype=np.int64)
    dst = np.empty(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for s in range(0, m, chunk):
        e = min(m, s + chunk)
        i = np.zeros(e - s, dtype=np.int64)
        j = np.zeros(e - s, dtype=np.int64)
        for level in range(scale):
            r = g.random(e - s)
            bit = np.int64(1) << np.int64(scale - 1 - level)
            ibit = r >= ab
            jbit = ((r >= a) & (r < ab)) | (r >= abc)
            i |= np.where(ibit, bit, 0)
            j |= np.where(jbit, bit, 0)
        src[s:e] = i
        dst[s:e] = j
    if permute:
        p = g.permutation(n).astype(np.int64)
        src, dst = p[src], p[dst]
    return canonical_csr(n, src, dst, name=f"rmat_s{scale}_ef{edge_factor}_s{seed}{'_perm' if permute else ''}")


def king_grid(rows: int, cols: int) -> Csr:
    """R x C grid, row-major ids, each cell adjacent to its 8 surrounding cells."""
    r, c = np.meshgrid(np.arange(rows, dtype=np.int64), np.arange(cols, dtype=np.int64), indexing="ij")
    r, c = r.ravel(), c.ravel()
    src, dst = [], []
    for dr, dc in ((0, 1), (1, 0), (1, 1), (1, -1)):
        ok = (r + dr < rows) & (c + dc >= 0) & (c + dc < cols)
        src.append(r[ok] * cols + c[ok])
        dst.append((r[ok] + dr) * cols + (c[ok] + dc))
    return canonical_csr(rows * cols, np.concatenate(src), np.concatenate(dst), name=f"king_{rows}x{cols}")


def grid4(rows: int, cols: int) -> Csr:
    """R x C grid, row-major ids, 4-neighbour connectivity."""
    r, c = np.meshgrid(np.arange(rows, dtype=np.int64), np.arange(cols, dtype=np.int64), indexing="ij")
    r, c = r.ravel(), c.ravel()
    src, dst = [], []
    for dr, dc in ((0, 1), (1, 0)):
        ok = (r + dr < rows) & (c + dc < cols)
        src.append(r[ok] * cols + c[ok])
        dst.append((r[ok] + dr) * cols + (c[ok] + dc))
    return canonical_csr(rows * cols, np.concatenate(src), np.concatenate(dst), name=f"grid4_{rows}x{cols}")


def torus(rows: int, cols: int) -> Csr:
    """4-regular wrap-around grid (rows, cols >= 3)."""
    r, c = np.meshgrid(np.arange(rows, dtype=np.int64), np.arange(cols, dtype=np.int64), indexing="ij")
    r, c = r.ravel(), c.ravel()
    src = np.concatenate([r * cols + c, r * cols + c])
    dst = np.concatenate([r * cols + (c + 1) % cols, ((r + 1) % rows) * cols + c])
    return canonical_csr(rows * cols, src, dst, name=f"torus_{rows}x{cols}")


def mycielski(k: int) -> Csr:
    """Mycielski graph M_k (k >= 2) in natural order.

    M_2 is K_2.  M_{k+1} lists the vertices v_i of M_k, then their shadows u_i
    (u_i is adjacent to every neighbour of v_i), then an apex w adjacent to all
    u_i.  M_k is triangle-free with n_k = 3 * 2**(k-2) - 1 vertices."""
    if k < 2:
        raise ValueError("k >= 2")
    n = 2
    src = np.array([0], dtype=np.int64)
    dst = np.array([1], dtype=np.int64)
    for _ in range(k - 2):
        shadow_a = np.concatenate([src + n, dst + n])   # u_i side
        shadow_b = np.concatenate([dst, src])           # neighbour v_j of v_i
        apex = np.full(n, 2 * n, dtype=np.int64)
        src = np.concatenate([src, shadow_a, np.arange(n, 2 * n, dtype=np.int64)])
        dst = np.concatenate([dst, shadow_b, apex])
        n = 2 * n + 1
    return canonical_csr(n, src, dst, name=f"mycielski{k}")


def chung_lu(n: int, avg_degree: float, gamma: float = 2.1, seed: int = 0) -> Csr:
    """Chung-Lu expected-degree power-law graph.

    Weights w_i ~ (i+1)^(-1/(gamma-1)), capped at sqrt(sum w), rescaled so the
    mean expected degree is ``avg_degree``; n*avg_degree/2 endpoint pairs are
    drawn independently proportional to w, then symmetrised and de-duplicated."""
    g = rng(seed)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= avg_degree * n / w.sum()
    cap = np.sqrt(w.sum())
    w = np.minimum(w, cap)
    p = w / w.sum()
    m = int(round(n * avg_degree / 2))
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    a = np.searchsorted(cdf, g.random(m), side="right")
    b = np.searchsorted(cdf, g.random(m), side="right")
    a = np.minimum(a, n - 1)
    b = np.minimum(b, n - 1)
    return canonical_csr(n, a, b, name=f"chunglu_n{n}_k{avg_degree:g}_s{seed}")


def path(n: int) -> Csr:
    i = np.arange(n - 1, dtype=np.int64)
    return canonical_csr(n, i, i + 1, name=f"path{n}")


def cycle(n: int) -> Csr:
    i = np.arange(n, dtype=np.int64)
    return canonical_csr(n, i, (i + 1) % n, name=f"cycle{n}")


def star(n: int) -> Csr:
    """Vertex 0 is the centre, 1..n-1 the leaves."""
    i = np.arange(1, n, dtype=np.int64)
    return canonical_csr(n, np.zeros_like(i), i, name=f"star{n}")


def wheel(n: int) -> Csr:
    """A cycle on 0..n-2 (the rim) and vertex n-1 (the hub) joined to all of
    them; n - 1 triangles when the rim has at least 4 vertices."""
    i = np.arange(n - 1, dtype=np.int64)
    src = np.concatenate([i, i])
    dst = np.concatenate([(i + 1) % (n - 1), np.full(n - 1, n - 1, dtype=np.int64)])
    return canonical_csr(n, src, dst, name=f"wheel{n}")


def complete(n: int) -> Csr:
    i, j = np.triu_indices(n, 1)
    return canonical_csr(n, i, j, name=f"K{n}")


def disjoint_union(*gs: Csr) -> Csr:
    off = 0
    src, dst = [], []
    for g in gs:
        rows = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
        src.append(rows + off)
        dst.append(g.colind.astype(np.int64) + off)
        off += g.n
    return canonical_csr(off, np.concatenate(src), np.concatenate(dst), name="union")


def batch_params(count: int = 256, seed: int = 1000):
    """Sizes and mean degrees of the batched workload: n log-uniform in
    [1024, 262144], mean degree uniform in [4, 32]."""
    r = rng(seed)
    n = np.floor(np.exp(r.uniform(np.log(1024), np.log(262144), count))).astype(np.int64)
    k = r.uniform(4, 32, count)
    return n, k


def _chung_lu_job(args):
    i, n, k, gamma, seed0 = args
    return chung_lu(int(n), float(k), gamma, seed=seed0 + i)


def chung_lu_batch(count: int = 256, gamma: float = 2.1, seed: int = 1000, workers: int = 8):
    """The batched workload: ``count`` Chung-Lu graphs (power-law exponent
    gamma), graph i drawn with seed ``seed + i``; generated in worker processes."""
    from concurrent.futures import ProcessPoolExecutor
    n, k = batch_params(count, seed)
    jobs = [(i, n[i], k[i], gamma, seed) for i in range(count)]
    if workers <= 1:
        return [_chung_lu_job(j) for j in jobs]
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_chung_lu_job, jobs, chunksize=4))


def random_graph_tiny(n: int, p: float, seed: int) -> Csr:
    """G(n, p) for brute-force checks on tiny graphs."""
    g = rng(seed)
    i, j = np.triu_indices(n, 1)
    keep = g.random(i.size) < p
    return canonical_csr(n, i[keep], j[keep], name=f"gnp_n{n}_p{p:g}_s{seed}")


def sample_sources(csr: Csr, k: int, seed: int) -> np.ndarray:
    """``k`` distinct vertices of degree >= 1, drawn without replacement."""
    cand = np.flatnonzero(csr.degrees() > 0)
    g = rng(seed)
    if k > cand.size:
        raise ValueError("not enough non-isolated vertices")
    return np.sort(g.choice(cand, size=k, replace=False)).astype(np.uint32)


def random_mask(n: int, density: float, seed: int) -> np.ndarray:
    """Boolean vector with each entry set independently with ``density``."""
    return rng(seed).random(n) < density


def rmat_pool_params(count: int = 64, seed: int = 2000):
    """Scales uniform in 12..20 and edge factors uniform in 8..32, seeded."""
    g = rng(seed)
    return g.integers(12, 21, size=count), g.integers(8, 33, size=count)


def _rmat_job(args):
    i, scale, ef, seed = args
    return rmat(int(scale), int(ef), seed=seed + i)


def rmat_pool(count: int = 64, seed: int = 2000, workers: int = 8):
    """The serving pool: ``count`` R-MAT graphs (parameters from
    rmat_pool_params; graph i drawn with seed ``seed + i``), generated in worker
    processes, largest first."""
    from concurrent.futures import ProcessPoolExecutor
    scales, efs = rmat_pool_params(count, seed)
    jobs = [(i, scales[i], efs[i], seed) for i in range(count)]
    order = sorted(range(count), key=lambda i: -(int(efs[i]) << int(scales[i])))
    if workers <= 1:
        out = {i: _rmat_job(jobs[i]) for i in order}
    else:
        with ProcessPoolExecutor(workers) as ex:
            out = dict(zip(order, ex.map(_rmat_job, [jobs[i] for i in order])))
    return [out[i] for i in range(count)]
