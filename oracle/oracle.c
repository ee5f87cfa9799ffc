/*
 * CPU oracle for the B2SR hot path.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It is a plain, slow, obviously correct statement of what
 * the bit-level GraphBLAS kernels of Bit-GraphBLAS (Chen et al., IPDPS 2022,
 * arXiv 2201.08560) compute.  It never touches the HIP product code: inputs are
 * plain CSR arrays (canonical: sorted, unique columns, no self loops, as built
 * by the repository's graph generators) and plain per-vertex vectors (one byte
 * per Boolean, double for reals, uint32 for labels and levels).
 *
 * Parallelism: independent output rows are computed by an OpenMP "parallel
 * for"; every per-row sum runs serially in CSR order, so results do not depend
 * on the thread count.
 *
 * Readings taken where the paper is silent or ambiguous are stated at each
 * function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_UNREACHED 0xFFFFFFFFu

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------------- */
/* B2SR by definition (Sec. III-A tile indexing, Sec. III-B / Table II packing) */
/* ------------------------------------------------------------------------- */

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Bytes of one bit-row for tile dimension T (Table II; T=4 uses the low nibble
 * of an unsigned char; T=64 uses the unsigned long long bit-packing type that
 * Sec. III-A lists for BitTiles). */
static size_t row_bytes(uint32_t T)
{
    return T == 64 ? 8 : T == 32 ? 4 : (T == 16 ? 2 : 1);
}

/*
 * Distinct tile columns of tile-row I, sorted ascending, written to out.
 * Returns the count.  out must hold the number of nonzeros of the tile-row.
 */
static uint32_t tile_row_columns(uint32_t n, const uint32_t *rowptr, const uint32_t *colind,
                                 uint32_t T, uint32_t I, uint32_t *out, int lower_only)
{
    uint32_t r0 = I * T, r1 = r0 + T < n ? r0 + T : n, k = 0;
    for (uint32_t i = r0; i < r1; ++i)
        for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (!lower_only || colind[e] < i) out[k++] = colind[e] / T;
    if (k == 0) return 0;
    qsort(out, k, sizeof(uint32_t), cmp_u32);
    uint32_t u = 1;
    for (uint32_t e = 1; e < k; ++e)
        if (out[e] != out[u - 1]) out[u++] = out[e];
    return u;
}

/*
 * Number of non-empty T x T tiles: |{(floor(i/T), floor(j/T)) : A_ij = 1}|.
 * lower_only restricts A to its strictly lower triangle (j < i).
 */
uint64_t orc_b2sr_count_tiles(uint32_t n, const uint32_t *rowptr, const uint32_t *colind,
                              uint32_t T, int lower_only)
{
    uint32_t ntr = (n + T - 1) / T;
    uint64_t total = 0;
#pragma omp parallel reduction(+ : total)
    {
        uint32_t *buf = NULL;
        size_t cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (uint32_t I = 0; I < ntr; ++I) {
            uint32_t r1 = I * T + T < n ? I * T + T : n;
            size_t need = rowptr[r1] - rowptr[I * T];
            if (need > cap) {
                free(buf);
                cap = need;
                buf = (uint32_t *)malloc(cap * sizeof(uint32_t));
            }
            total += tile_row_columns(n, rowptr, colind, T, I, buf, lower_only);
        }
        free(buf);
    }
    return total;
}

/*
 * Full B2SR arrays (Sec. III-A): TileRowPtr has nTileRow+1 entries (exclusive
 * prefix of non-empty tiles per tile-row), TileColInd lists tile columns in
 * ascending order within each tile-row, BitTiles holds T bit-rows per tile in
 * the same order.  Bit-row r of a tile is the word at index tile*T + r; bit c
 * of it (least significant first: "bits are indexed from right to left",
 * Sec. IV) is A[I*T + r][J*T + c].  Word width per Table II: 1 byte for T=4
 * (low nibble) and T=8, 2 bytes for T=16, 4 bytes for T=32; 8 bytes for T=64
 * (the 64-bit packing type of Sec. III-A, a tile size Sec. VI-B also names).
 * bits must be zero-filled by the caller.
 */
int orc_b2sr_build(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, uint32_t T,
                   int lower_only, uint32_t *tile_rowptr, uint32_t *tile_colind, void *bits)
{
    if (T != 4 && T != 8 && T != 16 && T != 32 && T != 64) return -1;
    uint32_t ntr = (n + T - 1) / T;
    size_t rb = row_bytes(T);
    uint32_t maxseg = 0;
    for (uint32_t I = 0; I < ntr; ++I) {
        uint32_t r1 = I * T + T < n ? I * T + T : n;
        uint32_t seg = rowptr[r1] - rowptr[I * T];
        if (seg > maxseg) maxseg = seg;
    }
    uint32_t *buf = (uint32_t *)malloc((maxseg ? maxseg : 1) * sizeof(uint32_t));
    tile_rowptr[0] = 0;
    for (uint32_t I = 0; I < ntr; ++I) {
        uint32_t cnt = tile_row_columns(n, rowptr, colind, T, I, buf, lower_only);
        memcpy(tile_colind + tile_rowptr[I], buf, cnt * sizeof(uint32_t));
        tile_rowptr[I + 1] = tile_rowptr[I] + cnt;
    }
    free(buf);
    uint8_t *b = (uint8_t *)bits;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t I = i / T, r = i % T;
        for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            uint32_t j = colind[e];
            if (lower_only && j >= i) continue;
            uint32_t J = j / T, c = j % T;
            /* binary search for J in tile-row I */
            uint32_t lo = tile_rowptr[I], hi = tile_rowptr[I + 1];
            while (lo < hi) {
                uint32_t mid = lo + (hi - lo) / 2;
                if (tile_colind[mid] < J) lo = mid + 1; else hi = mid;
            }
            size_t word = (size_t)lo * T + r;
            if (rb == 1) b[word] |= (uint8_t)(1u << c);
            else if (rb == 2) ((uint16_t *)b)[word] |= (uint16_t)(1u << c);
            else if (rb == 4) ((uint32_t *)b)[word] |= (1u << c);
            else ((uint64_t *)b)[word] |= ((uint64_t)1 << c);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Matrix-vector products on CSR (Sec. IV, Table III; semirings of Table V)    */
/* ------------------------------------------------------------------------- */

/* keep_i for an optional mask: without complement keep rows where mask_i != 0,
 * with complement keep rows where mask_i == 0 (the BFS "not visited" filter of
 * Sec. V applied before the store). */
static int keep_row(const uint8_t *mask, int complement, uint32_t i)
{
    if (!mask) return 1;
    return complement ? mask[i] == 0 : mask[i] != 0;
}

/* Boolean semiring, 1-bit in / 1-bit out (bmv_bin_bin_bin[_masked]):
 * y_i = OR_{j : A_ij = 1} x_j, then AND keep_i. */
void orc_spmv_or(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const uint8_t *x,
                 const uint8_t *mask, int complement, uint8_t *y)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint8_t v = 0;
        for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (x[colind[e]]) { v = 1; break; }
        y[i] = keep_row(mask, complement, (uint32_t)i) ? v : 0;
    }
}

/* Arithmetic semiring, 1-bit in / 32-bit out (bmv_bin_bin_full, Listing 1's
 * popcount dot product): y_i = |{j : A_ij = 1 and x_j = 1}|; masked rows 0. */
void orc_spmv_count(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const uint8_t *x,
                    const uint8_t *mask, int complement, uint32_t *y)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint32_t v = 0;
        for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) v += x[colind[e]] ? 1u : 0u;
        y[i] = keep_row(mask, complement, (uint32_t)i) ? v : 0;
    }
}

/* Arithmetic semiring, full-precision vector (bmv_bin_full_full):
 * y_i = sum_{j : A_ij = 1} x_j * s_j (s = 1 when absent), in double, summed in
 * ascending j.  Masked rows get 0. */
void orc_spmv_plus(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const double *x,
                   const double *s, const uint8_t *mask, int complement, double *y)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        double v = 0.0;
        for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            uint32_t j = colind[e];
            v += s ? x[j] * s[j] : x[j];
        }
        y[i] = keep_row(mask, complement, (uint32_t)i) ? v : 0.0;
    }
}

/* Tropical min-plus semiring (Sec. V, SSSP and CC): off-diagonal zeros of A are
 * +infinity, set bits carry the edge weight w, and with self != 0 the diagonal
 * is a real zero, so y_i = min(x_i, min_{j : A_ij = 1} x_j + w).  Without self
 * the x_i term is absent.  An empty minimum is +infinity.  Masked rows get
 * +infinity. */
void orc_spmv_min_plus(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const double *x,
                       double w, int self, const uint8_t *mask, int complement, double *y)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        double v = self ? x[i] : INFINITY;
        for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            double t = x[colind[e]] + w;
            if (t < v) v = t;
        }
        y[i] = keep_row(mask, complement, (uint32_t)i) ? v : INFINITY;
    }
}

/* Boolean semiring on 64 independent Boolean vectors at once (one bit per
 * source): y_i = (OR_{j : A_ij = 1} x_j) AND NOT v_i.  This is 64 copies of
 * the masked Boolean product above. */
void orc_spmv_or64(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const uint64_t *x,
                   const uint64_t *visited, uint64_t *y)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t v = 0;
        for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) v |= x[colind[e]];
        y[i] = visited ? (v & ~visited[i]) : v;
    }
}

/* ------------------------------------------------------------------------- */
/* Masked sparse matrix-matrix product, summed (Sec. IV, Table IV)            */
/* ------------------------------------------------------------------------- */

/* |N_A(i) ∩ N_B(j)| for two ascending column lists: a sorted merge. */
static uint64_t intersect_count(const uint32_t *a, uint32_t na, const uint32_t *b, uint32_t nb)
{
    uint32_t p = 0, q = 0;
    uint64_t c = 0;
    while (p < na && q < nb) {
        if (a[p] < b[q]) ++p;
        else if (a[p] > b[q]) ++q;
        else { ++c; ++p; ++q; }
    }
    return c;
}

/*
 * bmm_bin_bin_sum[_masked]: s = sum over (i, j) of (A * B)_ij, with B given by
 * its transpose Bt (row j of Bt lists the k with B_kj = 1), so
 * (A * B)_ij = |N_A(i) ∩ N_Bt(j)|.  The sum is arithmetic (a count of paths
 * i -> k -> j), not a count of nonzero output entries.  With a mask M only the
 * (i, j) with M_ij = 1 contribute; with M absent every (i, j) does (an O(n^2)
 * loop: only for small n).  All three matrices are n x n.
 */
uint64_t orc_masked_sum(uint32_t n, const uint32_t *arp, const uint32_t *aci, const uint32_t *brp,
                        const uint32_t *bci, const uint32_t *mrp, const uint32_t *mci)
{
    uint64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        const uint32_t *ai = aci + arp[i];
        uint32_t na = arp[i + 1] - arp[i];
        if (mrp) {
            for (uint32_t e = mrp[i]; e < mrp[i + 1]; ++e) {
                uint32_t j = mci[e];
                total += intersect_count(ai, na, bci + brp[j], brp[j + 1] - brp[j]);
            }
        } else {
            for (uint32_t j = 0; j < n; ++j)
                total += intersect_count(ai, na, bci + brp[j], brp[j + 1] - brp[j]);
        }
    }
    return total;
}

/* ------------------------------------------------------------------------- */
/* Graph algorithms (Sec. V), textbook formulations                          */
/* ------------------------------------------------------------------------- */

/* BFS levels from src by a FIFO queue.  level[src] = 0, unreachable vertices
 * keep 0xFFFFFFFF.  Levels (not parents) are the compared output: they are
 * unique. */
void orc_bfs(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, uint32_t src,
             uint32_t *level)
{
    for (uint32_t i = 0; i < n; ++i) level[i] = ORC_UNREACHED;
    if (src >= n) return;
    uint32_t *queue = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    uint32_t head = 0, tail = 0;
    level[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        uint32_t u = queue[head++];
        for (uint32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            uint32_t v = colind[e];
            if (level[v] == ORC_UNREACHED) {
                level[v] = level[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
}

/* BFS from several sources, one independent BFS each (out is k x n). */
void orc_bfs_multi(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, uint32_t k,
                   const uint32_t *srcs, uint32_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < (int64_t)k; ++s)
        orc_bfs(n, rowptr, colind, srcs[s], out + (size_t)s * n);
}

/* Single-source shortest paths with unit edge weights by Bellman-Ford:
 * relax every edge (dist_i = min(dist_i, dist_j + 1)) until nothing changes.
 * Unreachable vertices keep 0xFFFFFFFF.  Returns the number of sweeps. */
uint32_t orc_sssp_unit(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, uint32_t src,
                       uint32_t *dist)
{
    for (uint32_t i = 0; i < n; ++i) dist[i] = ORC_UNREACHED;
    if (src >= n) return 0;
    dist[src] = 0;
    uint32_t sweeps = 0;
    int changed = 1;
    while (changed) {
        changed = 0;
        ++sweeps;
        for (uint32_t i = 0; i < n; ++i)
            for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                uint32_t dj = dist[colind[e]];
                if (dj != ORC_UNREACHED && dj + 1 < dist[i]) {
                    dist[i] = dj + 1;
                    changed = 1;
                }
            }
    }
    return sweeps;
}

static uint32_t uf_find(uint32_t *parent, uint32_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

/* Connected components by union-find; the output label of every vertex is the
 * smallest vertex id in its component (a canonical, unique labelling). */
void orc_cc(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, uint32_t *label)
{
    uint32_t *parent = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    for (uint32_t i = 0; i < n; ++i) parent[i] = i;
    for (uint32_t i = 0; i < n; ++i)
        for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            uint32_t a = uf_find(parent, i), b = uf_find(parent, colind[e]);
            /* union by smaller id keeps every root the minimum of its set */
            if (a < b) parent[b] = a;
            else if (b < a) parent[a] = b;
        }
    for (uint32_t i = 0; i < n; ++i) label[i] = uf_find(parent, i);
    free(parent);
}

/*
 * PageRank by power iteration on the column-stochastic adjacency (Sec. V):
 * r^0_i = 1/n and, for iters steps,
 *     r'_i = (1 - d)/n + d * sum_{j : A_ij = 1} r_j / deg_j.
 * Reading: vertices of degree 0 contribute nothing (their mass leaks; there is
 * no renormalisation), and exactly iters steps are taken with no tolerance
 * test.  deg_j is the length of row j, which equals the out-degree because the
 * graphs are symmetric.
 */
void orc_pagerank(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, double d,
                  uint32_t iters, double *r)
{
    double *z = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    for (uint32_t i = 0; i < n; ++i) r[i] = 1.0 / (double)n;
    for (uint32_t it = 0; it < iters; ++it) {
        for (uint32_t j = 0; j < n; ++j) {
            uint32_t deg = rowptr[j + 1] - rowptr[j];
            z[j] = deg ? r[j] / (double)deg : 0.0;
        }
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < (int64_t)n; ++i) {
            double v = 0.0;
            for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) v += z[colind[e]];
            r[i] = (1.0 - d) / (double)n + d * v;
        }
    }
    free(z);
}

/* PageRank of a directed graph from its definition: with out-degree o(u) and
 * arcs u -> v (row u of the CSR lists the heads v),
 *     r'(v) = (1 - d) / n + d * sum_{u -> v} r(u) / o(u),
 * starting from r = 1/n.  Rank at vertices without out-arcs is not
 * redistributed (the reading taken for the undirected case too).  The sums
 * are pushed along rows in CSR order, one thread, so the result is fixed. */
void orc_pagerank_directed(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, double d,
                           uint32_t iters, double *r)
{
    double *acc = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    for (uint32_t i = 0; i < n; ++i) r[i] = 1.0 / (double)n;
    for (uint32_t it = 0; it < iters; ++it) {
        for (uint32_t v = 0; v < n; ++v) acc[v] = 0.0;
        for (uint32_t u = 0; u < n; ++u) {
            const uint32_t o = rowptr[u + 1] - rowptr[u];
            for (uint32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) acc[colind[e]] += r[u] / (double)o;
        }
        for (uint32_t v = 0; v < n; ++v) r[v] = (1.0 - d) / (double)n + d * acc[v];
    }
    free(acc);
}

/* Max-times on a binary matrix (Table V): y_i = max_{j in row i} x_j, 0 for an
 * empty row. */
void orc_spmv_max(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const uint64_t *x, uint64_t *y)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t m = 0;
        for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (x[colind[e]] > m) m = x[colind[e]];
        y[i] = m;
    }
}

/* Maximal independent set by rounds of local maxima (Luby's scheme with fixed
 * keys, the max-times use of Table V): a candidate whose key is at least every
 * candidate neighbour's joins the set; it and its neighbours stop being
 * candidates; repeat while candidates remain.  Vertices with key 0 are never
 * candidates.  in[v] = 1 for members.  Returns the number of rounds. */
uint32_t orc_mis(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const uint64_t *key, uint8_t *in)
{
    uint8_t *cand = (uint8_t *)malloc(n ? n : 1), *join = (uint8_t *)malloc(n ? n : 1);
    for (uint32_t v = 0; v < n; ++v) {
        cand[v] = key[v] != 0;
        in[v] = 0;
    }
    uint32_t rounds = 0;
    for (;;) {
        int any = 0;
        for (uint32_t v = 0; v < n; ++v) any |= cand[v];
        if (!any) break;
        ++rounds;
        for (uint32_t v = 0; v < n; ++v) {
            join[v] = cand[v];
            for (uint32_t e = rowptr[v]; e < rowptr[v + 1] && join[v]; ++e)
                if (cand[colind[e]] && key[colind[e]] > key[v]) join[v] = 0;
        }
        for (uint32_t v = 0; v < n; ++v)
            if (join[v]) {
                in[v] = 1;
                cand[v] = 0;
                for (uint32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) cand[colind[e]] = 0;
            }
    }
    free(cand);
    free(join);
    return rounds;
}

/* The sequential greedy independent set in decreasing key order: take a vertex
 * unless a neighbour was taken.  (With distinct keys it equals orc_mis.) */
void orc_mis_greedy(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const uint64_t *key, uint8_t *in)
{
    uint32_t *order = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    for (uint32_t v = 0; v < n; ++v) {
        order[v] = v;
        in[v] = 0;
    }
    /* insertion sort by decreasing key: small inputs only */
    for (uint32_t i = 1; i < n; ++i) {
        uint32_t v = order[i], j = i;
        while (j > 0 && key[order[j - 1]] < key[v]) {
            order[j] = order[j - 1];
            --j;
        }
        order[j] = v;
    }
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t v = order[i];
        if (!key[v]) continue;
        int free_v = 1;
        for (uint32_t e = rowptr[v]; e < rowptr[v + 1]; ++e)
            if (in[colind[e]]) free_v = 0;
        in[v] = (uint8_t)free_v;
    }
    free(order);
}

/* Colouring by successive independent sets: colour c is the orc_mis set of the
 * vertices still uncoloured (with the same keys).  colors[v] = colour of v;
 * returns the number of colours. */
uint32_t orc_color(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const uint64_t *key,
                   uint32_t *colors)
{
    uint64_t *k = (uint64_t *)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
    uint8_t *in = (uint8_t *)malloc(n ? n : 1);
    for (uint32_t v = 0; v < n; ++v) colors[v] = ORC_UNREACHED;
    uint32_t c = 0;
    for (;;) {
        int left = 0;
        for (uint32_t v = 0; v < n; ++v) {
            k[v] = colors[v] == ORC_UNREACHED ? key[v] : 0;
            left |= k[v] != 0;
        }
        if (!left) break;
        orc_mis(n, rowptr, colind, k, in);
        for (uint32_t v = 0; v < n; ++v)
            if (in[v]) colors[v] = c;
        ++c;
    }
    free(k);
    free(in);
    return c;
}

/* Eccentricity of each source: the largest finite BFS level (0 when nothing
 * else is reachable), one textbook BFS per source. */
void orc_eccentricity(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const uint32_t *srcs,
                      uint32_t nsrc, uint32_t *ecc)
{
#pragma omp parallel
    {
        uint32_t *lv = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < (int64_t)nsrc; ++s) {
            orc_bfs(n, rowptr, colind, srcs[s], lv);
            uint32_t m = 0;
            for (uint32_t v = 0; v < n; ++v)
                if (lv[v] != ORC_UNREACHED && lv[v] > m) m = lv[v];
            ecc[s] = m;
        }
        free(lv);
    }
}

/* Triangles of a simple undirected graph: for every edge (i, j) with j < i,
 * count the common neighbours k with k < j.  Each triangle k < j < i is
 * counted exactly once.  (Sec. V: the sum of (L L^T) masked by L.) */
uint64_t orc_tc(uint32_t n, const uint32_t *rowptr, const uint32_t *colind)
{
    uint64_t total = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        const uint32_t *ni = colind + rowptr[i];
        uint32_t li = 0;
        while (li < rowptr[i + 1] - rowptr[i] && ni[li] < (uint32_t)i) ++li; /* lower part of row i */
        for (uint32_t p = 0; p < li; ++p) {
            uint32_t j = ni[p];
            const uint32_t *nj = colind + rowptr[j];
            uint32_t lj = 0;
            while (lj < rowptr[j + 1] - rowptr[j] && nj[lj] < j) ++lj;
            total += intersect_count(ni, li, nj, lj);
        }
    }
    return total;
}

/* ------------------------------------------------------------------------- */
/* Local graph clustering (Table V, arithmetic semiring)                      */
/* ------------------------------------------------------------------------- */

/*
 * Personalised PageRank from one seed vertex by power iteration: p^0 = e_seed
 * and, for iters steps,
 *     p'_i = (1 - a) [i == seed] + a * sum_{j : A_ij = 1} p_j / deg_j,
 * vertices of degree 0 contributing nothing (the reading taken for PageRank).
 */
void orc_ppr(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, uint32_t seed, double a,
             uint32_t iters, double *p)
{
    double *z = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    for (uint32_t i = 0; i < n; ++i) p[i] = i == seed ? 1.0 : 0.0;
    for (uint32_t it = 0; it < iters; ++it) {
        for (uint32_t j = 0; j < n; ++j) {
            uint32_t deg = rowptr[j + 1] - rowptr[j];
            z[j] = deg ? p[j] / (double)deg : 0.0;
        }
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < (int64_t)n; ++i) {
            double v = 0.0;
            for (uint32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) v += z[colind[e]];
            p[i] = (i == (int64_t)seed ? 1.0 - a : 0.0) + a * v;
        }
    }
    free(z);
}

typedef struct {
    float q;
    uint32_t v;
} orc_sweep_item;

/* Decreasing q, then increasing vertex id. */
static int cmp_sweep(const void *pa, const void *pb)
{
    const orc_sweep_item *a = (const orc_sweep_item *)pa, *b = (const orc_sweep_item *)pb;
    if (a->q != b->q) return a->q > b->q ? -1 : 1;
    return a->v < b->v ? -1 : (a->v > b->v);
}

/*
 * Sweep cut over a score vector (the last step of local clustering).  The
 * vertices taken are those with deg_v > 0 whose quotient q_v = score_v / deg_v,
 * evaluated in single precision, is > 0; they are ordered by decreasing q_v,
 * ties by increasing id.  For each prefix S of k taken vertices (k >= 1),
 *     cut(S) = number of edges with exactly one end in S,
 *     vol(S) = sum of the degrees in S,
 *     conductance(S) = cut(S) / min(vol(S), vol(V) - vol(S)),
 * prefixes with a zero denominator not being candidates.  The prefix of least
 * conductance is chosen, the shortest one among equal conductances (compared
 * exactly, as cut_a * den_b against cut_b * den_a in 64-bit integers: both
 * factors are below 2^32).  With no candidate the chosen prefix is empty.
 *   order[n]: the taken vertices in sweep order, then every other vertex by
 *             increasing id.
 *   stats[5]: {k, cut, vol, vol(V), number taken}.
 * The graph must be undirected (cut is counted from the edges at each end).
 */
void orc_sweep_cut(uint32_t n, const uint32_t *rowptr, const uint32_t *colind, const float *score,
                   uint32_t *order, uint64_t *stats)
{
    orc_sweep_item *it = (orc_sweep_item *)malloc((size_t)(n ? n : 1) * sizeof *it);
    uint8_t *taken = (uint8_t *)calloc(n ? n : 1, 1), *in = (uint8_t *)calloc(n ? n : 1, 1);
    uint32_t m = 0;
    uint64_t vol_all = rowptr[n];
    for (uint32_t v = 0; v < n; ++v) {
        uint32_t deg = rowptr[v + 1] - rowptr[v];
        if (deg == 0) continue;
        float q = score[v] / (float)deg;
        if (q > 0.0f) {
            it[m].q = q;
            it[m].v = v;
            taken[v] = 1;
            ++m;
        }
    }
    qsort(it, m, sizeof *it, cmp_sweep);
    uint32_t o = 0;
    for (uint32_t r = 0; r < m; ++r) order[o++] = it[r].v;
    for (uint32_t v = 0; v < n; ++v)
        if (!taken[v]) order[o++] = v;

    uint64_t cut = 0, vol = 0, best_k = 0, best_cut = 0, best_vol = 0, best_den = 0;
    for (uint32_t k = 1; k <= m; ++k) {
        uint32_t v = it[k - 1].v;
        /* v joins S: its edges to S stop crossing, its other edges start */
        for (uint32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
            if (in[colind[e]]) --cut;
            else ++cut;
        }
        in[v] = 1;
        vol += rowptr[v + 1] - rowptr[v];
        uint64_t den = vol < vol_all - vol ? vol : vol_all - vol;
        if (den == 0) continue;
        if (best_k == 0 || cut * best_den < best_cut * den) {
            best_k = k;
            best_cut = cut;
            best_vol = vol;
            best_den = den;
        }
    }
    stats[0] = best_k;
    stats[1] = best_cut;
    stats[2] = best_vol;
    stats[3] = vol_all;
    stats[4] = m;
    free(it);
    free(taken);
    free(in);
}
