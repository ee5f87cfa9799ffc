/*
 * b2sr.h - C ABI of libb2sr.so: the Bit-Block Compressed Sparse Row (B2SR)
 * format and the bit-level GraphBLAS kernels on it, for AMD Instinct MI355X
 * (gfx950, wave64).
 *
 * The operations follow Bit-GraphBLAS (Chen, Sung, Shen, Tallent, Barker, Li;
 * IPDPS 2022, arXiv 2201.08560):
 *   - the format:                Sec. III-A (tile indexing), Sec. III-B and
 *                                Table II (bit packing);
 *   - matrix-vector schemes:     Sec. IV, Table III (bmv_bin_bin_bin,
 *                                bmv_bin_bin_full, bmv_bin_full_full and their
 *                                masked forms);
 *   - matrix-matrix schemes:     Sec. IV, Table IV (bmm_bin_bin_sum[_masked]);
 *   - semirings and algorithms:  Sec. V, Table V (Boolean, arithmetic and
 *                                tropical min-plus; BFS, SSSP, PR, CC, TC).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer to memory the caller
 *   allocated and owns (unless documented as a host pointer).  The library
 *   never allocates or frees caller-visible memory.  Scratch memory, where a
 *   call needs any, is a caller-supplied workspace whose size is returned by a
 *   *_workspace_bytes query; the workspace's contents on entry do not matter.
 * Streams.  Every call enqueues its kernels on `stream` (0 = the null stream)
 *   and returns without synchronising, except where documented (tile counting
 *   and the iterative algorithm drivers, which read a device flag back).
 * Errors.  Calls return B2SR_OK (0) or a negative status; arguments are
 *   validated on the host before any work is enqueued, so an error return
 *   means nothing was launched (B2SR_EHIP excepted).  No exception crosses
 *   the ABI.  b2sr_strerror() names a status; b2sr_last_hip_error() gives the
 *   text of the last HIP failure seen by the calling thread.
 * Threads.  There is no global mutable state besides that per-thread error
 *   text: calls on different streams may run concurrently.
 *
 * Matrix layout (the B2SR format)
 * -------------------------------
 * An n x n binary matrix A is cut into T x T tiles, T in {4, 8, 16, 32, 64};
 * nTR = ceil(n / T) tile-rows.  Only non-empty tiles are stored:
 *   tile_rowptr[nTR + 1]  exclusive prefix count of non-empty tiles per
 *                         tile-row (tile_rowptr[0] = 0; tiles of tile-row I
 *                         are [tile_rowptr[I], tile_rowptr[I+1]) );
 *   tile_colind[ntiles]   tile-column index of each tile, strictly ascending
 *                         within a tile-row;
 *   bits[ntiles * T]      T bit-rows per tile, in tile order.  Bit-row r of
 *                         tile t is the word bits[t*T + r]; its bit c (least
 *                         significant bit first) is A[I*T + r][J*T + c].
 *                         Word type (Table II): uint8_t for T = 4 (low nibble
 *                         used) and T = 8, uint16_t for T = 16, uint32_t for
 *                         T = 32; uint64_t for T = 64 (the 64-bit packing
 *                         type Sec. III-A lists).  Bits for rows or columns
 *                         >= n are zero.  bits must be 16-byte aligned for
 *                         T >= 16, 8-byte for T = 8, 4-byte for T = 4.
 * Indices are 32-bit: n, nnz and ntiles must be < 2^32.
 *
 * Vector layout
 * -------------
 * A bit vector over n entries is ceil(n / 32) uint32_t words; entry v is bit
 * (v % 32) of word v / 32.  On input the bits >= n must be zero; on output they
 * are written zero.  The same layout serves every T: the T-bit segment of
 * tile-column J is bits [J*T, J*T + T).
 * A full vector is n elements of the semiring's value type.
 */
#ifndef B2SR_H
#define B2SR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define B2SR_OK 0
#define B2SR_EINVAL (-1)  /* bad argument: tile size, NULL pointer, flags   */
#define B2SR_ERANGE (-2)  /* a size does not fit the 32-bit index space     */
#define B2SR_ENOSPC (-3)  /* workspace smaller than the query returned      */
#define B2SR_EHIP (-4)    /* a HIP runtime call failed                      */
#define B2SR_ENOTSUP (-5) /* unsupported semiring or combination            */

/* ---- flags ---------------------------------------------------------------- */
/* Build: keep only the strictly lower triangle (j < i) of the CSR input.  This
 * forms L for triangle counting (Sec. V, TC). */
#define B2SR_BUILD_LOWER 0x1u

/* Products. */
#define B2SR_MASK_COMPLEMENT 0x1u /* keep rows whose mask bit is 0 (BFS: not visited)    */
#define B2SR_OUT_COUNT 0x2u       /* spmv_bin_bin: y is uint32_t[n] counts (bin_bin_full)  */
#define B2SR_ACCUMULATE 0x4u      /* combine with the existing y (or *d_sum) instead of     */
                                  /* overwriting it                                          */
#define B2SR_SELF 0x8u            /* min-plus: the diagonal is a real zero (Sec. V, SSSP)   */
#define B2SR_SPARSE_X 0x10u       /* spmv_bin_bin hint: x has few set bits, so read a tile   */
                                  /* only after finding its x segment non-zero (results are  */
                                  /* the same either way; only the memory traffic differs)   */

/* Semirings for spmv_bin_full (Table V). */
#define B2SR_PLUS_TIMES_F32 1 /* arithmetic, float x / y                           */
#define B2SR_MIN_PLUS_F32 2   /* tropical min-plus, float x / y, +inf = unreachable */
#define B2SR_MIN_PLUS_U32 3   /* tropical min-plus, uint32_t x / y, 0xFFFFFFFF = inf,
                                 saturating addition                                */
#define B2SR_OR_U64 4         /* Boolean on 64 vectors at once: uint64_t x / y,
                                 y_i = OR_{A_ij = 1} x_j (multi-source BFS frontier) */
#define B2SR_MAX_TIMES_U64 5  /* the max-times semiring (Table V) on a binary matrix:
                                 y_i = max_{j : A_ij = 1} x_j over uint64_t, the empty
                                 maximum being 0 (MIS and colouring keys) */

/* A non-owning view of a B2SR matrix in device memory (layout above).
 * chunk_blocks sets how the matrix-vector products (spmv_bin_bin,
 * spmv_bin_full and the algorithms and batches built on them) divide the work:
 * each wave takes chunk_blocks consecutive blocks of tiles, a block being the
 * tiles whose loads a wave issues together (for T = 32: 64 tiles for the bit
 * and count products, 32 for 4-byte values, 16 for 8-byte values).  0 lets
 * the library size the chunks (about 65536 waves per launch); values above
 * 64 are EINVAL.  Results do not depend on it, except the rounding of float
 * sums (each split's order is fixed, so a given split is deterministic); the
 * plus-times workspace size does.  Other calls ignore it. */
typedef struct b2sr_matrix {
    uint32_t n;      /* rows = columns                         */
    uint32_t tile;   /* T: 4, 8, 16, 32 or 64                  */
    uint32_t ntiles; /* number of non-empty tiles              */
    uint32_t chunk_blocks; /* products' work split: 0 = the library's
                              choice, else 1..64 (see below)           */
    const uint32_t *tile_rowptr; /* device, nTR + 1 entries    */
    const uint32_t *tile_colind; /* device, ntiles entries     */
    const void *bits;            /* device, ntiles * T words   */
} b2sr_matrix;

/* ---- errors ------------------------------------------------------------- */
const char *b2sr_strerror(int status);
/* Text of the last HIP error seen by this thread ("" if none). */
const char *b2sr_last_hip_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int b2sr_version(void);

/* ---- format construction (Sec. III-A, III-B; Table II) -------------------
 * Conversion from CSR takes two calls, because the caller allocates the output
 * arrays once the tile count is known.
 *
 * b2sr_count_tiles: counts the non-empty T x T tiles of the CSR matrix
 *   (rowptr[n + 1], colind[nnz], device, uint32) and writes tile_rowptr
 *   (device, ceil(n/T) + 1 entries).  The total tile count is written to the
 *   HOST pointer *ntiles; the call synchronises `stream` to read it.
 *   Columns inside a row may be unsorted and may repeat.  Every column index
 *   must be < n (not checked on the device).
 *   flags: 0 or B2SR_BUILD_LOWER.
 *   Errors: EINVAL (tile not in {4,8,16,32,64}, NULL pointer with n > 0, unknown
 *   flag), ERANGE (nnz >= 2^32), EHIP.
 */
int b2sr_count_tiles(uint32_t n, uint64_t nnz, const uint32_t *rowptr, const uint32_t *colind,
                     uint32_t tile, unsigned flags, uint32_t *tile_rowptr, uint64_t *ntiles,
                     hipStream_t stream);

/*
 * b2sr_from_csr: fills tile_colind[ntiles] and bits[ntiles * T words] (device,
 *   caller-allocated) from the same CSR arrays, tile size and flags as the
 *   preceding b2sr_count_tiles, given its tile_rowptr and tile count.  Bits of
 *   repeated CSR entries are set once.  Does not synchronise.
 *   Errors: EINVAL, ERANGE, EHIP.
 */
int b2sr_from_csr(uint32_t n, uint64_t nnz, const uint32_t *rowptr, const uint32_t *colind,
                  uint32_t tile, unsigned flags, const uint32_t *tile_rowptr, uint64_t ntiles,
                  uint32_t *tile_colind, void *bits, hipStream_t stream);

/*
 * b2sr_csr_transpose: the CSR of the transposed matrix (for a directed graph,
 *   the pull matrix whose row v lists the tails u of the arcs u -> v).  Inputs
 *   as for b2sr_count_tiles (every column index < n, not checked on the
 *   device); outputs t_rowptr[n + 1] and t_colind[nnz] (device, caller
 *   allocated).  The columns within an output row come in no particular order
 *   (the B2SR build accepts that).  ws: b2sr_csr_transpose_workspace_bytes(n)
 *   bytes of device memory.  Does not synchronise.
 *   Errors: EINVAL (NULL pointer with n > 0 or nnz > 0), ENOSPC (workspace),
 *   ERANGE (nnz >= 2^32), EHIP.
 */
size_t b2sr_csr_transpose_workspace_bytes(uint32_t n);
int b2sr_csr_transpose(uint32_t n, uint64_t nnz, const uint32_t *rowptr, const uint32_t *colind,
                       uint32_t *t_rowptr, uint32_t *t_colind, void *ws, size_t ws_bytes,
                       hipStream_t stream);

/*
 * b2sr_pack_bits: vector binarisation (Sec. IV, Listing 1's packed operand):
 *   bits[ceil(n/32)] (device) receives bit v = (pred[v] != 0) for v < n, zero
 *   padding above n.  pred is n bytes (device).
 */
int b2sr_pack_bits(uint32_t n, const uint8_t *pred, uint32_t *bits, hipStream_t stream);

/* ---- matrix-vector products (Sec. IV, Table III) ------------------------
 * spmv_bin_bin: 1-bit matrix times 1-bit vector x (bit layout, ceil(n/32)
 *   words).
 *   Default (bmv_bin_bin_bin, Boolean semiring): y is a bit vector with
 *     y_i = OR_{j : A_ij = 1} x_j.
 *   B2SR_OUT_COUNT (bmv_bin_bin_full, Listing 1): y is uint32_t[n] with
 *     y_i = sum_J popcount(A's bit-row i in tile-column J AND x's segment J)
 *         = |{ j : A_ij = 1 and x_j = 1 }|.
 *   mask (nullable bit vector; the *_masked schemes of Table III, Sec. V BFS):
 *     row i is kept if its mask bit is 1, or 0 under B2SR_MASK_COMPLEMENT;
 *     the mask is applied to the result just before it is stored.  A dropped
 *     row gets the identity (0), or keeps its old value under ACCUMULATE.
 *   B2SR_ACCUMULATE: y |= result (bits) or y += result (counts).
 *   Otherwise y is overwritten.  y must not alias x or mask.
 *   B2SR_SPARSE_X: a performance hint for sparse frontiers (see the flag).
 *   Errors: EINVAL, EHIP.
 */
int spmv_bin_bin(const b2sr_matrix *A, const uint32_t *x, const uint32_t *mask, unsigned flags,
                 void *y, hipStream_t stream);

/*
 * spmv_bin_full (bmv_bin_full_full[_masked]): 1-bit matrix times a full
 *   vector x (n elements) under `semiring`:
 *   B2SR_PLUS_TIMES_F32: t_i = sum_{j : A_ij = 1} x_j * s_j, with s =
 *       col_scale (nullable: s = 1; PageRank's 1/out-degree vector, Sec. V);
 *       y_i = alpha * t_i + beta.
 *   B2SR_MIN_PLUS_F32 / _U32: t_i = min_{j : A_ij = 1} (x_j + alpha), the
 *       empty minimum being infinity; with B2SR_SELF also min'ed with x_i
 *       (the diagonal as a real zero, Sec. V SSSP); y_i = t_i.  For _U32,
 *       alpha must be a non-negative integer and additions saturate.
 *   B2SR_OR_U64: y_i = OR_{j : A_ij = 1} x_j over uint64_t words.
 *   B2SR_MAX_TIMES_U64: y_i = max_{j : A_ij = 1} x_j over uint64_t (0 when
 *       row i has no set bit).
 *   x_active (nullable bit vector over columns, the layout of x's indices):
 *   entries x_j whose bit is 0 are treated as the semiring's identity (0, or
 *   +infinity for min-plus) and tiles whose whole x segment is inactive are
 *   not read; the B2SR_SELF term still reads x_i.  Iterative algorithms pass
 *   the set of entries that changed (SSSP, CC) or are non-zero (multi-source
 *   BFS frontier words).
 *   mask / B2SR_MASK_COMPLEMENT: as for spmv_bin_bin; a dropped row gets 0
 *   (plus-times, or-u64, max-times) or infinity (min-plus), or keeps its old value under
 *   ACCUMULATE.  B2SR_ACCUMULATE: y_i = y_i + alpha t_i + beta (plus-times),
 *   min(y_i, t_i) (min-plus), y_i | t_i (or-u64), max(y_i, t_i) (max-times).
 *   Floating-point sums are deterministic: a fixed reduction order that does
 *   not depend on scheduling (rows split across work chunks are combined in
 *   chunk order by a second kernel).
 *   ws/ws_bytes: workspace of spmv_bin_full_workspace_bytes(A, semiring)
 *   bytes (may be NULL when that is 0).  For plus-times it holds the partial
 *   sums of tile-rows split across work chunks and, last, n floats for x * s;
 *   without col_scale those last 4n bytes may be left out.  With col_scale, ws
 *   must be 16-byte aligned.  y must not alias x, x_active or mask.
 *   x and col_scale must be 16-byte aligned (segments are read as vectors).
 *   Errors: EINVAL, ENOSPC, ENOTSUP (unknown semiring), EHIP.
 */
size_t spmv_bin_full_workspace_bytes(const b2sr_matrix *A, int semiring);
int spmv_bin_full(const b2sr_matrix *A, int semiring, const void *x, const float *col_scale,
                  const uint32_t *x_active, const uint32_t *mask, unsigned flags, double alpha,
                  double beta, void *y, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * spmv_bin_full_noalloc: spmv_bin_full for callers that cannot allocate device
 *   memory (code under HIP graph capture, tight serving loops, harnesses that
 *   forbid hipMalloc).  The same product, semantics, argument rules and errors
 *   as spmv_bin_full, without a workspace argument: the workspace is a
 *   library-owned device array of B2SR_NOALLOC_MAX_BYTES bytes, one per device
 *   (each device holds it from the library's first use there until the process
 *   ends).  The call allocates nothing and launches nothing when the workspace
 *   spmv_bin_full_workspace_bytes would size (without col_scale: that size less
 *   the 4n bytes of the scaled copy of x) exceeds the array: it returns
 *   B2SR_ENOSPC then.  The array is addressed on the device current at the call,
 *   so `stream` must belong to that device.  Every call on one device shares
 *   its array, and no part of it needs clearing between calls; calls whose
 *   execution overlaps on one device (different streams, or threads without
 *   ordering) race on it, so the caller orders them.
 */
#define B2SR_NOALLOC_MAX_BYTES (64u << 20)
int spmv_bin_full_noalloc(const b2sr_matrix *A, int semiring, const void *x, const float *col_scale,
                          const uint32_t *x_active, const uint32_t *mask, unsigned flags, double alpha,
                          double beta, void *y, hipStream_t stream);

/* ---- masked matrix-matrix product, summed (Sec. IV, Table IV, Listing 2) ---
 * spgemm_masked: *d_sum (device uint64_t) receives
 *     s = sum_{(i,j) : M_ij = 1} (A * B)_ij,   (A * B)_ij = sum_k A_ik B_kj,
 *   an arithmetic sum of products (not a count of nonzero outputs).  B is
 *   passed as its transpose Bt (row j of Bt holds column j of B), so that
 *   (A * B)_ij is a dot product of bit-rows of A and Bt.  M == NULL means the
 *   unmasked bmm_bin_bin_sum (every (i, j)).  A, Bt and M must have the same
 *   n and T and may alias.  Triangle counting (Sec. V) is A = Bt = M = L, the
 *   strictly lower triangle.
 *   B2SR_ACCUMULATE adds to *d_sum instead of overwriting it.
 *   ws: spgemm_masked_workspace_bytes(A, M) bytes.  Unmasked: required.
 *   Masked: optional.  When A and Bt are the same matrix (the same three
 *   arrays), a workspace of that size holds lists that let each mask tile (I, J)
 *   scan the shorter of A's tile-row I and Bt's tile-row J: about half the
 *   lookups on power-law graphs.  The result is the same with or without it:
 *   with ws NULL or smaller, every mask tile scans Bt's row J.
 *   Errors: EINVAL, ENOSPC, EHIP.
 */
size_t spgemm_masked_workspace_bytes(const b2sr_matrix *A, const b2sr_matrix *M);
int spgemm_masked(const b2sr_matrix *A, const b2sr_matrix *Bt, const b2sr_matrix *M,
                  unsigned flags, uint64_t *d_sum, void *ws, size_t ws_bytes, hipStream_t stream);

/* spgemm_masked_rows: spgemm_masked restricted to the mask's tile-rows
 *   [row_begin, row_end): *d_sum receives (or, with B2SR_ACCUMULATE, gains)
 *   the sum over the mask's ones in rows row_begin*T .. row_end*T - 1 only.
 *   Sums over consecutive ranges add up to spgemm_masked's.  M is required;
 *   no workspace (every mask tile scans Bt's row J).  It lets a caller cut one long product into shorter
 *   launches (a serving loop interleaving other work between them), and is
 *   the per-device call when mask tile-rows are split across devices.
 *   row_begin > row_end or row_end > ceil(n/T): EINVAL.  Errors: EINVAL, EHIP. */
int spgemm_masked_rows(const b2sr_matrix *A, const b2sr_matrix *Bt, const b2sr_matrix *M,
                       uint32_t row_begin, uint32_t row_end, unsigned flags, uint64_t *d_sum,
                       hipStream_t stream);

/* spgemm_masked_profile: the work spgemm_masked does for the same operands
 *   when every mask tile scans Bt's row J (no workspace)
 *   (M required), counted instead of the sum.  d_counts (device, 4 x uint64_t)
 *   receives: [0] mask tiles visited (those whose tile-row of A is non-empty),
 *   [1] tile columns of Bt looked up in A's tile-row, [2] matched tile pairs
 *   (A_IK, Bt_JK) = sum over visited mask tiles of |cols(A_I) n cols(Bt_J)|,
 *   [3] bit-row pair operations (AND + popcount of two T-bit rows) = sum over
 *   matched pairs of the mask tile's set bits.  Overwrites d_counts.
 *   Errors: EINVAL, EHIP. */
int spgemm_masked_profile(const b2sr_matrix *A, const b2sr_matrix *Bt, const b2sr_matrix *M,
                          uint64_t *d_counts, hipStream_t stream);

/* ---- graph algorithms on the products above (Sec. V) ---------------------
 * Each driver runs its iteration loop on the host, launching the kernels
 * above on `stream`, and synchronises `stream` to test convergence.  BFS,
 * multi-source BFS, SSSP, CC, eccentricity, MIS and colouring keep their
 * convergence state on the device:
 * every kernel of an iteration is gated on it, the host enqueues iterations in
 * batches of 2, 4, 8 and then 16 and reads the state once per batch, and the
 * iterations enqueued past the end return at once (MIS and colouring also read
 * one word before the first round: whether any vertex has a key).  PageRank
 * runs a fixed number of iterations and reads nothing.  These reads (and the tile count
 * of b2sr_count_tiles, and the batched BFS's flags) land in 64 bytes of pinned
 * host memory held per host thread, allocated on the thread's first read and
 * kept until the process ends (a read into pageable memory costs a staging
 * copy on the device).  The number of iterations run is
 * written to the HOST pointer *iters when it is not NULL.  ws is a workspace
 * of b2sr_algo_workspace_bytes(A, algo) bytes.  The drivers read A as the
 * pull matrix: row i lists the vertices whose edges reach i, so each product
 * y = A x moves the frontier one step along the edges.  For an undirected
 * graph that is its symmetric adjacency matrix (vxm and mxv are then the same
 * product); for a directed graph it is the transpose of the arc matrix
 * (row u of the arc matrix lists the heads of u's arcs), which
 * b2sr_csr_transpose forms from the arc CSR: BFS and SSSP then follow arcs
 * forward, and b2sr_pagerank_directed takes out-degrees from A's columns.
 * b2sr_cc needs an undirected graph.
 */
#define B2SR_ALGO_BFS 1
#define B2SR_ALGO_SSSP 2
#define B2SR_ALGO_CC 3
#define B2SR_ALGO_PAGERANK 4
#define B2SR_ALGO_MSBFS 5
#define B2SR_ALGO_MIS 6
#define B2SR_ALGO_COLOR 7
#define B2SR_ALGO_ECC 8
#define B2SR_ALGO_LGC 9
size_t b2sr_algo_workspace_bytes(const b2sr_matrix *A, int algo);

/* BFS (Sec. V): Boolean semiring, masked bin_bin_bin product per level with
 * the complement of the visited set as the mask (a level whose frontier holds
 * fewer vertices than A has tile-rows reads only the tiles behind a non-empty
 * frontier segment).  levels (uint32_t[n]): levels[src] = 0, unreachable =
 * 0xFFFFFFFF.  *iters = levels run, the last one finding nothing. */
int b2sr_bfs(const b2sr_matrix *A, uint32_t src, uint32_t *levels, void *ws, size_t ws_bytes,
             uint32_t *iters, hipStream_t stream);

/* Multi-source BFS: up to 64 sources at once as one uint64_t frontier word
 * per vertex (bit s = source s), each level one B2SR_OR_U64 product masked by
 * the visited words.  levels is nsrc x n uint32_t, row s for source srcs[s]
 * (srcs is a HOST array; sources must be distinct and < n). */
int b2sr_msbfs(const b2sr_matrix *A, const uint32_t *srcs, uint32_t nsrc, uint32_t *levels,
               void *ws, size_t ws_bytes, uint32_t *iters, hipStream_t stream);

/* SSSP with unit edge weights (Sec. V): tropical min-plus over uint32 with
 * saturating addition (B2SR_MIN_PLUS_U32, edge weight 1) and the diagonal as
 * zero, iterated to a fixpoint; exact for every n.  dist (uint32_t[n]) holds
 * hop distances, unreachable = 0xFFFFFFFF. */
int b2sr_sssp(const b2sr_matrix *A, uint32_t src, uint32_t *dist, void *ws, size_t ws_bytes,
              uint32_t *iters, hipStream_t stream);

/* Connected components (Sec. V): min-label propagation, x = min(x, A x) under
 * min-plus over uint32 with zero edge weight, from x_i = i to a fixpoint.
 * labels (uint32_t[n], 16-byte aligned: it is one of the two iterates the
 * product reads as x) ends as the smallest vertex id of each component. */
int b2sr_cc(const b2sr_matrix *A, uint32_t *labels, void *ws, size_t ws_bytes, uint32_t *iters,
            hipStream_t stream);

/* PageRank (Sec. V): r_0 = 1/n, then `iterations` steps of
 * r_i = (1 - d)/n + d * sum_{j : A_ij = 1} r_j / deg_j in float, degree-0
 * vertices contributing nothing.  rank is float[n]. */
int b2sr_pagerank(const b2sr_matrix *A, float damping, uint32_t iterations, float *rank, void *ws,
                  size_t ws_bytes, hipStream_t stream);

/* Maximal independent set (max-times, Table V): rounds of local maxima.  key
 * (device uint64_t[n], nonzero, distinct; ties let adjacent vertices both in)
 * ranks the vertices: a candidate whose key is at least every candidate
 * neighbour's (y = A max-times x over the candidates' keys) joins, then it and
 * its neighbours (an OR product) stop being candidates; repeat while any
 * remain.  With distinct keys the set equals the greedy one taken in
 * decreasing key order.  mis_bits: the set as a bit vector (device,
 * ceil(n/32) words).  *iters: rounds.  A must be undirected (symmetric). */
int b2sr_mis(const b2sr_matrix *A, const uint64_t *key, uint32_t *mis_bits, void *ws,
             size_t ws_bytes, uint32_t *iters, hipStream_t stream);

/* Graph colouring by successive independent sets (max-times, Table V): colour
 * c = 0, 1, ... is the b2sr_mis set of the vertices still uncoloured, with the
 * same keys.  colors: device uint32_t[n].  *ncolors: colours used.  A must be
 * undirected.  Workspace: b2sr_algo_workspace_bytes(A, B2SR_ALGO_COLOR). */
int b2sr_color(const b2sr_matrix *A, const uint64_t *key, uint32_t *colors, void *ws,
               size_t ws_bytes, uint32_t *ncolors, hipStream_t stream);

/* Eccentricities (BFS on the Boolean semiring, 64 sources at a time as bits of
 * one frontier word, as b2sr_msbfs, without storing levels): ecc[s] = the
 * largest finite BFS level from srcs[s] (0 for a vertex that reaches nothing).
 * srcs and ecc are HOST arrays of nsrc entries (any count; repeats allowed).
 * Convergence is kept on the device (as for b2sr_msbfs); the host reads the
 * state once per batch of levels and the eccentricities once per 64 sources,
 * so it synchronises `stream`.  Workspace:
 * b2sr_algo_workspace_bytes(A, B2SR_ALGO_ECC). */
int b2sr_eccentricity(const b2sr_matrix *A, const uint32_t *srcs, uint32_t nsrc, uint32_t *ecc,
                      void *ws, size_t ws_bytes, hipStream_t stream);

/* Diameter: the largest finite distance between two vertices, as the largest
 * eccentricity over every vertex (n / 64 batches of b2sr_eccentricity: exact,
 * and as costly as n/64 multi-source BFS runs).  *diameter is a HOST word.
 * Same workspace as b2sr_eccentricity. */
int b2sr_diameter(const b2sr_matrix *A, uint32_t *diameter, void *ws, size_t ws_bytes,
                  hipStream_t stream);

/* PageRank of a directed graph: At is the transpose of the arc matrix (the
 * pull matrix), r_0 = 1/n, then r_i(v) = (1 - d)/n + d * sum_{u -> v} r(u) / o(u)
 * with o(u) the out-degree of u, taken as the set bits of column u of At;
 * vertices without out-arcs contribute nothing.  Workspace as for
 * B2SR_ALGO_PAGERANK. */
int b2sr_pagerank_directed(const b2sr_matrix *At, float damping, uint32_t iterations, float *rank,
                           void *ws, size_t ws_bytes, hipStream_t stream);

/* Local graph clustering (Table V: arithmetic semiring).  Personalised
 * PageRank from `seed`: p_0 = e_seed, then `iterations` steps of
 *     p_i = (1 - alpha) [i == seed] + alpha * sum_{j : A_ij = 1} p_j / deg_j
 * in float (plus-times products; degree-0 vertices contribute nothing), then
 * b2sr_sweep_cut of p.  ppr: device float[n] (the final p).  cluster_bits and
 * stats as for b2sr_sweep_cut (cluster_bits nullable).  seed >= n or alpha
 * outside [0, 1]: EINVAL.  Workspace: b2sr_algo_workspace_bytes(A,
 * B2SR_ALGO_LGC).  A must be undirected. */
int b2sr_lgc(const b2sr_matrix *A, uint32_t seed, float alpha, uint32_t iterations, float *ppr,
             uint32_t *cluster_bits, uint64_t *stats, void *ws, size_t ws_bytes, hipStream_t stream);

/* Sweep cut of a score vector (the last step of local clustering).  The
 * vertices taken are those with deg_v > 0 (deg = set bits of row v) whose
 * single-precision quotient q_v = score_v / deg_v is > 0, ordered by
 * decreasing q_v, ties by increasing id.  Of the prefixes S of that order,
 * the one of least conductance cut(S) / min(vol S, vol V - vol S) is chosen
 * (cut = edges leaving S, vol = sum of degrees; the shortest prefix among
 * equal conductances, compared exactly; prefixes with a zero denominator are
 * not candidates).  Outputs (device):
 *   stats: uint64_t[5] = {size of the chosen prefix (0: none), its cut, its
 *          vol, vol V, number of vertices taken};
 *   order (nullable): uint32_t[n], the taken vertices in sweep order, then
 *          the others by increasing id;
 *   cluster_bits (nullable): ceil(n/32) words, bit v set iff v is in the
 *          chosen prefix (padding bits 0).
 * score: device float[n] (NaN and values <= 0 are not taken).  Workspace:
 * b2sr_algo_workspace_bytes(A, B2SR_ALGO_LGC).  A must be undirected. */
int b2sr_sweep_cut(const b2sr_matrix *A, const float *score, uint32_t *order, uint32_t *cluster_bits,
                   uint64_t *stats, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---- batched multi-source BFS over many graphs ---------------------------
 * Many graphs are placed in one vertex space of n vertices (each graph's ids
 * offset by a multiple of 64) and grouped by tile width; group k is the B2SR
 * matrix groups[k] (a HOST array of ngroups <= 8 views, each n x n and
 * block-diagonal).  The sources are nseeds distinct (vertex, bit) pairs given
 * as DEVICE arrays seed_vertex[] and seed_bit[] (bit < 64): bit s of a vertex's
 * 64-bit frontier word carries the BFS from the source seeded with bit s in
 * that vertex's graph, so up to 64 sources per graph run at once (seeds with
 * vertex >= n or bit >= 64 are ignored).  Each level
 * is one B2SR_OR_U64 product per group plus an element-wise update.
 * levels (DEVICE, n * 64 uint32_t, vertex-major: levels[v * 64 + s]) receives
 * the BFS level of v from source s of v's graph, 0xFFFFFFFF if unreached.
 * *iters (HOST, nullable) receives the number of levels run.
 *   mode B2SR_BATCH_LEVELS:     one product launch per group and one update
 *                               launch per level; reads one flag per level.
 *   mode B2SR_BATCH_PERSISTENT: one cooperative kernel runs all levels with
 *                               grid barriers (B2SR_ENOTSUP if the device has
 *                               no cooperative launch).
 * The call synchronises `stream` (it reads flags back).  ws: workspace of
 * b2sr_msbfs_batch_workspace_bytes(n) bytes.
 * Errors: EINVAL, ERANGE, ENOSPC, ENOTSUP, EHIP. */
#define B2SR_BATCH_LEVELS 0u
#define B2SR_BATCH_PERSISTENT 1u
size_t b2sr_msbfs_batch_workspace_bytes(uint32_t n);
int b2sr_msbfs_batch(uint32_t n, uint32_t ngroups, const b2sr_matrix *groups, uint32_t nseeds,
                     const uint32_t *seed_vertex, const uint32_t *seed_bit, uint32_t *levels,
                     unsigned mode, void *ws, size_t ws_bytes, uint32_t *iters,
                     hipStream_t stream);

/* b2sr_msbfs_batch_timed: b2sr_msbfs_batch in B2SR_BATCH_PERSISTENT mode that
 * also records where the persistent kernel's time goes.  For each of the first
 * stamp_levels levels and each of the first stamp_blocks blocks of the grid,
 * thread 0 of the block writes five readings of the device wall clock
 * (stamps[((level - 1) * stamp_blocks + block) * 5 + e], e = 0: level start,
 * 1: the block's product work done, 2: past the first grid barrier, 3: the
 * block's update done, 4: past the second barrier).  stamps: device uint64_t,
 * stamp_levels * stamp_blocks * 5 entries, zeroed first (levels not run stay
 * 0).  *grid_blocks and *clock_khz (HOST) receive the grid size and the wall
 * clock's rate in kHz.  Synchronises `stream`.  Errors as b2sr_msbfs_batch. */
int b2sr_msbfs_batch_timed(uint32_t n, uint32_t ngroups, const b2sr_matrix *groups, uint32_t nseeds,
                           const uint32_t *seed_vertex, const uint32_t *seed_bit, uint32_t *levels,
                           void *ws, size_t ws_bytes, uint64_t *stamps, uint32_t stamp_levels,
                           uint32_t stamp_blocks, uint32_t *grid_blocks, uint32_t *clock_khz,
                           uint32_t *iters, hipStream_t stream);

/* A plan instantiates the batched BFS as hipGraphs once; each launch replays
 * them.  mode B2SR_BATCH_LEVELS: the first graph holds the initialisation, the
 * seeding and 32 levels of per-level kernels, and a second graph 32 more
 * levels; the level count and a finished flag live on the device, so levels
 * after the BFS has finished return at once, and plan_launch replays the second
 * graph until the device reports the BFS finished (it synchronises `stream`).
 * mode B2SR_BATCH_PERSISTENT: one graph of initialisation, seeding and the
 * persistent kernel, whose kernel node is cooperative (the runtime checks at
 * each replay that the grid can be co-resident; plan_create returns
 * B2SR_ENOTSUP when the runtime refuses that attribute).  plan_launch
 * synchronises only when iters is not NULL, and then reports a grid barrier
 * that timed out (B2SR_EHIP).  Without iters the time-out flag stays set in the
 * plan's workspace, where it makes every later replay stop at once, until
 * b2sr_msbfs_batch_plan_status reads it: that call synchronises `stream`,
 * writes the levels run of the last replay to *iters (nullable) and returns
 * B2SR_EHIP, clearing the flag, when a barrier timed out since the last
 * status read.  The plan's workspace keeps that state between launches.
 * The plan keeps the pointers it was created with: rewrite the seed arrays in
 * device memory between launches to run other sources.  plan_create clears
 * the time-out flag with a synchronous hipMemset. */
typedef struct b2sr_msbfs_plan_s *b2sr_msbfs_plan;
int b2sr_msbfs_batch_plan_create(uint32_t n, uint32_t ngroups, const b2sr_matrix *groups,
                                 uint32_t nseeds, const uint32_t *seed_vertex,
                                 const uint32_t *seed_bit, uint32_t *levels, unsigned mode,
                                 void *ws, size_t ws_bytes, b2sr_msbfs_plan *plan);
int b2sr_msbfs_batch_plan_launch(b2sr_msbfs_plan plan, uint32_t *iters, hipStream_t stream);
int b2sr_msbfs_batch_plan_status(b2sr_msbfs_plan plan, uint32_t *iters, hipStream_t stream);
int b2sr_msbfs_batch_plan_destroy(b2sr_msbfs_plan plan);

/* ---- serving: continuous multi-source BFS sessions ------------------------
 * A session keeps the BFS state of up to 64 queries on one graph, one per bit
 * of a 64-bit frontier word per vertex (the Boolean-semiring product of
 * Sec. V's BFS, Table V, applied to 64 vectors at once).  Bit lanes are
 * independent, so queries need not start or finish together:
 *   join(slot, source): the query in `slot` starts from `source` at the
 *     session's current step (the slot must be free; slot < 64, source < n);
 *   step: one BFS level for every query in the session: Y = A (x) F over the
 *     non-zero frontier words, new = Y & ~V, V |= new, F = new.  When
 *     alive_host is not NULL, the 64-bit word whose bit s is set when slot s
 *     reached a new vertex in this step is copied to *alive_host (host memory,
 *     pinned for an asynchronous copy) in stream order; a query whose bit is 0
 *     in the first step after it joined, or in any later one, has finished;
 *   extract(slot, levels): writes the finished query's BFS levels (uint32_t[n],
 *     device; 0xFFFFFFFF = unreached) and frees the slot; levels == NULL just
 *     frees it (a cancelled query);
 *   info: steps run so far and the mask of busy slots.
 * ws: b2sr_bfs_session_bytes(n) bytes of device memory, owned by the caller
 * and used until destroy.  Calls on one session must use one stream (or be
 * ordered by the caller); sessions on different graphs or streams are
 * independent.  create zeroes the state on `stream`; destroy frees only the
 * host-side handle.  Errors: EINVAL (bad slot, busy slot on join, free slot on
 * extract, source >= n, NULL handle), ENOSPC (workspace too small), ERANGE
 * (step counter exhausted), EHIP.
 */
typedef struct b2sr_bfs_session_s *b2sr_bfs_session;
size_t b2sr_bfs_session_bytes(uint32_t n);
int b2sr_bfs_session_create(const b2sr_matrix *A, void *ws, size_t ws_bytes, hipStream_t stream,
                            b2sr_bfs_session *session);
int b2sr_bfs_session_join(b2sr_bfs_session session, uint32_t slot, uint32_t source,
                          hipStream_t stream);
int b2sr_bfs_session_step(b2sr_bfs_session session, uint64_t *alive_host, hipStream_t stream);
int b2sr_bfs_session_extract(b2sr_bfs_session session, uint32_t slot, uint32_t *levels,
                             hipStream_t stream);
int b2sr_bfs_session_info(b2sr_bfs_session session, uint32_t *step, uint64_t *busy);
int b2sr_bfs_session_destroy(b2sr_bfs_session session);

/* ---- calibration -----------------------------------------------------------
 * b2sr_stream_read: reads bytes / 16 consecutive 16-byte vectors at p (device,
 *   16-byte aligned) with nontemporal loads over B2SR_STREAM_READ_BLOCKS
 *   workgroups of 256 threads and writes to out (device,
 *   B2SR_STREAM_READ_BLOCKS words) one word per workgroup whose XOR over all
 *   workgroups is the XOR of every 32-bit word read.  Its time is the read-only
 *   bandwidth a product kernel's stream is compared with.  Errors: EINVAL, EHIP.
 */
#define B2SR_STREAM_READ_BLOCKS 8192
int b2sr_stream_read(const void *p, size_t bytes, uint32_t *out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* B2SR_H */
