// CSR -> B2SR conversion (Sec. III-A tile indexing, Sec. III-B bit packing) and
// vector binarisation.
//
// The paper converts through a float BSR intermediate produced by vendor
// library calls and then packs each tile.  Here the CSR is packed straight to
// bits: one workgroup owns one tile-row, marks the tile columns its nonzeros
// touch in an LDS bitmap (a window of up to 131072 tile columns at a time),
// counts them (pass 1), and in pass 2 turns the bitmap's popcount prefix into
// each tile's slot, writes TileColInd in ascending order and ORs every nonzero
// into its bit-row.  Unsorted and repeated CSR columns need no special case.
#include "common.h"

using namespace b2sr_dev;

namespace {

constexpr int kBuildThreads = 256;
constexpr uint32_t kWinWords = 4096;  // 16 KiB of LDS bitmap = 131072 tile columns per window
constexpr uint32_t kWinBits = kWinWords * 32;

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *s_red)
{
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
    const unsigned w = threadIdx.x / B2SR_WAVE;
    __syncthreads();
    if (lane_id() == 0) s_red[w] = v;
    __syncthreads();
    uint32_t t = 0;
    for (unsigned k = 0; k < blockDim.x / B2SR_WAVE; ++k) t += s_red[k];
    return t;
}

__device__ __forceinline__ uint32_t block_min(uint32_t v, uint32_t *s_red)
{
    for (int m = 32; m >= 1; m >>= 1) v = min(v, shfl_xor(v, m));
    const unsigned w = threadIdx.x / B2SR_WAVE;
    __syncthreads();
    if (lane_id() == 0) s_red[w] = v;
    __syncthreads();
    uint32_t t = 0xFFFFFFFFu;
    for (unsigned k = 0; k < blockDim.x / B2SR_WAVE; ++k) t = min(t, s_red[k]);
    return t;
}

__device__ __forceinline__ uint32_t block_max(uint32_t v, uint32_t *s_red)
{
    for (int m = 32; m >= 1; m >>= 1) v = max(v, shfl_xor(v, m));
    const unsigned w = threadIdx.x / B2SR_WAVE;
    __syncthreads();
    if (lane_id() == 0) s_red[w] = v;
    __syncthreads();
    uint32_t t = 0;
    for (unsigned k = 0; k < blockDim.x / B2SR_WAVE; ++k) t = max(t, s_red[k]);
    return t;
}

// Row of CSR entry e inside a tile-row whose T+1 row pointers sit in s_rp:
// the last r with s_rp[r] <= e.
__device__ __forceinline__ uint32_t row_of_entry(const uint32_t *s_rp, uint32_t nrows, uint32_t e)
{
    uint32_t lo = 0, hi = nrows;  // s_rp[lo] <= e < s_rp[hi]
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (s_rp[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

struct TileRowCtx {
    uint32_t r0, nrows, e0, e1, jmin, jmax;
};

// Loads the tile-row's row pointers and finds the range of tile columns its
// (optionally strictly-lower) nonzeros fall in.  jmin > jmax when it has none.
template <bool LOWER>
__device__ TileRowCtx tile_row_setup(uint32_t n, const uint32_t *rowptr, const uint32_t *colind,
                                     uint32_t logT, uint32_t I, uint32_t *s_rp, uint32_t *s_red)
{
    TileRowCtx c;
    const uint32_t T = 1u << logT;
    c.r0 = I * T;
    uint32_t r1 = min(c.r0 + T, n);
    c.nrows = r1 - c.r0;
    __syncthreads();
    if (threadIdx.x <= c.nrows) s_rp[threadIdx.x] = rowptr[c.r0 + threadIdx.x];
    __syncthreads();
    c.e0 = s_rp[0];
    c.e1 = s_rp[c.nrows];
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
    for (uint32_t e = c.e0 + threadIdx.x; e < c.e1; e += blockDim.x) {
        uint32_t j = colind[e];
        if (LOWER && j >= c.r0 + row_of_entry(s_rp, c.nrows, e)) continue;
        lo = min(lo, j >> logT);
        hi = max(hi, j >> logT);
    }
    c.jmin = block_min(lo, s_red);
    c.jmax = block_max(hi, s_red);
    return c;
}

// Marks the tile columns in [wbase, wbase + nw*32) of the tile-row's nonzeros.
template <bool LOWER>
__device__ void mark_window(const TileRowCtx &c, const uint32_t *colind, uint32_t logT, uint32_t wbase,
                            uint32_t nw, const uint32_t *s_rp, uint32_t *s_bm)
{
    for (uint32_t w = threadIdx.x; w < nw; w += blockDim.x) s_bm[w] = 0;
    __syncthreads();
    for (uint32_t e = c.e0 + threadIdx.x; e < c.e1; e += blockDim.x) {
        uint32_t j = colind[e];
        if (LOWER && j >= c.r0 + row_of_entry(s_rp, c.nrows, e)) continue;
        uint32_t off = (j >> logT) - wbase;
        if ((j >> logT) >= wbase && off < nw * 32) atomicOr(&s_bm[off >> 5], 1u << (off & 31));
    }
    __syncthreads();
}

template <bool LOWER>
__global__ void __launch_bounds__(kBuildThreads)
count_tiles_kernel(uint32_t n, const uint32_t *__restrict__ rowptr, const uint32_t *__restrict__ colind,
                   uint32_t logT, uint32_t ntr, uint32_t *__restrict__ tile_rowptr)
{
    __shared__ uint32_t s_bm[kWinWords];
    __shared__ uint32_t s_rp[65];
    __shared__ uint32_t s_red[kBuildThreads / B2SR_WAVE];
    for (uint32_t I = blockIdx.x; I < ntr; I += gridDim.x) {
        TileRowCtx c = tile_row_setup<LOWER>(n, rowptr, colind, logT, I, s_rp, s_red);
        uint32_t count = 0;
        if (c.jmin <= c.jmax) {
            for (uint64_t wb = c.jmin; wb <= c.jmax; wb += kWinBits) {
                uint32_t nw = (uint32_t)min<uint64_t>(kWinWords, (c.jmax - wb + 32) / 32);
                mark_window<LOWER>(c, colind, logT, (uint32_t)wb, nw, s_rp, s_bm);
                uint32_t local = 0;
                for (uint32_t w = threadIdx.x; w < nw; w += blockDim.x) local += __popc(s_bm[w]);
                count += block_sum(local, s_red);
            }
        }
        if (threadIdx.x == 0) tile_rowptr[I + 1] = count;
    }
}

// In-place scan: tile_rowptr[1..ntr] holds per-tile-row counts on entry and the
// inclusive prefix on exit; tile_rowptr[0] = 0.  One workgroup walks the array
// in blocks of 4096 entries with a running carry.
__global__ void __launch_bounds__(1024) scan_counts_kernel(uint32_t ntr, uint32_t *__restrict__ tile_rowptr)
{
    __shared__ uint32_t s_wave[1024 / B2SR_WAVE];
    constexpr uint32_t kItems = 4;
    uint32_t *p = tile_rowptr + 1;
    uint32_t carry = 0;
    if (threadIdx.x == 0) tile_rowptr[0] = 0;
    for (uint32_t base = 0; base < ntr; base += 1024 * kItems) {
        uint32_t v[kItems];
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t k = 0; k < kItems; ++k) {
            uint32_t idx = base + threadIdx.x * kItems + k;
            v[k] = idx < ntr ? p[idx] : 0;
            sum += v[k];
        }
        // inclusive scan of thread sums within the wave
        uint32_t inc = sum;
        for (unsigned d = 1; d < 64; d <<= 1) {
            uint32_t o = shfl_up(inc, d);
            if (lane_id() >= d) inc += o;
        }
        const unsigned w = threadIdx.x / B2SR_WAVE;
        if (lane_id() == 63) s_wave[w] = inc;
        __syncthreads();
        uint32_t before = carry, total = 0;
        for (unsigned k = 0; k < 1024 / B2SR_WAVE; ++k) {
            if (k < w) before += s_wave[k];
            total += s_wave[k];
        }
        uint32_t run = before + inc - sum;
#pragma unroll
        for (uint32_t k = 0; k < kItems; ++k) {
            run += v[k];
            uint32_t idx = base + threadIdx.x * kItems + k;
            if (idx < ntr) p[idx] = run;
        }
        carry += total;
        __syncthreads();
    }
}

template <bool LOWER>
__global__ void __launch_bounds__(kBuildThreads)
fill_tiles_kernel(uint32_t n, const uint32_t *__restrict__ rowptr, const uint32_t *__restrict__ colind,
                  uint32_t logT, uint32_t rbytes, uint32_t ntr, const uint32_t *__restrict__ tile_rowptr,
                  uint32_t *__restrict__ tile_colind, uint32_t *__restrict__ bits32)
{
    __shared__ uint32_t s_bm[kWinWords];
    __shared__ uint32_t s_pre[kWinWords];
    __shared__ uint32_t s_rp[65];
    __shared__ uint32_t s_red[kBuildThreads / B2SR_WAVE];
    __shared__ uint32_t s_thr[kBuildThreads];
    const uint32_t T = 1u << logT;
    for (uint32_t I = blockIdx.x; I < ntr; I += gridDim.x) {
        TileRowCtx c = tile_row_setup<LOWER>(n, rowptr, colind, logT, I, s_rp, s_red);
        if (c.jmin > c.jmax) continue;  // block-uniform
        uint32_t base = tile_rowptr[I];
        for (uint64_t wb64 = c.jmin; wb64 <= c.jmax; wb64 += kWinBits) {
            const uint32_t wb = (uint32_t)wb64;
            const uint32_t nw = (uint32_t)min<uint64_t>(kWinWords, (c.jmax - wb64 + 32) / 32);
            mark_window<LOWER>(c, colind, logT, wb, nw, s_rp, s_bm);
            // exclusive popcount prefix over bitmap words: each thread owns a run
            const uint32_t per = (nw + blockDim.x - 1) / blockDim.x;
            const uint32_t w0 = threadIdx.x * per, w1 = min(nw, w0 + per);
            uint32_t local = 0;
            for (uint32_t w = w0; w < w1; ++w) local += __popc(s_bm[w]);
            s_thr[threadIdx.x] = local;
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t run = 0;
                for (unsigned k = 0; k < blockDim.x; ++k) {
                    uint32_t t = s_thr[k];
                    s_thr[k] = run;
                    run += t;
                }
                s_red[0] = run;  // window total
            }
            __syncthreads();
            uint32_t run = s_thr[threadIdx.x];
            for (uint32_t w = w0; w < w1; ++w) {
                uint32_t m = s_bm[w];
                s_pre[w] = run;
                uint32_t k = run;
                while (m) {
                    uint32_t b = __builtin_ctz(m);
                    m &= m - 1;
                    tile_colind[base + k++] = wb + w * 32 + b;
                }
                run += __popc(s_bm[w]);
            }
            const uint32_t wtotal = s_red[0];
            __syncthreads();
            // OR every nonzero of the window into its bit-row
            for (uint32_t e = c.e0 + threadIdx.x; e < c.e1; e += blockDim.x) {
                uint32_t j = colind[e];
                uint32_t r = row_of_entry(s_rp, c.nrows, e);
                if (LOWER && j >= c.r0 + r) continue;
                uint32_t J = j >> logT;
                uint32_t off = J - wb;
                if (J < wb || off >= nw * 32) continue;
                uint32_t wi = off >> 5, bi = off & 31;
                uint32_t pos = s_pre[wi] + __popc(s_bm[wi] & ((1u << bi) - 1u));
                // bit (r, j % T) of the tile, counted from the start of bits
                const uint64_t bit = ((uint64_t)(base + pos) * T + r) * rbytes * 8 + (j & (T - 1));
                atomicOr(&bits32[bit >> 5], 1u << (bit & 31));
            }
            base += wtotal;
            __syncthreads();
        }
    }
}

__global__ void fill_u32_kernel(uint32_t *__restrict__ p, uint64_t count, uint32_t value)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// One wave turns 64 predicate bytes into two bit words with a 64-bit ballot.
__global__ void __launch_bounds__(256) pack_bits_kernel(uint32_t n, const uint8_t *__restrict__ pred,
                                                        uint32_t *__restrict__ bits)
{
    const uint32_t nwords = (n + 31) / 32;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE;
         wv * 2 < nwords; wv += waves) {
        uint64_t v = wv * 64 + lane_id();
        bool p = v < n && pred[v] != 0;
        uint64_t m = __ballot(p);
        uint64_t w = wv * 2 + lane_id();
        if (lane_id() < 2 && w < nwords) bits[w] = (uint32_t)(m >> (32 * lane_id()));
    }
}

inline uint32_t log2_tile(uint32_t T) { return T == 4 ? 2 : T == 8 ? 3 : T == 16 ? 4 : T == 32 ? 5 : 6; }

// ---- CSR transpose (directed graphs: the pull matrix A^T from the CSR of A)
// Counts land at t_rowptr[v + 1]; the in-place scan above turns them into row
// pointers; each arc u -> v then takes the next free position of row v.
__global__ void transpose_count_kernel(uint64_t nnz, const uint32_t *__restrict__ colind, uint32_t *t_rowptr)
{
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(t_rowptr + colind[e] + 1, 1u);
}

__global__ void transpose_cursor_kernel(uint32_t n, const uint32_t *__restrict__ t_rowptr, uint32_t *cursor)
{
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
        cursor[v] = t_rowptr[v];
}

// One wave per source row, lanes striding over its arcs.
__global__ void transpose_scatter_kernel(uint32_t n, const uint32_t *__restrict__ rowptr,
                                         const uint32_t *__restrict__ colind, uint32_t *cursor, uint32_t *t_colind)
{
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t u = (uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE; u < n; u += waves) {
        const uint32_t e1 = rowptr[u + 1];
        for (uint32_t e = rowptr[u] + lane_id(); e < e1; e += B2SR_WAVE) {
            const uint32_t v = colind[e];
            t_colind[atomicAdd(cursor + v, 1u)] = (uint32_t)u;
        }
    }
}

int validate_csr(uint32_t n, uint64_t nnz, const uint32_t *rowptr, const uint32_t *colind, uint32_t tile,
                 unsigned flags)
{
    if (!b2sr::valid_tile(tile)) return B2SR_EINVAL;
    if (flags & ~B2SR_BUILD_LOWER) return B2SR_EINVAL;
    if (nnz >= (1ull << 32) || n > 0xFFFFFF00u) return B2SR_ERANGE;
    if (n > 0 && !rowptr) return B2SR_EINVAL;
    if (nnz > 0 && !colind) return B2SR_EINVAL;
    return B2SR_OK;
}

}  // namespace

namespace b2sr {
int fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t stream)
{
    if (count == 0) return B2SR_OK;
    fill_u32_kernel<<<grid_for(count, 256, 65536), 256, 0, stream>>>(p, count, value);
    return check_launch("fill_u32_kernel");
}
}  // namespace b2sr

extern "C" {

int b2sr_count_tiles(uint32_t n, uint64_t nnz, const uint32_t *rowptr, const uint32_t *colind,
                     uint32_t tile, unsigned flags, uint32_t *tile_rowptr, uint64_t *ntiles,
                     hipStream_t stream)
{
    int rc = validate_csr(n, nnz, rowptr, colind, tile, flags);
    if (rc) return rc;
    if (!tile_rowptr || !ntiles) return B2SR_EINVAL;
    const uint32_t ntr = b2sr::n_tile_rows(n, tile);
    const unsigned grid = b2sr::grid_for(ntr, 1, 1u << 16);
    if (ntr > 0) {
        if (flags & B2SR_BUILD_LOWER)
            count_tiles_kernel<true><<<grid, kBuildThreads, 0, stream>>>(n, rowptr, colind, log2_tile(tile), ntr,
                                                                         tile_rowptr);
        else
            count_tiles_kernel<false><<<grid, kBuildThreads, 0, stream>>>(n, rowptr, colind, log2_tile(tile), ntr,
                                                                          tile_rowptr);
        if ((rc = b2sr::check_launch("count_tiles_kernel"))) return rc;
    }
    scan_counts_kernel<<<1, 1024, 0, stream>>>(ntr, tile_rowptr);
    if ((rc = b2sr::check_launch("scan_counts_kernel"))) return rc;
    uint32_t total = 0;
    if ((rc = b2sr::read_words(tile_rowptr + ntr, &total, 1, stream))) return rc;
    *ntiles = total;
    return B2SR_OK;
}

int b2sr_from_csr(uint32_t n, uint64_t nnz, const uint32_t *rowptr, const uint32_t *colind, uint32_t tile,
                  unsigned flags, const uint32_t *tile_rowptr, uint64_t ntiles, uint32_t *tile_colind, void *bits,
                  hipStream_t stream)
{
    int rc = validate_csr(n, nnz, rowptr, colind, tile, flags);
    if (rc) return rc;
    if (ntiles >= (1ull << 32)) return B2SR_ERANGE;
    if (n > 0 && !tile_rowptr) return B2SR_EINVAL;
    if (ntiles > 0 && (!tile_colind || !bits)) return B2SR_EINVAL;
    if (bits && ((uintptr_t)bits & 3)) return B2SR_EINVAL;
    if (ntiles == 0) return B2SR_OK;
    const uint32_t ntr = b2sr::n_tile_rows(n, tile);
    if ((rc = b2sr::fill_u32((uint32_t *)bits, b2sr::bits_bytes(ntiles, tile) / 4, 0, stream))) return rc;
    const unsigned grid = b2sr::grid_for(ntr, 1, 1u << 16);
    if (flags & B2SR_BUILD_LOWER)
        fill_tiles_kernel<true><<<grid, kBuildThreads, 0, stream>>>(n, rowptr, colind, log2_tile(tile),
                                                                    b2sr::row_bytes(tile), ntr, tile_rowptr,
                                                                    tile_colind, (uint32_t *)bits);
    else
        fill_tiles_kernel<false><<<grid, kBuildThreads, 0, stream>>>(n, rowptr, colind, log2_tile(tile),
                                                                     b2sr::row_bytes(tile), ntr, tile_rowptr,
                                                                     tile_colind, (uint32_t *)bits);
    return b2sr::check_launch("fill_tiles_kernel");
}

size_t b2sr_csr_transpose_workspace_bytes(uint32_t n) { return ((size_t)n * 4 + 255) & ~(size_t)255; }

int b2sr_csr_transpose(uint32_t n, uint64_t nnz, const uint32_t *rowptr, const uint32_t *colind, uint32_t *t_rowptr,
                       uint32_t *t_colind, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (nnz >= (1ull << 32)) return B2SR_ERANGE;
    if (n > 0 && (!rowptr || !t_rowptr)) return B2SR_EINVAL;
    if (nnz > 0 && (!colind || !t_colind)) return B2SR_EINVAL;
    if (n > 0 && (!ws || ws_bytes < b2sr_csr_transpose_workspace_bytes(n))) return B2SR_ENOSPC;
    if (n == 0) {
        if (t_rowptr) return b2sr::fill_u32(t_rowptr, 1, 0, stream);
        return B2SR_OK;
    }
    int rc = b2sr::fill_u32(t_rowptr, (uint64_t)n + 1, 0, stream);
    if (rc) return rc;
    if (nnz) {
        transpose_count_kernel<<<b2sr::grid_for(nnz, 256, 8192), 256, 0, stream>>>(nnz, colind, t_rowptr);
        if ((rc = b2sr::check_launch("transpose_count_kernel"))) return rc;
    }
    scan_counts_kernel<<<1, 1024, 0, stream>>>(n, t_rowptr);
    if ((rc = b2sr::check_launch("scan_counts_kernel"))) return rc;
    if (!nnz) return B2SR_OK;
    uint32_t *cursor = (uint32_t *)ws;
    transpose_cursor_kernel<<<b2sr::grid_for(n, 256, 8192), 256, 0, stream>>>(n, t_rowptr, cursor);
    if ((rc = b2sr::check_launch("transpose_cursor_kernel"))) return rc;
    transpose_scatter_kernel<<<b2sr::grid_for(n, 4, 16384), 256, 0, stream>>>(n, rowptr, colind, cursor, t_colind);
    return b2sr::check_launch("transpose_scatter_kernel");
}

int b2sr_pack_bits(uint32_t n, const uint8_t *pred, uint32_t *bits, hipStream_t stream)
{
    if (n > 0xFFFFFF00u) return B2SR_ERANGE;
    if (n > 0 && (!pred || !bits)) return B2SR_EINVAL;
    if (n == 0) return B2SR_OK;
    const uint32_t nwords = b2sr::n_words(n);
    pack_bits_kernel<<<b2sr::grid_for((nwords + 1) / 2, 4, 65536), 256, 0, stream>>>(n, pred, bits);
    return b2sr::check_launch("pack_bits_kernel");
}

}  // extern "C"
