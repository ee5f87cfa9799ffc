// Local graph clustering (Table V lists it under the arithmetic semiring):
// personalised PageRank from a seed by plus-times products, then a sweep cut
// over the vertices in decreasing p_v / deg_v.
//
// The sweep is data-parallel instead of a walk over the sorted vertices:
//   1. sort keys: ~bits(p_v / deg_v) for the vertices taken (a positive
//      quotient), all ones for the rest; a stable LSD radix sort of (key, id)
//      gives the sweep order with ties by increasing id;
//   2. rank[v] = position of v in that order;
//   3. vol_k = prefix sum of the degrees in sweep order;
//   4. cut_k: an edge (u, v) with rank_u < rank_v crosses the prefixes of size
//      k in (rank_u, rank_v], so it adds +1 at rank_u and -1 at rank_v of a
//      difference array whose prefix sum is the cut of every prefix;
//   5. the least cut_k / min(vol_k, vol_all - vol_k), compared exactly as
//      128-bit cross products, the smallest k among equals.
#include <algorithm>
#include <utility>

#include "common.h"
#include "scan.h"

using namespace b2sr_dev;

namespace b2sr {
int fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t stream);
size_t lgc_workspace_bytes(const b2sr_matrix *A);
}

namespace {

constexpr unsigned kThreads = 256;
constexpr unsigned kWaves = kThreads / 64;
static_assert(kThreads == 256, "the radix kernels give one thread per digit");

unsigned vgrid(uint64_t n) { return b2sr::grid_for(n, kThreads, 8192); }

// ---------------------------------------------------------------- prefix sums
using b2sr_scan::block_exclusive;
using b2sr_scan::device_scan;
using b2sr_scan::LoadArray;
using b2sr_scan::scan_blocks;

struct LoadDegreeInOrder {
    const uint32_t *deg, *order;
    __device__ uint64_t operator()(uint64_t i) const { return deg[order[i]]; }
};

// ---------------------------------------------------------------- radix sort
// Stable LSD sort of (key, value) pairs, 8 bits per pass.  A block owns
// kSortTile consecutive pairs and wave w of the block the w-th quarter, so
// the order inside a block is (wave, round, lane).  Histograms are stored
// digit-major (digit * nblocks + block): their exclusive scan is every
// block's first output slot per digit.
constexpr unsigned kSortItems = 16, kSortTile = kThreads * kSortItems, kSortWaveItems = kSortItems * 64;

uint32_t sort_blocks(uint32_t n) { return (uint32_t)(((uint64_t)n + kSortTile - 1) / kSortTile); }

__global__ void __launch_bounds__(kThreads) radix_hist_kernel(uint32_t n, const uint32_t *__restrict__ keys,
                                                              unsigned shift, uint32_t nb, uint32_t *hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    for (unsigned k = 0; k < kSortItems; ++k) {
        const uint64_t i = base + (uint64_t)k * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kThreads)
    radix_scatter_kernel(uint32_t n, const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                         unsigned shift, uint32_t nb, const uint32_t *__restrict__ offsets,
                         uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out)
{
    __shared__ uint32_t cursor[kWaves][256];
    const unsigned lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (unsigned i = threadIdx.x; i < kWaves * 256; i += kThreads) (&cursor[0][0])[i] = 0;
    __syncthreads();
    const uint64_t wbase = (uint64_t)blockIdx.x * kSortTile + (uint64_t)w * kSortWaveItems;
    for (unsigned r = 0; r < kSortItems; ++r) {
        const uint64_t i = wbase + r * 64 + lane;
        if (i < n) atomicAdd(&cursor[w][(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    {
        // thread d turns the per-wave counts of digit d into first slots
        const unsigned d = threadIdx.x;
        uint32_t run = offsets[(uint64_t)d * nb + blockIdx.x];
        for (unsigned v = 0; v < kWaves; ++v) {
            const uint32_t c = cursor[v][d];
            cursor[v][d] = run;
            run += c;
        }
    }
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    for (unsigned r = 0; r < kSortItems; ++r) {
        const uint64_t i = wbase + r * 64 + lane;
        const bool ok = i < n;
        const uint32_t key = ok ? keys[i] : 0u, d = (key >> shift) & 255u;
        // lanes holding the same digit: agree on all 8 digit bits
        uint64_t peers = __ballot(ok);
        for (unsigned b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        if (ok) {
            const uint32_t pos = cursor[w][d] + (uint32_t)__popcll(peers & below);
            keys_out[pos] = key;
            vals_out[pos] = vals[i];
            if ((peers >> lane) == 1ull) cursor[w][d] = pos + 1;  // the last peer moves the cursor
        }
    }
}

// ---------------------------------------------------------------- sweep steps
__global__ void sweep_keys_kernel(uint32_t n, const float *__restrict__ score, const uint32_t *__restrict__ deg,
                                  uint32_t *keys, uint32_t *vals, uint32_t *ntaken)
{
    uint32_t c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t dg = deg[i];
        const float q = dg ? score[i] / (float)dg : 0.0f;
        const bool take = dg != 0 && q > 0.0f;
        keys[i] = take ? ~__float_as_uint(q) : 0xFFFFFFFFu;
        vals[i] = (uint32_t)i;
        c += take;
    }
    uint32_t total;
    block_exclusive(c, &total);
    if (threadIdx.x == 0 && total) atomicAdd(ntaken, total);
}

__global__ void rank_kernel(uint32_t n, const uint32_t *__restrict__ order, uint32_t *rank)
{
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x)
        rank[order[r]] = (uint32_t)r;
}

template <int T> __device__ __forceinline__ row_t<T> row_word(const void *bits, uint64_t t, uint32_t r)
{
    if constexpr (T == 64) return ((const uint64_t *)bits)[t * 64 + r];
    else if constexpr (T == 32) return ((const uint32_t *)bits)[t * 32 + r];
    else if constexpr (T == 16) return ((const uint16_t *)bits)[t * 16 + r];
    else if constexpr (T == 8) return ((const uint8_t *)bits)[t * 8 + r];
    else return ((const uint8_t *)bits)[t * 4 + r] & 0xFu;
}

// Difference array of the prefix cuts.  A wave takes kEdgeChunk consecutive
// tiles, 64 / T at a time, lane = (tile, bit-row); each lane finds its tile-row
// once by binary search and then walks forward.  The +1s of one row are summed
// in a register until the row changes.
constexpr uint32_t kEdgeChunk = 256;

template <int T>
__global__ void __launch_bounds__(kThreads)
    sweep_edges_kernel(uint32_t n, uint32_t ntr, uint32_t ntiles, const uint32_t *__restrict__ tile_rowptr,
                       const uint32_t *__restrict__ tile_colind, const void *__restrict__ bits,
                       const uint32_t *__restrict__ rank, const uint32_t *__restrict__ ntaken_p,
                       unsigned long long *diff)
{
    constexpr uint32_t kPerStep = 64 / T;
    const uint32_t ntaken = *ntaken_p;
    const unsigned lane = threadIdx.x & 63, sub = lane / T, r = lane % T;
    const uint64_t wave = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kThreads) >> 6;
    const uint64_t nchunks = ((uint64_t)ntiles + kEdgeChunk - 1) / kEdgeChunk;
    for (uint64_t c = wave; c < nchunks; c += nwaves) {
        const uint32_t t0 = (uint32_t)(c * kEdgeChunk);
        const uint32_t t1 = (uint32_t)std::min<uint64_t>(ntiles, (uint64_t)t0 + kEdgeChunk);
        uint32_t t = t0 + sub;
        if (t >= t1) continue;
        uint32_t lo = 0, hi = ntr;  // largest tr with tile_rowptr[tr] <= t; tile_rowptr[ntr] = ntiles > t
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo + 1) / 2;
            if (tile_rowptr[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        uint32_t tr = lo, row = 0xFFFFFFFFu, ru = 0xFFFFFFFFu, plus = 0;
        for (; t < t1; t += kPerStep) {
            while (tr + 1 < ntr && tile_rowptr[tr + 1] <= t) ++tr;
            const uint32_t u = tr * T + r;
            if (u != row) {
                if (plus) atomicAdd(&diff[ru], (unsigned long long)plus);
                plus = 0;
                row = u;
                ru = u < n ? rank[u] : 0xFFFFFFFFu;
            }
            if (ru >= ntaken) continue;
            row_t<T> word = row_word<T>(bits, t, r);
            const uint32_t cbase = tile_colind[t] * T;
            while (word) {
                const uint32_t v = cbase + (uint32_t)(T == 64 ? __builtin_ctzll(word) : __builtin_ctz((uint32_t)word));
                word &= word - 1;
                const uint32_t rv = v < n ? rank[v] : 0u;  // bits past n are never set in a valid matrix
                if (ru < rv) {
                    ++plus;
                    if (rv < ntaken) atomicAdd(&diff[rv], ~0ull);  // -1 modulo 2^64
                }
            }
        }
        if (plus) atomicAdd(&diff[ru], (unsigned long long)plus);
    }
}

// Candidate prefix (k = 0: none) and its exact comparison.
struct Best {
    uint64_t cut, den;
    uint32_t k;
};

__device__ __forceinline__ bool less128(uint64_t a, uint64_t b, uint64_t c, uint64_t d)  // a*b < c*d
{
    const uint64_t h1 = __umul64hi(a, b), h2 = __umul64hi(c, d);
    return h1 != h2 ? h1 < h2 : a * b < c * d;
}

__device__ __forceinline__ bool better(const Best &a, const Best &b)
{
    if (!a.k) return false;
    if (!b.k) return true;
    if (less128(a.cut, b.den, b.cut, a.den)) return true;
    if (less128(b.cut, a.den, a.cut, b.den)) return false;
    return a.k < b.k;
}

__device__ Best block_best(Best b)
{
    __shared__ uint64_t s_cut[kWaves], s_den[kWaves];
    __shared__ uint32_t s_k[kWaves];
    for (int m = 32; m >= 1; m >>= 1) {
        Best o{shfl_xor(b.cut, m), shfl_xor(b.den, m), shfl_xor(b.k, m)};
        if (better(o, b)) b = o;
    }
    const unsigned w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_cut[w] = b.cut;
        s_den[w] = b.den;
        s_k[w] = b.k;
    }
    __syncthreads();
    Best r{0, 0, 0};
    for (unsigned i = 0; i < kWaves; ++i) {
        Best o{s_cut[i], s_den[i], s_k[i]};
        if (better(o, r)) r = o;
    }
    return r;
}

constexpr unsigned kBestBlocks = 1024;

// cut and vol hold the inclusive prefix sums over ranks: prefix k ends at rank k - 1.
__global__ void __launch_bounds__(kThreads)
    sweep_best_kernel(uint32_t n, const uint32_t *__restrict__ ntaken_p, const uint64_t *__restrict__ cut,
                      const uint64_t *__restrict__ vol, uint64_t *part)
{
    const uint32_t ntaken = *ntaken_p;
    const uint64_t vol_all = vol[n - 1];
    Best b{0, 0, 0};
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ntaken; r += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t v = vol[r], den = v < vol_all - v ? v : vol_all - v;
        Best o{cut[r], den, (uint32_t)r + 1};
        if (den && better(o, b)) b = o;
    }
    b = block_best(b);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = b.cut;
        part[3 * blockIdx.x + 1] = b.den;
        part[3 * blockIdx.x + 2] = b.k;
    }
}

__global__ void __launch_bounds__(kThreads)
    sweep_final_kernel(uint32_t n, uint32_t nparts, const uint64_t *__restrict__ part, const uint32_t *__restrict__ ntaken_p,
                       const uint64_t *__restrict__ vol, uint64_t *stats)
{
    Best b{0, 0, 0};
    for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x) {
        Best o{part[3 * i], part[3 * i + 1], (uint32_t)part[3 * i + 2]};
        if (better(o, b)) b = o;
    }
    b = block_best(b);
    if (threadIdx.x == 0) {
        stats[0] = b.k;
        stats[1] = b.k ? b.cut : 0;
        stats[2] = b.k ? vol[b.k - 1] : 0;
        stats[3] = vol[n - 1];
        stats[4] = *ntaken_p;
    }
}

__global__ void cluster_bits_kernel(uint32_t n, const uint32_t *__restrict__ rank, const uint64_t *__restrict__ stats,
                                    uint32_t *bits)
{
    const uint64_t k = stats[0];
    const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t wv = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; wv * 64 < n; wv += waves) {
        const uint64_t v = wv * 64 + lane_id();
        const uint64_t m = __ballot(v < n && rank[v] < k);
        const uint64_t w = wv * 2 + lane_id();
        if (lane_id() < 2 && w < (n + 31u) / 32u) bits[w] = (uint32_t)(m >> (32 * lane_id()));
    }
}

// ---------------------------------------------------------------- personalised PageRank
__global__ void ones_bits_kernel(uint32_t n, uint32_t *bits)
{
    const uint32_t nw = (n + 31) / 32;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t hi = (uint32_t)std::min<uint64_t>(32, n - w * 32);
        bits[w] = hi == 32 ? 0xFFFFFFFFu : ((1u << hi) - 1u);
    }
}

__global__ void ppr_init_kernel(uint32_t n, uint32_t seed, const uint32_t *__restrict__ deg, float *inv, float *p)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        inv[i] = deg[i] ? 1.0f / (float)deg[i] : 0.0f;
        p[i] = i == seed ? 1.0f : 0.0f;
    }
}

__global__ void ppr_scale_kernel(uint32_t n, const float *__restrict__ p, const float *__restrict__ inv, float *z)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        z[i] = p[i] * inv[i];
}

__global__ void ppr_restart_kernel(float *p, uint32_t seed, float restart) { p[seed] += restart; }

__global__ void copy_u32_kernel(uint64_t n, const uint32_t *__restrict__ a, uint32_t *b)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// ---------------------------------------------------------------- workspace
struct Carver {
    char *base;
    size_t off = 0;
    template <class P> P *take(size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        P *p = base ? (P *)(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

struct Layout {
    uint32_t *deg, *ones, *keys0, *vals0, *keys1, *vals1, *rank, *hist, *ntaken;
    uint64_t *vol, *cut, *sums, *part;
    float *z, *inv, *p2;
    void *spmv_ws;
    size_t spmv_ws_bytes, bytes;
};

Layout carve(const b2sr_matrix *A, void *ws)
{
    Carver c{(char *)ws};
    Layout L;
    const size_t n = A->n, nw = b2sr::n_words(A->n);
    const uint32_t nbs = sort_blocks(A->n);
    const uint64_t nsums = std::max<uint64_t>(scan_blocks(n), scan_blocks((uint64_t)256 * nbs));
    L.deg = c.take<uint32_t>(n * 4);
    L.ones = c.take<uint32_t>(nw * 4);
    L.keys0 = c.take<uint32_t>(n * 4);
    L.vals0 = c.take<uint32_t>(n * 4);
    L.keys1 = c.take<uint32_t>(n * 4);
    L.vals1 = c.take<uint32_t>(n * 4);
    L.rank = c.take<uint32_t>(n * 4);
    L.hist = c.take<uint32_t>((size_t)256 * nbs * 4);
    L.ntaken = c.take<uint32_t>(4);
    L.vol = c.take<uint64_t>(n * 8);
    L.cut = c.take<uint64_t>(n * 8);
    L.sums = c.take<uint64_t>(nsums * 8);
    L.part = c.take<uint64_t>((size_t)3 * kBestBlocks * 8);
    L.z = c.take<float>(n * 4);
    L.inv = c.take<float>(n * 4);
    L.p2 = c.take<float>(n * 4);
    L.spmv_ws_bytes = spmv_bin_full_workspace_bytes(A, B2SR_PLUS_TIMES_F32);
    L.spmv_ws = c.take<char>(L.spmv_ws_bytes);
    L.bytes = c.off;
    return L;
}

int check_args(const b2sr_matrix *A, void *ws, size_t ws_bytes, Layout *L)
{
    if (int rc = b2sr::validate_matrix(A)) return rc;
    if (!ws) return B2SR_ENOSPC;
    *L = carve(A, ws);
    return ws_bytes < L->bytes ? B2SR_ENOSPC : B2SR_OK;
}

// Row degrees as the count product with the all-ones vector (bin_bin_full).
int degrees(const b2sr_matrix *A, const Layout &L, hipStream_t s)
{
    ones_bits_kernel<<<vgrid(b2sr::n_words(A->n)), kThreads, 0, s>>>(A->n, L.ones);
    if (int rc = b2sr::check_launch("ones_bits_kernel")) return rc;
    return spmv_bin_bin(A, L.ones, nullptr, B2SR_OUT_COUNT, L.deg, s);
}

template <int T> int launch_edges(const b2sr_matrix *A, const Layout &L, hipStream_t s)
{
    const uint64_t nchunks = ((uint64_t)A->ntiles + kEdgeChunk - 1) / kEdgeChunk;
    sweep_edges_kernel<T><<<b2sr::grid_for(nchunks, kWaves, 65536), kThreads, 0, s>>>(
        A->n, b2sr::n_tile_rows(A->n, A->tile), A->ntiles, A->tile_rowptr, A->tile_colind, A->bits, L.rank,
        L.ntaken, (unsigned long long *)L.cut);
    return b2sr::check_launch("sweep_edges_kernel");
}

// The sweep of `score` once L.deg holds the degrees.
int sweep(const b2sr_matrix *A, const float *score, const Layout &L, uint32_t *order, uint32_t *cluster_bits,
          uint64_t *stats, hipStream_t s)
{
    const uint32_t n = A->n;
    int rc;
    if (n == 0) return b2sr::fill_u32((uint32_t *)stats, 10, 0, s);
    if ((rc = b2sr::fill_u32(L.ntaken, 1, 0, s))) return rc;
    sweep_keys_kernel<<<vgrid(n), kThreads, 0, s>>>(n, score, L.deg, L.keys0, L.vals0, L.ntaken);
    if ((rc = b2sr::check_launch("sweep_keys_kernel"))) return rc;

    const uint32_t nbs = sort_blocks(n);
    uint32_t *kin = L.keys0, *vin = L.vals0, *kout = L.keys1, *vout = L.vals1;
    for (unsigned shift = 0; shift < 32; shift += 8) {
        radix_hist_kernel<<<nbs, kThreads, 0, s>>>(n, kin, shift, nbs, L.hist);
        if ((rc = b2sr::check_launch("radix_hist_kernel"))) return rc;
        if ((rc = device_scan<uint32_t>((uint64_t)256 * nbs, LoadArray<uint32_t>{L.hist}, L.hist, false,
                                        (uint32_t *)L.sums, s)))
            return rc;
        radix_scatter_kernel<<<nbs, kThreads, 0, s>>>(n, kin, vin, shift, nbs, L.hist, kout, vout);
        if ((rc = b2sr::check_launch("radix_scatter_kernel"))) return rc;
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    // four passes: the sorted ids are back in vals0
    rank_kernel<<<vgrid(n), kThreads, 0, s>>>(n, vin, L.rank);
    if ((rc = b2sr::check_launch("rank_kernel"))) return rc;
    if ((rc = device_scan<uint64_t>(n, LoadDegreeInOrder{L.deg, vin}, L.vol, true, L.sums, s))) return rc;
    if ((rc = b2sr::fill_u32((uint32_t *)L.cut, (uint64_t)n * 2, 0, s))) return rc;
    switch (A->tile) {
    case 4: rc = launch_edges<4>(A, L, s); break;
    case 8: rc = launch_edges<8>(A, L, s); break;
    case 16: rc = launch_edges<16>(A, L, s); break;
    case 64: rc = launch_edges<64>(A, L, s); break;
    default: rc = launch_edges<32>(A, L, s); break;
    }
    if (rc) return rc;
    if ((rc = device_scan<uint64_t>(n, LoadArray<uint64_t>{L.cut}, L.cut, true, L.sums, s))) return rc;
    const unsigned nparts = b2sr::grid_for(n, kThreads, kBestBlocks);
    sweep_best_kernel<<<nparts, kThreads, 0, s>>>(n, L.ntaken, L.cut, L.vol, L.part);
    if ((rc = b2sr::check_launch("sweep_best_kernel"))) return rc;
    sweep_final_kernel<<<1, kThreads, 0, s>>>(n, nparts, L.part, L.ntaken, L.vol, stats);
    if ((rc = b2sr::check_launch("sweep_final_kernel"))) return rc;
    if (cluster_bits) {
        cluster_bits_kernel<<<vgrid(n), kThreads, 0, s>>>(n, L.rank, stats, cluster_bits);
        if ((rc = b2sr::check_launch("cluster_bits_kernel"))) return rc;
    }
    if (order) {
        copy_u32_kernel<<<vgrid(n), kThreads, 0, s>>>(n, vin, order);
        if ((rc = b2sr::check_launch("copy_u32_kernel"))) return rc;
    }
    return B2SR_OK;
}

}  // namespace

namespace b2sr {
size_t lgc_workspace_bytes(const b2sr_matrix *A) { return carve(A, nullptr).bytes; }
}  // namespace b2sr

extern "C" {

int b2sr_sweep_cut(const b2sr_matrix *A, const float *score, uint32_t *order, uint32_t *cluster_bits,
                   uint64_t *stats, void *ws, size_t ws_bytes, hipStream_t stream)
{
    Layout L;
    int rc = check_args(A, ws, ws_bytes, &L);
    if (rc) return rc;
    if (!stats || (A->n && !score)) return B2SR_EINVAL;
    if (A->n && (rc = degrees(A, L, stream))) return rc;
    return sweep(A, score, L, order, cluster_bits, stats, stream);
}

int b2sr_lgc(const b2sr_matrix *A, uint32_t seed, float alpha, uint32_t iterations, float *ppr,
             uint32_t *cluster_bits, uint64_t *stats, void *ws, size_t ws_bytes, hipStream_t stream)
{
    Layout L;
    int rc = check_args(A, ws, ws_bytes, &L);
    if (rc) return rc;
    if (!ppr || !stats || seed >= A->n || !(alpha >= 0.0f && alpha <= 1.0f)) return B2SR_EINVAL;
    const uint32_t n = A->n;
    if ((rc = degrees(A, L, stream))) return rc;
    float *p = ppr, *p_next = L.p2;
    ppr_init_kernel<<<vgrid(n), kThreads, 0, stream>>>(n, seed, L.deg, L.inv, p);
    if ((rc = b2sr::check_launch("ppr_init_kernel"))) return rc;
    const float restart = (float)(1.0 - (double)alpha);
    for (uint32_t it = 0; it < iterations; ++it) {
        ppr_scale_kernel<<<vgrid(n), kThreads, 0, stream>>>(n, p, L.inv, L.z);
        if ((rc = b2sr::check_launch("ppr_scale_kernel"))) return rc;
        if ((rc = spmv_bin_full(A, B2SR_PLUS_TIMES_F32, L.z, nullptr, nullptr, nullptr, 0, alpha, 0.0, p_next,
                                L.spmv_ws, L.spmv_ws_bytes, stream)))
            return rc;
        ppr_restart_kernel<<<1, 1, 0, stream>>>(p_next, seed, restart);
        if ((rc = b2sr::check_launch("ppr_restart_kernel"))) return rc;
        std::swap(p, p_next);
    }
    if (p != ppr) {
        copy_u32_kernel<<<vgrid(n), kThreads, 0, stream>>>(n, (const uint32_t *)p, (uint32_t *)ppr);
        if ((rc = b2sr::check_launch("copy_u32_kernel"))) return rc;
    }
    return sweep(A, ppr, L, nullptr, cluster_bits, stats, stream);
}

}  // extern "C"
