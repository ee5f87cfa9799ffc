// Masked B2SR matrix-matrix product, reduced to one sum (Sec. IV, Table IV:
// bmm_bin_bin_sum and bmm_bin_bin_sum_masked; Sec. V: triangle counting).
//
//   s = sum_{(i,j) : M_ij = 1} sum_k A_ik * B_kj,  B supplied as Bt (rows of Bt
//   are columns of B), so (A B)_ij is the dot product of bit-row i of A with
//   bit-row j of Bt.
//
// The paper's kernel walks A's tile-row, multiplies whole tile pairs with
// shuffles and popcounts, and masks afterwards.  Here the mask drives the work
// (a masked dot product): only output positions with M_ij = 1 are computed.
//   * A workgroup owns one tile-row I.  It marks the tile columns of A's
//     tile-row I in an LDS bitmap with a popcount prefix per word, which turns
//     "is there a tile A_IK, and where" into two LDS reads.
//   * Its waves take the mask tiles (I, J) of M's tile-row I in turn.  A wave
//     lists the set bits (r, c) of the mask tile in LDS, then streams Bt's
//     tile-row J one tile column K per lane and looks K up in A's tile-row.
//   * T <= 8: a tile is one word, so each lane with a match loads both tiles
//     whole and adds popcount(A_IK[r] & Bt_JK[c]) over the listed (r, c).
//   * T >= 16: the matches of a round are listed in LDS with a ballot, and the
//     wave spreads (match, listed bit) items over its lanes: each item loads
//     its two bit-rows, independent of every other, so the wave keeps many
//     loads in flight instead of a few lanes walking the list serially.
//   * Lanes accumulate in 64-bit registers; one atomic add per wave at the end.
// For triangle counting (A = Bt = M = L, the strict lower triangle) row I of L
// is read once per workgroup and Bt's rows are re-read from L2/MALL.
#include <type_traits>

#include <algorithm>

#include "common.h"
#include "scan.h"

using namespace b2sr_dev;

namespace b2sr {
int fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t stream);
}

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / B2SR_WAVE;
constexpr uint32_t kMapWords = 4096;  // bitmap of up to 131072 tile columns
constexpr unsigned kMaxGroups = 8192;  // workgroups of a masked-product launch
#ifndef B2SR_TC_FLAT_SWAP
#define B2SR_TC_FLAT_SWAP 1  // orientation lists built one thread per mask tile
#endif

template <int T> __device__ __forceinline__ row_t<T> load_word(const void *bits, size_t idx)
{
    if constexpr (T == 64) return ((const uint64_t *)bits)[idx];
    else if constexpr (T == 32) return ((const uint32_t *)bits)[idx];
    else if constexpr (T == 16) return ((const uint16_t *)bits)[idx];
    else return ((const uint8_t *)bits)[idx];
}

__device__ __forceinline__ uint32_t popc_word(uint32_t v) { return (uint32_t)__popc(v); }
__device__ __forceinline__ uint32_t popc_word(uint64_t v) { return (uint32_t)__popcll(v); }
__device__ __forceinline__ uint32_t ctz_word(uint32_t v) { return (uint32_t)__builtin_ctz(v); }
__device__ __forceinline__ uint32_t ctz_word(uint64_t v) { return (uint32_t)__builtin_ctzll(v); }

#ifndef B2SR_TC_UB
#define B2SR_TC_UB 4
#endif
constexpr int kUB = B2SR_TC_UB;  // streamed tile columns per lane per round
#ifndef B2SR_TC_IU
#define B2SR_TC_IU 4
#endif
constexpr int kIU = B2SR_TC_IU;  // (tile pair, mask bit) items per lane in flight, T >= 16
constexpr uint32_t kHitCap = 64 * kUB;  // matched tile pairs of one round (T >= 16)
#ifndef B2SR_TC_SWAP_CHUNK
#define B2SR_TC_SWAP_CHUNK 128
#endif
constexpr uint32_t kSwapChunk = B2SR_TC_SWAP_CHUNK;  // swapped mask tiles per work item
#ifndef B2SR_TC_OWN_CHUNK
#define B2SR_TC_OWN_CHUNK 64
#endif
constexpr uint32_t kOwnChunk = B2SR_TC_OWN_CHUNK;  // a row's own mask tiles per work item

struct GemmArgs {
    const uint32_t *a_rp, *a_ci;
    const void *a_bits;
    const uint32_t *b_rp, *b_ci;
    const void *b_bits;
    const uint32_t *m_rp, *m_ci;
    const void *m_bits;
    uint32_t ntr;
    uint32_t map_words;  // LDS bitmap words: enough for every tile column, at most kMapWords
    unsigned long long *sum;
    uint32_t row0, row1;  // the mask tile-rows taken: [row0, row1)
    // Orientation (A and Bt the same matrix): the mask tiles (I, J) with
    // 0 < |A_I| < |Bt_J| tiles are listed under J as (I, mask tile) pairs,
    // sw_list[2 e], sw_list[2 e + 1] for e in [sw_off[J], sw_off[J + 1]); the
    // workgroup of tile-row J then scans A's shorter row I against its bitmap.
    // Null: every mask tile scans Bt's row J.
    const uint32_t *sw_off, *sw_list;
    // Work items when sw_off is set: (row | 2^31 for a swapped chunk, e0, e1)
    // triples; item_off[ntr] of them.  A row's own mask tiles are cut into
    // ranges of kOwnChunk tiles [e0, e1) of M's tile list, its list of swapped
    // tiles into chunks of kSwapChunk entries, so that the work of a long row
    // is spread over many workgroups.
    const uint32_t *item_off, *items;
    uint32_t items_bound;  // an upper bound of item_off[ntr] (the launch's grid)
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Whether mask tile (I, J) is taken from J's side: A and Bt alias, and A's row
// I is the shorter non-empty one.
__device__ __forceinline__ bool swapped(uint32_t len_ai, uint32_t len_btj)
{
    return len_ai > 0 && len_ai < len_btj;
}

// T <= 8: sum over the listed mask bits (r, c) of popcount(A_tile[r] &
// Bt_tile[c]) for the tiles at positions ia (A) and kb (Bt), each loaded whole
// (T bytes) once.
template <int T>
__device__ __forceinline__ uint32_t pair_sum_small(const GemmArgs &g, size_t ia, uint32_t kb, const uint16_t *pairs,
                                                   uint32_t npairs)
{
    static_assert(T <= 8, "whole-tile words");
    using W = typename std::conditional<T == 8, uint64_t, uint32_t>::type;
    const W a = ((const W *)g.a_bits)[ia], b = ((const W *)g.b_bits)[kb];
    uint32_t part = 0;
    for (uint32_t q = 0; q < npairs; ++q) {
        const uint32_t rc = pairs[q];
        part += __popc((uint32_t)((a >> (8 * (rc >> 8))) & (b >> (8 * (rc & 0xFFu)))) & 0xFFu);
    }
    return part;
}

// T >= 16: the products of nh matched tile pairs (hits[h] = A tile position,
// Bt tile position) over the npairs listed mask bits, as nh * npairs items
// spread over the wave's lanes: item x is tile pair x / npairs and mask bit
// x % npairs, and costs two independent row loads.  Each lane keeps kIU items'
// loads in flight.  inv = 1 / npairs (the quotient is corrected to exact).
template <int T>
__device__ __forceinline__ uint32_t items_sum(const GemmArgs &g, const uint2 *hits, uint32_t nh, const uint16_t *pairs,
                                              uint32_t npairs, float inv)
{
    const uint32_t lane = lane_id();
    const uint32_t nitems = nh * npairs;  // <= kHitCap * T * T < 2^24, exact in float
    uint32_t part = 0;
    for (uint32_t x0 = 0; x0 < nitems; x0 += 64 * kIU) {
        row_t<T> a[kIU], b[kIU];
#pragma unroll
        for (int u = 0; u < kIU; ++u) {
            const uint32_t x = x0 + 64 * u + lane;
            const bool ok = x < nitems;
            const uint32_t xc = ok ? x : 0u;
            int h = (int)((float)xc * inv);
            int q = (int)xc - h * (int)npairs;
            if (q < 0) { --h; q += (int)npairs; }
            else if (q >= (int)npairs) { ++h; q -= (int)npairs; }
            const uint2 hp = hits[h];
            const uint32_t rc = pairs[q];
            a[u] = ok ? load_word<T>(g.a_bits, (size_t)hp.x * T + (rc >> 8)) : (row_t<T>)0;
            b[u] = ok ? load_word<T>(g.b_bits, (size_t)hp.y * T + (rc & 0xFFu)) : (row_t<T>)0;
        }
#pragma unroll
        for (int u = 0; u < kIU; ++u) part += popc_word(a[u] & b[u]);
    }
    return part;
}

// PROFILE: instead of the sum, count the work into g.sum[0..3]: mask tiles
// visited, Bt tile columns looked up, matched tile pairs, and bit-row pair
// operations (matched pairs times the mask tile's set bits).
template <int T, bool PROFILE = false> __global__ void __launch_bounds__(kThreads) spgemm_masked_kernel(GemmArgs g)
{
    using R = row_t<T>;
    constexpr bool kItems = T >= 16;
    // the bitmap and its prefix are sized at launch to the matrix's tile columns,
    // so that small matrices leave room for more workgroups per CU
    extern __shared__ uint32_t s_dyn[];
    uint32_t *const s_map = s_dyn, *const s_pre = s_dyn + g.map_words;
    __shared__ uint32_t s_thr[kWaves];
    __shared__ uint16_t s_pairs[kWaves][T * T];
    __shared__ uint2 s_hits[kItems ? kWaves : 1][kItems ? kHitCap : 1];
    const uint32_t lane = lane_id(), wv = threadIdx.x / B2SR_WAVE;
    unsigned long long acc = 0;
    [[maybe_unused]] unsigned long long n_tiles = 0, n_lookups = 0, n_matches = 0;

    const uint32_t nwork = g.sw_off ? g.item_off[g.ntr] : g.row1 - g.row0;
    for (uint32_t wk = blockIdx.x; wk < nwork; wk += gridDim.x) {
        uint32_t I = g.row0 + wk, s0 = 0, s1 = 0, m0 = 0, m1 = 0;
        if (g.sw_off) {
            // a range of this row's own mask tiles, or a chunk of its swapped list
            const uint32_t x = g.items[3 * (size_t)wk];
            I = x & 0x7FFFFFFFu;
            uint32_t e0 = g.items[3 * (size_t)wk + 1], e1 = g.items[3 * (size_t)wk + 2];
            if (x >> 31) { s0 = e0; s1 = e1; }
            else { m0 = e0; m1 = e1; }
        } else {
            m0 = g.m_rp[I];
            m1 = g.m_rp[I + 1];
        }
        const uint32_t a0 = g.a_rp[I], a1 = g.a_rp[I + 1];
        if ((m0 == m1 && s0 == s1) || a0 == a1) continue;  // workgroup-uniform
        const uint32_t jlo = g.a_ci[a0], jhi = g.a_ci[a1 - 1];
        const uint32_t span = jhi - jlo + 1;
        const bool use_map = span <= g.map_words * 32;
        __syncthreads();
        if (use_map) {
            const uint32_t nw = (span + 31) / 32;
            for (uint32_t w = threadIdx.x; w < nw; w += kThreads) s_map[w] = 0;
            __syncthreads();
            for (uint32_t e = a0 + threadIdx.x; e < a1; e += kThreads) {
                const uint32_t off = g.a_ci[e] - jlo;
                atomicOr(&s_map[off >> 5], 1u << (off & 31));
            }
            __syncthreads();
            const uint32_t per = (nw + kThreads - 1) / kThreads;
            const uint32_t w0 = threadIdx.x * per, w1 = min(nw, w0 + per);
            uint32_t local = 0;
            for (uint32_t w = w0; w < w1; ++w) local += __popc(s_map[w]);
            // exclusive prefix of the threads' counts: a scan within each wave,
            // then the totals of the waves before
            uint32_t inc = local;
            for (uint32_t d = 1; d < 64; d <<= 1) {
                const uint32_t o = shfl_up(inc, d);
                if (lane >= d) inc += o;
            }
            if (lane == 63) s_thr[wv] = inc;
            __syncthreads();
            uint32_t run = inc - local;
            for (uint32_t k = 0; k < wv; ++k) run += s_thr[k];
            for (uint32_t w = w0; w < w1; ++w) {
                s_pre[w] = run;
                run += __popc(s_map[w]);
            }
            __syncthreads();
        }
        // Position of tile column K in A's tile-row I, or -1.
        auto lookup = [&](uint32_t K) -> int64_t {
            if (K < jlo || K > jhi) return -1;
            if (use_map) {
                const uint32_t off = K - jlo, w = off >> 5, b = off & 31;
                const uint32_t m = s_map[w];
                if (!((m >> b) & 1u)) return -1;
                return (int64_t)a0 + s_pre[w] + __popc(m & ((1u << b) - 1u));
            }
            uint32_t lo = a0, hi = a1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (g.a_ci[mid] < K) lo = mid + 1; else hi = mid;
            }
            return (lo < a1 && g.a_ci[lo] == K) ? (int64_t)lo : -1;
        };

        // One mask tile m: its set bits (r, c) are listed, then the tile columns
        // ci[p0 .. p1) of the streamed row are looked up in this row's bitmap.
        // Normal orientation: the stream is Bt's row J and the bitmap gives A_IK;
        // swapped: the stream is A's row (the mask tile's row) and the bitmap,
        // this row of Bt = A, gives Bt_JK.
        auto do_tile = [&](uint32_t m, uint32_t p0, uint32_t p1, const uint32_t *ci, bool swap) {
            // list the set bits (r, c) of mask tile m
            const R mw = lane < (uint32_t)T ? load_word<T>(g.m_bits, (size_t)m * T + lane) : (R)0;
            const uint32_t cnt = popc_word(mw);
            uint32_t inc = cnt;
            for (uint32_t d = 1; d < 64; d <<= 1) {
                const uint32_t o = shfl_up(inc, d);
                if (lane >= d) inc += o;
            }
            const uint32_t npairs = readlane(inc, 63);
            uint32_t pos = inc - cnt;
            R w = mw;
            while (w) {
                const uint32_t c = ctz_word(w);
                w &= w - 1;
                s_pairs[wv][pos++] = (uint16_t)((lane << 8) | c);
            }
            wave_sync();
            const float inv = 1.0f / (float)npairs;
            // the streamed row, kUB tile columns per lane per round: the column
            // loads and lookups of a round are independent, so they overlap
            unsigned long long part = 0;
            for (uint32_t base = p0; base < p1; base += 64 * kUB) {
                uint32_t ps[kUB], K[kUB];
#pragma unroll
                for (int u = 0; u < kUB; ++u) {
                    ps[u] = base + 64 * u + lane;
                    K[u] = ci[min(ps[u], p1 - 1)];
                }
                int64_t hit[kUB];
#pragma unroll
                for (int u = 0; u < kUB; ++u) hit[u] = ps[u] < p1 ? lookup(K[u]) : -1;
                uint32_t nh = 0;  // T >= 16: the round's matched tile pairs, listed in s_hits
#pragma unroll
                for (int u = 0; u < kUB; ++u) {
                    const size_t ia = swap ? (size_t)ps[u] : (size_t)hit[u];
                    const uint32_t kb = swap ? (uint32_t)hit[u] : ps[u];
                    if constexpr (PROFILE) {
                        n_lookups += ps[u] < p1;
                        if (hit[u] >= 0) {
                            ++n_matches;
                            part += npairs;
                        }
                    } else if constexpr (kItems) {
                        const uint64_t bal = __ballot(hit[u] >= 0);
                        if (hit[u] >= 0)
                            s_hits[wv][nh + __popcll(bal & ((1ull << lane) - 1ull))] = uint2{(uint32_t)ia, kb};
                        nh += (uint32_t)__popcll(bal);
                    } else if (hit[u] >= 0) {
                        part += pair_sum_small<T>(g, ia, kb, s_pairs[wv], npairs);
                    }
                }
                if constexpr (kItems && !PROFILE) {
                    if (nh) {
                        wave_sync();
                        part += items_sum<T>(g, s_hits[wv], nh, s_pairs[wv], npairs, inv);
                        wave_sync();  // the next round rewrites s_hits
                    }
                }
            }
            acc += part;
            if constexpr (PROFILE) n_tiles += lane == 0;
            wave_sync();  // s_pairs and s_hits are rewritten by the next tile
        };

        for (uint32_t m = m0 + wv; m < m1; m += kWaves) {
            const uint32_t J = g.m_ci[m];
            const uint32_t b0 = g.b_rp[J], b1 = g.b_rp[J + 1];
            if (g.sw_off && swapped(a1 - a0, b1 - b0)) continue;  // taken from J's side
            do_tile(m, b0, b1, g.b_ci, false);
        }
        for (uint32_t e = s0 + wv; e < s1; e += kWaves) {
            const uint32_t Ir = g.sw_list[2 * (size_t)e], m = g.sw_list[2 * (size_t)e + 1];
            do_tile(m, g.a_rp[Ir], g.a_rp[Ir + 1], g.a_ci, true);
        }
    }
    for (int d = 32; d >= 1; d >>= 1) acc += shfl_xor((uint64_t)acc, d);
    if constexpr (PROFILE) {
        for (int d = 32; d >= 1; d >>= 1) {
            n_tiles += shfl_xor((uint64_t)n_tiles, d);
            n_lookups += shfl_xor((uint64_t)n_lookups, d);
            n_matches += shfl_xor((uint64_t)n_matches, d);
        }
        if (lane == 0) {
            if (n_tiles) atomicAdd(g.sum, n_tiles);
            if (n_lookups) atomicAdd(g.sum + 1, n_lookups);
            if (n_matches) atomicAdd(g.sum + 2, n_matches);
            if (acc) atomicAdd(g.sum + 3, acc);
        }
    } else if (lane == 0 && acc) {
        atomicAdd(g.sum, acc);
    }
}

// Unmasked sum: sum_{i,j} (A B)_ij = sum_k colsum_A(k) * colsum_Bt(k).
// One thread per (tile, column) counts that column's bits.
template <int T>
__global__ void column_counts_kernel(const uint32_t *__restrict__ ci, const void *__restrict__ bits, uint32_t ntiles,
                                     uint32_t *__restrict__ colsum)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t)ntiles * T;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t t = (uint32_t)(i / T), c = (uint32_t)(i % T);
        uint32_t cnt = 0;
#pragma unroll
        for (int r = 0; r < T; ++r) cnt += (load_word<T>(bits, (size_t)t * T + r) >> c) & 1u;
        if (cnt) atomicAdd(&colsum[(size_t)ci[t] * T + c], cnt);
    }
}

__global__ void __launch_bounds__(256) dot_counts_kernel(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                                                         uint64_t len, unsigned long long *sum)
{
    unsigned long long acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (uint64_t)gridDim.x * blockDim.x)
        acc += (unsigned long long)a[i] * b[i];
    for (int d = 32; d >= 1; d >>= 1) acc += shfl_xor((uint64_t)acc, d);
    if (lane_id() == 0 && acc) atomicAdd(sum, acc);
}

__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0; }

template <int T, bool PROFILE = false> int launch_masked(GemmArgs g, hipStream_t s)
{
    g.map_words = std::max<uint32_t>(1, std::min<uint32_t>(kMapWords, (g.ntr + 31) / 32));
    // At T = 32 every match reads tile rows from global memory, and more resident
    // workgroups measured slower: its blocks keep the full-size bitmap's LDS,
    // which holds them to 3 per CU.
    const uint32_t lds_words = T == 32 ? kMapWords : g.map_words;
    if (!g.sw_off && g.row1 <= g.row0) return B2SR_OK;
    const uint32_t work = g.sw_off ? g.items_bound : g.row1 - g.row0;
    // At most kMaxGroups workgroups, each looping over work items: one workgroup
    // per item (up to 65,536) measured slower wherever items are short, their
    // launches then dominating (king grid T = 32: 3.23 -> 1.07 ms; R-MAT s18 T = 8:
    // 2.98 -> 2.47 ms).
    spgemm_masked_kernel<T, PROFILE><<<b2sr::grid_for(work, 1, kMaxGroups), kThreads, 2 * lds_words * 4, s>>>(g);
    return b2sr::check_launch("spgemm_masked_kernel");
}

__global__ void zero_u64x4_kernel(unsigned long long *p)
{
    if (threadIdx.x < 4) p[threadIdx.x] = 0;
}

template <int T>
int launch_unmasked(const b2sr_matrix *A, const b2sr_matrix *Bt, uint32_t *ws, uint64_t len,
                    unsigned long long *sum, hipStream_t s)
{
    column_counts_kernel<T><<<b2sr::grid_for((uint64_t)A->ntiles * T, 256, 65536), 256, 0, s>>>(
        A->tile_colind, A->bits, A->ntiles, ws);
    if (int rc = b2sr::check_launch("column_counts_kernel")) return rc;
    column_counts_kernel<T><<<b2sr::grid_for((uint64_t)Bt->ntiles * T, 256, 65536), 256, 0, s>>>(
        Bt->tile_colind, Bt->bits, Bt->ntiles, ws + len);
    if (int rc = b2sr::check_launch("column_counts_kernel")) return rc;
    dot_counts_kernel<<<b2sr::grid_for(len, 256, 4096), 256, 0, s>>>(ws, ws + len, len, sum);
    return b2sr::check_launch("dot_counts_kernel");
}

// ---- orientation lists (A and Bt the same matrix) ------------------------------
// One wave per mask tile-row I, its lanes over the row's tiles.
__global__ void swap_count_kernel(GemmArgs g, uint32_t *counts)
{
    const uint32_t lane = lane_id();
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t I = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / B2SR_WAVE; I < g.ntr; I += nwaves) {
        const uint32_t lai = g.a_rp[I + 1] - g.a_rp[I];
        for (uint32_t m = g.m_rp[I] + lane; m < g.m_rp[I + 1]; m += B2SR_WAVE) {
            const uint32_t J = g.m_ci[m];
            if (swapped(lai, g.b_rp[J + 1] - g.b_rp[J])) atomicAdd(&counts[J], 1u);
        }
    }
}

// The tile-row of every mask tile: rowof[m] = I for m in [m_rp[I], m_rp[I + 1]),
// one wave per tile-row writing its range with contiguous stores.
__global__ void tile_rows_kernel(GemmArgs g, uint32_t *rowof)
{
    const uint32_t lane = lane_id();
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t I = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / B2SR_WAVE; I < g.ntr; I += nwaves)
        for (uint32_t m = g.m_rp[I] + lane; m < g.m_rp[I + 1]; m += B2SR_WAVE) rowof[m] = (uint32_t)I;
}

// The same counts and lists as swap_count_kernel and swap_fill_kernel, one
// thread per mask tile: its loads are independent of every other thread's, where
// a wave per tile-row leaves most lanes idle on short rows.
template <bool FILL>
__global__ void swap_flat_kernel(GemmArgs g, const uint32_t *rowof, uint32_t ntiles_m, uint32_t *counts,
                                 uint32_t *list)
{
    for (uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; m < ntiles_m;
         m += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t I = rowof[m], J = g.m_ci[m];
        if (!swapped(g.a_rp[I + 1] - g.a_rp[I], g.b_rp[J + 1] - g.b_rp[J])) continue;
        const uint32_t e = atomicAdd(&counts[J], 1u);
        if constexpr (FILL) {
            list[2 * (size_t)e] = I;
            list[2 * (size_t)e + 1] = (uint32_t)m;
        }
    }
}

__global__ void swap_fill_kernel(GemmArgs g, uint32_t *cursor, uint32_t *list)
{
    const uint32_t lane = lane_id();
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t I = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / B2SR_WAVE; I < g.ntr; I += nwaves) {
        const uint32_t lai = g.a_rp[I + 1] - g.a_rp[I];
        for (uint32_t m = g.m_rp[I] + lane; m < g.m_rp[I + 1]; m += B2SR_WAVE) {
            const uint32_t J = g.m_ci[m];
            if (!swapped(lai, g.b_rp[J + 1] - g.b_rp[J])) continue;
            const uint32_t e = atomicAdd(&cursor[J], 1u);
            list[2 * (size_t)e] = (uint32_t)I;
            list[2 * (size_t)e + 1] = m;
        }
    }
}

// Work items per row: one per kOwnChunk of its own mask tiles (when A's row is
// not empty), one per kSwapChunk entries of its swapped list.
__global__ void item_count_kernel(GemmArgs g, const uint32_t *off, uint32_t *counts)
{
    for (uint32_t X = blockIdx.x * blockDim.x + threadIdx.x; X < g.ntr; X += gridDim.x * blockDim.x) {
        const uint32_t own = g.a_rp[X + 1] > g.a_rp[X] ? g.m_rp[X + 1] - g.m_rp[X] : 0u;
        counts[X] = (own + kOwnChunk - 1) / kOwnChunk + (off[X + 1] - off[X] + kSwapChunk - 1) / kSwapChunk;
    }
}

__global__ void item_fill_kernel(GemmArgs g, const uint32_t *off, const uint32_t *item_off, uint32_t *items)
{
    for (uint32_t X = blockIdx.x * blockDim.x + threadIdx.x; X < g.ntr; X += gridDim.x * blockDim.x) {
        size_t w = item_off[X];
        if (g.a_rp[X + 1] > g.a_rp[X]) {
            for (uint32_t e = g.m_rp[X]; e < g.m_rp[X + 1]; e += kOwnChunk, ++w) {
                items[3 * w] = X;
                items[3 * w + 1] = e;
                items[3 * w + 2] = min(g.m_rp[X + 1], e + kOwnChunk);
            }
        }
        for (uint32_t e = off[X]; e < off[X + 1]; e += kSwapChunk, ++w) {
            items[3 * w] = X | 0x80000000u;
            items[3 * w + 1] = e;
            items[3 * w + 2] = min(off[X + 1], e + kSwapChunk);
        }
    }
}

__global__ void copy_u32_kernel(uint32_t n, const uint32_t *__restrict__ a, uint32_t *__restrict__ b)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = a[i];
}

struct SwapLayout {
    uint32_t *off, *cursor, *list, *item_off, *items, *sums, *rowof;
    size_t bytes;
};

SwapLayout swap_layout(const b2sr_matrix *A, const b2sr_matrix *M, void *ws)
{
    const size_t ntr = b2sr::n_tile_rows(A->n, A->tile);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        o = (o + 255) & ~(size_t)255;
        char *p = ws ? (char *)ws + o : nullptr;
        o += bytes;
        return (uint32_t *)p;
    };
    SwapLayout L;
    L.off = take((ntr + 1) * 4);
    L.cursor = take(ntr * 4);
    L.list = take((size_t)M->ntiles * 8);
    L.item_off = take((ntr + 1) * 4);
    // per row, one item per started chunk of its own tiles and of its swapped list
    L.items = take((2 * ntr + (size_t)M->ntiles / kOwnChunk + (size_t)M->ntiles / kSwapChunk + 1) * 12);
    L.sums = take(b2sr_scan::scan_blocks(ntr) * 4);
    L.rowof = B2SR_TC_FLAT_SWAP ? take((size_t)M->ntiles * 4) : nullptr;
    L.bytes = o;
    return L;
}

size_t swap_bytes(const b2sr_matrix *A, const b2sr_matrix *M) { return swap_layout(A, M, nullptr).bytes; }

// Lists, under each tile-row J, the mask tiles (I, J) whose row I of A is the
// shorter: counts, their prefix (the list offsets), then a scatter through a
// copy of the offsets.  The order inside a list follows the atomics, which
// does not change the integer sum.
int build_swap_lists(GemmArgs &g, const b2sr_matrix *A, const b2sr_matrix *M, void *ws, hipStream_t s)
{
    using b2sr_scan::device_scan;
    using b2sr_scan::LoadArray;
    const SwapLayout L = swap_layout(A, M, ws);
    const uint32_t ntr = g.ntr;
    int rc;
    // list offsets: off[0] = 0, off[J + 1] = swapped tiles of rows 0 .. J
    if ((rc = b2sr::fill_u32(L.off, (uint64_t)ntr + 1, 0, s))) return rc;
    const unsigned wgrid = b2sr::grid_for(ntr, 256 / B2SR_WAVE, kMaxGroups);  // grid-stride over tile-rows
    const unsigned tgrid = b2sr::grid_for(M->ntiles, 256, kMaxGroups);       // grid-stride over mask tiles
    if constexpr (B2SR_TC_FLAT_SWAP) {
        tile_rows_kernel<<<wgrid, 256, 0, s>>>(g, L.rowof);
        if ((rc = b2sr::check_launch("tile_rows_kernel"))) return rc;
        swap_flat_kernel<false><<<tgrid, 256, 0, s>>>(g, L.rowof, M->ntiles, L.off + 1, nullptr);
        if ((rc = b2sr::check_launch("swap_flat_kernel"))) return rc;
    } else {
        swap_count_kernel<<<wgrid, 256, 0, s>>>(g, L.off + 1);
        if ((rc = b2sr::check_launch("swap_count_kernel"))) return rc;
    }
    if ((rc = device_scan<uint32_t>(ntr, LoadArray<uint32_t>{L.off + 1}, L.off + 1, true, L.sums, s))) return rc;
    copy_u32_kernel<<<b2sr::grid_for(ntr, 256, 4096), 256, 0, s>>>(ntr, L.off, L.cursor);
    if ((rc = b2sr::check_launch("copy_u32_kernel"))) return rc;
    if constexpr (B2SR_TC_FLAT_SWAP) {
        swap_flat_kernel<true><<<tgrid, 256, 0, s>>>(g, L.rowof, M->ntiles, L.cursor, L.list);
        if ((rc = b2sr::check_launch("swap_flat_kernel"))) return rc;
    } else {
        swap_fill_kernel<<<wgrid, 256, 0, s>>>(g, L.cursor, L.list);
        if ((rc = b2sr::check_launch("swap_fill_kernel"))) return rc;
    }
    // work items: item_off[0] = 0, item_off[X + 1] = items of rows 0 .. X
    if ((rc = b2sr::fill_u32(L.item_off, 1, 0, s))) return rc;
    item_count_kernel<<<b2sr::grid_for(ntr, 256, 4096), 256, 0, s>>>(g, L.off, L.item_off + 1);
    if ((rc = b2sr::check_launch("item_count_kernel"))) return rc;
    if ((rc = device_scan<uint32_t>(ntr, LoadArray<uint32_t>{L.item_off + 1}, L.item_off + 1, true, L.sums, s)))
        return rc;
    item_fill_kernel<<<b2sr::grid_for(ntr, 256, 4096), 256, 0, s>>>(g, L.off, L.item_off, L.items);
    if ((rc = b2sr::check_launch("item_fill_kernel"))) return rc;
    g.sw_off = L.off;
    g.sw_list = L.list;
    g.item_off = L.item_off;
    g.items = L.items;
    g.items_bound = (uint32_t)std::min<uint64_t>(
        0xFFFFFFFFu, 2ull * ntr + M->ntiles / kOwnChunk + M->ntiles / kSwapChunk + 1);
    return B2SR_OK;
}

}  // namespace

namespace b2sr {
// colsum[c] = number of set bits in column c, for c < nTR * T (the columns of
// A's last tile column past n count nothing).
int column_counts(const b2sr_matrix *A, uint32_t *colsum, hipStream_t s)
{
    const uint64_t len = (uint64_t)n_tile_rows(A->n, A->tile) * A->tile;
    if (int rc = fill_u32(colsum, len, 0, s)) return rc;
    if (!A->ntiles) return B2SR_OK;
    const unsigned grid = grid_for((uint64_t)A->ntiles * A->tile, 256, 65536);
    switch (A->tile) {
    case 4: column_counts_kernel<4><<<grid, 256, 0, s>>>(A->tile_colind, A->bits, A->ntiles, colsum); break;
    case 8: column_counts_kernel<8><<<grid, 256, 0, s>>>(A->tile_colind, A->bits, A->ntiles, colsum); break;
    case 16: column_counts_kernel<16><<<grid, 256, 0, s>>>(A->tile_colind, A->bits, A->ntiles, colsum); break;
    case 64: column_counts_kernel<64><<<grid, 256, 0, s>>>(A->tile_colind, A->bits, A->ntiles, colsum); break;
    default: column_counts_kernel<32><<<grid, 256, 0, s>>>(A->tile_colind, A->bits, A->ntiles, colsum); break;
    }
    return check_launch("column_counts_kernel");
}
}  // namespace b2sr

extern "C" {

size_t spgemm_masked_workspace_bytes(const b2sr_matrix *A, const b2sr_matrix *M)
{
    if (!A || !b2sr::valid_tile(A->tile)) return 0;
    if (M) return swap_bytes(A, M);
    return (size_t)2 * b2sr::n_tile_rows(A->n, A->tile) * A->tile * sizeof(uint32_t);
}

int spgemm_masked_profile(const b2sr_matrix *A, const b2sr_matrix *Bt, const b2sr_matrix *M, uint64_t *d_counts,
                          hipStream_t stream)
{
    int rc = b2sr::validate_matrix(A);
    if (rc) return rc;
    if ((rc = b2sr::validate_matrix(Bt))) return rc;
    if (!M || (rc = b2sr::validate_matrix(M))) return rc ? rc : B2SR_EINVAL;
    if (!d_counts) return B2SR_EINVAL;
    if (Bt->n != A->n || Bt->tile != A->tile || M->n != A->n || M->tile != A->tile) return B2SR_EINVAL;
    unsigned long long *c = (unsigned long long *)d_counts;
    zero_u64x4_kernel<<<1, 64, 0, stream>>>(c);
    if ((rc = b2sr::check_launch("zero_u64x4_kernel"))) return rc;
    if (A->n == 0 || A->ntiles == 0 || Bt->ntiles == 0 || M->ntiles == 0) return B2SR_OK;
    GemmArgs g{A->tile_rowptr, A->tile_colind, A->bits, Bt->tile_rowptr, Bt->tile_colind, Bt->bits,
               M->tile_rowptr, M->tile_colind, M->bits, b2sr::n_tile_rows(A->n, A->tile), 0, c,
               0, b2sr::n_tile_rows(A->n, A->tile), nullptr, nullptr, nullptr, nullptr, 0};
    switch (A->tile) {
    case 4: return launch_masked<4, true>(g, stream);
    case 8: return launch_masked<8, true>(g, stream);
    case 16: return launch_masked<16, true>(g, stream);
    case 64: return launch_masked<64, true>(g, stream);
    default: return launch_masked<32, true>(g, stream);
    }
}

int spgemm_masked(const b2sr_matrix *A, const b2sr_matrix *Bt, const b2sr_matrix *M, unsigned flags,
                  uint64_t *d_sum, void *ws, size_t ws_bytes, hipStream_t stream)
{
    int rc = b2sr::validate_matrix(A);
    if (rc) return rc;
    if ((rc = b2sr::validate_matrix(Bt))) return rc;
    if (M && (rc = b2sr::validate_matrix(M))) return rc;
    if (flags & ~B2SR_ACCUMULATE) return B2SR_EINVAL;
    if (!d_sum) return B2SR_EINVAL;
    if (Bt->n != A->n || Bt->tile != A->tile) return B2SR_EINVAL;
    if (M && (M->n != A->n || M->tile != A->tile)) return B2SR_EINVAL;
    // the unmasked sum needs its workspace; the masked one uses it when given
    const size_t need = M ? 0 : spgemm_masked_workspace_bytes(A, M);
    if (ws_bytes < need || (need && !ws)) return B2SR_ENOSPC;
    unsigned long long *sum = (unsigned long long *)d_sum;
    if (!(flags & B2SR_ACCUMULATE)) {
        zero_u64_kernel<<<1, 1, 0, stream>>>(sum);
        if ((rc = b2sr::check_launch("zero_u64_kernel"))) return rc;
    }
    if (A->n == 0 || A->ntiles == 0 || Bt->ntiles == 0 || (M && M->ntiles == 0)) return B2SR_OK;
    if (!M) {
        const uint64_t len = (uint64_t)b2sr::n_tile_rows(A->n, A->tile) * A->tile;
        if ((rc = b2sr::fill_u32((uint32_t *)ws, 2 * len, 0, stream))) return rc;
        switch (A->tile) {
        case 4: return launch_unmasked<4>(A, Bt, (uint32_t *)ws, len, sum, stream);
        case 8: return launch_unmasked<8>(A, Bt, (uint32_t *)ws, len, sum, stream);
        case 16: return launch_unmasked<16>(A, Bt, (uint32_t *)ws, len, sum, stream);
        case 64: return launch_unmasked<64>(A, Bt, (uint32_t *)ws, len, sum, stream);
        default: return launch_unmasked<32>(A, Bt, (uint32_t *)ws, len, sum, stream);
        }
    }
    GemmArgs g{A->tile_rowptr, A->tile_colind, A->bits, Bt->tile_rowptr, Bt->tile_colind, Bt->bits,
               M->tile_rowptr, M->tile_colind, M->bits, b2sr::n_tile_rows(A->n, A->tile), 0, sum,
               0, b2sr::n_tile_rows(A->n, A->tile), nullptr, nullptr, nullptr, nullptr, 0};
    // A and Bt the same matrix, and room for the lists: each mask tile scans the
    // shorter of its two tile-rows
    const bool alias = Bt->tile_rowptr == A->tile_rowptr && Bt->tile_colind == A->tile_colind &&
                       Bt->bits == A->bits && Bt->ntiles == A->ntiles;
    if (alias && ws && ws_bytes >= swap_bytes(A, M)) {
        if ((rc = build_swap_lists(g, A, M, ws, stream))) return rc;
    }
    switch (A->tile) {
    case 4: return launch_masked<4>(g, stream);
    case 8: return launch_masked<8>(g, stream);
    case 16: return launch_masked<16>(g, stream);
    case 64: return launch_masked<64>(g, stream);
    default: return launch_masked<32>(g, stream);
    }
}

int spgemm_masked_rows(const b2sr_matrix *A, const b2sr_matrix *Bt, const b2sr_matrix *M, uint32_t row_begin,
                       uint32_t row_end, unsigned flags, uint64_t *d_sum, hipStream_t stream)
{
    int rc = b2sr::validate_matrix(A);
    if (rc) return rc;
    if ((rc = b2sr::validate_matrix(Bt))) return rc;
    if (!M) return B2SR_EINVAL;
    if ((rc = b2sr::validate_matrix(M))) return rc;
    if (flags & ~B2SR_ACCUMULATE) return B2SR_EINVAL;
    if (!d_sum) return B2SR_EINVAL;
    if (Bt->n != A->n || Bt->tile != A->tile || M->n != A->n || M->tile != A->tile) return B2SR_EINVAL;
    const uint32_t ntr = b2sr::n_tile_rows(A->n, A->tile);
    if (row_begin > row_end || row_end > ntr) return B2SR_EINVAL;
    unsigned long long *sum = (unsigned long long *)d_sum;
    if (!(flags & B2SR_ACCUMULATE)) {
        zero_u64_kernel<<<1, 1, 0, stream>>>(sum);
        if ((rc = b2sr::check_launch("zero_u64_kernel"))) return rc;
    }
    if (A->n == 0 || A->ntiles == 0 || Bt->ntiles == 0 || M->ntiles == 0) return B2SR_OK;
    GemmArgs g{A->tile_rowptr, A->tile_colind, A->bits, Bt->tile_rowptr, Bt->tile_colind, Bt->bits,
               M->tile_rowptr, M->tile_colind, M->bits, ntr, 0, sum, row_begin, row_end, nullptr, nullptr, nullptr,
               nullptr, 0};
    switch (A->tile) {
    case 4: return launch_masked<4>(g, stream);
    case 8: return launch_masked<8>(g, stream);
    case 16: return launch_masked<16>(g, stream);
    case 64: return launch_masked<64>(g, stream);
    default: return launch_masked<32>(g, stream);
    }
}

}  // extern "C"
