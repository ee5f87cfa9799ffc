// Matrix-vector products on B2SR (Sec. IV, Table III; semirings of Table V).
//
// Work decomposition (wave64, gfx950).  The paper gives one warp a whole
// tile-row and one lane a bit-row.  On power-law graphs that leaves a few
// waves with thousands of tiles, so here every wave takes a fixed CHUNK of
// consecutive tiles instead, whatever rows they belong to:
//   * a wave step covers TPW consecutive tiles; LPT lanes share a tile and each
//     reads one 16/8/4-byte piece holding RPL bit-rows (TileShape), so the
//     wave's loads are one contiguous run of tile bytes;
//   * the tile-row of the chunk's first tile comes from a 64-way search of
//     TileRowPtr (3 rounds for 2^18 tile-rows);
//   * when a whole step lies inside the current tile-row (the common case on
//     long rows) each lane just folds its partial into a register accumulator;
//   * when a step crosses row ends, each lane finds its tile's row from the
//     next 64 row pointers held one per lane, and a segmented scan over the
//     wave combines partials of equal rows;
//   * a finished row is written once per chunk.  Bit, count and min results
//     use atomics (exact and order-free); float sums write rows owned by one
//     chunk directly and park the partials of rows that straddle chunks in the
//     workspace, where a second kernel adds them in chunk order, so every float
//     result is deterministic.
// Masks are applied when a row is stored (Sec. V, BFS), and tiles whose rows
// are all masked out or whose vector segment is empty are not read.
#include "common.h"

using namespace b2sr_dev;

namespace {

enum Kind : int { kBits = 0, kCount = 1, kPlusF32 = 2, kMinF32 = 3, kMinU32 = 4, kOr64 = 5 };

template <int K> struct KindTraits;
template <> struct KindTraits<kCount> {
    using V = uint32_t;
    static __device__ __forceinline__ V id() { return 0u; }
    static __device__ __forceinline__ V op(V a, V b) { return a + b; }
};
template <> struct KindTraits<kPlusF32> {
    using V = float;
    static __device__ __forceinline__ V id() { return 0.0f; }
    static __device__ __forceinline__ V op(V a, V b) { return a + b; }
};
template <> struct KindTraits<kMinF32> {
    using V = float;
    static __device__ __forceinline__ V id() { return __builtin_huge_valf(); }
    static __device__ __forceinline__ V op(V a, V b) { return b < a ? b : a; }
};
template <> struct KindTraits<kMinU32> {
    using V = uint32_t;
    static __device__ __forceinline__ V id() { return 0xFFFFFFFFu; }
    static __device__ __forceinline__ V op(V a, V b) { return b < a ? b : a; }
};
template <> struct KindTraits<kOr64> {
    using V = uint64_t;
    static __device__ __forceinline__ V id() { return 0ull; }
    static __device__ __forceinline__ V op(V a, V b) { return a | b; }
};

struct SpmvArgs {
    const uint32_t *trp;
    const uint32_t *tci;
    const void *bits;
    uint32_t n, ntr, ntiles, chunk;
    const void *x;
    const float *s;
    const uint32_t *mask;
    unsigned flags;
    float alpha, beta;
    uint32_t w_u32;
    void *y;
    uint32_t *ws_rows;  // float sums: first and last row of each chunk
    float *ws_part;     // float sums: partials of straddling rows, 2*T per chunk
};

// Tiles per wave chunk.
template <int T> constexpr uint32_t chunk_tiles() { return T == 32 ? 256u : (T == 16 ? 512u : 1024u); }
inline uint32_t chunk_tiles_rt(uint32_t T)
{
    return T == 32 ? chunk_tiles<32>() : T == 16 ? chunk_tiles<16>() : T == 8 ? chunk_tiles<8>() : chunk_tiles<4>();
}

// Tile-row holding tile t: the last r with trp[r] <= t (trp[ntr] > t).  A
// 64-way search: every lane probes one pointer per round.
__device__ __forceinline__ uint32_t find_row(const uint32_t *trp, uint32_t ntr, uint32_t t)
{
    uint32_t lo = 0, hi = ntr;  // trp[lo] <= t < trp[hi]
    const uint32_t lane = lane_id();
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t probe = lo + (lane + 1) * step;
        const bool le = lane < 63 && probe < hi && trp[probe] <= t;
        const uint32_t c = (uint32_t)__popcll(__ballot(le));
        const uint32_t nlo = lo + c * step;
        hi = min(hi, nlo + step);
        lo = nlo;
    }
    return lo;
}

// Row of this lane's tile t, given that every tile of the step lies at or after
// row r_cur: the rows r_base+1 .. r_base+64 have their first tiles loaded one
// per lane, and a 6-step search through them counts how many start at or
// before t.  Repeats (rarely) when more than 64 rows end inside the step.
__device__ __forceinline__ uint32_t lane_row(const uint32_t *trp, uint32_t ntr, uint32_t r_cur, uint32_t t)
{
    const uint32_t lane = lane_id();
    uint32_t r_base = r_cur, row = 0;
    bool done = false;
    while (true) {
        const uint32_t idx = r_base + 1 + lane;
        const uint32_t rb = idx <= ntr ? trp[idx] : 0xFFFFFFFFu;
        uint32_t cnt = 0;
#pragma unroll
        for (uint32_t step = 32; step >= 1; step >>= 1) {
            const uint32_t v = shfl(rb, (int)(cnt + step - 1));
            if (v <= t) cnt += step;
        }
        if (readlane(rb, 63) <= t) cnt = 64;
        if (!done && cnt < 64) {
            row = r_base + cnt;
            done = true;
        }
        if (__all(done)) break;
        r_base += 64;
    }
    return row;
}

// Rows of tile-row I that the mask keeps, as T bits.
template <int T> __device__ __forceinline__ uint32_t keep_bits(const uint32_t *mask, unsigned flags, uint32_t I)
{
    constexpr uint32_t full = T == 32 ? 0xFFFFFFFFu : ((1u << T) - 1u);
    if (!mask) return full;
    const uint32_t w = bit_segment<T>(mask, I);
    return (flags & B2SR_MASK_COMPLEMENT) ? (~w & full) : w;
}

// ---------------------------------------------------------------------------
// Boolean product, bit output (bmv_bin_bin_bin[_masked])
// ---------------------------------------------------------------------------

// OR-test of this lane's bit-rows of tile t against x's segment, placed at the
// rows' bit positions inside the tile-row.
template <int T> __device__ __forceinline__ uint32_t bits_partial(const SpmvArgs &p, uint32_t t, uint32_t sub)
{
    using S = TileShape<T>;
    const uint32_t seg = bit_segment<T>((const uint32_t *)p.x, p.tci[t]);
    if (!seg) return 0;  // frontier-empty segment: the tile cannot contribute
    uint32_t a[S::RPL];
    load_rows<T>(p.bits, t, sub, a);
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < S::RPL; ++k) m |= (uint32_t)((a[k] & seg) != 0) << (sub * S::RPL + k);
    return m;
}

template <int T> __device__ __forceinline__ void store_bits(const SpmvArgs &p, uint32_t I, uint32_t m)
{
    if (!m) return;
    const uint32_t bit = I * T;
    atomicOr((uint32_t *)p.y + (bit >> 5), m << (bit & 31u));
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) v |= shfl_xor(v, d);
    return v;
}

template <int T> __global__ void __launch_bounds__(256) spmv_bits_kernel(SpmvArgs p)
{
    using S = TileShape<T>;
    const uint32_t lane = lane_id(), grp = lane / S::LPT, sub = lane % S::LPT;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE;
    if (wave * p.chunk >= p.ntiles) return;
    const uint32_t t_begin = (uint32_t)(wave * p.chunk);
    const uint32_t t_end = min(t_begin + p.chunk, p.ntiles);

    uint32_t r_cur = find_row(p.trp, p.ntr, t_begin);
    uint32_t r_end = p.trp[r_cur + 1];
    uint32_t keep = keep_bits<T>(p.mask, p.flags, r_cur);
    uint32_t acc = 0;
    uint32_t base = t_begin;
    while (base < t_end) {
        const uint32_t last = min(base + S::TPW, t_end) - 1;
        const bool valid = base + grp < t_end;
        const uint32_t t = valid ? base + grp : t_end - 1;
        if (last < r_end) {
            if (!keep) {  // every row of this tile-row is masked out
                base = min(r_end, t_end);
                continue;
            }
            if (valid) acc |= bits_partial<T>(p, t, sub);
            base += S::TPW;
            continue;
        }
        // the step crosses the end of row r_cur
        const uint32_t row = lane_row(p.trp, p.ntr, r_cur, t);
        const uint32_t rkeep = row == r_cur ? keep : keep_bits<T>(p.mask, p.flags, row);
        const uint32_t part = (valid && rkeep) ? bits_partial<T>(p, t, sub) : 0u;
        const uint32_t acc_all = wave_or(acc);
        uint32_t v = part;
        if (readlane(row, 0) != r_cur) {
            if (lane == 0) store_bits<T>(p, r_cur, acc_all & keep);
        } else if (lane == 0) {
            v |= acc_all;
        }
#pragma unroll
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t o = shfl_up(v, d), ro = shfl_up(row, d);
            if (lane >= d && ro == row) v |= o;
        }
        const uint32_t r_last = readlane(row, 63);
        const uint32_t next_row = shfl(row, (int)min(lane + 1, 63u));
        if ((lane == 63 || next_row != row) && row != r_last) store_bits<T>(p, row, v & rkeep);
        acc = row == r_last ? part : 0u;
        r_cur = r_last;
        r_end = p.trp[r_cur + 1];
        keep = keep_bits<T>(p.mask, p.flags, r_cur);
        base += S::TPW;
    }
    const uint32_t acc_all = wave_or(acc);
    if (lane == 0) store_bits<T>(p, r_cur, acc_all & keep);
}

// ---------------------------------------------------------------------------
// Value outputs: counts (bmv_bin_bin_full), and bmv_bin_full_full under
// plus-times, min-plus and 64-wide OR
// ---------------------------------------------------------------------------

template <int T, int K>
__device__ __forceinline__ void value_partial(const SpmvArgs &p, uint32_t t, uint32_t sub,
                                              typename KindTraits<K>::V (&part)[TileShape<T>::RPL])
{
    using S = TileShape<T>;
    using KT = KindTraits<K>;
    const uint32_t J = p.tci[t];
    uint32_t a[S::RPL];
    if constexpr (K == kCount) {
        const uint32_t seg = bit_segment<T>((const uint32_t *)p.x, J);
        if (!seg) return;  // frontier-empty segment
        load_rows<T>(p.bits, t, sub, a);
#pragma unroll
        for (int k = 0; k < S::RPL; ++k) part[k] = (uint32_t)__popc(a[k] & seg);  // Listing 1's dot product
    } else {
        load_rows<T>(p.bits, t, sub, a);
        const size_t col0 = (size_t)J * T;
#pragma unroll
        for (int k = 0; k < S::RPL; ++k) {
            uint32_t w = a[k];
            while (w) {
                const uint32_t c = __builtin_ctz(w);
                w &= w - 1;
                if constexpr (K == kPlusF32) {
                    float xv = ((const float *)p.x)[col0 + c];
                    if (p.s) xv *= p.s[col0 + c];
                    part[k] += xv;
                } else if constexpr (K == kMinF32) {
                    part[k] = KT::op(part[k], ((const float *)p.x)[col0 + c]);
                } else if constexpr (K == kMinU32) {
                    part[k] = KT::op(part[k], ((const uint32_t *)p.x)[col0 + c]);
                } else {
                    part[k] |= ((const uint64_t *)p.x)[col0 + c];
                }
            }
        }
    }
}

// Stores the RPL rows [sub*RPL, sub*RPL + RPL) of tile-row I.
template <int T, int K>
__device__ __forceinline__ void store_values(const SpmvArgs &p, uint32_t I, uint32_t sub, uint32_t keep,
                                             const typename KindTraits<K>::V (&v)[TileShape<T>::RPL],
                                             bool straddles, uint32_t chunk_id, uint32_t slot)
{
    using S = TileShape<T>;
    using KT = KindTraits<K>;
#pragma unroll
    for (int k = 0; k < S::RPL; ++k) {
        const uint32_t r = sub * S::RPL + k;
        const uint32_t row = I * T + r;
        if constexpr (K == kPlusF32) {
            if (straddles) {
                p.ws_part[((size_t)chunk_id * 2 + slot) * T + r] = v[k];
                continue;
            }
        }
        if (row >= p.n || !((keep >> r) & 1u)) continue;
        if constexpr (K == kCount) {
            if (v[k]) atomicAdd((uint32_t *)p.y + row, v[k]);
        } else if constexpr (K == kPlusF32) {
            float *y = (float *)p.y + row;
            if (p.flags & B2SR_ACCUMULATE) *y = *y + p.alpha * v[k];
            else *y = p.alpha * v[k] + p.beta;
        } else if constexpr (K == kMinF32) {
            if (v[k] != KT::id()) atomic_min_f32((float *)p.y + row, v[k] + p.alpha);
        } else if constexpr (K == kMinU32) {
            if (v[k] != KT::id()) atomicMin((uint32_t *)p.y + row, sat_add_u32(v[k], p.w_u32));
        } else {
            if (v[k]) atomicOr((unsigned long long *)p.y + row, (unsigned long long)v[k]);
        }
    }
}

template <int T, int K> __global__ void __launch_bounds__(256) spmv_values_kernel(SpmvArgs p)
{
    using S = TileShape<T>;
    using KT = KindTraits<K>;
    using V = typename KT::V;
    constexpr int RPL = S::RPL, LPT = S::LPT, TPW = S::TPW;
    const uint32_t lane = lane_id(), grp = lane / LPT, sub = lane % LPT;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE;
    if (wave * p.chunk >= p.ntiles) return;
    const uint32_t chunk_id = (uint32_t)wave;
    const uint32_t t_begin = chunk_id * p.chunk;
    const uint32_t t_end = min(t_begin + p.chunk, p.ntiles);

    const uint32_t r_first = find_row(p.trp, p.ntr, t_begin);
    uint32_t r_cur = r_first;
    uint32_t r_end = p.trp[r_cur + 1];
    uint32_t keep = keep_bits<T>(p.mask, p.flags, r_cur);
    // A row straddles chunks when it starts before t_begin or ends after t_end;
    // only the chunk's first and last rows can.
    auto straddles = [&](uint32_t I) { return p.trp[I] < t_begin || p.trp[I + 1] > t_end; };

    V acc[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) acc[k] = KT::id();
    uint32_t base = t_begin;
    while (base < t_end) {
        const uint32_t last = min(base + TPW, t_end) - 1;
        const bool valid = base + grp < t_end;
        const uint32_t t = valid ? base + grp : t_end - 1;
        if (last < r_end) {
            if (!keep && K != kPlusF32) {  // all rows masked out (float sums still park partials)
                base = min(r_end, t_end);
                continue;
            }
            if (valid) {
                V part[RPL];
#pragma unroll
                for (int k = 0; k < RPL; ++k) part[k] = KT::id();
                value_partial<T, K>(p, t, sub, part);
#pragma unroll
                for (int k = 0; k < RPL; ++k) acc[k] = KT::op(acc[k], part[k]);
            }
            base += TPW;
            continue;
        }
        const uint32_t row = lane_row(p.trp, p.ntr, r_cur, t);
        const uint32_t rkeep = row == r_cur ? keep : keep_bits<T>(p.mask, p.flags, row);
        V part[RPL], v[RPL], tot[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) part[k] = KT::id();
        if (valid && (rkeep || K == kPlusF32)) value_partial<T, K>(p, t, sub, part);
        // total of the running accumulator over the groups (rows by sub)
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            tot[k] = acc[k];
#pragma unroll
            for (int d = LPT; d < 64; d <<= 1) tot[k] = KT::op(tot[k], shfl_xor(tot[k], d));
            v[k] = part[k];
        }
        if (readlane(row, 0) != r_cur) {
            if (grp == 0) store_values<T, K>(p, r_cur, sub, keep, tot, straddles(r_cur), chunk_id, r_cur == r_first ? 0 : 1);
        } else if (grp == 0) {
#pragma unroll
            for (int k = 0; k < RPL; ++k) v[k] = KT::op(tot[k], part[k]);
        }
        // segmented inclusive scan over groups, keyed by row
#pragma unroll
        for (int d = 1; d < TPW; d <<= 1) {
            const uint32_t ro = shfl_up(row, d * LPT);
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const V o = shfl_up(v[k], d * LPT);
                if (grp >= (uint32_t)d && ro == row) v[k] = KT::op(v[k], o);
            }
        }
        const uint32_t r_last = readlane(row, 63);
        const uint32_t next_row = shfl(row, (int)min(lane + LPT, 63u));
        if ((grp == TPW - 1 || next_row != row) && row != r_last)
            store_values<T, K>(p, row, sub, rkeep, v, straddles(row), chunk_id, row == r_first ? 0 : 1);
#pragma unroll
        for (int k = 0; k < RPL; ++k) acc[k] = row == r_last ? part[k] : KT::id();
        r_cur = r_last;
        r_end = p.trp[r_cur + 1];
        keep = keep_bits<T>(p.mask, p.flags, r_cur);
        base += TPW;
    }
    V tot[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        tot[k] = acc[k];
#pragma unroll
        for (int d = LPT; d < 64; d <<= 1) tot[k] = KT::op(tot[k], shfl_xor(tot[k], d));
    }
    if (grp == 0) store_values<T, K>(p, r_cur, sub, keep, tot, straddles(r_cur), chunk_id, r_cur == r_first ? 0 : 1);
    if constexpr (K == kPlusF32) {
        if (lane == 0) {
            p.ws_rows[2 * chunk_id] = r_first;
            p.ws_rows[2 * chunk_id + 1] = r_cur;
        }
    }
}

// Float sums of rows that straddle chunks: the chunk where such a row starts
// adds its own partial and those of the following chunks, in chunk order.
template <int T> __global__ void __launch_bounds__(256) plus_fixup_kernel(SpmvArgs p, uint32_t nchunks)
{
    const uint64_t c64 = (uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE;
    if (c64 >= nchunks) return;
    const uint32_t c = (uint32_t)c64, lane = lane_id();
    const uint32_t t_begin = c * p.chunk, t_end = min(t_begin + p.chunk, p.ntiles);
    const uint32_t r_first = p.ws_rows[2 * c], R = p.ws_rows[2 * c + 1];
    if (p.trp[R + 1] <= t_end || p.trp[R] < t_begin) return;  // R does not start here or ends here
    if (lane >= (uint32_t)T) return;
    float sum = p.ws_part[((size_t)c * 2 + (R == r_first ? 0 : 1)) * T + lane];
    for (uint32_t c2 = c + 1; c2 < nchunks && p.ws_rows[2 * c2] == R; ++c2)
        sum += p.ws_part[(size_t)c2 * 2 * T + lane];
    const uint32_t row = R * T + lane;
    if (row >= p.n || !((keep_bits<T>(p.mask, p.flags, R) >> lane) & 1u)) return;
    float *y = (float *)p.y + row;
    if (p.flags & B2SR_ACCUMULATE) *y = *y + p.alpha * sum;
    else *y = p.alpha * sum + p.beta;
}

// Output initialisation: identity (or the diagonal term under SELF) for every
// row, so rows without tiles and masked rows end with the right value.
template <int K> __global__ void init_values_kernel(SpmvArgs p)
{
    using KT = KindTraits<K>;
    using V = typename KT::V;
    const bool accumulate = p.flags & B2SR_ACCUMULATE;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += (uint64_t)gridDim.x * blockDim.x) {
        bool keep = true;
        if (p.mask) {
            const bool bit = (p.mask[i >> 5] >> (i & 31)) & 1u;
            keep = (p.flags & B2SR_MASK_COMPLEMENT) ? !bit : bit;
        }
        V *y = (V *)p.y + i;
        if constexpr (K == kPlusF32) {
            if (accumulate) { if (keep && p.beta != 0.0f) *y = *y + p.beta; }
            else *y = keep ? p.beta : 0.0f;
        } else if constexpr (K == kMinF32 || K == kMinU32) {
            const V self = (keep && (p.flags & B2SR_SELF)) ? ((const V *)p.x)[i] : KT::id();
            if (accumulate) *y = KT::op(*y, self);
            else *y = self;
        } else {
            if (!accumulate) *y = KT::id();
        }
    }
}

template <int T, int K> int launch_values(SpmvArgs p, hipStream_t stream)
{
    const uint32_t nchunks = (uint32_t)((p.ntiles + (uint64_t)p.chunk - 1) / p.chunk);
    if (p.n) {
        init_values_kernel<K><<<b2sr::grid_for(p.n, 256, 65536), 256, 0, stream>>>(p);
        if (int rc = b2sr::check_launch("init_values_kernel")) return rc;
    }
    if (nchunks == 0) return B2SR_OK;
    spmv_values_kernel<T, K><<<b2sr::grid_for(nchunks, 4), 256, 0, stream>>>(p);
    if (int rc = b2sr::check_launch("spmv_values_kernel")) return rc;
    if constexpr (K == kPlusF32) {
        plus_fixup_kernel<T><<<b2sr::grid_for(nchunks, 4), 256, 0, stream>>>(p, nchunks);
        if (int rc = b2sr::check_launch("plus_fixup_kernel")) return rc;
    }
    return B2SR_OK;
}

template <int K> int dispatch_values(uint32_t T, const SpmvArgs &p, hipStream_t s)
{
    switch (T) {
    case 4: return launch_values<4, K>(p, s);
    case 8: return launch_values<8, K>(p, s);
    case 16: return launch_values<16, K>(p, s);
    default: return launch_values<32, K>(p, s);
    }
}

template <int T> int launch_bits(const SpmvArgs &p, hipStream_t stream)
{
    const uint32_t nchunks = (uint32_t)((p.ntiles + (uint64_t)p.chunk - 1) / p.chunk);
    if (nchunks == 0) return B2SR_OK;
    spmv_bits_kernel<T><<<b2sr::grid_for(nchunks, 4), 256, 0, stream>>>(p);
    return b2sr::check_launch("spmv_bits_kernel");
}

SpmvArgs make_args(const b2sr_matrix *A)
{
    SpmvArgs p{};
    p.trp = A->tile_rowptr;
    p.tci = A->tile_colind;
    p.bits = A->bits;
    p.n = A->n;
    p.ntr = b2sr::n_tile_rows(A->n, A->tile);
    p.ntiles = A->ntiles;
    p.chunk = chunk_tiles_rt(A->tile);
    return p;
}

}  // namespace

namespace b2sr {
int fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t stream);
}

extern "C" {

int spmv_bin_bin(const b2sr_matrix *A, const uint32_t *x, const uint32_t *mask, unsigned flags, void *y,
                 hipStream_t stream)
{
    int rc = b2sr::validate_matrix(A);
    if (rc) return rc;
    if (flags & ~(B2SR_MASK_COMPLEMENT | B2SR_OUT_COUNT | B2SR_ACCUMULATE)) return B2SR_EINVAL;
    if (A->n > 0 && (!x || !y)) return B2SR_EINVAL;
    if (A->n == 0) return B2SR_OK;
    if ((const void *)x == y || (const void *)mask == y) return B2SR_EINVAL;
    SpmvArgs p = make_args(A);
    p.x = x;
    p.mask = mask;
    p.flags = flags;
    p.y = y;
    if (flags & B2SR_OUT_COUNT) {
        if (!(flags & B2SR_ACCUMULATE) && (rc = b2sr::fill_u32((uint32_t *)y, A->n, 0, stream))) return rc;
        return dispatch_values<kCount>(A->tile, p, stream);
    }
    if (!(flags & B2SR_ACCUMULATE) && (rc = b2sr::fill_u32((uint32_t *)y, b2sr::n_words(A->n), 0, stream)))
        return rc;
    switch (A->tile) {
    case 4: return launch_bits<4>(p, stream);
    case 8: return launch_bits<8>(p, stream);
    case 16: return launch_bits<16>(p, stream);
    default: return launch_bits<32>(p, stream);
    }
}

size_t spmv_bin_full_workspace_bytes(const b2sr_matrix *A, int semiring)
{
    if (!A || !b2sr::valid_tile(A->tile) || semiring != B2SR_PLUS_TIMES_F32) return 0;
    const uint64_t nchunks = ((uint64_t)A->ntiles + chunk_tiles_rt(A->tile) - 1) / chunk_tiles_rt(A->tile);
    const uint64_t rows_bytes = (nchunks * 2 * 4 + 255) & ~255ull;
    return (size_t)(rows_bytes + nchunks * 2 * A->tile * 4);
}

int spmv_bin_full(const b2sr_matrix *A, int semiring, const void *x, const float *col_scale,
                  const uint32_t *mask, unsigned flags, double alpha, double beta, void *y, void *ws,
                  size_t ws_bytes, hipStream_t stream)
{
    int rc = b2sr::validate_matrix(A);
    if (rc) return rc;
    if (semiring < B2SR_PLUS_TIMES_F32 || semiring > B2SR_OR_U64) return B2SR_ENOTSUP;
    if (flags & ~(B2SR_MASK_COMPLEMENT | B2SR_ACCUMULATE | B2SR_SELF)) return B2SR_EINVAL;
    if ((flags & B2SR_SELF) && semiring != B2SR_MIN_PLUS_F32 && semiring != B2SR_MIN_PLUS_U32) return B2SR_EINVAL;
    if (col_scale && semiring != B2SR_PLUS_TIMES_F32) return B2SR_EINVAL;
    if (semiring == B2SR_MIN_PLUS_U32 && !(alpha >= 0.0 && alpha <= 4294967295.0 && alpha == (double)(uint32_t)alpha))
        return B2SR_EINVAL;
    if (A->n > 0 && (!x || !y)) return B2SR_EINVAL;
    if (A->n == 0) return B2SR_OK;
    if (x == y) return B2SR_EINVAL;
    const size_t need = spmv_bin_full_workspace_bytes(A, semiring);
    if (ws_bytes < need || (need && !ws)) return B2SR_ENOSPC;
    SpmvArgs p = make_args(A);
    p.x = x;
    p.s = col_scale;
    p.mask = mask;
    p.flags = flags;
    p.alpha = (float)alpha;
    p.beta = (float)beta;
    p.w_u32 = semiring == B2SR_MIN_PLUS_U32 ? (uint32_t)alpha : 0u;
    p.y = y;
    if (need) {
        const uint64_t nchunks = ((uint64_t)A->ntiles + p.chunk - 1) / p.chunk;
        p.ws_rows = (uint32_t *)ws;
        p.ws_part = (float *)((char *)ws + ((nchunks * 2 * 4 + 255) & ~255ull));
    }
    switch (semiring) {
    case B2SR_PLUS_TIMES_F32: return dispatch_values<kPlusF32>(A->tile, p, stream);
    case B2SR_MIN_PLUS_F32: return dispatch_values<kMinF32>(A->tile, p, stream);
    case B2SR_MIN_PLUS_U32: return dispatch_values<kMinU32>(A->tile, p, stream);
    default: return dispatch_values<kOr64>(A->tile, p, stream);
    }
}

}  // extern "C"
