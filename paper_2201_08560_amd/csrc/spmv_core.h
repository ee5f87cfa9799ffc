// Device-side machinery of the B2SR matrix-vector products, shared by the
// product kernels (spmv.hip) and the persistent batched BFS (batch.hip).
// Internal to libb2sr.so.
#pragma once

#include <type_traits>

#include "common.h"

// Tuning knobs (compile-time; the defaults are the measured choices).
#ifndef B2SR_TARGET_WAVES
#define B2SR_TARGET_WAVES 65536  // waves per product launch the chunk size aims at
#endif
#ifndef B2SR_BITS_STEPS
#define B2SR_BITS_STEPS 8        // steps per block for bit and count products, T = 32
#endif
#ifndef B2SR_BITS_STEPS_SMALL
#define B2SR_BITS_STEPS_SMALL 8  // the same for T <= 16
#endif
#ifndef B2SR_BITS_STEPS_SHORT
#define B2SR_BITS_STEPS_SHORT 4  // the same for short tile-rows and sparse frontiers
#endif
#ifndef B2SR_STAGE_BYTES
#define B2SR_STAGE_BYTES 4096    // LDS bytes per wave for staged x segments
#endif
#ifndef B2SR_X_DMA
#define B2SR_X_DMA 1             // stage 4-byte x segments at T = 32 with global-to-LDS loads
#endif
#ifndef B2SR_NT_TILES
#define B2SR_NT_TILES 1          // stream tile bits with nontemporal loads
#endif
#ifndef B2SR_FAST_BLOCKS
#define B2SR_FAST_BLOCKS 1       // value products at T >= 32: the lean path for whole in-row blocks
#endif
#ifndef B2SR_FAST_PIPE
#define B2SR_FAST_PIPE 1         // runs of lean blocks load the next block's tiles before a block's wait
#endif
#ifndef B2SR_ACT_PREFETCH
#define B2SR_ACT_PREFETCH 1      // products with x_active load the next block's tile columns a block ahead
#endif

namespace b2sr_core {

using namespace b2sr_dev;

template <class P> __device__ __forceinline__ P load_stream(const P *p)
{
#if B2SR_NT_TILES
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

enum Kind : int { kBits = 0, kCount = 1, kPlusF32 = 2, kMinF32 = 3, kMinU32 = 4, kOr64 = 5, kMaxU64 = 6 };

template <int K> struct KindTraits;
template <> struct KindTraits<kBits> {
    using V = uint32_t;
    static __device__ __forceinline__ V id() { return 0u; }
    static __device__ __forceinline__ V op(V a, V b) { return a | b; }
};
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
template <> struct KindTraits<kMaxU64> {
    using V = uint64_t;
    static __device__ __forceinline__ V id() { return 0ull; }
    static __device__ __forceinline__ V op(V a, V b) { return b > a ? b : a; }
};

struct SpmvArgs {
    const uint32_t *trp;
    const uint32_t *tci;
    const void *bits;
    uint32_t n, ntr, ntiles, chunk;
    const void *x;
    const uint32_t *xact;  // value products: columns whose x entries take part (nullable: all)
    const uint32_t *mask;
    unsigned flags;
    float alpha, beta;
    uint32_t w_u32;
    void *y;
    uint32_t *ws_rows;  // float sums: first and last row of each chunk
    float *ws_part;     // float sums: partials of straddling rows, 2*T per chunk
    uint32_t x_whole;   // n is a multiple of T: no x segment is cut short
    uint32_t chunk_blocks;  // blocks per wave chunk (0: sized from the tile count)
    // Iteration gating (the algorithm drivers): when gate is set, every kernel
    // of the product returns at once unless *gate == gate_val.
    const uint32_t *gate;
    uint32_t gate_val;
};

__device__ __forceinline__ bool gated_off(const SpmvArgs &p) { return p.gate && *p.gate != p.gate_val; }

// Block shape per tile width and kind.  Bit and count products read the x
// segment as T bits; the others stage T values per tile in LDS (a fixed budget
// per wave, so the block shrinks as the vector values widen).  At T = 64 a
// bit-product block holds half the steps, so that a lane keeps as many tile
// bytes in flight (8 KiB per wave) as at T = 32.
// SHORT (bit and count products): fewer steps per block, for matrices whose
// tile-rows are shorter than a block and for sparse frontiers; fewer
// registers then buy occupancy where the long blocks' loads would be cut short.
template <int T, int K, bool SHORT = false> struct Cfg {
    using S = TileShape<T>;
    static constexpr int LPT = S::LPT, RPL = S::RPL, TPW = S::TPW;
    static constexpr bool kStage = K >= kPlusF32;
    static constexpr int VB = sizeof(typename KindTraits<K>::V);
    static constexpr int U = kStage ? B2SR_STAGE_BYTES / (TPW * T * VB)
                           : SHORT  ? (T == 64 ? (B2SR_BITS_STEPS_SHORT + 1) / 2 : B2SR_BITS_STEPS_SHORT)
                           : T == 64 ? (B2SR_BITS_STEPS + 1) / 2
                                    : (T == 32 ? B2SR_BITS_STEPS : B2SR_BITS_STEPS_SMALL);
    static constexpr int BT = U * TPW;                 // tiles per block
    static constexpr int JK = BT >= 64 ? BT / 64 : 1;  // tile-column registers per lane
    static constexpr int XW = T / LPT;                 // staged x values per lane per tile
    static_assert(U >= 1 && (64 % TPW) == 0, "block shape");
};

// Tiles per wave chunk: `blocks` whole blocks when given (the matrix view's
// chunk_blocks), else aiming at about B2SR_TARGET_WAVES waves per launch,
// between 1 and 16 blocks.  A pure function of (T, kind, ntiles, blocks), so
// the float-sum workspace query and the launch agree.
template <int T, int K, bool SHORT = false> inline uint32_t chunk_tiles(uint32_t ntiles, uint32_t blocks = 0)
{
    constexpr uint32_t bt = Cfg<T, K, SHORT>::BT;
    if (blocks) return bt * blocks;
    constexpr uint64_t waves = B2SR_TARGET_WAVES;
    uint64_t nb = ((uint64_t)ntiles + waves * bt - 1) / (waves * bt);
    nb = nb < 1 ? 1 : (nb > 16 ? 16 : nb);
    return (uint32_t)(bt * nb);
}

// One lane's raw piece of a tile.
template <int T> struct PieceT { using type = u32x4; };
template <> struct PieceT<64> { using type = u32x8; };
template <> struct PieceT<8> { using type = u32x2; };
template <> struct PieceT<4> { using type = uint32_t; };

template <int T> __device__ __forceinline__ typename PieceT<T>::type load_piece(const void *bits, uint32_t t, uint32_t sub)
{
    if constexpr (T == 64) {
        // two 16-byte loads (rows 4 sub .. 4 sub + 3 of the 512-byte tile)
        const u32x4 *q = (const u32x4 *)bits + ((size_t)t * 32 + 2 * sub);
        const u32x4 lo = load_stream(q), hi = load_stream(q + 1);
        return u32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    }
    else if constexpr (T == 32) return load_stream((const u32x4 *)bits + ((size_t)t * 8 + sub));
    else if constexpr (T == 16) return load_stream((const u32x4 *)bits + ((size_t)t * 2 + sub));
    else if constexpr (T == 8) return load_stream((const u32x2 *)bits + t);
    else return load_stream((const uint32_t *)bits + t);
}

// 512 zero bytes (the largest tile), the stand-in tile of lanes that skip
// their tile: every lane issues every load of a block, so waits count the
// loads exactly.
static __device__ __align__(16) uint32_t g_zero_tile[128];

// The piece of tile t when `use`, else the same piece of the zero tile.
template <int T>
__device__ __forceinline__ typename PieceT<T>::type load_piece_or_zero(const void *bits, uint32_t t, uint32_t sub, bool use)
{
    return load_piece<T>(use ? bits : (const void *)g_zero_tile, use ? t : 0u, sub);
}

template <int T> __device__ __forceinline__ typename PieceT<T>::type zero_piece()
{
    typename PieceT<T>::type z;
    if constexpr (T == 4) z = 0u;
    else z = 0u;  // splat
    return z;
}

// The RPL bit-rows of a piece as T-bit values (Table II word layout).
template <int T>
__device__ __forceinline__ void piece_rows(const typename PieceT<T>::type &v, row_t<T> (&a)[TileShape<T>::RPL])
{
    if constexpr (T == 64) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] = ((uint64_t)v[2 * k + 1] << 32) | v[2 * k];
    } else if constexpr (T == 32) {
        a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
    } else if constexpr (T == 16) {
        a[0] = v.x & 0xFFFFu; a[1] = v.x >> 16; a[2] = v.y & 0xFFFFu; a[3] = v.y >> 16;
        a[4] = v.z & 0xFFFFu; a[5] = v.z >> 16; a[6] = v.w & 0xFFFFu; a[7] = v.w >> 16;
    } else if constexpr (T == 8) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = (v.x >> (8 * k)) & 0xFFu;
            a[4 + k] = (v.y >> (8 * k)) & 0xFFu;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] = (v >> (8 * k)) & 0xFu;
    }
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

// Rows of tile-row I that the mask keeps, as T bits (n: the vector length).
template <int T>
__device__ __forceinline__ row_t<T> keep_bits(const uint32_t *mask, unsigned flags, uint32_t I, uint32_t n)
{
    using R = row_t<T>;
    constexpr R full = T >= 32 ? ~(R)0 : (R)((1u << T) - 1u);
    if (!mask) return full;
    const R w = bit_segment<T>(mask, I, n);
    return (flags & B2SR_MASK_COMPLEMENT) ? (R)(~w & full) : w;
}

__device__ __forceinline__ uint32_t popc_row(uint32_t v) { return (uint32_t)__popc(v); }
__device__ __forceinline__ uint32_t popc_row(uint64_t v) { return (uint32_t)__popcll(v); }
__device__ __forceinline__ uint32_t ctz_row(uint32_t v) { return (uint32_t)__builtin_ctz(v); }
__device__ __forceinline__ uint32_t ctz_row(uint64_t v) { return (uint32_t)__builtin_ctzll(v); }

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Row stores
// ---------------------------------------------------------------------------

template <int T> __device__ __forceinline__ void store_bits(const SpmvArgs &p, uint32_t I, row_t<T> m)
{
    if (!m) return;
    if constexpr (T == 64) {
        // the two words of the segment; the upper one exists whenever a row in
        // it does (rows >= n hold no bits)
        const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
        if (lo) atomicOr((uint32_t *)p.y + 2 * (size_t)I, lo);
        if (hi) atomicOr((uint32_t *)p.y + 2 * (size_t)I + 1, hi);
    } else {
        const uint32_t bit = I * T;
        atomicOr((uint32_t *)p.y + (bit >> 5), m << (bit & 31u));
    }
}

// Stores the RPL rows [sub*RPL, sub*RPL + RPL) of tile-row I.
template <int T, int K>
__device__ __forceinline__ void store_values(const SpmvArgs &p, uint32_t I, uint32_t sub, row_t<T> keep,
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
        } else if constexpr (K == kMaxU64) {
            if (v[k]) atomicMax((unsigned long long *)p.y + row, (unsigned long long)v[k]);
        } else {
            if (v[k]) atomicOr((unsigned long long *)p.y + row, (unsigned long long)v[k]);
        }
    }
}

// ---------------------------------------------------------------------------
// The product kernel, one template for every kind
// ---------------------------------------------------------------------------

// LDS per wave for the staged kinds (the same for every T and kind).
constexpr uint32_t kStageBytesPerWave = B2SR_STAGE_BYTES;
// A wave's LDS slice: the staged segments, then 16 bytes whose first value is
// the semiring's identity (the value an empty bit-row reads).
constexpr uint32_t kSliceBytes = kStageBytesPerWave + 16;

// The staged x value a bit-row selects first: the value of its lowest set bit
// in the tile's staged segment xt, or, for an empty row, the identity slot
// after the wave's slice xs.
template <class V, class R> __device__ __forceinline__ V xt_or_id(const V *xt, R row, const V *xs)
{
    return row ? xt[ctz_row(row)] : xs[kStageBytesPerWave / sizeof(V)];
}

// A whole block of BT tiles of one tile-row, for the value products with
// 4-byte values at T >= 32 (wave-uniform conditions checked by the caller: the
// block lies before the chunk's end and inside the current tile-row, every x
// segment is whole, no x_active).  Lane l reads piece l of each step's run of
// tiles at a fixed offset from the block's first tile (no per-lane bounds or
// zero-tile selection), the x segments go to LDS by global-to-LDS loads, and
// each bit-row costs one LDS read for its lowest set bit; rows with more set
// bits (rare at these widths on sparse graphs) take a loop.  Sums are folded
// into acc in bit order, the same fixed order as the general path.
// J holds the block's tile columns (lane l: tile blk + l) on entry and the next
// block's on exit, loaded ahead so that the x loads never wait for them.
template <int T, int K>
__device__ __forceinline__ void fast_block(const SpmvArgs &p, uint32_t blk, uint32_t t_end,
                                           typename KindTraits<K>::V *xs,
                                           typename KindTraits<K>::V (&acc)[TileShape<T>::RPL], uint32_t &J)
{
    using C = Cfg<T, K>;
    using KT = KindTraits<K>;
    using V = typename KT::V;
    using R = row_t<T>;
    using Piece = typename PieceT<T>::type;
    constexpr int RPL = C::RPL, TPW = C::TPW, U = C::U, BT = C::BT, XW = C::XW, LPT = C::LPT;
    static_assert(BT <= 64 && C::VB == 4 && T >= 32, "fast block shape");
    const uint32_t lane = lane_id(), grp = lane / LPT, sub = lane % LPT;
    // the x offsets first, from the columns loaded a block ago (landed at the
    // last block's barrier), so that nothing below waits on a load of this block
    uint32_t xo[U];
#pragma unroll
    for (int i = 0; i < U; ++i) xo[i] = shfl(J, (int)(i * TPW + grp)) * T + sub * XW;
    __builtin_amdgcn_sched_barrier(0);  // no load of this block is moved above the offsets
    J = p.tci[min(blk + BT + min(lane, (uint32_t)BT - 1), t_end - 1)];
    Piece pc[U];
    if constexpr (T == 64) {
        const u32x4 *q = (const u32x4 *)p.bits + (size_t)blk * 32;
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const u32x4 lo = load_stream(q + (i * 128 + 2 * lane)), hi = load_stream(q + (i * 128 + 2 * lane + 1));
            pc[i] = u32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
        }
    } else {
        const u32x4 *q = (const u32x4 *)p.bits + (size_t)blk * 8;
#pragma unroll
        for (int i = 0; i < U; ++i) pc[i] = load_stream(q + (i * 64 + lane));
    }
    const uint32_t xs_lds = readfirstlane((uint32_t)(uintptr_t)xs);
#pragma unroll
    for (int i = 0; i < U; ++i)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)((const V *)p.x + xo[i]),
                                         (__attribute__((address_space(3))) void *)(uintptr_t)(xs_lds + i * TPW * T * 4),
                                         16, 0, 0);
    __builtin_amdgcn_sched_barrier(0);  // every load is issued before the first wait
    // the global-to-LDS loads count in vmcnt: wait for all of them explicitly
    // before any LDS read, rather than rely on the compiler's alias analysis
    __builtin_amdgcn_s_waitcnt(0);
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < U; ++i) {
        R a[RPL];
        piece_rows<T>(pc[i], a);
        const V *xt = xs + (i * TPW + grp) * T;
        V v[RPL];
#pragma unroll
        // an empty row reads the identity slot after the slice: one address for
        // all such lanes is a broadcast (each tile's own first value would
        // conflict across the step's tiles, whose segments all start at bank 0)
        for (int k = 0; k < RPL; ++k) v[k] = xt_or_id(xt, a[k], xs);
        R more = 0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            acc[k] = KT::op(acc[k], v[k]);
            a[k] &= a[k] - 1;
            more |= a[k];
        }
        if (more) {
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                R w = a[k];
                while (w) {
                    const uint32_t c = ctz_row(w);
                    w &= w - 1;
                    acc[k] = KT::op(acc[k], xt[c]);
                }
            }
        }
    }
    wave_lds_sync();  // the next block's LDS writes follow these reads
}

// s_waitcnt limiting only the vector-memory counter (the gfx9 encoding: vmcnt
// in bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima).
template <int N> __device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// nb >= 1 consecutive lean blocks from blk, all inside one tile-row and the
// chunk, software-pipelined: block b + 1's tile pieces are loaded before block
// b's wait, so they stream in while block b is reduced.  Vector loads complete
// in issue order, so waiting until at most the next block's piece loads remain
// covers this block's pieces, columns and x segments.  The run's last block
// has no successor to load and waits for everything.  On entry J holds the
// tile columns of block blk (loaded, one per lane); on return those of the
// block after the run.
template <int T, int K>
__device__ __forceinline__ void fast_run(const SpmvArgs &p, uint32_t blk, uint32_t nb, uint32_t t_end,
                                         typename KindTraits<K>::V *xs,
                                         typename KindTraits<K>::V (&acc)[TileShape<T>::RPL], uint32_t &J)
{
    using C = Cfg<T, K>;
    using KT = KindTraits<K>;
    using V = typename KT::V;
    using R = row_t<T>;
    using Piece = typename PieceT<T>::type;
    constexpr int RPL = C::RPL, TPW = C::TPW, U = C::U, BT = C::BT, XW = C::XW, LPT = C::LPT;
    constexpr int kPieceLoads = (T == 64 ? 2 : 1) * U;  // vector loads per block's pieces
    static_assert(BT <= 64 && C::VB == 4 && T >= 32, "fast block shape");
    const uint32_t lane = lane_id(), grp = lane / LPT, sub = lane % LPT;
    const uint32_t xs_lds = readfirstlane((uint32_t)(uintptr_t)xs);
    Piece cur[U], nxt[U];
    auto load_pieces = [&](uint32_t b, Piece(&pc)[U]) {
        if constexpr (T == 64) {
            const u32x4 *q = (const u32x4 *)p.bits + (size_t)b * 32;
#pragma unroll
            for (int i = 0; i < U; ++i) {
                const u32x4 lo = load_stream(q + (i * 128 + 2 * lane)), hi = load_stream(q + (i * 128 + 2 * lane + 1));
                pc[i] = u32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
            }
        } else {
            const u32x4 *q = (const u32x4 *)p.bits + (size_t)b * 8;
#pragma unroll
            for (int i = 0; i < U; ++i) pc[i] = load_stream(q + (i * 64 + lane));
        }
    };
    // the next block's columns, then this block's x segments into LDS
    auto stage_x = [&]() {
        uint32_t xo[U];
#pragma unroll
        for (int i = 0; i < U; ++i) xo[i] = shfl(J, (int)(i * TPW + grp)) * T + sub * XW;
        __builtin_amdgcn_sched_barrier(0);
        J = p.tci[min(blk + BT + min(lane, (uint32_t)BT - 1), t_end - 1)];
#pragma unroll
        for (int i = 0; i < U; ++i)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)((const V *)p.x + xo[i]),
                                             (__attribute__((address_space(3))) void *)(uintptr_t)(xs_lds + i * TPW * T * 4),
                                             16, 0, 0);
    };
    auto reduce = [&]() {
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < U; ++i) {
            R a[RPL];
            piece_rows<T>(cur[i], a);
            const V *xt = xs + (i * TPW + grp) * T;
            V v[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k) v[k] = xt_or_id(xt, a[k], xs);  // empty rows: a broadcast
            R rest = 0;
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                acc[k] = KT::op(acc[k], v[k]);
                a[k] &= a[k] - 1;
                rest |= a[k];
            }
            if (rest) {
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    R w = a[k];
                    while (w) {
                        const uint32_t c = ctz_row(w);
                        w &= w - 1;
                        acc[k] = KT::op(acc[k], xt[c]);
                    }
                }
            }
        }
        wave_lds_sync();  // the next block's LDS writes follow these reads
        blk += BT;
    };
    load_pieces(blk, cur);
    for (uint32_t k = 1; k < nb; ++k) {
        stage_x();
        load_pieces(blk + BT, nxt);
        __builtin_amdgcn_sched_barrier(0);  // every load is issued before the wait
        wait_vmcnt<kPieceLoads>();
        reduce();
#pragma unroll
        for (int i = 0; i < U; ++i) cur[i] = nxt[i];
    }
    stage_x();
    __builtin_amdgcn_sched_barrier(0);
    wait_vmcnt<0>();
    reduce();
}

// Processes tile chunk chunk_id (wave-uniform) of the product described by p.
// xs is this wave's LDS slice (unused by bit and count products).
template <int T, int K, bool ACT = false, bool SHORT = false>
__device__ __forceinline__ void spmv_chunk(const SpmvArgs &p, uint32_t chunk_id, typename KindTraits<K>::V *xs)
{
    using C = Cfg<T, K, SHORT>;
    using KT = KindTraits<K>;
    using V = typename KT::V;
    using Piece = typename PieceT<T>::type;
    constexpr int LPT = C::LPT, RPL = C::RPL, TPW = C::TPW, U = C::U, BT = C::BT, JK = C::JK, XW = C::XW;
    static_assert(!C::kStage || BT * T * sizeof(V) <= kStageBytesPerWave, "LDS slice");
    // Partials of one lane: a bit mask for kBits, RPL values otherwise.
    constexpr int NV = K == kBits ? 1 : RPL;
    using R = row_t<T>;                                                  // one bit-row
    using AV = typename std::conditional<K == kBits, R, V>::type;        // a partial

    const uint32_t lane = lane_id(), grp = lane / LPT, sub = lane % LPT;
    const uint32_t t_begin = chunk_id * p.chunk;
    const uint32_t t_end = min(t_begin + p.chunk, p.ntiles);

    if constexpr (C::kStage) {
        // the identity slot after the slice (read by empty rows, after the first
        // staging's LDS sync)
        if (lane == 0) xs[kStageBytesPerWave / sizeof(V)] = KT::id();
    }
    const uint32_t r_first = find_row(p.trp, p.ntr, t_begin);
    uint32_t r_cur = r_first;
    uint32_t r_end = p.trp[r_cur + 1];
    R keep = keep_bits<T>(p.mask, p.flags, r_cur, p.n);
    // A row straddles chunks when it starts before t_begin or ends after t_end;
    // only the chunk's first and last rows can.
    auto straddles = [&](uint32_t I) { return p.trp[I] < t_begin || p.trp[I + 1] > t_end; };
    auto slot_of = [&](uint32_t I) { return I == r_first ? 0u : 1u; };

    AV acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = KT::id();
    // Bit products fold raw AND words per bit-row in the common case and form
    // the row bits only when a row is finished.
    R raw[K == kBits ? RPL : 1];
#pragma unroll
    for (int k = 0; k < (K == kBits ? RPL : 1); ++k) raw[k] = 0;
    auto fold_raw = [&]() {
        if constexpr (K == kBits) {
            R m = 0;
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                m |= (R)(raw[k] != 0) << (sub * RPL + k);
                raw[k] = 0;
            }
            acc[0] |= m;
        }
    };

    uint32_t blk = t_begin;
    // fast blocks: the tile columns of block jf_blk, loaded one block ahead
    [[maybe_unused]] uint32_t jf = 0, jf_blk = 0xFFFFFFFFu;
    // products with x_active: the next block's tile columns, loaded while this
    // block is examined (most blocks of a small frontier are skipped after
    // reading only their columns and those columns' activity bits)
    [[maybe_unused]] uint32_t jn[JK], jn_blk = 0xFFFFFFFFu;
    while (blk < t_end) {
        if (min(blk + BT, t_end) - 1 < r_end && !keep) {  // the block lies in a row masked out entirely
            blk = min(r_end, t_end);
            continue;
        }
        if constexpr (B2SR_FAST_BLOCKS && C::kStage && !ACT && T >= 32 && C::VB == 4) {
            if (p.x_whole && blk + BT <= t_end && blk + BT - 1 < r_end) {
                if (jf_blk != blk) jf = p.tci[blk + min(lane, (uint32_t)BT - 1)];
                if constexpr (B2SR_FAST_PIPE) {
                    const uint32_t nb = (min(r_end, t_end) - blk) / BT;  // >= 1
                    fast_run<T, K>(p, blk, nb, t_end, xs, acc, jf);
                    blk += nb * BT;
                } else {
                    fast_block<T, K>(p, blk, t_end, xs, acc, jf);
                    blk += BT;
                }
                jf_blk = blk;
                continue;
            }
        }
        // ---- load phase: tile columns (one per lane), tile pieces, x segments.
        // No load sits under a per-lane branch (lanes past the chunk read its
        // last column and the zero tile), so a wait covers just the loads it needs:
        // the column loads come first, and the x reads that depend on them are
        // issued while the tile pieces are still in flight.
        uint32_t Jr[JK];
        if constexpr (ACT && B2SR_ACT_PREFETCH) {
            if (jn_blk == blk) {
#pragma unroll
                for (int k = 0; k < JK; ++k) Jr[k] = jn[k];
            } else {
#pragma unroll
                for (int k = 0; k < JK; ++k) Jr[k] = p.tci[min(blk + 64 * k + lane, t_end - 1)];
            }
            jn_blk = blk + BT;
#pragma unroll
            for (int k = 0; k < JK; ++k) jn[k] = p.tci[min(jn_blk + 64 * k + lane, t_end - 1)];
        } else {
#pragma unroll
            for (int k = 0; k < JK; ++k) Jr[k] = p.tci[min(blk + 64 * k + lane, t_end - 1)];
        }
        Piece pc[U];
        R seg[U];
        if constexpr (!C::kStage) {
            R Sr[JK];
            // (At T = 32 the measured best is a per-lane branch for the sparse
            // hint and a clamped tile index for the dense case; below T = 32 the
            // zero tile in both.)
            if (p.flags & B2SR_SPARSE_X) {
                // read a tile only when its x segment has a set bit
#pragma unroll
                for (int k = 0; k < JK; ++k) Sr[k] = bit_segment<T>((const uint32_t *)p.x, Jr[k], p.n);
                if constexpr (K == kBits && SHORT) {
                    // A block inside the current row none of whose tiles meets a set x
                    // bit adds nothing to it (a block across a row end takes the
                    // general path, which stores the row).  Only in the short-block
                    // form, which sparse frontiers use: in the long one the test costs
                    // the dense path registers.
                    if (min(blk + BT, t_end) - 1 < r_end) {
                        bool seg_any = false;
#pragma unroll
                        for (int k = 0; k < JK; ++k)
                            seg_any |= Sr[k] != 0 && 64 * k + lane < (uint32_t)BT && blk + 64 * k + lane < t_end;
                        if (!__any(seg_any)) {
                            blk += BT;
                            continue;
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    const uint32_t ti = i * TPW + grp;
                    seg[i] = shfl(Sr[(i * TPW) / 64], (int)(ti % 64));
                    const bool use = blk + ti < t_end && seg[i];
                    if constexpr (T >= 32) pc[i] = use ? load_piece<T>(p.bits, blk + ti, sub) : zero_piece<T>();
                    else pc[i] = load_piece_or_zero<T>(p.bits, blk + ti, sub, use);
                }
            } else if constexpr (T >= 32) {
                // lanes past the chunk read its last tile; their segment is cleared
#pragma unroll
                for (int i = 0; i < U; ++i) pc[i] = load_piece<T>(p.bits, min(blk + i * TPW + grp, t_end - 1), sub);
#pragma unroll
                for (int k = 0; k < JK; ++k) Sr[k] = bit_segment<T>((const uint32_t *)p.x, Jr[k], p.n);
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    const uint32_t ti = i * TPW + grp;
                    seg[i] = shfl(Sr[(i * TPW) / 64], (int)(ti % 64));
                    if (blk + ti >= t_end) seg[i] = 0;
                }
            } else {
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    const uint32_t t = blk + i * TPW + grp;
                    pc[i] = load_piece_or_zero<T>(p.bits, t, sub, t < t_end);
                }
                // a tile past the chunk holds no bits, whatever its segment
#pragma unroll
                for (int k = 0; k < JK; ++k) Sr[k] = bit_segment<T>((const uint32_t *)p.x, Jr[k], p.n);
#pragma unroll
                for (int i = 0; i < U; ++i) seg[i] = shfl(Sr[(i * TPW) / 64], (int)((i * TPW + grp) % 64));
            }
        } else {
            if constexpr (ACT) {
                // active columns only: a tile whose x segment is wholly inactive is not read
                R Sr[JK];
#pragma unroll
                for (int k = 0; k < JK; ++k) Sr[k] = bit_segment<T>(p.xact, Jr[k], p.n);
                // A block none of whose tiles has an active column contributes the
                // identity: nothing of it is loaded or staged; only the row the
                // block ends in is followed, and a row that ends inside it is stored.
                bool act_any = false;
#pragma unroll
                for (int k = 0; k < JK; ++k)
                    act_any |= Sr[k] != 0 && 64 * k + lane < (uint32_t)BT && blk + 64 * k + lane < t_end;
                if (!__any(act_any)) {
                    const uint32_t last = min(blk + BT, t_end) - 1;
                    if (last >= r_end) {
                        V tot[NV];
#pragma unroll
                        for (int k = 0; k < NV; ++k) {
                            tot[k] = acc[k];
#pragma unroll
                            for (int d = LPT; d < 64; d <<= 1) tot[k] = KT::op(tot[k], shfl_xor(tot[k], d));
                            acc[k] = KT::id();
                        }
                        if (grp == 0)
                            store_values<T, K>(p, r_cur, sub, keep, tot, straddles(r_cur), chunk_id, slot_of(r_cur));
                        r_cur = readfirstlane(lane_row(p.trp, p.ntr, r_cur, last));
                        r_end = p.trp[r_cur + 1];
                        keep = keep_bits<T>(p.mask, p.flags, r_cur, p.n);
                    }
                    blk += BT;
                    continue;
                }
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    const uint32_t ti = i * TPW + grp;
                    seg[i] = shfl(Sr[(i * TPW) / 64], (int)(ti % 64));
                    pc[i] = load_piece_or_zero<T>(p.bits, blk + ti, sub, blk + ti < t_end && seg[i]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    const uint32_t t = blk + i * TPW + grp;
                    pc[i] = load_piece_or_zero<T>(p.bits, t, sub, t < t_end);
                }
            }
            // x segments: every lane reads its XW values of every step's segment as
            // 16-byte quads, all steps at once; a lane whose tile is skipped reads
            // x's first quad instead (its tile holds no bits, so the values are
            // never selected).  A segment cut by n (the last tile column) is
            // completed value by value afterwards.
            constexpr int QV = 16 / C::VB;  // values per 16-byte quad
            constexpr int NQ = XW / QV;
            const bool quads = p.n >= (uint32_t)XW;
            u32x4 xq[U][NQ];
            uint32_t off[U];
            uint32_t partial = 0;
#pragma unroll
            for (int i = 0; i < U; ++i) {
                const uint32_t ti = i * TPW + grp;
                const uint32_t J = shfl(Jr[(i * TPW) / 64], (int)(ti % 64));
                bool use = blk + ti < t_end;
                if constexpr (ACT) use = use && seg[i];
                const uint32_t c0 = J * T + sub * XW;  // < n + T <= 2^32
                const bool full = (uint64_t)c0 + XW <= p.n;
                off[i] = use && full ? c0 : 0u;
                partial |= (uint32_t)(use && !full) << i;
            }
            // At T = 32 with 4-byte values a step's segments are one 16-byte quad per
            // lane at slot i * 1024 + 16 * lane: exactly where a global-to-LDS load
            // puts lane l's quad, so those bytes need no registers.
            constexpr bool kDma = B2SR_X_DMA && T >= 32 && NQ == 1;
            if (kDma && quads) {
#pragma unroll
                for (int i = 0; i < U; ++i)
                    __builtin_amdgcn_global_load_lds(
                        (const __attribute__((address_space(1))) void *)((const V *)p.x + off[i]),
                        (__attribute__((address_space(3))) void *)(xs + i * TPW * T), 16, 0, 0);
            } else if (quads) {
#pragma unroll
                for (int i = 0; i < U; ++i)
#pragma unroll
                    for (int q = 0; q < NQ; ++q) xq[i][q] = ((const u32x4 *)((const V *)p.x + off[i]))[q];
            } else {
#pragma unroll
                for (int i = 0; i < U; ++i)
#pragma unroll
                    for (int q = 0; q < NQ; ++q) xq[i][q] = u32x4{0u, 0u, 0u, 0u};
            }
            if (!(kDma && quads)) {
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    V *dst = xs + (i * TPW + grp) * T + sub * XW;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) ((u32x4 *)dst)[q] = xq[i][q];
                }
            }
            if (partial) {
                if constexpr (kDma) __builtin_amdgcn_s_waitcnt(0);  // the quads have landed before they are overwritten
                // only the last tile column can be cut by n; values past n are never selected
                const uint32_t c0 = (p.n - 1) / T * T + sub * XW;
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    if (!((partial >> i) & 1u)) continue;
                    V *dst = xs + (i * TPW + grp) * T + sub * XW;
                    for (int q = 0; q < XW; ++q) {
                        V v = KT::id();
                        if (c0 + q < p.n) v = ((const V *)p.x)[c0 + q];
                        dst[q] = v;
                    }
                }
            }
            if constexpr (kDma) __builtin_amdgcn_s_waitcnt(0);  // the global-to-LDS loads have landed
            wave_lds_sync();
        }

        // ---- compute phase, one step at a time
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t base = blk + i * TPW;
            if (base >= t_end) break;
            const uint32_t last = min(base + TPW, t_end) - 1;
            const bool valid = base + grp < t_end;
            const uint32_t t = valid ? base + grp : t_end - 1;
            const uint32_t ti = i * TPW + grp;
            AV part[NV];
            auto compute = [&]() {
                R a[RPL];
                piece_rows<T>(pc[i], a);
                if constexpr (K == kBits) {
                    R m = 0;
#pragma unroll
                    for (int k = 0; k < RPL; ++k) m |= (R)((a[k] & seg[i]) != 0) << (sub * RPL + k);
                    part[0] = m;
                } else if constexpr (K == kCount) {
#pragma unroll
                    for (int k = 0; k < RPL; ++k) part[k] = popc_row(a[k] & seg[i]);  // Listing 1's dot
                } else {
#pragma unroll
                    for (int k = 0; k < RPL; ++k) part[k] = KT::id();
                    R any = 0;
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        if constexpr (ACT) a[k] &= seg[i];  // inactive columns contribute the identity
                        any |= a[k];
                    }
                    if (any) {  // most lanes of a sparse tile hold no set bit
                        const V *xt = xs + ti * T;
                        if constexpr (T >= 32) {
                            // the lowest set bit of every row first, the rows' LDS reads
                            // together (about two set bits per tile on power-law graphs);
                            // the sum order within a row is unchanged
                            V v[RPL];
#pragma unroll
                            for (int k = 0; k < RPL; ++k) v[k] = xt_or_id(xt, a[k], xs);  // empty rows: a broadcast
                            any = 0;
#pragma unroll
                            for (int k = 0; k < RPL; ++k) {
                                part[k] = KT::op(part[k], v[k]);
                                a[k] &= a[k] - 1;
                                any |= a[k];
                            }
                        }
                        if (any) {
#pragma unroll
                            for (int k = 0; k < RPL; ++k) {
                                R w = a[k];
                                while (w) {
                                    const uint32_t c = ctz_row(w);
                                    w &= w - 1;
                                    part[k] = KT::op(part[k], xt[c]);
                                }
                            }
                        }
                    }
                }
            };
            if (last < r_end) {
                if constexpr (K == kBits) {
                    R a[RPL];
                    piece_rows<T>(pc[i], a);
#pragma unroll
                    for (int k = 0; k < RPL; ++k) raw[k] |= a[k] & seg[i];
                } else {
                    compute();
#pragma unroll
                    for (int k = 0; k < NV; ++k) acc[k] = KT::op(acc[k], part[k]);
                }
                continue;
            }
            fold_raw();
            // the step crosses the end of row r_cur
            const uint32_t row = lane_row(p.trp, p.ntr, r_cur, t);
            const R rkeep = row == r_cur ? keep : keep_bits<T>(p.mask, p.flags, row, p.n);
            if (valid && rkeep) compute();
            else {
#pragma unroll
                for (int k = 0; k < NV; ++k) part[k] = KT::id();
            }
            const uint32_t r_last = readlane(row, 63);
            const bool first_in_cur = readlane(row, 0) == r_cur;
            if constexpr (K == kBits) {
                R acc_all = acc[0];
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) acc_all |= shfl_xor(acc_all, d);
                R v = part[0];
                if (!first_in_cur) {
                    if (lane == 0) store_bits<T>(p, r_cur, acc_all & keep);
                } else if (lane == 0) {
                    v |= acc_all;
                }
#pragma unroll
                for (uint32_t d = 1; d < 64; d <<= 1) {
                    const R o = shfl_up(v, d);
                    const uint32_t ro = shfl_up(row, d);
                    if (lane >= d && ro == row) v |= o;
                }
                const uint32_t next_row = shfl(row, (int)min(lane + 1, 63u));
                if ((lane == 63 || next_row != row) && row != r_last) store_bits<T>(p, row, v & rkeep);
                acc[0] = row == r_last ? part[0] : (R)0;
            } else {
                V v[NV], tot[NV];
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    tot[k] = acc[k];
#pragma unroll
                    for (int d = LPT; d < 64; d <<= 1) tot[k] = KT::op(tot[k], shfl_xor(tot[k], d));
                    v[k] = part[k];
                }
                if (!first_in_cur) {
                    if (grp == 0) store_values<T, K>(p, r_cur, sub, keep, tot, straddles(r_cur), chunk_id, slot_of(r_cur));
                } else if (grp == 0) {
#pragma unroll
                    for (int k = 0; k < NV; ++k) v[k] = KT::op(tot[k], part[k]);
                }
                // segmented inclusive scan over groups, keyed by row
#pragma unroll
                for (int d = 1; d < TPW; d <<= 1) {
                    const uint32_t ro = shfl_up(row, d * LPT);
#pragma unroll
                    for (int k = 0; k < NV; ++k) {
                        const V o = shfl_up(v[k], d * LPT);
                        if (grp >= (uint32_t)d && ro == row) v[k] = KT::op(v[k], o);
                    }
                }
                const uint32_t next_row = shfl(row, (int)min(lane + LPT, 63u));
                if ((grp == TPW - 1 || next_row != row) && row != r_last)
                    store_values<T, K>(p, row, sub, rkeep, v, straddles(row), chunk_id, slot_of(row));
#pragma unroll
                for (int k = 0; k < NV; ++k) acc[k] = row == r_last ? part[k] : KT::id();
            }
            r_cur = r_last;
            r_end = p.trp[r_cur + 1];
            keep = keep_bits<T>(p.mask, p.flags, r_cur, p.n);
        }
        blk += BT;
        if constexpr (C::kStage) wave_lds_sync();  // the next block's LDS writes follow this block's reads
    }
    // flush the row the chunk ends in
    if constexpr (K == kBits) {
        fold_raw();
        R acc_all = acc[0];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) acc_all |= shfl_xor(acc_all, d);
        if (lane == 0) store_bits<T>(p, r_cur, acc_all & keep);
    } else {
        V tot[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            tot[k] = acc[k];
#pragma unroll
            for (int d = LPT; d < 64; d <<= 1) tot[k] = KT::op(tot[k], shfl_xor(tot[k], d));
        }
        if (grp == 0) store_values<T, K>(p, r_cur, sub, keep, tot, straddles(r_cur), chunk_id, slot_of(r_cur));
        if constexpr (K == kPlusF32) {
            if (lane == 0) {
                p.ws_rows[2 * chunk_id] = r_first;
                p.ws_rows[2 * chunk_id + 1] = r_cur;
            }
        }
    }
}

}  // namespace b2sr_core
