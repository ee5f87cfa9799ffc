// Batched multi-source BFS over many graphs at once.
//
// Many graphs share one vertex space (each graph's ids offset by a multiple
// of 64) and are grouped by tile width; each group is one block-diagonal B2SR
// matrix over the whole space.  Every vertex carries a 64-bit frontier word, so
// one level of 64-source BFS on every graph is one OR_U64 product per group
// (the Boolean semiring of Table V on 64 vectors at once) plus an element-wise
// update:
//     Y = OR over groups of (A_g (x) F);  new = Y & ~V;  V |= new;  F = new;
//     level[v][s] = current level for every new bit s of v.
// Three ways to run the levels:
//   * B2SR_BATCH_LEVELS:     one product launch per group and one update launch
//                            per level, with one flag read back per level;
//   * B2SR_BATCH_PERSISTENT: one kernel runs every level, separating the product
//                            and update phases with grid barriers.  The grid is
//                            sized from the occupancy API and launched
//                            cooperatively (the runtime refuses a grid that
//                            cannot be co-resident); the barrier itself is a
//                            generation counter whose waits are bounded: a wait
//                            that runs out raises an error flag, every block
//                            leaves the level loop, and the call reports an
//                            error instead of hanging;
//   * a plan: the persistent launch (with its initialisation) instantiated as a
//     hipGraph once and replayed.
// A work item (one chunk of one group) whose tile columns meet no frontier
// vertex is skipped after two reads: each call first records every item's
// column range, and each level's update marks, one bit per 1024 vertices,
// which ranges hold frontier vertices.  Late levels, when most graphs of the
// batch have finished, then skip those graphs' items instead of reading all
// their tile columns (every per-level product; in the persistent kernel the
// levels whose summary has under a quarter of its bits set, which it runs at
// a fixed stride rather than by claims).
#include <algorithm>
#include <new>
#include <utility>

#include "spmv_core.h"

using namespace b2sr_dev;
using namespace b2sr_core;

namespace {

constexpr uint32_t kMaxGroups = 8;
// Flag words: [0..7] as listed in BatchArgs; the barrier's arrival count and
// generation, and the persistent kernel's two work counters (one per level
// parity), 256 bytes apart, each on a line of its own.
constexpr uint32_t kBarrierCount = 64, kBarrierGen = 128, kClaim = 192, kFlagWords = 320;
// Words 8 and 9 (by level parity): the persistent kernel's count of summary
// bits its update set.
constexpr uint32_t kLiveBits = 8;
constexpr uint32_t kUnreached = 0xFFFFFFFFu;

struct Group {
    SpmvArgs p;      // product A_g (x) F -> Y (OR_U64 atomics), chunked as spmv_bin_full does
    uint32_t tile;
    uint32_t item0;  // first global work item (chunk) of the group
    uint32_t nchunks;
};

// Activity summary for skipping work items: bit k of a summary is set when a
// vertex in [k * 1024, (k + 1) * 1024) is in the frontier.
constexpr uint32_t kCoarseShift = 10;
// At most this many items have a recorded column range (beyond it no item is
// skipped): 8 MiB of workspace.
constexpr uint64_t kMaxRangeItems = 1u << 20;

struct BatchArgs {
    uint32_t n, ngroups, nitems, max_levels;
    Group g[kMaxGroups];
    uint64_t *F, *V, *Y;
    uint32_t *act;     // bit vector: vertices whose frontier word is non-zero
    // per item, the summary bits its tile columns fall in: [lo, hi] (nullptr:
    // no item is skipped); two summaries by level parity: the update of level l
    // writes coarse + (l & 1) * coarse_words (level 0: the seeds) and clears the
    // other, which the product of level l has just read
    uint32_t *ranges, *coarse;
    uint32_t coarse_words;
    uint32_t *levels;  // n x 64, vertex-major
    uint32_t *flags;   // [0], [1]: per-level parity flags; [2]: levels run;
                       // [5]: barrier timed out (the barrier's own words are further on);
                       // [6]: BFS finished (per-level kernels return at once)
    const uint32_t *seed_vertex, *seed_bit;
    uint32_t nseeds;
    uint32_t sticky_timeout;  // plans: initialisation leaves flags[5] for the status call to read
    unsigned tmask;  // tile widths present: bit 0 for 4, 1 for 8, 2 for 16, 3 for 32, 4 for 64
    // persistent kernel, optional: five wall-clock readings per (level, block)
    unsigned long long *stamps;
    uint32_t stamp_levels, stamp_blocks;
};

// Phase timestamps of the persistent kernel (when b.stamps is set): thread 0 of
// each block records the device wall clock at event ev of `level`.
__device__ __forceinline__ void stamp(const BatchArgs &b, uint32_t level, uint32_t ev)
{
    if (threadIdx.x == 0 && level <= b.stamp_levels && blockIdx.x < b.stamp_blocks)
        b.stamps[((size_t)(level - 1) * b.stamp_blocks + blockIdx.x) * 5 + ev] = wall_clock64();
}

__global__ void batch_init_kernel(BatchArgs b)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = tid; i < (uint64_t)b.n * 64; i += stride) b.levels[i] = kUnreached;
    for (uint64_t i = tid; i < b.n; i += stride) {
        b.F[i] = 0;
        b.V[i] = 0;
        b.Y[i] = 0;
    }
    for (uint64_t w = tid; w < (b.n + 31) / 32; w += stride) b.act[w] = 0;
    for (uint64_t w = tid; w < 2ull * b.coarse_words; w += stride) b.coarse[w] = 0;
    if (tid < 8 && !(tid == 5 && b.sticky_timeout)) b.flags[tid] = 0;
    if (tid == 8) b.flags[kBarrierCount] = 0;
    if (tid == 9) b.flags[kClaim] = 0;
    if (tid == 10) b.flags[kClaim + 64] = 0;
    if (tid == 11 || tid == 12) b.flags[kLiveBits + tid - 11] = 0;
}

// Seeds are distinct (vertex, bit) pairs, so the level writes never collide and
// the frontier words are combined with atomics.
__global__ void batch_seed_kernel(BatchArgs b)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b.nseeds;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = b.seed_vertex[i], s = b.seed_bit[i];
        if (v >= b.n || s >= 64) continue;  // out-of-range seeds are ignored
        atomicOr((unsigned long long *)b.F + v, 1ull << s);
        atomicOr((unsigned long long *)b.V + v, 1ull << s);
        atomicOr(b.act + (v >> 5), 1u << (v & 31));
        atomicOr(b.coarse + (v >> kCoarseShift) / 32, 1u << ((v >> kCoarseShift) & 31));  // level 0's summary
        b.levels[(size_t)v * 64 + s] = 0;
    }
}

// Every item's column range, as the summary bits [lo, hi] its tile columns
// fall in: one wave per item, a min and max over its tiles.
__global__ void batch_ranges_kernel(BatchArgs b)
{
    const uint32_t lane = lane_id();
    const uint32_t waves = gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint32_t item = blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE; item < b.nitems;
         item += waves) {
        uint32_t gi = 0;
        while (gi + 1 < b.ngroups && item >= b.g[gi + 1].item0) ++gi;
        const Group &g = b.g[gi];
        const uint32_t t0 = (item - g.item0) * g.p.chunk, t1 = min(t0 + g.p.chunk, g.p.ntiles);
        uint32_t lo = 0xFFFFFFFFu, hi = 0;
        // eight independent loads per lane in flight (a load per iteration left
        // the kernel waiting on each in turn)
        for (uint32_t t = t0 + lane; t < t1; t += 8 * B2SR_WAVE) {
            uint32_t j[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) j[u] = g.p.tci[min(t + u * B2SR_WAVE, t1 - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                lo = min(lo, j[u]);
                hi = max(hi, j[u]);
            }
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            lo = min(lo, shfl_xor(lo, d));
            hi = max(hi, shfl_xor(hi, d));
        }
        if (lane == 0) {
            const bool empty = lo > hi;  // no tiles: never live
            // (the last tile column's padding past n would reach one bit past the summary)
            const uint32_t last = (uint32_t)(((uint64_t)b.n - 1) >> kCoarseShift);
            b.ranges[2 * (size_t)item] = empty ? 1u : (uint32_t)(((uint64_t)lo * g.tile) >> kCoarseShift);
            b.ranges[2 * (size_t)item + 1] =
                empty ? 0u : min(last, (uint32_t)(((uint64_t)hi * g.tile + g.tile - 1) >> kCoarseShift));
        }
    }
}

// Whether work item `item` may meet the frontier summarised in `coarse` (wave-
// uniform): any summary bit set within the item's range.  The summary is read
// with agent-scope loads, past any stale cached copy of an earlier level's.
// Not inlined: inside the persistent kernel's claim loop the inlined check
// raised the kernel's registers from 76 to 84 VGPRs (6 -> 5 waves per SIMD);
// as a call it costs 80 and keeps 6.
__device__ __attribute__((noinline)) bool item_live(const uint32_t *ranges, const uint32_t *coarse, uint32_t item)
{
    if (!ranges) return true;
    const uint32_t lo = readfirstlane(ranges[2 * (size_t)item]), hi = readfirstlane(ranges[2 * (size_t)item + 1]);
    if (lo > hi) return false;
    bool any = false;
    for (uint32_t w = lo / 32 + lane_id(); w <= hi / 32; w += B2SR_WAVE) {
        uint32_t m = __hip_atomic_load(coarse + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w == lo / 32) m &= ~0u << (lo & 31);
        if (w == hi / 32) m &= ~0u >> (31 - (hi & 31));
        any |= m != 0;
    }
    return __any(any);
}


// Updates the vertices [base, base + 64), held one per lane (base a multiple
// of 64): takes each one's new frontier bits Y & ~V, marks them visited, clears
// Y for the next level's product, writes the two words of the active bit
// vector, and records the level of every new (vertex, source) pair.  The level
// rows are vertex-major (64 words per vertex), so the wave writes them one
// vertex at a time, lane s storing source s: one store per vertex covers its
// row's contiguous words, where a lane per vertex would scatter 4-byte stores
// over 64 rows.  Returns whether this lane's vertex has new bits.
__device__ __forceinline__ bool update_group(const BatchArgs &b, uint64_t base, uint32_t level)
{
    const uint32_t lane = lane_id();
    const uint64_t i = base + lane;
    uint64_t y = 0;
    if (i < b.n) {
        y = b.Y[i] & ~b.V[i];
        b.Y[i] = 0;
        b.F[i] = y;
        if (y) b.V[i] |= y;
    }
    const uint64_t m = __ballot(y != 0);
    const uint64_t w = base / 32 + lane;
    if (lane < 2 && w < (b.n + 31u) / 32u) b.act[w] = (uint32_t)(m >> (32 * lane));
    for (uint64_t todo = m; todo;) {
        const uint32_t k = (uint32_t)__builtin_ctzll(todo);
        todo &= todo - 1;
        const uint64_t yk = ((uint64_t)readlane((uint32_t)(y >> 32), (int)k) << 32) | readlane((uint32_t)y, (int)k);
        if ((yk >> lane) & 1) b.levels[(base + k) * 64 + lane] = level;
    }
    return y != 0;
}

// The update of `level` for wave `wave` of `nwaves`: runs of RUN groups of 64
// vertices in a grid-stride order, so that the wave sets a run's summary bit
// once (a wave per group put an atomic per group on the summary's few cache
// lines, and the update took 20 % longer; one contiguous stretch per wave was
// slower still at light levels).  The per-level kernel takes whole 1024-vertex
// runs (one summary bit each); the persistent kernel, whose update ends at a
// grid barrier, takes 256-vertex runs, which balance its waves better (256-graph
// batch: 20.05 -> 19.7 ms).  Returns the number of vertices with new bits; with
// BITS, *fresh_bits receives the number of summary bits this wave set first.
template <bool BITS = false, uint32_t RUN = (1u << kCoarseShift) / 64>
__device__ __forceinline__ uint32_t update_run(const BatchArgs &b, uint64_t wave, uint64_t nwaves, uint32_t level,
                                               uint32_t *fresh_bits = nullptr)
{
    static_assert(RUN >= 1 && ((1u << kCoarseShift) / 64) % RUN == 0, "a run lies inside one summary bit");
    constexpr uint32_t kRunGroups = RUN;
    const uint32_t groups = (uint32_t)(((uint64_t)b.n + 63) / 64);
    const uint32_t runs = (groups + kRunGroups - 1) / kRunGroups;
    uint32_t *const c = b.coarse + (level & 1) * b.coarse_words;
    uint32_t count = 0, fresh = 0;
    for (uint64_t r = wave; r < runs; r += nwaves) {
        const uint32_t g0 = (uint32_t)r * kRunGroups, g1 = min(g0 + kRunGroups, groups);
        uint32_t found = 0;
        for (uint32_t g = g0; g < g1; ++g) found += (uint32_t)__popcll(__ballot(update_group(b, (uint64_t)g * 64, level)));
        if (!found) continue;
        count += found;
        uint32_t f = 0;
        if (lane_id() == 0) {
            const uint32_t k = (uint32_t)((r * kRunGroups * 64) >> kCoarseShift);  // the run's summary bit
            const uint32_t bit = 1u << (k & 31);
            if constexpr (BITS) f = (atomicOr(c + k / 32, bit) & bit) ? 0u : 1u;
            else atomicOr(c + k / 32, bit);
        }
        if constexpr (BITS) fresh += readfirstlane(f);
    }
    if constexpr (BITS) *fresh_bits = fresh;
    return count;
}

// The update of `level` clears the summary the product of `level` read (the
// one the update of level + 1 writes).
__device__ __forceinline__ void clear_other_summary(const BatchArgs &b, uint32_t level, uint64_t tid, uint64_t stride)
{
    uint32_t *c = b.coarse + ((level + 1) & 1) * b.coarse_words;
    for (uint64_t w = tid; w < b.coarse_words; w += stride) c[w] = 0;
}

// Per-level kernels keep the level count and the finished flag on the device,
// so a fixed sequence of levels can be replayed from a hipGraph: once the BFS
// has finished, every later kernel returns at once.
__global__ void batch_update_kernel(BatchArgs b)
{
    if (b.flags[6]) return;
    const uint32_t level = b.flags[2] + 1;
    clear_other_summary(b, level, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    const bool any = update_run(b, (uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE, waves, level) != 0;
    if (__syncthreads_or(any) && threadIdx.x == 0) atomicOr(b.flags + (level & 1), 1u);
}

// One thread: count the level, finish when it found nothing (or the level
// bound is reached), and clear the next level's flag.
__global__ void batch_advance_kernel(uint32_t *flags, uint32_t max_levels)
{
    if (flags[6]) return;
    const uint32_t level = flags[2] + 1;
    flags[2] = level;
    if (!flags[level & 1] || level >= max_levels) flags[6] = 1;
    flags[(level + 1) & 1] = 0;
}

// One group's product for one level (per-level modes): one wave per chunk.
// The item skip's arguments for one group's per-level product.
struct Skip {
    const uint32_t *ranges, *coarse;
    uint32_t coarse_words, item0;
};

template <int T>
__global__ void __launch_bounds__(256) batch_product_kernel(SpmvArgs p, uint32_t nchunks, const uint32_t *flags, Skip sk)
{
    __shared__ __align__(16) uint64_t s_x[4 * kSliceBytes / sizeof(uint64_t)];
    if (flags[6]) return;
    const uint32_t wave = blockIdx.x * (blockDim.x / B2SR_WAVE) + readfirstlane(threadIdx.x / B2SR_WAVE);
    if (wave >= nchunks) return;
    // this level's product reads the summary of the last level's frontier
    if (!item_live(sk.ranges, sk.coarse + (flags[2] & 1) * sk.coarse_words, sk.item0 + wave)) return;
    spmv_chunk<T, kOr64, true>(p, wave, s_x + (threadIdx.x / B2SR_WAVE) * (kSliceBytes / sizeof(uint64_t)));
}

template <int T> __device__ __forceinline__ void run_chunk(const Group &g, uint32_t c, uint64_t *xs)
{
    spmv_chunk<T, kOr64, true>(g.p, c, xs);
}

#ifndef B2SR_BARRIER_FAST_POLLS
#define B2SR_BARRIER_FAST_POLLS 0
#endif
#ifndef B2SR_BARRIER_MAX_POLLS
#define B2SR_BARRIER_MAX_POLLS (1u << 19)  // about 2 s of long sleeps
#endif
#ifndef B2SR_BARRIER_SLEEP
#define B2SR_BARRIER_SLEEP 127
#endif

// Grid-wide barrier for the persistent kernel: block leaders count arrivals;
// the last one resets the count and advances the generation the others wait
// on.  The count and the generation sit on cache lines of their own, away
// from the flags every block reads.  Fences around it publish each block's
// writes device-wide.  A wait is bounded (B2SR_BARRIER_MAX_POLLS polls, each
// after a sleep: about two seconds): when it runs out, flags[5] is raised and
// the caller leaves its loop.  Returns, as read once per block after the barrier,
// bit 0 = flags[5] (timed out) and bit 1 = (*extra != 0) when extra is given.
__device__ __forceinline__ uint32_t grid_barrier(uint32_t *flags, const uint32_t *extra)
{
    __shared__ uint32_t s_state;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *count = flags + kBarrierCount, *gen = flags + kBarrierGen, *timed_out = flags + 5;
        const uint32_t g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        if (atomicAdd(count, 1u) + 1 == gridDim.x) {
            atomicExch(count, 0u);
            __threadfence();
            atomicAdd(gen, 1u);
        } else {
            uint32_t spins = 0;
            // relaxed polls: the fence after the wait is the acquire that pairs with
            // the last arriver's fence before it advanced the generation
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                // a long sleep between polls: a thousand waiting blocks polling
                // often crowd the arrivals on the counter's memory channel
                if (spins < B2SR_BARRIER_FAST_POLLS) __builtin_amdgcn_s_sleep(1);
                else __builtin_amdgcn_s_sleep(B2SR_BARRIER_SLEEP);
                if (++spins == B2SR_BARRIER_MAX_POLLS) {
                    atomicOr(timed_out, 1u);
                    break;
                }
            }
        }
        __threadfence();
        uint32_t st = __hip_atomic_load(timed_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
        if (extra && __hip_atomic_load(extra, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) st |= 2u;
        s_state = st;
    }
    __syncthreads();
    return s_state;
}

// Every level of every graph in one launch.  Waves take work items (chunks of
// every group) in a grid-stride loop; grid barriers separate the product from
// the update, and the update from the convergence test.  All threads read the
// same flags after the barrier, so they leave the level loop together; the loop
// is also bounded by max_levels and left at once if a barrier timed out.
// TMASK holds the tile widths present (bit 0: 4, 1: 8, 2: 16, 3: 32, 4: 64):
// only their product paths are compiled in, so the registers, and with them the
// waves per SIMD, are those of the widest path present rather than of all five.
#ifndef B2SR_PW_SMALL
#define B2SR_PW_SMALL 1  // waves per SIMD asked for masks without T = 8 and 16
#endif
#ifndef B2SR_PW_WIDE
#define B2SR_PW_WIDE 1   // the same for masks holding T = 8 or 16
#endif
#ifndef B2SR_PW_T4
#define B2SR_PW_T4 6     // the same for a batch all at T = 4: 80 VGPRs with a few 8-byte
                         // spills outside the product loop, 6 waves per SIMD instead of 5
#endif
constexpr int persistent_waves(unsigned tmask)
{
    return tmask == 1u ? B2SR_PW_T4 : (tmask & 6u) ? B2SR_PW_WIDE : B2SR_PW_SMALL;
}

#ifndef B2SR_PERSIST_MAX_PER_CU
#define B2SR_PERSIST_MAX_PER_CU 3
#endif
#ifndef B2SR_PERSIST_THREADS
#define B2SR_PERSIST_THREADS 512  // threads per block of the persistent kernel
#endif
constexpr unsigned kPersistThreads = B2SR_PERSIST_THREADS;
#ifndef B2SR_PERSIST_CLAIM
#define B2SR_PERSIST_CLAIM 1         // work items per claim after a large frontier
#endif
#ifndef B2SR_PERSIST_CLAIM_SPARSE
#define B2SR_PERSIST_CLAIM_SPARSE 2  // the same after a small one
#endif
#ifndef B2SR_PERSIST_STRIDE_BELOW
#define B2SR_PERSIST_STRIDE_BELOW 4  // a fixed stride when under 1/4 of the summary bits are set
#endif
#ifndef B2SR_PERSIST_SPARSE_FACTOR
#define B2SR_PERSIST_SPARSE_FACTOR 4  // a frontier is small below this many vertices per item
#endif

template <unsigned TMASK>
__global__ void __launch_bounds__(kPersistThreads, persistent_waves(TMASK)) batch_persistent_kernel(BatchArgs b)
{
    __shared__ __align__(16) uint64_t s_x[kPersistThreads / B2SR_WAVE * kSliceBytes / sizeof(uint64_t)];
    uint64_t *xs = s_x + (threadIdx.x / B2SR_WAVE) * (kSliceBytes / sizeof(uint64_t));
    const uint32_t wave = blockIdx.x * (blockDim.x / B2SR_WAVE) + readfirstlane(threadIdx.x / B2SR_WAVE);
    const uint32_t nwaves = gridDim.x * (blockDim.x / B2SR_WAVE);
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t level = 1; level <= b.max_levels; ++level) {
        if (b.stamps) stamp(b, level, 0);
        // Waves claim per_claim consecutive work items at a time from this
        // level's counter, so a wave that drew light chunks takes more of them
        // (a fixed stride left the heaviest wave 30 % behind the median).  The
        // counter only grows during the product phase, so every wave leaves
        // once it passes nitems; the claims a wave makes are also capped at
        // nitems.  The other parity's counter is reset in the update phase,
        // between the two barriers, when no wave claims from it.
        // A level whose items are light (most chunks inactive after a small
        // frontier: fewer than 4 frontier vertices per item; the seeds before
        // level 1) claims two items at a time, halving its claims on the one
        // counter (256-graph batch: 24.9 -> 22.7 ms; 4 items 23.3, 8 items 24.1).
        uint32_t *const counter = b.flags + kClaim + (level & 1) * 64;
        const uint32_t frontier = readfirstlane(level == 1 ? b.nseeds : b.flags[(level - 1) & 1]);
        // When under 1/4 of the summary bits are set (and every item has a
        // column range), waves take items at a fixed stride instead: per_claim
        // 0, and test each item against the summary.  Most items are then
        // dead, and a claim per item on the one counter (about 18 ns each,
        // serialised) set the level's time whatever the work.  Claimed items
        // are not tested: at those levels almost all are live.  Level 1's
        // summary (the seeds) is not counted: it claims.
        const uint32_t live_bits = level == 1 ? 0xFFFFFFFFu : readfirstlane(b.flags[kLiveBits + ((level - 1) & 1)]);
        const uint64_t summary_bits = ((uint64_t)b.n + (1u << kCoarseShift) - 1) >> kCoarseShift;
        const bool few = b.ranges && (uint64_t)live_bits * B2SR_PERSIST_STRIDE_BELOW < summary_bits;
        const bool small = (uint64_t)frontier < (uint64_t)b.nitems * B2SR_PERSIST_SPARSE_FACTOR;
        const uint32_t per_claim = few ? 0u : small ? B2SR_PERSIST_CLAIM_SPARSE : B2SR_PERSIST_CLAIM;
        uint32_t claims = 0, next = wave;
        for (;;) {
            uint32_t first = 0;
            if (per_claim) {
                if (lane_id() == 0) first = atomicAdd(counter, per_claim);
                first = readfirstlane(shfl(first, 0));
            } else {
                first = next;
                next += nwaves;
            }
            if (first >= b.nitems || ++claims > b.nitems) break;
            const uint32_t stop = min(b.nitems, first + max(per_claim, 1u));
            for (uint32_t item = first; item < stop; ++item) {
            // (this level reads the summary of the last level's frontier)
            if (!per_claim && !item_live(b.ranges, b.coarse + ((level - 1) & 1) * b.coarse_words, item)) continue;
            uint32_t gi = 0;
            while (gi + 1 < b.ngroups && item >= b.g[gi + 1].item0) ++gi;
            const Group &g = b.g[gi];
            const uint32_t c = item - g.item0;
            if constexpr ((TMASK & 1u) != 0) {
                if (g.tile == 4) { run_chunk<4>(g, c, xs); continue; }
            }
            if constexpr ((TMASK & 2u) != 0) {
                if (g.tile == 8) { run_chunk<8>(g, c, xs); continue; }
            }
            if constexpr ((TMASK & 4u) != 0) {
                if (g.tile == 16) { run_chunk<16>(g, c, xs); continue; }
            }
            if constexpr ((TMASK & 8u) != 0) {
                if (g.tile == 32) { run_chunk<32>(g, c, xs); continue; }
            }
            if constexpr ((TMASK & 16u) != 0) {
                if (g.tile == 64) run_chunk<64>(g, c, xs);
            }
            }
        }
        if (b.stamps) {  // uniform: every thread of the grid takes this branch or none
            __syncthreads();
            stamp(b, level, 1);
        }
        if (grid_barrier(b.flags, nullptr) & 1u) break;
        if (b.stamps) stamp(b, level, 2);
        // the level's count of new frontier vertices: the convergence test (zero
        // or not) and the next level's claim size
        __shared__ uint32_t s_count, s_fresh;
        if (threadIdx.x == 0) s_count = s_fresh = 0;
        __syncthreads();
        clear_other_summary(b, level, tid, (uint64_t)gridDim.x * blockDim.x);
        uint32_t fresh = 0;
        const uint32_t count = update_run<true, 4>(b, wave, nwaves, level, &fresh);
        if (lane_id() == 0 && count) atomicAdd(&s_count, count);
        if (lane_id() == 0 && fresh) atomicAdd(&s_fresh, fresh);
        __syncthreads();
        if (threadIdx.x == 0 && s_count) atomicAdd(b.flags + (level & 1), s_count);
        if (threadIdx.x == 0 && s_fresh) atomicAdd(b.flags + kLiveBits + (level & 1), s_fresh);
        if (tid == 0) {
            b.flags[(level + 1) & 1] = 0;
            b.flags[kLiveBits + ((level + 1) & 1)] = 0;
            b.flags[2] = level;
            b.flags[kClaim + ((level + 1) & 1) * 64] = 0;  // the next level's work counter
        }
        if (b.stamps) {
            __syncthreads();
            stamp(b, level, 3);
        }
        const uint32_t st = grid_barrier(b.flags, b.flags + (level & 1));
        if (b.stamps) stamp(b, level, 4);
        if ((st & 1u) || !(st & 2u)) break;
    }
}

struct Layout {
    uint64_t *F, *V, *Y;
    uint32_t *act, *flags, *coarse, *ranges;
    uint32_t coarse_words, range_items;
    size_t bytes;
};

Layout carve(uint32_t n, void *ws)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        char *p = ws ? (char *)ws + off : nullptr;
        off += bytes;
        return p;
    };
    L.F = (uint64_t *)take((size_t)n * 8);
    L.V = (uint64_t *)take((size_t)n * 8);
    L.Y = (uint64_t *)take((size_t)n * 8);
    L.act = (uint32_t *)take(((size_t)n + 31) / 32 * 4);
    L.flags = (uint32_t *)take(kFlagWords * 4);
    L.coarse_words = (uint32_t)((((uint64_t)n + (1u << kCoarseShift) - 1) >> kCoarseShift) + 31) / 32;
    L.coarse = (uint32_t *)take((size_t)L.coarse_words * 2 * 4);
    // no more items than tiles: at most 8 groups of (n / 4)^2 tiles
    const uint64_t ntr4 = ((uint64_t)n + 3) / 4;
    L.range_items = (uint32_t)(ntr4 > 362 ? kMaxRangeItems : std::min<uint64_t>(kMaxRangeItems, 8 * ntr4 * ntr4));
    L.ranges = (uint32_t *)take((size_t)L.range_items * 2 * 4);
    L.bytes = off;
    return L;
}

template <int T> uint32_t or64_chunk(const b2sr_matrix *A) { return chunk_tiles<T, kOr64>(A->ntiles, A->chunk_blocks); }

int make_args(uint32_t n, uint32_t ngroups, const b2sr_matrix *groups, uint32_t nseeds, const uint32_t *seed_vertex,
              const uint32_t *seed_bit, uint32_t *levels, void *ws, size_t ws_bytes, BatchArgs *out)
{
    if (n == 0 || ngroups == 0 || ngroups > kMaxGroups || !groups || !levels) return B2SR_EINVAL;
    if (n > 0xFFFFFF00u) return B2SR_ERANGE;
    if (nseeds > 0 && (!seed_vertex || !seed_bit)) return B2SR_EINVAL;
    const Layout L = carve(n, ws);
    if (!ws || ws_bytes < L.bytes) return B2SR_ENOSPC;
    BatchArgs b{};
    b.n = n;
    b.ngroups = ngroups;
    b.F = L.F;
    b.V = L.V;
    b.Y = L.Y;
    b.act = L.act;
    b.levels = levels;
    b.flags = L.flags;
    b.seed_vertex = seed_vertex;
    b.seed_bit = seed_bit;
    b.nseeds = nseeds;
    b.max_levels = n + 1;  // a BFS level adds at least one vertex, so n + 1 levels always suffice
    uint64_t items = 0;
    for (uint32_t k = 0; k < ngroups; ++k) {
        const b2sr_matrix *A = groups + k;
        if (int rc = b2sr::validate_matrix(A)) return rc;
        if (A->n != n) return B2SR_EINVAL;
        Group &g = b.g[k];
        g.p = SpmvArgs{};
        g.p.trp = A->tile_rowptr;
        g.p.tci = A->tile_colind;
        g.p.bits = A->bits;
        g.p.n = n;
        g.p.ntr = b2sr::n_tile_rows(n, A->tile);
        g.p.ntiles = A->ntiles;
        g.p.chunk = A->tile == 4 ? or64_chunk<4>(A) : A->tile == 8 ? or64_chunk<8>(A)
                  : A->tile == 16 ? or64_chunk<16>(A) : A->tile == 32 ? or64_chunk<32>(A) : or64_chunk<64>(A);
        g.p.x = L.F;
        g.p.xact = L.act;  // only non-zero frontier words take part
        g.p.y = L.Y;
        g.p.flags = B2SR_ACCUMULATE;
        g.tile = A->tile;
        b.tmask |= A->tile == 4 ? 1u : A->tile == 8 ? 2u : A->tile == 16 ? 4u : A->tile == 32 ? 8u : 16u;
        g.item0 = (uint32_t)items;
        g.nchunks = (uint32_t)(((uint64_t)A->ntiles + g.p.chunk - 1) / g.p.chunk);
        items += g.nchunks;
    }
    // the persistent kernel's work counter runs past nitems by at most one claim per wave
    if (items >= (1ull << 32) - (1ull << 24)) return B2SR_ERANGE;
    b.nitems = (uint32_t)items;
    b.coarse = L.coarse;
    b.coarse_words = L.coarse_words;
    b.ranges = items <= L.range_items ? L.ranges : nullptr;
    *out = b;
    return B2SR_OK;
}

unsigned vgrid(uint64_t n) { return b2sr::grid_for(n, 256, 8192); }

int launch_init(const BatchArgs &b, hipStream_t stream)
{
    batch_init_kernel<<<vgrid((uint64_t)b.n * 64), 256, 0, stream>>>(b);
    if (int rc = b2sr::check_launch("batch_init_kernel")) return rc;
    if (b.ranges && b.nitems) {
        batch_ranges_kernel<<<b2sr::grid_for(b.nitems, 4, 16384), 256, 0, stream>>>(b);
        if (int rc = b2sr::check_launch("batch_ranges_kernel")) return rc;
    }
    if (b.nseeds) {
        batch_seed_kernel<<<vgrid(b.nseeds), 256, 0, stream>>>(b);
        if (int rc = b2sr::check_launch("batch_seed_kernel")) return rc;
    }
    return B2SR_OK;
}

// The persistent kernel compiled for exactly the tile widths present.
template <unsigned... M> const void *persistent_pick(unsigned tmask, std::integer_sequence<unsigned, M...>)
{
    static const void *const table[] = {(const void *)batch_persistent_kernel<M + 1>...};
    return tmask >= 1 && tmask <= sizeof...(M) ? table[tmask - 1] : nullptr;
}

const void *persistent_kernel(unsigned tmask) { return persistent_pick(tmask, std::make_integer_sequence<unsigned, 31>{}); }

int persistent_grid(const void *kernel, unsigned *grid)
{
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (!kernel) return B2SR_EINVAL;
    if (int rc = b2sr::check(hipGetDevice(&dev), "hipGetDevice")) return rc;
    if (int rc = b2sr::check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties")) return rc;
    if (int rc = b2sr::check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kPersistThreads, 0),
                             "hipOccupancyMaxActiveBlocksPerMultiprocessor"))
        return rc;
    if (per_cu < 1 || !prop.cooperativeLaunch) return B2SR_ENOTSUP;
    // at most B2SR_PERSIST_MAX_PER_CU blocks per CU (the occupancy API's own
    // figure is lower for the wider tile widths): with work claimed from a
    // counter, 3 blocks of 512 threads measured best on the 256-graph batch
    if (per_cu > B2SR_PERSIST_MAX_PER_CU) per_cu = B2SR_PERSIST_MAX_PER_CU;
    *grid = (unsigned)per_cu * (unsigned)prop.multiProcessorCount;
    return B2SR_OK;
}

int launch_persistent(BatchArgs &b, hipStream_t stream)
{
    unsigned grid = 0;
    const void *kernel = persistent_kernel(b.tmask);
    if (int rc = persistent_grid(kernel, &grid)) return rc;
    void *args[] = {&b};
    return b2sr::check(hipLaunchCooperativeKernel(kernel, dim3(grid), dim3(kPersistThreads), args, 0, stream),
                       "hipLaunchCooperativeKernel(batch_persistent_kernel)");
}

// Reads the levels run and the barrier time-out flag after a persistent run.
int finish_persistent(const BatchArgs &b, uint32_t *iters, hipStream_t s)
{
    uint32_t h[6] = {0, 0, 0, 0, 0, 0};
    if (int rc = b2sr::read_words(b.flags, h, 6, s)) return rc;
    if (h[5]) {
        // clear the flag so that the next launch runs again, then report the time-out
        if (int rc = b2sr::fill_u32(b.flags + 5, 1, 0, s)) return rc;
        if (int rc = b2sr::check(hipStreamSynchronize(s), "hipStreamSynchronize")) return rc;
        b2sr::set_hip_error(hipErrorLaunchTimeOut, "batch_persistent_kernel grid barrier timed out");
        return B2SR_EHIP;
    }
    if (iters) *iters = h[2];
    return B2SR_OK;
}

// The per-level update's grid: up to 4096 blocks of 4 waves, so that a wave
// takes about one 1024-vertex run (1024 blocks: 17.9 ms for the 256-graph
// batch; 4096: 17.75).
unsigned update_grid(uint32_t n) { return b2sr::grid_for(n, 256, 4096); }

Skip skip_of(const BatchArgs &b, const Group &g) { return Skip{b.ranges, b.coarse, b.coarse_words, g.item0}; }

// One level: each group's product, the update, the advance (stream order).
int launch_level(const BatchArgs &b, hipStream_t stream)
{
    for (uint32_t k = 0; k < b.ngroups; ++k) {
        const Group &g = b.g[k];
        if (!g.nchunks) continue;
        const unsigned grid = b2sr::grid_for(g.nchunks, 4);
        const Skip sk = skip_of(b, g);
        switch (g.tile) {
        case 4: batch_product_kernel<4><<<grid, 256, 0, stream>>>(g.p, g.nchunks, b.flags, sk); break;
        case 8: batch_product_kernel<8><<<grid, 256, 0, stream>>>(g.p, g.nchunks, b.flags, sk); break;
        case 16: batch_product_kernel<16><<<grid, 256, 0, stream>>>(g.p, g.nchunks, b.flags, sk); break;
        case 64: batch_product_kernel<64><<<grid, 256, 0, stream>>>(g.p, g.nchunks, b.flags, sk); break;
        default: batch_product_kernel<32><<<grid, 256, 0, stream>>>(g.p, g.nchunks, b.flags, sk); break;
        }
        if (int rc = b2sr::check_launch("batch_product_kernel")) return rc;
    }
    batch_update_kernel<<<update_grid(b.n), 256, 0, stream>>>(b);
    if (int rc = b2sr::check_launch("batch_update_kernel")) return rc;
    batch_advance_kernel<<<1, 1, 0, stream>>>(b.flags, b.max_levels);
    return b2sr::check_launch("batch_advance_kernel");
}

// Levels per graph replay of a per-level plan.
constexpr uint32_t kPlanLevels = 32;

}  // namespace

struct b2sr_msbfs_plan_s {
    unsigned mode = 0;
    hipGraph_t first = nullptr, more = nullptr;  // first replay (init, seeds, levels); continuation (levels)
    hipGraphExec_t first_exec = nullptr, more_exec = nullptr;
    BatchArgs args{};
};

namespace {

int add_node(hipGraph_t g, hipGraphNode_t *last, const void *func, unsigned grid, unsigned block, void **params,
             hipGraphNode_t *out = nullptr)
{
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(func);
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(block);
    kp.kernelParams = params;
    hipGraphNode_t node = nullptr;
    const int rc = b2sr::check(hipGraphAddKernelNode(&node, g, *last ? last : nullptr, *last ? 1 : 0, &kp),
                               "hipGraphAddKernelNode");
    if (!rc) {
        *last = node;
        if (out) *out = node;
    }
    return rc;
}

// Appends `levels` levels (products, update, advance) after *last.
int add_levels(hipGraph_t g, hipGraphNode_t *last, BatchArgs &b, uint32_t levels)
{
    void *args_b[] = {&b};
    void *args_adv[] = {&b.flags, &b.max_levels};
    for (uint32_t l = 0; l < levels; ++l) {
        for (uint32_t k = 0; k < b.ngroups; ++k) {
            Group &gr = b.g[k];
            if (!gr.nchunks) continue;
            Skip sk = skip_of(b, gr);  // (a node copies its arguments)
            void *args_p[] = {&gr.p, &gr.nchunks, &b.flags, &sk};
            const void *f = gr.tile == 4    ? (const void *)batch_product_kernel<4>
                            : gr.tile == 8  ? (const void *)batch_product_kernel<8>
                            : gr.tile == 16 ? (const void *)batch_product_kernel<16>
                            : gr.tile == 32 ? (const void *)batch_product_kernel<32>
                                            : (const void *)batch_product_kernel<64>;
            if (int rc = add_node(g, last, f, b2sr::grid_for(gr.nchunks, 4), 256, args_p)) return rc;
        }
        if (int rc = add_node(g, last, (const void *)batch_update_kernel, update_grid(b.n), 256, args_b))
            return rc;
        if (int rc = add_node(g, last, (const void *)batch_advance_kernel, 1, 1, args_adv)) return rc;
    }
    return B2SR_OK;
}

}  // namespace

extern "C" {

size_t b2sr_msbfs_batch_workspace_bytes(uint32_t n) { return carve(n, nullptr).bytes; }

int b2sr_msbfs_batch(uint32_t n, uint32_t ngroups, const b2sr_matrix *groups, uint32_t nseeds,
                     const uint32_t *seed_vertex, const uint32_t *seed_bit, uint32_t *levels, unsigned mode, void *ws,
                     size_t ws_bytes, uint32_t *iters, hipStream_t stream)
{
    if (mode != B2SR_BATCH_LEVELS && mode != B2SR_BATCH_PERSISTENT) return B2SR_EINVAL;
    BatchArgs b;
    int rc = make_args(n, ngroups, groups, nseeds, seed_vertex, seed_bit, levels, ws, ws_bytes, &b);
    if (rc) return rc;
    if ((rc = launch_init(b, stream))) return rc;
    if (mode == B2SR_BATCH_PERSISTENT) {
        if ((rc = launch_persistent(b, stream))) return rc;
        return finish_persistent(b, iters, stream);
    }
    uint32_t h[8] = {0};
    do {
        if ((rc = launch_level(b, stream))) return rc;
        if ((rc = b2sr::read_words(b.flags, h, 8, stream))) return rc;
    } while (!h[6]);
    if (iters) *iters = h[2];
    return B2SR_OK;
}

int b2sr_msbfs_batch_timed(uint32_t n, uint32_t ngroups, const b2sr_matrix *groups, uint32_t nseeds,
                           const uint32_t *seed_vertex, const uint32_t *seed_bit, uint32_t *levels, void *ws,
                           size_t ws_bytes, uint64_t *stamps, uint32_t stamp_levels, uint32_t stamp_blocks,
                           uint32_t *grid_blocks, uint32_t *clock_khz, uint32_t *iters, hipStream_t stream)
{
    if (!stamps || !grid_blocks || !clock_khz || stamp_levels == 0 || stamp_blocks == 0) return B2SR_EINVAL;
    BatchArgs b;
    int rc = make_args(n, ngroups, groups, nseeds, seed_vertex, seed_bit, levels, ws, ws_bytes, &b);
    if (rc) return rc;
    unsigned grid = 0;
    if ((rc = persistent_grid(persistent_kernel(b.tmask), &grid))) return rc;
    int dev = 0, khz = 0;
    if ((rc = b2sr::check(hipGetDevice(&dev), "hipGetDevice"))) return rc;
    if ((rc = b2sr::check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "hipDeviceGetAttribute")))
        return rc;
    *grid_blocks = grid;
    *clock_khz = (uint32_t)khz;
    b.stamps = (unsigned long long *)stamps;
    b.stamp_levels = stamp_levels;
    b.stamp_blocks = stamp_blocks;
    if ((rc = b2sr::fill_u32((uint32_t *)stamps, (uint64_t)stamp_levels * stamp_blocks * 10, 0, stream))) return rc;
    if ((rc = launch_init(b, stream))) return rc;
    if ((rc = launch_persistent(b, stream))) return rc;
    return finish_persistent(b, iters, stream);
}

int b2sr_msbfs_batch_plan_create(uint32_t n, uint32_t ngroups, const b2sr_matrix *groups, uint32_t nseeds,
                                 const uint32_t *seed_vertex, const uint32_t *seed_bit, uint32_t *levels, unsigned mode,
                                 void *ws, size_t ws_bytes, b2sr_msbfs_plan *plan)
{
    if (!plan) return B2SR_EINVAL;
    *plan = nullptr;
    if (mode != B2SR_BATCH_LEVELS && mode != B2SR_BATCH_PERSISTENT) return B2SR_EINVAL;
    b2sr_msbfs_plan_s *P = new (std::nothrow) b2sr_msbfs_plan_s();
    if (!P) return B2SR_ENOSPC;
    P->mode = mode;
    int rc = make_args(n, ngroups, groups, nseeds, seed_vertex, seed_bit, levels, ws, ws_bytes, &P->args);
    BatchArgs &b = P->args;
    void *args_b[] = {&b};
    hipGraphNode_t last = nullptr;
    // the time-out flag outlives a replay: cleared here once, then only by the
    // status read that reports it
    b.sticky_timeout = 1;
    if (!rc) rc = b2sr::check(hipMemset(b.flags + 5, 0, sizeof(uint32_t)), "hipMemset(time-out flag)");
    if (!rc) rc = b2sr::check(hipGraphCreate(&P->first, 0), "hipGraphCreate");
    if (!rc) rc = add_node(P->first, &last, (const void *)batch_init_kernel, vgrid((uint64_t)n * 64), 256, args_b);
    if (!rc && b.ranges && b.nitems)
        rc = add_node(P->first, &last, (const void *)batch_ranges_kernel, b2sr::grid_for(b.nitems, 4, 16384), 256, args_b);
    if (!rc && nseeds) rc = add_node(P->first, &last, (const void *)batch_seed_kernel, vgrid(nseeds), 256, args_b);
    if (!rc && mode == B2SR_BATCH_PERSISTENT) {
        unsigned grid = 0;
        hipGraphNode_t run = nullptr;
        rc = persistent_grid(persistent_kernel(b.tmask), &grid);
        if (!rc) rc = add_node(P->first, &last, persistent_kernel(b.tmask), grid, kPersistThreads, args_b, &run);
        if (!rc) {
            // a cooperative node: the runtime checks at each replay that the grid
            // can be co-resident, as hipLaunchCooperativeKernel does
            hipKernelNodeAttrValue v{};
            v.cooperative = 1;
            if (hipGraphKernelNodeSetAttribute(run, hipKernelNodeAttributeCooperative, &v) != hipSuccess) {
                (void)hipGetLastError();
                rc = B2SR_ENOTSUP;
            }
        }
    } else if (!rc) {
        rc = add_levels(P->first, &last, b, kPlanLevels);
        hipGraphNode_t last2 = nullptr;
        if (!rc) rc = b2sr::check(hipGraphCreate(&P->more, 0), "hipGraphCreate");
        if (!rc) rc = add_levels(P->more, &last2, b, kPlanLevels);
        if (!rc) rc = b2sr::check(hipGraphInstantiate(&P->more_exec, P->more, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
    if (!rc) rc = b2sr::check(hipGraphInstantiate(&P->first_exec, P->first, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (rc) {
        b2sr_msbfs_batch_plan_destroy(P);
        return rc;
    }
    *plan = P;
    return B2SR_OK;
}

int b2sr_msbfs_batch_plan_launch(b2sr_msbfs_plan plan, uint32_t *iters, hipStream_t stream)
{
    if (!plan || !plan->first_exec) return B2SR_EINVAL;
    int rc = b2sr::check(hipGraphLaunch(plan->first_exec, stream), "hipGraphLaunch");
    if (rc) return rc;
    if (plan->mode == B2SR_BATCH_PERSISTENT) return iters ? finish_persistent(plan->args, iters, stream) : B2SR_OK;
    // per-level plan: replay the continuation until the device says the BFS finished
    uint32_t h[8] = {0};
    for (;;) {
        if ((rc = b2sr::read_words(plan->args.flags, h, 8, stream))) return rc;
        if (h[6]) break;
        if ((rc = b2sr::check(hipGraphLaunch(plan->more_exec, stream), "hipGraphLaunch"))) return rc;
    }
    if (iters) *iters = h[2];
    return B2SR_OK;
}

int b2sr_msbfs_batch_plan_status(b2sr_msbfs_plan plan, uint32_t *iters, hipStream_t stream)
{
    if (!plan || !plan->first_exec) return B2SR_EINVAL;
    return finish_persistent(plan->args, iters, stream);
}

int b2sr_msbfs_batch_plan_destroy(b2sr_msbfs_plan plan)
{
    if (!plan) return B2SR_OK;
    int rc = B2SR_OK;
    auto keep = [&](int r) { if (!rc) rc = r; };
    if (plan->first_exec) keep(b2sr::check(hipGraphExecDestroy(plan->first_exec), "hipGraphExecDestroy"));
    if (plan->more_exec) keep(b2sr::check(hipGraphExecDestroy(plan->more_exec), "hipGraphExecDestroy"));
    if (plan->first) keep(b2sr::check(hipGraphDestroy(plan->first), "hipGraphDestroy"));
    if (plan->more) keep(b2sr::check(hipGraphDestroy(plan->more), "hipGraphDestroy"));
    delete plan;
    return rc;
}

}  // extern "C"
