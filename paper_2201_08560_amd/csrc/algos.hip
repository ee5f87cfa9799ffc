// Graph algorithms on the B2SR products (Sec. V): BFS, multi-source BFS,
// SSSP, connected components and PageRank.  Each driver launches the product
// kernels plus a small element-wise update kernel per iteration.
//
// BFS, multi-source BFS, SSSP and CC keep their convergence on the device: a
// state word says how the next iteration runs (a dense or a sparse-frontier
// product) or that the algorithm has finished, and every kernel of an
// iteration returns at once when the state does not select it.  The host
// enqueues iterations in growing batches (2, 4, 8, then 16) and reads the
// state once per batch, instead of once per iteration; iterations enqueued
// after the end cost one empty launch each.  Per-iteration counts alternate
// between two words so the kernel that advances the state can clear the next
// one.
#include <algorithm>
#include <utility>

#include "common.h"

using namespace b2sr_dev;

namespace b2sr {
int column_counts(const b2sr_matrix *A, uint32_t *colsum, hipStream_t s);
size_t lgc_workspace_bytes(const b2sr_matrix *A);
// The products with every kernel gated on *gate == gate_val (spmv.hip); the
// full product takes B2SR_MIN_PLUS_U32, B2SR_OR_U64 and B2SR_MAX_TIMES_U64.
int spmv_bits_gated(const b2sr_matrix *A, const uint32_t *x, const uint32_t *mask, unsigned flags, void *y,
                    const uint32_t *gate, uint32_t gate_val, hipStream_t stream);
int spmv_full_gated(const b2sr_matrix *A, int semiring, const void *x, const uint32_t *x_active, unsigned flags,
                    double alpha, void *y, const uint32_t *gate, uint32_t gate_val, hipStream_t stream);
}

namespace {

constexpr uint32_t kUnreached = 0xFFFFFFFFu;

// Carves aligned pieces out of a caller workspace (or just sizes them when
// base is null).
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

// The drivers' flag words: two 64-bit accumulators, one per iteration
// parity, each the count of finished update blocks (high half) and the
// iteration's count of found units (low half); then the next iteration's run
// state, the iterations run, and the last two iterations' counts.
constexpr uint32_t kRunDense = 0, kRunSparse = 1, kDone = 2;
constexpr uint32_t kState = 4, kIters = 5, kLast = 6, kPrev = 7, kFlagWords = 10;
// MIS and colouring also keep: whether the next round starts a colour pass,
// and the current colour.
constexpr uint32_t kPass = 8, kColor = 9;

// Ends a gated update kernel (every thread calls it; found_wave is this wave's
// count, read from lane 0).  Each block adds its count and itself to the
// iteration's accumulator in one 64-bit atomic, so the block that sees every
// other block counted is the last and holds the total, with no fence between
// the two.  It then advances the state: none found ends the run (as does the
// iteration bound), otherwise the next iteration runs the sparse-frontier
// product when fewer than sparse_below were found; and it clears the
// accumulator for iteration it + 2.
// Returns true in thread 0 of the last block only.
__device__ bool finish_iteration(uint32_t *flags, uint32_t it, uint32_t found_wave, uint32_t sparse_below,
                                 uint32_t max_iters)
{
    __shared__ uint32_t s_found;
    if (threadIdx.x == 0) s_found = 0;
    __syncthreads();
    if (lane_id() == 0 && found_wave) atomicAdd(&s_found, found_wave);
    __syncthreads();
    if (threadIdx.x != 0) return false;
    unsigned long long *acc = (unsigned long long *)flags + (it & 1);
    const unsigned long long old = atomicAdd(acc, (1ull << 32) | s_found);
    if ((uint32_t)(old >> 32) != gridDim.x - 1) return false;
    const uint32_t found = (uint32_t)old + s_found;
    atomicExch(acc, 0ull);
    atomicExch(flags + kPrev, atomicExch(flags + kLast, found));
    atomicExch(flags + kIters, it);
    atomicExch(flags + kState, (found == 0 || it >= max_iters) ? kDone : (found < sparse_below ? kRunSparse : kRunDense));
    return true;
}

// Runs `one(iteration index)` in batches, reading the device state after each
// batch (which synchronises the stream), until the device reports the run
// finished (the last block of an update ends it by max_iters at the latest).
// Batches double from 2 up to 16 iterations while the counts grow or hold,
// and fall back to 2 once they shrink: a shrinking frontier is near its end,
// where every iteration enqueued after the last costs empty launches.
template <class F> int run_gated(const uint32_t *flags, uint32_t max_iters, uint32_t *iters, hipStream_t s, F one)
{
    uint32_t enq = 0, batch = 2;
    uint32_t h[4] = {kRunDense, 0, 0, 0};  // state, iterations run, last and previous counts
    for (;;) {
        for (uint32_t k = 0; k < batch; ++k)
            if (int rc = one(++enq)) return rc;
        if (int rc = b2sr::read_words(flags + kState, h, 4, s)) return rc;
        if (h[0] == kDone) break;
        if (enq > max_iters + 1) return B2SR_EHIP;  // cannot happen: the run ends by max_iters
        batch = h[2] < h[3] ? 2u : std::min<uint32_t>(batch * 2, 16);
    }
    if (iters) *iters = h[1];
    return B2SR_OK;
}

int read_flag(const uint32_t *d_flag, uint32_t *h, hipStream_t s) { return b2sr::read_words(d_flag, h, 1, s); }

// ---------------------------------------------------------------- BFS
__global__ void bfs_init_kernel(uint32_t n, uint32_t src, uint32_t *levels, uint32_t *frontier, uint32_t *visited,
                                uint32_t *next, uint32_t *flags, uint32_t first_state)
{
    const uint32_t nw = (n + 31) / 32;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        levels[i] = i == src ? 0u : kUnreached;
        if (i < nw) {
            const uint32_t w = (i == src / 32) ? (1u << (src % 32)) : 0u;
            frontier[i] = w;
            visited[i] = w;
            next[i] = 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < kFlagWords) flags[threadIdx.x] = threadIdx.x == kState ? first_state : 0u;
}

// Newly reached vertices (next is already masked by NOT visited) get this
// level, join the visited set and form the next frontier; next is cleared for
// the next product, which accumulates into it; the level's count of found
// vertices goes to its parity's word.
__global__ void bfs_update_gated_kernel(uint32_t nw, uint32_t *next, uint32_t *frontier, uint32_t *visited,
                                        uint32_t *levels, uint32_t *flags, uint32_t sparse_below, uint32_t max_iters)
{
    if (flags[kState] == kDone) return;
    const uint32_t level = flags[kIters] + 1;
    uint32_t found = 0;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t nb = next[w];
        frontier[w] = nb;
        if (!nb) continue;
        next[w] = 0;
        found += __popc(nb);
        visited[w] |= nb;
        while (nb) {
            const uint32_t b = __builtin_ctz(nb);
            nb &= nb - 1;
            levels[w * 32 + b] = level;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) found += shfl_xor(found, d);
    finish_iteration(flags, level, found, sparse_below, max_iters);
}

// ---------------------------------------------------------------- multi-source BFS
__global__ void msbfs_init_kernel(uint32_t n, uint32_t nsrc, const uint32_t *srcs, uint64_t *F, uint64_t *V,
                                  uint32_t *levels, uint32_t *flags)
{
    const uint64_t total = (uint64_t)nsrc * n;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x)
        levels[i] = kUnreached;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        F[i] = 0;
        V[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x < kFlagWords) flags[threadIdx.x] = 0;  // state: dense
}

__global__ void msbfs_seed_kernel(uint32_t n, uint32_t nsrc, const uint32_t *srcs, uint64_t *F, uint64_t *V,
                                  uint32_t *levels, uint32_t *act)
{
    // one thread seeds every source so repeated vertices (rejected on the host) cannot race
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (uint32_t s = 0; s < nsrc; ++s) {
            F[srcs[s]] |= 1ull << s;
            V[srcs[s]] |= 1ull << s;
            act[srcs[s] >> 5] |= 1u << (srcs[s] & 31);
            levels[(size_t)s * n + srcs[s]] = 0;
        }
}

// Writes the bit vector of predicate p for vertices [base, base + 64) held one
// per lane (base is a multiple of 64): two words, the second only if it exists.
__device__ __forceinline__ void store_pred_bits(uint32_t *bits, uint64_t base, uint32_t n, bool p)
{
    const uint64_t m = __ballot(p);
    const uint64_t w = base / 32 + lane_id();
    if (lane_id() < 2 && w < (n + 31u) / 32u) bits[w] = (uint32_t)(m >> (32 * lane_id()));
}

// ---------------------------------------------------------------- eccentricity
// 64 sources at a time as bits of one frontier word per vertex, as the
// multi-source BFS does, but no levels are stored per vertex: each level ORs
// the sources that reached new vertices into one word for that level, and a
// source's eccentricity is the last level whose word holds its bit.
__global__ void ecc_init_kernel(uint32_t n, uint64_t *F, uint64_t *V, uint32_t *act, uint64_t *hist, uint32_t *flags)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = tid; i < n; i += stride) {
        F[i] = 0;
        V[i] = 0;
    }
    for (uint64_t w = tid; w < (n + 31) / 32; w += stride) act[w] = 0;
    if (tid < 2) hist[1 + tid] = 0;  // level 1's word (later levels are cleared as the run goes)
    if (tid < kFlagWords) flags[tid] = 0;  // state: dense
}

__global__ void ecc_seed_kernel(uint32_t nsrc, const uint32_t *srcs, uint64_t *F, uint64_t *V, uint32_t *act)
{
    // one thread seeds every source, so repeated vertices cannot race
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (uint32_t s = 0; s < nsrc; ++s) {
            F[srcs[s]] |= 1ull << s;
            V[srcs[s]] |= 1ull << s;
            act[srcs[s] >> 5] |= 1u << (srcs[s] & 31);
        }
}

// The gated form: the level comes from the device state, every wave ORs the
// sources that reached new vertices into hist[level] (one 64-bit word per
// level), and the last block clears hist[level + 1] for the next level.  After
// the run, a source's eccentricity is the last level whose word holds its bit.
__global__ void ecc_update_gated_kernel(uint32_t n, const uint64_t *Y, uint64_t *F, uint64_t *V, uint32_t *act,
                                        uint64_t *hist, uint32_t *flags, uint32_t max_iters)
{
    if (flags[kState] == kDone) return;
    const uint32_t level = flags[kIters] + 1;
    uint64_t seen = 0;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + lane_id();
        uint64_t y = 0;
        if (i < n) {
            y = Y[i] & ~V[i];
            F[i] = y;
            if (y) V[i] |= y;
        }
        seen |= y;
        store_pred_bits(act, base, n, y != 0);
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) seen |= shfl_xor(seen, d);
    if (lane_id() == 0 && seen) atomicOr((unsigned long long *)hist + level, (unsigned long long)seen);
    if (finish_iteration(flags, level, seen ? 1u : 0u, 0, max_iters)) atomicExch((unsigned long long *)hist + level + 1, 0ull);
}

// Eccentricities of the k sources of a batch from the per-level words: lane s
// takes the last level 1 .. flags[kIters] whose word holds bit s (0 if none).
__global__ void ecc_final_kernel(const uint64_t *hist, const uint32_t *flags, uint32_t k, uint32_t *ecc)
{
    const uint32_t s = threadIdx.x, levels = flags[kIters];
    uint32_t e = 0;
    for (uint32_t l = 1; l <= levels; ++l)
        if ((hist[l] >> s) & 1u) e = l;
    if (s < k) ecc[s] = e;
}

// New frontier words: Y & ~V.  Marks them visited, records levels, and writes
// the active bit vector (frontier word non-zero) for the next product.  Each
// wave walks 64 consecutive vertices at a time, so the ballot forms whole words.
__global__ void msbfs_update_kernel(uint32_t n, const uint64_t *Y, uint64_t *F, uint64_t *V, uint32_t *levels,
                                    uint32_t *act, uint32_t *flags, uint32_t max_iters)
{
    if (flags[kState] == kDone) return;
    const uint32_t level = flags[kIters] + 1;
    bool any = false;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + lane_id();
        uint64_t y = 0;
        if (i < n) {
            y = Y[i] & ~V[i];
            F[i] = y;
            if (y) {
                any = true;
                V[i] |= y;
            }
        }
        store_pred_bits(act, base, n, y != 0);
        // levels are source-major: one source at a time, the lanes' consecutive
        // vertices make one store into that source's row
        uint64_t srcs = y;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) srcs |= shfl_xor(srcs, d);
        while (srcs) {
            const uint32_t s = __builtin_ctzll(srcs);
            srcs &= srcs - 1;
            if ((y >> s) & 1) levels[(size_t)s * n + i] = level;
        }
    }
    finish_iteration(flags, level, __any(any) ? 1u : 0u, 0, max_iters);
}

// ---------------------------------------------------------------- SSSP / CC
__global__ void sssp_init_kernel(uint32_t n, uint32_t src, uint32_t *d, uint32_t *act, uint32_t *flags)
{
    const uint32_t nw = (n + 31) / 32;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        d[i] = i == src ? 0u : kUnreached;
        if (i < nw) act[i] = i == src / 32 ? 1u << (src % 32) : 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x < kFlagWords) flags[threadIdx.x] = 0;  // state: dense
}

// Entries that changed between two iterates: the active bit vector of the next
// product and the iteration's count (of blocks with a change).
__global__ void changed_kernel(uint32_t n, const uint32_t *a, const uint32_t *b, uint32_t *act, uint32_t *flags,
                               uint32_t max_iters)
{
    if (flags[kState] == kDone) return;
    const uint32_t it = flags[kIters] + 1;
    bool diff = false;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + lane_id();
        const bool d = i < n && a[i] != b[i];
        diff |= d;
        store_pred_bits(act, base, n, d);
    }
    finish_iteration(flags, it, __any(diff) ? 1u : 0u, 0, max_iters);
}

__global__ void iota_kernel(uint32_t n, uint32_t *x, uint32_t *flags)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        x[i] = (uint32_t)i;
    if (blockIdx.x == 0 && threadIdx.x < kFlagWords) flags[threadIdx.x] = 0;  // state: dense
}

__global__ void copy_u32_kernel(uint32_t n, const uint32_t *a, uint32_t *b)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// ---------------------------------------------------------------- PageRank
__global__ void ones_bits_kernel(uint32_t n, uint32_t *bits)
{
    const uint32_t nw = (n + 31) / 32;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t hi = (uint32_t)min<uint64_t>(32, n - w * 32);
        bits[w] = hi == 32 ? 0xFFFFFFFFu : ((1u << hi) - 1u);
    }
}

__global__ void pr_init_kernel(uint32_t n, const uint32_t *deg, float *inv, float *r)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        inv[i] = deg[i] ? 1.0f / (float)deg[i] : 0.0f;
        r[i] = 1.0f / (float)n;
    }
}

__global__ void pr_scale_kernel(uint32_t n, const float *r, const float *inv, float *z)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        z[i] = r[i] * inv[i];
}

// ---------------------------------------------------------------- MIS / colouring
// Candidates carry their key in X (0 = not a candidate).  Each wave walks 64
// consecutive vertices at a time so ballots form whole bit-vector words.

// X = key for the vertices still to place (uncoloured when colors is given).
__global__ void mis_start_kernel(uint32_t n, const uint64_t *key, const uint32_t *colors, uint64_t *X, uint32_t *act,
                                 uint32_t *flag_now, uint32_t *flag_next)
{
    bool any = false;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + lane_id();
        uint64_t x = 0;
        if (i < n) {
            x = (!colors || colors[i] == kUnreached) ? key[i] : 0ull;
            X[i] = x;
        }
        any |= x != 0;
        store_pred_bits(act, base, n, x != 0);
    }
    if (__syncthreads_or(any) && threadIdx.x == 0) atomicOr(flag_now, 1u);
    if (blockIdx.x == 0 && threadIdx.x == 0) *flag_next = 0;
}

// A candidate joins when its key is at least the largest candidate key among
// its neighbours (Y = A max-times X); joined vertices and their neighbours
// (nb = A OR joined) stop being candidates.
// The gated rounds.  A round is: (colouring, when the last round ended a
// pass) a new pass's candidates; Y = A max-times X; the joins; the joined
// vertices' neighbours; the removals.  The removal kernel's last block sets
// the next round's state from two per-block tallies packed into the one
// 64-bit accumulator: blocks that still hold candidates (low 16 bits) and,
// when colouring, blocks that hold uncoloured vertices with a key (high 16;
// at most 1024 blocks, so neither field overflows).  No candidates left ends
// the pass: colouring starts the next one while vertices remain uncoloured.
__device__ bool finish_round(uint32_t *flags, uint32_t it, bool cand, bool uncol, bool colouring, uint32_t max_iters)
{
    __shared__ uint32_t s_found;
    if (threadIdx.x == 0) s_found = 0;
    __syncthreads();
    if (lane_id() == 0 && (cand || uncol)) atomicOr(&s_found, (cand ? 1u : 0u) | (uncol ? 0x10000u : 0u));
    __syncthreads();
    if (threadIdx.x != 0) return false;
    unsigned long long *acc = (unsigned long long *)flags + (it & 1);
    const unsigned long long old = atomicAdd(acc, (1ull << 32) | s_found);
    if ((uint32_t)(old >> 32) != gridDim.x - 1) return false;
    const uint32_t found = (uint32_t)old + s_found;
    atomicExch(acc, 0ull);
    const uint32_t cand_blocks = found & 0xFFFFu, uncol_blocks = found >> 16;
    const bool next_pass = cand_blocks == 0 && colouring && uncol_blocks != 0;
    atomicExch(flags + kPrev, atomicExch(flags + kLast, cand_blocks));
    atomicExch(flags + kIters, it);
    atomicExch(flags + kPass, next_pass ? 1u : 0u);
    if (next_pass) atomicAdd(flags + kColor, 1u);
    atomicExch(flags + kState, ((cand_blocks == 0 && !next_pass) || it >= max_iters) ? kDone : kRunDense);
    return true;
}

__global__ void mis_start_gated_kernel(uint32_t n, const uint64_t *key, const uint32_t *colors, uint64_t *X,
                                       uint32_t *act, const uint32_t *flags)
{
    if (flags[kState] != kRunDense || !flags[kPass]) return;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + lane_id();
        uint64_t x = 0;
        if (i < n) {
            x = colors[i] == kUnreached ? key[i] : 0ull;
            X[i] = x;
        }
        store_pred_bits(act, base, n, x != 0);
    }
}

__global__ void mis_join_gated_kernel(uint32_t n, const uint64_t *X, const uint64_t *Y, uint32_t *joined,
                                      uint32_t *mis_bits, uint32_t *colors, const uint32_t *flags)
{
    if (flags[kState] != kRunDense) return;
    const uint32_t color = flags[kColor];
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + lane_id();
        bool j = false;
        if (i < n) {
            const uint64_t x = X[i];
            j = x != 0 && x >= Y[i];
            if (j && colors) colors[i] = color;
        }
        const uint64_t m = __ballot(j);
        const uint64_t w = base / 32 + lane_id();
        if (lane_id() < 2 && w < (n + 31u) / 32u) {
            const uint32_t word = (uint32_t)(m >> (32 * lane_id()));
            joined[w] = word;
            if (mis_bits) mis_bits[w] |= word;  // this wave owns the word
        }
    }
}

__global__ void mis_remove_gated_kernel(uint32_t n, uint64_t *X, const uint32_t *joined, const uint32_t *nb,
                                        uint32_t *act, const uint64_t *key, const uint32_t *colors, uint32_t *flags,
                                        uint32_t max_iters)
{
    if (flags[kState] != kRunDense) return;
    const uint32_t it = flags[kIters] + 1;
    bool cand = false, uncol = false;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + lane_id();
        uint64_t x = 0;
        if (i < n) {
            x = X[i];
            if (x && (((joined[i >> 5] | nb[i >> 5]) >> (i & 31)) & 1u)) {
                x = 0;
                X[i] = 0;
            }
            if (colors) uncol |= colors[i] == kUnreached && key[i] != 0;
        }
        cand |= x != 0;
        store_pred_bits(act, base, n, x != 0);
    }
    finish_round(flags, it, __any(cand), __any(uncol), colors != nullptr, max_iters);
}

unsigned vgrid(uint64_t n) { return b2sr::grid_for(n, 256, 8192); }
// Grids of the kernels that raise a convergence flag: at most 1024 blocks, so
// at most 1024 atomics on the flag word.
unsigned fgrid(uint64_t n) { return b2sr::grid_for(n, 256, 1024); }

struct Layout {
    // BFS
    uint32_t *frontier = nullptr, *visited = nullptr, *next = nullptr;
    // MSBFS
    uint64_t *F = nullptr, *V = nullptr, *Y = nullptr;
    uint32_t *srcs = nullptr;
    // SSSP / CC / PR
    float *f0 = nullptr, *f1 = nullptr, *f2 = nullptr;
    uint32_t *u0 = nullptr, *u1 = nullptr, *ones = nullptr, *act = nullptr;
    uint64_t *alive = nullptr;
    void *spmv_ws = nullptr;
    size_t spmv_ws_bytes = 0;
    uint32_t *flags = nullptr;
    size_t bytes = 0;
};

Layout carve(const b2sr_matrix *A, int algo, void *ws)
{
    Carver c{(char *)ws};
    Layout L;
    const size_t n = A->n, nw = b2sr::n_words(A->n);
    switch (algo) {
    case B2SR_ALGO_BFS:
        L.frontier = c.take<uint32_t>(nw * 4);
        L.visited = c.take<uint32_t>(nw * 4);
        L.next = c.take<uint32_t>(nw * 4);
        break;
    case B2SR_ALGO_MSBFS:
        L.F = c.take<uint64_t>(n * 8);
        L.V = c.take<uint64_t>(n * 8);
        L.Y = c.take<uint64_t>(n * 8);
        L.srcs = c.take<uint32_t>(64 * 4);
        L.act = c.take<uint32_t>(nw * 4);
        break;
    case B2SR_ALGO_SSSP:
        L.u0 = c.take<uint32_t>(n * 4);
        L.u1 = c.take<uint32_t>(n * 4);
        L.act = c.take<uint32_t>(nw * 4);
        break;
    case B2SR_ALGO_CC:
        L.u0 = c.take<uint32_t>(n * 4);
        L.act = c.take<uint32_t>(nw * 4);
        break;
    case B2SR_ALGO_ECC:
        L.F = c.take<uint64_t>(n * 8);
        L.V = c.take<uint64_t>(n * 8);
        L.Y = c.take<uint64_t>(n * 8);
        L.srcs = c.take<uint32_t>(64 * 4);
        L.act = c.take<uint32_t>(nw * 4);
        L.alive = c.take<uint64_t>(((size_t)n + 3) * 8);  // one word per level 0 .. n + 2
        L.u0 = c.take<uint32_t>(64 * 4);                   // the batch's eccentricities
        break;
    case B2SR_ALGO_MIS:
    case B2SR_ALGO_COLOR:
        L.F = c.take<uint64_t>(n * 8);  // candidate keys X
        L.Y = c.take<uint64_t>(n * 8);  // max-times product
        L.frontier = c.take<uint32_t>(nw * 4);  // joined this round
        L.next = c.take<uint32_t>(nw * 4);      // neighbours of the joined
        L.act = c.take<uint32_t>(nw * 4);       // candidates
        break;
    case B2SR_ALGO_PAGERANK:
        L.f0 = c.take<float>(n * 4);  // z = r / deg
        L.f1 = c.take<float>(n * 4);  // 1 / deg
        L.f2 = c.take<float>(n * 4);  // second rank buffer
        // degrees; column counts (directed graphs) cover every column of the last tile
        L.u0 = c.take<uint32_t>((size_t)b2sr::n_tile_rows(A->n, A->tile) * A->tile * 4);
        L.ones = c.take<uint32_t>(nw * 4);
        L.spmv_ws_bytes = spmv_bin_full_workspace_bytes(A, B2SR_PLUS_TIMES_F32);
        L.spmv_ws = c.take<char>(L.spmv_ws_bytes);
        break;
    default: break;
    }
    L.flags = c.take<uint32_t>(kFlagWords * 4);
    L.bytes = c.off;
    return L;
}

int check_algo_args(const b2sr_matrix *A, int algo, void *ws, size_t ws_bytes, Layout *L)
{
    int rc = b2sr::validate_matrix(A);
    if (rc) return rc;
    if (!ws) return B2SR_ENOSPC;
    *L = carve(A, algo, ws);
    return ws_bytes < L->bytes ? B2SR_ENOSPC : B2SR_OK;
}

}  // namespace

extern "C" {

size_t b2sr_algo_workspace_bytes(const b2sr_matrix *A, int algo)
{
    if (!A || !b2sr::valid_tile(A->tile)) return 0;
    if (algo == B2SR_ALGO_LGC) return b2sr::lgc_workspace_bytes(A);
    if (algo < B2SR_ALGO_BFS || algo > B2SR_ALGO_ECC) return 0;
    return carve(A, algo, nullptr).bytes;
}

int b2sr_bfs(const b2sr_matrix *A, uint32_t src, uint32_t *levels, void *ws, size_t ws_bytes, uint32_t *iters,
             hipStream_t stream)
{
    Layout L;
    int rc = check_algo_args(A, B2SR_ALGO_BFS, ws, ws_bytes, &L);
    if (rc) return rc;
    if (!levels || src >= A->n) return B2SR_EINVAL;
    const uint32_t n = A->n, nw = b2sr::n_words(n), max_iters = n + 1;
    // A frontier with fewer vertices than there are tile columns leaves most x
    // segments empty: then tiles are read only behind a non-empty segment.
    const uint32_t sparse_below = b2sr::n_tile_rows(n, A->tile);
    bfs_init_kernel<<<vgrid(n), 256, 0, stream>>>(n, src, levels, L.frontier, L.visited, L.next, L.flags,
                                                  1 < sparse_below ? kRunSparse : kRunDense);
    if ((rc = b2sr::check_launch("bfs_init_kernel"))) return rc;
    const uint32_t *state = L.flags + kState;
    // next = A frontier over unvisited rows, OR-ed into the cleared next; the
    // update consumes and clears next, so no buffers swap
    return run_gated(L.flags, max_iters, iters, stream, [&](uint32_t) {
        // the dense form or the sparse-frontier one, as the state says (the
        // other returns at once); the sparse form has a kernel of its own
        const unsigned fl = B2SR_MASK_COMPLEMENT | B2SR_ACCUMULATE;
        if (int r = b2sr::spmv_bits_gated(A, L.frontier, L.visited, fl, L.next, state, kRunDense, stream)) return r;
        if (int r = b2sr::spmv_bits_gated(A, L.frontier, L.visited, fl | B2SR_SPARSE_X, L.next, state, kRunSparse,
                                          stream))
            return r;
        bfs_update_gated_kernel<<<fgrid(nw), 256, 0, stream>>>(nw, L.next, L.frontier, L.visited, levels, L.flags,
                                                               sparse_below, max_iters);
        return b2sr::check_launch("bfs_update_gated_kernel");
    });
}

int b2sr_msbfs(const b2sr_matrix *A, const uint32_t *srcs, uint32_t nsrc, uint32_t *levels, void *ws,
               size_t ws_bytes, uint32_t *iters, hipStream_t stream)
{
    Layout L;
    int rc = check_algo_args(A, B2SR_ALGO_MSBFS, ws, ws_bytes, &L);
    if (rc) return rc;
    if (!levels || !srcs || nsrc == 0 || nsrc > 64) return B2SR_EINVAL;
    for (uint32_t s = 0; s < nsrc; ++s) {
        if (srcs[s] >= A->n) return B2SR_EINVAL;
        for (uint32_t q = 0; q < s; ++q)
            if (srcs[q] == srcs[s]) return B2SR_EINVAL;
    }
    const uint32_t n = A->n, max_iters = n + 1;
    if ((rc = b2sr::check(hipMemcpyAsync(L.srcs, srcs, nsrc * 4, hipMemcpyHostToDevice, stream), "hipMemcpyAsync(srcs)")))
        return rc;
    msbfs_init_kernel<<<vgrid((uint64_t)nsrc * n), 256, 0, stream>>>(n, nsrc, L.srcs, L.F, L.V, levels, L.flags);
    if ((rc = b2sr::check_launch("msbfs_init_kernel"))) return rc;
    if ((rc = b2sr::fill_u32(L.act, b2sr::n_words(n), 0, stream))) return rc;
    msbfs_seed_kernel<<<1, 64, 0, stream>>>(n, nsrc, L.srcs, L.F, L.V, levels, L.act);
    if ((rc = b2sr::check_launch("msbfs_seed_kernel"))) return rc;
    // srcs is read by the seed kernel above; the caller may reuse it once the
    // first state read has synchronised the stream
    return run_gated(L.flags, max_iters, iters, stream, [&](uint32_t) {
        // only frontier words that are non-zero take part in the product
        if (int r = b2sr::spmv_full_gated(A, B2SR_OR_U64, L.F, L.act, 0, 0.0, L.Y, L.flags + kState, kRunDense, stream))
            return r;
        msbfs_update_kernel<<<fgrid(n), 256, 0, stream>>>(n, L.Y, L.F, L.V, levels, L.act, L.flags, max_iters);
        return b2sr::check_launch("msbfs_update_kernel");
    });
}

// Min-plus iterations with the SELF term until no entry changes.  Iteration k
// reads buf[(k - 1) & 1] and writes buf[k & 1]; the enqueued iterations that run
// are exactly the first ones, so the host picks the buffers by enqueue index.
// Only entries that changed last iteration can improve a neighbour (the others
// were folded in when they changed), so the product reads those alone.  Leaves
// the result in buf[0].
int min_plus_to_fixpoint(const b2sr_matrix *A, uint32_t weight, uint32_t *buf0, uint32_t *buf1, const Layout &L,
                         uint32_t *iters, hipStream_t stream)
{
    const uint32_t n = A->n, max_iters = n + 1;
    uint32_t *buf[2] = {buf0, buf1};
    uint32_t done = 0;
    int rc = run_gated(L.flags, max_iters, &done, stream, [&](uint32_t k) {
        const uint32_t *cur = buf[(k - 1) & 1];
        uint32_t *nxt = buf[k & 1];
        if (int r = b2sr::spmv_full_gated(A, B2SR_MIN_PLUS_U32, cur, L.act, B2SR_SELF, (double)weight, nxt,
                                          L.flags + kState, kRunDense, stream))
            return r;
        changed_kernel<<<fgrid(n), 256, 0, stream>>>(n, cur, nxt, L.act, L.flags, max_iters);
        return b2sr::check_launch("changed_kernel");
    });
    if (rc) return rc;
    // the last iteration changed nothing, so both buffers hold the result; the
    // iteration bound (never reached: a change lowers some entry, and entries
    // settle within n rounds) would leave it in buf[done & 1]
    if (done & 1) {
        copy_u32_kernel<<<vgrid(n), 256, 0, stream>>>(n, buf1, buf0);
        if ((rc = b2sr::check_launch("copy_u32_kernel"))) return rc;
    }
    if (iters) *iters = done;
    return B2SR_OK;
}

int b2sr_sssp(const b2sr_matrix *A, uint32_t src, uint32_t *dist, void *ws, size_t ws_bytes, uint32_t *iters,
              hipStream_t stream)
{
    Layout L;
    int rc = check_algo_args(A, B2SR_ALGO_SSSP, ws, ws_bytes, &L);
    if (rc) return rc;
    if (!dist || src >= A->n) return B2SR_EINVAL;
    const uint32_t n = A->n;
    sssp_init_kernel<<<vgrid(n), 256, 0, stream>>>(n, src, L.u0, L.act, L.flags);
    if ((rc = b2sr::check_launch("sssp_init_kernel"))) return rc;
    // hop counts in uint32 with saturating addition: exact for every n
    if ((rc = min_plus_to_fixpoint(A, 1, L.u0, L.u1, L, iters, stream))) return rc;
    copy_u32_kernel<<<vgrid(n), 256, 0, stream>>>(n, L.u0, dist);
    return b2sr::check_launch("copy_u32_kernel");
}

int b2sr_cc(const b2sr_matrix *A, uint32_t *labels, void *ws, size_t ws_bytes, uint32_t *iters, hipStream_t stream)
{
    Layout L;
    int rc = check_algo_args(A, B2SR_ALGO_CC, ws, ws_bytes, &L);
    if (rc) return rc;
    if (!labels) return B2SR_EINVAL;
    if ((uintptr_t)labels & 15) return B2SR_EINVAL;  // the product reads x as 16-byte vectors
    const uint32_t n = A->n;
    iota_kernel<<<vgrid(n), 256, 0, stream>>>(n, labels, L.flags);
    if ((rc = b2sr::check_launch("iota_kernel"))) return rc;
    ones_bits_kernel<<<vgrid(b2sr::n_words(n)), 256, 0, stream>>>(n, L.act);  // every label starts active
    if ((rc = b2sr::check_launch("ones_bits_kernel"))) return rc;
    return min_plus_to_fixpoint(A, 0, labels, L.u0, L, iters, stream);
}

}  // extern "C"

namespace {

// PageRank on A read as the pull matrix: r'(i) = (1-d)/n + d * sum_{j : A_ij} r(j) / o(j).
// Undirected graphs: o = row degrees of A.  Directed graphs (A = the transpose
// of the arc matrix): o = out-degrees = column counts of A.
int pagerank(const b2sr_matrix *A, bool directed, float damping, uint32_t iterations, float *rank, void *ws,
             size_t ws_bytes, hipStream_t stream)
{
    Layout L;
    int rc = check_algo_args(A, B2SR_ALGO_PAGERANK, ws, ws_bytes, &L);
    if (rc) return rc;
    if (!rank || !(damping >= 0.0f && damping <= 1.0f)) return B2SR_EINVAL;
    const uint32_t n = A->n, nw = b2sr::n_words(n);
    if (directed) {
        if ((rc = b2sr::column_counts(A, L.u0, stream))) return rc;
    } else {
        // degrees as a count product with the all-ones vector (bmv_bin_bin_full)
        ones_bits_kernel<<<vgrid(nw), 256, 0, stream>>>(n, L.ones);
        if ((rc = b2sr::check_launch("ones_bits_kernel"))) return rc;
        if ((rc = spmv_bin_bin(A, L.ones, nullptr, B2SR_OUT_COUNT, L.u0, stream))) return rc;
    }
    float *r = rank, *r_next = L.f2;
    pr_init_kernel<<<vgrid(n), 256, 0, stream>>>(n, L.u0, L.f1, r);
    if ((rc = b2sr::check_launch("pr_init_kernel"))) return rc;
    const double beta = (1.0 - (double)damping) / (double)n;
    for (uint32_t it = 0; it < iterations; ++it) {
        pr_scale_kernel<<<vgrid(n), 256, 0, stream>>>(n, r, L.f1, L.f0);
        if ((rc = b2sr::check_launch("pr_scale_kernel"))) return rc;
        if ((rc = spmv_bin_full(A, B2SR_PLUS_TIMES_F32, L.f0, nullptr, nullptr, nullptr, 0, damping, beta, r_next,
                                L.spmv_ws, L.spmv_ws_bytes, stream)))
            return rc;
        std::swap(r, r_next);
    }
    if (r != rank) {
        copy_u32_kernel<<<vgrid(n), 256, 0, stream>>>(n, (const uint32_t *)r, (uint32_t *)rank);
        if ((rc = b2sr::check_launch("copy_u32_kernel"))) return rc;
    }
    return B2SR_OK;
}

}  // namespace

extern "C" {

int b2sr_pagerank(const b2sr_matrix *A, float damping, uint32_t iterations, float *rank, void *ws, size_t ws_bytes,
                  hipStream_t stream)
{
    return pagerank(A, false, damping, iterations, rank, ws, ws_bytes, stream);
}

int b2sr_pagerank_directed(const b2sr_matrix *At, float damping, uint32_t iterations, float *rank, void *ws,
                           size_t ws_bytes, hipStream_t stream)
{
    return pagerank(At, true, damping, iterations, rank, ws, ws_bytes, stream);
}

}  // extern "C"

namespace {

// Rounds of local maxima under max-times (Table V: MIS and colouring).  With
// colors == nullptr: one independent set into mis_bits.  Otherwise colour c is
// the independent set of the vertices still uncoloured, c = 0, 1, ...
int independent_sets(const b2sr_matrix *A, const uint64_t *key, uint32_t *mis_bits, uint32_t *colors, void *ws,
                     size_t ws_bytes, uint32_t *iters, uint32_t *ncolors, hipStream_t stream)
{
    Layout L;
    int rc = check_algo_args(A, colors ? B2SR_ALGO_COLOR : B2SR_ALGO_MIS, ws, ws_bytes, &L);
    if (rc) return rc;
    const uint32_t n = A->n, nw = b2sr::n_words(n);
    if (n > 0 && (!key || (!mis_bits && !colors))) return B2SR_EINVAL;
    if (mis_bits && (rc = b2sr::fill_u32(mis_bits, nw, 0, stream))) return rc;
    if (colors && (rc = b2sr::fill_u32(colors, n, kUnreached, stream))) return rc;
    if (iters) *iters = 0;
    if (ncolors) *ncolors = 0;
    if (n == 0) return B2SR_OK;
    // state dense, no pass pending, colour 0; the first pass's candidates, and
    // whether there are any (in kLast)
    if ((rc = b2sr::fill_u32(L.flags, kFlagWords, 0, stream))) return rc;
    mis_start_kernel<<<fgrid(n), 256, 0, stream>>>(n, key, colors, L.F, L.act, L.flags + kLast, L.flags + kPrev);
    if ((rc = b2sr::check_launch("mis_start_kernel"))) return rc;
    uint32_t any = 0;
    if ((rc = read_flag(L.flags + kLast, &any, stream))) return rc;
    if (!any) return B2SR_OK;
    // every round places at least the candidate of largest key, so n rounds suffice
    const uint32_t max_iters = n + 1;
    uint32_t rounds = 0;
    if ((rc = run_gated(L.flags, max_iters, &rounds, stream, [&](uint32_t) {
             if (colors) {
                 mis_start_gated_kernel<<<fgrid(n), 256, 0, stream>>>(n, key, colors, L.F, L.act, L.flags);
                 if (int r = b2sr::check_launch("mis_start_gated_kernel")) return r;
             }
             if (int r = b2sr::spmv_full_gated(A, B2SR_MAX_TIMES_U64, L.F, L.act, 0, 0.0, L.Y, L.flags + kState,
                                               kRunDense, stream))
                 return r;
             mis_join_gated_kernel<<<fgrid(n), 256, 0, stream>>>(n, L.F, L.Y, L.frontier, mis_bits, colors, L.flags);
             if (int r = b2sr::check_launch("mis_join_gated_kernel")) return r;
             if (int r = b2sr::spmv_bits_gated(A, L.frontier, nullptr, 0, L.next, L.flags + kState, kRunDense, stream))
                 return r;
             mis_remove_gated_kernel<<<fgrid(n), 256, 0, stream>>>(n, L.F, L.frontier, L.next, L.act, key, colors,
                                                                   L.flags, max_iters);
             return b2sr::check_launch("mis_remove_gated_kernel");
         })))
        return rc;
    if (iters) *iters = rounds;
    if (ncolors && colors) {
        uint32_t last = 0;
        if ((rc = b2sr::read_words(L.flags + kColor, &last, 1, stream))) return rc;
        *ncolors = last + 1;
    }
    return B2SR_OK;
}

}  // namespace

extern "C" {

int b2sr_mis(const b2sr_matrix *A, const uint64_t *key, uint32_t *mis_bits, void *ws, size_t ws_bytes,
             uint32_t *iters, hipStream_t stream)
{
    return independent_sets(A, key, mis_bits, nullptr, ws, ws_bytes, iters, nullptr, stream);
}

int b2sr_color(const b2sr_matrix *A, const uint64_t *key, uint32_t *colors, void *ws, size_t ws_bytes,
               uint32_t *ncolors, hipStream_t stream)
{
    return independent_sets(A, key, nullptr, colors, ws, ws_bytes, nullptr, ncolors, stream);
}

int b2sr_eccentricity(const b2sr_matrix *A, const uint32_t *srcs, uint32_t nsrc, uint32_t *ecc, void *ws,
                      size_t ws_bytes, hipStream_t stream)
{
    Layout L;
    int rc = check_algo_args(A, B2SR_ALGO_ECC, ws, ws_bytes, &L);
    if (rc) return rc;
    if (nsrc && (!srcs || !ecc)) return B2SR_EINVAL;
    const uint32_t n = A->n;
    for (uint32_t s = 0; s < nsrc; ++s)
        if (srcs[s] >= n) return B2SR_EINVAL;
    for (uint32_t b = 0; b < nsrc; b += 64) {
        const uint32_t k = std::min<uint32_t>(64, nsrc - b);
        if ((rc = b2sr::check(hipMemcpyAsync(L.srcs, srcs + b, k * 4, hipMemcpyHostToDevice, stream),
                              "hipMemcpyAsync(srcs)")))
            return rc;
        ecc_init_kernel<<<vgrid(n), 256, 0, stream>>>(n, L.F, L.V, L.act, L.alive, L.flags);
        if ((rc = b2sr::check_launch("ecc_init_kernel"))) return rc;
        ecc_seed_kernel<<<1, 64, 0, stream>>>(k, L.srcs, L.F, L.V, L.act);
        if ((rc = b2sr::check_launch("ecc_seed_kernel"))) return rc;
        const uint32_t max_iters = n + 1;
        if ((rc = run_gated(L.flags, max_iters, nullptr, stream, [&](uint32_t) {
                 if (int r = b2sr::spmv_full_gated(A, B2SR_OR_U64, L.F, L.act, 0, 0.0, L.Y, L.flags + kState, kRunDense,
                                                   stream))
                     return r;
                 ecc_update_gated_kernel<<<fgrid(n), 256, 0, stream>>>(n, L.Y, L.F, L.V, L.act, L.alive, L.flags,
                                                                       max_iters);
                 return b2sr::check_launch("ecc_update_gated_kernel");
             })))
            return rc;
        ecc_final_kernel<<<1, 64, 0, stream>>>(L.alive, L.flags, k, L.u0);
        if ((rc = b2sr::check_launch("ecc_final_kernel"))) return rc;
        if ((rc = b2sr::check(hipMemcpyAsync(ecc + b, L.u0, k * 4, hipMemcpyDeviceToHost, stream), "hipMemcpyAsync(ecc)")))
            return rc;
        if ((rc = b2sr::check(hipStreamSynchronize(stream), "hipStreamSynchronize"))) return rc;
    }
    return B2SR_OK;
}

int b2sr_diameter(const b2sr_matrix *A, uint32_t *diameter, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!diameter) return B2SR_EINVAL;
    if (int rc = b2sr::validate_matrix(A)) return rc;
    *diameter = 0;
    uint32_t srcs[64], ecc[64];
    for (uint32_t b = 0; b < A->n; b += 64) {
        const uint32_t k = std::min<uint32_t>(64, A->n - b);
        for (uint32_t s = 0; s < k; ++s) srcs[s] = b + s;
        if (int rc = b2sr_eccentricity(A, srcs, k, ecc, ws, ws_bytes, stream)) return rc;
        for (uint32_t s = 0; s < k; ++s) *diameter = std::max(*diameter, ecc[s]);
    }
    return B2SR_OK;
}

}  // extern "C"
