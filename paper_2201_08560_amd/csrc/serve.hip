// Continuous multi-source BFS sessions: the device half of query serving.
//
// A session holds the BFS state of up to 64 queries on one resident graph, one
// per bit of a 64-bit word per vertex, as the batched BFS does (the Boolean
// semiring of Table V applied to 64 frontier vectors at once):
//     Y = A (x) F;  new = Y & ~V;  V |= new;  F = new.
// Queries are independent bit lanes, so they need not start together: a query
// joins a free bit between two levels (its source is seeded at the session's
// current step) and leaves when its bit reaches no new vertex, while the other
// bits go on.  Each vertex records, per bit, the session step at which that bit
// reached it; a query's level of v is that step minus the step it joined at.
//
// Per step: one OR_U64 product over the active frontier words (spmv_bin_full
// with x_active) and one update kernel, which also ORs every new word into a
// 64-bit "alive" word (bit s set: query s reached a new vertex this step).
// The alive word is copied to a host buffer so the caller can retire finished
// queries and admit new ones without waiting on the device.
#include <new>

#include "common.h"

using namespace b2sr_dev;

namespace {

constexpr uint32_t kUnreached = 0xFFFFFFFFu;

struct SessionLayout {
    uint64_t *F, *V, *Y;
    uint32_t *act;     // bit vector: vertices whose frontier word is non-zero
    uint64_t *alive;   // two words, used in turn by consecutive steps
    uint32_t *steps;   // n x 64, vertex-major: step at which bit s reached v
    size_t bytes;
};

SessionLayout carve(uint32_t n, void *ws)
{
    SessionLayout L{};
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
    L.alive = (uint64_t *)take(16);
    L.steps = (uint32_t *)take((size_t)n * 64 * 4);
    L.bytes = off;
    return L;
}

unsigned vgrid(uint64_t work) { return b2sr::grid_for(work, 256, 8192); }

__global__ void session_init_kernel(uint32_t n, uint64_t *F, uint64_t *V, uint64_t *Y, uint32_t *act, uint64_t *alive)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = tid; i < n; i += stride) {
        F[i] = 0;
        V[i] = 0;
        Y[i] = 0;
    }
    for (uint64_t w = tid; w < (n + 31) / 32; w += stride) act[w] = 0;
    if (tid < 2) alive[tid] = 0;
}

// Clears bit `slot` everywhere (the previous query in the slot may have left
// visited bits, or frontier bits if it was cancelled), then seeds `src`.  The
// thread of vertex src does both for it, so nothing races.
__global__ void session_join_kernel(uint32_t n, uint64_t *F, uint64_t *V, uint32_t *act, uint32_t *steps,
                                    uint32_t slot, uint32_t src, uint32_t step)
{
    const uint64_t bit = 1ull << slot;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t f = F[i] & ~bit, v = V[i] & ~bit;
        if (i == src) {
            f |= bit;
            v |= bit;
            steps[i * 64 + slot] = step;
            atomicOr(act + (i >> 5), 1u << (i & 31));
        }
        F[i] = f;
        V[i] = v;
    }
}

// new = Y & ~V for 64 vertices per wave pass; records the step of every new
// bit, rewrites the active bit vector, clears Y, and ORs the new words into
// alive[step & 1] (the other word, for the next step, is cleared here).
__global__ void session_update_kernel(uint32_t n, uint64_t *Y, uint64_t *F, uint64_t *V, uint32_t *act,
                                      uint32_t *steps, uint32_t step, uint64_t *alive)
{
    uint64_t seen = 0;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / B2SR_WAVE);
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + threadIdx.x / B2SR_WAVE) * 64; base < n;
         base += waves * 64) {
        const uint64_t i = base + lane_id();
        uint64_t y = 0;
        if (i < n) {
            y = Y[i] & ~V[i];
            Y[i] = 0;
            F[i] = y;
            if (y) V[i] |= y;
        }
        const uint64_t m = __ballot(y != 0);
        const uint64_t w = base / 32 + lane_id();
        if (lane_id() < 2 && w < (n + 31u) / 32u) act[w] = (uint32_t)(m >> (32 * lane_id()));
        seen |= y;
        // the step rows are vertex-major (64 words per vertex): one vertex at a
        // time, lane s storing slot s, so one store covers the row's words
        for (uint64_t todo = m; todo;) {
            const uint32_t k = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint64_t yk = ((uint64_t)readlane((uint32_t)(y >> 32), (int)k) << 32) | readlane((uint32_t)y, (int)k);
            if ((yk >> lane_id()) & 1) steps[(base + k) * 64 + lane_id()] = step;
        }
    }
    // OR over the wave, then one atomic per wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) seen |= shfl_xor(seen, d);
    if (lane_id() == 0 && seen) atomicOr((unsigned long long *)alive + (step & 1), (unsigned long long)seen);
    if (blockIdx.x == 0 && threadIdx.x == 0) alive[(step + 1) & 1] = 0;
}

__global__ void session_extract_kernel(uint32_t n, const uint64_t *V, const uint32_t *steps, uint32_t slot,
                                       uint32_t start, uint32_t *levels)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        levels[i] = ((V[i] >> slot) & 1u) ? steps[i * 64 + slot] - start : kUnreached;
}

}  // namespace

struct b2sr_bfs_session_s {
    b2sr_matrix A;
    SessionLayout L;
    uint32_t step = 0;        // steps run so far
    uint32_t start[64] = {};  // step at which each slot's query joined
    uint64_t busy = 0;        // slots holding a query
};

extern "C" {

size_t b2sr_bfs_session_bytes(uint32_t n) { return carve(n, nullptr).bytes; }

int b2sr_bfs_session_create(const b2sr_matrix *A, void *ws, size_t ws_bytes, hipStream_t stream,
                            b2sr_bfs_session *out)
{
    if (!out) return B2SR_EINVAL;
    *out = nullptr;
    if (int rc = b2sr::validate_matrix(A)) return rc;
    if (A->n == 0) return B2SR_EINVAL;
    const SessionLayout L = carve(A->n, ws);
    if (!ws || ws_bytes < L.bytes) return B2SR_ENOSPC;
    b2sr_bfs_session_s *s = new (std::nothrow) b2sr_bfs_session_s();
    if (!s) return B2SR_ENOSPC;
    s->A = *A;
    s->L = L;
    session_init_kernel<<<vgrid(A->n), 256, 0, stream>>>(A->n, L.F, L.V, L.Y, L.act, L.alive);
    if (int rc = b2sr::check_launch("session_init_kernel")) {
        delete s;
        return rc;
    }
    *out = s;
    return B2SR_OK;
}

int b2sr_bfs_session_join(b2sr_bfs_session s, uint32_t slot, uint32_t source, hipStream_t stream)
{
    if (!s || slot >= 64 || source >= s->A.n || ((s->busy >> slot) & 1u)) return B2SR_EINVAL;
    session_join_kernel<<<vgrid(s->A.n), 256, 0, stream>>>(s->A.n, s->L.F, s->L.V, s->L.act, s->L.steps, slot, source,
                                                           s->step);
    if (int rc = b2sr::check_launch("session_join_kernel")) return rc;
    s->start[slot] = s->step;
    s->busy |= 1ull << slot;
    return B2SR_OK;
}

int b2sr_bfs_session_step(b2sr_bfs_session s, uint64_t *alive_host, hipStream_t stream)
{
    if (!s) return B2SR_EINVAL;
    if (s->step == 0xFFFFFFFEu) return B2SR_ERANGE;
    const SessionLayout &L = s->L;
    const uint32_t n = s->A.n;
    // only frontier words that are non-zero take part in the product
    if (int rc = spmv_bin_full(&s->A, B2SR_OR_U64, L.F, nullptr, L.act, nullptr, B2SR_ACCUMULATE, 0.0, 0.0, L.Y,
                               nullptr, 0, stream))
        return rc;
    const uint32_t step = s->step + 1;
    session_update_kernel<<<b2sr::grid_for(n, 256, 1024), 256, 0, stream>>>(n, L.Y, L.F, L.V, L.act, L.steps, step,
                                                                            L.alive);
    if (int rc = b2sr::check_launch("session_update_kernel")) return rc;
    if (alive_host) {
        if (int rc = b2sr::check(hipMemcpyAsync(alive_host, L.alive + (step & 1), 8, hipMemcpyDeviceToHost, stream),
                                 "hipMemcpyAsync(alive)"))
            return rc;
    }
    s->step = step;
    return B2SR_OK;
}

int b2sr_bfs_session_extract(b2sr_bfs_session s, uint32_t slot, uint32_t *levels, hipStream_t stream)
{
    if (!s || slot >= 64 || !((s->busy >> slot) & 1u)) return B2SR_EINVAL;
    if (levels) {
        session_extract_kernel<<<vgrid(s->A.n), 256, 0, stream>>>(s->A.n, s->L.V, s->L.steps, slot, s->start[slot],
                                                                  levels);
        if (int rc = b2sr::check_launch("session_extract_kernel")) return rc;
    }
    s->busy &= ~(1ull << slot);
    return B2SR_OK;
}

int b2sr_bfs_session_info(b2sr_bfs_session s, uint32_t *step, uint64_t *busy)
{
    if (!s) return B2SR_EINVAL;
    if (step) *step = s->step;
    if (busy) *busy = s->busy;
    return B2SR_OK;
}

int b2sr_bfs_session_destroy(b2sr_bfs_session s)
{
    delete s;
    return B2SR_OK;
}

}  // extern "C"
