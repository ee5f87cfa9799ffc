// Matrix-vector products on B2SR (Sec. IV, Table III; semirings of Table V).
//
// Work decomposition (wave64, gfx950).  The paper gives one warp a whole
// tile-row and one lane a bit-row.  On power-law graphs that leaves a few
// waves with thousands of tiles, so here every wave takes a fixed CHUNK of
// consecutive tiles instead, whatever rows they belong to:
//   * a wave step covers TPW consecutive tiles; LPT lanes share a tile and each
//     reads one 32/16/8/4-byte piece holding RPL bit-rows (TileShape), so a step
//     reads one contiguous run of tile bytes;
//   * steps are grouped into blocks of U steps whose loads are all issued before
//     any of them is used (U * 16 bytes of tile data in flight per lane for
//     T = 32), together with the block's tile-column indices, one per lane;
//   * full-precision vector segments (T values per tile, Sec. IV "efficient
//     full-precision vector load") are read with coalesced vector loads and
//     staged in LDS, so a set bit costs one LDS read instead of a dependent
//     global gather;
//   * the tile-row of the chunk's first tile comes from a 64-way search of
//     TileRowPtr; when a whole step lies inside the current tile-row each lane
//     folds its partial into a register accumulator;
//   * when a step crosses row ends, each lane finds its tile's row from the
//     next 64 row pointers held one per lane, and a segmented scan over the
//     wave combines partials of equal rows;
//   * a finished row is written once per chunk.  Bit, count and min results
//     use atomics (exact and order-free); float sums write rows owned by one
//     chunk directly and park the partials of rows that straddle chunks in the
//     workspace, where a second kernel adds them in chunk order, so every float
//     result is deterministic.
// Masks are applied when a row is stored (Sec. V, BFS).  Blocks whose rows are
// all masked out are not read, and with B2SR_SPARSE_X tiles whose x segment is
// empty are not read either.
#include <atomic>

#include "spmv_core.h"

using namespace b2sr_dev;
using namespace b2sr_core;

namespace {

// Minimum waves per SIMD asked of the compiler (the second __launch_bounds__
// argument) per tile width and kind: set where the product measured faster and
// nothing spills; 1 is no request.
#ifndef B2SR_W32_PLUS
#define B2SR_W32_PLUS 5
#endif
#ifndef B2SR_W32_MIN
#define B2SR_W32_MIN 5
#endif
#ifndef B2SR_W32_U64
#define B2SR_W32_U64 6
#endif
#ifndef B2SR_W32_BITS
#define B2SR_W32_BITS 5
#endif
#ifndef B2SR_W16_PLUS
#define B2SR_W16_PLUS 5
#endif
#ifndef B2SR_W16_MIN
#define B2SR_W16_MIN 5
#endif
#ifndef B2SR_W16_U64
#define B2SR_W16_U64 1
#endif
#ifndef B2SR_W8_PLUS
#define B2SR_W8_PLUS 1
#endif
#ifndef B2SR_W8_U64
#define B2SR_W8_U64 1
#endif
constexpr int waves_hint(int T, int K)
{
    const bool plus = K == kPlusF32, mins = K == kMinF32 || K == kMinU32, u64 = K == kOr64 || K == kMaxU64;
    if (T == 32) return plus ? B2SR_W32_PLUS : mins ? B2SR_W32_MIN : u64 ? B2SR_W32_U64 : B2SR_W32_BITS;
    if (T == 16) return plus ? B2SR_W16_PLUS : mins ? B2SR_W16_MIN : u64 ? B2SR_W16_U64 : 1;
    if (T == 8) return plus ? B2SR_W8_PLUS : u64 ? B2SR_W8_U64 : 1;
    return 1;
}

template <int T, int K, bool ACT, bool SHORT = false>
__global__ void __launch_bounds__(256, waves_hint(T, K)) spmv_kernel(SpmvArgs p)
{
    using V = typename KindTraits<K>::V;
    constexpr bool stage = Cfg<T, K>::kStage;
    __shared__ __align__(16) V s_x[stage ? 4 * kSliceBytes / sizeof(V) : 1];
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / B2SR_WAVE) + readfirstlane(threadIdx.x / B2SR_WAVE);
    if (wave * p.chunk >= p.ntiles || gated_off(p)) return;
    spmv_chunk<T, K, ACT, SHORT>(p, (uint32_t)wave,
                                 s_x + (stage ? (threadIdx.x / B2SR_WAVE) * kSliceBytes / sizeof(V) : 0));
}

// Float sums of rows that straddle chunks.  One thread per (chunk, row of a
// tile-row): when the chunk's last tile-row starts in it and continues into the
// next chunk, the thread adds that row's partials over every chunk the
// tile-row spans, in chunk order.  The partials' addresses are known up front,
// so the loads overlap.
template <int T> __global__ void __launch_bounds__(256) plus_fixup_kernel(SpmvArgs p, uint32_t nchunks)
{
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (uint64_t)nchunks * T || gated_off(p)) return;
    const uint32_t c = (uint32_t)(id / T), r = (uint32_t)(id % T);
    const uint32_t t_begin = c * p.chunk, t_end = min(t_begin + p.chunk, p.ntiles);
    const uint32_t r_first = p.ws_rows[2 * c], R = p.ws_rows[2 * c + 1];
    const uint32_t R_end = p.trp[R + 1];
    if (R_end <= t_end || p.trp[R] < t_begin) return;  // R ends here, or started in an earlier chunk
    const uint32_t c_last = (R_end - 1) / p.chunk;
    float sum = p.ws_part[((size_t)c * 2 + (R == r_first ? 0 : 1)) * T + r];
#pragma unroll 8
    for (uint32_t c2 = c + 1; c2 <= c_last; ++c2) sum += p.ws_part[(size_t)c2 * 2 * T + r];
    const uint32_t row = R * T + r;
    if (row >= p.n || !((keep_bits<T>(p.mask, p.flags, R, p.n) >> r) & 1u)) return;
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
    if (gated_off(p)) return;
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

__global__ void scale_x_kernel(uint32_t n, const float *__restrict__ x, const float *__restrict__ s, float *z)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        z[i] = x[i] * s[i];
}

__global__ void zero_words_kernel(SpmvArgs p, uint32_t nwords)
{
    if (gated_off(p)) return;
    uint32_t *__restrict__ y = (uint32_t *)p.y;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x) y[i] = 0;
}

template <int T, int K> int launch(SpmvArgs p, hipStream_t stream)
{
    // bit and count products: short blocks when the mean tile-row is shorter
    // than a long block, or under the sparse-frontier hint
    bool short_blocks = false;
    if constexpr (!Cfg<T, K>::kStage)
        short_blocks = (p.flags & B2SR_SPARSE_X) || (uint64_t)p.ntiles < (uint64_t)p.ntr * Cfg<T, K>::BT;
    p.chunk = short_blocks ? chunk_tiles<T, K, true>(p.ntiles, p.chunk_blocks)
                           : chunk_tiles<T, K>(p.ntiles, p.chunk_blocks);
    p.x_whole = p.n % T == 0;
    const uint32_t nchunks = (uint32_t)((p.ntiles + (uint64_t)p.chunk - 1) / p.chunk);
    if (!(p.flags & B2SR_ACCUMULATE) || K >= kPlusF32) {
        if constexpr (K == kBits) {
            const uint32_t nw = b2sr::n_words(p.n);
            zero_words_kernel<<<b2sr::grid_for(nw, 256, 4096), 256, 0, stream>>>(p, nw);
        } else {
            init_values_kernel<K><<<b2sr::grid_for(p.n, 256, 8192), 256, 0, stream>>>(p);
        }
        if (int rc = b2sr::check_launch("init kernel")) return rc;
    }
    if (nchunks == 0) return B2SR_OK;
    if constexpr (Cfg<T, K>::kStage) {
        if (p.xact) spmv_kernel<T, K, true><<<b2sr::grid_for(nchunks, 4), 256, 0, stream>>>(p);
        else spmv_kernel<T, K, false><<<b2sr::grid_for(nchunks, 4), 256, 0, stream>>>(p);
    } else if (short_blocks) {
        spmv_kernel<T, K, false, true><<<b2sr::grid_for(nchunks, 4), 256, 0, stream>>>(p);
    } else {
        spmv_kernel<T, K, false><<<b2sr::grid_for(nchunks, 4), 256, 0, stream>>>(p);
    }
    if (int rc = b2sr::check_launch("spmv_kernel")) return rc;
    if constexpr (K == kPlusF32) {
        plus_fixup_kernel<T><<<b2sr::grid_for((uint64_t)nchunks * T, 256), 256, 0, stream>>>(p, nchunks);
        if (int rc = b2sr::check_launch("plus_fixup_kernel")) return rc;
    }
    return B2SR_OK;
}

template <int K> int dispatch(uint32_t T, const SpmvArgs &p, hipStream_t s)
{
    switch (T) {
    case 4: return launch<4, K>(p, s);
    case 8: return launch<8, K>(p, s);
    case 16: return launch<16, K>(p, s);
    case 64: return launch<64, K>(p, s);
    default: return launch<32, K>(p, s);
    }
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
    p.chunk_blocks = A->chunk_blocks;
    return p;
}

uint32_t plus_chunk(const b2sr_matrix *A)
{
    const uint32_t nt = A->ntiles, cb = A->chunk_blocks;
    switch (A->tile) {
    case 4: return chunk_tiles<4, kPlusF32>(nt, cb);
    case 8: return chunk_tiles<8, kPlusF32>(nt, cb);
    case 16: return chunk_tiles<16, kPlusF32>(nt, cb);
    case 64: return chunk_tiles<64, kPlusF32>(nt, cb);
    default: return chunk_tiles<32, kPlusF32>(nt, cb);
    }
}

// Plus-times workspace: the first and last row of every chunk, then the
// straddling rows' partials (256-byte aligned pieces); x * col_scale follows.
size_t plus_partials_bytes(const b2sr_matrix *A)
{
    const uint32_t chunk = plus_chunk(A);
    const uint64_t nchunks = ((uint64_t)A->ntiles + chunk - 1) / chunk;
    const uint64_t rows_bytes = (nchunks * 2 * 4 + 255) & ~255ull;
    return (size_t)((rows_bytes + nchunks * 2 * A->tile * 4 + 255) & ~255ull);
}

int full_product(const b2sr_matrix *A, int semiring, const void *x, const float *col_scale,
                 const uint32_t *x_active, const uint32_t *mask, unsigned flags, double alpha, double beta,
                 void *y, void *ws, size_t ws_bytes, hipStream_t stream)
{
    int rc = b2sr::validate_matrix(A);
    if (rc) return rc;
    if (semiring < B2SR_PLUS_TIMES_F32 || semiring > B2SR_MAX_TIMES_U64) return B2SR_ENOTSUP;
    if (flags & ~(B2SR_MASK_COMPLEMENT | B2SR_ACCUMULATE | B2SR_SELF)) return B2SR_EINVAL;
    if ((flags & B2SR_SELF) && semiring != B2SR_MIN_PLUS_F32 && semiring != B2SR_MIN_PLUS_U32) return B2SR_EINVAL;
    if (col_scale && semiring != B2SR_PLUS_TIMES_F32) return B2SR_EINVAL;
    if (semiring == B2SR_MIN_PLUS_U32 && !(alpha >= 0.0 && alpha <= 4294967295.0 && alpha == (double)(uint32_t)alpha))
        return B2SR_EINVAL;
    if (A->n > 0 && (!x || !y)) return B2SR_EINVAL;
    if (A->n == 0) return B2SR_OK;
    if (x == y || (const void *)x_active == y || (const void *)mask == y) return B2SR_EINVAL;
    // x segments are read as 16-byte vectors
    if (((uintptr_t)x & 15) || ((uintptr_t)col_scale & 15)) return B2SR_EINVAL;
    // the scaled copy of x is needed only with col_scale
    const size_t need = semiring != B2SR_PLUS_TIMES_F32 ? 0
                      : col_scale ? spmv_bin_full_workspace_bytes(A, semiring) : plus_partials_bytes(A);
    if (ws_bytes < need || (need && !ws)) return B2SR_ENOSPC;
    if (col_scale && ((uintptr_t)ws & 15)) return B2SR_EINVAL;
    SpmvArgs p = make_args(A);
    p.x = x;
    if (col_scale) {
        float *z = (float *)((char *)ws + plus_partials_bytes(A));
        scale_x_kernel<<<b2sr::grid_for(A->n, 256, 8192), 256, 0, stream>>>(A->n, (const float *)x, col_scale, z);
        if ((rc = b2sr::check_launch("scale_x_kernel"))) return rc;
        p.x = z;
    }
    p.xact = x_active;
    p.mask = mask;
    p.flags = flags;
    p.alpha = (float)alpha;
    p.beta = (float)beta;
    p.w_u32 = semiring == B2SR_MIN_PLUS_U32 ? (uint32_t)alpha : 0u;
    p.y = y;
    if (semiring == B2SR_PLUS_TIMES_F32) {
        const uint64_t nchunks = ((uint64_t)A->ntiles + plus_chunk(A) - 1) / plus_chunk(A);
        p.ws_rows = (uint32_t *)ws;
        p.ws_part = (float *)((char *)ws + ((nchunks * 2 * 4 + 255) & ~255ull));
    }
    switch (semiring) {
    case B2SR_PLUS_TIMES_F32: return dispatch<kPlusF32>(A->tile, p, stream);
    case B2SR_MIN_PLUS_F32: return dispatch<kMinF32>(A->tile, p, stream);
    case B2SR_MIN_PLUS_U32: return dispatch<kMinU32>(A->tile, p, stream);
    case B2SR_MAX_TIMES_U64: return dispatch<kMaxU64>(A->tile, p, stream);
    default: return dispatch<kOr64>(A->tile, p, stream);
    }
}



// ---- the no-allocation variant's scratch ------------------------------------
// A file-scope device array serves spmv_bin_full_noalloc as its workspace, so
// that the call allocates nothing.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in for the symbol): its device
// address is taken once per device with hipGetSymbolAddress, with that device
// current, and kept here.
static __device__ __align__(256) unsigned char scratch[B2SR_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch_ptr[kMaxDevices];  // per device; null until its first call

int scratch_on_current_device(void **out)
{
    int dev = 0;
    if (int rc = b2sr::check(hipGetDevice(&dev), "hipGetDevice")) return rc;
    if (dev < 0 || dev >= kMaxDevices) return B2SR_ENOTSUP;
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        // two threads racing here store the same address
        if (int rc = b2sr::check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))
            return rc;
        if (!p) return B2SR_EHIP;
        g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return B2SR_OK;
}

}  // namespace

extern "C" {

int spmv_bin_bin(const b2sr_matrix *A, const uint32_t *x, const uint32_t *mask, unsigned flags, void *y,
                 hipStream_t stream)
{
    int rc = b2sr::validate_matrix(A);
    if (rc) return rc;
    if (flags & ~(B2SR_MASK_COMPLEMENT | B2SR_OUT_COUNT | B2SR_ACCUMULATE | B2SR_SPARSE_X)) return B2SR_EINVAL;
    if (A->n > 0 && (!x || !y)) return B2SR_EINVAL;
    if (A->n == 0) return B2SR_OK;
    if ((const void *)x == y || (const void *)mask == y) return B2SR_EINVAL;
    SpmvArgs p = make_args(A);
    p.x = x;
    p.mask = mask;
    p.flags = flags;
    p.y = y;
    if (flags & B2SR_OUT_COUNT) return dispatch<kCount>(A->tile, p, stream);
    return dispatch<kBits>(A->tile, p, stream);
}

size_t spmv_bin_full_workspace_bytes(const b2sr_matrix *A, int semiring)
{
    if (!A || !b2sr::valid_tile(A->tile) || semiring != B2SR_PLUS_TIMES_F32) return 0;
    return plus_partials_bytes(A) + (size_t)A->n * 4;
}

int spmv_bin_full(const b2sr_matrix *A, int semiring, const void *x, const float *col_scale,
                  const uint32_t *x_active, const uint32_t *mask, unsigned flags, double alpha, double beta,
                  void *y, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return full_product(A, semiring, x, col_scale, x_active, mask, flags, alpha, beta, y, ws, ws_bytes, stream);
}

int spmv_bin_full_noalloc(const b2sr_matrix *A, int semiring, const void *x, const float *col_scale,
                          const uint32_t *x_active, const uint32_t *mask, unsigned flags, double alpha,
                          double beta, void *y, hipStream_t stream)
{
    // sizes are checked on the host first: nothing is launched for a call that
    // does not fit the scratch array
    if (int rc = b2sr::validate_matrix(A)) return rc;
    const size_t need = semiring != B2SR_PLUS_TIMES_F32 ? 0
                      : col_scale ? spmv_bin_full_workspace_bytes(A, semiring) : plus_partials_bytes(A);
    if (need > B2SR_NOALLOC_MAX_BYTES) return B2SR_ENOSPC;
    void *ws = nullptr;
    if (int rc = scratch_on_current_device(&ws)) return rc;
    return full_product(A, semiring, x, col_scale, x_active, mask, flags, alpha, beta, y, ws,
                        B2SR_NOALLOC_MAX_BYTES, stream);
}

}  // extern "C"

namespace b2sr {
// The products for the algorithm drivers' gated iterations: every kernel of the
// launch returns at once unless *gate == gate_val (arguments as the public
// calls, validated by the drivers; no plus-times, so no workspace).
int spmv_bits_gated(const b2sr_matrix *A, const uint32_t *x, const uint32_t *mask, unsigned flags, void *y,
                    const uint32_t *gate, uint32_t gate_val, hipStream_t stream)
{
    SpmvArgs p = make_args(A);
    p.x = x;
    p.mask = mask;
    p.flags = flags;
    p.y = y;
    p.gate = gate;
    p.gate_val = gate_val;
    if (flags & B2SR_OUT_COUNT) return dispatch<kCount>(A->tile, p, stream);
    return dispatch<kBits>(A->tile, p, stream);
}

int spmv_full_gated(const b2sr_matrix *A, int semiring, const void *x, const uint32_t *x_active, unsigned flags,
                    double alpha, void *y, const uint32_t *gate, uint32_t gate_val, hipStream_t stream)
{
    SpmvArgs p = make_args(A);
    p.x = x;
    p.xact = x_active;
    p.flags = flags;
    p.alpha = (float)alpha;
    p.w_u32 = semiring == B2SR_MIN_PLUS_U32 ? (uint32_t)alpha : 0u;
    p.y = y;
    p.gate = gate;
    p.gate_val = gate_val;
    switch (semiring) {
    case B2SR_MIN_PLUS_U32: return dispatch<kMinU32>(A->tile, p, stream);
    case B2SR_OR_U64: return dispatch<kOr64>(A->tile, p, stream);
    case B2SR_MAX_TIMES_U64: return dispatch<kMaxU64>(A->tile, p, stream);
    default: return B2SR_ENOTSUP;
    }
}
}  // namespace b2sr
