// Internal helpers shared by the HIP sources of libb2sr.so (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "b2sr.h"

#define B2SR_WAVE 64

// ---------------------------------------------------------------------------
// Host-side error plumbing
// ---------------------------------------------------------------------------
namespace b2sr {

void set_hip_error(hipError_t e, const char *where);
void clear_hip_error();
// Reads `count` (<= 16) words of device memory at d into the host array h and
// synchronises `stream`.  The copy lands in pinned host words held per host
// thread (allocated on the thread's first read, kept until the process ends):
// a copy into pageable memory goes through a staging blit of about 20 us.
// Falls back to copying into h directly if that allocation failed.
int read_words(const uint32_t *d, uint32_t *h, uint32_t count, hipStream_t stream);

// Returns B2SR_EHIP (recording the text) when e is not hipSuccess.
inline int check(hipError_t e, const char *where)
{
    if (e == hipSuccess) return B2SR_OK;
    set_hip_error(e, where);
    return B2SR_EHIP;
}

// Checks the launch status of the kernel just enqueued.
inline int check_launch(const char *where) { return check(hipGetLastError(), where); }

inline bool valid_tile(uint32_t t) { return t == 4 || t == 8 || t == 16 || t == 32 || t == 64; }
inline uint32_t n_tile_rows(uint32_t n, uint32_t T) { return (n + T - 1) / T; }
inline uint32_t n_words(uint32_t n) { return (n + 31) / 32; }
// Bytes of one bit-row (Table II; 8 for T = 64, the 64-bit packing type of
// Sec. III-A).
inline uint32_t row_bytes(uint32_t T) { return T == 64 ? 8 : T == 32 ? 4 : (T == 16 ? 2 : 1); }
inline uint64_t bits_bytes(uint64_t ntiles, uint32_t T) { return ntiles * T * row_bytes(T); }

// Host validation of a B2SR view; returns B2SR_OK or an error code.
int validate_matrix(const b2sr_matrix *A);

// Enqueues p[0 .. count) = value on the stream (a fill kernel: no memset nodes
// in captured graphs).
int fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t stream);

inline unsigned grid_for(uint64_t work, unsigned per_block, unsigned cap = 1u << 20)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g == 0) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

}  // namespace b2sr

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
namespace b2sr_dev {

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Cross-lane reads.  Each lowers to ds_bpermute_b32 (or a DPP move when the
// pattern allows); 64-bit values move as two 32-bit halves.
__device__ __forceinline__ uint32_t shfl(uint32_t v, int src) { return (uint32_t)__shfl((int)v, src, 64); }
__device__ __forceinline__ float shfl(float v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ uint64_t shfl(uint64_t v, int src)
{
    uint32_t lo = shfl((uint32_t)v, src), hi = shfl((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t shfl_up(uint32_t v, unsigned d) { return (uint32_t)__shfl_up((int)v, d, 64); }
__device__ __forceinline__ float shfl_up(float v, unsigned d) { return __shfl_up(v, d, 64); }
__device__ __forceinline__ uint64_t shfl_up(uint64_t v, unsigned d)
{
    uint32_t lo = shfl_up((uint32_t)v, d), hi = shfl_up((uint32_t)(v >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t shfl_xor(uint32_t v, int m) { return (uint32_t)__shfl_xor((int)v, m, 64); }
__device__ __forceinline__ float shfl_xor(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ uint64_t shfl_xor(uint64_t v, int m)
{
    uint32_t lo = shfl_xor((uint32_t)v, m), hi = shfl_xor((uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}
// Value of v held by a wave-uniform lane, as a scalar.
__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
__device__ __forceinline__ uint32_t readfirstlane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Float minimum as an atomic on its bit pattern: non-negative values order like
// signed integers; negative ones order in reverse like unsigned integers.
__device__ __forceinline__ void atomic_min_f32(float *addr, float v)
{
    if (!signbit(v))
        atomicMin((int *)addr, __float_as_int(v));
    else
        atomicMax((unsigned int *)addr, __float_as_uint(v));
}

__device__ __forceinline__ uint32_t sat_add_u32(uint32_t a, uint32_t b)
{
    uint32_t s = a + b;
    return s < a ? 0xFFFFFFFFu : s;
}

// The register type of one bit-row: T-bit values in 32-bit registers, 64-bit
// ones for T = 64.
template <int T> struct RowWord { using type = uint32_t; };
template <> struct RowWord<64> { using type = uint64_t; };
template <int T> using row_t = typename RowWord<T>::type;

// Per tile width: lanes per tile (LPT), bit-rows per lane (RPL) and tiles per
// wave step (TPW).  One lane reads a 32-byte (T = 64), 16-byte (T = 32, 16),
// 8-byte (T = 8) or 4-byte (T = 4) piece of a tile, so a wave step reads a
// contiguous run of whole tiles: 2 KiB for T = 64, 1 KiB for T = 32 and 16,
// 512 B for T = 8 and 256 B for T = 4.
template <int T> struct TileShape;
template <> struct TileShape<64> { static constexpr int LPT = 16, RPL = 4, TPW = 4; };
template <> struct TileShape<32> { static constexpr int LPT = 8, RPL = 4, TPW = 8; };
template <> struct TileShape<16> { static constexpr int LPT = 2, RPL = 8, TPW = 32; };
template <> struct TileShape<8> { static constexpr int LPT = 1, RPL = 8, TPW = 64; };
template <> struct TileShape<4> { static constexpr int LPT = 1, RPL = 4, TPW = 64; };

typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// T-bit segment J of a bit vector over n entries (bits [J*T, J*T + T)).  At
// T = 64 the segment's upper word lies past the vector's last word when n
// ends in its lower half; it reads as zero then.
template <int T> __device__ __forceinline__ row_t<T> bit_segment(const uint32_t *x, uint32_t J, uint32_t n)
{
    if constexpr (T == 64) {
        const uint32_t lo = x[2 * (size_t)J];
        const uint32_t hi = (uint64_t)J * 64 + 32 < n ? x[2 * (size_t)J + 1] : 0u;
        return ((uint64_t)hi << 32) | lo;
    } else if constexpr (T == 32) {
        (void)n;
        return x[J];
    } else {
        (void)n;
        uint32_t w = x[(J * T) >> 5];
        return (w >> ((J * T) & 31u)) & ((1u << T) - 1u);
    }
}

}  // namespace b2sr_dev
