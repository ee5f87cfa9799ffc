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

// Returns B2SR_EHIP (recording the text) when e is not hipSuccess.
inline int check(hipError_t e, const char *where)
{
    if (e == hipSuccess) return B2SR_OK;
    set_hip_error(e, where);
    return B2SR_EHIP;
}

// Checks the launch status of the kernel just enqueued.
inline int check_launch(const char *where) { return check(hipGetLastError(), where); }

inline bool valid_tile(uint32_t t) { return t == 4 || t == 8 || t == 16 || t == 32; }
inline uint32_t n_tile_rows(uint32_t n, uint32_t T) { return (n + T - 1) / T; }
inline uint32_t n_words(uint32_t n) { return (n + 31) / 32; }
// Bytes of one bit-row (Table II).
inline uint32_t row_bytes(uint32_t T) { return T == 32 ? 4 : (T == 16 ? 2 : 1); }
inline uint64_t bits_bytes(uint64_t ntiles, uint32_t T) { return ntiles * T * row_bytes(T); }

// Host validation of a B2SR view; returns B2SR_OK or an error code.
int validate_matrix(const b2sr_matrix *A);

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

// Per tile width: lanes per tile (LPT), bit-rows per lane (RPL) and tiles per
// wave step (TPW).  One lane reads a 16-byte (T = 32, 16), 8-byte (T = 8) or
// 4-byte (T = 4) piece of a tile, so a wave step reads a contiguous run of
// whole tiles: 1 KiB for T = 32, 1 KiB for T = 16, 512 B for T = 8 and 256 B
// for T = 4.
template <int T> struct TileShape;
template <> struct TileShape<32> { static constexpr int LPT = 8, RPL = 4, TPW = 8; };
template <> struct TileShape<16> { static constexpr int LPT = 2, RPL = 8, TPW = 32; };
template <> struct TileShape<8> { static constexpr int LPT = 1, RPL = 8, TPW = 64; };
template <> struct TileShape<4> { static constexpr int LPT = 1, RPL = 4, TPW = 64; };

// Loads the RPL bit-rows [sub*RPL, sub*RPL + RPL) of tile t as T-bit values.
template <int T> __device__ __forceinline__ void load_rows(const void *bits, uint32_t t, uint32_t sub,
                                                           uint32_t (&a)[TileShape<T>::RPL]);

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <> __device__ __forceinline__ void load_rows<32>(const void *bits, uint32_t t, uint32_t sub,
                                                          uint32_t (&a)[4])
{
    u32x4 v = __builtin_nontemporal_load((const u32x4 *)bits + ((size_t)t * 8 + sub));
    a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
}
template <> __device__ __forceinline__ void load_rows<16>(const void *bits, uint32_t t, uint32_t sub,
                                                          uint32_t (&a)[8])
{
    u32x4 v = __builtin_nontemporal_load((const u32x4 *)bits + ((size_t)t * 2 + sub));
    a[0] = v.x & 0xFFFFu; a[1] = v.x >> 16; a[2] = v.y & 0xFFFFu; a[3] = v.y >> 16;
    a[4] = v.z & 0xFFFFu; a[5] = v.z >> 16; a[6] = v.w & 0xFFFFu; a[7] = v.w >> 16;
}
template <> __device__ __forceinline__ void load_rows<8>(const void *bits, uint32_t t, uint32_t,
                                                         uint32_t (&a)[8])
{
    u32x2 v = __builtin_nontemporal_load((const u32x2 *)bits + t);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = (v.x >> (8 * k)) & 0xFFu;
        a[4 + k] = (v.y >> (8 * k)) & 0xFFu;
    }
}
template <> __device__ __forceinline__ void load_rows<4>(const void *bits, uint32_t t, uint32_t,
                                                         uint32_t (&a)[4])
{
    uint32_t v = __builtin_nontemporal_load((const uint32_t *)bits + t);
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = (v >> (8 * k)) & 0xFu;
}

// T-bit segment J of a bit vector (bits [J*T, J*T + T)).
template <int T> __device__ __forceinline__ uint32_t bit_segment(const uint32_t *x, uint32_t J)
{
    if constexpr (T == 32) {
        return x[J];
    } else {
        uint32_t w = x[(J * T) >> 5];
        return (w >> ((J * T) & 31u)) & ((1u << T) - 1u);
    }
}

}  // namespace b2sr_dev
