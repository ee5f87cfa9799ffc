// Device-wide prefix sums: per-block totals, one workgroup scanning the
// totals, and a per-block scan offset by its total's prefix.  Each thread
// owns kScanItems consecutive elements.  Shared by the kernels that need a
// scan of more than a few thousand entries.
#pragma once

#include "common.h"

namespace b2sr_scan {

using namespace b2sr_dev;

constexpr unsigned kScanThreads = 256, kScanWaves = kScanThreads / 64;
constexpr unsigned kScanItems = 8, kScanTile = kScanThreads * kScanItems;

template <class V> struct LoadArray {
    const V *a;
    __device__ V operator()(uint64_t i) const { return a[i]; }
};

// Exclusive prefix of v over the block's threads; *total gets the block sum.
template <class V> __device__ V block_exclusive(V v, V *total)
{
    __shared__ V wsum[kScanWaves];
    const unsigned lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    V x = v;
    for (unsigned d = 1; d < 64; d <<= 1) {
        V y = shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    V before = 0, all = 0;
    for (unsigned i = 0; i < kScanWaves; ++i) {
        V s = wsum[i];
        if (i < w) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

template <class V, class Load>
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(uint64_t n, Load load, V *sums)
{
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    V s = 0;
    for (unsigned k = 0; k < kScanItems; ++k)
        if (base + k < n) s += load(base + k);
    V total;
    block_exclusive(s, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <class V> __global__ void __launch_bounds__(kScanThreads) scan_sums_kernel(uint32_t nb, V *sums)
{
    V carry = 0;
    for (uint32_t base = 0; base < nb; base += kScanThreads) {
        const uint32_t i = base + threadIdx.x;
        const V v = i < nb ? sums[i] : 0;
        V total;
        const V ex = block_exclusive(v, &total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
}

// out may be the array load reads: each element is read before it is written,
// by the same thread.
template <class V, class Load>
__global__ void __launch_bounds__(kScanThreads) scan_apply_kernel(uint64_t n, Load load, const V *sums, V *out,
                                                                  bool inclusive)
{
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    V v[kScanItems];
    V s = 0;
    for (unsigned k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? load(base + k) : 0;
        s += v[k];
    }
    V total;
    V run = sums[blockIdx.x] + block_exclusive(s, &total);
    for (unsigned k = 0; k < kScanItems; ++k) {
        if (inclusive) run += v[k];
        if (base + k < n) out[base + k] = run;
        if (!inclusive) run += v[k];
    }
}

// Entries of the block-total buffer a scan of n elements needs.
inline uint64_t scan_blocks(uint64_t n) { return (n + kScanTile - 1) / kScanTile; }

// out[i] = sum of load(0 .. i) (inclusive) or of load(0 .. i - 1) (exclusive);
// sums: scan_blocks(n) entries of V.
template <class V, class Load>
inline int device_scan(uint64_t n, Load load, V *out, bool inclusive, V *sums, hipStream_t s)
{
    if (n == 0) return B2SR_OK;
    const unsigned nb = (unsigned)scan_blocks(n);
    scan_reduce_kernel<V, Load><<<nb, kScanThreads, 0, s>>>(n, load, sums);
    if (int rc = b2sr::check_launch("scan_reduce_kernel")) return rc;
    scan_sums_kernel<V><<<1, kScanThreads, 0, s>>>(nb, sums);
    if (int rc = b2sr::check_launch("scan_sums_kernel")) return rc;
    scan_apply_kernel<V, Load><<<nb, kScanThreads, 0, s>>>(n, load, sums, out, inclusive);
    return b2sr::check_launch("scan_apply_kernel");
}

}  // namespace b2sr_scan
