// Calibration for the roofline: a plain streaming read, so that the bandwidth
// a product reaches can be set beside the bandwidth a read-only stream of the
// same bytes reaches on the same device (the HBM peak of the data sheet is not
// attainable by reads alone).
#include "common.h"

using namespace b2sr_dev;

namespace {

constexpr int kUnroll = 8;

__global__ void __launch_bounds__(256) stream_read_kernel(const u32x4 *__restrict__ p, uint64_t n16, uint32_t *out)
{
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (uint64_t i = tid; i < n16; i += stride * kUnroll) {
        u32x4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t j = i + (uint64_t)u * stride;
            v[u] = j < n16 ? __builtin_nontemporal_load(p + j) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    // the XOR of the block's words, one word per block: it keeps the loads alive
    // and lets a test check that every byte was read
    __shared__ uint32_t s_acc[256 / B2SR_WAVE];
#pragma unroll
    for (int d = 1; d < B2SR_WAVE; d <<= 1) acc ^= shfl_xor(acc, d);
    if (lane_id() == 0) s_acc[threadIdx.x / B2SR_WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0;
        for (int w = 0; w < 256 / B2SR_WAVE; ++w) x ^= s_acc[w];
        out[blockIdx.x] = x;
    }
}

}  // namespace

extern "C" {

int b2sr_stream_read(const void *p, size_t bytes, uint32_t *out, hipStream_t stream)
{
    if (bytes && (!p || !out)) return B2SR_EINVAL;
    if ((uintptr_t)p & 15) return B2SR_EINVAL;
    if (bytes < 16) return B2SR_OK;
    stream_read_kernel<<<B2SR_STREAM_READ_BLOCKS, 256, 0, stream>>>((const u32x4 *)p, bytes / 16, out);
    return b2sr::check_launch("stream_read_kernel");
}

}  // extern "C"
