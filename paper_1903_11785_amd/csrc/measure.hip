// A measurement aid for the gather roofline of the carve: the rate at which
// the GPU serves 4-byte words from a table the size of a frame's packed
// silhouettes, read coalesced within a wave (one word per lane, 64
// consecutive words) at pseudo-random wave offsets -- the fastest any carve
// could fetch silhouette words from that table.  Not part of the path.
#include "measure.h"

namespace fvv {

constexpr int kGatherIters = 256;   // words per lane and launch

__global__ __launch_bounds__(kBlock) void gather_peak_kernel(const uint32_t* __restrict__ table,
                                                             uint32_t n_words,
                                                             uint32_t* __restrict__ sink) {
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    // per-wave linear congruential sequence (uniform over the wave), offsets
    // in [0, n_words - 64] by a multiply-high
    uint32_t x = (gid / kWave) * 2654435761u + 12345u;
    const uint32_t span = n_words - (uint32_t)kWave + 1u;
    uint32_t acc = 0;
#pragma unroll 8
    for (int i = 0; i < kGatherIters; ++i) {
        x = x * 1664525u + 1013904223u;
        const uint32_t base = (uint32_t)(((uint64_t)x * span) >> 32);
        acc += table[base + lane_id()];
    }
    sink[gid] = acc;
}

hipError_t launch_gather_peak(fvv_ctx* ctx, const uint32_t* table, uint32_t n_words,
                              uint32_t* sink, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL(gather_peak_kernel, dim3(blocks), dim3(kBlock), 0, s, table, n_words, sink);
    return hipGetLastError();
}

uint64_t gather_peak_words(uint32_t blocks) { return (uint64_t)blocks * kBlock * kGatherIters; }

}  // namespace fvv
