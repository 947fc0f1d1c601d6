// The gather-rate measurement aid (measure.hip).
#pragma once
#include "fvv_internal.h"

namespace fvv {

// blocks x kBlock lanes each read gather_peak_words(blocks) / (blocks x
// kBlock) words of `table` (n_words >= 64); lane sums go to sink.
hipError_t launch_gather_peak(fvv_ctx* ctx, const uint32_t* table, uint32_t n_words,
                              uint32_t* sink, uint32_t blocks, hipStream_t s);
uint64_t gather_peak_words(uint32_t blocks);

}  // namespace fvv
