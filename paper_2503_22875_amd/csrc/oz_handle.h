// oz_handle.h -- accessors of the library handle shared by the host sources.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/oz.h"

#include <vector>

namespace oz {
// One autotuner result: the best GEMM block shape and tile order measured for
// a batch of square problems of size n with slice count s.
struct TuneEntry {
    int cplx;
    int64_t n;
    int s;
    int tile;   // 1: 128 x 64 blocks, 2: 64 x 64 blocks
    int order;  // 0: tiles by work, problem by problem; 1: problems dealt to per-XCD queues
};
}  // namespace oz

bool oz_handle_valid(oz_handle_t h);
const std::vector<oz::TuneEntry>& oz_handle_tuning(oz_handle_t h);
int oz_handle_use_device(oz_handle_t h);  // makes the handle's device current (OZ_OK / OZ_ERR_HIP)
hipStream_t oz_handle_stream(oz_handle_t h);
int oz_handle_device(oz_handle_t h);
hipError_t oz_handle_mark(oz_handle_t h);  // timing event (no-op unless oz_timing_enable)
