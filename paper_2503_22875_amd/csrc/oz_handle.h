// oz_handle.h -- accessors of the library handle shared by the host sources.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/oz.h"
#include "oz_internal.h"

#include <vector>

namespace oz {
// One autotuner result: the best GEMM block shape and tile order measured for
// a batch of square problems of size n with slice count s.
struct TuneEntry {
    int cplx;
    int64_t n;
    int s;
    int tile;   // 1: 128 x 64 blocks, 2: 64 x 64 blocks, 4: 128 x 64 blocks of two-tile waves
    int order;  // 0: tiles by work, problem by problem; 1: problems dealt to per-XCD queues
};
}  // namespace oz

bool oz_handle_valid(oz_handle_t h);
const std::vector<oz::TuneEntry>& oz_handle_tuning(oz_handle_t h);
int oz_handle_use_device(oz_handle_t h);  // makes the handle's device current (OZ_OK / OZ_ERR_HIP)
hipStream_t oz_handle_stream(oz_handle_t h);
int oz_handle_device(oz_handle_t h);
hipError_t oz_handle_mark(oz_handle_t h);  // timing event (no-op unless oz_timing_enable)
// library-owned workspace of at least `bytes` (grown on demand); null and
// *status set on failure
char* oz_handle_ws(oz_handle_t h, size_t bytes, int* status);
// LU: the handle's look-ahead stream and three events (created on the first
// call, kept until oz_destroy), and a grow-only device buffer of at least
// `bytes` apart from the GEMM workspace (null and *status set on failure)
int oz_handle_lu_stream(oz_handle_t h, hipStream_t* s2, hipEvent_t* ev);
char* oz_handle_lu_ws(oz_handle_t h, size_t bytes, int* status);
// learned slice-count selector attached to the handle (may be null)
oz_mlp_t oz_handle_selector(oz_handle_t h);
void oz_handle_set_selector(oz_handle_t h, oz_mlp_t mlp);

// learned selection (oz_learn.hip): device scratch bytes of one selection
// and the selection itself (synchronises the stream; msa, msb: m and n doubles)
size_t oz_learned_scratch_bytes();
int oz_learned_start(oz_handle_t h, oz_mlp_t mlp, const oz::OperandView& va, const oz::OperandView& vb,
                     const uint64_t* maxa, const uint64_t* maxb, double* msa, double* msb, int64_t m, int64_t n,
                     int64_t k, int cplx, double tol, int smax, char* scratch, int* s_out);

// selector network (oz_mlp.hip)
bool oz_mlp_valid(oz_mlp_t p);
// y = network(X) for rows feature rows, then s = clamp(floor(y + 1/2), smin, smax)
hipError_t oz_mlp_predict_device(oz_mlp_t p, int64_t rows, const float* X, float* y, int smin, int smax,
                                 int32_t* s_out, hipStream_t st);
