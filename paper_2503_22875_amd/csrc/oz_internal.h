// oz_internal.h -- shapes, argument blocks and launchers shared by the HIP
// sources of the library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oz {

// Rows of a slice buffer are padded to a multiple of the largest GEMM block
// tile side, so any tile shape reads whole tiles without bounds checks.
constexpr int kRowPad = 128;
// Terms per MFMA step (v_mfma_i32_32x32x32_i8 consumes 32 int8 per row).
constexpr int kStep = 32;
// Terms per 16-byte chunk of the slice layout.
constexpr int kHalf = 16;
// Largest slice count the all-diagonal kernel keeps in registers.
constexpr int kMaxLiveSlices = 8;
// Scale exponent marking a vector that holds Inf or NaN.
constexpr int32_t kNonFiniteExp = INT32_MIN;

inline int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// Where the vectors of one operand come from.  Vector v, term l:
//   element index  idx = v*sv + l*sl   (in elements of 1 or 2 doubles)
struct OperandView {
    const double* X;
    int64_t sv, sl;     // element strides along vectors / along terms
    int64_t nv, k;      // vectors, terms (complex elements count once)
    int cplx;           // interleaved (re, im) doubles
    int conj;           // negate imaginary parts ('C')
    int side_a;         // complex side 'A' writes the two-row (re, im) form
};

// Layout of the slices of one operand (see oz.h).
struct SliceLayout {
    int64_t rows_pad;   // padded vector count (multiple of kRowPad)
    int64_t kpad;       // padded term count (multiple of kStep)
    int s;              // slices
};

SliceLayout slice_layout(int side_a, int cplx, int64_t nv, int64_t k, int s);

// Split: per-vector max magnitude bits (uint64) -> exponent + digits.
hipError_t launch_zero_u64(uint64_t* p, int64_t n, hipStream_t st);
hipError_t launch_scan(const OperandView& op, uint64_t* maxbits, hipStream_t st);
hipError_t launch_digits(const OperandView& op, const uint64_t* maxbits, const SliceLayout& lay,
                         int32_t* E, int8_t* slices, hipStream_t st);

// GEMM over slice buffers with fused FP64 epilogue.
struct GemmArgs {
    const int8_t* SA;   // slices of A' (rows_pad = Mp)
    const int8_t* SB;   // slices of B' (rows_pad = Np)
    const int32_t* EA;  // scale exponents of A (per row / complex row)
    const int32_t* FB;  // scale exponents of B (per column)
    int64_t Mp, Np, kpad;
    int64_t chunk_steps;   // MFMA steps (of kStep terms) per INT32 chunk
    int s;
    int cplx;
    int tile;              // 0 auto, 1: 128 x 64 block, 2: 64 x 64 block, 3: per-diagonal streaming
    // epilogue
    double* C;
    int64_t ldc;
    int64_t m, n;          // valid output rows (complex rows) and columns
    double alpha_r, alpha_i, beta_r, beta_i;
    int beta_zero;
    // verification mode: write INT32 anti-diagonal sums instead of C
    int32_t* diag_out;
};
hipError_t launch_gemm(const GemmArgs& g, hipStream_t st);

// C = beta*C for the alpha == 0 / k == 0 quick return.
hipError_t launch_scale_c(double* C, int64_t ldc, int64_t m, int64_t n, int cplx, double br, double bi,
                          int beta_zero, hipStream_t st);

}  // namespace oz
