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
constexpr int kMaxWideSlices = 14;  // the all-diagonal tile at one wave per SIMD serves s = 9 .. 14
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

// Vectors of op(X): side 'A' rows of op(A) (nv = m), side 'B' columns of
// op(B) (nv = n); trans 'N', 'T' or 'C' (upper case).
inline OperandView operand_view(char trans, const double* X, int64_t ld, int64_t nv, int64_t k, int cplx,
                                int side_a) {
    OperandView v;
    const bool t = trans != 'N';
    v.X = X;
    v.sv = side_a ? (t ? ld : 1) : (t ? 1 : ld);
    v.sl = side_a ? (t ? 1 : ld) : (t ? ld : 1);
    v.nv = nv;
    v.k = k;
    v.cplx = cplx;
    v.conj = cplx && trans == 'C';
    v.side_a = side_a;
    return v;
}

// Layout of the slices of one operand (see oz.h).
struct SliceLayout {
    int64_t rows_pad;   // padded vector count (multiple of kRowPad)
    int64_t kpad;       // padded term count (multiple of kStep)
    int s;              // slices
    int bal;            // 1: balanced (round-to-nearest) digits, all s planes at once
};

SliceLayout slice_layout(int side_a, int cplx, int64_t nv, int64_t k, int s);

// Split: per-vector max magnitude bits (uint64) -> exponent + digits.
hipError_t launch_zero_u64(uint64_t* p, int64_t n, hipStream_t st);
hipError_t launch_scan(const OperandView& op, uint64_t* maxbits, hipStream_t st);
// Digit planes p_lo .. p_hi - 1 (0-based; p_hi < 0: all planes of the layout).
// The scale exponents E are written by every call.
hipError_t launch_digits(const OperandView& op, const uint64_t* maxbits, const SliceLayout& lay,
                         int32_t* E, int8_t* slices, hipStream_t st, int p_lo = 0, int p_hi = -1);

// Split of a complex operand into the three real operands of the
// 3-real-product form (parts: real, imaginary, their sum) in one pass each for
// the scan and the digits; the view is the complex operand (cplx = 1), the
// layout the real one.  maxbits[q] are cleared by the caller.
struct Split3Out {
    uint64_t* maxbits[3];
    int32_t* E[3];
    int8_t* slices[3];
};
hipError_t launch_scan3(const OperandView& op, const Split3Out& o, hipStream_t st);
// Digit planes p_lo .. p_hi - 1 of every part (p_hi < 0: all planes of the
// layout; balanced digits: all planes only).
hipError_t launch_digits3(const OperandView& op, const SliceLayout& lay, const Split3Out& o, hipStream_t st,
                          int p_lo = 0, int p_hi = -1);
// Batched three-part split: one block per item (operand op of the list, block
// coordinates as in the one-operand launches; digits3_blocks gives the grid).
struct Split3Op {
    OperandView op;  // the complex operand
    SliceLayout lay;  // the real layout of each part
    Split3Out o;
};
struct BlockItem;
void digits3_blocks(const SliceLayout& lay, int64_t* bx, int64_t* by);
hipError_t launch_scan3_batched(const Split3Op* ops, const BlockItem* items, int64_t nitems, hipStream_t st);
hipError_t launch_digits3_batched(const Split3Op* ops, const BlockItem* items, int64_t nitems, hipStream_t st);

// Batched split: one block per item; an item names its operand and the block
// coordinates the one-operand launch would have used.
struct SplitOp {
    OperandView op;
    uint64_t* maxbits;
    int32_t* E;
    int8_t* slices;
    SliceLayout lay;
};
struct BlockItem {
    int32_t op;
    int32_t bx;
    int32_t by;
    int32_t pad;
};
void scan_blocks(const OperandView& op, int64_t* bx, int64_t* by);
void digits_blocks(const OperandView& op, const SliceLayout& lay, int64_t* bx, int64_t* by);
hipError_t launch_scan_batched(const SplitOp* ops, const BlockItem* items, int64_t nitems, hipStream_t st);
// prange (device, 2 ints per operand, may be null = all planes): digit planes
// [prange[2 op], prange[2 op + 1]) of operand op; an empty range skips it.
hipError_t launch_digits_batched(const SplitOp* ops, const BlockItem* items, int64_t nitems, hipStream_t st,
                                 const int32_t* prange = nullptr);
// One-pass split (scan and all digit planes of a fixed-s layout) of operands
// whose vectors hold at most 1024 doubles (complex k <= 512, real k <= 1024)
// and whose vectors or terms are contiguous: one block per item (op, by = block
// of 8 of the operand's vectors; fused_split_blocks gives the count).  The
// padding rows of the layout past the last block are not written.
bool split_fusable(const OperandView& op);
void fused_split_blocks(const OperandView& op, int64_t* by);
hipError_t launch_split_fused_batched(const SplitOp* ops, const BlockItem* items, int64_t nitems, hipStream_t st);

// GEMM over slice buffers with fused FP64 epilogue.
struct GemmArgs {
    const int8_t* SA;   // slices of A' (rows_pad = Mp)
    const int8_t* SB;   // slices of B' (rows_pad = Np)
    const int32_t* EA;  // scale exponents of A (per row / complex row)
    const int32_t* FB;  // scale exponents of B (per column)
    int64_t Mp, Np, kpad;
    int64_t chunk_steps;   // MFMA steps (of kStep terms) per INT32 chunk
    int s;                 // slices used: pairs p + q <= s + 1
    int s_lay;             // digit planes in the slice layout (>= s)
    int top;               // 1: only the anti-diagonal d = s + 1 (growth s-1 -> s)
    int cplx;
    int tile;              // 0 auto, 1: 128 x 64 block, 2: 64 x 64 block, 3: per-diagonal streaming
    int mode;              // kFinal, kRawWrite, kRawAdd (see below)
    int bal;               // 0: fold weights 2^(-7d) (truncated digits); 1: 2^(2-8d) (balanced)
    double* acc;           // raw FP64 tile sums acc[col * Mp + row] for the raw modes
    // epilogue
    double* C;
    int64_t ldc;
    int64_t m, n;          // valid output rows (complex rows) and columns
    double alpha_r, alpha_i, beta_r, beta_i;
    int beta_zero;
    // verification mode: write INT32 anti-diagonal sums instead of C
    int32_t* diag_out;
    // kCombine3M: the other two real products (m x n, leading dimension ldt)
    const double* t1;
    const double* t2;
    int64_t ldt;
    // kFinalDD: the low parts of the double-double result (same layout as C)
    double* c_lo;
};
// Epilogue modes: kFinal writes alpha*ldexp(acc, E+F) + beta*C into C; kRawWrite
// stores the FP64 tile sum acc (before ldexp) into g.acc; kRawAdd adds the new
// anti-diagonal terms onto the acc already in g.acc (chunk by chunk);
// kRawWriteFinal does both kRawWrite and kFinal (for beta = 0, where C can be
// rewritten from acc if the slice count grows); kRawAddFinal does both kRawAdd
// and kFinal (a growth step with beta = 0 writes C itself); kCombine3M finishes a complex
// product in the 3-real-product form: this product is T3, t1 / t2 hold T1 / T2,
// and C (complex) receives alpha (T1 - T2 + i ((T3 - T1) - T2)) + beta C;
// kFinalDD (streaming kernel only) folds the anti-diagonal sums into a
// double-double (hi, lo) in the FP64 fold order and writes ldexp(hi, E+F) to C
// and ldexp(lo, E+F) to c_lo (alpha = 1, beta = 0).
constexpr int kFinal = 0, kRawWrite = 1, kRawAdd = 2, kRawWriteFinal = 3, kCombine3M = 4, kFinalDD = 5,
              kRawAddFinal = 6;
hipError_t launch_gemm(const GemmArgs& g, hipStream_t st);

// Batched products: one persistent launch over a list of tiles of many
// problems (all with the same s); tile 1 = 128 x 64 blocks, 2 = 64 x 64.
struct TileItem {
    int32_t prob;
    int32_t tm;
    int32_t tn;
    int32_t s;  // slice count of this tile's problem (read by the mixed-s launch)
};
// Flag in TileItem::s of a mixed-s launch: a 128 x 64 two-tile block (tm in
// units of 128 rows; s <= 6 and one INT32 chunk).
constexpr int32_t kTwoTileItem = 0x100;
hipError_t launch_gemm_persistent(const GemmArgs* probs, const TileItem* items, int64_t nitems, int s, int tile,
                                  int blocks, bool top, bool multi, hipStream_t st);
// Same for any s with the per-diagonal streaming body (64 x 64 tiles).
hipError_t launch_gemm_stream_persistent(const GemmArgs* probs, const TileItem* items, int64_t nitems, int s,
                                         bool top, int blocks, hipStream_t st);
// Tiles of problems with different slice counts (each s <= kMaxLiveSlices, read
// from its GemmArgs) in one persistent launch of 64 x 64 blocks.
hipError_t launch_gemm_persistent_mixed(const GemmArgs* probs, const TileItem* items, int64_t nitems, int blocks,
                                        bool top, bool multi, hipStream_t st);
// Fused 3-real-product tiles of complex products (item.prob: the first of
// three consecutive descriptors T1, T2, T3 of real products): high = false
// for tiles with s <= 6 (two blocks per CU), true for s = 7, 8 (one).
hipError_t launch_gemm_persistent_3m(const GemmArgs* probs, const TileItem* items, int64_t nitems, int blocks,
                                     bool high, hipStream_t st);
// Tiles of problems with 9 <= s <= kMaxWideSlices (each its own s, from the
// tile item) on the wide all-diagonal tile (64 x 64, one block per compute
// unit), over one slice range named by its top s_hi: without multi 9..12
// (s_hi 11 or 12) or 13..14 (s_hi 14); with multi (several INT32 chunks)
// 9..11 (s_hi 11) or 12 (s_hi 12).  Every tile's s must lie in the range.
// Other s_hi: hipErrorInvalidValue.
hipError_t launch_gemm_wide_persistent(const GemmArgs* probs, const TileItem* items, int64_t nitems, int blocks,
                                       bool top, bool multi, int s_hi, hipStream_t st);

// Tolerance-driven calls: operand statistics, residual check, final scaling.
// Per-vector mean square of x * 2^-E (E from maxbits); part: scratch of
// red_entries(nv, k) doubles for the per-chunk partial sums.
hipError_t launch_vec_stats(const OperandView& op, const uint64_t* maxbits, double* ms, double* part, hipStream_t st);
// (chunk, output) entries a split reduction of R outputs over L terms may use.
int64_t red_entries(int64_t R, int64_t L);
// Bytes of each of the two partial-sum buffers of a single-product check
// (and of the statistics pass) of an m x n x k product.
size_t check_part_bytes(int64_t m, int64_t n, int64_t k);
struct CheckArgs {
    OperandView opa, opb;      // op(A) rows and op(B) columns as vectors
    const uint64_t* maxa;      // max |.| bits per row of op(A) / column of op(B)
    const uint64_t* maxb;
    const double* acc;         // raw FP64 tile sums, acc[col * Mp + slice row]
    int64_t Mp;
    const int32_t* EA;
    const int32_t* FB;
    uint64_t seed;             // probe vector seed
    double* t;                 // n      : sigma_j / max|B_:j|
    double* u;                 // 4k     : op(B) t in double-double (re, im)
    double* diff;              // 2m     : y1 - y2
    double* ref;               // 2m     : y2
    double* norms;             // 2      : sum diff^2, sum ref^2
    double* part1;             // check_part_bytes: per-chunk partial sums (single product)
    double* part2;
    // 3-real-product form (z3 = 1, single product): C_emu is formed from the
    // raw sums and scales of T1, T2, T3 (real layout, rows_pad Mp) as
    // (T1 - T2) + i ((T3 - T1) - T2); acc, EA and FB are then unused
    int z3 = 0;
    const double* acc3[3] = {nullptr, nullptr, nullptr};
    const int32_t* EA3[3] = {nullptr, nullptr, nullptr};
    const int32_t* FB3[3] = {nullptr, nullptr, nullptr};
};
hipError_t launch_residual(const CheckArgs& c, hipStream_t st);
hipError_t launch_finalize(const double* acc, int64_t Mp, const int32_t* EA, const int32_t* FB, double* C,
                           int64_t ldc, int64_t m, int64_t n, int cplx, double ar, double ai, double br, double bi,
                           int beta_zero, hipStream_t st);
// The 3-real-product form: C = alpha ((T1 - T2) + i ((T3 - T1) - T2)) + beta C
// with T_q = ldexp(acc_q, E_q + F_q) (NaN where a scale marks Inf/NaN input),
// the arithmetic of the combining GEMM epilogue.
hipError_t launch_finalize3(const double* const* acc3, int64_t Mp, const int32_t* const* EA3,
                            const int32_t* const* FB3, double* C, int64_t ldc, int64_t m, int64_t n, double ar,
                            double ai, double br, double bi, int beta_zero, hipStream_t st);
// Many products: items of the weights (256 columns of op(B) per block), gemv
// (64 terms) and rows (64 rows of op(A)) phases name the product (op) and the
// block (bx); the norms phase runs one block per product.  Products whose
// active flag is 0 are skipped.
hipError_t launch_residual_batched(const CheckArgs* c, int64_t nprob, const int32_t* active, const BlockItem* wt_items,
                                   int64_t n_wt, const BlockItem* gv_items, int64_t n_gv, const BlockItem* row_items,
                                   int64_t n_row, hipStream_t st);
struct FinalArgs {
    const double* acc;
    int64_t Mp;
    const int32_t* EA;
    const int32_t* FB;
    double* C;
    int64_t ldc, m, n;
    int cplx;
    double ar, ai, br, bi;
    int beta_zero;
};
// items: (product, block of 256 rows); every block walks all columns; products
// whose flag is 0 are skipped
hipError_t launch_finalize_batched(const FinalArgs* f, const int32_t* active, const BlockItem* items, int64_t nitems,
                                   hipStream_t st);

// ---- slice-count selection ------------------------------------------------
// Margin of the a-posteriori check: a tolerance-driven call selects its
// starting s for tol / kCheckMargin and grows until the one-probe estimate is
// at most tol / kCheckMargin.  The estimate scatters around the true
// scale-weighted error (measured within 0.70x .. 1.40x of it on the selector's
// instance distribution), so the margin keeps the true error within tol.
constexpr double kCheckMargin = 2.0;

// Rule for the starting slice count of a tolerance-driven call: the
// scale-weighted error of the emulation behaves like
//   eps(s) ~ c (s + 1) 2^(-7s) sqrt((1/M_A + 1/M_B) / 3),
// M = mean over vectors of the mean square of x * 2^-E (truncation leaves
// about 2^-7s per scaled operand entry; the dropped pairs add a term growing
// with s).  c = 2.5 covers the data families measured (0.7 .. 2.0).  The
// smallest s in [1, smax] meeting tol (smax if none; 1 for a zero operand).
// Balanced digits carry one bit more in every slice but the first:
// eps(s) / 2^(s-1).
constexpr double kRuleC = 2.5;
__host__ __device__ inline int rule_slices_of(double ma, double mb, double tol, int smax, bool bal = false) {
    if (!(ma > 0.0) || !(mb > 0.0)) return 1;
    const double spread = sqrt((1.0 / ma + 1.0 / mb) / 3.0);
    int s = 1;
    while (s < smax && kRuleC * (s + 1) * ldexp(1.0, bal ? 1 - 8 * s : -7 * s) * spread > tol) ++s;
    return s;
}

// splitmix64 (Steele, Lea, Flood 2014): output number c (0-based) of the
// stream seeded with key.
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm64_draw(uint64_t key, uint64_t c) { return mix64(key + (c + 1) * kGamma); }

// One operand of a synthetic selector instance (see oz.h, oz_gen_t).
struct GenSide {
    double* X;
    int64_t rows, cols, ld;
    uint64_t ekey, vkey;   // entry stream, vector-exponent stream
    int vec_axis;          // 0: vectors are rows (A), 1: columns (B)
    int sig_el, sig_vec, bits, family;
    int64_t zero_q;
};
hipError_t launch_gen(const GenSide& g, hipStream_t st);

// Exponent statistics of one operand: per-vector mean square of x 2^-E and
// histograms of the gap g = E - exponent(x) and the width w = g + bit length
// of the odd significand of x (both capped at kHistCap) over its non-zero
// entries, plus the zero count.
constexpr int kHistCap = 127;
constexpr int kHistBins = kHistCap + 1;
constexpr int kHistLen = 2 * kHistBins + 1;  // [g bins | w bins | zeros]
struct StatSide {
    OperandView op;
    const uint64_t* maxbits;
    double* msq;                 // nv
    unsigned long long* hist;    // kHistLen, cleared by the caller
};
void stat_blocks(const OperandView& op, int64_t* blocks);
hipError_t launch_stats(const StatSide& s, hipStream_t st);
hipError_t launch_stats_batched(const StatSide* sides, const BlockItem* items, int64_t nitems, hipStream_t st);

// The 16 selector features of one product (rows for ntol tolerances), the
// rule's slice count per row, and (with an error table) the label per row.
constexpr int kNumFeat = 16;
struct FeatProb {
    const double* msq[2];
    const unsigned long long* hist[2];
    int64_t nv[2];
    int64_t m, n, k;
    int cplx;
    int ntol;
    const double* tols;     // ntol
    float* feat;            // ntol x kNumFeat
    int32_t* s_rule;        // ntol (may be null)
    int smax;
    const double* eps;      // s_ref entries, eps of s = 1..s_ref (may be null)
    int s_ref;
    float* label;           // ntol (with eps)
    double* mstat;          // 2: M_A, M_B (may be null)
};
hipError_t launch_features(const FeatProb* probs, int64_t nprob, hipStream_t st);

// Error table of a labelled instance from the INT32 anti-diagonal sums of the
// s_ref emulation (one chunk): eps_s = ||W o (C_s - C_ref)||_F / ||W o C_ref||_F.
constexpr int kMaxRef = 18;
hipError_t launch_eps_table(const int32_t* diag, int64_t Mp, int64_t Np, int s_ref, const int32_t* EA,
                            const int32_t* FB, const uint64_t* maxa, const uint64_t* maxb, int64_t m, int64_t n,
                            double* partial, double* eps, hipStream_t st);
int64_t eps_partial_len(int64_t m, int64_t n);

// C = beta*C for the alpha == 0 / k == 0 quick return.
hipError_t launch_scale_c(double* C, int64_t ldc, int64_t m, int64_t n, int cplx, double br, double bi,
                          int beta_zero, hipStream_t st);

}  // namespace oz
