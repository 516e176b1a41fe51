// oz_split.hip -- scale exponents and INT8 digits of one operand (the
// splitting step of the Ozaki scheme, paper Sec. 2.2).
//
// Pure integer work on the IEEE-754 bit pattern: no FP64 arithmetic runs
// here.  Two passes, both bound by HBM bandwidth:
//   scan   : per vector (row of op(A) / column of op(B)) the largest magnitude
//            as raw bits; the unsigned order of |x| bit patterns is the order
//            of |x|, so a max over uint64 is the max over values (atomicMax
//            merges the partial maxima of a 2-D grid).
//   digits : E = frexp exponent of that maximum; digit p of x is
//            floor(|x| * 2^(7p - E)) mod 128 with the sign of x, read off the
//            53-bit significand by one shift; written in the K-blocked slice
//            layout the GEMM kernel streams (see oz.h).
#include "oz_internal.h"

namespace oz {

namespace {

constexpr uint64_t kMagMask = 0x7fffffffffffffffull;
constexpr uint64_t kMantMask = (1ull << 52) - 1;
constexpr uint64_t kInfBits = 0x7ff0000000000000ull;

__device__ __forceinline__ uint64_t mag_bits(double x) {
    return static_cast<uint64_t>(__double_as_longlong(x)) & kMagMask;
}

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// frexp exponent of the value whose magnitude bits are b (b finite, nonzero).
__device__ __forceinline__ int frexp_exp_bits(uint64_t b) {
    int eb = static_cast<int>(b >> 52);
    if (eb > 0) return eb - 1022;
    // subnormal: value = mant * 2^-1074, frexp exponent = bitlength(mant) - 1074
    return (64 - __clzll(static_cast<long long>(b & kMantMask))) - 1074;
}

__device__ __forceinline__ int32_t exponent_of_max(uint64_t b) {
    if (b == 0) return 0;
    if (b >= kInfBits) return kNonFiniteExp;
    return frexp_exp_bits(b);
}

// Digit decomposition of one double under scale exponent E.
struct Sig {
    uint64_t M;  // significand as an integer (with the hidden bit when normal)
    int sh0;     // right shift giving floor(|x| * 2^-E) scaled by 2^0 ... see digit()
    bool neg;
};

__device__ __forceinline__ Sig sig_of(double x, int E) {
    uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    Sig g;
    g.neg = (b >> 63) != 0;
    uint64_t mag = b & kMagMask;
    int eb = static_cast<int>(mag >> 52);
    g.M = (mag & kMantMask) | (eb ? (1ull << 52) : 0ull);
    int e_eff = eb ? eb : 1;  // |x| = M * 2^(e_eff - 1075)
    // digit p = floor(M * 2^(e_eff - 1075 + 7p - E)) mod 128: right shift by sh0 - 7p
    g.sh0 = 1075 + E - e_eff;
    return g;
}

__device__ __forceinline__ int digit(const Sig& g, int p /* 1-based */) {
    int sh = g.sh0 - 7 * p;
    uint32_t t;
    if (sh >= 64)
        t = 0;
    else if (sh >= 0)
        t = static_cast<uint32_t>(g.M >> sh) & 127u;
    else if (sh > -7)
        t = static_cast<uint32_t>(g.M << (-sh)) & 127u;
    else
        t = 0;
    return g.neg ? -static_cast<int>(t) : static_cast<int>(t);
}

// The first 64 fractional bits of |x| * 2^-E, floor(M * 2^(64 - sh0)): digit
// p <= 9 is bits [64 - 7p, 71 - 7p) of it (one shift and mask per digit).
// |x| < 2^E gives sh0 >= 53 for a normal x (a left shift of at most 11) and
// sh0 >= bitlength(M) for a subnormal one, so the left shift never overflows.
constexpr int kWindowDigits = 9;
__device__ __forceinline__ uint64_t frac_window(const Sig& g) {
    const int sh = g.sh0 - 64;
    if (sh >= 64) return 0;
    if (sh >= 0) return g.M >> sh;
    return g.M << (-sh);
}

// Digit p (1-based) of x under scale exponent E; W = frac_window(sig_of(x, E)).
// Digits past the window are taken from the significand again.
__device__ __forceinline__ int digit_of(double x, int E, uint64_t W, int p) {
    if (p > kWindowDigits) return digit(sig_of(x, E), p);
    const int t = static_cast<int>(static_cast<uint32_t>(W >> (64 - 7 * p)) & 127u);
    return __double_as_longlong(x) < 0 ? -t : t;
}

// Balanced (round-to-nearest) digits, s <= 8.  The vector exponent is E' =
// E, or E + 1 when its largest magnitude M has M * 2^(7-E) > 127 (so that the
// top digit stays within [-127, 127]); N = |x| * 2^(7 - E' + 8(s-1)) rounded to
// the nearest integer (ties away from zero) with the sign of x -- one shift of
// the significand, N below 2^63 -- then the s digits are N's bytes read as
// signed digits (see balanced_digit), the top digit taking the rest.
__device__ __forceinline__ int balanced_bump(uint64_t maxb, int E) {
    // M * 2^(7-E) > 127 with M = Mi * 2^(e_eff - 1075): Mi > 127 * 2^(sh0 - 7)
    if (maxb == 0 || maxb >= kInfBits) return 0;
    const Sig g = sig_of(__longlong_as_double(static_cast<long long>(maxb)), E);
    // sh0 is 53 for a normal M and its bit length for a subnormal one; below 7,
    // M * 2^(7-E) = Mi * 2^(7-sh0) is an integer below 128, so at most 127
    if (g.sh0 < 7) return 0;
    return g.M > (127ull << (g.sh0 - 7)) ? 1 : 0;
}

__device__ __forceinline__ int64_t balanced_int(double x, int E, int s) {
    const Sig g = sig_of(x, E);
    const int sh = g.sh0 - 7 - 8 * (s - 1);
    uint64_t n;
    if (sh <= 0)
        n = g.M << (-sh);
    else if (sh <= 54)
        n = (g.M + (1ull << (sh - 1))) >> sh;  // M < 2^53: no overflow
    else
        n = 0;  // M < 2^53 < 2^(sh-1): below one half
    return g.neg ? -static_cast<int64_t>(n) : static_cast<int64_t>(n);
}

// The digits of N all at once: with C = 0x80...80 over the s - 1 low bytes,
// N + C = sum_{p>=2} (d_p + 128) 256^(s-p) + d_1 256^(s-1) with every
// d_p + 128 in [0, 255], so plane p >= 1 (0-based) is byte s-1-p of N + C
// minus 128 and plane 0 is N + C shifted right by 8(s-1) (arithmetic).
// |N| <= 127 * 256^(s-1) keeps N + C below 2^63.
__device__ __forceinline__ int64_t balanced_bias(int s) {
    return static_cast<int64_t>(0x0080808080808080ull >> (8 * (8 - s)));
}

__device__ __forceinline__ int balanced_digit(int64_t nb, int p, int s) {
    if (p == 0) return static_cast<int>(nb >> (8 * (s - 1)));
    return static_cast<int>((static_cast<uint64_t>(nb) >> (8 * (s - 1 - p))) & 255u) - 128;
}

__global__ void zero_u64_kernel(uint64_t* p, int64_t n) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// One block: 64 vectors x lspan terms.
// LCONTIG: terms of a vector are contiguous (sl == 1): each wave walks 16
//          vectors, 4 at a time with 16 lanes each reading 16 consecutive
//          terms (a 16-lane reduction per vector instead of a 64-lane one).
// else   : vectors are contiguous (sv == 1): lane = vector, the 4 waves
//          split the terms, partial maxima merged through LDS.
template <bool LCONTIG, bool CPLX>
__device__ __forceinline__ void scan_body(const OperandView& op, uint64_t* maxbits, int64_t lspan, int64_t bx,
                                          int64_t by) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t v0 = by * 64;
    const int64_t l0 = bx * lspan;
    const int64_t l1 = (l0 + lspan < op.k) ? l0 + lspan : op.k;
    const int w = CPLX ? 2 : 1;
    if (LCONTIG) {
        // 16 lanes per vector, 4 vectors of the wave's 16 at a time
        const int grp = lane >> 4, gl = lane & 15;
        for (int r = 0; r < 4; ++r) {
            const int64_t v = v0 + wave * 16 + r * 4 + grp;
            uint64_t mx = 0;
            if (v < op.nv) {
                const double* base = op.X + v * op.sv * w;
                for (int64_t l = l0 + gl; l < l1; l += 16) {
                    mx = umax64(mx, mag_bits(base[l * w]));
                    if (CPLX) mx = umax64(mx, mag_bits(base[l * w + 1]));
                }
            }
            for (int off = 8; off > 0; off >>= 1) mx = umax64(mx, __shfl_xor(mx, off));
            if (gl == 0 && v < op.nv && mx != 0) atomicMax(reinterpret_cast<unsigned long long*>(maxbits + v), mx);
        }
    } else {
        __shared__ uint64_t red[4][64];
        const int64_t v = v0 + lane;
        uint64_t mx = 0;
        if (v < op.nv) {
            for (int64_t l = l0 + wave; l < l1; l += 4) {
                const double* e = op.X + (v + l * op.sl) * w;
                mx = umax64(mx, mag_bits(e[0]));
                if (CPLX) mx = umax64(mx, mag_bits(e[1]));
            }
        }
        red[wave][lane] = mx;
        __syncthreads();
        if (wave == 0 && v < op.nv) {
            mx = umax64(umax64(red[0][lane], red[1][lane]), umax64(red[2][lane], red[3][lane]));
            if (mx != 0) atomicMax(reinterpret_cast<unsigned long long*>(maxbits + v), mx);
        }
    }
}

template <bool LCONTIG, bool CPLX>
__global__ __launch_bounds__(256) void scan_kernel(OperandView op, uint64_t* maxbits, int64_t lspan) {
    scan_body<LCONTIG, CPLX>(op, maxbits, lspan, blockIdx.x, blockIdx.y);
}

// Slice byte offset of (term t, digit p 0-based, vector r) in the layout of oz.h.
__device__ __forceinline__ int64_t slice_off(int64_t t, int p, int64_t r, int s, int64_t rows_pad) {
    return (((t >> 4) * s + p) * rows_pad + r) * 16 + (t & 15);
}

__device__ __forceinline__ uint64_t pack8(const int* d) {
    uint64_t r = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) r |= static_cast<uint64_t>(static_cast<uint8_t>(static_cast<int8_t>(d[i]))) << (8 * i);
    return r;
}

// Digits of the 8 terms t0 .. t0+7 of vector v (x: 8 real elements, or 4
// complex elements as (re, im) pairs; zeros for a non-finite vector or past k)
// under scale exponent ex, written as one 8-byte chunk per digit plane (and
// per row of the two-row form); planes p_lo .. p_hi - 1 (balanced digits: all
// p_hi planes of an s = p_hi split).
template <bool CPLX, bool SIDE_A, bool BAL>
__device__ __forceinline__ void emit_digits(const double (&x)[8], int32_t ex, int64_t v, int64_t t0,
                                            const SliceLayout& lay, int8_t* slices, int p_lo, int p_hi) {
    if constexpr (BAL) {
        // all p_hi planes at once (p_lo = 0): the digits of an s = p_hi split
        // (a tolerance-driven plan lays out more planes than it fills)
        const int s = p_hi;
        if (CPLX && SIDE_A) {
            const int64_t r_re = 32 * (v >> 4) + 16 * ((v >> 3) & 1) + (v & 7);
            const int64_t r_im = r_re + 8;
            if (r_re >= lay.rows_pad) return;
            // real-part row (ar, -ai): the digits of the value -ai are those of -N(ai)
            const int64_t bias = balanced_bias(s);
            int64_t nr[4], ni[4], nn[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t r = balanced_int(x[2 * e], ex, s), i = balanced_int(x[2 * e + 1], ex, s);
                nr[e] = r + bias;
                ni[e] = i + bias;
                nn[e] = bias - i;
            }
            for (int p = 0; p < s; ++p) {
                int dre[8], dim[8];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ar = balanced_digit(nr[e], p, s);
                    const int ai = balanced_digit(ni[e], p, s);
                    const int an = balanced_digit(nn[e], p, s);
                    dre[2 * e] = ar;
                    dre[2 * e + 1] = an;
                    dim[2 * e] = ai;
                    dim[2 * e + 1] = ar;
                }
                *reinterpret_cast<uint64_t*>(slices + slice_off(t0, p, r_re, lay.s, lay.rows_pad)) = pack8(dre);
                *reinterpret_cast<uint64_t*>(slices + slice_off(t0, p, r_im, lay.s, lay.rows_pad)) = pack8(dim);
            }
        } else {
            if (v >= lay.rows_pad) return;
            const int64_t bias = balanced_bias(s);
            int64_t nv8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) nv8[e] = balanced_int(x[e], ex, s) + bias;
            for (int p = 0; p < s; ++p) {
                int d[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) d[e] = balanced_digit(nv8[e], p, s);
                *reinterpret_cast<uint64_t*>(slices + slice_off(t0, p, v, lay.s, lay.rows_pad)) = pack8(d);
            }
        }
        return;
    }

    uint64_t w[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = frac_window(sig_of(x[e], ex));

    if (CPLX && SIDE_A) {
        // real-part row holds (ar, -ai), imaginary-part row holds (ai, ar)
        const int64_t r_re = 32 * (v >> 4) + 16 * ((v >> 3) & 1) + (v & 7);
        const int64_t r_im = r_re + 8;
        if (r_re >= lay.rows_pad) return;
        for (int p = p_lo; p < p_hi; ++p) {
            int dre[8], dim[8];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ar = digit_of(x[2 * e], ex, w[2 * e], p + 1);
                const int ai = digit_of(x[2 * e + 1], ex, w[2 * e + 1], p + 1);
                dre[2 * e] = ar;
                dre[2 * e + 1] = -ai;
                dim[2 * e] = ai;
                dim[2 * e + 1] = ar;
            }
            *reinterpret_cast<uint64_t*>(slices + slice_off(t0, p, r_re, lay.s, lay.rows_pad)) = pack8(dre);
            *reinterpret_cast<uint64_t*>(slices + slice_off(t0, p, r_im, lay.s, lay.rows_pad)) = pack8(dim);
        }
    } else {
        if (v >= lay.rows_pad) return;
        for (int p = p_lo; p < p_hi; ++p) {
            int d[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) d[e] = digit_of(x[e], ex, w[e], p + 1);
            *reinterpret_cast<uint64_t*>(slices + slice_off(t0, p, v, lay.s, lay.rows_pad)) = pack8(d);
        }
    }
}

// One block: 64 vectors (64 complex rows for a complex side-'A' operand) x one
// MFMA step of 32 terms.  Each thread owns 8 consecutive terms of one vector:
// 8 real elements, or 4 complex elements (terms 2l, 2l+1).
template <bool LCONTIG, bool CPLX, bool SIDE_A, bool BAL = false>
__device__ __forceinline__ void digits_body(const OperandView& op, const uint64_t* maxbits, const SliceLayout& lay,
                                            int32_t* E, int8_t* slices, int64_t bx, int64_t by, int p_lo, int p_hi) {
    const int tid = threadIdx.x;
    const int vi = LCONTIG ? (tid >> 2) : (tid & 63);
    const int sub = LCONTIG ? (tid & 3) : (tid >> 6);
    const int64_t v = by * 64 + vi;
    const int64_t step = bx;
    const int64_t t0 = step * kStep + sub * 8;  // first term of this thread
    const bool live = v < op.nv;

    int32_t ex = 0;
    if (live) ex = exponent_of_max(maxbits[v]);
    const bool bad = ex == kNonFiniteExp;
    if constexpr (BAL)
        if (live && !bad) ex += balanced_bump(maxbits[v], ex);
    if (live && step == 0 && sub == 0) E[v] = ex;

    // 8 doubles: real -> elements l = t0 .. t0+7; complex -> l = t0/2 .. t0/2+3 (re, im)
    double x[8];
    constexpr int NEL = CPLX ? 4 : 8;
    const int64_t lbase = CPLX ? t0 / 2 : t0;
#pragma unroll
    for (int e = 0; e < NEL; ++e) {
        const int64_t l = lbase + e;
        double re = 0.0, im = 0.0;
        if (live && !bad && l < op.k) {
            const double* src = op.X + (v * op.sv + l * op.sl) * (CPLX ? 2 : 1);
            re = src[0];
            if (CPLX) im = op.conj ? -src[1] : src[1];
        }
        if (CPLX) {
            x[2 * e] = re;
            x[2 * e + 1] = im;
        } else {
            x[e] = re;
        }
    }
    emit_digits<CPLX, SIDE_A, BAL>(x, ex, v, t0, lay, slices, p_lo, p_hi);
}

template <bool LCONTIG, bool CPLX, bool SIDE_A, bool BAL>
__global__ __launch_bounds__(256) void digits_kernel(OperandView op, const uint64_t* maxbits, SliceLayout lay,
                                                     int32_t* E, int8_t* slices, int p_lo, int p_hi) {
    digits_body<LCONTIG, CPLX, SIDE_A, BAL>(op, maxbits, lay, E, slices, blockIdx.x, blockIdx.y, p_lo, p_hi);
}

// Batched forms: block b runs item b of a list naming the operand and the
// block coordinates its one-operand launch would have had.
__global__ __launch_bounds__(256) void scan_batched_kernel(const SplitOp* __restrict__ ops,
                                                           const BlockItem* __restrict__ items, int64_t lspan) {
    const BlockItem it = items[blockIdx.x];
    const SplitOp& o = ops[it.op];
    const bool lc = o.op.sl == 1;
    if (lc && o.op.cplx) scan_body<true, true>(o.op, o.maxbits, lspan, it.bx, it.by);
    else if (lc) scan_body<true, false>(o.op, o.maxbits, lspan, it.bx, it.by);
    else if (o.op.cplx) scan_body<false, true>(o.op, o.maxbits, lspan, it.bx, it.by);
    else scan_body<false, false>(o.op, o.maxbits, lspan, it.bx, it.by);
}

__global__ __launch_bounds__(256) void digits_batched_kernel(const SplitOp* __restrict__ ops,
                                                             const BlockItem* __restrict__ items,
                                                             const int32_t* __restrict__ prange) {
    const BlockItem it = items[blockIdx.x];
    const SplitOp& o = ops[it.op];
    const int p_lo = prange ? prange[2 * it.op] : 0, p_hi = prange ? prange[2 * it.op + 1] : o.lay.s;
    if (p_lo >= p_hi) return;  // nothing to split for this operand (uniform over the block)
    const bool lc = o.op.sl == 1, two_row = o.op.cplx && o.op.side_a;
    // balanced operands (fixed s only) fill all their planes: p_lo = 0, p_hi = s
#define OZ_DB(LC, CP, SA)                                                                                   \
    do {                                                                                                    \
        if (o.lay.bal)                                                                                      \
            digits_body<LC, CP, SA, true>(o.op, o.maxbits, o.lay, o.E, o.slices, it.bx, it.by, 0, o.lay.s); \
        else                                                                                                \
            digits_body<LC, CP, SA>(o.op, o.maxbits, o.lay, o.E, o.slices, it.bx, it.by, p_lo, p_hi);       \
    } while (0)
    if (lc) {
        if (two_row) OZ_DB(true, true, true);
        else if (o.op.cplx) OZ_DB(true, true, false);
        else OZ_DB(true, false, false);
    } else {
        if (two_row) OZ_DB(false, true, true);
        else if (o.op.cplx) OZ_DB(false, true, false);
        else OZ_DB(false, false, false);
    }
#undef OZ_DB
}

// ---- one-pass split of short vectors ----------------------------------------
// Block = kFuseV vectors, each at most kFuseMaxDoubles doubles long (complex
// k <= 512, real k <= 1024): the vectors are read once from HBM into LDS
// (consecutive lanes on consecutive doubles of a vector when its terms are
// contiguous, on consecutive vectors otherwise), the per-vector maxima are
// taken from LDS, and the digits are emitted from LDS with the arithmetic of
// digits_body (emit_digits): the FP64 operand is read once instead of twice.
// Threads of the digit phase: (vector v, 8-term half h, 16-term chunk c) with v
// fastest, so the chunks of the block's rows for one (c, plane) are one
// contiguous run of 16-byte rows.
constexpr int kFuseV = 4;
constexpr int kFuseMaxDoubles = 1024;
constexpr int kFuseRow = kFuseMaxDoubles + 2;  // LDS doubles per staged vector (+2 spreads the banks)

template <bool LCONTIG, bool CPLX, bool SIDE_A, bool BAL>
__device__ __forceinline__ void fused_split_body(const SplitOp& o, int64_t by, double* stage, uint64_t* vmax) {
    const OperandView& op = o.op;
    const int tid = threadIdx.x;
    constexpr int W = CPLX ? 2 : 1;  // doubles per element
    const int64_t K = op.k;
    const int64_t v0 = by * kFuseV;
    const int nvb = op.nv - v0 < kFuseV ? static_cast<int>(op.nv - v0 > 0 ? op.nv - v0 : 0) : kFuseV;
    // phase 1: stage the block's vectors, stage[v * kFuseRow + l * W + part];
    // each thread owns kLoads doubles, all loaded before any is stored so that
    // the loads are in flight together
    constexpr int kLoads = kFuseV * kFuseMaxDoubles / 256;
    double buf[kLoads];
    static_assert(kFuseMaxDoubles == 4 * 256 && kFuseV * 4 == kLoads, "4 doubles of a vector per thread");
    if constexpr (LCONTIG) {
        // double i of the thread: vector i / 4, double tid + 256 (i % 4) of it
#pragma unroll
        for (int i = 0; i < kLoads; ++i) {
            const int v = i >> 2;
            const int64_t d = tid + 256 * (i & 3);
            buf[i] = (v < nvb && d < K * W) ? op.X[(v0 + v) * op.sv * W + d] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kLoads; ++i) {
            const int64_t d = tid + 256 * (i & 3);
            if (d < K * W) stage[(i >> 2) * kFuseRow + d] = buf[i];
        }
    } else {
        // kFuseV consecutive vectors of one term are contiguous (sv == 1):
        // double i of the thread is term lo + LPER i of vector v, part `part`
        constexpr int LPER = 256 / (kFuseV * W);  // terms per pass
        const int part = tid % W, v = (tid / W) % kFuseV, lo = tid / (kFuseV * W);
#pragma unroll
        for (int i = 0; i < kLoads; ++i) {
            const int64_t l = lo + static_cast<int64_t>(LPER) * i;
            buf[i] = (v < nvb && l < K) ? op.X[(v0 + v + l * op.sl) * W + part] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kLoads; ++i) {
            const int64_t l = lo + static_cast<int64_t>(LPER) * i;
            if (l < K) stage[v * kFuseRow + l * W + part] = buf[i];
        }
    }
    __syncthreads();
    // per-vector max of |x| bits: TPV threads per vector
    {
        constexpr int TPV = 256 / kFuseV;
        const int v = tid / TPV, j = tid % TPV;
        uint64_t mx = 0;
        for (int64_t d = j; d < K * W; d += TPV) mx = umax64(mx, mag_bits(stage[v * kFuseRow + d]));
        for (int off = TPV / 2; off > 0; off >>= 1) mx = umax64(mx, __shfl_xor(mx, off, TPV));
        if (j == 0) {
            vmax[v] = mx;
            if (v < nvb) o.maxbits[v0 + v] = mx;
        }
    }
    __syncthreads();
    // phase 2: digits from LDS
    const int v = tid % kFuseV, h = (tid / kFuseV) & 1;
    const int64_t vg = v0 + v;
    const bool live = v < nvb;
    int32_t ex = 0;
    if (live) ex = exponent_of_max(vmax[v]);
    const bool bad = ex == kNonFiniteExp;
    if constexpr (BAL)
        if (live && !bad) ex += balanced_bump(vmax[v], ex);
    if (live && tid < kFuseV) o.E[vg] = ex;
    const bool take = live && !bad;
    const int64_t nchunks = o.lay.kpad / 16;
    for (int64_t c = tid / (2 * kFuseV); c < nchunks; c += 256 / (2 * kFuseV)) {
        const int64_t t0 = c * 16 + h * 8;
        double x[8];
        constexpr int NEL = CPLX ? 4 : 8;
        const int64_t lbase = CPLX ? t0 / 2 : t0;
#pragma unroll
        for (int e = 0; e < NEL; ++e) {
            const int64_t l = lbase + e;
            double re = 0.0, im = 0.0;
            if (take && l < K) {
                re = stage[v * kFuseRow + l * W];
                if (CPLX) im = op.conj ? -stage[v * kFuseRow + l * W + 1] : stage[v * kFuseRow + l * W + 1];
            }
            if (CPLX) {
                x[2 * e] = re;
                x[2 * e + 1] = im;
            } else {
                x[e] = re;
            }
        }
        emit_digits<CPLX, SIDE_A, BAL>(x, ex, vg, t0, o.lay, o.slices, 0, o.lay.s);
    }
}

__global__ __launch_bounds__(256) void split_fused_batched_kernel(const SplitOp* __restrict__ ops,
                                                                  const BlockItem* __restrict__ items) {
    __shared__ double stage[kFuseV * kFuseRow];
    __shared__ uint64_t vmax[kFuseV];
    const BlockItem it = items[blockIdx.x];
    const SplitOp& o = ops[it.op];
    const bool lc = o.op.sl == 1, two_row = o.op.cplx && o.op.side_a;  // uniform over the block
#define OZ_FS(LC, CP, SA)                                                                  \
    do {                                                                                   \
        if (o.lay.bal) fused_split_body<LC, CP, SA, true>(o, it.by, stage, vmax);          \
        else fused_split_body<LC, CP, SA, false>(o, it.by, stage, vmax);                   \
    } while (0)
    if (lc) {
        if (two_row) OZ_FS(true, true, true);
        else if (o.op.cplx) OZ_FS(true, true, false);
        else OZ_FS(true, false, false);
    } else {
        if (two_row) OZ_FS(false, true, true);
        else if (o.op.cplx) OZ_FS(false, true, false);
        else OZ_FS(false, false, false);
    }
#undef OZ_FS
}

// ---- three real operands of one complex operand in one pass ---------------
// Parts q = 0, 1, 2: the real parts, the imaginary parts (negated for 'C')
// and their FP64 sums, each a real operand with its own scales and slices
// (the complex product in its 3-real-product form).
__device__ __forceinline__ void parts3(const OperandView& op, const double* e, double (&x)[3]) {
    const double re = e[0], im = op.conj ? -e[1] : e[1];
    x[0] = re;
    x[1] = im;
    x[2] = re + im;
}

template <bool LCONTIG>
__device__ __forceinline__ void scan3_body(const OperandView& op, const Split3Out& o, int64_t lspan, int64_t bx,
                                           int64_t by) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t v0 = by * 64;
    const int64_t l0 = bx * lspan;
    const int64_t l1 = (l0 + lspan < op.k) ? l0 + lspan : op.k;
    if (LCONTIG) {
        // 16 lanes per vector, 4 vectors of the wave's 16 at a time
        const int grp = lane >> 4, gl = lane & 15;
        for (int r = 0; r < 4; ++r) {
            const int64_t v = v0 + wave * 16 + r * 4 + grp;
            uint64_t mx[3] = {0, 0, 0};
            if (v < op.nv) {
                const double* base = op.X + v * op.sv * 2;
                for (int64_t l = l0 + gl; l < l1; l += 16) {
                    double x[3];
                    parts3(op, base + l * 2, x);
#pragma unroll
                    for (int q = 0; q < 3; ++q) mx[q] = umax64(mx[q], mag_bits(x[q]));
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                for (int off = 8; off > 0; off >>= 1) mx[q] = umax64(mx[q], __shfl_xor(mx[q], off));
                if (gl == 0 && v < op.nv && mx[q] != 0)
                    atomicMax(reinterpret_cast<unsigned long long*>(o.maxbits[q] + v), mx[q]);
            }
        }
    } else {
        __shared__ uint64_t red[3][4][64];
        const int64_t v = v0 + lane;
        uint64_t mx[3] = {0, 0, 0};
        if (v < op.nv) {
            for (int64_t l = l0 + wave; l < l1; l += 4) {
                double x[3];
                parts3(op, op.X + (v + l * op.sl) * 2, x);
#pragma unroll
                for (int q = 0; q < 3; ++q) mx[q] = umax64(mx[q], mag_bits(x[q]));
            }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) red[q][wave][lane] = mx[q];
        __syncthreads();
        if (wave == 0 && v < op.nv) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const uint64_t m = umax64(umax64(red[q][0][lane], red[q][1][lane]), umax64(red[q][2][lane], red[q][3][lane]));
                if (m != 0) atomicMax(reinterpret_cast<unsigned long long*>(o.maxbits[q] + v), m);
            }
        }
    }
}

template <bool LCONTIG>
__global__ __launch_bounds__(256) void scan3_kernel(OperandView op, Split3Out o, int64_t lspan) {
    scan3_body<LCONTIG>(op, o, lspan, blockIdx.x, blockIdx.y);
}

// One block: 64 vectors x one step of 32 terms; each thread owns 8 consecutive
// terms (complex elements) of one vector and writes them into all three parts.
// Contiguous terms: the block's 64 x 32 elements are first read with 32
// neighbouring lanes per vector (512 contiguous bytes) into LDS; each thread
// then takes its 8 elements from there (a direct read would have every lane
// of a load touch its own 128-byte line).
template <bool LCONTIG, bool BAL>
__device__ __forceinline__ void digits3_body(const OperandView& op, const SliceLayout& lay, const Split3Out& o,
                                             int64_t bx, int64_t by, int p_lo = 0, int p_hi = -1) {
    // truncated digits: planes p_lo .. p_hi - 1 (all with p_hi < 0); balanced
    // digits depend on s and are written all at once
    if (p_hi < 0) p_hi = lay.s;
    constexpr int kStagePad = 33;  // 16-byte entries per staged vector: 32 elements + 1 to spread LDS banks
    __shared__ double2 stage[LCONTIG ? 64 * kStagePad : 1];
    if constexpr (LCONTIG) {
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int idx = it * 256 + static_cast<int>(threadIdx.x);
            const int sv = idx >> 5, se = idx & 31;
            const int64_t vv = by * 64 + sv;
            const int64_t l = bx * kStep + se;
            double2 val = make_double2(0.0, 0.0);
            if (vv < op.nv && l < op.k) {
                const double* src = op.X + (vv * op.sv + l) * 2;
                val = make_double2(src[0], src[1]);
            }
            stage[sv * kStagePad + se] = val;
        }
        __syncthreads();
    }
    const int tid = threadIdx.x;
    const int vi = LCONTIG ? (tid >> 2) : (tid & 63);
    const int sub = LCONTIG ? (tid & 3) : (tid >> 6);
    const int64_t v = by * 64 + vi;
    const int64_t step = bx;
    const int64_t t0 = step * kStep + sub * 8;
    const bool live = v < op.nv;
    if (v >= lay.rows_pad) return;
    int32_t ex[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (live) ex[q] = exponent_of_max(o.maxbits[q][v]);
        if constexpr (BAL)
            if (live && ex[q] != kNonFiniteExp) ex[q] += balanced_bump(o.maxbits[q][v], ex[q]);
        if (live && step == 0 && sub == 0) o.E[q][v] = ex[q];
    }
    // the 8 complex elements of this thread, read once
    double re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t l = t0 + e;
        double px[3] = {0.0, 0.0, 0.0};
        if (live && l < op.k) {
            if constexpr (LCONTIG) {
                const double2 val = stage[vi * kStagePad + sub * 8 + e];
                const double pair[2] = {val.x, val.y};
                parts3(op, pair, px);
            } else {
                parts3(op, op.X + (v * op.sv + l * op.sl) * 2, px);
            }
        }
        re[e] = px[0];
        im[e] = px[1];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const bool bad = ex[q] == kNonFiniteExp;
        double x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)  // part 2 is the FP64 sum of the two parts (as in the scan)
            x[e] = bad ? 0.0 : (q == 0 ? re[e] : q == 1 ? im[e] : re[e] + im[e]);
        if constexpr (BAL) {
            // balanced digits (no part is negated in this form)
            const int64_t bias = balanced_bias(lay.s);
            int64_t nv8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) nv8[e] = balanced_int(x[e], ex[q], lay.s) + bias;
            for (int p = 0; p < lay.s; ++p) {
                int d[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) d[e] = balanced_digit(nv8[e], p, lay.s);
                *reinterpret_cast<uint64_t*>(o.slices[q] + slice_off(t0, p, v, lay.s, lay.rows_pad)) = pack8(d);
            }
            continue;
        }
        uint64_t w[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = frac_window(sig_of(x[e], ex[q]));
        for (int p = p_lo; p < p_hi; ++p) {
            int d[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) d[e] = digit_of(x[e], ex[q], w[e], p + 1);
            *reinterpret_cast<uint64_t*>(o.slices[q] + slice_off(t0, p, v, lay.s, lay.rows_pad)) = pack8(d);
        }
    }
}

template <bool LCONTIG, bool BAL>
__global__ __launch_bounds__(256) void digits3_kernel(OperandView op, SliceLayout lay, Split3Out o, int p_lo,
                                                      int p_hi) {
    digits3_body<LCONTIG, BAL>(op, lay, o, blockIdx.x, blockIdx.y, p_lo, p_hi);
}

// Batched three-part split: block b runs item b (operand, block coordinates).
__global__ __launch_bounds__(256) void scan3_batched_kernel(const Split3Op* __restrict__ ops,
                                                            const BlockItem* __restrict__ items, int64_t lspan) {
    const BlockItem it = items[blockIdx.x];
    const Split3Op& o = ops[it.op];
    if (o.op.sl == 1) scan3_body<true>(o.op, o.o, lspan, it.bx, it.by);
    else scan3_body<false>(o.op, o.o, lspan, it.bx, it.by);
}

__global__ __launch_bounds__(256) void digits3_batched_kernel(const Split3Op* __restrict__ ops,
                                                              const BlockItem* __restrict__ items) {
    const BlockItem it = items[blockIdx.x];
    const Split3Op& o = ops[it.op];
    const bool lc = o.op.sl == 1;  // uniform over the block
    if (o.lay.bal) {
        if (lc) digits3_body<true, true>(o.op, o.lay, o.o, it.bx, it.by);
        else digits3_body<false, true>(o.op, o.lay, o.o, it.bx, it.by);
    } else {
        if (lc) digits3_body<true, false>(o.op, o.lay, o.o, it.bx, it.by);
        else digits3_body<false, false>(o.op, o.lay, o.o, it.bx, it.by);
    }
}

}  // namespace

// Terms per exponent-scan block: 128 gives n = 4096 operands 2048 blocks of 64
// vectors (8 per CU), enough loads in flight to stream the operand.
int64_t scan_lspan() { return 128; }

hipError_t launch_scan3(const OperandView& op, const Split3Out& o, hipStream_t st) {
    if (op.nv <= 0 || op.k <= 0) return hipSuccess;
    const int64_t lspan = scan_lspan();
    dim3 grid(static_cast<unsigned>((op.k + lspan - 1) / lspan), static_cast<unsigned>((op.nv + 63) / 64));
    if (op.sl == 1) hipLaunchKernelGGL(scan3_kernel<true>, grid, dim3(256), 0, st, op, o, lspan);
    else hipLaunchKernelGGL(scan3_kernel<false>, grid, dim3(256), 0, st, op, o, lspan);
    return hipGetLastError();
}

hipError_t launch_digits3(const OperandView& op, const SliceLayout& lay, const Split3Out& o, hipStream_t st, int p_lo,
                          int p_hi) {
    if (p_hi < 0) p_hi = lay.s;
    if (p_lo < 0 || p_hi > lay.s || p_lo > p_hi) return hipErrorInvalidValue;
    if (lay.bal && (p_lo != 0 || p_hi != lay.s)) return hipErrorInvalidValue;  // balanced: all planes at once
    if (p_lo == p_hi) return hipSuccess;
    dim3 grid(static_cast<unsigned>(lay.kpad / kStep), static_cast<unsigned>((lay.rows_pad + 63) / 64));
    if (lay.bal) {
        if (op.sl == 1) hipLaunchKernelGGL((digits3_kernel<true, true>), grid, dim3(256), 0, st, op, lay, o, p_lo, p_hi);
        else hipLaunchKernelGGL((digits3_kernel<false, true>), grid, dim3(256), 0, st, op, lay, o, p_lo, p_hi);
    } else {
        if (op.sl == 1)
            hipLaunchKernelGGL((digits3_kernel<true, false>), grid, dim3(256), 0, st, op, lay, o, p_lo, p_hi);
        else
            hipLaunchKernelGGL((digits3_kernel<false, false>), grid, dim3(256), 0, st, op, lay, o, p_lo, p_hi);
    }
    return hipGetLastError();
}

SliceLayout slice_layout(int side_a, int cplx, int64_t nv, int64_t k, int s) {
    SliceLayout L;
    int64_t rows = (cplx && side_a) ? 2 * round_up(nv, 16) : nv;
    L.rows_pad = round_up(rows > 0 ? rows : 1, kRowPad);
    int64_t terms = cplx ? 2 * k : k;
    L.kpad = round_up(terms > 0 ? terms : 1, kStep);
    L.s = s;
    L.bal = 0;
    return L;
}


void scan_blocks(const OperandView& op, int64_t* bx, int64_t* by) {
    *bx = op.k > 0 ? (op.k + scan_lspan() - 1) / scan_lspan() : 0;
    *by = op.nv > 0 ? (op.nv + 63) / 64 : 0;
}

void digits3_blocks(const SliceLayout& lay, int64_t* bx, int64_t* by) {
    *bx = lay.kpad / kStep;
    *by = (lay.rows_pad + 63) / 64;
}

hipError_t launch_scan3_batched(const Split3Op* ops, const BlockItem* items, int64_t nitems, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(scan3_batched_kernel, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, st, ops, items,
                       scan_lspan());
    return hipGetLastError();
}

bool split_fusable(const OperandView& op) {
    return op.k * (op.cplx ? 2 : 1) <= kFuseMaxDoubles && (op.sl == 1 || op.sv == 1);
}

// Blocks over the operand's own vectors only: a GEMM tile that reaches into
// the padding rows of the layout reads whatever they hold, but those rows only
// feed rows (columns) of C' that are never stored, so they need no digits.
void fused_split_blocks(const OperandView& op, int64_t* by) { *by = (op.nv + kFuseV - 1) / kFuseV; }

hipError_t launch_split_fused_batched(const SplitOp* ops, const BlockItem* items, int64_t nitems, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(split_fused_batched_kernel, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, st, ops,
                       items);
    return hipGetLastError();
}

hipError_t launch_digits3_batched(const Split3Op* ops, const BlockItem* items, int64_t nitems, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(digits3_batched_kernel, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, st, ops, items);
    return hipGetLastError();
}

void digits_blocks(const OperandView& op, const SliceLayout& lay, int64_t* bx, int64_t* by) {
    const bool two_row = op.cplx && op.side_a;
    const int64_t vec_cover = two_row ? lay.rows_pad / 2 : lay.rows_pad;
    *bx = lay.kpad / kStep;
    *by = (vec_cover + 63) / 64;
}

hipError_t launch_scan_batched(const SplitOp* ops, const BlockItem* items, int64_t nitems, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(scan_batched_kernel, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, st, ops, items,
                       scan_lspan());
    return hipGetLastError();
}

hipError_t launch_digits_batched(const SplitOp* ops, const BlockItem* items, int64_t nitems, hipStream_t st,
                                 const int32_t* prange) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(digits_batched_kernel, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, st, ops, items,
                       prange);
    return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_scan(const OperandView& op, uint64_t* maxbits, hipStream_t st) {
    if (op.nv <= 0 || op.k <= 0) return hipSuccess;
    const bool lcontig = op.sl == 1;
    const int64_t lspan = scan_lspan();
    dim3 grid(static_cast<unsigned>((op.k + lspan - 1) / lspan), static_cast<unsigned>((op.nv + 63) / 64));
    if (lcontig) {
        if (op.cplx) hipLaunchKernelGGL((scan_kernel<true, true>), grid, dim3(256), 0, st, op, maxbits, lspan);
        else hipLaunchKernelGGL((scan_kernel<true, false>), grid, dim3(256), 0, st, op, maxbits, lspan);
    } else {
        if (op.cplx) hipLaunchKernelGGL((scan_kernel<false, true>), grid, dim3(256), 0, st, op, maxbits, lspan);
        else hipLaunchKernelGGL((scan_kernel<false, false>), grid, dim3(256), 0, st, op, maxbits, lspan);
    }
    return hipGetLastError();
}

hipError_t launch_digits(const OperandView& op, const uint64_t* maxbits, const SliceLayout& lay, int32_t* E,
                         int8_t* slices, hipStream_t st, int p_lo, int p_hi) {
    if (p_hi < 0) p_hi = lay.s;
    if (p_lo < 0 || p_hi > lay.s || p_lo >= p_hi) return p_lo == p_hi ? hipSuccess : hipErrorInvalidValue;
    const bool lcontig = op.sl == 1;
    const bool two_row = op.cplx && op.side_a;
    // blocks along vectors: 64 vectors each (64 complex rows = 128 slice rows for two_row)
    const int64_t vec_cover = two_row ? lay.rows_pad / 2 : lay.rows_pad;
    dim3 grid(static_cast<unsigned>(lay.kpad / kStep), static_cast<unsigned>((vec_cover + 63) / 64));
    // balanced digits depend on s: planes 0 .. p_hi - 1 of an s = p_hi split, in one pass
    if (lay.bal && p_lo != 0) return hipErrorInvalidValue;
#define OZ_DIG(LC, CP, SA, BL) \
    hipLaunchKernelGGL((digits_kernel<LC, CP, SA, BL>), grid, dim3(256), 0, st, op, maxbits, lay, E, slices, p_lo, \
                       p_hi)
#define OZ_DIG_ALL(BL)                                    \
    if (lcontig) {                                        \
        if (two_row) OZ_DIG(true, true, true, BL);        \
        else if (op.cplx) OZ_DIG(true, true, false, BL);  \
        else OZ_DIG(true, false, false, BL);              \
    } else {                                              \
        if (two_row) OZ_DIG(false, true, true, BL);       \
        else if (op.cplx) OZ_DIG(false, true, false, BL); \
        else OZ_DIG(false, false, false, BL);             \
    }
    if (lay.bal) {
        OZ_DIG_ALL(true)
    } else {
        OZ_DIG_ALL(false)
    }
#undef OZ_DIG_ALL
#undef OZ_DIG
    return hipGetLastError();
}

}  // namespace oz
