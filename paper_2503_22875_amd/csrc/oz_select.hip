// oz_select.hip -- kernels of the learned slice-count selection: the
// counter-based generator of synthetic instances, per-operand exponent
// statistics and the 16 selector features, and the error table that labels a
// training instance.
//
// The paper suggests adjusting the number of splits to the operator (Sec. 4);
// the selector predicts, from cheap statistics of the operands and the target
// tolerance, the smallest s whose emulation meets the tolerance.
#include "oz_internal.h"

namespace oz {

namespace {

constexpr uint64_t kMagMask = 0x7fffffffffffffffull;
constexpr uint64_t kMantMask = (1ull << 52) - 1;
constexpr uint64_t kInfBits = 0x7ff0000000000000ull;

__device__ __forceinline__ double max_value(uint64_t b) { return __longlong_as_double(static_cast<long long>(b)); }

// frexp exponent of the scale of a vector whose largest magnitude has bits b
__device__ __forceinline__ int scale_exp(uint64_t b) {
    if (b == 0) return 0;
    if (b >= kInfBits) return kNonFiniteExp;
    const int eb = static_cast<int>(b >> 52);
    if (eb > 0) return eb - 1022;
    return (64 - __clzll(static_cast<long long>(b & kMantMask))) - 1074;
}

// ---- generator ----------------------------------------------------------------
// Entry (i, j) of a rows x cols operand, idx = i + j*rows, uses draws
// 5 idx .. 5 idx + 4 of the entry stream:
//   family 0: sign (bit 0) and 53-bit significand (bits 11..63) of draw 0,
//             value in [1/2, 1);
//   family 1: u_c = (draw c >> 11) 2^-53, value ((u0 + u1) + u2) + u3 - 2;
//   then the significand keeps its top `bits` bits; draw 4 gives zero when
//   (d4 >> 40) < zero_q and the entry exponent (d4 mod 2^32) mod (sig_el + 1)
//   - sig_el/2; the vector exponent of row i (A) / column j (B) is draw i / j
//   of the vector stream mod (sig_vec + 1) - sig_vec/2.  All steps are exact
//   or single IEEE additions, so every implementation gets the same bits.
__global__ void gen_kernel(GenSide g) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= g.rows * g.cols) return;
    const int64_t i = idx % g.rows, j = idx / g.rows;
    const uint64_t base = 5ull * static_cast<uint64_t>(idx);
    double x;
    if (g.family == 0) {
        const uint64_t d0 = sm64_draw(g.ekey, base);
        const uint64_t mant = (d0 >> 11) | (1ull << 52);
        x = static_cast<double>(mant) * 0x1p-53;
        if (d0 & 1ull) x = -x;
    } else {
        double u[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) u[c] = static_cast<double>(sm64_draw(g.ekey, base + c) >> 11) * 0x1p-53;
        x = (((u[0] + u[1]) + u[2]) + u[3]) - 2.0;
    }
    if (g.bits < 53) {
        const uint64_t keep = ~((1ull << (53 - g.bits)) - 1ull);
        x = __longlong_as_double(static_cast<long long>(static_cast<uint64_t>(__double_as_longlong(x)) & keep));
    }
    const uint64_t d4 = sm64_draw(g.ekey, base + 4);
    const bool zero = static_cast<int64_t>(d4 >> 40) < g.zero_q;
    const int e_el = static_cast<int>((d4 & 0xffffffffull) % static_cast<uint64_t>(g.sig_el + 1)) - g.sig_el / 2;
    const uint64_t dv = sm64_draw(g.vkey, static_cast<uint64_t>(g.vec_axis == 0 ? i : j));
    const int e_vec = static_cast<int>(dv % static_cast<uint64_t>(g.sig_vec + 1)) - g.sig_vec / 2;
    g.X[i + j * g.ld] = zero ? 0.0 : ldexp(x, e_el + e_vec);
}

// ---- exponent statistics ---------------------------------------------------------
// The block's histogram is kept in kHistCopies copies, lane l adding to copy
// l % kHistCopies: most entries of a vector share a few gap and width values,
// and 64 lanes adding to one LDS word serialise (one lane per clock), which
// held the pass to a third of the HBM rate.  Copy c starts kHistLen words
// after copy c - 1 (kHistLen = 1 mod 32), so one bin lies in a different bank
// in every copy.
constexpr int kHistCopies = 16;
static_assert(kHistLen % 32 == 1 && (kHistCopies & (kHistCopies - 1)) == 0, "histogram copy layout");
__device__ __forceinline__ void lane_hist_add(uint32_t* h, int bin) {
    if (bin >= 0) atomicAdd(&h[(threadIdx.x & (kHistCopies - 1)) * kHistLen + bin], 1u);
}

// One entry: its gap bin and width bin (the zero bin and -1 for a zero), and
// its term of the mean square.
__device__ __forceinline__ void stat_entry(double x, int E, int& gbin, int& wbin, double& sq) {
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x)) & kMagMask;
    if (b == 0) {
        gbin = 2 * kHistBins;
        wbin = -1;
        return;
    }
    const int eb = static_cast<int>(b >> 52);
    const uint64_t M = (b & kMantMask) | (eb ? (1ull << 52) : 0ull);
    const int bl = 64 - __clzll(static_cast<long long>(M));
    const int ex = eb ? eb - 1022 : bl - 1074;          // frexp exponent of x
    const int tz = __builtin_ctzll(M);
    const int gap = E - ex;
    const int wid = gap + bl - tz;
    gbin = gap < kHistCap ? gap : kHistCap;
    wbin = kHistBins + (wid < kHistCap ? wid : kHistCap);
    const double y = ldexp(x, -E);
    sq += y * y;
}

// Histogram counts and mean-square terms of one entry per active lane (CPLX:
// the two parts), from values already loaded.
template <bool CPLX>
__device__ __forceinline__ void stat_terms(double re, double im, int E, uint32_t* lh, double& sq) {
    int g0, w0;
    stat_entry(re, E, g0, w0, sq);
    lane_hist_add(lh, g0);
    lane_hist_add(lh, w0);
    if (CPLX) {
        int g1, w1;
        stat_entry(im, E, g1, w1, sq);
        lane_hist_add(lh, g1);
        lane_hist_add(lh, w1);
    }
}

// Terms per lane whose loads are issued before any of them is processed (one
// load round trip per term left the pass latency-bound).
constexpr int kStatBatch = 8;

// One block: 64 vectors, all their terms.
// LCONTIG (terms contiguous): each wave walks 16 vectors, lanes along terms,
//   per-vector sums by a fixed butterfly.
// else (vectors contiguous): lane = vector, the 4 waves split the terms,
//   partial sums combined through LDS in wave order.
// Each lane adds its terms in ascending order; lh and red are the block's
// shared arrays (one allocation for every instantiation).
template <bool LCONTIG, bool CPLX>
__device__ __forceinline__ void stats_body(const StatSide& s, int64_t by, uint32_t* lh, double (*red)[64]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int b = tid; b < kHistCopies * kHistLen; b += 256) lh[b] = 0;
    __syncthreads();
    const OperandView& op = s.op;
    const int w = CPLX ? 2 : 1;
    const double denom = static_cast<double>(op.k) * w;
    if (LCONTIG) {
        for (int vi = 0; vi < 16; ++vi) {
            const int64_t v = by * 64 + wave * 16 + vi;
            if (v >= op.nv) break;  // wave-uniform
            const int E = scale_exp(s.maxbits[v]);
            double sq = 0.0;
            if (E != kNonFiniteExp) {
                const double* base = op.X + v * op.sv * w;
                for (int64_t l0 = lane; l0 < op.k; l0 += 64 * kStatBatch) {
                    double re[kStatBatch], im[kStatBatch];
#pragma unroll
                    for (int q = 0; q < kStatBatch; ++q) {
                        const int64_t l = l0 + 64 * q;
                        const double* e = base + (l < op.k ? l : l0) * op.sl * w;
                        re[q] = e[0];
                        im[q] = CPLX ? e[1] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < kStatBatch; ++q)
                        if (l0 + 64 * q < op.k) stat_terms<CPLX>(re[q], im[q], E, lh, sq);
                }
            }
            for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
            if (lane == 0) s.msq[v] = op.k > 0 ? sq / denom : 0.0;
        }
    } else {
        const int64_t v = by * 64 + lane;
        double sq = 0.0;
        if (v < op.nv) {
            const int E = scale_exp(s.maxbits[v]);
            if (E != kNonFiniteExp)
                for (int64_t l0 = wave; l0 < op.k; l0 += 4 * kStatBatch) {
                    double re[kStatBatch], im[kStatBatch];
#pragma unroll
                    for (int q = 0; q < kStatBatch; ++q) {
                        const int64_t l = l0 + 4 * q;
                        const double* e = op.X + (v * op.sv + (l < op.k ? l : l0) * op.sl) * w;
                        re[q] = e[0];
                        im[q] = CPLX ? e[1] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < kStatBatch; ++q)
                        if (l0 + 4 * q < op.k) stat_terms<CPLX>(re[q], im[q], E, lh, sq);
                }
        }
        red[wave][lane] = sq;
        __syncthreads();
        if (wave == 0 && v < op.nv) {
            const double t = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
            s.msq[v] = op.k > 0 ? t / denom : 0.0;
        }
    }
    __syncthreads();
    for (int b = tid; b < kHistLen; b += 256) {
        unsigned long long t = 0;
        for (int c = 0; c < kHistCopies; ++c) t += lh[c * kHistLen + b];
        if (t) atomicAdd(&s.hist[b], t);
    }
}

__device__ __forceinline__ void stats_dispatch(const StatSide& s, int64_t by) {
    __shared__ uint32_t lh[kHistCopies * kHistLen];
    __shared__ double red[4][64];
    const bool lc = s.op.sl == 1 && s.op.sv != 1;
    if (lc) {
        if (s.op.cplx) stats_body<true, true>(s, by, lh, red);
        else stats_body<true, false>(s, by, lh, red);
    } else {
        if (s.op.cplx) stats_body<false, true>(s, by, lh, red);
        else stats_body<false, false>(s, by, lh, red);
    }
}

__global__ __launch_bounds__(256) void stats_kernel(StatSide s) { stats_dispatch(s, blockIdx.x); }

__global__ __launch_bounds__(256) void stats_batched_kernel(const StatSide* sides, const BlockItem* items) {
    const BlockItem it = items[blockIdx.x];
    stats_dispatch(sides[it.op], it.by);
}

// ---- features ----------------------------------------------------------------------
struct HistMoments {
    double zero_frac, gm, gs, g90, wm, w90;
};

__device__ double quantile90(const unsigned long long* h, unsigned long long nz) {
    if (nz == 0) return 0.0;
    unsigned long long cum = 0;
    for (int v = 0; v < kHistBins; ++v) {
        cum += h[v];
        if (cum * 10ull >= 9ull * nz) return static_cast<double>(v);
    }
    return static_cast<double>(kHistCap);
}

__device__ HistMoments moments(const unsigned long long* h, int64_t total) {
    HistMoments r;
    unsigned long long nz = 0, s1 = 0, s2 = 0, w1 = 0;
    for (int v = 0; v < kHistBins; ++v) {
        nz += h[v];
        s1 += h[v] * static_cast<unsigned long long>(v);
        s2 += h[v] * static_cast<unsigned long long>(v * v);
        w1 += h[kHistBins + v] * static_cast<unsigned long long>(v);
    }
    const double dnz = static_cast<double>(nz);
    r.zero_frac = total > 0 ? static_cast<double>(h[2 * kHistBins]) / static_cast<double>(total) : 0.0;
    r.gm = nz ? static_cast<double>(s1) / dnz : 0.0;
    const double var = nz ? static_cast<double>(s2) / dnz - r.gm * r.gm : 0.0;
    r.gs = var > 0.0 ? sqrt(var) : 0.0;
    r.g90 = quantile90(h, nz);
    r.wm = nz ? static_cast<double>(w1) / dnz : 0.0;
    r.w90 = quantile90(h + kHistBins, nz);
    return r;
}

// One block per problem: fixed-order sums of the per-vector mean squares,
// then one thread turns the histograms into the feature rows.
__global__ __launch_bounds__(256) void features_kernel(const FeatProb* probs) {
    const FeatProb& p = probs[blockIdx.x];
    __shared__ double red[2][256];
    for (int side = 0; side < 2; ++side) {
        double a = 0.0;
        for (int64_t v = threadIdx.x; v < p.nv[side]; v += 256) a += p.msq[side][v];
        red[side][threadIdx.x] = a;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double ma = p.nv[0] > 0 ? red[0][0] / static_cast<double>(p.nv[0]) : 0.0;
    const double mb = p.nv[1] > 0 ? red[1][0] / static_cast<double>(p.nv[1]) : 0.0;
    if (p.mstat) {
        p.mstat[0] = ma;
        p.mstat[1] = mb;
    }
    const int64_t terms = p.k * (p.cplx ? 2 : 1);
    const HistMoments ha = moments(p.hist[0], p.nv[0] * terms);
    const HistMoments hb = moments(p.hist[1], p.nv[1] * terms);
    const double spread = (ma > 0.0 && mb > 0.0) ? 0.5 * log2((1.0 / ma + 1.0 / mb) / 3.0) : 0.0;
    const double f_k = log2(static_cast<double>(terms));
    const double f_mn = 0.5 * log2(static_cast<double>(p.m) * static_cast<double>(p.n));
    for (int t = 0; t < p.ntol; ++t) {
        const double tol = p.tols[t];
        float* f = p.feat + static_cast<int64_t>(t) * kNumFeat;
        const double vals[kNumFeat] = {ha.zero_frac, ha.gm, ha.gs, ha.g90, ha.wm, ha.w90,
                                       hb.zero_frac, hb.gm, hb.gs, hb.g90, hb.wm, hb.w90,
                                       f_k, f_mn, -log10(tol), spread};
        for (int q = 0; q < kNumFeat; ++q) f[q] = static_cast<float>(vals[q]);
        if (p.s_rule) p.s_rule[t] = rule_slices_of(ma, mb, tol, p.smax);
        if (p.eps) {
            int lab = p.s_ref;
            for (int s = 2; s <= p.s_ref; ++s)
                if (p.eps[s - 1] <= tol) {
                    lab = s;
                    break;
                }
            p.label[t] = static_cast<float>(lab);
        }
    }
}

// ---- error table ---------------------------------------------------------------------
// Thread (i, j): C_s = ldexp(acc_s, E_i + F_j) with acc_s the sum, from d = s+1
// down to 2, of S_d 2^(-7d) -- the accumulation of the fixed-s emulation with
// one INT32 chunk.  W_ij C_ij = acc * r_i * c_j with r_i = 2^E_i / max|A_i:|,
// c_j = 2^F_j / max|B_:j| (in (1, 2]).  Per block: the sums over its entries of
// (W (C_s - C_ref))^2 for s < s_ref and of (W C_ref)^2.
__global__ __launch_bounds__(256) void eps_partial_kernel(const int32_t* diag, int64_t Mp, int64_t Np, int s_ref,
                                                          const int32_t* EA, const int32_t* FB,
                                                          const uint64_t* maxa, const uint64_t* maxb, int64_t m,
                                                          double* partial) {
    __shared__ double red[kMaxRef][256];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t j = blockIdx.y;
    double part[kMaxRef];
#pragma unroll
    for (int q = 0; q < kMaxRef; ++q) part[q] = 0.0;
    if (i < m && maxa[i] != 0 && maxb[j] != 0) {
        const double r = 1.0 / ldexp(max_value(maxa[i]), -EA[i]);
        const double c = 1.0 / ldexp(max_value(maxb[j]), -FB[j]);
        double S[kMaxRef + 2];
        for (int d = 2; d <= s_ref + 1; ++d) S[d] = static_cast<double>(diag[((d - 2) * Np + j) * Mp + i]);
        double acc_ref = 0.0;
        for (int d = s_ref + 1; d >= 2; --d) acc_ref = acc_ref + S[d] * ldexp(1.0, -7 * d);
        const double wref = acc_ref * r * c;
        part[s_ref - 1] = wref * wref;
        for (int s = 1; s < s_ref; ++s) {
            double acc = 0.0;
            for (int d = s + 1; d >= 2; --d) acc = acc + S[d] * ldexp(1.0, -7 * d);
            const double diff = (acc - acc_ref) * r * c;
            part[s - 1] = diff * diff;
        }
    }
    for (int q = 0; q < s_ref; ++q) red[q][threadIdx.x] = part[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < s_ref; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < s_ref)
        partial[(static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * kMaxRef + threadIdx.x] =
            red[threadIdx.x][0];
}

// eps[s - 1] = sqrt(num_s / den) for s < s_ref, eps[s_ref - 1] = 0; the block
// sums are added in block order.
__global__ void eps_final_kernel(const double* partial, int64_t nblocks, int s_ref, double* eps) {
    const int q = threadIdx.x;
    __shared__ double den;
    if (q == 0) {
        double d = 0.0;
        for (int64_t b = 0; b < nblocks; ++b) d += partial[b * kMaxRef + s_ref - 1];
        den = d;
    }
    __syncthreads();
    if (q >= s_ref) return;
    if (q == s_ref - 1) {
        eps[q] = 0.0;
        return;
    }
    double num = 0.0;
    for (int64_t b = 0; b < nblocks; ++b) num += partial[b * kMaxRef + q];
    eps[q] = den > 0.0 ? sqrt(num / den) : sqrt(num);
}

}  // namespace

hipError_t launch_gen(const GenSide& g, hipStream_t st) {
    const int64_t total = g.rows * g.cols;
    if (total <= 0) return hipSuccess;
    if (g.sig_el < 0 || g.sig_vec < 0 || g.bits < 1 || g.bits > 53 || g.ld < g.rows) return hipErrorInvalidValue;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gen_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, g);
    return hipGetLastError();
}

void stat_blocks(const OperandView& op, int64_t* blocks) { *blocks = (op.nv + 63) / 64; }

hipError_t launch_stats(const StatSide& s, hipStream_t st) {
    int64_t blocks;
    stat_blocks(s.op, &blocks);
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stats_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_stats_batched(const StatSide* sides, const BlockItem* items, int64_t nitems, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (nitems > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stats_batched_kernel, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, st, sides, items);
    return hipGetLastError();
}

hipError_t launch_features(const FeatProb* probs, int64_t nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3(static_cast<unsigned>(nprob)), dim3(256), 0, st, probs);
    return hipGetLastError();
}

int64_t eps_partial_len(int64_t m, int64_t n) { return ((m + 255) / 256) * n * kMaxRef; }

hipError_t launch_eps_table(const int32_t* diag, int64_t Mp, int64_t Np, int s_ref, const int32_t* EA,
                            const int32_t* FB, const uint64_t* maxa, const uint64_t* maxb, int64_t m, int64_t n,
                            double* partial, double* eps, hipStream_t st) {
    if (s_ref < 2 || s_ref > kMaxRef || m <= 0 || n <= 0 || n > 65535 || Mp < m || Np < n)
        return hipErrorInvalidValue;
    const int64_t bx = (m + 255) / 256;
    hipLaunchKernelGGL(eps_partial_kernel, dim3(static_cast<unsigned>(bx), static_cast<unsigned>(n)), dim3(256), 0,
                       st, diag, Mp, Np, s_ref, EA, FB, maxa, maxb, m, partial);
    hipLaunchKernelGGL(eps_final_kernel, dim3(1), dim3(64), 0, st, partial, bx * n, s_ref, eps);
    return hipGetLastError();
}

}  // namespace oz
