// oz_check.hip -- tolerance-driven slice count: operand statistics for the
// a-priori rule, the a-posteriori residual check, and the final scaling pass.
//
// Residual check (randomised, one probe vector): with D1 = diag(1/max|op(A)_i:|),
// D2 = diag(1/max|op(B)_:j|) and sigma a +-1 vector drawn from a counter-based
// hash,
//   y1 = D1 * C_emu * D2 * sigma        (C_emu = ldexp(acc, E_i + F_j))
//   y2 = D1 * op(A) * (op(B) * (D2 * sigma))
// are formed in double-double arithmetic, and
//   eps_est = || y1 - y2 || / || y2 ||
// A single product splits each of its three reductions (op(B) t, the rows of
// op(A) against u, the rows of C_emu against t) over many blocks with
// fixed-order partial sums; a batch of small products runs one block per 64
// vectors of each product.
// estimates the scale-weighted Frobenius error || D1 (C_emu - AB) D2 ||_F /
// || D1 AB D2 ||_F (for +-1 entries E||X sigma||^2 = ||X||_F^2).  Both sides use
// the same rounded weights t_j = D2_jj * sigma_j and w_i = D1_ii, so y1 - y2
// carries the emulation error only.  The work is O(mk + kn + mn), against
// O(mnk) for the product itself.
#include <algorithm>

#include "oz_internal.h"

namespace oz {

namespace {

// ---- double-double helpers (FMA TwoProduct, Knuth TwoSum) ----------------
struct dd {
    double hi, lo;
};
__device__ __forceinline__ dd two_sum(double a, double b) {
    const double s = a + b, z = s - a;
    return {s, (a - (s - z)) + (b - z)};
}
__device__ __forceinline__ dd dd_add_prod(dd acc, double a, double b) {
    // acc + a*b, Dot2 style: error terms gathered in lo
    const double p = a * b, e = fma(a, b, -p);
    const dd s = two_sum(acc.hi, p);
    return {s.hi, acc.lo + (s.lo + e)};
}
__device__ __forceinline__ dd dd_norm(dd x) { return two_sum(x.hi, x.lo); }
__device__ __forceinline__ dd dd_mul_d(dd x, double w) {
    const double p = x.hi * w, e = fma(x.hi, w, -p);
    return dd_norm({p, e + x.lo * w});
}
__device__ __forceinline__ double dd_sub_to_d(dd a, dd b) {
    const dd s = two_sum(a.hi, -b.hi);
    return s.hi + (s.lo + (a.lo - b.lo));
}

__device__ __forceinline__ double max_of_bits(uint64_t b) { return __longlong_as_double(static_cast<long long>(b)); }

// +-1 from the splitmix64 mixer of (seed, j)
__device__ __forceinline__ double rademacher(uint64_t seed, int64_t j) {
    uint64_t z = seed + static_cast<uint64_t>(j + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (z >> 63) ? -1.0 : 1.0;
}

__device__ __forceinline__ void load_elem(const OperandView& op, int64_t v, int64_t l, double& re, double& im) {
    const double* e = op.X + (v * op.sv + l * op.sl) * (op.cplx ? 2 : 1);
    re = e[0];
    im = op.cplx ? (op.conj ? -e[1] : e[1]) : 0.0;
}

// ---- t_j = sigma_j / max|op(B)_:j| ------------------------------------------
__device__ __forceinline__ void weights_body(const CheckArgs& c, int64_t j) {
    if (j >= c.opb.nv) return;
    const double mx = max_of_bits(c.maxb[j]);
    c.t[j] = mx > 0.0 ? rademacher(c.seed, j) / mx : 0.0;
}

// ---- many products: u = op(B) t in double-double; u[l] = (re.hi, re.lo,
// im.hi, im.lo).  Block: 64 terms (lanes) x 4 parts (waves); part w sums the columns
// j = w, w + 4, ...; the four partial sums are added in part order.
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    const dd s = two_sum(a.hi, b.hi);
    return {s.hi, s.lo + (a.lo + b.lo)};
}
constexpr int kParts = 4;
constexpr int kLanes = 64;
// Terms per wave whose loads are issued before any of them is added: the
// reductions below are chains of double-double additions, and one load
// round trip per term left them latency-bound.
constexpr int kBatch = 8;
// an index past the end reads the last element (in bounds; its term is not added)
__device__ __forceinline__ int64_t clamp_index(int64_t x, int64_t n) { return x < n ? x : n - 1; }

__device__ __forceinline__ void gemv_b_body(const CheckArgs& c, int64_t lb) {
    __shared__ dd red[kParts][2][kLanes];
    const OperandView& opb = c.opb;
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int64_t l = lb * kLanes + lane;
    dd sr = {0.0, 0.0}, si = {0.0, 0.0};
    if (l < opb.k) {
        // kBatch columns' loads issued together, then added in column order
        for (int64_t j0 = part; j0 < opb.nv; j0 += kParts * kBatch) {
            double re[kBatch], im[kBatch], tj[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const int64_t j = clamp_index(j0 + q * kParts, opb.nv);
                load_elem(opb, j, l, re[q], im[q]);
                tj[q] = c.t[j];
            }
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                if (j0 + q * kParts >= opb.nv) break;
                sr = dd_add_prod(sr, re[q], tj[q]);
                si = dd_add_prod(si, im[q], tj[q]);
            }
        }
    }
    red[part][0][lane] = sr;
    red[part][1][lane] = si;
    __syncthreads();
    if (part != 0 || l >= opb.k) return;
    for (int q = 1; q < kParts; ++q) {
        sr = dd_add(sr, red[q][0][lane]);
        si = dd_add(si, red[q][1][lane]);
    }
    sr = dd_norm(sr);
    si = dd_norm(si);
    c.u[4 * l] = sr.hi;
    c.u[4 * l + 1] = sr.lo;
    c.u[4 * l + 2] = si.hi;
    c.u[4 * l + 3] = si.lo;
}

// ---- many products, per row i of op(A): y2 = w_i op(A)_i: u, y1 = w_i sum_j C_emu_ij t_j
// Writes diff[i] = y1 - y2 and ref[i] = y2 (real, or real and imaginary parts
// at 2i, 2i+1 for complex).  Block: 64 rows (lanes) x 4 parts (waves); part w
// takes the terms l = w, w + 4, ... and the columns j = w, w + 4, ...; the
// partial sums are added in part order.
template <bool CPLX>
__device__ __forceinline__ void rows_body_t(const CheckArgs& c, int64_t rb) {
    __shared__ dd red[kParts][4][kLanes];
    const OperandView& opa = c.opa;
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int64_t i = rb * kLanes + lane;
    const int64_t Mp = c.Mp, n = c.opb.nv;
    const double* u = c.u;
    dd y2r = {0.0, 0.0}, y2i = {0.0, 0.0}, y1r = {0.0, 0.0}, y1i = {0.0, 0.0};
    if (i < opa.nv) {
        // y2 = a_i . u  (complex: (ar + i ai)(ur + i ui))
        for (int64_t l0 = part; l0 < opa.k; l0 += kParts * kBatch) {
            double ar[kBatch], ai[kBatch], uu[kBatch][4];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const int64_t l = clamp_index(l0 + q * kParts, opa.k);
                load_elem(opa, i, l, ar[q], ai[q]);
#pragma unroll
                for (int r = 0; r < 4; ++r) uu[q][r] = u[4 * l + r];
            }
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                if (l0 + q * kParts >= opa.k) break;
                const double urh = uu[q][0], url = uu[q][1], uih = uu[q][2], uil = uu[q][3];
                y2r = dd_add_prod(y2r, ar[q], urh);
                y2r = dd_add_prod(y2r, ar[q], url);
                if (CPLX) {
                    y2r = dd_add_prod(y2r, -ai[q], uih);
                    y2r = dd_add_prod(y2r, -ai[q], uil);
                    y2i = dd_add_prod(y2i, ar[q], uih);
                    y2i = dd_add_prod(y2i, ar[q], uil);
                    y2i = dd_add_prod(y2i, ai[q], urh);
                    y2i = dd_add_prod(y2i, ai[q], url);
                }
            }
        }
        // y1 = sum_j ldexp(acc_ij, E_i + F_j) t_j over the slice-row(s) of row i
        const int64_t r_re = CPLX ? 32 * (i >> 4) + 16 * ((i >> 3) & 1) + (i & 7) : i;
        const int64_t r_im = r_re + 8;
        const int32_t e = c.EA[i];
        for (int64_t j0 = part; j0 < n; j0 += kParts * kBatch) {
            int fb[kBatch];
            double tj[kBatch], cr[kBatch], ci[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const int64_t j = clamp_index(j0 + q * kParts, n);
                fb[q] = c.FB[j];
                tj[q] = c.t[j];
                cr[q] = c.acc[j * Mp + r_re];
                if (CPLX) ci[q] = c.acc[j * Mp + r_im];
            }
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                if (j0 + q * kParts >= n) break;
                const int ef = e + fb[q];
                y1r = dd_add_prod(y1r, ldexp(cr[q], ef), tj[q]);
                if (CPLX) y1i = dd_add_prod(y1i, ldexp(ci[q], ef), tj[q]);
            }
        }
    }
    red[part][0][lane] = y1r;
    red[part][1][lane] = y1i;
    red[part][2][lane] = y2r;
    red[part][3][lane] = y2i;
    __syncthreads();
    if (part != 0 || i >= opa.nv) return;
    for (int q = 1; q < kParts; ++q) {
        y1r = dd_add(y1r, red[q][0][lane]);
        y1i = dd_add(y1i, red[q][1][lane]);
        y2r = dd_add(y2r, red[q][2][lane]);
        y2i = dd_add(y2i, red[q][3][lane]);
    }
    const double mx = max_of_bits(c.maxa[i]);
    const double w = mx > 0.0 ? 1.0 / mx : 0.0;
    y1r = dd_mul_d(dd_norm(y1r), w);
    y2r = dd_mul_d(dd_norm(y2r), w);
    if (!CPLX) {
        c.diff[i] = dd_sub_to_d(y1r, y2r);
        c.ref[i] = y2r.hi + y2r.lo;
    } else {
        y1i = dd_mul_d(dd_norm(y1i), w);
        y2i = dd_mul_d(dd_norm(y2i), w);
        c.diff[2 * i] = dd_sub_to_d(y1r, y2r);
        c.diff[2 * i + 1] = dd_sub_to_d(y1i, y2i);
        c.ref[2 * i] = y2r.hi + y2r.lo;
        c.ref[2 * i + 1] = y2i.hi + y2i.lo;
    }
}
__device__ __forceinline__ void rows_body(const CheckArgs& c, int64_t rb) {
    if (c.opa.cplx) rows_body_t<true>(c, rb);
    else rows_body_t<false>(c, rb);
}

// ---- split reductions (single product) --------------------------------------
// A reduction of R outputs over L terms, o[r] = sum_c f(r, c), runs in one of
// two shapes chosen by which index is contiguous in memory:
//   out: one thread per output, consecutive outputs on consecutive lanes, the
//        terms cut into nch chunks along grid.y;
//   in:  one wave per output, consecutive terms on consecutive lanes, the
//        lanes' sums merged by a fixed butterfly; nch chunks along grid.y.
// Each (chunk, output) partial goes to part[chunk * R + r]; a second pass adds
// the chunks in chunk order.  The result is deterministic for a given shape.
struct DC {
    dd re, im;
};
__device__ __forceinline__ void acc_zero(DC& a) { a = {{0.0, 0.0}, {0.0, 0.0}}; }
__device__ __forceinline__ void acc_zero(double& a) { a = 0.0; }
__device__ __forceinline__ DC acc_merge(DC a, DC b) { return {dd_add(a.re, b.re), dd_add(a.im, b.im)}; }
__device__ __forceinline__ double acc_merge(double a, double b) { return a + b; }
__device__ __forceinline__ DC acc_xor(DC a, int off) {
    return {{__shfl_xor(a.re.hi, off), __shfl_xor(a.re.lo, off)}, {__shfl_xor(a.im.hi, off), __shfl_xor(a.im.lo, off)}};
}
__device__ __forceinline__ double acc_xor(double a, int off) { return __shfl_xor(a, off); }

// u = op(B) t: output = term l of op(B), reduction over its columns j
struct OpU {
    OperandView opb;
    const double* t;
    __device__ int64_t row(int64_t l) const { return l; }
    __device__ void add(DC& a, int64_t l, int64_t j) const {
        double re, im;
        load_elem(opb, j, l, re, im);
        const double tj = t[j];
        a.re = dd_add_prod(a.re, re, tj);
        a.im = dd_add_prod(a.im, im, tj);
    }
};

// y2 = op(A)_i: u: output = row i of op(A), reduction over its terms l
struct OpY2 {
    OperandView opa;
    const double* u;
    __device__ int64_t row(int64_t i) const { return i; }
    __device__ void add(DC& a, int64_t i, int64_t l) const {
        double ar, ai;
        load_elem(opa, i, l, ar, ai);
        const double urh = u[4 * l], url = u[4 * l + 1], uih = u[4 * l + 2], uil = u[4 * l + 3];
        a.re = dd_add_prod(a.re, ar, urh);
        a.re = dd_add_prod(a.re, ar, url);
        if (opa.cplx) {
            a.re = dd_add_prod(a.re, -ai, uih);
            a.re = dd_add_prod(a.re, -ai, uil);
            a.im = dd_add_prod(a.im, ar, uih);
            a.im = dd_add_prod(a.im, ar, uil);
            a.im = dd_add_prod(a.im, ai, urh);
            a.im = dd_add_prod(a.im, ai, url);
        }
    }
};

// y1 = sum_j ldexp(acc_ij, E_i + F_j) t_j: output = row i, reduction over j
struct RowY1 {
    int64_t r_re;
    int32_t e;
};
struct OpY1 {
    const double* acc;
    int64_t Mp;
    const int32_t* EA;
    const int32_t* FB;
    const double* t;
    int cplx;
    __device__ RowY1 row(int64_t i) const {
        return {cplx ? 32 * (i >> 4) + 16 * ((i >> 3) & 1) + (i & 7) : i, EA[i]};
    }
    __device__ void add(DC& a, const RowY1& r, int64_t j) const {
        const int ef = r.e + FB[j];
        const double tj = t[j];
        a.re = dd_add_prod(a.re, ldexp(acc[j * Mp + r.r_re], ef), tj);
        if (cplx) a.im = dd_add_prod(a.im, ldexp(acc[j * Mp + r.r_re + 8], ef), tj);
    }
};

// 3-real-product form: y1 = sum_j C_ij t_j with C_ij = (T1 - T2) + i ((T3 - T1)
// - T2), T_q = ldexp(acc_q, E_q,i + F_q,j) (real layout), each difference
// rounded as in the combining epilogue; NaN where a scale marks Inf/NaN input
struct RowY13 {
    int64_t i;
    int32_t e[3];
};
struct OpY1z3 {
    const double* acc[3];
    int64_t Mp;
    const int32_t* EA[3];
    const int32_t* FB[3];
    const double* t;
    __device__ RowY13 row(int64_t i) const { return {i, {EA[0][i], EA[1][i], EA[2][i]}}; }
    __device__ void add(DC& a, const RowY13& r, int64_t j) const {
        double T[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int32_t f = FB[q][j];
            T[q] = (r.e[q] == kNonFiniteExp || f == kNonFiniteExp) ? __longlong_as_double(0x7ff8000000000000ll)
                                                                    : ldexp(acc[q][j * Mp + r.i], r.e[q] + f);
        }
        const double cr = T[0] - T[1];
        const double ci = (T[2] - T[0]) - T[1];
        const double tj = t[j];
        a.re = dd_add_prod(a.re, cr, tj);
        a.im = dd_add_prod(a.im, ci, tj);
    }
};

// sum over the terms of vector v of |x * 2^-E_v|^2 (the rule's statistic)
struct RowMsq {
    int64_t v;
    int E;
};
struct OpMsq {
    OperandView op;
    const uint64_t* maxbits;
    __device__ RowMsq row(int64_t v) const {
        const uint64_t mb = maxbits[v];
        int E = 0;
        if (mb != 0 && mb < 0x7ff0000000000000ull) frexp(max_of_bits(mb), &E);
        return {v, E};
    }
    __device__ void add(double& a, const RowMsq& r, int64_t l) const {
        double re, im;
        load_elem(op, r.v, l, re, im);
        const double x = ldexp(re, -r.E), y = ldexp(im, -r.E);
        a += x * x + y * y;
    }
};

template <class Op, class Acc>
__global__ __launch_bounds__(256) void red_out_kernel(Op op, int64_t R, int64_t L, int64_t chunk, Acc* part) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (r >= R) return;
    const int64_t c0 = static_cast<int64_t>(blockIdx.y) * chunk;
    const int64_t c1 = c0 + chunk < L ? c0 + chunk : L;
    Acc a;
    acc_zero(a);
    const auto rs = op.row(r);
    for (int64_t c = c0; c < c1; ++c) op.add(a, rs, c);
    part[static_cast<int64_t>(blockIdx.y) * R + r] = a;
}

template <class Op, class Acc>
__global__ __launch_bounds__(256) void red_in_kernel(Op op, int64_t R, int64_t L, int64_t chunk, Acc* part) {
    const int lane = threadIdx.x & 63;
    const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (r >= R) return;  // uniform over the wave; no barrier follows
    const int64_t c0 = static_cast<int64_t>(blockIdx.y) * chunk;
    const int64_t c1 = c0 + chunk < L ? c0 + chunk : L;
    Acc a;
    acc_zero(a);
    const auto rs = op.row(r);
    for (int64_t c = c0 + lane; c < c1; c += 64) op.add(a, rs, c);
    for (int off = 32; off > 0; off >>= 1) a = acc_merge(a, acc_xor(a, off));
    if (lane == 0) part[static_cast<int64_t>(blockIdx.y) * R + r] = a;
}

// Chunk sums: a block takes 32 outputs (consecutive lanes, coalesced reads)
// x 8 chunk groups; group g adds the chunks g, g + 8, ... in order, and the 8
// group sums are merged in group order.
constexpr int kSumOut = 32;
constexpr int kSumGroups = 8;

template <class Acc>
__device__ __forceinline__ Acc group_sum(const Acc* part, int64_t R, int64_t nch, int64_t r, int g) {
    Acc a;
    acc_zero(a);
    if (r < R)
        for (int64_t q = g; q < nch; q += kSumGroups) a = acc_merge(a, part[q * R + r]);
    return a;
}

template <class Acc>
__device__ __forceinline__ Acc merge_groups(Acc a, Acc (*red)[kSumOut], int o) {
    for (int q = 1; q < kSumGroups; ++q) a = acc_merge(a, red[q][o]);
    return a;
}

// u[l] = (re.hi, re.lo, im.hi, im.lo) of the chunk sum, normalised
__global__ __launch_bounds__(256) void u_sum_kernel(const DC* part, int64_t R, int64_t nch, double* u) {
    __shared__ DC red[kSumGroups][kSumOut];
    const int o = threadIdx.x % kSumOut, g = threadIdx.x / kSumOut;
    const int64_t l = static_cast<int64_t>(blockIdx.x) * kSumOut + o;
    DC a = group_sum(part, R, nch, l, g);
    red[g][o] = a;
    __syncthreads();
    if (g != 0 || l >= R) return;
    a = merge_groups(a, red, o);
    const dd re = dd_norm(a.re), im = dd_norm(a.im);
    u[4 * l] = re.hi;
    u[4 * l + 1] = re.lo;
    u[4 * l + 2] = im.hi;
    u[4 * l + 3] = im.lo;
}

__global__ __launch_bounds__(256) void msq_sum_kernel(const double* part, int64_t R, int64_t nch, double denom,
                                                      double* ms) {
    __shared__ double red[kSumGroups][kSumOut];
    const int o = threadIdx.x % kSumOut, g = threadIdx.x / kSumOut;
    const int64_t v = static_cast<int64_t>(blockIdx.x) * kSumOut + o;
    double a = group_sum(part, R, nch, v, g);
    red[g][o] = a;
    __syncthreads();
    if (g != 0 || v >= R) return;
    a = merge_groups(a, red, o);
    ms[v] = denom > 0.0 ? a / denom : 0.0;
}

// diff[i] = w_i (y1 - y2), ref[i] = w_i y2 from the chunk sums of y1 and y2
__global__ __launch_bounds__(256) void rows_combine_kernel(CheckArgs c, int64_t nch1, int64_t nch2) {
    __shared__ DC red1[kSumGroups][kSumOut], red2[kSumGroups][kSumOut];
    const int o = threadIdx.x % kSumOut, g = threadIdx.x / kSumOut;
    const int64_t m = c.opa.nv;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kSumOut + o;
    DC y1 = group_sum(reinterpret_cast<const DC*>(c.part1), m, nch1, i, g);
    DC y2 = group_sum(reinterpret_cast<const DC*>(c.part2), m, nch2, i, g);
    red1[g][o] = y1;
    red2[g][o] = y2;
    __syncthreads();
    if (g != 0 || i >= m) return;
    y1 = merge_groups(y1, red1, o);
    y2 = merge_groups(y2, red2, o);
    const double mx = max_of_bits(c.maxa[i]);
    const double w = mx > 0.0 ? 1.0 / mx : 0.0;
    const dd y1r = dd_mul_d(dd_norm(y1.re), w), y2r = dd_mul_d(dd_norm(y2.re), w);
    if (!c.opa.cplx) {
        c.diff[i] = dd_sub_to_d(y1r, y2r);
        c.ref[i] = y2r.hi + y2r.lo;
    } else {
        const dd y1i = dd_mul_d(dd_norm(y1.im), w), y2i = dd_mul_d(dd_norm(y2.im), w);
        c.diff[2 * i] = dd_sub_to_d(y1r, y2r);
        c.diff[2 * i + 1] = dd_sub_to_d(y1i, y2i);
        c.ref[2 * i] = y2r.hi + y2r.lo;
        c.ref[2 * i + 1] = y2i.hi + y2i.lo;
    }
}

// ---- out[0] = sum diff^2, out[1] = sum ref^2 (one block, fixed order) ------
__device__ __forceinline__ void norms_body(const double* diff, const double* ref, int64_t len, double* out) {
    __shared__ double sd[256], sr[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < len; i += 256) {
        a += diff[i] * diff[i];
        b += ref[i] * ref[i];
    }
    sd[threadIdx.x] = a;
    sr[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sd[threadIdx.x] += sd[threadIdx.x + w];
            sr[threadIdx.x] += sr[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sd[0];
        out[1] = sr[0];
    }
}

// ---- C = alpha * ldexp(acc, E+F) + beta * C (same arithmetic as the fused
// GEMM epilogue); NaN where a scale marks Inf/NaN input ---------------------
__device__ __forceinline__ void finalize_body(const double* acc, int64_t Mp, const int32_t* EA, const int32_t* FB,
                                              double* C, int64_t ldc, int64_t m, int64_t n, int cplx, double ar,
                                              double ai, double br, double bi, int beta_zero, int64_t i, int64_t j0,
                                              int64_t jstep) {
    if (i >= m) return;
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    const int32_t e = EA[i];
    const int64_t r_re = cplx ? 32 * (i >> 4) + 16 * ((i >> 3) & 1) + (i & 7) : i;
    for (int64_t j = j0; j < n; j += jstep) {
        const int32_t f = FB[j];
        const bool bad = e == kNonFiniteExp || f == kNonFiniteExp;
        if (!cplx) {
            double* c = C + i + j * ldc;
            double out = nan;
            if (!bad) {
                const double v = ldexp(acc[j * Mp + r_re], e + f);
                out = ar * v;
                if (!beta_zero) out = out + br * (*c);
            }
            *c = out;
        } else {
            double* c = C + 2 * (i + j * ldc);
            double outr = nan, outi = nan;
            if (!bad) {
                const double vr = ldexp(acc[j * Mp + r_re], e + f);
                const double vi = ldexp(acc[j * Mp + r_re + 8], e + f);
                outr = ar * vr - ai * vi;
                outi = ar * vi + ai * vr;
                if (!beta_zero) {
                    const double cr = c[0], cim = c[1];
                    outr = outr + (br * cr - bi * cim);
                    outi = outi + (br * cim + bi * cr);
                }
            }
            c[0] = outr;
            c[1] = outi;
        }
    }
}

// ---- the 3-real-product form: combine the raw sums of T1, T2, T3 into C ----
struct Final3 {
    const double* acc[3];
    int64_t Mp;
    const int32_t* EA[3];
    const int32_t* FB[3];
    double* C;
    int64_t ldc, m, n;
    double ar, ai, br, bi;
    int beta_zero;
};

__global__ void finalize3_kernel(Final3 f) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= f.m) return;
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    const int32_t e0 = f.EA[0][i], e1 = f.EA[1][i], e2 = f.EA[2][i];
    for (int64_t j = blockIdx.y; j < f.n; j += gridDim.y) {
        const int32_t g0 = f.FB[0][j], g1 = f.FB[1][j], g2 = f.FB[2][j];
        const double T1 = (e0 == kNonFiniteExp || g0 == kNonFiniteExp) ? nan : ldexp(f.acc[0][j * f.Mp + i], e0 + g0);
        const double T2 = (e1 == kNonFiniteExp || g1 == kNonFiniteExp) ? nan : ldexp(f.acc[1][j * f.Mp + i], e1 + g1);
        const double T3 = (e2 == kNonFiniteExp || g2 == kNonFiniteExp) ? nan : ldexp(f.acc[2][j * f.Mp + i], e2 + g2);
        const double cr = T1 - T2;
        const double ci = (T3 - T1) - T2;
        double* c = f.C + 2 * (i + j * f.ldc);
        double outr = f.ar * cr - f.ai * ci;
        double outi = f.ar * ci + f.ai * cr;
        if (!f.beta_zero) {
            const double c0 = c[0], c1 = c[1];
            outr = outr + (f.br * c0 - f.bi * c1);
            outi = outi + (f.br * c1 + f.bi * c0);
        }
        c[0] = outr;
        c[1] = outi;
    }
}

// ---- kernels: one product -------------------------------------------------------
__global__ void weights_kernel(CheckArgs c) { weights_body(c, static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x); }
__global__ __launch_bounds__(256) void norms_kernel(const double* diff, const double* ref, int64_t len,
                                                    double* out) {
    norms_body(diff, ref, len, out);
}
__global__ void finalize_kernel(const double* acc, int64_t Mp, const int32_t* EA, const int32_t* FB, double* C,
                                int64_t ldc, int64_t m, int64_t n, int cplx, double ar, double ai, double br,
                                double bi, int beta_zero) {
    finalize_body(acc, Mp, EA, FB, C, ldc, m, n, cplx, ar, ai, br, bi, beta_zero,
                  static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x, blockIdx.y, gridDim.y);
}

// ---- kernels: many products; an item names the product (op) and the block
// index along its phase (bx); products whose flag is 0 are skipped -------------
__global__ void weights_batched_kernel(const CheckArgs* c, const int32_t* active, const BlockItem* items) {
    const BlockItem it = items[blockIdx.x];
    if (!active[it.op]) return;
    weights_body(c[it.op], static_cast<int64_t>(it.bx) * 256 + threadIdx.x);
}
__global__ __launch_bounds__(256) void gemv_b_batched_kernel(const CheckArgs* c, const int32_t* active,
                                                             const BlockItem* items) {
    const BlockItem it = items[blockIdx.x];
    if (!active[it.op]) return;  // uniform over the block
    gemv_b_body(c[it.op], it.bx);
}
__global__ __launch_bounds__(256) void rows_batched_kernel(const CheckArgs* c, const int32_t* active,
                                                           const BlockItem* items) {
    const BlockItem it = items[blockIdx.x];
    if (!active[it.op]) return;  // uniform over the block
    rows_body(c[it.op], it.bx);
}
__global__ __launch_bounds__(256) void norms_batched_kernel(const CheckArgs* c, const int32_t* active) {
    const int p = blockIdx.x;
    if (!active[p]) return;
    norms_body(c[p].diff, c[p].ref, c[p].opa.cplx ? 2 * c[p].opa.nv : c[p].opa.nv, c[p].norms);
}
__global__ void finalize_batched_kernel(const FinalArgs* f, const int32_t* active, const BlockItem* items) {
    const BlockItem it = items[blockIdx.x];
    if (!active[it.op]) return;
    const FinalArgs& a = f[it.op];
    finalize_body(a.acc, a.Mp, a.EA, a.FB, a.C, a.ldc, a.m, a.n, a.cplx, a.ar, a.ai, a.br, a.bi, a.beta_zero,
                  static_cast<int64_t>(it.bx) * 256 + threadIdx.x, 0, 1);
}

}  // namespace

// ---- chunking of the split reductions ----------------------------------------
namespace {
constexpr int64_t kOutBlocks = 2048;  // target blocks of the output-contiguous shape
constexpr int64_t kInWaves = 8192;    // target waves of the term-contiguous shape

struct RedSplit {
    bool out;
    int64_t L, nch, chunk;  // terms, chunks, terms per chunk (nch * chunk >= L)
};

RedSplit red_split(int64_t R, int64_t L, bool out) {
    int64_t nch = 1;
    if (L > 0 && R > 0) {
        if (out) {  // at least 16 terms per thread
            nch = std::min((kOutBlocks + (R + 255) / 256 - 1) / ((R + 255) / 256), (L + 15) / 16);
        } else {    // at least 8 terms per lane
            nch = std::min((kInWaves + R - 1) / R, (L + 511) / 512);
        }
        nch = std::max<int64_t>(nch, 1);
    }
    const int64_t chunk = L > 0 ? (L + nch - 1) / nch : 0;
    if (L > 0) nch = (L + chunk - 1) / chunk;  // no empty chunk
    return {out, L, nch, chunk};
}

template <class Op, class Acc>
hipError_t launch_red(const Op& op, int64_t R, const RedSplit& sp, Acc* part, hipStream_t st) {
    if (R <= 0) return hipSuccess;
    if ((R + 3) / 4 > INT32_MAX || sp.nch > 65535) return hipErrorInvalidValue;
    if (sp.out) {
        dim3 grid(static_cast<unsigned>((R + 255) / 256), static_cast<unsigned>(sp.nch));
        hipLaunchKernelGGL((red_out_kernel<Op, Acc>), grid, dim3(256), 0, st, op, R, sp.L, sp.chunk, part);
    } else {
        dim3 grid(static_cast<unsigned>((R + 3) / 4), static_cast<unsigned>(sp.nch));
        hipLaunchKernelGGL((red_in_kernel<Op, Acc>), grid, dim3(256), 0, st, op, R, sp.L, sp.chunk, part);
    }
    return hipGetLastError();
}
}  // namespace

int64_t red_entries(int64_t R, int64_t L) {
    const RedSplit a = red_split(R, L, true), b = red_split(R, L, false);
    return std::max(a.nch, b.nch) * std::max<int64_t>(R, 1);
}

size_t check_part_bytes(int64_t m, int64_t n, int64_t k) {
    const int64_t e = std::max(std::max(red_entries(k, n), red_entries(m, n)),
                               std::max(red_entries(m, k), red_entries(n, k)));
    return sizeof(double) * 4 * static_cast<size_t>(e);
}

hipError_t launch_vec_stats(const OperandView& op, const uint64_t* maxbits, double* ms, double* part, hipStream_t st) {
    if (op.nv <= 0) return hipSuccess;
    const RedSplit sp = red_split(op.nv, op.k, op.sv == 1);
    hipError_t e = launch_red(OpMsq{op, maxbits}, op.nv, sp, part, st);
    if (e != hipSuccess) return e;
    const double denom = static_cast<double>(op.k) * (op.cplx ? 2.0 : 1.0);
    hipLaunchKernelGGL(msq_sum_kernel, dim3(static_cast<unsigned>((op.nv + 31) / 32)), dim3(256), 0, st, part, op.nv,
                       sp.nch, denom, ms);
    return hipGetLastError();
}

hipError_t launch_residual(const CheckArgs& c, hipStream_t st) {
    const int64_t n = c.opb.nv, k = c.opa.k, m = c.opa.nv;
    if (m <= 0 || n <= 0) return hipSuccess;
    DC* p1 = reinterpret_cast<DC*>(c.part1);
    DC* p2 = reinterpret_cast<DC*>(c.part2);
    hipLaunchKernelGGL(weights_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, c);
    hipError_t e = hipGetLastError();
    // u = op(B) t over the n columns (partials in part1), then summed into u
    if (e == hipSuccess && k > 0) {
        const RedSplit su = red_split(k, n, c.opb.sl == 1);
        e = launch_red(OpU{c.opb, c.t}, k, su, p1, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(u_sum_kernel, dim3(static_cast<unsigned>((k + 31) / 32)), dim3(256), 0, st, p1, k,
                               su.nch, c.u);
            e = hipGetLastError();
        }
    }
    // y1 over the n columns of the FP64 sums (part1), y2 over the k terms (part2)
    const RedSplit s1 = red_split(m, n, true), s2 = red_split(m, k, c.opa.sv == 1);
    if (e == hipSuccess) {
        if (c.z3)
            e = launch_red(OpY1z3{{c.acc3[0], c.acc3[1], c.acc3[2]}, c.Mp, {c.EA3[0], c.EA3[1], c.EA3[2]},
                                  {c.FB3[0], c.FB3[1], c.FB3[2]}, c.t},
                           m, s1, p1, st);
        else
            e = launch_red(OpY1{c.acc, c.Mp, c.EA, c.FB, c.t, c.opa.cplx}, m, s1, p1, st);
    }
    if (e == hipSuccess) e = launch_red(OpY2{c.opa, c.u}, m, s2, p2, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rows_combine_kernel, dim3(static_cast<unsigned>((m + 31) / 32)), dim3(256), 0, st, c, s1.nch,
                       s2.nch);
    const int64_t len = c.opa.cplx ? 2 * m : m;
    hipLaunchKernelGGL(norms_kernel, dim3(1), dim3(256), 0, st, c.diff, c.ref, len, c.norms);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* acc, int64_t Mp, const int32_t* EA, const int32_t* FB, double* C,
                           int64_t ldc, int64_t m, int64_t n, int cplx, double ar, double ai, double br, double bi,
                           int beta_zero, hipStream_t st) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>(n < 65535 ? n : 65535));
    hipLaunchKernelGGL(finalize_kernel, grid, dim3(256), 0, st, acc, Mp, EA, FB, C, ldc, m, n, cplx, ar, ai, br, bi,
                       beta_zero);
    return hipGetLastError();
}

hipError_t launch_finalize3(const double* const* acc3, int64_t Mp, const int32_t* const* EA3,
                            const int32_t* const* FB3, double* C, int64_t ldc, int64_t m, int64_t n, double ar,
                            double ai, double br, double bi, int beta_zero, hipStream_t st) {
    if (m <= 0 || n <= 0) return hipSuccess;
    Final3 f;
    for (int q = 0; q < 3; ++q) {
        f.acc[q] = acc3[q];
        f.EA[q] = EA3[q];
        f.FB[q] = FB3[q];
    }
    f.Mp = Mp;
    f.C = C;
    f.ldc = ldc;
    f.m = m;
    f.n = n;
    f.ar = ar;
    f.ai = ai;
    f.br = br;
    f.bi = bi;
    f.beta_zero = beta_zero;
    dim3 grid(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>(n < 65535 ? n : 65535));
    hipLaunchKernelGGL(finalize3_kernel, grid, dim3(256), 0, st, f);
    return hipGetLastError();
}

hipError_t launch_residual_batched(const CheckArgs* c, int64_t nprob, const int32_t* active, const BlockItem* wt_items,
                                   int64_t n_wt, const BlockItem* gv_items, int64_t n_gv, const BlockItem* row_items,
                                   int64_t n_row, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    if (n_wt > 0)
        hipLaunchKernelGGL(weights_batched_kernel, dim3(static_cast<unsigned>(n_wt)), dim3(256), 0, st, c, active,
                           wt_items);
    if (n_gv > 0)
        hipLaunchKernelGGL(gemv_b_batched_kernel, dim3(static_cast<unsigned>(n_gv)), dim3(256), 0, st, c, active,
                           gv_items);
    if (n_row > 0)
        hipLaunchKernelGGL(rows_batched_kernel, dim3(static_cast<unsigned>(n_row)), dim3(256), 0, st, c, active,
                           row_items);
    hipLaunchKernelGGL(norms_batched_kernel, dim3(static_cast<unsigned>(nprob)), dim3(256), 0, st, c, active);
    return hipGetLastError();
}

hipError_t launch_finalize_batched(const FinalArgs* f, const int32_t* active, const BlockItem* items, int64_t nitems,
                                   hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_batched_kernel, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, st, f, active,
                       items);
    return hipGetLastError();
}

}  // namespace oz
