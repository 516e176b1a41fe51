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
// estimates the scale-weighted Frobenius error || D1 (C_emu - AB) D2 ||_F /
// || D1 AB D2 ||_F (for +-1 entries E||X sigma||^2 = ||X||_F^2).  Both sides use
// the same rounded weights t_j = D2_jj * sigma_j and w_i = D1_ii, so y1 - y2
// carries the emulation error only.  The work is O(mk + kn + mn), against
// O(mnk) for the product itself.
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

// ---- per-vector mean square of x * 2^-E ------------------------------------
// One block per 64 vectors; 4 waves split the terms; fixed-order reduction.
__global__ __launch_bounds__(256) void vec_stats_kernel(OperandView op, const uint64_t* maxbits, double* ms) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t v = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    double acc = 0.0;
    if (v < op.nv) {
        const uint64_t mb = maxbits[v];
        int E = 0;
        if (mb != 0 && mb < 0x7ff0000000000000ull) frexp(max_of_bits(mb), &E);
        for (int64_t l = wave; l < op.k; l += 4) {
            double re, im;
            load_elem(op, v, l, re, im);
            const double a = ldexp(re, -E), b = ldexp(im, -E);
            acc += a * a + b * b;
        }
    }
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && v < op.nv) {
        const double t = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        ms[v] = op.k > 0 ? t / (static_cast<double>(op.k) * (op.cplx ? 2.0 : 1.0)) : 0.0;
    }
}

// ---- t_j = sigma_j / max|op(B)_:j| ------------------------------------------
__device__ __forceinline__ void weights_body(const CheckArgs& c, int64_t j) {
    if (j >= c.opb.nv) return;
    const double mx = max_of_bits(c.maxb[j]);
    c.t[j] = mx > 0.0 ? rademacher(c.seed, j) / mx : 0.0;
}

// ---- u = op(B) t in double-double; u[l] = (re.hi, re.lo, im.hi, im.lo) ------
// Block: 64 terms (lanes) x 4 parts (waves); part w sums the columns
// j = w, w + 4, ...; the four partial sums are added in part order.
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    const dd s = two_sum(a.hi, b.hi);
    return {s.hi, s.lo + (a.lo + b.lo)};
}
constexpr int kParts = 4;
constexpr int kLanes = 64;

__device__ __forceinline__ void gemv_b_body(const CheckArgs& c, int64_t lb) {
    __shared__ dd red[kParts][2][kLanes];
    const OperandView& opb = c.opb;
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int64_t l = lb * kLanes + lane;
    dd sr = {0.0, 0.0}, si = {0.0, 0.0};
    if (l < opb.k) {
        for (int64_t j = part; j < opb.nv; j += kParts) {
            double re, im;
            load_elem(opb, j, l, re, im);
            const double tj = c.t[j];
            sr = dd_add_prod(sr, re, tj);
            si = dd_add_prod(si, im, tj);
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

// ---- per row i of op(A): y2 = w_i op(A)_i: u, y1 = w_i sum_j C_emu_ij t_j ----
// Writes diff[i] = y1 - y2 and ref[i] = y2 (real, or real and imaginary parts
// at 2i, 2i+1 for complex).  Block: 64 rows (lanes) x 4 parts (waves); part w
// takes the terms l = w, w + 4, ... and the columns j = w, w + 4, ...; the
// partial sums are added in part order.
__device__ __forceinline__ void rows_body(const CheckArgs& c, int64_t rb) {
    __shared__ dd red[kParts][4][kLanes];
    const OperandView& opa = c.opa;
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int64_t i = rb * kLanes + lane;
    const int64_t Mp = c.Mp, n = c.opb.nv;
    const double* u = c.u;
    dd y2r = {0.0, 0.0}, y2i = {0.0, 0.0}, y1r = {0.0, 0.0}, y1i = {0.0, 0.0};
    if (i < opa.nv) {
        // y2 = a_i . u  (complex: (ar + i ai)(ur + i ui))
        for (int64_t l = part; l < opa.k; l += kParts) {
            double ar, ai;
            load_elem(opa, i, l, ar, ai);
            const double urh = u[4 * l], url = u[4 * l + 1], uih = u[4 * l + 2], uil = u[4 * l + 3];
            y2r = dd_add_prod(y2r, ar, urh);
            y2r = dd_add_prod(y2r, ar, url);
            if (opa.cplx) {
                y2r = dd_add_prod(y2r, -ai, uih);
                y2r = dd_add_prod(y2r, -ai, uil);
                y2i = dd_add_prod(y2i, ar, uih);
                y2i = dd_add_prod(y2i, ar, uil);
                y2i = dd_add_prod(y2i, ai, urh);
                y2i = dd_add_prod(y2i, ai, url);
            }
        }
        // y1 = sum_j ldexp(acc_ij, E_i + F_j) t_j over the slice-row(s) of row i
        const int64_t r_re = opa.cplx ? 32 * (i >> 4) + 16 * ((i >> 3) & 1) + (i & 7) : i;
        const int64_t r_im = r_re + 8;
        const int32_t e = c.EA[i];
        for (int64_t j = part; j < n; j += kParts) {
            const int ef = e + c.FB[j];
            const double tj = c.t[j];
            y1r = dd_add_prod(y1r, ldexp(c.acc[j * Mp + r_re], ef), tj);
            if (opa.cplx) y1i = dd_add_prod(y1i, ldexp(c.acc[j * Mp + r_im], ef), tj);
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
    if (!opa.cplx) {
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

// ---- kernels: one product -------------------------------------------------------
__global__ void weights_kernel(CheckArgs c) { weights_body(c, static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x); }
__global__ __launch_bounds__(256) void gemv_b_kernel(CheckArgs c) { gemv_b_body(c, blockIdx.x); }
__global__ __launch_bounds__(256) void rows_kernel(CheckArgs c) { rows_body(c, blockIdx.x); }
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

hipError_t launch_vec_stats(const OperandView& op, const uint64_t* maxbits, double* ms, hipStream_t st) {
    if (op.nv <= 0) return hipSuccess;
    hipLaunchKernelGGL(vec_stats_kernel, dim3(static_cast<unsigned>((op.nv + 63) / 64)), dim3(256), 0, st, op, maxbits,
                       ms);
    return hipGetLastError();
}

hipError_t launch_residual(const CheckArgs& c, hipStream_t st) {
    const int64_t n = c.opb.nv, k = c.opa.k, m = c.opa.nv;
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(weights_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, c);
    if (k > 0) hipLaunchKernelGGL(gemv_b_kernel, dim3(static_cast<unsigned>((k + 63) / 64)), dim3(256), 0, st, c);
    hipLaunchKernelGGL(rows_kernel, dim3(static_cast<unsigned>((m + 63) / 64)), dim3(256), 0, st, c);
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
