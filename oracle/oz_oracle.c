/*
 * oz_oracle.c -- CPU oracle for FP64 / complex-FP64 GEMM and its Ozaki-scheme
 * INT8 emulation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the GPU path.
 *
 * Plain, slow and written to be checked by eye.  Storage is BLAS column-major:
 * op(A) is m x k, op(B) is k x n, C is m x n, element (i, j) of C at
 * C[i + j*ldc].  trans is 'N', 'T' or 'C' ('C' conjugates; for real data it
 * equals 'T').
 *
 * Part I, the product the method approximates (Sec. 2.2: the emulation
 * stands in for an FP64 GEMM; double-double arithmetic is named there as the
 * classic way to go beyond FP64):
 *   O1  oro_gemm_plain : FP64 GEMM, one dot product per entry in l order.
 *   O2  oro_gemm_dd    : compensated dot product (Dot2, Ogita-Rump-Oishi
 *                        2005) per entry, alpha/beta in double-double,
 *                        rounded once.  Accuracy reference.
 *
 * Part II, the emulation (Sec. 2.2: split each matrix into low-precision
 * slices, multiply slices on INT8 units with INT32 accumulation, accumulate
 * at higher precision; Sec. 3.1: precision set by the number of splits s;
 * Sec. 4: cost grows quadratically in s).  The readings used where the paper
 * is silent:
 *   - one power-of-two scale per row of op(A) and per column of op(B): the
 *     frexp exponent E of the largest magnitude (0 for an all-zero vector);
 *     for complex data the largest real or imaginary part of the vector;
 *   - digits: x*2^(7-E) has magnitude < 128; digit p (p = 1..s) is the
 *     integer part taken toward zero after peeling p-1 base-128 digits, so
 *     every digit lies in [-127, 127] and carries the sign of x;
 *   - slice pairs (p, q) with p + q <= s + 1; the pairs of one anti-diagonal
 *     d = p + q are summed exactly as integers (an INT32 sum on the device);
 *   - k is cut into chunks of kc terms so that an anti-diagonal sum of one
 *     chunk cannot leave INT32; per entry the FP64 value is
 *       acc = sum over chunks (in order), then over d = s+1 down to 2,
 *             of S_{d,chunk} * 2^(-7d)   (plain FP64 adds, in that order)
 *       v   = ldexp(acc, E_i + F_j)
 *   - real:    C = alpha*v + beta*C (two rounded products, one rounded add);
 *              with beta == 0 the old C is not read;
 *   - incremental growth s0 -> s1 (the fallback of a tolerance-driven call):
 *     starting from acc at s0, for s = s0 .. s1-1 the new anti-diagonal
 *     d = s + 2 (pairs p + q = d, 1 <= p, q <= s + 1) is added chunk by chunk:
 *     acc = acc + S_{d,c} * 2^(-7d); digits do not depend on s, so digit s+1
 *     comes from the same scale exponents;
 *   - complex: Cr = sum_l (ar*br - ai*bi), Ci = sum_l (ar*bi + ai*br), every
 *     product of two slices is an exact integer, both parts use the shared
 *     scales, each chunk holds kc/2 values of l (kc even);
 *     out_r = (xr*vr - xi*vi) + (yr*cr - yi*ci),
 *     out_i = (xr*vi + xi*vr) + (yr*ci + yi*cr)  with (xr, xi) = alpha and
 *     (yr, yi) = beta, every product and sum rounded, evaluated as
 *     bracketed; with beta == 0 only the alpha part is formed.
 *
 *
 * Balanced digits (round to nearest; a variant of this library's own, since
 * the paper does not say how the digits are rounded; it gains about one bit
 * per slice over truncation), fixed s <= 8 only:
 *   - the vector's exponent is E' = E, or E + 1 when its largest magnitude M
 *     has M * 2^(7-E) > 127 (then the top digit could round to 128);
 *   - N = |x| * 2^(7 - E' + 8(s-1)) rounded to the nearest integer (ties
 *     away from zero), with the sign of x; |N| <= 127 * 256^(s-1);
 *   - the digits are the unique d_1..d_s with N = sum_p d_p 256^(s-p) and
 *     d_2..d_s in [-128, 127] (d_p = N mod 256 taken in that range, then
 *     N = (N - d_p) / 256); d_1 is what remains, |d_1| <= 127;
 *   - so x = 2^(E'+1) sum_p d_p 2^(-8p) up to half a unit of the last digit,
 *     and the fold weight of anti-diagonal d is 2^(2 - 8d), the final scale
 *     2^(E'_i + F'_j):
 *       acc = sum over chunks, then d = s+1 down to 2, of S_{d,c} * 2^(2-8d);
 *   - every digit product is at most 128^2 in magnitude, so the INT32 chunk
 *     bound is s * kc * 128^2 <= 2^31 - 1;
 *   - complex: Re C is the real emulated product of the rows (ar, -ai)
 *     against (br, bi) over 2k terms, so it takes the digits of the value
 *     -ai, which need not be the negated digits of ai; Im C pairs (ar, ai)
 *     with (bi, br).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (see build.py).
 * -ffp-contract=off keeps every multiply and add separately rounded; the only
 * fused multiply-add is the explicit fma() inside TwoProduct.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } zval;

/* malloc that never returns NULL: the oracle stops loudly when out of memory */
static void* xmalloc(size_t bytes) {
    void* p = malloc(bytes);
    if (p == NULL) {
        fprintf(stderr, "oz_oracle: out of memory (%zu bytes)\n", bytes);
        abort();
    }
    return p;
}

/* ---- operand access -------------------------------------------------- */

static int is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }
static int is_conj(char t) { return t == 'C' || t == 'c'; }

/* element (i, l) of op(A), real storage */
static double opA_d(char ta, const double* A, int64_t lda, int64_t i, int64_t l) {
    return is_trans(ta) ? A[l + i * lda] : A[i + l * lda];
}
/* element (l, j) of op(B), real storage */
static double opB_d(char tb, const double* B, int64_t ldb, int64_t l, int64_t j) {
    return is_trans(tb) ? B[j + l * ldb] : B[l + j * ldb];
}
/* complex storage: interleaved (re, im) doubles */
static zval opA_z(char ta, const double* A, int64_t lda, int64_t i, int64_t l) {
    int64_t idx = is_trans(ta) ? (l + i * lda) : (i + l * lda);
    zval z = { A[2 * idx], A[2 * idx + 1] };
    if (is_conj(ta)) z.im = -z.im;
    return z;
}
static zval opB_z(char tb, const double* B, int64_t ldb, int64_t l, int64_t j) {
    int64_t idx = is_trans(tb) ? (j + l * ldb) : (l + j * ldb);
    zval z = { B[2 * idx], B[2 * idx + 1] };
    if (is_conj(tb)) z.im = -z.im;
    return z;
}

/* row/column subsets: NULL means all, in order */
static int64_t pick(const int64_t* sel, int64_t t) { return sel ? sel[t] : t; }

/* ---- O1: plain FP64 ---------------------------------------------------- */

void oro_dgemm_plain(char ta, char tb, int64_t m, int64_t n, int64_t k, double alpha,
                     const double* A, int64_t lda, const double* B, int64_t ldb,
                     double beta, double* C, int64_t ldc) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int64_t l = 0; l < k; ++l) acc = acc + opA_d(ta, A, lda, i, l) * opB_d(tb, B, ldb, l, j);
            double r = alpha * acc;
            if (beta != 0.0) r = r + beta * C[i + j * ldc];
            C[i + j * ldc] = r;
        }
}

void oro_zgemm_plain(char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                     const double* A, int64_t lda, const double* B, int64_t ldb,
                     const double* beta, double* C, int64_t ldc) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double ar = 0.0, ai = 0.0;
            for (int64_t l = 0; l < k; ++l) {
                zval a = opA_z(ta, A, lda, i, l), b = opB_z(tb, B, ldb, l, j);
                ar = ar + (a.re * b.re - a.im * b.im);
                ai = ai + (a.re * b.im + a.im * b.re);
            }
            double* c = C + 2 * (i + j * ldc);
            double rr = alpha[0] * ar - alpha[1] * ai;
            double ri = alpha[0] * ai + alpha[1] * ar;
            if (beta[0] != 0.0 || beta[1] != 0.0) {
                double cr = c[0], ci = c[1];
                rr = rr + (beta[0] * cr - beta[1] * ci);
                ri = ri + (beta[0] * ci + beta[1] * cr);
            }
            c[0] = rr;
            c[1] = ri;
        }
}

/* ---- O2: double-double ------------------------------------------------- */

typedef struct { double hi, lo; } dd;

static void two_sum(double a, double b, double* s, double* e) {
    double x = a + b, z = x - a;
    *s = x;
    *e = (a - (x - z)) + (b - z);
}
static void two_prod(double a, double b, double* p, double* e) {
    double x = a * b;
    *p = x;
    *e = fma(a, b, -x);
}
static dd dd_norm(double hi, double lo) {
    dd r;
    two_sum(hi, lo, &r.hi, &r.lo);
    return r;
}
static dd dd_add(dd a, dd b) {
    double s, e;
    two_sum(a.hi, b.hi, &s, &e);
    e = e + (a.lo + b.lo);
    return dd_norm(s, e);
}
static dd dd_mul_d(dd a, double b) {
    double p, e;
    two_prod(a.hi, b, &p, &e);
    e = e + a.lo * b;
    return dd_norm(p, e);
}

/* Dot2 state: running sum p and running error s */
typedef struct { double p, s; } dot2;
static void dot2_add(dot2* st, double x, double y) {
    double h, r, q;
    two_prod(x, y, &h, &r);
    two_sum(st->p, h, &st->p, &q);
    st->s = st->s + (q + r);
}
static dd dot2_result(dot2 st) { return dd_norm(st.p, st.s); }

void oro_dgemm_dd(char ta, char tb, int64_t m, int64_t n, int64_t k, double alpha,
                  const double* A, int64_t lda, const double* B, int64_t ldb,
                  double beta, double* C, int64_t ldc, const int64_t* rows, int64_t nr,
                  const int64_t* cols, int64_t nc, double* out, int64_t ldo) {
    /* rows/cols select a sub-block of C; out (nr x nc, ld ldo) receives it.
       C supplies beta*C for the selected entries (indexed in full C). */
    (void)m; (void)n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t jj = 0; jj < nc; ++jj)
        for (int64_t ii = 0; ii < nr; ++ii) {
            int64_t i = pick(rows, ii), j = pick(cols, jj);
            dot2 st = { 0.0, 0.0 };
            for (int64_t l = 0; l < k; ++l) dot2_add(&st, opA_d(ta, A, lda, i, l), opB_d(tb, B, ldb, l, j));
            dd r = dd_mul_d(dot2_result(st), alpha);
            if (beta != 0.0) {
                double p, e;
                two_prod(beta, C[i + j * ldc], &p, &e);
                r = dd_add(r, dd_norm(p, e));
            }
            out[ii + jj * ldo] = r.hi + r.lo;
        }
}

void oro_zgemm_dd(char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                  const double* A, int64_t lda, const double* B, int64_t ldb,
                  const double* beta, const double* C, int64_t ldc, const int64_t* rows, int64_t nr,
                  const int64_t* cols, int64_t nc, double* out, int64_t ldo) {
    (void)m; (void)n;
    int bnz = beta[0] != 0.0 || beta[1] != 0.0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t jj = 0; jj < nc; ++jj)
        for (int64_t ii = 0; ii < nr; ++ii) {
            int64_t i = pick(rows, ii), j = pick(cols, jj);
            dot2 sr = { 0.0, 0.0 }, si = { 0.0, 0.0 };
            for (int64_t l = 0; l < k; ++l) {
                zval a = opA_z(ta, A, lda, i, l), b = opB_z(tb, B, ldb, l, j);
                dot2_add(&sr, a.re, b.re);
                dot2_add(&sr, -a.im, b.im);
                dot2_add(&si, a.re, b.im);
                dot2_add(&si, a.im, b.re);
            }
            dd vr = dot2_result(sr), vi = dot2_result(si);
            /* alpha*v in double-double: (ar*vr - ai*vi, ar*vi + ai*vr) */
            dd rr = dd_add(dd_mul_d(vr, alpha[0]), dd_mul_d(vi, -alpha[1]));
            dd ri = dd_add(dd_mul_d(vi, alpha[0]), dd_mul_d(vr, alpha[1]));
            if (bnz) {
                dd cr = { C[2 * (i + j * ldc)], 0.0 }, ci = { C[2 * (i + j * ldc) + 1], 0.0 };
                rr = dd_add(rr, dd_add(dd_mul_d(cr, beta[0]), dd_mul_d(ci, -beta[1])));
                ri = dd_add(ri, dd_add(dd_mul_d(ci, beta[0]), dd_mul_d(cr, beta[1])));
            }
            out[2 * (ii + jj * ldo)] = rr.hi + rr.lo;
            out[2 * (ii + jj * ldo) + 1] = ri.hi + ri.lo;
        }
}

/* ---- O4: the emulation, step by step ----------------------------------- */

/* Scale exponent of one vector: frexp exponent of its largest magnitude,
   0 for an all-zero vector.  vals holds len doubles (for complex data both
   parts, so the maximum runs over real and imaginary parts). */
static int vec_exponent(const double* vals, int64_t len) {
    double mx = 0.0;
    for (int64_t t = 0; t < len; ++t) {
        double a = fabs(vals[t]);
        if (a > mx) mx = a;
    }
    if (mx == 0.0) return 0;
    int e;
    frexp(mx, &e);
    return e;
}

/* Digits of x under scale exponent E: x*2^(7-E) = t1 + t2/128 + t3/128^2 + ...
   Each step is exact in FP64: ldexp is exact away from underflow (and where
   it underflows every digit up to p = 18 is zero anyway), x - trunc(x) is the
   exact fractional part, and *128 is exact. */
static void digits_of(double a, int E, int s, int8_t* out, int64_t stride) {
    double x = ldexp(a, 7 - E);
    for (int p = 0; p < s; ++p) {
        double t = trunc(x);
        out[p * stride] = (int8_t)t;
        x = (x - t) * 128.0;
    }
}

/* Balanced digits of x under scale exponent E (the vector's E') and slice
   count s (s <= 8).  ldexp is exact here: the result is below 2^63, and where
   it would be subnormal it is below 1/2, which rounds to 0 whatever ldexp
   returns. */
static void digits_bal_of(double a, int E, int s, int8_t* out, int64_t stride) {
    int64_t N = 0;
    if (isfinite(a)) {
        double y = ldexp(fabs(a), 7 - E + 8 * (s - 1));
        double ip = floor(y);
        N = (int64_t)ip + ((y - ip) >= 0.5 ? 1 : 0);
        if (a < 0) N = -N;
    }
    for (int p = s - 1; p >= 1; --p) {
        int64_t r = ((N % 256) + 256) % 256;
        if (r >= 128) r -= 256;
        out[p * stride] = (int8_t)r;
        N = (N - r) / 256;
    }
    out[0] = (int8_t)N;
}

/* Fold weight of anti-diagonal d: 2^(-7d) (truncated digits) or 2^(2-8d)
   (balanced digits). */
static double diag_weight(int d, int bal) { return ldexp(1.0, bal ? 2 - 8 * d : -7 * d); }

/* Split the vectors of an operand.  side 'A': vector v is row v of op(A)
   (nv = m); side 'B': vector v is column v of op(B) (nv = n); length k.
   Real:    dig[(p*nv + v)*k + l]            = digit p+1 of element (v, l)
   Complex: dig[((p*nv + v)*k + l)*2 + part] = digit p+1 of the real (part 0)
            or imaginary (part 1) part, after conjugation by 'C'.
   E[v] receives the scale exponent. */
static void split_impl(char side, char trans, int cplx, int64_t nv, int64_t k, const double* X,
                       int64_t ldx, int s, int32_t* E, int8_t* dig, int bal) {
    int w = cplx ? 2 : 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t v = 0; v < nv; ++v) {
        double* vals = (double*)xmalloc(sizeof(double) * (size_t)(k * w + 1));
        for (int64_t l = 0; l < k; ++l) {
            if (cplx) {
                zval z = (side == 'A') ? opA_z(trans, X, ldx, v, l) : opB_z(trans, X, ldx, l, v);
                vals[2 * l] = z.re;
                vals[2 * l + 1] = z.im;
            } else {
                vals[l] = (side == 'A') ? opA_d(trans, X, ldx, v, l) : opB_d(trans, X, ldx, l, v);
            }
        }
        int e = vec_exponent(vals, k * w);
        if (bal) { /* the top digit must stay within [-127, 127] */
            double mx = 0.0;
            for (int64_t t = 0; t < k * w; ++t)
                if (fabs(vals[t]) > mx) mx = fabs(vals[t]);
            if (mx > 0.0 && isfinite(mx) && ldexp(mx, 7 - e) > 127.0) e = e + 1;
        }
        E[v] = e;
        int64_t stride = nv * k * w; /* distance between digit planes */
        for (int64_t t = 0; t < k * w; ++t) {
            if (bal)
                digits_bal_of(vals[t], e, s, dig + v * k * w + t, stride);
            else
                digits_of(vals[t], e, s, dig + v * k * w + t, stride);
        }
        free(vals);
    }
}

void oro_split(char side, char trans, int cplx, int64_t nv, int64_t k, const double* X,
               int64_t ldx, int s, int32_t* E, int8_t* dig) {
    split_impl(side, trans, cplx, nv, k, X, ldx, s, E, dig, 0);
}

void oro_split_bal(char side, char trans, int cplx, int64_t nv, int64_t k, const double* X,
                   int64_t ldx, int s, int32_t* E, int8_t* dig) {
    split_impl(side, trans, cplx, nv, k, X, ldx, s, E, dig, 1);
}

/* Anti-diagonal sums for one output entry and one chunk [l0, l1) of l:
   S_d = sum over p + q = d (1 <= p, q <= s) of sum_l a_p(l) * b_q(l), exact in
   int64.  da/db point at digit p=1 of this row / column; plane strides ps. */
static void diag_sums_real(const int8_t* da, const int8_t* db, int64_t ps_a, int64_t ps_b,
                           int s, int64_t l0, int64_t l1, int64_t* S /* [s+2] */) {
    for (int d = 0; d < s + 2; ++d) S[d] = 0;
    for (int p = 1; p <= s; ++p)
        for (int q = 1; p + q <= s + 1; ++q) {
            const int8_t* a = da + (p - 1) * ps_a;
            const int8_t* b = db + (q - 1) * ps_b;
            int64_t acc = 0;
            for (int64_t l = l0; l < l1; ++l) acc += (int64_t)a[l] * (int64_t)b[l];
            S[p + q] += acc;
        }
}

static void diag_sums_cplx(const int8_t* da, const int8_t* db, int64_t ps_a, int64_t ps_b,
                           int s, int64_t l0, int64_t l1, int64_t* Sr, int64_t* Si) {
    for (int d = 0; d < s + 2; ++d) Sr[d] = Si[d] = 0;
    for (int p = 1; p <= s; ++p)
        for (int q = 1; p + q <= s + 1; ++q) {
            const int8_t* a = da + (p - 1) * ps_a;
            const int8_t* b = db + (q - 1) * ps_b;
            int64_t accr = 0, acci = 0;
            for (int64_t l = l0; l < l1; ++l) {
                int64_t ar = a[2 * l], ai = a[2 * l + 1], br = b[2 * l], bi = b[2 * l + 1];
                accr += ar * br - ai * bi;
                acci += ar * bi + ai * br;
            }
            Sr[p + q] += accr;
            Si[p + q] += acci;
        }
}

/* Balanced complex sums: the real part is the real emulated product of the
   row (ar, -ai) against (br, bi), so it takes the digits of the value -ai
   (dn, the split of A with negated imaginary parts), which with balanced
   digits need not be the negated digits of ai. */
static void diag_sums_cplx_bal(const int8_t* da, const int8_t* dn, const int8_t* db, int64_t ps_a, int64_t ps_b,
                               int s, int64_t l0, int64_t l1, int64_t* Sr, int64_t* Si) {
    for (int d = 0; d < s + 2; ++d) Sr[d] = Si[d] = 0;
    for (int p = 1; p <= s; ++p)
        for (int q = 1; p + q <= s + 1; ++q) {
            const int8_t* a = da + (p - 1) * ps_a;
            const int8_t* an = dn + (p - 1) * ps_a;
            const int8_t* b = db + (q - 1) * ps_b;
            int64_t accr = 0, acci = 0;
            for (int64_t l = l0; l < l1; ++l) {
                int64_t ar = a[2 * l], ai = a[2 * l + 1], nai = an[2 * l + 1], br = b[2 * l], bi = b[2 * l + 1];
                accr += ar * br + nai * bi;
                acci += ar * bi + ai * br;
            }
            Sr[p + q] += accr;
            Si[p + q] += acci;
        }
}

static double pow2i(int e) { return ldexp(1.0, e); }

/* S_d of one diagonal d only, slices 1..s available (real / complex) */
static void one_diag_real(const int8_t* da, const int8_t* db, int64_t ps_a, int64_t ps_b, int s, int d,
                          int64_t l0, int64_t l1, int64_t* out) {
    int64_t acc = 0;
    for (int p = 1; p <= s; ++p) {
        int q = d - p;
        if (q < 1 || q > s) continue;
        const int8_t* a = da + (p - 1) * ps_a;
        const int8_t* b = db + (q - 1) * ps_b;
        for (int64_t l = l0; l < l1; ++l) acc += (int64_t)a[l] * (int64_t)b[l];
    }
    *out = acc;
}

static void one_diag_cplx(const int8_t* da, const int8_t* db, int64_t ps_a, int64_t ps_b, int s, int d,
                          int64_t l0, int64_t l1, int64_t* outr, int64_t* outi) {
    int64_t accr = 0, acci = 0;
    for (int p = 1; p <= s; ++p) {
        int q = d - p;
        if (q < 1 || q > s) continue;
        const int8_t* a = da + (p - 1) * ps_a;
        const int8_t* b = db + (q - 1) * ps_b;
        for (int64_t l = l0; l < l1; ++l) {
            int64_t ar = a[2 * l], ai = a[2 * l + 1], br = b[2 * l], bi = b[2 * l + 1];
            accr += ar * br - ai * bi;
            acci += ar * bi + ai * br;
        }
    }
    *outr = accr;
    *outi = acci;
}

/* Exported anti-diagonal sums for parity of the integer stage.
   out[((c*(s) + (d-2)) * nc + jj) * nr + ii] = S_{d,c}(rows[ii], cols[jj]) for
   d = 2..s+1, chunk c = 0..nchunks-1 (real: one plane set; complex: the real
   part planes then the imaginary part planes, i.e. out_im = out + nchunks*s*nr*nc). */
void oro_diag_sums(int cplx, int s, int64_t k, int64_t kc, const int8_t* digA, int64_t nvA,
                   const int8_t* digB, int64_t nvB, const int64_t* rows, int64_t nr,
                   const int64_t* cols, int64_t nc, int64_t* out) {
    int w = cplx ? 2 : 1;
    int64_t lchunk = cplx ? kc / 2 : kc;
    int64_t nch = (k + lchunk - 1) / lchunk;
    if (k == 0) nch = 0;
    int64_t plane = nr * nc;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t jj = 0; jj < nc; ++jj) {
        int64_t Sr[64], Si[64];
        for (int64_t ii = 0; ii < nr; ++ii) {
            int64_t i = pick(rows, ii), j = pick(cols, jj);
            const int8_t* da = digA + i * k * w;
            const int8_t* db = digB + j * k * w;
            for (int64_t c = 0; c < nch; ++c) {
                int64_t l0 = c * lchunk, l1 = l0 + lchunk < k ? l0 + lchunk : k;
                if (cplx)
                    diag_sums_cplx(da, db, nvA * k * 2, nvB * k * 2, s, l0, l1, Sr, Si);
                else
                    diag_sums_real(da, db, nvA * k, nvB * k, s, l0, l1, Sr);
                for (int d = 2; d <= s + 1; ++d) {
                    out[((c * s + (d - 2)) * nc + jj) * nr + ii] = Sr[d];
                    if (cplx) out[nch * s * plane + ((c * s + (d - 2)) * nc + jj) * nr + ii] = Si[d];
                }
            }
        }
    }
}

/* Emulated DGEMM on the selected block.  C (full, ldc) provides beta*C for the
   selected entries; out (nr x nc, ldo) receives the result. */
static void emu_dgemm_impl(char ta, char tb, int64_t m, int64_t n, int64_t k, double alpha,
                           const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                           const double* C, int64_t ldc, int s, int s1, int64_t kc, const int64_t* rows,
                           int64_t nr, const int64_t* cols, int64_t nc, double* out, int64_t ldo, int bal) {
    /* s1 >= s: grow incrementally from s to s1 (s1 == s: plain emulation) */
    int sd = s1 > s ? s1 : s; /* digits needed */
    int32_t* EA = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t* FB = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    int8_t* dA = (int8_t*)xmalloc((size_t)(sd * m * k + 1));
    int8_t* dB = (int8_t*)xmalloc((size_t)(sd * n * k + 1));
    split_impl('A', ta, 0, m, k, A, lda, sd, EA, dA, bal);
    split_impl('B', tb, 0, n, k, B, ldb, sd, FB, dB, bal);
    int64_t nch = k > 0 ? (k + kc - 1) / kc : 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t jj = 0; jj < nc; ++jj) {
        int64_t S[64];
        for (int64_t ii = 0; ii < nr; ++ii) {
            int64_t i = pick(rows, ii), j = pick(cols, jj);
            double acc = 0.0;
            for (int64_t c = 0; c < nch; ++c) {
                int64_t l0 = c * kc, l1 = l0 + kc < k ? l0 + kc : k;
                diag_sums_real(dA + i * k, dB + j * k, m * k, n * k, s, l0, l1, S);
                for (int d = s + 1; d >= 2; --d) acc = acc + (double)S[d] * diag_weight(d, bal);
            }
            for (int st = s; st < sd; ++st) {
                int d = st + 2;
                for (int64_t c = 0; c < nch; ++c) {
                    int64_t l0 = c * kc, l1 = l0 + kc < k ? l0 + kc : k, Sd;
                    one_diag_real(dA + i * k, dB + j * k, m * k, n * k, st + 1, d, l0, l1, &Sd);
                    acc = acc + (double)Sd * diag_weight(d, bal);
                }
            }
            double v = ldexp(acc, EA[i] + FB[j]);
            double r = alpha * v;
            if (beta != 0.0) r = r + beta * C[i + j * ldc];
            out[ii + jj * ldo] = r;
        }
    }
    free(EA); free(FB); free(dA); free(dB);
}

void oro_emu_dgemm(char ta, char tb, int64_t m, int64_t n, int64_t k, double alpha,
                   const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                   const double* C, int64_t ldc, int s, int s1, int64_t kc, const int64_t* rows, int64_t nr,
                   const int64_t* cols, int64_t nc, double* out, int64_t ldo) {
    emu_dgemm_impl(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s, s1, kc, rows, nr, cols, nc, out, ldo,
                   0);
}

/* Balanced digits (fixed s: s1 is ignored) */
void oro_emu_dgemm_bal(char ta, char tb, int64_t m, int64_t n, int64_t k, double alpha,
                       const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                       const double* C, int64_t ldc, int s, int64_t kc, const int64_t* rows, int64_t nr,
                       const int64_t* cols, int64_t nc, double* out, int64_t ldo) {
    emu_dgemm_impl(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s, s, kc, rows, nr, cols, nc, out, ldo, 1);
}

static void emu_zgemm_impl(char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                           const double* A, int64_t lda, const double* B, int64_t ldb, const double* beta,
                           const double* C, int64_t ldc, int s, int s1, int64_t kc, const int64_t* rows,
                           int64_t nr, const int64_t* cols, int64_t nc, double* out, int64_t ldo, int bal) {
    int sd = s1 > s ? s1 : s;
    int32_t* EA = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t* FB = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    int8_t* dA = (int8_t*)xmalloc((size_t)(2 * sd * m * k + 1));
    int8_t* dB = (int8_t*)xmalloc((size_t)(2 * sd * n * k + 1));
    split_impl('A', ta, 1, m, k, A, lda, sd, EA, dA, bal);
    split_impl('B', tb, 1, n, k, B, ldb, sd, FB, dB, bal);
    int8_t* dN = NULL; /* balanced: digits of A with negated imaginary parts */
    if (bal) {
        int64_t ra = (ta == 'N' || ta == 'n') ? m : k, ca = (ta == 'N' || ta == 'n') ? k : m;
        double* An = (double*)xmalloc(sizeof(double) * (size_t)(2 * lda * (ca > 0 ? ca : 1) + 2));
        for (int64_t c = 0; c < ca; ++c)
            for (int64_t r = 0; r < ra; ++r) {
                An[2 * (r + c * lda)] = A[2 * (r + c * lda)];
                An[2 * (r + c * lda) + 1] = -A[2 * (r + c * lda) + 1];
            }
        int32_t* En = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(m + 1));
        dN = (int8_t*)xmalloc((size_t)(2 * sd * m * k + 1));
        split_impl('A', ta, 1, m, k, An, lda, sd, En, dN, 1);
        free(An);
        free(En);
    }
    int64_t lchunk = kc / 2;
    int64_t nch = k > 0 ? (k + lchunk - 1) / lchunk : 0;
    int bnz = beta[0] != 0.0 || beta[1] != 0.0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t jj = 0; jj < nc; ++jj) {
        int64_t Sr[64], Si[64];
        for (int64_t ii = 0; ii < nr; ++ii) {
            int64_t i = pick(rows, ii), j = pick(cols, jj);
            double accr = 0.0, acci = 0.0;
            for (int64_t c = 0; c < nch; ++c) {
                int64_t l0 = c * lchunk, l1 = l0 + lchunk < k ? l0 + lchunk : k;
                if (bal)
                    diag_sums_cplx_bal(dA + i * k * 2, dN + i * k * 2, dB + j * k * 2, m * k * 2, n * k * 2, s, l0,
                                       l1, Sr, Si);
                else
                    diag_sums_cplx(dA + i * k * 2, dB + j * k * 2, m * k * 2, n * k * 2, s, l0, l1, Sr, Si);
                for (int d = s + 1; d >= 2; --d) {
                    accr = accr + (double)Sr[d] * diag_weight(d, bal);
                    acci = acci + (double)Si[d] * diag_weight(d, bal);
                }
            }
            for (int st = s; st < sd; ++st) {
                int d = st + 2;
                for (int64_t c = 0; c < nch; ++c) {
                    int64_t l0 = c * lchunk, l1 = l0 + lchunk < k ? l0 + lchunk : k, Sdr, Sdi;
                    one_diag_cplx(dA + i * k * 2, dB + j * k * 2, m * k * 2, n * k * 2, st + 1, d, l0, l1, &Sdr, &Sdi);
                    accr = accr + (double)Sdr * diag_weight(d, bal);
                    acci = acci + (double)Sdi * diag_weight(d, bal);
                }
            }
            double vr = ldexp(accr, EA[i] + FB[j]);
            double vi = ldexp(acci, EA[i] + FB[j]);
            double rr = alpha[0] * vr - alpha[1] * vi;
            double ri = alpha[0] * vi + alpha[1] * vr;
            if (bnz) {
                double cr = C[2 * (i + j * ldc)], ci = C[2 * (i + j * ldc) + 1];
                rr = rr + (beta[0] * cr - beta[1] * ci);
                ri = ri + (beta[0] * ci + beta[1] * cr);
            }
            out[2 * (ii + jj * ldo)] = rr;
            out[2 * (ii + jj * ldo) + 1] = ri;
        }
    }
    free(EA); free(FB); free(dA); free(dB); free(dN);
}

void oro_emu_zgemm(char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                   const double* A, int64_t lda, const double* B, int64_t ldb, const double* beta,
                   const double* C, int64_t ldc, int s, int s1, int64_t kc, const int64_t* rows, int64_t nr,
                   const int64_t* cols, int64_t nc, double* out, int64_t ldo) {
    emu_zgemm_impl(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s, s1, kc, rows, nr, cols, nc, out, ldo,
                   0);
}

void oro_emu_zgemm_bal(char ta, char tb, int64_t m, int64_t n, int64_t k, const double* alpha,
                       const double* A, int64_t lda, const double* B, int64_t ldb, const double* beta,
                       const double* C, int64_t ldc, int s, int64_t kc, const int64_t* rows, int64_t nr,
                       const int64_t* cols, int64_t nc, double* out, int64_t ldo) {
    emu_zgemm_impl(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s, s, kc, rows, nr, cols, nc, out, ldo, 1);
}

/* ---- products beyond FP64: the same sums folded into a double-double ---- */

/* (hi, lo) + x, x exactly representable: TwoSum of hi and x, the error added
   to lo, then a fast TwoSum renormalisation. */
static void dd_add_exact(double* hi, double* lo, double x) {
    double s = *hi + x;
    double bb = s - *hi;
    double err = (*hi - (s - bb)) + (x - bb);
    double t = *lo + err;
    double h = s + t;
    *lo = t - (h - s);
    *hi = h;
}

/* C = op(A) op(B) at s slices, the anti-diagonal sums of each INT32 chunk
   folded from d = s+1 down to 2 into (hi, lo); outputs ldexp(hi, E+F) and
   ldexp(lo, E+F) for the selected block (ldo). */
void oro_emu_dgemm_x2(char ta, char tb, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                      const double* B, int64_t ldb, int s, int64_t kc, const int64_t* rows, int64_t nr,
                      const int64_t* cols, int64_t nc, double* out_hi, double* out_lo, int64_t ldo) {
    int32_t* EA = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t* FB = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    int8_t* dA = (int8_t*)xmalloc((size_t)(s * m * k + 1));
    int8_t* dB = (int8_t*)xmalloc((size_t)(s * n * k + 1));
    oro_split('A', ta, 0, m, k, A, lda, s, EA, dA);
    oro_split('B', tb, 0, n, k, B, ldb, s, FB, dB);
    int64_t nch = k > 0 ? (k + kc - 1) / kc : 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t jj = 0; jj < nc; ++jj) {
        int64_t S[64];
        for (int64_t ii = 0; ii < nr; ++ii) {
            int64_t i = pick(rows, ii), j = pick(cols, jj);
            double hi = 0.0, lo = 0.0;
            for (int64_t c = 0; c < nch; ++c) {
                int64_t l0 = c * kc, l1 = l0 + kc < k ? l0 + kc : k;
                diag_sums_real(dA + i * k, dB + j * k, m * k, n * k, s, l0, l1, S);
                for (int d = s + 1; d >= 2; --d) dd_add_exact(&hi, &lo, (double)S[d] * pow2i(-7 * d));
            }
            out_hi[ii + jj * ldo] = ldexp(hi, EA[i] + FB[j]);
            out_lo[ii + jj * ldo] = ldexp(lo, EA[i] + FB[j]);
        }
    }
    free(EA); free(FB); free(dA); free(dB);
}

/* Complex form: real and imaginary parts each a double-double (interleaved). */
void oro_emu_zgemm_x2(char ta, char tb, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                      const double* B, int64_t ldb, int s, int64_t kc, const int64_t* rows, int64_t nr,
                      const int64_t* cols, int64_t nc, double* out_hi, double* out_lo, int64_t ldo) {
    int32_t* EA = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t* FB = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    int8_t* dA = (int8_t*)xmalloc((size_t)(2 * s * m * k + 1));
    int8_t* dB = (int8_t*)xmalloc((size_t)(2 * s * n * k + 1));
    oro_split('A', ta, 1, m, k, A, lda, s, EA, dA);
    oro_split('B', tb, 1, n, k, B, ldb, s, FB, dB);
    int64_t lchunk = kc / 2;
    int64_t nch = k > 0 ? (k + lchunk - 1) / lchunk : 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t jj = 0; jj < nc; ++jj) {
        int64_t Sr[64], Si[64];
        for (int64_t ii = 0; ii < nr; ++ii) {
            int64_t i = pick(rows, ii), j = pick(cols, jj);
            double hr = 0.0, lr = 0.0, hi_ = 0.0, li = 0.0;
            for (int64_t c = 0; c < nch; ++c) {
                int64_t l0 = c * lchunk, l1 = l0 + lchunk < k ? l0 + lchunk : k;
                diag_sums_cplx(dA + i * k * 2, dB + j * k * 2, m * k * 2, n * k * 2, s, l0, l1, Sr, Si);
                for (int d = s + 1; d >= 2; --d) {
                    dd_add_exact(&hr, &lr, (double)Sr[d] * pow2i(-7 * d));
                    dd_add_exact(&hi_, &li, (double)Si[d] * pow2i(-7 * d));
                }
            }
            int e = EA[i] + FB[j];
            out_hi[2 * (ii + jj * ldo)] = ldexp(hr, e);
            out_hi[2 * (ii + jj * ldo) + 1] = ldexp(hi_, e);
            out_lo[2 * (ii + jj * ldo)] = ldexp(lr, e);
            out_lo[2 * (ii + jj * ldo) + 1] = ldexp(li, e);
        }
    }
    free(EA); free(FB); free(dA); free(dB);
}

int oro_num_threads(void) {
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}
