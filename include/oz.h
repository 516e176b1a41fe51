/*
 * oz.h -- C ABI of the Ozaki-scheme FP64 / complex-FP64 GEMM emulation on
 * INT8 matrix cores (AMD Instinct MI355X, gfx950).
 *
 * The method (paper Sec. 2.2): each FP64 operand is split into s INT8 slices
 * under a power-of-two scale per row of op(A) and per column of op(B); the
 * slice products run on INT8 matrix units with INT32 accumulation and are
 * rescaled and summed in FP64.  The number of splits s sets the precision
 * (Sec. 3.1, modes with 3 to 18 splits; Sec. 4: about two decimal digits per
 * split, cost quadratic in s).  The paper reaches the emulation through
 * intercepted BLAS dgemm/zgemm calls (Sec. 3.1), so the entry points below
 * keep the BLAS argument list.
 *
 * Conventions shared by every entry point
 *  - Storage is BLAS column-major.  op(A) is m x k, op(B) is k x n, C is
 *    m x n; element (i, j) of C lives at C[i + j*ldc].  trans is 'N', 'T' or
 *    'C' (either case); for real data 'C' means 'T'.
 *  - A, B, C and every other array argument named "device" are device
 *    pointers owned by the caller; alpha and beta are host pointers.
 *  - Work is enqueued on the handle's stream and the call returns without
 *    waiting, unless a report is requested (rep != NULL), in which case the
 *    call waits for its own work so that it can fill the report.
 *  - C must not overlap A or B.  Calls on one handle must not overlap in time
 *    from several host threads (the handle owns one workspace).
 *  - Return value: 0 on success; a positive value is the position of the
 *    first invalid argument, counted as in reference BLAS (1 transa,
 *    2 transb, 3 m, 4 n, 5 k, 8 lda, 10 ldb, 13 ldc, 14 prec); a negative
 *    value is one of the OZ_ERR_* codes below.  Nothing is enqueued when a
 *    call returns nonzero.
 *  - Quick returns as in reference BLAS: m = 0 or n = 0 does nothing; when
 *    alpha = 0 or k = 0, C = beta*C (exact zeros when beta = 0, C not read).
 *  - Non-finite inputs: the scale of a row of op(A) or column of op(B) that
 *    holds an Inf or NaN is undefined; every entry of C that depends on such
 *    a row or column is set to NaN, the other entries are computed normally,
 *    and the report (if requested) carries status OZ_ERR_NONFINITE.
 */
#ifndef OZ_H
#define OZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    OZ_OK = 0,
    OZ_ERR_HIP = -1,         /* a HIP runtime call failed                         */
    OZ_ERR_ALLOC = -2,       /* device workspace allocation failed or too small   */
    OZ_ERR_NONFINITE = -3,   /* an input row / column held Inf or NaN (report only) */
    OZ_ERR_HANDLE = -4,      /* NULL or destroyed handle                          */
    OZ_ERR_UNSUPPORTED = -5, /* no gfx950 device, or a size beyond the int32 grid  */
    OZ_ERR_ARG = -6          /* invalid argument of a non-BLAS entry point        */
};

/* Largest slice count accepted (the paper's modes run up to 18 splits). */
#define OZ_MAX_SLICES 18

typedef struct oz_handle_s* oz_handle_t;

/* Precision request.
 *  slices : s in 1..OZ_MAX_SLICES, the number of INT8 slices per operand
 *           (Sec. 3.1 "fp64_int8_<s>" modes); 0 selects s from tol.
 *  tol    : target when slices == 0 (must then be > 0): the scale-weighted
 *           relative error || D1 (C - AB) D2 ||_F / || D1 AB D2 ||_F with
 *           D1 = diag(1 / max|op(A)_i:|), D2 = diag(1 / max|op(B)_:j|), on
 *           the product before alpha/beta.  The call picks a starting s for
 *           tol/2 by a rule on operand statistics (oz_select_slices) or the
 *           learned selector, emulates, checks the result a posteriori with a
 *           randomised double-double residual, and while the estimate exceeds
 *           tol/2 adds ceil(log2(estimate / (tol/2)) / 6) slices, at least one
 *           (each the next digit and the next anti-diagonal, added last, in
 *           turn) up to smax, then checks again.  The one-probe estimate lies
 *           within about 0.7x .. 1.4x of the true error, so the margin of 2
 *           keeps the true error within tol; the error falls by at least about
 *           2^6 per slice.  Sec. 4 of the paper motivates adjusting the split
 *           number to the operator.
 *           Tolerance-driven calls synchronise their stream.
 *  smax   : largest s the tol-driven selection may use (0: 12).
 *  kchunk : products per INT32 chunk along k; 0 picks the largest multiple of
 *           64 with s*kchunk*127^2 <= 2^31-1; a nonzero value must be a
 *           positive multiple of 64 not above that bound (used to exercise
 *           the chunked accumulation on small k).
 *  zmode  : complex only.  4: the 4-real-product form -- one real
 *           emulated product over the two-row form of op(A) (see oz_zgemm).
 *           0 (and a NULL prec): the form measured faster -- the 3-real-
 *           product form for a single fixed-s call (not the double-double
 *           one) with m, n and k all at least 2048, the 4-product form
 *           otherwise (tolerance-driven and batched calls, small products,
 *           k below 2048 as in the LU updates); oz_report_t.zmode_used tells.
 *           3: the 3-real-product form (batched calls: fixed slice counts up
 *           to 8; tolerance-driven single calls: truncated digits, and 14
 *           with digits = 1): with
 *           op(A) = Ar + i Ai, op(B) = Br + i Bi and the FP64 sums As = Ar + Ai,
 *           Bs = Br + Bi (each rounded once), T1 = Ar Br, T2 = Ai Bi and
 *           T3 = As Bs are three real emulated products, each with its own
 *           per-row / per-column scales and INT32 chunks of kchunk real terms;
 *           then Cr = T1 - T2, Ci = (T3 - T1) - T2 and alpha, beta as for
 *           zmode 4.  Three quarters of the INT8 work; the error is of the same
 *           order (the sums can double the scale of T3).  A row or column
 *           whose sum overflows counts as non-finite.  A tolerance-driven
 *           call picks its start from the complex operands as for zmode 4,
 *           keeps the raw sums of T1, T2 and T3, checks the combined result,
 *           grows each product by its top anti-diagonals (T1, T2, T3 in turn)
 *           and combines the sums into C at the end: bit-identical to three
 *           real tolerance products grown the same way and combined once.
 *  kernel : GEMM kernel shape; 0 = the default (for s <= 6 with one INT32
 *           chunk and at least 512 tiles of 128 x 64, shape 4; else the
 *           64 x 64 block for s <= 8; for 9 <= s <= 14 the same all-diagonal
 *           block at one wave per SIMD, except where its registers would not
 *           hold the chunked sums (several INT32 chunks at s >= 13);
 *           streaming otherwise), 1 = 128 x 64 block of 8 waves with a
 *           3-stage LDS ring, 2 = 64 x 64 block of 4 waves (both for s <= 8),
 *           3 = per-diagonal streaming (any s), 4 = 128 x 64 block of 4
 *           waves owning two 32-row tiles each, 5 = 128 x 128 block of 8 such
 *           waves (4 and 5: s <= 6 with one INT32 chunk, the 64 x 64 block
 *           otherwise).  Batched plans take 0, 1, 2 and 4.  Every shape gives
 *           the same bits.
 *  sstart : tolerance-driven calls only: the starting slice count; 0 lets
 *           `selector` choose it.
 *  selector: tolerance-driven calls with sstart == 0: 0 = the rule of
 *           oz_select_slices, 1 = the learned selector attached to the handle
 *           (oz_set_selector; OZ_ERR_ARG without one), see oz_predict_slices.
 *  digits : 0 = truncated digits (the default, as described above).
 *           1 = balanced, round-to-nearest digits (this library's own
 *           variant: the paper does not say how digits are rounded; rounding
 *           gains about one bit per slice over truncation), fixed slice
 *           counts 1..8, real products and both complex forms, and
 *           tolerance-driven calls (smax capped at 8; the rule's estimate is
 *           divided by 2^(s-1), and the selector's start lowered by one from
 *           7 on; growth splits again at s + 1 and recomputes the sums, since
 *           the digits depend on s), and batched calls with fixed slice counts
 *           (the 4-product form; each problem's s from 1 to 8).  A
 *           double-double call, a tolerance-driven batch, or s > 8 returns
 *           14.  The vector exponent is E' = E, or E + 1 when the
 *           largest magnitude M has M 2^(7-E) > 127; N = |x| 2^(7-E'+8(s-1))
 *           rounded to the nearest integer (ties away from zero) with the
 *           sign of x; digits d_1..d_s with N = sum_p d_p 256^(s-p), all in
 *           [-128, 127] (|d_1| <= 127), so x is 2^(E'+1) sum_p d_p 2^(-8p) to
 *           half a unit of the last digit; the anti-diagonal weights are
 *           2^(2-8d), the result is scaled by 2^(E'_i + F'_j), and kchunk is
 *           bounded by s*kchunk*128^2 <= 2^31-1.  Complex, 4-product form: the
 *           real-part row (ar, -ai) takes the digits of the value -ai;
 *           3-product form: the three real products take balanced digits.
 */
typedef struct {
    int32_t slices;
    int32_t smax;
    int32_t kchunk;
    int32_t zmode;
    int32_t kernel;
    int32_t sstart;
    int32_t selector;
    int32_t digits;
    double tol;
} oz_prec_t;

/* Per-call report, filled when rep != NULL (the call then synchronises). */
typedef struct {
    int32_t status;        /* OZ_OK or OZ_ERR_NONFINITE                      */
    int32_t slices_used;   /* s of the final result                          */
    int32_t fallbacks;     /* slices added after the residual check failed   */
    int32_t kchunks;       /* INT32 chunks along k                           */
    int32_t zmode_used;    /* complex form used (3 or 4), 0 for real         */
    int32_t reserved;
    double resid_est;      /* a-posteriori error estimate (tol mode), else 0 */
} oz_report_t;

/* Create a handle bound to HIP device `device` (made current for the call)
 * with the null stream and a library-owned, grow-only workspace.
 * Returns OZ_ERR_UNSUPPORTED when the device is not gfx950. */
int oz_create(oz_handle_t* handle, int device);

/* Free the handle and its library-owned workspace (waits for its stream). */
int oz_destroy(oz_handle_t handle);

/* Set the stream (a hipStream_t) every later call enqueues on; NULL is the
 * null stream.  The stream stays owned by the caller. */
int oz_set_stream(oz_handle_t handle, void* stream);

/* Text of a status code (static storage). */
const char* oz_status_string(int status);

/* Device workspace bytes oz_dgemm (is_complex = 0) or oz_zgemm (1) needs for
 * these sizes and precision (prec->slices must be nonzero). */
int oz_workspace_size(oz_handle_t handle, char transa, char transb, int64_t m, int64_t n, int64_t k,
                      int is_complex, const oz_prec_t* prec, size_t* bytes);

/* Hand the handle a caller-owned device workspace (NULL releases it and
 * returns to library-owned allocation).  A call whose need exceeds the bytes
 * given returns OZ_ERR_ALLOC. */
int oz_set_workspace(oz_handle_t handle, void* dptr, size_t bytes);

/* C = alpha*op(A)*op(B) + beta*C, FP64, emulated with prec->slices INT8
 * slices (Sec. 2.2 / 3.1).  prec NULL means s = 7.  With beta == 0, C is not
 * read.  Per entry the result is ldexp(acc, E_i + F_j) scaled by alpha,
 * where acc sums, chunk by chunk and then from the highest anti-diagonal
 * d = s+1 down to d = 2, the INT32 sums S_d of the slice-pair products with
 * p + q = d, each times 2^(-7d); the products alpha*v and beta*C are rounded
 * separately and added (no fused multiply-add). */
int oz_dgemm(oz_handle_t handle, char transa, char transb, int64_t m, int64_t n, int64_t k,
             const double* alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
             const double* beta, double* C, int64_t ldc, const oz_prec_t* prec, oz_report_t* rep);

/* Complex version (interleaved real/imaginary FP64 pairs, i.e. the memory
 * layout of double _Complex / hipDoubleComplex).  alpha and beta point at
 * two doubles each (real, imaginary).  One power-of-two scale serves both
 * parts of a row of op(A) / column of op(B): the exponent of its largest real
 * or imaginary part.  Re C and Im C are each a real emulated product over 2k
 * terms (ar*br - ai*bi and ar*bi + ai*br), so the INT8 work is that of four
 * real products.  out = (xr*vr - xi*vi) + (yr*cr - yi*ci) for the real part
 * and (xr*vi + xi*vr) + (yr*ci + yi*cr) for the imaginary part, with
 * alpha = (xr, xi), beta = (yr, yi), each product and sum rounded. */
int oz_zgemm(oz_handle_t handle, char transa, char transb, int64_t m, int64_t n, int64_t k,
             const double* alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
             const double* beta, double* C, int64_t ldc, const oz_prec_t* prec, oz_report_t* rep);

/* Allocation-free variant of oz_dgemm (is_complex = 0) and oz_zgemm
 * (is_complex = 1), for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, semantics, kernels and bits as oz_dgemm /
 * oz_zgemm with the same prec (both complex forms, both digit kinds, any
 * kernel choice), with these differences:
 *  - the workspace is a fixed device array inside the library,
 *    OZ_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, held from the first
 *    oz_create on that GPU until the process ends; the call allocates
 *    nothing (no hipMalloc, no timing events);
 *  - a call whose workspace need (oz_workspace_size) exceeds that size
 *    returns OZ_ERR_ALLOC and enqueues nothing;
 *  - fixed slice counts only: prec->slices == 0 (tolerance mode) returns 14;
 *    prec NULL means s = 7;
 *  - no report;
 *  - every call on one GPU shares the array (the library zeroes what must
 *    start at zero): calls that overlap in time on one GPU -- from several
 *    handles, streams or threads -- race and give undefined results.
 * Argument errors are numbered as in oz_dgemm / oz_zgemm (without the
 * is_complex argument); is_complex other than 0 or 1 returns OZ_ERR_ARG. */
#define OZ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int oz_gemm_noalloc(oz_handle_t handle, int is_complex, char transa, char transb, int64_t m, int64_t n,
                    int64_t k, const double* alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                    const double* beta, double* C, int64_t ldc, const oz_prec_t* prec);

/* Products beyond FP64 (paper Sec. 1: some computations need more than FP64;
 * with s >= 9 the emulated product carries more bits than one double holds).
 * C = op(A) op(B) as a double-double (C_hi + C_lo, both m x n with leading
 * dimension ldc, device memory, distinct buffers; complex: interleaved pairs,
 * real parts and imaginary parts each a double-double).  The digits, pairs and
 * INT32 anti-diagonal sums are those of oz_dgemm with the same prec; the sums
 * are folded in the same order (d = s+1 down to 2, chunk by chunk) but into a
 * double-double: hi + x by TwoSum, its error added to lo, then a fast TwoSum
 * renormalisation.  C_hi = ldexp(hi, E_i + F_j), C_lo = ldexp(lo, E_i + F_j);
 * NaN in both for a row or column with Inf/NaN input (rep->status
 * OZ_ERR_NONFINITE).  alpha = 1 and beta = 0 (C is not read).  Fixed slice
 * counts only (prec->slices 1..18, tolerance mode returns 14); complex uses the
 * 4-product form (zmode 3 returns 14); runs the all-diagonal kernel at one
 * wave per SIMD for s <= 14 (one INT32 chunk, or several up to s = 11) and
 * the per-diagonal streaming kernel otherwise, or when prec->kernel is 3.
 * Returns 12 when C_lo is NULL or equals C_hi;
 * argument errors otherwise as oz_dgemm. */
int oz_dgemm_x2(oz_handle_t handle, char transa, char transb, int64_t m, int64_t n, int64_t k,
                const double* A, int64_t lda, const double* B, int64_t ldb, double* C_hi, double* C_lo,
                int64_t ldc, const oz_prec_t* prec, oz_report_t* rep);
int oz_zgemm_x2(oz_handle_t handle, char transa, char transb, int64_t m, int64_t n, int64_t k,
                const double* A, int64_t lda, const double* B, int64_t ldb, double* C_hi, double* C_lo,
                int64_t ldc, const oz_prec_t* prec, oz_report_t* rep);

/* ---- LU-based complex inversion (the paper's application, Sec. 3.2) --------
 *
 * The application's solver inverts complex matrices through an LU
 * factorisation whose level-3 work is ZGEMM; here every such product is the
 * emulated oz_zgemm at the precision `prec` (NULL: s = 7), on the handle's
 * stream.  The panel factorisation, the row interchanges and the triangular
 * solves run in FP64 kernels of this library.  Complex arithmetic outside the
 * products is written out on the parts: a b = (ar br - ai bi, ar bi + ai br),
 * 1/p = (pr / (pr^2 + pi^2), -pi / (pr^2 + pi^2)), each operation rounded.
 *
 * oz_zgetrf: A = P L U in place (n x n, interleaved complex, column-major,
 * leading dimension lda >= max(1, n), device memory), right-looking in panels
 * of nb columns (nb 0: 128).  For column j the pivot is the first row r >= j
 * with the largest |Re a_rj| + |Im a_rj|; ipiv[j] = r (device int32, n
 * entries, 0-based row numbers; interchanges apply in order j = 0 .. n-1).
 * A panel is factored column by column (swap across the panel, scale the
 * column below the diagonal by the pivot's reciprocal, rank-1 update of the
 * panel columns to its right); its interchanges are then applied to the other
 * columns, U12 = L11^-1 A12 by forward substitution (sums in index order), and
 * A22 = A22 - L21 U12 by oz_zgemm (alpha = -1, beta = 1).  *info (host) = 0,
 * or j + 1 for the first exactly zero pivot (the column is then left unscaled
 * and the factorisation continues).  The next panel is factored on a second,
 * library-created stream while the handle's stream runs the rest of the
 * trailing product (issued as two products split by columns, which changes no
 * entry of a fixed-s product); both streams are drained before the call
 * returns.  Synchronises.  Argument errors: 2 (n < 0),
 * 4 (lda), 6 (nb < 0), 7 (prec), 8 (info NULL), OZ_ERR_ARG (A or ipiv NULL
 * with n > 0); errors of oz_zgemm are passed on.  Inputs with Inf or NaN are
 * not supported (the pivot search skips NaN entries).
 *
 * oz_zgetri: X = A^-1 (n x n, leading dimension ldx, device memory distinct
 * from LU) from the output of oz_zgetrf, by solving A X = I: X = P I, then for
 * block rows of nb (nb 0: 256) from the first, X_i = X_i - L[i, :i] X[:i]
 * (oz_zgemm) followed by X_i = L_ii^-1 X_i, then from the last block row,
 * X_i = X_i - U[i, i+1:] X[i+1:] (oz_zgemm) followed by back substitution
 * with U_ii (each row multiplied by the reciprocal of its diagonal entry).
 * The solves run against I in a library-allocated n x n work matrix and the
 * columns are permuted into X at the end (the same bits, without the
 * structural zeros of L^-1).  ipiv must hold the pivots oz_zgetrf wrote
 * (other values give an unspecified X but no access outside it).
 * Synchronises.  Argument errors: 2 (n), 4 (lda), 7 (ldx), 8 (nb), 9 (prec),
 * OZ_ERR_ARG (a NULL pointer with n > 0, or X == LU). */
int oz_zgetrf(oz_handle_t handle, int64_t n, double* A, int64_t lda, int32_t* ipiv, int32_t nb,
              const oz_prec_t* prec, int32_t* info);
int oz_zgetri(oz_handle_t handle, int64_t n, const double* LU, int64_t lda, const int32_t* ipiv, double* X,
              int64_t ldx, int32_t nb, const oz_prec_t* prec);

/* The starting slice count of a tolerance-driven call: the smallest s in
 * [1, smax] (smax 0: 12) with 2.5 (s+1) 2^(-7s) sqrt((1/M_A + 1/M_B)/3) <= tol,
 * M_A / M_B the mean over rows of op(A) / columns of op(B) of the mean square
 * of x * 2^-E.  Synchronises the handle's stream.  Arguments as oz_dgemm /
 * oz_zgemm (is_complex selects interleaved complex storage). */
int oz_select_slices(oz_handle_t handle, char transa, char transb, int64_t m, int64_t n, int64_t k,
                     int is_complex, const double* A, int64_t lda, const double* B, int64_t ldb,
                     double tol, int32_t smax, int32_t* s_out);

/* ---- Learned slice-count selection ------------------------------------------
 *
 * The paper proposes adjusting the split number to the operator (Sec. 4).
 * The learned selector predicts the starting s of a tolerance-driven call
 * from 16 statistics of the operands and the tolerance, with a small network
 * (16 -> 64 -> 64 -> 1, ReLU, FP32) trained on the GPU against labels that
 * the emulation itself produces.  The residual check and the incremental
 * growth of the tolerance-driven call still guarantee the tolerance; a good
 * start only saves work (a start below the final s costs check rounds, a start
 * above it costs slice pairs).
 *
 * Features of a product op(A) op(B) at tolerance tol (FP32, in this order).
 * For each operand -- rows of op(A), then columns of op(B); a complex operand
 * contributes real and imaginary parts as separate entries under the shared
 * scale -- with E_v the scale exponent of vector v, over its non-zero entries
 * x the gap g = E_v - exponent(x) (frexp convention) and the width
 * w = g + bit length of the odd significand of x (the entry is exact with
 * ceil(w/7) digits), both capped at 127:
 *   zero fraction, mean g, std g, 90th percentile g, mean w, 90th percentile w
 * (percentile: smallest v with at least 90% of the entries at or below v);
 * then log2 of the term count (k, or 2k for complex), log2(m n) / 2,
 * -log10(tol), and log2 sqrt((1/M_A + 1/M_B)/3) with M as in
 * oz_select_slices (0 when an operand is zero). */
#define OZ_NUM_FEATURES 16
#define OZ_MLP_NIN 16
#define OZ_MLP_NHIDDEN 64
#define OZ_MLP_NPARAM 5313

typedef struct oz_mlp_s* oz_mlp_t;

/* One synthetic instance of the selector's training distribution, drawn by a
 * counter-based generator (splitmix64: draw c of the stream with key K is
 * mix64(K + (c+1) * 0x9E3779B97F4A7C15)).  Sub-stream keys are draws 0..3 of
 * `key`: entries of A, entries of B, row exponents of A, column exponents of
 * B.  Entry (i, j) of a rows x cols operand uses draws 5 idx .. 5 idx + 4 of
 * its entry stream, idx = i + j*rows:
 *   family 0: sign = bit 0 and significand = (draw 0 >> 11) | 2^52 of draw 0,
 *             value (-1)^sign * significand * 2^-53, in [1/2, 1);
 *   family 1: u_c = (draw c >> 11) * 2^-53, value ((u0 + u1) + u2) + u3 - 2;
 *   the significand then keeps its top `bits` bits; draw 4 makes the entry
 *   zero when (draw 4 >> 40) < zero_q, else scales it by 2^(e_el + e_vec),
 *   e_el = ((draw 4) mod 2^32) mod (sig_el + 1) - sig_el/2 and e_vec = (draw r
 *   of the row / column exponent stream) mod (sig_vec + 1) - sig_vec/2, r the
 *   row of A or column of B.  Every step is exact or one IEEE addition, so any
 *   implementation reproduces the same operands. */
typedef struct {
    int64_t m, n, k;
    int32_t sig_el;   /* exponent spread per entry, >= 0       */
    int32_t sig_vec;  /* exponent spread per row / column, >= 0 */
    int32_t bits;     /* significand bits kept, 1..53          */
    int32_t family;   /* 0 or 1                                */
    int64_t zero_q;   /* zero threshold, 0..2^24               */
    uint64_t key;
} oz_gen_t;

/* A (m x k, lda >= m) and B (k x n, ldb >= k), column-major device arrays,
 * of instance p.  Asynchronous on the handle's stream. */
int oz_gen_operands(oz_handle_t handle, const oz_gen_t* p, double* A, int64_t lda, double* B, int64_t ldb);

/* Feature rows of op(A) op(B) for ntol tolerances (host array tols): feat is
 * a device array of ntol x OZ_NUM_FEATURES floats (row-major); s_rule (host,
 * ntol entries, may be NULL) receives oz_select_slices' choice per tolerance
 * with smax (0: 12).  Operand arguments as oz_dgemm / oz_zgemm.
 * Synchronises the handle's stream. */
int oz_features(oz_handle_t handle, char transa, char transb, int64_t m, int64_t n, int64_t k, int is_complex,
                const double* A, int64_t lda, const double* B, int64_t ldb, int32_t ntol, const double* tols,
                int32_t smax, float* feat, int32_t* s_rule);

/* Training / test data of the selector, generated and labelled on the GPU.
 * For each instance b (params[b], real operands, k <= 11072 so that the
 * reference emulation needs one INT32 chunk) the library draws the operands,
 * runs the s_ref emulation (2 <= s_ref <= 18) keeping its INT32 anti-diagonal
 * sums, and from them forms every C_s, s < s_ref, exactly as the fixed-s
 * emulation would (one chunk: sum from d = s+1 down to 2 of S_d 2^-7d), and
 *   eps_s = || W o (C_s - C_ref) ||_F / || W o C_ref ||_F,
 *   W_ij = 1 / (max|A_i:| max|B_:j|).
 * Row r = b*ntol + t of the output is the feature row of instance b at
 * tolerance tols[r] (host array), with label y[r] = the smallest s in
 * [2, s_ref] with eps_s <= tol.  X (device, rows x OZ_NUM_FEATURES floats)
 * and y (device, rows floats) receive the data; s_rule (host, rows entries)
 * the rule's choice with smax_rule; eps (host, count x s_ref doubles) the
 * table eps_1 .. eps_s_ref (eps_s_ref = 0).  s_rule and eps may be NULL.
 * Synchronises the handle's stream. */
int oz_selector_dataset(oz_handle_t handle, int32_t count, const oz_gen_t* params, int32_t ntol,
                        const double* tols, int32_t s_ref, int32_t smax_rule, float* X, float* y,
                        int32_t* s_rule, double* eps);

/* The network.  Parameters (OZ_MLP_NPARAM floats, host order): W1[64][16]
 * (row = hidden unit), b1[64], W2[64][64], b2[64], W3[64], b3; inputs are
 * normalised as (x - mu) / sd per feature before the first layer.
 *   y = W3 . relu(W2 relu(W1 xn + b1) + b2) + b3.
 * Loss of a batch of B rows with targets t: (1/B) sum rho(t - y) with
 * rho(r) = tau r for r > 0, (tau - 1) r otherwise (pinball loss; tau near 1
 * penalises predictions below the target, which cost extra check rounds, more
 * than those above).  Optimiser: Adam, beta1 0.9, beta2 0.999, eps 1e-8. */
/* New network: He-uniform weights drawn from the splitmix64 stream of seed,
 * zero biases, mu = 0, sd = 1.  Bound to the handle's device and stream. */
int oz_mlp_create(oz_handle_t handle, uint64_t seed, oz_mlp_t* mlp);
int oz_mlp_destroy(oz_mlp_t mlp);
/* Host copies in and out (any pointer may be NULL).  Setting the parameters
 * restarts Adam.  Both synchronise the handle's stream. */
int oz_mlp_set_params(oz_mlp_t mlp, const float* params, const float* mu, const float* sd);
int oz_mlp_get_params(oz_mlp_t mlp, float* params, float* mu, float* sd);
/* mu, sd = per-feature mean and standard deviation of the rows of X (device,
 * rows x 16; a deviation below 1e-6 is taken as 1). */
int oz_mlp_fit_norm(oz_mlp_t mlp, int64_t rows, const float* X);
/* y (device, rows) = network(X (device, rows x 16)).  Asynchronous. */
int oz_mlp_forward(oz_mlp_t mlp, int64_t rows, const float* X, float* y);
/* Gradient of the batch loss with respect to the parameters (host,
 * OZ_MLP_NPARAM floats, may be NULL) and the loss (host, may be NULL), for
 * device rows X and targets t.  Synchronous. */
int oz_mlp_grad(oz_mlp_t mlp, int64_t rows, const float* X, const float* t, float tau, float* grad, float* loss);
/* One Adam step on one batch; loss (host, may be NULL) is the batch loss
 * before the step (then the call synchronises). */
int oz_mlp_train_step(oz_mlp_t mlp, int64_t rows, const float* X, const float* t, float tau, float lr,
                      float* loss);
/* epochs passes over the rows in batches of `batch`, each pass in an order
 * shuffled by the splitmix64 stream of seed; an untrained network first sets
 * b3 to the mean target.  epoch_loss (host, epochs entries, may be NULL)
 * receives the mean loss of each pass.  Synchronous. */
int oz_mlp_train(oz_mlp_t mlp, int64_t rows, const float* X, const float* t, int32_t epochs, int32_t batch,
                 float tau, float lr, uint64_t seed, float* epoch_loss);
/* Binary file: 8-byte magic "OZMLP001", int32 16, 64, 5313, then the 5313
 * parameters, mu[16] and sd[16] as little-endian floats. */
int oz_mlp_save(oz_mlp_t mlp, const char* path);
int oz_mlp_load(oz_handle_t handle, const char* path, oz_mlp_t* mlp);

/* Attach a network as the handle's learned selector (NULL detaches).  The
 * network is not copied and must outlive its use. */
int oz_set_selector(oz_handle_t handle, oz_mlp_t mlp);

/* The learned starting slice count: s = clamp(floor(y + 1/2), 2, smax)
 * (smax 0: 12) for the network output y on the features of the product at
 * tol (y estimates an upper quantile of the smallest passing s).  Operand
 * arguments as oz_select_slices.  Synchronises the handle's stream. */
int oz_predict_slices(oz_handle_t handle, char transa, char transb, int64_t m, int64_t n, int64_t k,
                      int is_complex, const double* A, int64_t lda, const double* B, int64_t ldb, double tol,
                      int32_t smax, int32_t* s_out);

/* ---- Measured peaks -------------------------------------------------------
 *
 * Rates of this GPU that roofline reports divide by, measured by the
 * library's own microbenchmarks on the handle's stream (synchronises):
 *  kind 0: INT8 matrix cores, back-to-back v_mfma_i32_32x32x32_i8 on every
 *          SIMD, iters instructions per accumulator chain -> ops per second;
 *  kind 1: FP64 matrix cores, v_mfma_f64_16x16x4_f64 -> flops per second;
 *  kind 2: device copy of `bytes` (a multiple of 16) from src to dst (device
 *          buffers of the caller), iters repetitions -> bytes read plus bytes
 *          written per second;
 *  kind 3: INT8 matrix cores in the 16 x 16 x 64 shape,
 *          v_mfma_i32_16x16x64_i8 -> ops per second;
 *  kind 4: as kind 0 with two pairs of full-range pseudo-random operand
 *          bytes used by alternate instructions (consecutive MFMAs see
 *          different data, as in a GEMM over random digits; kind 0 feeds
 *          the same small bytes to every instruction) -> ops per second.
 * src, dst and bytes are ignored for kinds 0, 1, 3 and 4.  OZ_ERR_ARG for a bad
 * kind, iters < 1, a NULL rate, or a bad copy buffer. */
int oz_peak(oz_handle_t handle, int kind, int64_t iters, const void* src, void* dst, size_t bytes, double* rate);

/* ---- Batched products ----------------------------------------------------
 *
 * Many independent products of uneven sizes (real: is_complex = 0, complex:
 * 1).  All array arguments are host arrays of `batch` entries (alpha and beta:
 * one double per problem, or two -- real, imaginary -- for complex); A[b],
 * B[b], C[b] are device pointers.  Each problem follows the oz_dgemm /
 * oz_zgemm semantics with its own slice count: slices[b] if the array is given,
 * else prec->slices (1..8; prec NULL: 7), and prec->digits = 1 gives every
 * problem balanced digits.  Errors are reported for the first
 * problem that has one, at the reference-BLAS argument position.
 *
 * A plan computes the layouts, carves one device allocation (owned by the
 * plan) for every problem's scales, slices and the work lists, and uploads the
 * descriptors.  Executing it enqueues a fixed sequence on the handle's stream:
 * one launch clearing the scale scratch, one batched exponent scan, one
 * batched digit split, and persistent GEMM launches whose blocks walk a tile
 * list ordered by work: one for every problem with s <= 8 (each tile at its
 * problem's s), one for those with 9 <= s <= 14 on a second stream beside it.
 * With zmode 3 (complex, s <= 8) the scan and split write the three real
 * parts of each operand, and one block computes the three real products of
 * a tile in turn (T1 and T2 held in registers) and combines them: one launch
 * for s <= 6, one on the second stream for s = 7, 8.  Tiles that cover only
 * padding are never computed.  No host synchronisation and no allocation happen in
 * an execution, so it can be captured: oz_batch_graph_launch captures it into
 * a HIP graph on its first call (the handle's stream must not be the null
 * stream) and replays the graph afterwards.  The operand and output buffers
 * must stay valid while the plan is used. */
typedef struct oz_batch_s* oz_batch_t;

int oz_gemm_batched_plan(oz_handle_t handle, int is_complex, int32_t batch, const char* transa,
                         const char* transb, const int64_t* m, const int64_t* n, const int64_t* k,
                         const double* alpha, const double* const* A, const int64_t* lda,
                         const double* const* B, const int64_t* ldb, const double* beta, double* const* C,
                         const int64_t* ldc, const oz_prec_t* prec, const int32_t* slices, const double* tols,
                         oz_batch_t* plan);
int oz_batch_execute(oz_batch_t plan);
/* Replay the captured execution (fixed slice counts only; a tolerance-driven
 * plan returns OZ_ERR_ARG). */
int oz_batch_graph_launch(oz_batch_t plan);
int oz_batch_destroy(oz_batch_t plan);
/* Tolerance-driven batches: prec->slices == 0 with prec->tol > 0 (slices
 * array NULL) plans every problem as a tolerance-driven oz_dgemm / oz_zgemm
 * call with its own tolerance -- tols[b] (every entry > 0) when the array is
 * given, else prec->tol -- and the same smax (0: 12, up to OZ_MAX_SLICES),
 * sstart and selector; tols given with a fixed slice count returns 14.  An
 * execution then runs: the batched scan; the starting s of every problem
 * (sstart, or one batched statistics pass and the rule or the handle's
 * learned selector); the split of digit planes 1..s; raw sums at those s
 * (every problem with s <= 8 in one mixed-s persistent launch, those with
 * 9 <= s <= 14 in wide launches on a second stream beside it, streaming
 * launches above); then rounds of a batched residual check over the problems
 * still open, and for those whose estimate exceeds tol/2 the slices the
 * single call would add (new digit planes, then one anti-diagonal at a time,
 * each added last), until all pass or reach smax; finally one batched
 * scaling pass into C for the problems with beta != 0 (with beta = 0 every
 * GEMM pass writes C).  Each problem's result is bit-identical to the single
 * tolerance-driven call that starts and ends at the same s.  The execution
 * synchronises the stream at every round. */
/* Per-problem reports of the last execution (batch entries): slices used,
 * slices added by the check, INT32 chunks, the final error estimate (tol
 * plans), status OZ_ERR_NONFINITE for non-finite input.  Synchronises. */
int oz_batch_report(oz_batch_t plan, oz_report_t* reps);
/* Plan facts: GEMM launches, tiles, device bytes held, slices per problem
 * (array of batch entries; any pointer may be NULL).  For a tolerance-driven
 * plan the launch and tile counts are those of a fixed plan (0) and the slices
 * are the final ones of the last execution. */
int oz_batch_info(oz_batch_t plan, int32_t* launches, int64_t* tiles, size_t* device_bytes, int32_t* slices);

/* Load the batched-plan tuning table written by the package's autotuner
 * (JSON: an "entries" array of {"complex", "n", "s", "tile", "order", ...}).
 * Later plans take, per slice-count group, the block shape and tile order of
 * the entry nearest (in log n) to each problem, weighted by its work; without
 * a table, or with prec->kernel set, a size rule decides.  NULL clears it. */
int oz_load_tuning(oz_handle_t handle, const char* path);

/* One-shot batched calls: plan, execute, destroy. */
int oz_zgemm_batched(oz_handle_t handle, int32_t batch, const char* transa, const char* transb,
                     const int64_t* m, const int64_t* n, const int64_t* k, const double* alpha,
                     const double* const* A, const int64_t* lda, const double* const* B, const int64_t* ldb,
                     const double* beta, double* const* C, const int64_t* ldc, const oz_prec_t* prec,
                     const int32_t* slices);
int oz_dgemm_batched(oz_handle_t handle, int32_t batch, const char* transa, const char* transb,
                     const int64_t* m, const int64_t* n, const int64_t* k, const double* alpha,
                     const double* const* A, const int64_t* lda, const double* const* B, const int64_t* ldb,
                     const double* beta, double* const* C, const int64_t* ldc, const oz_prec_t* prec,
                     const int32_t* slices);

/* Profiling aid.  While enabled, every oz_dgemm / oz_zgemm call records HIP
 * events on the handle's stream before its split kernels, between the split
 * kernels and the GEMM kernel, and after the GEMM kernel.  oz_timing_read
 * waits for the stream, returns the summed milliseconds of the split phase
 * and of the GEMM kernel and the number of timed calls since the previous
 * read, and starts a new count.  Any output pointer may be NULL. */
int oz_timing_enable(oz_handle_t handle, int enable);
int oz_timing_read(oz_handle_t handle, double* split_ms, double* gemm_ms, int64_t* calls);

/* ---- The steps of the method, exposed for verification ------------------
 *
 * Slice layout (the library's own, shared by its kernels):
 *   An operand is a set of vectors: the rows of op(A) (side 'A') or the
 *   columns of op(B) (side 'B').  A real operand has nv vectors of K' = k
 *   terms.  A complex side-'B' operand has nv vectors of K' = 2k terms, term
 *   2l holding the real and 2l+1 the imaginary part of element l.  A complex
 *   side-'A' operand has 2*ceil(nv/16)*16 vectors of K' = 2k terms: complex
 *   row c maps to vector r = 32*(c/16) + 16*((c/8)%2) + (c%8) for the
 *   real-part row (terms: ar, -ai) and r + 8 for the imaginary-part row
 *   (terms: ai, ar).  Vectors are padded with zeros to rows_pad (a multiple
 *   of 128) and terms to kpad (a multiple of 32).
 *   Digit p (1..s) of term t of vector v is the int8 at byte offset
 *     (((t/16)*s + (p-1)) * rows_pad + v) * 16 + t%16.
 *   The scale exponent of vector v (per complex row c for a complex side 'A')
 *   is the int32 E[v]; INT32_MIN marks a vector that holds Inf or NaN.
 */

/* Sizes of the slice layout above. */
int oz_split_layout(char side, int is_complex, int64_t nv, int64_t k, int32_t slices,
                    int64_t* rows_pad, int64_t* kpad, size_t* slice_bytes);

/* Step 1-2 of the method for one operand: scale exponents and INT8 digits.
 * X is the device operand (real or interleaved complex doubles) with leading
 * dimension ldx; vectors are taken from op(X) as described above (side 'A':
 * op(X) is nv x k; side 'B': op(X) is k x nv).  E (device int32, nv entries)
 * and slices (device, slice_bytes of oz_split_layout) receive the result. */
int oz_split(oz_handle_t handle, char side, char trans, int is_complex, int64_t nv, int64_t k,
             const double* X, int64_t ldx, int32_t slices, int32_t* E, int8_t* slices_out);

/* Step 3: the exact anti-diagonal sums S_{d,c} = sum over p + q = d of the
 * INT32 slice-pair products over chunk c of kchunk terms, from two slice
 * buffers laid out by oz_split (A: rows_pad_a vectors, B: rows_pad_b vectors,
 * same kpad), computed by the GEMM kernel `kernel` (as in oz_prec_t).
 * out (device int32) receives
 *   out[((c*s + (d-2)) * rows_pad_b + j) * rows_pad_a + i]
 * for every chunk c < ceil(kpad/kchunk), d = 2..s+1, and all padded i, j. */
int oz_diag_sums(oz_handle_t handle, int32_t slices, int64_t kchunk, int32_t kernel, int64_t rows_pad_a,
                 int64_t rows_pad_b, int64_t kpad, const int8_t* slices_a, const int8_t* slices_b,
                 int32_t* out);

#ifdef __cplusplus
}
#endif
#endif /* OZ_H */
