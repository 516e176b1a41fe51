/* oz_blas.h -- Fortran-ABI level-3 BLAS entry points that run dgemm/zgemm
 * on one MI355X through the emulated path of oz.h (liboz_blas.so).
 *
 * The paper runs an unmodified CPU program on the GPU's integer units by
 * intercepting its level-3 BLAS calls (Sec. 2.1) and choosing the arithmetic
 * per run through an environment variable that names either native FP64 or
 * INT8 emulation with a given split number (Sec. 3.1).  This library is that
 * offload layer for a discrete GPU: a program linked against it (ahead of its
 * CPU BLAS) gets dgemm_ and zgemm_ from here.  The paper's Grace-Hopper setup
 * shares memory between CPU and GPU; here every host operand is copied over
 * PCIe for each call, and operands that already live in device memory are
 * used in place (checked per pointer).
 *
 * Mode (environment variable OZ_COMPUTE_MODE, read at the first call, or
 * oz_blas_set_mode):
 *   "fp64_int8_<s>"        emulation with s slices, 1 <= s <= 18 (default s = 7);
 *   "fp64_int8_tol<tol>"   tolerance-driven emulation (oz_prec_t.tol = tol,
 *                          smax 12), e.g. "fp64_int8_tol1e-12";
 *   "fp64_int8_bal<s>"     emulation with s balanced (round-to-nearest) digits,
 *                          1 <= s <= 8 (oz_prec_t.digits = 1), e.g.
 *                          "fp64_int8_bal6";
 *   "dgemm"                native FP64 on the GPU (rocBLAS), for comparison.
 * OZ_ZMODE = 0, 3 or 4 selects the complex form of zgemm_ in the emulated
 * modes (default 0: the library's choice by size, oz_prec_t.zmode); OZ_DEVICE
 * selects the GPU (default 0).
 *
 * Error behaviour: an illegal argument is reported as the reference BLAS does
 * (a message naming the routine and the 1-based parameter number, written to
 * stderr), C is left untouched and oz_blas_stats().last_info holds that
 * number.  A failure of the GPU runtime or of the emulation library (no
 * device, out of memory, a kernel error) is reported on stderr and aborts the
 * process: there is no CPU fallback.
 *
 * Threads: calls are serialised by one lock; each call is synchronous (C holds
 * the result when it returns).  Not re-entrant from inside a HIP callback.
 */
#ifndef OZ_BLAS_H
#define OZ_BLAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C <- alpha * op(A) * op(B) + beta * C, column-major, Fortran calling
 * convention (every argument by reference; 32-bit integers; trailing hidden
 * string lengths, if a Fortran caller passes them, are ignored).
 * transa, transb: 'N', 'T' or 'C' (either case); m, n, k >= 0;
 * lda >= max(1, rows of the stored A), likewise ldb, ldc >= max(1, m).
 * Pointers may be host or device memory; host arrays are read (A, B, and C
 * when beta != 0) and C is written back before the call returns. */
void dgemm_(const char* transa, const char* transb, const int32_t* m, const int32_t* n, const int32_t* k,
            const double* alpha, const double* A, const int32_t* lda, const double* B, const int32_t* ldb,
            const double* beta, double* C, const int32_t* ldc);

/* The complex*16 form: alpha, beta, A, B and C hold interleaved (re, im)
 * double pairs; 'C' takes the conjugate transpose. */
void zgemm_(const char* transa, const char* transb, const int32_t* m, const int32_t* n, const int32_t* k,
            const double* alpha, const double* A, const int32_t* lda, const double* B, const int32_t* ldb,
            const double* beta, double* C, const int32_t* ldc);

/* Select the mode (syntax as OZ_COMPUTE_MODE).  Returns 0, or -1 when the
 * string is not a mode (the mode is then unchanged). */
int oz_blas_set_mode(const char* mode);

/* Counters since the first call (or the last oz_blas_finalize). */
typedef struct {
    int64_t calls;           /* dgemm_ + zgemm_ calls that ran */
    int64_t bytes_to_device; /* host operand bytes copied in */
    int64_t bytes_to_host;   /* result bytes copied out */
    double copy_ms;          /* time in host<->device copies (HIP events) */
    double compute_ms;       /* time in the emulated (or native) product */
    int32_t last_info;       /* 0, or the illegal parameter of the last call */
    int32_t last_slices;     /* slice count used by the last emulated call */
    int32_t mode;            /* 0 = native FP64, 1 = fixed s, 2 = tolerance-driven,
                                3 = fixed s with balanced digits */
    int32_t slices;          /* fixed s of modes 1 and 3 */
    double tol;              /* tolerance of mode 2 */
} oz_blas_stats_t;

void oz_blas_stats(oz_blas_stats_t* out);

/* Release the device buffers and handles (the next call sets them up again)
 * and reset the counters. */
void oz_blas_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* OZ_BLAS_H */
