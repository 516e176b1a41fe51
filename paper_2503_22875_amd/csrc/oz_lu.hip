// oz_lu.hip -- LU-based complex inversion with emulated trailing products
// (the paper's application: an LU-based matrix inverse rich in ZGEMM, with
// every ZGEMM emulated at the chosen split number, Sec. 3.2 and Table 1).
//
// Right-looking blocked LU with partial pivoting; each panel of nb columns is
// factored by one block (pivot = first row of largest |re| + |im|, row swap
// across the panel, scaling by the pivot's reciprocal, rank-1 updates), the
// interchanges are applied to the other columns, U12 = L11^-1 A12 by forward
// substitution, and A22 -= L21 U12 runs as an emulated ZGEMM (oz_zgemm with
// alpha = -1, beta = 1).  The inverse solves A X = I: X = P I, then block by
// block X_i -= L[i, :i] X[:i] (emulated) and X_i = L_ii^-1 X_i, then from the
// last block X_i -= U[i, i+1:] X[i+1:] (emulated) and X_i = U_ii^-1 X_i.
// Complex arithmetic is written out on the parts, (ar br - ai bi, ar bi + ai br),
// with no fused multiply-add (the library is built with -ffp-contract=off).
#include <hip/hip_runtime.h>

#include "oz_handle.h"

namespace {

constexpr int kPanelThreads = 1024;

__device__ __forceinline__ double* at(double* X, int64_t ld, int64_t r, int64_t c) { return X + 2 * (r + c * ld); }
__device__ __forceinline__ const double* at(const double* X, int64_t ld, int64_t r, int64_t c) {
    return X + 2 * (r + c * ld);
}

// One panel (columns j0 .. j0 + b - 1, rows j0 .. n - 1), one block.
__global__ __launch_bounds__(kPanelThreads) void panel_kernel(double* A, int64_t lda, int64_t n, int64_t j0, int b,
                                                              int32_t* ipiv, int32_t* info) {
    __shared__ double red_v[kPanelThreads];
    __shared__ int64_t red_i[kPanelThreads];
    __shared__ double s_rr, s_ri;
    __shared__ int s_zero;
    const int tid = threadIdx.x;
    for (int c = 0; c < b; ++c) {
        const int64_t j = j0 + c;
        // pivot: largest |re| + |im| at or below the diagonal, first row on ties
        double best = -1.0;
        int64_t bi = j;
        for (int64_t r = j + tid; r < n; r += kPanelThreads) {
            const double* e = at(A, lda, r, j);
            const double v = fabs(e[0]) + fabs(e[1]);
            if (v > best) {
                best = v;
                bi = r;
            }
        }
        red_v[tid] = best;
        red_i[tid] = bi;
        __syncthreads();
        for (int off = kPanelThreads / 2; off > 0; off >>= 1) {
            if (tid < off) {
                const double v = red_v[tid + off];
                const int64_t i = red_i[tid + off];
                if (v > red_v[tid] || (v == red_v[tid] && i < red_i[tid])) {
                    red_v[tid] = v;
                    red_i[tid] = i;
                }
            }
            __syncthreads();
        }
        const int64_t p = red_i[0];
        if (tid == 0) ipiv[j] = static_cast<int32_t>(p);
        // swap rows j and p across the panel
        for (int c2 = tid; p != j && c2 < b; c2 += kPanelThreads) {
            double* x = at(A, lda, j, j0 + c2);
            double* y = at(A, lda, p, j0 + c2);
            const double t0 = x[0], t1 = x[1];
            x[0] = y[0];
            x[1] = y[1];
            y[0] = t0;
            y[1] = t1;
        }
        __syncthreads();
        if (tid == 0) {
            const double* d = at(A, lda, j, j);
            const double pr = d[0], pi = d[1];
            s_zero = (pr == 0.0 && pi == 0.0) ? 1 : 0;
            if (s_zero) {
                if (*info == 0) *info = static_cast<int32_t>(j + 1);
            } else {
                const double q = pr * pr + pi * pi;
                s_rr = pr / q;
                s_ri = -pi / q;
            }
        }
        __syncthreads();
        // l_rj = a_rj * (1 / pivot)
        if (!s_zero) {
            const double rr = s_rr, ri = s_ri;
            for (int64_t r = j + 1 + tid; r < n; r += kPanelThreads) {
                double* e = at(A, lda, r, j);
                const double ar = e[0], ai = e[1];
                e[0] = ar * rr - ai * ri;
                e[1] = ar * ri + ai * rr;
            }
        }
        __syncthreads();
        // rank-1 update of the panel columns right of j
        for (int64_t r = j + 1 + tid; r < n; r += kPanelThreads) {
            const double* l = at(A, lda, r, j);
            const double lr = l[0], li = l[1];
            for (int64_t k = j + 1; k < j0 + b; ++k) {
                const double* u = at(A, lda, j, k);
                const double ur = u[0], ui = u[1];
                const double tr = lr * ur - li * ui, ti = lr * ui + li * ur;
                double* e = at(A, lda, r, k);
                e[0] = e[0] - tr;
                e[1] = e[1] - ti;
            }
        }
        __syncthreads();
    }
}

// Row interchanges j = r0 .. r1 - 1 (in order) on the columns c0 .. c1 - 1.
__global__ void laswp_kernel(double* X, int64_t ld, int64_t c0, int64_t c1, int64_t r0, int64_t r1,
                             const int32_t* ipiv) {
    const int64_t c = c0 + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    for (int64_t j = r0; j < r1; ++j) {
        const int64_t p = ipiv[j];
        if (p == j) continue;
        double* x = at(X, ld, j, c);
        double* y = at(X, ld, p, c);
        const double t0 = x[0], t1 = x[1];
        x[0] = y[0];
        x[1] = y[1];
        y[0] = t0;
        y[1] = t1;
    }
}

// Where the one of column c of P I lands: the interchanges j = 0 .. n - 1 in
// order move it from row c (one block; the pivots staged through LDS).
__global__ __launch_bounds__(1024) void perm_pos_kernel(const int32_t* ipiv, int64_t n, int32_t* pos) {
    __shared__ int32_t sp[1024];
    for (int64_t c0 = 0; c0 < n; c0 += 1024) {
        const int64_t c = c0 + threadIdx.x;
        int64_t at_row = c;
        for (int64_t j0 = 0; j0 < n; j0 += 1024) {
            __syncthreads();
            if (j0 + threadIdx.x < n) sp[threadIdx.x] = ipiv[j0 + threadIdx.x];
            __syncthreads();
            const int64_t jn = n - j0 < 1024 ? n - j0 : 1024;
            for (int64_t t = 0; t < jn; ++t) {
                const int64_t j = j0 + t, p = sp[t];
                if (at_row == j)
                    at_row = p;
                else if (at_row == p)
                    at_row = j;
            }
        }
        if (c < n) pos[c] = static_cast<int32_t>(at_row);
    }
}

// X = P I from the landing rows: X[r, c] = 1 where r = pos[c], else 0.
__global__ void perm_fill_kernel(double* X, int64_t ld, int64_t n, const int32_t* pos) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int64_t c = blockIdx.y; c < n; c += gridDim.y) {
        double* e = at(X, ld, r, c);
        e[0] = r == pos[c] ? 1.0 : 0.0;
        e[1] = 0.0;
    }
}

// B <- L^-1 B, L unit lower b x b (at L, leading dimension ldl), B b x ncols:
// one column per thread, rows in order, sums in index order.
__global__ void trsm_lower_unit_kernel(const double* L, int64_t ldl, int b, double* B, int64_t ldb, int64_t ncols) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    for (int i = 0; i < b; ++i) {
        double* bi = at(B, ldb, i, c);
        double accr = bi[0], acci = bi[1];
        for (int k = 0; k < i; ++k) {
            const double* l = at(L, ldl, i, k);
            const double* x = at(B, ldb, k, c);
            const double lr = l[0], li = l[1], xr = x[0], xi = x[1];
            const double tr = lr * xr - li * xi, ti = lr * xi + li * xr;
            accr = accr - tr;
            acci = acci - ti;
        }
        bi[0] = accr;
        bi[1] = acci;
    }
}

// B <- U^-1 B, U upper b x b: rows from the last, sums in index order, each row
// multiplied by the reciprocal (ur - i ui) / (ur^2 + ui^2) of its diagonal.
__global__ void trsm_upper_kernel(const double* U, int64_t ldu, int b, double* B, int64_t ldb, int64_t ncols) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    for (int i = b - 1; i >= 0; --i) {
        double* bi = at(B, ldb, i, c);
        double accr = bi[0], acci = bi[1];
        for (int k = i + 1; k < b; ++k) {
            const double* u = at(U, ldu, i, k);
            const double* x = at(B, ldb, k, c);
            const double ur = u[0], ui = u[1], xr = x[0], xi = x[1];
            const double tr = ur * xr - ui * xi, ti = ur * xi + ui * xr;
            accr = accr - tr;
            acci = acci - ti;
        }
        const double* d = at(U, ldu, i, i);
        const double pr = d[0], pi = d[1];
        const double q = pr * pr + pi * pi;
        const double rr = pr / q, ri = -pi / q;
        bi[0] = accr * rr - acci * ri;
        bi[1] = accr * ri + acci * rr;
    }
}

hipError_t launch_laswp(double* X, int64_t ld, int64_t c0, int64_t c1, int64_t r0, int64_t r1, const int32_t* ipiv,
                        hipStream_t st) {
    if (c1 <= c0 || r1 <= r0) return hipSuccess;
    hipLaunchKernelGGL(laswp_kernel, dim3(static_cast<unsigned>((c1 - c0 + 255) / 256)), dim3(256), 0, st, X, ld, c0,
                       c1, r0, r1, ipiv);
    return hipGetLastError();
}

hipError_t launch_trsm(bool upper, const double* T, int64_t ldt, int b, double* B, int64_t ldb, int64_t ncols,
                       hipStream_t st) {
    if (ncols <= 0 || b <= 0) return hipSuccess;
    dim3 grid(static_cast<unsigned>((ncols + 63) / 64));
    if (upper)
        hipLaunchKernelGGL(trsm_upper_kernel, grid, dim3(64), 0, st, T, ldt, b, B, ldb, ncols);
    else
        hipLaunchKernelGGL(trsm_lower_unit_kernel, grid, dim3(64), 0, st, T, ldt, b, B, ldb, ncols);
    return hipGetLastError();
}

bool prec_ok(const oz_prec_t* p) { return p == nullptr || p->slices > 0 || p->tol > 0.0; }

}  // namespace

extern "C" {

int oz_zgetrf(oz_handle_t h, int64_t n, double* A, int64_t lda, int32_t* ipiv, int32_t nb, const oz_prec_t* prec,
              int32_t* info) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (n < 0) return 2;
    if (lda < (n > 1 ? n : 1)) return 4;
    if (nb < 0) return 6;
    if (!prec_ok(prec)) return 7;
    if (!info) return 8;
    *info = 0;
    if (n == 0) return OZ_OK;
    if (!A || !ipiv) return OZ_ERR_ARG;
    if (nb == 0) nb = 64;
    int st = oz_handle_use_device(h);
    if (st) return st;
    hipStream_t s = oz_handle_stream(h);
    int32_t* dinfo = nullptr;
    if (hipMalloc(&dinfo, sizeof(int32_t)) != hipSuccess) return OZ_ERR_HIP;
    int rc = OZ_OK;
    if (hipMemsetAsync(dinfo, 0, sizeof(int32_t), s) != hipSuccess) rc = OZ_ERR_HIP;
    const double minus_one[2] = {-1.0, 0.0}, one[2] = {1.0, 0.0};
    for (int64_t j0 = 0; rc == OZ_OK && j0 < n; j0 += nb) {
        const int b = static_cast<int>(n - j0 < nb ? n - j0 : nb);
        hipLaunchKernelGGL(panel_kernel, dim3(1), dim3(kPanelThreads), 0, s, A, lda, n, j0, b, ipiv, dinfo);
        if (hipGetLastError() != hipSuccess || launch_laswp(A, lda, 0, j0, j0, j0 + b, ipiv, s) != hipSuccess) {
            rc = OZ_ERR_HIP;
            break;
        }
        const int64_t rest = n - j0 - b;
        if (rest <= 0) break;
        double* A12 = A + 2 * (j0 + (j0 + b) * lda);
        if (launch_laswp(A, lda, j0 + b, n, j0, j0 + b, ipiv, s) != hipSuccess ||
            launch_trsm(false, A + 2 * (j0 + j0 * lda), lda, b, A12, lda, rest, s) != hipSuccess) {
            rc = OZ_ERR_HIP;
            break;
        }
        rc = oz_zgemm(h, 'N', 'N', rest, rest, b, minus_one, A + 2 * ((j0 + b) + j0 * lda), lda, A12, lda, one,
                      A + 2 * ((j0 + b) + (j0 + b) * lda), lda, prec, nullptr);
    }
    if (rc == OZ_OK && (hipMemcpyAsync(info, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
        rc = OZ_ERR_HIP;
    hipStreamSynchronize(s);
    hipFree(dinfo);
    return rc;
}

int oz_zgetri(oz_handle_t h, int64_t n, const double* LU, int64_t lda, const int32_t* ipiv, double* X, int64_t ldx,
              int32_t nb, const oz_prec_t* prec) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (n < 0) return 2;
    if (lda < (n > 1 ? n : 1)) return 4;
    if (ldx < (n > 1 ? n : 1)) return 7;
    if (nb < 0) return 8;
    if (!prec_ok(prec)) return 9;
    if (n == 0) return OZ_OK;
    if (!LU || !ipiv || !X || X == LU) return OZ_ERR_ARG;
    if (nb == 0) nb = 64;
    int st = oz_handle_use_device(h);
    if (st) return st;
    hipStream_t s = oz_handle_stream(h);
    const double minus_one[2] = {-1.0, 0.0}, one[2] = {1.0, 0.0};
    int32_t* pos = nullptr;
    if (hipMalloc(&pos, sizeof(int32_t) * n) != hipSuccess) return OZ_ERR_HIP;
    dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n < 65535 ? n : 65535));
    hipLaunchKernelGGL(perm_pos_kernel, dim3(1), dim3(1024), 0, s, ipiv, n, pos);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(perm_fill_kernel, grid, dim3(256), 0, s, X, ldx, n, pos);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(pos);
    if (e != hipSuccess) return OZ_ERR_HIP;
    // forward: L Y = P I
    for (int64_t j0 = 0; j0 < n; j0 += nb) {
        const int b = static_cast<int>(n - j0 < nb ? n - j0 : nb);
        if (j0 > 0) {
            const int rc = oz_zgemm(h, 'N', 'N', b, n, j0, minus_one, LU + 2 * j0, lda, X, ldx, one, X + 2 * j0, ldx,
                                    prec, nullptr);
            if (rc) return rc;
        }
        if (launch_trsm(false, LU + 2 * (j0 + j0 * lda), lda, b, X + 2 * j0, ldx, n, s) != hipSuccess)
            return OZ_ERR_HIP;
    }
    // backward: U X = Y
    const int64_t last = ((n - 1) / nb) * nb;
    for (int64_t j0 = last; j0 >= 0; j0 -= nb) {
        const int b = static_cast<int>(n - j0 < nb ? n - j0 : nb);
        const int64_t rest = n - j0 - b;
        if (rest > 0) {
            const int rc = oz_zgemm(h, 'N', 'N', b, n, rest, minus_one, LU + 2 * (j0 + (j0 + b) * lda), lda,
                                    X + 2 * (j0 + b), ldx, one, X + 2 * j0, ldx, prec, nullptr);
            if (rc) return rc;
        }
        if (launch_trsm(true, LU + 2 * (j0 + j0 * lda), lda, b, X + 2 * j0, ldx, n, s) != hipSuccess)
            return OZ_ERR_HIP;
    }
    return hipStreamSynchronize(s) == hipSuccess ? OZ_OK : OZ_ERR_HIP;
}

}  // extern "C"
