// oz_lu.hip -- LU-based complex inversion with emulated trailing products
// (the paper's application: an LU-based matrix inverse rich in ZGEMM, with
// every ZGEMM emulated at the chosen split number, Sec. 3.2 and Table 1).
//
// Right-looking blocked LU with partial pivoting.  Within a panel of nb
// columns the arithmetic is that of the column-by-column algorithm (pivot =
// first row of largest |re| + |im|, row swap across the panel, scaling by the
// pivot's reciprocal, rank-1 updates of the panel columns to the right), so
// every entry receives its updates one at a time in ascending column order.
// The panel is worked through in narrow sub-panels: one block factors the
// sub-panel with its rows in registers (the pivot chain), applies its
// interchanges to the other panel columns and solves their top rows, and a
// many-block kernel then applies the sub-panel's rank-w update to the rows
// below -- the same operations on every entry in the same order, so the
// result is that of the column-by-column panel bit for bit.  After the panel:
// the interchanges on the other columns, U12 = L11^-1 A12, and
// A22 -= L21 U12 as an emulated ZGEMM (oz_zgemm with alpha = -1, beta = 1).
// The inverse solves A X = I: X = P I, then block by block
// X_i -= L[i, :i] X[:i] (emulated) and X_i = L_ii^-1 X_i, then from the last
// block X_i -= U[i, i+1:] X[i+1:] (emulated) and X_i = U_ii^-1 X_i -- run
// against I with the columns permuted at the end, which gives the same bits
// and skips the structural zeros of L^-1.
// Complex arithmetic is written out on the parts, (ar br - ai bi, ar bi + ai br),
// with no fused multiply-add (the library is built with -ffp-contract=off).
#include <hip/hip_runtime.h>

#include "oz_handle.h"

namespace {

constexpr int kPanelThreads = 1024;
// Register panel of width 8 (up to 2048 rows): 512 threads of 4 rows; 1024
// threads of 2 rows spilled 88 registers.  Widths 4 and 2 keep 1024
// threads: 512 threads of 8 rows measured the same at width 4 (28.0 us per
// launch either way), and 16 rows per thread would spill at width 2.
constexpr int kRegPanelThreads = 512;
constexpr int kMaxRegRows = 8192;
constexpr int kMaxWaveTrsm = 256; // wave-per-column triangular solves: b <= 256
constexpr int kMaxGatherSwaps = 256;
constexpr int kDefaultPanel = 128;       // oz_zgetrf nb = 0
constexpr int kDefaultSolveBlock = 256;  // oz_zgetri nb = 0

__device__ __forceinline__ double* at(double* X, int64_t ld, int64_t r, int64_t c) { return X + 2 * (r + c * ld); }
__device__ __forceinline__ const double* at(const double* X, int64_t ld, int64_t r, int64_t c) {
    return X + 2 * (r + c * ld);
}

// (ar + i ai)(br + i bi), each product and sum rounded
__device__ __forceinline__ void cmul(double ar, double ai, double br, double bi, double& cr, double& ci) {
    cr = ar * br - ai * bi;
    ci = ar * bi + ai * br;
}

// 1 / (pr + i pi) = (pr - i pi) / (pr^2 + pi^2)
__device__ __forceinline__ void crecip(double pr, double pi, double& rr, double& ri) {
    const double q = pr * pr + pi * pi;
    rr = pr / q;
    ri = -pi / q;
}

// value of lane `src` (wave-uniform) to every lane
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffull), src);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                                       static_cast<unsigned>(lo)));
}

// (v, i) beats (bv, bi): larger value, or equal value and smaller row
__device__ __forceinline__ bool pivot_better(double v, int i, double bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

// ---------------------------------------------------------------------------
// Panel, sub-panel step 1 (one block of NT threads): factor the sub-panel
// columns c0 .. c0 + w - 1 over rows c0 .. n - 1, thread t holding rows
// c0 + t + NT s (s < R) of those columns in registers; then, for every other
// panel column (j0 .. j0 + b - 1), apply the sub-panel's interchanges and, to
// the right of it, solve the w top rows with the unit lower w x w block.
template <int NT, int R, int W>
__global__ __launch_bounds__(NT) void panel_reg_kernel(double* A, int64_t lda, int64_t n, int64_t j0, int b,
                                                       int64_t c0, int w, int32_t* ipiv, int32_t* info) {
    __shared__ double red_v[NT / 64];
    __shared__ int red_i[NT / 64];
    __shared__ double rowj[2 * W], rowp[2 * W];
    __shared__ double l11[W][2 * W];
    __shared__ int psub[W];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = static_cast<int>(n - c0);
    double xr[R][W], xi[R][W];
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const int r = tid + NT * s;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            xr[s][c] = 0.0;
            xi[s][c] = 0.0;
            if (r < m && c < w) {
                const double* e = at(A, lda, c0 + r, c0 + c);
                xr[s][c] = e[0];
                xi[s][c] = e[1];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < W; ++c) {
        if (c < w) {
            // pivot: first row >= c (relative) of largest |re| + |im|
            double best = -1.0;
            int bi = c;
    #pragma unroll
            for (int s = 0; s < R; ++s) {
                const int r = tid + NT * s;
                if (r >= c && r < m) {
                    const double v = fabs(xr[s][c]) + fabs(xi[s][c]);
                    if (v > best) {
                        best = v;
                        bi = r;
                    }
                }
            }
    #pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double v2 = __shfl_xor(best, off);
                const int i2 = __shfl_xor(bi, off);
                if (pivot_better(v2, i2, best, bi)) {
                    best = v2;
                    bi = i2;
                }
            }
            if (lane == 0) {
                red_v[wave] = best;
                red_i[wave] = bi;
            }
            __syncthreads();
            best = red_v[0];
            bi = red_i[0];
            for (int q = 1; q < NT / 64; ++q)
                if (pivot_better(red_v[q], red_i[q], best, bi)) {
                    best = red_v[q];
                    bi = red_i[q];
                }
            const int p = bi;
            const int owner = p % NT, slot = p / NT;
            // exchange rows c and p of the sub-panel through LDS (row c: thread c, slot 0)
            if (tid == c) {
    #pragma unroll
                for (int k = 0; k < W; ++k) {
                    rowj[2 * k] = xr[0][k];
                    rowj[2 * k + 1] = xi[0][k];
                }
            }
            if (tid == owner) {
    #pragma unroll
                for (int s = 0; s < R; ++s)
                    if (s == slot) {
    #pragma unroll
                        for (int k = 0; k < W; ++k) {
                            rowp[2 * k] = xr[s][k];
                            rowp[2 * k + 1] = xi[s][k];
                        }
                    }
            }
            __syncthreads();
            if (p != c) {
                if (tid == c) {
    #pragma unroll
                    for (int k = 0; k < W; ++k) {
                        xr[0][k] = rowp[2 * k];
                        xi[0][k] = rowp[2 * k + 1];
                    }
                }
                if (tid == owner) {
    #pragma unroll
                    for (int s = 0; s < R; ++s)
                        if (s == slot) {
    #pragma unroll
                            for (int k = 0; k < W; ++k) {
                                xr[s][k] = rowj[2 * k];
                                xi[s][k] = rowj[2 * k + 1];
                            }
                        }
                }
            }
            if (tid == 0) {
                ipiv[c0 + c] = static_cast<int32_t>(c0 + p);
                psub[c] = p;
            }
            const double ppr = rowp[2 * c], ppi = rowp[2 * c + 1];
            const bool zero = ppr == 0.0 && ppi == 0.0;
            if (zero) {
                if (tid == 0 && *info == 0) *info = static_cast<int32_t>(c0 + c + 1);
            } else {
                double rr, ri;
                crecip(ppr, ppi, rr, ri);
    #pragma unroll
                for (int s = 0; s < R; ++s) {
                    const int r = tid + NT * s;
                    if (r > c && r < m) {
                        double lr, li;
                        cmul(xr[s][c], xi[s][c], rr, ri, lr, li);
                        xr[s][c] = lr;
                        xi[s][c] = li;
                    }
                }
            }
            // rank-1 update of the sub-panel columns right of c
    #pragma unroll
            for (int s = 0; s < R; ++s) {
                const int r = tid + NT * s;
                if (r > c && r < m) {
    #pragma unroll
                    for (int k = c + 1; k < W; ++k) {
                        if (k < w) {
                            double tr, ti;
                            cmul(xr[s][c], xi[s][c], rowp[2 * k], rowp[2 * k + 1], tr, ti);
                            xr[s][k] = xr[s][k] - tr;
                            xi[s][k] = xi[s][k] - ti;
                        }
                    }
                }
            }
        }
    }
    // write the factored sub-panel back; keep its top w x w block in LDS
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const int r = tid + NT * s;
#pragma unroll
        for (int c = 0; c < W; ++c)
            if (r < m && c < w) {
                double* e = at(A, lda, c0 + r, c0 + c);
                e[0] = xr[s][c];
                e[1] = xi[s][c];
            }
    }
    if (tid < w) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            l11[tid][2 * k] = xr[0][k];
            l11[tid][2 * k + 1] = xi[0][k];
        }
    }
    // net effect of the w interchanges on the rows they touch (the block rows
    // c0 + e and the pivot rows): row dst[e] ends up holding row src[e]
    __shared__ int dst[2 * W], src[2 * W];
    if (tid < 2 * w) {
        const int x = tid < w ? tid : psub[tid - w];
        int y = x;
        for (int i = w - 1; i >= 0; --i) {
            const int p = psub[i];
            if (y == i)
                y = p;
            else if (y == p)
                y = i;
        }
        dst[tid] = x;
        src[tid] = y;
    }
    __syncthreads();
    // the other panel columns: the interchanges (all loads, then the stores of
    // the pivot rows), then right of the sub-panel u_i = a_i - sum_{k < i}
    // l_ik u_k over the w top rows, in registers
    const int left = static_cast<int>(c0 - j0), right = b - left - w;
    for (int t = tid; t < left + right; t += NT) {
        const int64_t col = t < left ? j0 + t : c0 + w + (t - left);
        double vr[2 * W], vi[2 * W];
#pragma unroll
        for (int e = 0; e < 2 * W; ++e) {
            vr[e] = 0.0;
            vi[e] = 0.0;
            if (e < 2 * w) {
                const double* q = at(A, lda, c0 + src[e], col);
                vr[e] = q[0];
                vi[e] = q[1];
            }
        }
#pragma unroll
        for (int e = 0; e < 2 * W; ++e) {
            if (e >= w && e < 2 * w && src[e] != dst[e]) {
                double* q = at(A, lda, c0 + dst[e], col);
                q[0] = vr[e];
                q[1] = vi[e];
            }
        }
        if (t >= left) {
#pragma unroll
            for (int i = 1; i < W; ++i) {
                if (i < w) {
#pragma unroll
                    for (int k = 0; k < i; ++k) {
                        double tr, ti;
                        cmul(l11[i][2 * k], l11[i][2 * k + 1], vr[k], vi[k], tr, ti);
                        vr[i] = vr[i] - tr;
                        vi[i] = vi[i] - ti;
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < W; ++i) {
            if (i < w) {
                double* q = at(A, lda, c0 + i, col);
                q[0] = vr[i];
                q[1] = vi[i];
            }
        }
    }
}

// Panel, sub-panel step 2: rows c0 + w .. n - 1 of the panel columns
// c0 + w .. cend - 1 get a_rk - sum_{i < w} l_{r,c0+i} u_{c0+i,k}, one term at
// a time in ascending i (grid.x over rows, grid.y over columns).
__global__ __launch_bounds__(256) void panel_update_kernel(double* A, int64_t lda, int64_t n, int64_t c0, int w) {
    __shared__ double u[2 * 8];
    const int64_t k = c0 + w + blockIdx.y;
    if (threadIdx.x < w) {
        const double* e = at(A, lda, c0 + threadIdx.x, k);
        u[2 * threadIdx.x] = e[0];
        u[2 * threadIdx.x + 1] = e[1];
    }
    __syncthreads();
    const int64_t r = c0 + w + static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (r >= n) return;
    double* e = at(A, lda, r, k);
    double accr = e[0], acci = e[1];
    for (int i = 0; i < w; ++i) {
        const double* l = at(A, lda, r, c0 + i);
        double tr, ti;
        cmul(l[0], l[1], u[2 * i], u[2 * i + 1], tr, ti);
        accr = accr - tr;
        acci = acci - ti;
    }
    e[0] = accr;
    e[1] = acci;
}

// Whole panel in one block through global memory (rows n - j0 beyond the
// register panel's reach): the column-by-column algorithm as written.
__global__ __launch_bounds__(kPanelThreads) void panel_kernel(double* A, int64_t lda, int64_t n, int64_t j0, int b,
                                                              int32_t* ipiv, int32_t* info) {
    __shared__ double red_v[kPanelThreads];
    __shared__ int64_t red_i[kPanelThreads];
    __shared__ double s_rr, s_ri;
    __shared__ int s_zero;
    const int tid = threadIdx.x;
    for (int c = 0; c < b; ++c) {
        const int64_t j = j0 + c;
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
            s_zero = (d[0] == 0.0 && d[1] == 0.0) ? 1 : 0;
            if (s_zero) {
                if (*info == 0) *info = static_cast<int32_t>(j + 1);
            } else {
                double rr, ri;
                crecip(d[0], d[1], rr, ri);
                s_rr = rr;
                s_ri = ri;
            }
        }
        __syncthreads();
        if (!s_zero) {
            const double rr = s_rr, ri = s_ri;
            for (int64_t r = j + 1 + tid; r < n; r += kPanelThreads) {
                double* e = at(A, lda, r, j);
                double lr, li;
                cmul(e[0], e[1], rr, ri, lr, li);
                e[0] = lr;
                e[1] = li;
            }
        }
        __syncthreads();
        for (int64_t r = j + 1 + tid; r < n; r += kPanelThreads) {
            const double* l = at(A, lda, r, j);
            const double lr = l[0], li = l[1];
            for (int64_t k = j + 1; k < j0 + b; ++k) {
                const double* u = at(A, lda, j, k);
                double tr, ti;
                cmul(lr, li, u[0], u[1], tr, ti);
                double* e = at(A, lda, r, k);
                e[0] = e[0] - tr;
                e[1] = e[1] - ti;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Row interchanges r0 .. r0 + nsw - 1 (in order) on columns c0 .. c1 - 1 as one
// gather: the affected rows are the block rows and the pivot rows; the final
// content of row x is the original row found by undoing the interchanges from
// the last (one wave per column, loads before stores).
__global__ __launch_bounds__(256) void laswp_gather_kernel(double* X, int64_t ld, int64_t c0, int64_t c1, int64_t r0,
                                                           int nsw, const int32_t* ipiv) {
    constexpr int kE = 2 * kMaxGatherSwaps / 64;
    __shared__ int32_t piv[kMaxGatherSwaps];
    __shared__ int64_t dst[2 * kMaxGatherSwaps], src[2 * kMaxGatherSwaps];
    for (int t = threadIdx.x; t < nsw; t += 256) piv[t] = ipiv[r0 + t];
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * nsw; e += 256) {
        const int64_t x = e < nsw ? r0 + e : static_cast<int64_t>(piv[e - nsw]);
        int64_t y = x;
        for (int j = nsw - 1; j >= 0; --j) {
            const int64_t jj = r0 + j, pp = piv[j];
            if (y == jj)
                y = pp;
            else if (y == pp)
                y = jj;
        }
        dst[e] = x;
        src[e] = y;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * 4;
    for (int64_t c = c0 + static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6); c < c1; c += waves) {
        double vr[kE], vi[kE];
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const int e = lane + 64 * q;
            vr[q] = 0.0;
            vi[q] = 0.0;
            if (e < 2 * nsw && src[e] != dst[e]) {
                const double* s = at(X, ld, src[e], c);
                vr[q] = s[0];
                vi[q] = s[1];
            }
        }
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const int e = lane + 64 * q;
            if (e < 2 * nsw && src[e] != dst[e]) {
                double* d = at(X, ld, dst[e], c);
                d[0] = vr[q];
                d[1] = vi[q];
            }
        }
    }
}

// Row interchanges one column per thread (blocks of more than
// kMaxGatherSwaps interchanges).
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

// src[x] = the row of I that row x of P I holds: undo the interchanges
// j = n - 1 .. 0 starting from x (one thread per row, pivots staged in LDS).
__global__ __launch_bounds__(256) void perm_src_kernel(const int32_t* ipiv, int64_t n, int32_t* src) {
    __shared__ int32_t sp[1024];
    const int64_t x = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    int64_t y = x;
    for (int64_t hi = n; hi > 0; hi -= 1024) {
        const int64_t lo = hi > 1024 ? hi - 1024 : 0;
        __syncthreads();
        for (int64_t t = lo + threadIdx.x; t < hi; t += 256) sp[t - lo] = ipiv[t];
        __syncthreads();
        for (int64_t j = hi - 1; j >= lo; --j) {
            const int64_t p = sp[j - lo];
            if (y == j)
                y = p;
            else if (y == p)
                y = j;
        }
    }
    if (x < n) src[x] = static_cast<int32_t>(y);
}

// T = I (n x n).
__global__ void identity_kernel(double* T, int64_t ldt, int64_t n) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int64_t c = blockIdx.y; c < n; c += gridDim.y) {
        double* e = at(T, ldt, r, c);
        e[0] = r == c ? 1.0 : 0.0;
        e[1] = 0.0;
    }
}

// X[:, src[c]] = T[:, c]: the column permutation that turns L^-1-based
// columns into those of the inverse (grid.x over rows, grid.y over columns).
__global__ void col_scatter_kernel(const double* T, int64_t ldt, double* X, int64_t ldx, int64_t n,
                                   const int32_t* src) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int64_t c = blockIdx.y; c < n; c += gridDim.y) {
        const int64_t d = src[c];
        if (d < 0 || d >= n) continue;  // pivots not from oz_zgetrf: no access outside X
        const double* t = at(T, ldt, r, c);
        double* x = at(X, ldx, r, d);
        x[0] = t[0];
        x[1] = t[1];
    }
}

// ---------------------------------------------------------------------------
// Triangular solves with b x ncols right-hand sides B, one wave per column
// (16 per block), lane l holding rows l + 64 t (t < R2), the triangle staged
// through LDS 16 columns at a time.  Column-oriented: once x_k is final it is
// broadcast and every row still open subtracts t_ik x_k, so each row's sum runs
// over the unknowns in the order they are solved (ascending for the unit lower
// solve; descending for the upper one, where x_k is the open sum times the
// reciprocal of u_kk).
constexpr int kTrsmWaves = 16;
constexpr int kTrsmChunk = 16;

template <int R2, bool UPPER>
__global__ __launch_bounds__(64 * kTrsmWaves) void trsm_wave_kernel(const double* T, int64_t ldt, int b, double* B,
                                                                    int64_t ldb, int64_t ncols) {
    __shared__ double tk[kTrsmChunk][2 * 64 * R2];
    __shared__ double rec[2 * 64 * R2];
    constexpr int kThreads = 64 * kTrsmWaves;
    if (UPPER) {
        for (int i = threadIdx.x; i < b; i += kThreads) {
            const double* d = at(T, ldt, i, i);
            double rr, ri;
            crecip(d[0], d[1], rr, ri);
            rec[2 * i] = rr;
            rec[2 * i + 1] = ri;
        }
    }
    const int lane = threadIdx.x & 63;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kTrsmWaves + (threadIdx.x >> 6);
    const bool active = c < ncols;
    double xr[R2], xi[R2];
#pragma unroll
    for (int t = 0; t < R2; ++t) {
        const int i = lane + 64 * t;
        xr[t] = 0.0;
        xi[t] = 0.0;
        if (active && i < b) {
            const double* e = at(B, ldb, i, c);
            xr[t] = e[0];
            xi[t] = e[1];
        }
    }
    const int nchunks = (b + kTrsmChunk - 1) / kTrsmChunk;
    for (int q = 0; q < nchunks; ++q) {
        // columns k_lo .. k_lo + kc - 1 of the triangle
        const int k_lo = UPPER ? (b - (q + 1) * kTrsmChunk > 0 ? b - (q + 1) * kTrsmChunk : 0) : q * kTrsmChunk;
        const int k_hi = UPPER ? b - q * kTrsmChunk : (b < (q + 1) * kTrsmChunk ? b : (q + 1) * kTrsmChunk);
        const int kc = k_hi - k_lo;
        __syncthreads();
        for (int e = threadIdx.x; e < b * kc; e += kThreads) {
            const int kk = e / b, i = e - kk * b;
            const double* v = at(T, ldt, i, k_lo + kk);
            tk[kk][2 * i] = v[0];
            tk[kk][2 * i + 1] = v[1];
        }
        __syncthreads();
        if (!active) continue;
        for (int s = 0; s < kc; ++s) {
            const int k = UPPER ? k_hi - 1 - s : k_lo + s;
            const int kk = k - k_lo;
            const int tk_ = k >> 6, src = k & 63;
            double ar = xr[0], ai = xi[0];
#pragma unroll
            for (int t = 1; t < R2; ++t)
                if (tk_ == t) {
                    ar = xr[t];
                    ai = xi[t];
                }
            double vr = ar, vi = ai;
            if (UPPER) cmul(ar, ai, rec[2 * k], rec[2 * k + 1], vr, vi);
            vr = lane_bcast(vr, src);
            vi = lane_bcast(vi, src);
            if (UPPER && lane == src) {
#pragma unroll
                for (int t = 0; t < R2; ++t)
                    if (tk_ == t) {
                        xr[t] = vr;
                        xi[t] = vi;
                    }
            }
#pragma unroll
            for (int t = 0; t < R2; ++t) {
                // slots whose rows are all solved (wave-uniform test) are skipped
                if (UPPER ? 64 * t >= k : 64 * t + 63 <= k) continue;
                const int i = lane + 64 * t;
                if (UPPER ? i < k : (i > k && i < b)) {
                    double tr, ti;
                    cmul(tk[kk][2 * i], tk[kk][2 * i + 1], vr, vi, tr, ti);
                    xr[t] = xr[t] - tr;
                    xi[t] = xi[t] - ti;
                }
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int t = 0; t < R2; ++t) {
        const int i = lane + 64 * t;
        if (i < b) {
            double* e = at(B, ldb, i, c);
            e[0] = xr[t];
            e[1] = xi[t];
        }
    }
}

// The same solves one column per thread (b beyond kMaxWaveTrsm).
__global__ void trsm_lower_unit_kernel(const double* L, int64_t ldl, int b, double* B, int64_t ldb, int64_t ncols) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    for (int i = 0; i < b; ++i) {
        double* bi = at(B, ldb, i, c);
        double accr = bi[0], acci = bi[1];
        for (int k = 0; k < i; ++k) {
            const double* l = at(L, ldl, i, k);
            const double* x = at(B, ldb, k, c);
            double tr, ti;
            cmul(l[0], l[1], x[0], x[1], tr, ti);
            accr = accr - tr;
            acci = acci - ti;
        }
        bi[0] = accr;
        bi[1] = acci;
    }
}

__global__ void trsm_upper_kernel(const double* U, int64_t ldu, int b, double* B, int64_t ldb, int64_t ncols) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    for (int i = b - 1; i >= 0; --i) {
        double* bi = at(B, ldb, i, c);
        double accr = bi[0], acci = bi[1];
        for (int k = b - 1; k > i; --k) {
            const double* u = at(U, ldu, i, k);
            const double* x = at(B, ldb, k, c);
            double tr, ti;
            cmul(u[0], u[1], x[0], x[1], tr, ti);
            accr = accr - tr;
            acci = acci - ti;
        }
        const double* d = at(U, ldu, i, i);
        double rr, ri, vr, vi;
        crecip(d[0], d[1], rr, ri);
        cmul(accr, acci, rr, ri, vr, vi);
        bi[0] = vr;
        bi[1] = vi;
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_laswp(double* X, int64_t ld, int64_t c0, int64_t c1, int64_t r0, int64_t r1, const int32_t* ipiv,
                        hipStream_t st) {
    if (c1 <= c0 || r1 <= r0) return hipSuccess;
    if (r1 - r0 <= kMaxGatherSwaps) {
        const int64_t blocks = (c1 - c0 + 3) / 4;
        hipLaunchKernelGGL(laswp_gather_kernel, dim3(static_cast<unsigned>(blocks < 2048 ? blocks : 2048)), dim3(256),
                           0, st, X, ld, c0, c1, r0, static_cast<int>(r1 - r0), ipiv);
    } else {
        hipLaunchKernelGGL(laswp_kernel, dim3(static_cast<unsigned>((c1 - c0 + 255) / 256)), dim3(256), 0, st, X, ld,
                           c0, c1, r0, r1, ipiv);
    }
    return hipGetLastError();
}

template <bool UPPER>
void launch_trsm_wave(int r2, dim3 grid, hipStream_t st, const double* T, int64_t ldt, int b, double* B, int64_t ldb,
                      int64_t ncols) {
    const dim3 blk(64 * kTrsmWaves);
    switch (r2) {
        case 1: hipLaunchKernelGGL((trsm_wave_kernel<1, UPPER>), grid, blk, 0, st, T, ldt, b, B, ldb, ncols); break;
        case 2: hipLaunchKernelGGL((trsm_wave_kernel<2, UPPER>), grid, blk, 0, st, T, ldt, b, B, ldb, ncols); break;
        case 3: hipLaunchKernelGGL((trsm_wave_kernel<3, UPPER>), grid, blk, 0, st, T, ldt, b, B, ldb, ncols); break;
        default: hipLaunchKernelGGL((trsm_wave_kernel<4, UPPER>), grid, blk, 0, st, T, ldt, b, B, ldb, ncols); break;
    }
}

hipError_t launch_trsm(bool upper, const double* T, int64_t ldt, int b, double* B, int64_t ldb, int64_t ncols,
                       hipStream_t st) {
    if (ncols <= 0 || b <= 0) return hipSuccess;
    if (b <= kMaxWaveTrsm) {
        const dim3 grid(static_cast<unsigned>((ncols + kTrsmWaves - 1) / kTrsmWaves));
        const int r2 = (b + 63) / 64;
        if (upper)
            launch_trsm_wave<true>(r2, grid, st, T, ldt, b, B, ldb, ncols);
        else
            launch_trsm_wave<false>(r2, grid, st, T, ldt, b, B, ldb, ncols);
    } else {
        const dim3 grid(static_cast<unsigned>((ncols + 63) / 64));
        if (upper)
            hipLaunchKernelGGL(trsm_upper_kernel, grid, dim3(64), 0, st, T, ldt, b, B, ldb, ncols);
        else
            hipLaunchKernelGGL(trsm_lower_unit_kernel, grid, dim3(64), 0, st, T, ldt, b, B, ldb, ncols);
    }
    return hipGetLastError();
}

// One panel (columns j0 .. j0 + b - 1): sub-panels in registers when the rows
// fit (width 8: 4 rows per thread of 512; widths 4 and 2: 4 and 8 rows per
// thread of 1024), else the global-memory panel kernel.
hipError_t launch_panel(double* A, int64_t lda, int64_t n, int64_t j0, int b, int32_t* ipiv, int32_t* info,
                        hipStream_t st) {
    if (n - j0 > kMaxRegRows) {
        hipLaunchKernelGGL(panel_kernel, dim3(1), dim3(kPanelThreads), 0, st, A, lda, n, j0, b, ipiv, info);
        return hipGetLastError();
    }
    for (int64_t c0 = j0; c0 < j0 + b;) {
        const int64_t m = n - c0;
        // sub-panel width 8, 4, 2 for up to 2048, 4096, 8192 rows
        const int W = m <= 2048 ? 8 : m <= 4096 ? 4 : 2;
        const int w = static_cast<int>(j0 + b - c0 < W ? j0 + b - c0 : W);
        const dim3 grid(1), small(kRegPanelThreads), large(kPanelThreads);
        switch (W) {
            case 8: hipLaunchKernelGGL((panel_reg_kernel<kRegPanelThreads, 4, 8>), grid, small, 0, st, A, lda, n, j0, b, c0, w, ipiv, info); break;
            case 4: hipLaunchKernelGGL((panel_reg_kernel<kPanelThreads, 4, 4>), grid, large, 0, st, A, lda, n, j0, b, c0, w, ipiv, info); break;
            default: hipLaunchKernelGGL((panel_reg_kernel<kPanelThreads, 8, 2>), grid, large, 0, st, A, lda, n, j0, b, c0, w, ipiv, info); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t cols = j0 + b - c0 - w, rows = n - c0 - w;
        if (cols > 0 && rows > 0) {
            hipLaunchKernelGGL(panel_update_kernel, dim3(static_cast<unsigned>((rows + 255) / 256),
                                                         static_cast<unsigned>(cols)),
                               dim3(256), 0, st, A, lda, n, c0, w);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        c0 += w;
    }
    return hipSuccess;
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
    if (n > INT32_MAX) return OZ_ERR_UNSUPPORTED;
    if (nb == 0) nb = kDefaultPanel;
    int st = oz_handle_use_device(h);
    if (st) return st;
    hipStream_t s = oz_handle_stream(h);
    // Look-ahead: panel k + 1 is factored on a second stream while the handle's
    // stream runs the rest of panel k's trailing product.  The trailing product
    // is issued as two products split by columns (first the next panel's
    // columns, then the rest); an entry of an emulated product depends only on
    // its row of op(A) and its column of op(B), so the split changes no result.
    // the second stream, its events and the info word come from the handle
    // (created on the first call, reused after): nothing is allocated per call
    hipStream_t s2 = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    int rc = oz_handle_lu_stream(h, &s2, ev);
    if (rc) return rc;
    hipEvent_t ev_start = ev[0], ev_panel = ev[1], ev_next = ev[2];
    int32_t* dinfo = reinterpret_cast<int32_t*>(oz_handle_lu_ws(h, 256, &rc));
    if (rc) return rc;
    if (rc == OZ_OK && (hipMemsetAsync(dinfo, 0, sizeof(int32_t), s) != hipSuccess ||
                        hipEventRecord(ev_start, s) != hipSuccess || hipStreamWaitEvent(s2, ev_start, 0) != hipSuccess))
        rc = OZ_ERR_HIP;
    const double minus_one[2] = {-1.0, 0.0}, one[2] = {1.0, 0.0};
    for (int64_t j0 = 0; rc == OZ_OK && j0 < n; j0 += nb) {
        const int b = static_cast<int>(n - j0 < nb ? n - j0 : nb);
        if (launch_panel(A, lda, n, j0, b, ipiv, dinfo, s2) != hipSuccess || hipEventRecord(ev_panel, s2) != hipSuccess ||
            hipStreamWaitEvent(s, ev_panel, 0) != hipSuccess ||
            launch_laswp(A, lda, 0, j0, j0, j0 + b, ipiv, s) != hipSuccess) {
            rc = OZ_ERR_HIP;
            break;
        }
        const int64_t rest = n - j0 - b;
        if (rest <= 0) break;
        const double* L21 = A + 2 * ((j0 + b) + j0 * lda);
        double* A12 = A + 2 * (j0 + (j0 + b) * lda);
        double* A22 = A + 2 * ((j0 + b) + (j0 + b) * lda);
        if (launch_laswp(A, lda, j0 + b, n, j0, j0 + b, ipiv, s) != hipSuccess ||
            launch_trsm(false, A + 2 * (j0 + j0 * lda), lda, b, A12, lda, rest, s) != hipSuccess) {
            rc = OZ_ERR_HIP;
            break;
        }
        const int64_t next = rest < nb ? rest : nb;
        rc = oz_zgemm(h, 'N', 'N', rest, next, b, minus_one, L21, lda, A12, lda, one, A22, lda, prec, nullptr);
        if (rc) break;
        if (hipEventRecord(ev_next, s) != hipSuccess || hipStreamWaitEvent(s2, ev_next, 0) != hipSuccess) {
            rc = OZ_ERR_HIP;
            break;
        }
        if (rest > next)
            rc = oz_zgemm(h, 'N', 'N', rest, rest - next, b, minus_one, L21, lda, A12 + 2 * next * lda, lda, one,
                          A22 + 2 * next * lda, lda, prec, nullptr);
    }
    if (rc == OZ_OK && (hipMemcpyAsync(info, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
        rc = OZ_ERR_HIP;
    if (s2 && hipStreamSynchronize(s2) != hipSuccess) rc = OZ_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) rc = OZ_ERR_HIP;
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
    if (n > INT32_MAX) return OZ_ERR_UNSUPPORTED;
    if (nb == 0) nb = kDefaultSolveBlock;
    int st = oz_handle_use_device(h);
    if (st) return st;
    hipStream_t s = oz_handle_stream(h);
    const double minus_one[2] = {-1.0, 0.0}, one[2] = {1.0, 0.0};
    // The solves run against I into a work matrix T, and the columns are
    // permuted at the end: column j of L^-1 (P I) is column r of L^-1 for the
    // row r of P I that holds the one of column j (src[r] = j).  Each column
    // takes exactly the same operations either way -- an entry of an emulated
    // product depends only on its row of op(A) and its column of op(B), and
    // the triangular solves work column by column -- so the inverse is the
    // same bit for bit.  Against I, block row i of L^-1 is zero right of
    // column (i+1) nb: those columns are neither multiplied nor solved (they
    // stay +0, as subtracting +-0 from them would leave them).
    // T (n x n complex) and the column sources from the handle's LU buffer
    // (grow-only): nothing is allocated per call once it is large enough
    const int64_t ldt = n;
    const size_t t_bytes = sizeof(double) * 2 * static_cast<size_t>(n) * static_cast<size_t>(n);
    int wst = OZ_OK;
    char* ws = oz_handle_lu_ws(h, t_bytes + ((sizeof(int32_t) * static_cast<size_t>(n) + 255) & ~size_t(255)), &wst);
    if (wst) return wst;
    double* T = reinterpret_cast<double*>(ws);
    int32_t* src = reinterpret_cast<int32_t*>(ws + t_bytes);
    const dim3 grid_nn(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n < 65535 ? n : 65535));
    hipLaunchKernelGGL(perm_src_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, ipiv, n, src);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(identity_kernel, grid_nn, dim3(256), 0, s, T, ldt, n);
        e = hipGetLastError();
    }
    int rc = e == hipSuccess ? OZ_OK : OZ_ERR_HIP;
    // forward: L Y = I, block row i over columns [0, (i+1) nb)
    for (int64_t j0 = 0; rc == OZ_OK && j0 < n; j0 += nb) {
        const int b = static_cast<int>(n - j0 < nb ? n - j0 : nb);
        if (j0 > 0) {
            rc = oz_zgemm(h, 'N', 'N', b, j0, j0, minus_one, LU + 2 * j0, lda, T, ldt, one, T + 2 * j0, ldt, prec,
                          nullptr);
            if (rc) break;
        }
        if (launch_trsm(false, LU + 2 * (j0 + j0 * lda), lda, b, T + 2 * j0, ldt, j0 + b, s) != hipSuccess)
            rc = OZ_ERR_HIP;
    }
    // backward: U T = Y, all columns
    const int64_t last = ((n - 1) / nb) * nb;
    for (int64_t j0 = last; rc == OZ_OK && j0 >= 0; j0 -= nb) {
        const int b = static_cast<int>(n - j0 < nb ? n - j0 : nb);
        const int64_t rest = n - j0 - b;
        if (rest > 0) {
            rc = oz_zgemm(h, 'N', 'N', b, n, rest, minus_one, LU + 2 * (j0 + (j0 + b) * lda), lda, T + 2 * (j0 + b),
                          ldt, one, T + 2 * j0, ldt, prec, nullptr);
            if (rc) break;
        }
        if (launch_trsm(true, LU + 2 * (j0 + j0 * lda), lda, b, T + 2 * j0, ldt, n, s) != hipSuccess)
            rc = OZ_ERR_HIP;
    }
    if (rc == OZ_OK) {
        hipLaunchKernelGGL(col_scatter_kernel, grid_nn, dim3(256), 0, s, T, ldt, X, ldx, n, src);
        if (hipGetLastError() != hipSuccess) rc = OZ_ERR_HIP;
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == OZ_OK) rc = OZ_ERR_HIP;
    return rc;
}

}  // extern "C"
