// oz_blas.cpp -- dgemm_ / zgemm_ with the Fortran BLAS calling convention,
// run on the GPU through the emulated path (or native FP64 for comparison).
// The offload layer of the method (paper Sec. 2.1 and 3.1): a program linked
// against this library gets its level-3 products from the GPU's INT8 units,
// with the arithmetic chosen per run by OZ_COMPUTE_MODE.  See oz_blas.h.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "oz.h"
#include "oz_blas.h"

namespace {

enum Mode { kNative = 0, kFixed = 1, kTol = 2, kBalanced = 3 };

struct Config {
    int mode = kFixed;
    int slices = 7;
    double tol = 0.0;
    int zmode = 0;  // the library's measured choice
    int device = 0;
};

// Parses a mode string; false when it is not one.
bool parse_mode(const char* s, Config* c) {
    if (!s) return false;
    const std::string m(s);
    if (m == "dgemm") {
        c->mode = kNative;
        return true;
    }
    const std::string tol_prefix = "fp64_int8_tol", bal_prefix = "fp64_int8_bal", fix_prefix = "fp64_int8_";
    if (m.compare(0, bal_prefix.size(), bal_prefix) == 0) {
        char* end = nullptr;
        const long v = std::strtol(m.c_str() + bal_prefix.size(), &end, 10);
        if (!end || *end != '\0' || end == m.c_str() + bal_prefix.size() || v < 1 || v > 8) return false;
        c->mode = kBalanced;
        c->slices = static_cast<int>(v);
        return true;
    }
    if (m.compare(0, tol_prefix.size(), tol_prefix) == 0) {
        char* end = nullptr;
        const double t = std::strtod(m.c_str() + tol_prefix.size(), &end);
        if (!end || *end != '\0' || !(t > 0.0)) return false;
        c->mode = kTol;
        c->tol = t;
        return true;
    }
    if (m.compare(0, fix_prefix.size(), fix_prefix) == 0) {
        char* end = nullptr;
        const long v = std::strtol(m.c_str() + fix_prefix.size(), &end, 10);
        if (!end || *end != '\0' || end == m.c_str() + fix_prefix.size() || v < 1 || v > 18) return false;
        c->mode = kFixed;
        c->slices = static_cast<int>(v);
        return true;
    }
    return false;
}

// A device buffer that only grows.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

// Host<->device copies of host operands go through two pinned staging
// buffers: the columns of one chunk are packed (by several threads for large
// chunks) while the DMA of the other chunk runs.  Pageable memory cannot be
// registered here, and the runtime's own staging of pageable copies is slower.
constexpr size_t kStageBytes = size_t(32) << 20;
constexpr size_t kThreadedBytes = size_t(4) << 20;  // chunks above this are packed by several threads

struct Ctx {
    std::mutex mu;
    bool configured = false;  // environment read
    bool ready = false;       // device objects created
    Config cfg;
    oz_handle_t oz = nullptr;
    rocblas_handle rb = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    DevBuf buf[3];
    void* pin[2] = {nullptr, nullptr};
    hipEvent_t pin_free[2] = {nullptr, nullptr};  // the DMA that last used a staging buffer
    int copy_threads = 1;
    oz_blas_stats_t st{};
};

Ctx& ctx() {
    static Ctx c;
    return c;
}

[[noreturn]] void die(const char* what, const char* detail) {
    std::fprintf(stderr, "oz_blas: %s: %s\n", what, detail);
    std::fflush(stderr);
    std::abort();
}

void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) die(what, hipGetErrorString(e));
}

void configure(Ctx& c) {
    if (c.configured) return;
    c.configured = true;
    if (const char* m = std::getenv("OZ_COMPUTE_MODE")) {
        if (!parse_mode(m, &c.cfg)) die("OZ_COMPUTE_MODE is not a mode", m);
    }
    if (const char* z = std::getenv("OZ_ZMODE")) {
        const int v = std::atoi(z);
        if (v != 0 && v != 3 && v != 4) die("OZ_ZMODE must be 0, 3 or 4", z);
        c.cfg.zmode = v;
    }
    if (const char* d = std::getenv("OZ_DEVICE")) c.cfg.device = std::atoi(d);
}

void setup(Ctx& c) {
    if (c.ready) return;
    check_hip(hipSetDevice(c.cfg.device), "hipSetDevice");
    check_hip(hipStreamCreate(&c.stream), "hipStreamCreate");
    for (auto& e : c.ev) check_hip(hipEventCreate(&e), "hipEventCreate");
    int s = oz_create(&c.oz, c.cfg.device);
    if (s) die("oz_create", oz_status_string(s));
    s = oz_set_stream(c.oz, c.stream);
    if (s) die("oz_set_stream", oz_status_string(s));
    if (rocblas_create_handle(&c.rb) != rocblas_status_success) die("rocblas_create_handle", "failed");
    if (rocblas_set_stream(c.rb, c.stream) != rocblas_status_success) die("rocblas_set_stream", "failed");
    for (int b = 0; b < 2; ++b) {
        check_hip(hipHostMalloc(&c.pin[b], kStageBytes, hipHostMallocDefault), "hipHostMalloc");
        check_hip(hipEventCreateWithFlags(&c.pin_free[b], hipEventDisableTiming), "hipEventCreate");
        check_hip(hipEventRecord(c.pin_free[b], c.stream), "hipEventRecord");
    }
    const unsigned hw = std::thread::hardware_concurrency();
    c.copy_threads = static_cast<int>(std::max(1u, std::min(8u, hw / 2)));
    c.ready = true;
}

void teardown(Ctx& c) {
    if (!c.ready) return;
    check_hip(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    for (auto& b : c.buf) {
        if (b.p) check_hip(hipFree(b.p), "hipFree");
        b = DevBuf{};
    }
    for (int b = 0; b < 2; ++b) {
        check_hip(hipHostFree(c.pin[b]), "hipHostFree");
        check_hip(hipEventDestroy(c.pin_free[b]), "hipEventDestroy");
        c.pin[b] = nullptr;
    }
    rocblas_destroy_handle(c.rb);
    oz_destroy(c.oz);
    for (auto& e : c.ev) check_hip(hipEventDestroy(e), "hipEventDestroy");
    check_hip(hipStreamDestroy(c.stream), "hipStreamDestroy");
    c.rb = nullptr;
    c.oz = nullptr;
    c.stream = nullptr;
    c.ready = false;
}

void* reserve(DevBuf& b, size_t bytes) {
    if (bytes > b.cap) {
        if (b.p) check_hip(hipFree(b.p), "hipFree");
        b.p = nullptr;
        check_hip(hipMalloc(&b.p, bytes), "hipMalloc");
        b.cap = bytes;
    }
    return b.p;
}

// Copy `cols` columns of `colb` bytes between a strided and a packed layout
// (dst column j at dst + j * dld, src column j at src + j * sld), split over
// up to `threads` threads when large.
void copy_cols(char* dst, size_t dld, const char* src, size_t sld, size_t colb, int64_t cols, int threads) {
    auto run = [&](int64_t j0, int64_t j1) {
        if (dld == colb && sld == colb) {
            std::memcpy(dst + j0 * dld, src + j0 * sld, colb * (j1 - j0));
            return;
        }
        for (int64_t j = j0; j < j1; ++j) std::memcpy(dst + j * dld, src + j * sld, colb);
    };
    const size_t total = colb * static_cast<size_t>(cols);
    const int nt = total >= kThreadedBytes ? static_cast<int>(std::min<int64_t>(threads, cols)) : 1;
    if (nt <= 1) {
        run(0, cols);
        return;
    }
    std::vector<std::thread> pool;
    const int64_t per = (cols + nt - 1) / nt;
    for (int t = 1; t < nt; ++t) {
        const int64_t j0 = t * per, j1 = std::min(cols, j0 + per);
        if (j0 < j1) pool.emplace_back(run, j0, j1);
    }
    run(0, std::min(cols, per));
    for (auto& th : pool) th.join();
}

// Host (leading dimension ld) -> device (packed, leading dimension rows).
void to_device(Ctx& c, void* dst, const void* src, int64_t ld, int64_t rows, int64_t cols, size_t es) {
    const size_t colb = es * static_cast<size_t>(rows);
    if (colb > kStageBytes) {  // one column larger than a stage: the runtime copies it
        check_hip(hipMemcpy2DAsync(dst, colb, src, es * ld, colb, cols, hipMemcpyHostToDevice, c.stream), "copy in");
        return;
    }
    const int64_t per = static_cast<int64_t>(kStageBytes / colb);
    int b = 0;
    for (int64_t j0 = 0; j0 < cols; j0 += per, b ^= 1) {
        const int64_t nc = std::min(per, cols - j0);
        check_hip(hipEventSynchronize(c.pin_free[b]), "hipEventSynchronize");
        copy_cols(static_cast<char*>(c.pin[b]), colb, static_cast<const char*>(src) + j0 * es * ld, es * ld, colb, nc,
                  c.copy_threads);
        check_hip(hipMemcpyAsync(static_cast<char*>(dst) + j0 * colb, c.pin[b], colb * nc, hipMemcpyHostToDevice,
                                 c.stream),
                  "copy in");
        check_hip(hipEventRecord(c.pin_free[b], c.stream), "hipEventRecord");
    }
}

// Device (packed, leading dimension rows) -> host (leading dimension ld).
void to_host(Ctx& c, void* dst, int64_t ld, const void* src, int64_t rows, int64_t cols, size_t es) {
    const size_t colb = es * static_cast<size_t>(rows);
    if (colb > kStageBytes) {
        check_hip(hipMemcpy2DAsync(dst, es * ld, src, colb, colb, cols, hipMemcpyDeviceToHost, c.stream), "copy out");
        check_hip(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
        return;
    }
    const int64_t per = static_cast<int64_t>(kStageBytes / colb);
    const int64_t nchunks = (cols + per - 1) / per;
    auto issue = [&](int64_t i) {
        const int64_t j0 = i * per, nc = std::min(per, cols - j0);
        const int b = static_cast<int>(i & 1);
        check_hip(hipMemcpyAsync(c.pin[b], static_cast<const char*>(src) + j0 * colb, colb * nc,
                                 hipMemcpyDeviceToHost, c.stream),
                  "copy out");
        check_hip(hipEventRecord(c.pin_free[b], c.stream), "hipEventRecord");
    };
    issue(0);
    for (int64_t i = 0; i < nchunks; ++i) {
        if (i + 1 < nchunks) issue(i + 1);  // the other buffer was unpacked in the previous round
        const int b = static_cast<int>(i & 1);
        check_hip(hipEventSynchronize(c.pin_free[b]), "hipEventSynchronize");
        const int64_t j0 = i * per, nc = std::min(per, cols - j0);
        copy_cols(static_cast<char*>(dst) + j0 * es * ld, es * ld, static_cast<const char*>(c.pin[b]), colb, colb, nc,
                  c.copy_threads);
    }
}

// True when the GPU can use ptr directly (device or managed memory).
bool on_device(const void* ptr) {
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    const hipError_t e = hipPointerGetAttributes(&a, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // pageable host memory: clear the sticky error
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

char up(char c) { return static_cast<char>(std::toupper(static_cast<unsigned char>(c))); }
bool trans_ok(char c) { return c == 'N' || c == 'T' || c == 'C'; }

// The shared body of dgemm_ and zgemm_ (cplx: elements are (re, im) pairs).
void gemm(const char* name, int cplx, const char* transa, const char* transb, const int32_t* pm, const int32_t* pn,
          const int32_t* pk, const double* alpha, const double* A, const int32_t* plda, const double* B,
          const int32_t* pldb, const double* beta, double* C, const int32_t* pldc) {
    Ctx& c = ctx();
    std::lock_guard<std::mutex> lock(c.mu);
    configure(c);
    const char ta = up(*transa), tb = up(*transb);
    const int64_t m = *pm, n = *pn, k = *pk, lda = *plda, ldb = *pldb, ldc = *pldc;
    const int64_t rows_a = ta == 'N' ? m : k, cols_a = ta == 'N' ? k : m;
    const int64_t rows_b = tb == 'N' ? k : n, cols_b = tb == 'N' ? n : k;
    int info = 0;
    if (!trans_ok(ta)) info = 1;
    else if (!trans_ok(tb)) info = 2;
    else if (m < 0) info = 3;
    else if (n < 0) info = 4;
    else if (k < 0) info = 5;
    else if (lda < (rows_a > 1 ? rows_a : 1)) info = 8;
    else if (ldb < (rows_b > 1 ? rows_b : 1)) info = 10;
    else if (ldc < (m > 1 ? m : 1)) info = 13;
    c.st.last_info = info;
    if (info) {
        std::fprintf(stderr, " ** On entry to %s parameter number %2d had an illegal value\n", name, info);
        return;
    }
    const bool alpha_zero = alpha[0] == 0.0 && (!cplx || alpha[1] == 0.0);
    const bool beta_one = beta[0] == 1.0 && (!cplx || beta[1] == 0.0);
    const bool beta_zero = beta[0] == 0.0 && (!cplx || beta[1] == 0.0);
    if (m == 0 || n == 0 || ((alpha_zero || k == 0) && beta_one)) return;  // nothing changes

    setup(c);
    const size_t es = cplx ? 16 : 8;
    const bool use_a = !alpha_zero && k > 0;  // A and B are not read otherwise
    const bool host_a = use_a && !on_device(A), host_b = use_a && !on_device(B), host_c = !on_device(C);
    const double* dA = A;
    const double* dB = B;
    double* dC = C;
    int64_t la = lda, lb = ldb, lc = ldc;

    check_hip(hipEventRecord(c.ev[0], c.stream), "hipEventRecord");
    if (host_a) {
        dA = static_cast<const double*>(reserve(c.buf[0], es * rows_a * cols_a));
        la = rows_a;
        to_device(c, const_cast<double*>(dA), A, lda, rows_a, cols_a, es);
        c.st.bytes_to_device += static_cast<int64_t>(es * rows_a * cols_a);
    }
    if (host_b) {
        dB = static_cast<const double*>(reserve(c.buf[1], es * rows_b * cols_b));
        lb = rows_b;
        to_device(c, const_cast<double*>(dB), B, ldb, rows_b, cols_b, es);
        c.st.bytes_to_device += static_cast<int64_t>(es * rows_b * cols_b);
    }
    if (host_c) {
        dC = static_cast<double*>(reserve(c.buf[2], es * m * n));
        lc = m;
        if (!beta_zero) {  // with beta = 0 C is write-only
            to_device(c, dC, C, ldc, m, n, es);
            c.st.bytes_to_device += static_cast<int64_t>(es * m * n);
        }
    }
    check_hip(hipEventRecord(c.ev[1], c.stream), "hipEventRecord");

    if (c.cfg.mode == kNative) {
        auto op = [](char t) {
            return t == 'N' ? rocblas_operation_none
                            : (t == 'T' ? rocblas_operation_transpose : rocblas_operation_conjugate_transpose);
        };
        rocblas_status r;
        if (!cplx) {
            r = rocblas_dgemm(c.rb, op(ta), op(tb), static_cast<rocblas_int>(m), static_cast<rocblas_int>(n),
                              static_cast<rocblas_int>(k), alpha, dA, static_cast<rocblas_int>(la), dB,
                              static_cast<rocblas_int>(lb), beta, dC, static_cast<rocblas_int>(lc));
        } else {
            r = rocblas_zgemm(c.rb, op(ta), op(tb), static_cast<rocblas_int>(m), static_cast<rocblas_int>(n),
                              static_cast<rocblas_int>(k), reinterpret_cast<const rocblas_double_complex*>(alpha),
                              reinterpret_cast<const rocblas_double_complex*>(dA), static_cast<rocblas_int>(la),
                              reinterpret_cast<const rocblas_double_complex*>(dB), static_cast<rocblas_int>(lb),
                              reinterpret_cast<const rocblas_double_complex*>(beta),
                              reinterpret_cast<rocblas_double_complex*>(dC), static_cast<rocblas_int>(lc));
        }
        if (r != rocblas_status_success) die(cplx ? "rocblas_zgemm" : "rocblas_dgemm", rocblas_status_to_string(r));
    } else {
        oz_prec_t p;
        std::memset(&p, 0, sizeof(p));
        if (c.cfg.mode == kFixed || c.cfg.mode == kBalanced) {
            p.slices = c.cfg.slices;
            p.digits = c.cfg.mode == kBalanced ? 1 : 0;
        } else {
            p.slices = 0;
            p.tol = c.cfg.tol;
            p.smax = 12;
        }
        if (cplx) p.zmode = c.cfg.zmode;
        if (cplx && c.cfg.mode == kTol && p.zmode == 3) p.zmode = 4;  // tolerance-driven calls: 4-product form
        oz_report_t rep;
        const int s = cplx ? oz_zgemm(c.oz, ta, tb, m, n, k, alpha, dA, la, dB, lb, beta, dC, lc, &p, &rep)
                           : oz_dgemm(c.oz, ta, tb, m, n, k, alpha, dA, la, dB, lb, beta, dC, lc, &p, &rep);
        if (s) die(cplx ? "oz_zgemm" : "oz_dgemm", oz_status_string(s));
        c.st.last_slices = rep.slices_used;
    }
    check_hip(hipEventRecord(c.ev[2], c.stream), "hipEventRecord");
    if (host_c) {
        to_host(c, C, ldc, dC, m, n, es);
        c.st.bytes_to_host += static_cast<int64_t>(es * m * n);
    }
    check_hip(hipEventRecord(c.ev[3], c.stream), "hipEventRecord");
    check_hip(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    float t01 = 0.f, t12 = 0.f, t23 = 0.f;
    check_hip(hipEventElapsedTime(&t01, c.ev[0], c.ev[1]), "hipEventElapsedTime");
    check_hip(hipEventElapsedTime(&t12, c.ev[1], c.ev[2]), "hipEventElapsedTime");
    check_hip(hipEventElapsedTime(&t23, c.ev[2], c.ev[3]), "hipEventElapsedTime");
    c.st.copy_ms += t01 + t23;
    c.st.compute_ms += t12;
    c.st.calls += 1;
}

}  // namespace

extern "C" {

void dgemm_(const char* transa, const char* transb, const int32_t* m, const int32_t* n, const int32_t* k,
            const double* alpha, const double* A, const int32_t* lda, const double* B, const int32_t* ldb,
            const double* beta, double* C, const int32_t* ldc) {
    gemm("DGEMM ", 0, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

void zgemm_(const char* transa, const char* transb, const int32_t* m, const int32_t* n, const int32_t* k,
            const double* alpha, const double* A, const int32_t* lda, const double* B, const int32_t* ldb,
            const double* beta, double* C, const int32_t* ldc) {
    gemm("ZGEMM ", 1, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

int oz_blas_set_mode(const char* mode) {
    Ctx& c = ctx();
    std::lock_guard<std::mutex> lock(c.mu);
    configure(c);
    Config next = c.cfg;
    if (!parse_mode(mode, &next)) return -1;
    c.cfg = next;
    return 0;
}

void oz_blas_stats(oz_blas_stats_t* out) {
    Ctx& c = ctx();
    std::lock_guard<std::mutex> lock(c.mu);
    configure(c);
    if (!out) return;
    *out = c.st;
    out->mode = c.cfg.mode;
    out->slices = c.cfg.slices;
    out->tol = c.cfg.tol;
}

void oz_blas_finalize(void) {
    Ctx& c = ctx();
    std::lock_guard<std::mutex> lock(c.mu);
    teardown(c);
    const int32_t info = c.st.last_info;
    c.st = oz_blas_stats_t{};
    c.st.last_info = info;
}

}  // extern "C"
