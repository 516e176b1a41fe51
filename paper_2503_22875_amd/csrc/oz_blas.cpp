// oz_blas.cpp -- dgemm_ / zgemm_ with the Fortran BLAS calling convention,
// run on the GPU through the emulated path (or native FP64 for comparison).
// The offload layer of the method (paper Sec. 2.1 and 3.1): a program linked
// against this library gets its level-3 products from the GPU's INT8 units,
// with the arithmetic chosen per run by OZ_COMPUTE_MODE.  See oz_blas.h.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "oz.h"
#include "oz_blas.h"

namespace {

enum Mode { kNative = 0, kFixed = 1, kTol = 2 };

struct Config {
    int mode = kFixed;
    int slices = 7;
    double tol = 0.0;
    int zmode = 4;
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
    const std::string tol_prefix = "fp64_int8_tol", fix_prefix = "fp64_int8_";
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
        if (v != 3 && v != 4) die("OZ_ZMODE must be 3 or 4", z);
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
    c.ready = true;
}

void teardown(Ctx& c) {
    if (!c.ready) return;
    check_hip(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    for (auto& b : c.buf) {
        if (b.p) check_hip(hipFree(b.p), "hipFree");
        b = DevBuf{};
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
        check_hip(hipMemcpy2DAsync(const_cast<double*>(dA), es * rows_a, A, es * lda, es * rows_a, cols_a,
                                   hipMemcpyHostToDevice, c.stream),
                  "copy A");
        c.st.bytes_to_device += static_cast<int64_t>(es * rows_a * cols_a);
    }
    if (host_b) {
        dB = static_cast<const double*>(reserve(c.buf[1], es * rows_b * cols_b));
        lb = rows_b;
        check_hip(hipMemcpy2DAsync(const_cast<double*>(dB), es * rows_b, B, es * ldb, es * rows_b, cols_b,
                                   hipMemcpyHostToDevice, c.stream),
                  "copy B");
        c.st.bytes_to_device += static_cast<int64_t>(es * rows_b * cols_b);
    }
    if (host_c) {
        dC = static_cast<double*>(reserve(c.buf[2], es * m * n));
        lc = m;
        if (!beta_zero) {  // with beta = 0 C is write-only
            check_hip(hipMemcpy2DAsync(dC, es * m, C, es * ldc, es * m, n, hipMemcpyHostToDevice, c.stream),
                      "copy C");
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
        if (c.cfg.mode == kFixed) {
            p.slices = c.cfg.slices;
        } else {
            p.slices = 0;
            p.tol = c.cfg.tol;
            p.smax = 12;
        }
        if (cplx) p.zmode = c.cfg.zmode;
        if (cplx && c.cfg.mode == kTol) p.zmode = 4;  // tolerance-driven calls use the 4-product form
        oz_report_t rep;
        const int s = cplx ? oz_zgemm(c.oz, ta, tb, m, n, k, alpha, dA, la, dB, lb, beta, dC, lc, &p, &rep)
                           : oz_dgemm(c.oz, ta, tb, m, n, k, alpha, dA, la, dB, lb, beta, dC, lc, &p, &rep);
        if (s) die(cplx ? "oz_zgemm" : "oz_dgemm", oz_status_string(s));
        c.st.last_slices = rep.slices_used;
    }
    check_hip(hipEventRecord(c.ev[2], c.stream), "hipEventRecord");
    if (host_c) {
        check_hip(hipMemcpy2DAsync(C, es * ldc, dC, es * m, es * m, n, hipMemcpyDeviceToHost, c.stream), "copy C back");
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
