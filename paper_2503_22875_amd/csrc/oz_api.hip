// oz_api.hip -- the C ABI of include/oz.h: argument checks in reference-BLAS
// order, quick returns, the INT32 chunk plan, workspace, launch sequence.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/oz.h"
#include "oz_internal.h"

struct oz_handle_s {
    uint32_t magic;
    int device;
    hipStream_t stream;
    void* ws;
    size_t ws_bytes;
    bool ws_owned;
    // profiling: event triples (before split, before GEMM, after GEMM) per call
    bool timing;
    std::vector<hipEvent_t> ev_pool;
    std::vector<hipEvent_t> ev_pending;
};

namespace {

constexpr uint32_t kMagic = 0x6f7a3335u;  // "oz35"
constexpr int kDefaultSlices = 7;

bool valid(oz_handle_t h) { return h != nullptr && h->magic == kMagic; }

char up(char c) { return (c >= 'a' && c <= 'z') ? static_cast<char>(c - 'a' + 'A') : c; }
bool trans_ok(char c) {
    c = up(c);
    return c == 'N' || c == 'T' || c == 'C';
}

int use_device(oz_handle_t h) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return OZ_ERR_HIP;
    if (cur != h->device && hipSetDevice(h->device) != hipSuccess) return OZ_ERR_HIP;
    return OZ_OK;
}

// Largest multiple of 64 with s * kc * 127^2 <= 2^31 - 1: the INT32 sum of one
// anti-diagonal (at most s pair products per term, each |.| <= 127^2) over kc
// terms cannot overflow.
int64_t kchunk_bound(int s) {
    int64_t kc = static_cast<int64_t>(INT32_MAX) / (static_cast<int64_t>(s) * 127 * 127);
    return kc - kc % 64;
}

// Workspace carve-up for one GEMM call.
struct Plan {
    oz::SliceLayout la, lb;
    int64_t nva, nvb;
    size_t off_maxa, off_maxb, off_ea, off_fb, off_sa, off_sb, total;
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

Plan make_plan(int cplx, int64_t m, int64_t n, int64_t k, int s) {
    Plan p;
    p.nva = m;
    p.nvb = n;
    p.la = oz::slice_layout(1, cplx, m, k, s);
    p.lb = oz::slice_layout(0, cplx, n, k, s);
    size_t o = 0;
    p.off_maxa = o; o = align256(o + sizeof(uint64_t) * static_cast<size_t>(m));
    p.off_maxb = o; o = align256(o + sizeof(uint64_t) * static_cast<size_t>(n));
    p.off_ea = o;   o = align256(o + sizeof(int32_t) * static_cast<size_t>(m));
    p.off_fb = o;   o = align256(o + sizeof(int32_t) * static_cast<size_t>(p.lb.rows_pad));
    p.off_sa = o;   o = align256(o + static_cast<size_t>(s) * p.la.rows_pad * p.la.kpad);
    p.off_sb = o;   o = align256(o + static_cast<size_t>(s) * p.lb.rows_pad * p.lb.kpad);
    p.total = o;
    return p;
}

int ensure_ws(oz_handle_t h, size_t bytes) {
    if (bytes <= h->ws_bytes) return OZ_OK;
    if (!h->ws_owned) return OZ_ERR_ALLOC;
    if (h->ws) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) return OZ_ERR_HIP;
        hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return OZ_ERR_ALLOC;
    h->ws = p;
    h->ws_bytes = bytes;
    return OZ_OK;
}

// op(A) rows as vectors: 'N' -> A[i + l*lda]; 'T'/'C' -> A[l + i*lda]
oz::OperandView view_a(char ta, const double* A, int64_t lda, int64_t m, int64_t k, int cplx) {
    oz::OperandView v;
    v.X = A;
    const bool t = up(ta) != 'N';
    v.sv = t ? lda : 1;
    v.sl = t ? 1 : lda;
    v.nv = m;
    v.k = k;
    v.cplx = cplx;
    v.conj = cplx && up(ta) == 'C';
    v.side_a = 1;
    return v;
}

// op(B) columns as vectors: 'N' -> B[l + j*ldb]; 'T'/'C' -> B[j + l*ldb]
oz::OperandView view_b(char tb, const double* B, int64_t ldb, int64_t n, int64_t k, int cplx) {
    oz::OperandView v;
    v.X = B;
    const bool t = up(tb) != 'N';
    v.sv = t ? 1 : ldb;
    v.sl = t ? ldb : 1;
    v.nv = n;
    v.k = k;
    v.cplx = cplx;
    v.conj = cplx && up(tb) == 'C';
    v.side_a = 0;
    return v;
}

int hip_status(hipError_t e) { return e == hipSuccess ? OZ_OK : OZ_ERR_HIP; }

// Record a timing event on the handle's stream (no-op unless timing is on).
hipError_t mark(oz_handle_t h) {
    if (!h->timing) return hipSuccess;
    hipEvent_t ev;
    if (!h->ev_pool.empty()) {
        ev = h->ev_pool.back();
        h->ev_pool.pop_back();
    } else {
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return e;
    }
    h->ev_pending.push_back(ev);
    return hipEventRecord(ev, h->stream);
}

bool grid_fits(const Plan& p) {
    // split grids run 64 vectors per block along grid.y (at most 65535)
    return p.la.rows_pad / 64 <= 65535 && p.lb.rows_pad / 64 <= 65535;
}

int gemm_common(oz_handle_t h, int cplx, char transa, char transb, int64_t m, int64_t n, int64_t k,
                const double* alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                const double* beta, double* C, int64_t ldc, const oz_prec_t* prec, oz_report_t* rep) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    if (!trans_ok(transa)) return 1;
    if (!trans_ok(transb)) return 2;
    if (m < 0) return 3;
    if (n < 0) return 4;
    if (k < 0) return 5;
    const int64_t rows_a = up(transa) == 'N' ? m : k;
    const int64_t rows_b = up(transb) == 'N' ? k : n;
    if (lda < (rows_a > 1 ? rows_a : 1)) return 8;
    if (ldb < (rows_b > 1 ? rows_b : 1)) return 10;
    if (ldc < (m > 1 ? m : 1)) return 13;
    int s = kDefaultSlices;
    int64_t kc = 0;
    int kernel = 0;
    if (prec) {
        if (prec->slices < 0 || prec->slices > OZ_MAX_SLICES) return 14;
        if (prec->slices == 0) return OZ_ERR_UNSUPPORTED;  // tolerance-driven selection: not in this build
        if (prec->zmode != 0 && prec->zmode != 4) return 14;
        if (prec->kernel < 0 || prec->kernel > 3) return 14;
        s = prec->slices;
        kc = prec->kchunk;
        kernel = prec->kernel;
    }
    if (s > oz::kMaxLiveSlices && (kernel == 1 || kernel == 2)) return 14;
    if (kc < 0 || kc % 64 != 0 || (kc > 0 && kc > kchunk_bound(s))) return 14;
    if (kc == 0) kc = kchunk_bound(s);
    if (!alpha || !beta) return OZ_ERR_ARG;

    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->slices_used = s;
        rep->zmode_used = cplx ? 4 : 0;
    }
    int st = use_device(h);
    if (st) return st;
    if (m == 0 || n == 0) return OZ_OK;

    const double ar = alpha[0], ai = cplx ? alpha[1] : 0.0;
    const double br = beta[0], bi = cplx ? beta[1] : 0.0;
    const bool alpha_zero = ar == 0.0 && ai == 0.0;
    const bool beta_zero = br == 0.0 && bi == 0.0;
    const bool beta_one = br == 1.0 && bi == 0.0;
    if (alpha_zero || k == 0) {
        if (beta_one) return OZ_OK;
        st = hip_status(oz::launch_scale_c(C, ldc, m, n, cplx, br, bi, beta_zero, h->stream));
        if (st == OZ_OK && rep && hipStreamSynchronize(h->stream) != hipSuccess) st = OZ_ERR_HIP;
        return st;
    }

    Plan p = make_plan(cplx, m, n, k, s);
    if (!grid_fits(p)) return OZ_ERR_UNSUPPORTED;
    st = ensure_ws(h, p.total);
    if (st) return st;
    char* ws = static_cast<char*>(h->ws);
    uint64_t* maxa = reinterpret_cast<uint64_t*>(ws + p.off_maxa);
    uint64_t* maxb = reinterpret_cast<uint64_t*>(ws + p.off_maxb);
    int32_t* EA = reinterpret_cast<int32_t*>(ws + p.off_ea);
    int32_t* FB = reinterpret_cast<int32_t*>(ws + p.off_fb);
    int8_t* SA = reinterpret_cast<int8_t*>(ws + p.off_sa);
    int8_t* SB = reinterpret_cast<int8_t*>(ws + p.off_sb);

    oz::OperandView va = view_a(transa, A, lda, m, k, cplx);
    oz::OperandView vb = view_b(transb, B, ldb, n, k, cplx);
    hipError_t e = mark(h);
    if (e == hipSuccess) e = oz::launch_zero_u64(maxa, static_cast<int64_t>((p.off_ea - p.off_maxa) / 8), h->stream);
    if (e == hipSuccess) e = oz::launch_scan(va, maxa, h->stream);
    if (e == hipSuccess) e = oz::launch_scan(vb, maxb, h->stream);
    if (e == hipSuccess) e = oz::launch_digits(va, maxa, p.la, EA, SA, h->stream);
    if (e == hipSuccess) e = oz::launch_digits(vb, maxb, p.lb, FB, SB, h->stream);
    if (e != hipSuccess) return OZ_ERR_HIP;

    oz::GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.SA = SA;
    g.SB = SB;
    g.EA = EA;
    g.FB = FB;
    g.Mp = p.la.rows_pad;
    g.Np = p.lb.rows_pad;
    g.kpad = p.la.kpad;
    g.chunk_steps = kc / oz::kStep;
    g.s = s;
    g.cplx = cplx;
    g.tile = kernel;
    g.C = C;
    g.ldc = ldc;
    g.m = m;
    g.n = n;
    g.alpha_r = ar;
    g.alpha_i = ai;
    g.beta_r = br;
    g.beta_i = bi;
    g.beta_zero = beta_zero ? 1 : 0;
    g.diag_out = nullptr;
    e = mark(h);
    if (e == hipSuccess) e = oz::launch_gemm(g, h->stream);
    if (e == hipSuccess) e = mark(h);
    if (e != hipSuccess) return OZ_ERR_HIP;

    if (rep) {
        rep->kchunks = static_cast<int32_t>((p.la.kpad + kc - 1) / kc);
        if (hipStreamSynchronize(h->stream) != hipSuccess) return OZ_ERR_HIP;
        std::vector<int32_t> ea(static_cast<size_t>(m)), fb(static_cast<size_t>(n));
        if (hipMemcpy(ea.data(), EA, sizeof(int32_t) * m, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(fb.data(), FB, sizeof(int32_t) * n, hipMemcpyDeviceToHost) != hipSuccess)
            return OZ_ERR_HIP;
        for (int32_t x : ea)
            if (x == oz::kNonFiniteExp) rep->status = OZ_ERR_NONFINITE;
        for (int32_t x : fb)
            if (x == oz::kNonFiniteExp) rep->status = OZ_ERR_NONFINITE;
    }
    return OZ_OK;
}

}  // namespace

extern "C" {

int oz_create(oz_handle_t* handle, int device) {
    if (!handle) return OZ_ERR_ARG;
    *handle = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return OZ_ERR_UNSUPPORTED;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return OZ_ERR_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return OZ_ERR_UNSUPPORTED;
    if (hipSetDevice(device) != hipSuccess) return OZ_ERR_HIP;
    oz_handle_s* h = new (std::nothrow) oz_handle_s;
    if (!h) return OZ_ERR_ALLOC;
    h->magic = kMagic;
    h->device = device;
    h->stream = nullptr;
    h->ws = nullptr;
    h->ws_bytes = 0;
    h->ws_owned = true;
    h->timing = false;
    *handle = h;
    return OZ_OK;
}

int oz_destroy(oz_handle_t h) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    use_device(h);
    hipStreamSynchronize(h->stream);
    if (h->ws_owned && h->ws) hipFree(h->ws);
    for (hipEvent_t ev : h->ev_pool) hipEventDestroy(ev);
    for (hipEvent_t ev : h->ev_pending) hipEventDestroy(ev);
    h->magic = 0;
    delete h;
    return OZ_OK;
}

int oz_timing_enable(oz_handle_t h, int enable) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    h->timing = enable != 0;
    return OZ_OK;
}

int oz_timing_read(oz_handle_t h, double* split_ms, double* gemm_ms, int64_t* calls) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    if (use_device(h)) return OZ_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return OZ_ERR_HIP;
    double ts = 0.0, tg = 0.0;
    const size_t n = h->ev_pending.size() / 3;
    int st = OZ_OK;
    for (size_t c = 0; c < n; ++c) {
        float a = 0.f, b = 0.f;
        hipEvent_t* e = &h->ev_pending[3 * c];
        if (hipEventElapsedTime(&a, e[0], e[1]) != hipSuccess || hipEventElapsedTime(&b, e[1], e[2]) != hipSuccess)
            st = OZ_ERR_HIP;
        ts += a;
        tg += b;
    }
    for (hipEvent_t ev : h->ev_pending) h->ev_pool.push_back(ev);
    h->ev_pending.clear();
    if (split_ms) *split_ms = ts;
    if (gemm_ms) *gemm_ms = tg;
    if (calls) *calls = static_cast<int64_t>(n);
    return st;
}

int oz_set_stream(oz_handle_t h, void* stream) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    h->stream = static_cast<hipStream_t>(stream);
    return OZ_OK;
}

const char* oz_status_string(int status) {
    switch (status) {
        case OZ_OK: return "success";
        case OZ_ERR_HIP: return "HIP runtime error";
        case OZ_ERR_ALLOC: return "device workspace allocation failed or too small";
        case OZ_ERR_NONFINITE: return "input holds Inf or NaN";
        case OZ_ERR_HANDLE: return "invalid handle";
        case OZ_ERR_UNSUPPORTED: return "unsupported device, size or mode";
        case OZ_ERR_ARG: return "invalid argument";
        default: return status > 0 ? "invalid BLAS argument (position = status)" : "unknown status";
    }
}

int oz_workspace_size(oz_handle_t h, char transa, char transb, int64_t m, int64_t n, int64_t k, int is_complex,
                      const oz_prec_t* prec, size_t* bytes) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    if (!trans_ok(transa)) return 1;
    if (!trans_ok(transb)) return 2;
    if (m < 0) return 3;
    if (n < 0) return 4;
    if (k < 0) return 5;
    if (!bytes) return OZ_ERR_ARG;
    int s = prec ? prec->slices : kDefaultSlices;
    if (s < 1 || s > OZ_MAX_SLICES) return 14;
    *bytes = make_plan(is_complex ? 1 : 0, m, n, k, s).total;
    return OZ_OK;
}

int oz_set_workspace(oz_handle_t h, void* dptr, size_t bytes) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    if (use_device(h)) return OZ_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return OZ_ERR_HIP;
    if (h->ws_owned && h->ws) hipFree(h->ws);
    if (dptr) {
        h->ws = dptr;
        h->ws_bytes = bytes;
        h->ws_owned = false;
    } else {
        h->ws = nullptr;
        h->ws_bytes = 0;
        h->ws_owned = true;
    }
    return OZ_OK;
}

int oz_dgemm(oz_handle_t h, char transa, char transb, int64_t m, int64_t n, int64_t k, const double* alpha,
             const double* A, int64_t lda, const double* B, int64_t ldb, const double* beta, double* C, int64_t ldc,
             const oz_prec_t* prec, oz_report_t* rep) {
    return gemm_common(h, 0, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, prec, rep);
}

int oz_zgemm(oz_handle_t h, char transa, char transb, int64_t m, int64_t n, int64_t k, const double* alpha,
             const double* A, int64_t lda, const double* B, int64_t ldb, const double* beta, double* C, int64_t ldc,
             const oz_prec_t* prec, oz_report_t* rep) {
    return gemm_common(h, 1, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, prec, rep);
}

int oz_split_layout(char side, int is_complex, int64_t nv, int64_t k, int32_t slices, int64_t* rows_pad,
                    int64_t* kpad, size_t* slice_bytes) {
    if (up(side) != 'A' && up(side) != 'B') return OZ_ERR_ARG;
    if (nv < 0 || k < 0 || slices < 1 || slices > OZ_MAX_SLICES) return OZ_ERR_ARG;
    oz::SliceLayout L = oz::slice_layout(up(side) == 'A', is_complex ? 1 : 0, nv, k, slices);
    if (rows_pad) *rows_pad = L.rows_pad;
    if (kpad) *kpad = L.kpad;
    if (slice_bytes) *slice_bytes = static_cast<size_t>(slices) * L.rows_pad * L.kpad;
    return OZ_OK;
}

int oz_split(oz_handle_t h, char side, char trans, int is_complex, int64_t nv, int64_t k, const double* X,
             int64_t ldx, int32_t slices, int32_t* E, int8_t* slices_out) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    const bool sa = up(side) == 'A';
    if (!sa && up(side) != 'B') return OZ_ERR_ARG;
    if (!trans_ok(trans) || nv < 0 || k < 0 || slices < 1 || slices > OZ_MAX_SLICES) return OZ_ERR_ARG;
    const bool t = up(trans) != 'N';
    // stored rows of X: side A 'N' -> nv, 'T' -> k; side B 'N' -> k, 'T' -> nv
    const int64_t rows = sa ? (t ? k : nv) : (t ? nv : k);
    if (ldx < (rows > 1 ? rows : 1)) return OZ_ERR_ARG;
    if (use_device(h)) return OZ_ERR_HIP;
    const int cplx = is_complex ? 1 : 0;
    oz::OperandView v = sa ? view_a(trans, X, ldx, nv, k, cplx) : view_b(trans, X, ldx, nv, k, cplx);
    oz::SliceLayout L = oz::slice_layout(sa, cplx, nv, k, slices);
    if (L.rows_pad / 64 > 65535) return OZ_ERR_UNSUPPORTED;
    int st = ensure_ws(h, align256(sizeof(uint64_t) * static_cast<size_t>(nv > 0 ? nv : 1)));
    if (st) return st;
    uint64_t* mx = static_cast<uint64_t*>(h->ws);
    hipError_t e = oz::launch_zero_u64(mx, nv, h->stream);
    if (e == hipSuccess) e = oz::launch_scan(v, mx, h->stream);
    if (e == hipSuccess) e = oz::launch_digits(v, mx, L, E, slices_out, h->stream);
    return hip_status(e);
}

int oz_diag_sums(oz_handle_t h, int32_t slices, int64_t kchunk, int32_t kernel, int64_t rows_pad_a,
                 int64_t rows_pad_b, int64_t kpad, const int8_t* slices_a, const int8_t* slices_b, int32_t* out) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    if (slices < 1 || slices > OZ_MAX_SLICES) return OZ_ERR_ARG;
    if (kernel < 0 || kernel > 3 || (slices > oz::kMaxLiveSlices && (kernel == 1 || kernel == 2))) return OZ_ERR_ARG;
    if (kchunk <= 0 || kchunk % 64 != 0 || kchunk > kchunk_bound(slices)) return OZ_ERR_ARG;
    if (rows_pad_a <= 0 || rows_pad_b <= 0 || rows_pad_a % oz::kRowPad || rows_pad_b % oz::kRowPad) return OZ_ERR_ARG;
    if (kpad <= 0 || kpad % oz::kStep) return OZ_ERR_ARG;
    if (use_device(h)) return OZ_ERR_HIP;
    oz::GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.SA = slices_a;
    g.SB = slices_b;
    g.Mp = rows_pad_a;
    g.Np = rows_pad_b;
    g.kpad = kpad;
    g.chunk_steps = kchunk / oz::kStep;
    g.s = slices;
    g.tile = kernel;
    g.diag_out = out;
    return hip_status(oz::launch_gemm(g, h->stream));
}

}  // extern "C"
