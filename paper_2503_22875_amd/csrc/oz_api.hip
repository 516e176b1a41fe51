// oz_api.hip -- the C ABI of include/oz.h: argument checks in reference-BLAS
// order, quick returns, the INT32 chunk plan, workspace, launch sequence.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <new>
#include <vector>

#include "../../include/oz.h"
#include "oz_handle.h"
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
    // batched plans: autotuner results (oz_load_tuning)
    std::vector<oz::TuneEntry> tune;
    // learned slice-count selector (oz_set_selector), not owned
    oz_mlp_t selector;
    // LU factorisation / inverse: the look-ahead stream and its events, and a
    // grow-only device buffer apart from the GEMM workspace (created on first use)
    hipStream_t lu_stream;
    hipEvent_t lu_ev[3];
    void* lu_ws;
    size_t lu_ws_bytes;
};

// Device scratch of the allocation-free entry point oz_gemm_noalloc: every
// workspace buffer of one fixed-s call (scale scratch, exponents, slices, the
// 3-product form's T1 / T2) is carved from it.  Each GPU the library runs on
// holds its own copy for the life of the process.  Host code never uses the
// name `scratch` as an address: its device address is looked up once per
// device (scratch_setup) and kept in g_scratch_ptr.
constexpr size_t kNoAllocScratchBytes = OZ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices];

// Device address of `scratch` on `device`, which must be the current device;
// looked up on the first call per device.
int scratch_setup(int device, char** out) {
    if (device < 0 || device >= kMaxScratchDevices) return OZ_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return OZ_ERR_HIP;
        g_scratch_ptr[device] = p;
    }
    if (out) *out = static_cast<char*>(g_scratch_ptr[device]);
    return OZ_OK;
}

constexpr uint32_t kMagic = 0x6f7a3335u;  // "oz35"
constexpr int kDefaultSlices = 7;
constexpr int kDefaultSmax = 12;
constexpr uint64_t kProbeSeed = 0x6f7a5eedull;

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
// terms cannot overflow.  Balanced digits reach -128: 128^2 per product.
int64_t kchunk_bound(int s, bool bal = false) {
    const int64_t dmax = bal ? 128 : 127;
    int64_t kc = static_cast<int64_t>(INT32_MAX) / (static_cast<int64_t>(s) * dmax * dmax);
    return kc - kc % 64;
}

constexpr int kMaxBalancedSlices = 8;  // balanced digits: N below 2^62 in one int64

// Workspace carve-up for one GEMM call (s_lay digit planes; the tol buffers
// only when a tolerance-driven call needs them).
struct Plan {
    oz::SliceLayout la, lb;
    int64_t nva, nvb;
    size_t off_maxa, off_maxb, off_ea, off_fb, off_sa, off_sb;
    size_t off_acc, off_msa, off_msb, off_t, off_u, off_diff, off_ref, off_norms, off_sel, off_part1, off_part2,
        total;
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

Plan make_plan(int cplx, int64_t m, int64_t n, int64_t k, int s_lay, bool tol_bufs) {
    Plan p;
    p.nva = m;
    p.nvb = n;
    p.la = oz::slice_layout(1, cplx, m, k, s_lay);
    p.lb = oz::slice_layout(0, cplx, n, k, s_lay);
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    p.off_maxa = take(sizeof(uint64_t) * static_cast<size_t>(m));
    p.off_maxb = take(sizeof(uint64_t) * static_cast<size_t>(n));
    p.off_ea = take(sizeof(int32_t) * static_cast<size_t>(m));
    p.off_fb = take(sizeof(int32_t) * static_cast<size_t>(p.lb.rows_pad));
    p.off_sa = take(static_cast<size_t>(s_lay) * p.la.rows_pad * p.la.kpad);
    p.off_sb = take(static_cast<size_t>(s_lay) * p.lb.rows_pad * p.lb.kpad);
    p.off_acc = p.off_msa = p.off_msb = p.off_t = p.off_u = p.off_diff = p.off_ref = p.off_norms = p.off_sel = 0;
    p.off_part1 = p.off_part2 = 0;
    if (tol_bufs) {
        p.off_acc = take(sizeof(double) * static_cast<size_t>(p.la.rows_pad) * p.lb.rows_pad);
        p.off_msa = take(sizeof(double) * static_cast<size_t>(m));
        p.off_msb = take(sizeof(double) * static_cast<size_t>(n));
        p.off_t = take(sizeof(double) * static_cast<size_t>(n));
        p.off_u = take(sizeof(double) * 4 * static_cast<size_t>(k));
        p.off_diff = take(sizeof(double) * 2 * static_cast<size_t>(m));
        p.off_ref = take(sizeof(double) * 2 * static_cast<size_t>(m));
        p.off_norms = take(sizeof(double) * 2);
        p.off_sel = take(oz_learned_scratch_bytes());
        p.off_part1 = take(oz::check_part_bytes(m, n, k));
        p.off_part2 = take(oz::check_part_bytes(m, n, k));
    }
    p.total = o;
    return p;
}

// Workspace of a complex product in the 3-real-product form: per real operand
// (parts 1: real, 2: imaginary, 3: their sum) the scale scratch, exponents and
// slices of A and B (s_lay digit planes), then the real products T1, T2
// (m x n) of a fixed-s call, or for a tolerance-driven call the raw sums of
// T1, T2, T3, the complex operands' own maxima and the check and statistics
// buffers.
struct Plan3 {
    oz::SliceLayout la, lb;
    size_t off_max, off_ea[3], off_fb[3], off_sa[3], off_sb[3], off_t1, off_t2, total;
    size_t off_acc[3], off_maxc, off_msa, off_msb, off_t, off_u, off_diff, off_ref, off_norms, off_sel, off_part1,
        off_part2;
    int64_t nmax;
};

Plan3 make_plan3(int64_t m, int64_t n, int64_t k, int s, bool tol_bufs = false) {
    Plan3 p;
    p.la = oz::slice_layout(1, 0, m, k, s);
    p.lb = oz::slice_layout(0, 0, n, k, s);
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    p.nmax = 3 * (m + n);
    p.off_max = take(sizeof(uint64_t) * static_cast<size_t>(p.nmax));
    for (int q = 0; q < 3; ++q) {
        p.off_ea[q] = take(sizeof(int32_t) * static_cast<size_t>(m));
        p.off_fb[q] = take(sizeof(int32_t) * static_cast<size_t>(p.lb.rows_pad));
        p.off_sa[q] = take(static_cast<size_t>(s) * p.la.rows_pad * p.la.kpad);
        p.off_sb[q] = take(static_cast<size_t>(s) * p.lb.rows_pad * p.lb.kpad);
    }
    p.off_t1 = p.off_t2 = 0;
    for (int q = 0; q < 3; ++q) p.off_acc[q] = 0;
    p.off_maxc = p.off_msa = p.off_msb = p.off_t = p.off_u = p.off_diff = p.off_ref = p.off_norms = p.off_sel = 0;
    p.off_part1 = p.off_part2 = 0;
    if (!tol_bufs) {
        p.off_t1 = take(sizeof(double) * static_cast<size_t>(m) * n);
        p.off_t2 = take(sizeof(double) * static_cast<size_t>(m) * n);
    } else {
        for (int q = 0; q < 3; ++q)
            p.off_acc[q] = take(sizeof(double) * static_cast<size_t>(p.la.rows_pad) * p.lb.rows_pad);
        p.off_maxc = take(sizeof(uint64_t) * static_cast<size_t>(m + n));
        p.off_msa = take(sizeof(double) * static_cast<size_t>(m));
        p.off_msb = take(sizeof(double) * static_cast<size_t>(n));
        p.off_t = take(sizeof(double) * static_cast<size_t>(n));
        p.off_u = take(sizeof(double) * 4 * static_cast<size_t>(k));
        p.off_diff = take(sizeof(double) * 2 * static_cast<size_t>(m));
        p.off_ref = take(sizeof(double) * 2 * static_cast<size_t>(m));
        p.off_norms = take(sizeof(double) * 2);
        p.off_sel = take(oz_learned_scratch_bytes());
        p.off_part1 = take(oz::check_part_bytes(m, n, k));
        p.off_part2 = take(oz::check_part_bytes(m, n, k));
    }
    p.total = o;
    return p;
}

// A caller-fixed workspace (the allocation-free entry point's scratch), or
// none: the handle's own.
struct FixedWs {
    char* ptr = nullptr;
    size_t bytes = 0;
};

int ensure_ws(oz_handle_t h, size_t bytes);

// Workspace of `bytes` for one call: the fixed buffer when given (too small:
// OZ_ERR_ALLOC, nothing allocated), else the handle's.
int take_ws(oz_handle_t h, const FixedWs& fixed, size_t bytes, char** ws) {
    if (fixed.ptr) {
        if (bytes > fixed.bytes) return OZ_ERR_ALLOC;
        *ws = fixed.ptr;
        return OZ_OK;
    }
    const int st = ensure_ws(h, bytes);
    if (st) return st;
    *ws = static_cast<char*>(h->ws);
    return OZ_OK;
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

// Mean over vectors of the per-vector mean square of x * 2^-E (stats kernel).
int vector_msq(oz_handle_t h, const oz::OperandView& v, const uint64_t* mx, double* ms, double* part, double* mean) {
    if (oz::launch_vec_stats(v, mx, ms, part, h->stream) != hipSuccess) return OZ_ERR_HIP;
    std::vector<double> host(static_cast<size_t>(v.nv));
    if (v.nv > 0 && (hipMemcpyAsync(host.data(), ms, sizeof(double) * v.nv, hipMemcpyDeviceToHost, h->stream) !=
                         hipSuccess ||
                     hipStreamSynchronize(h->stream) != hipSuccess))
        return OZ_ERR_HIP;
    double sum = 0.0;
    for (double x : host) sum += x;
    *mean = v.nv > 0 ? sum / static_cast<double>(v.nv) : 0.0;
    return OZ_OK;
}

// Smallest s in [1, smax] whose rule estimate meets tol (smax if none does).
int rule_slices(oz_handle_t h, const oz::OperandView& va, const oz::OperandView& vb, const uint64_t* maxa,
                const uint64_t* maxb, double* msa, double* msb, double* part, double tol, int smax, int* s_out,
                bool bal = false) {
    double ma = 0.0, mb = 0.0;
    int st = vector_msq(h, va, maxa, msa, part, &ma);
    if (!st) st = vector_msq(h, vb, maxb, msb, part, &mb);
    if (st) return st;
    if (!(ma > 0.0) || !(mb > 0.0)) {  // a zero operand: every s is exact
        *s_out = 1;
        return OZ_OK;
    }
    *s_out = oz::rule_slices_of(ma, mb, tol, smax, bal);
    return OZ_OK;
}

// Complex product in the 3-real-product form (zmode 3): with op(A) = Ar + i Ai
// and op(B) = Br + i Bi, T1 = Ar Br, T2 = Ai Bi and T3 = (Ar + Ai)(Br + Bi)
// are three real emulated products (each with its own scales; the pre-added
// operands rounded once in FP64 as the split reads them); the last one's
// epilogue forms Cr = T1 - T2, Ci = (T3 - T1) - T2 and applies alpha, beta.
// Three quarters of the INT8 work of the 4-product form.
//
// Tolerance-driven (tp != nullptr, truncated digits): the starting s comes from
// the complex operands' statistics as for the 4-product form; the three
// products write raw FP64 sums; the residual check forms C from them with the
// combine's roundings; each growth step adds a digit plane to every part and
// the new top anti-diagonal to each product (T1, T2, T3 in turn); a last pass
// combines the sums into C.
struct Tol3 {
    double tol;
    int smax, sstart, selector;
};

int zgemm_3m(oz_handle_t h, char transa, char transb, int64_t m, int64_t n, int64_t k, const double* alpha,
             const double* A, int64_t lda, const double* B, int64_t ldb, const double* beta, double* C, int64_t ldc,
             int s, int64_t kc, int kernel, bool bal, oz_report_t* rep, const FixedWs& fixed,
             const Tol3* tp = nullptr) {
    const bool tol_mode = tp != nullptr;
    const int s_lay = tol_mode ? tp->smax : s;
    Plan3 p = make_plan3(m, n, k, s_lay, tol_mode);
    if (p.la.rows_pad / 64 > 65535 || p.lb.rows_pad / 64 > 65535) return OZ_ERR_UNSUPPORTED;
    p.la.bal = p.lb.bal = bal ? 1 : 0;
    char* ws = nullptr;
    int st = take_ws(h, fixed, p.total, &ws);
    if (st) return st;
    uint64_t* mx = reinterpret_cast<uint64_t*>(ws + p.off_max);
    const double ar = alpha[0], ai = alpha[1], br = beta[0], bi = beta[1];
    const int beta_zero = (br == 0.0 && bi == 0.0) ? 1 : 0;
    // no timing events on the allocation-free path (events are created on demand)
    auto mark = [&](oz_handle_t hh) { return fixed.ptr ? hipSuccess : ::mark(hh); };
    hipError_t e = tol_mode ? hipSuccess : mark(h);
    if (e == hipSuccess) e = oz::launch_zero_u64(mx, p.nmax, h->stream);
    // the three real operands of each side (real parts, imaginary parts,
    // their sums) in one scan and one digit pass over the complex operand
    const oz::OperandView va = view_a(transa, A, lda, m, k, 1);
    const oz::OperandView vb = view_b(transb, B, ldb, n, k, 1);
    oz::Split3Out oa, ob;
    for (int q = 0; q < 3; ++q) {
        oa.maxbits[q] = mx + q * (m + n);
        ob.maxbits[q] = oa.maxbits[q] + m;
        oa.E[q] = reinterpret_cast<int32_t*>(ws + p.off_ea[q]);
        ob.E[q] = reinterpret_cast<int32_t*>(ws + p.off_fb[q]);
        oa.slices[q] = reinterpret_cast<int8_t*>(ws + p.off_sa[q]);
        ob.slices[q] = reinterpret_cast<int8_t*>(ws + p.off_sb[q]);
    }
    if (e == hipSuccess) e = oz::launch_scan3(va, oa, h->stream);
    if (e == hipSuccess) e = oz::launch_scan3(vb, ob, h->stream);
    oz::GemmArgs g3[3];
    for (int q = 0; q < 3; ++q) {
        oz::GemmArgs& g = g3[q];
        std::memset(&g, 0, sizeof(g));
        g.SA = reinterpret_cast<const int8_t*>(ws + p.off_sa[q]);
        g.SB = reinterpret_cast<const int8_t*>(ws + p.off_sb[q]);
        g.EA = reinterpret_cast<const int32_t*>(ws + p.off_ea[q]);
        g.FB = reinterpret_cast<const int32_t*>(ws + p.off_fb[q]);
        g.Mp = p.la.rows_pad;
        g.Np = p.lb.rows_pad;
        g.kpad = p.la.kpad;
        g.chunk_steps = kc / oz::kStep;
        g.s = s;
        g.s_lay = s_lay;
        g.tile = kernel;
        g.m = m;
        g.n = n;
        g.bal = bal ? 1 : 0;
    }
    int fallbacks = 0;
    double eps = 0.0;
    if (!tol_mode) {
        if (e == hipSuccess) e = oz::launch_digits3(va, p.la, oa, h->stream);
        if (e == hipSuccess) e = oz::launch_digits3(vb, p.lb, ob, h->stream);
        if (e == hipSuccess) e = mark(h);
        double* T[2] = {reinterpret_cast<double*>(ws + p.off_t1), reinterpret_cast<double*>(ws + p.off_t2)};
        for (int q = 0; q < 3 && e == hipSuccess; ++q) {
            oz::GemmArgs& g = g3[q];
            if (q < 2) {
                // T1, T2: plain FP64 results (alpha = 1, beta = 0: 1 * v is exact)
                g.mode = oz::kFinal;
                g.C = T[q];
                g.ldc = m;
                g.alpha_r = 1.0;
                g.beta_zero = 1;
            } else {
                g.mode = oz::kCombine3M;
                g.C = C;
                g.ldc = ldc;
                g.alpha_r = ar;
                g.alpha_i = ai;
                g.beta_r = br;
                g.beta_i = bi;
                g.beta_zero = beta_zero;
                g.t1 = T[0];
                g.t2 = T[1];
                g.ldt = m;
            }
            e = oz::launch_gemm(g, h->stream);
        }
        if (e == hipSuccess) e = mark(h);
        if (e != hipSuccess) return OZ_ERR_HIP;
    } else {
        if (e != hipSuccess) return OZ_ERR_HIP;
        // (1) starting s from the complex operands' statistics (their own
        // maxima), for the checked target
        uint64_t* maxa = reinterpret_cast<uint64_t*>(ws + p.off_maxc);
        uint64_t* maxb = maxa + m;
        double* msa = reinterpret_cast<double*>(ws + p.off_msa);
        double* msb = reinterpret_cast<double*>(ws + p.off_msb);
        const double tol_eff = tp->tol / oz::kCheckMargin;
        const int smax = tp->smax;
        if (oz::launch_zero_u64(maxa, m + n, h->stream) != hipSuccess ||
            oz::launch_scan(va, maxa, h->stream) != hipSuccess || oz::launch_scan(vb, maxb, h->stream) != hipSuccess)
            return OZ_ERR_HIP;
        if (tp->sstart > 0) {
            s = tp->sstart;
        } else if (tp->selector == 1) {
            st = oz_learned_start(h, h->selector, va, vb, maxa, maxb, msa, msb, m, n, k, 1, tol_eff, smax,
                                  ws + p.off_sel, &s);
            if (st) return st;
        } else {
            st = rule_slices(h, va, vb, maxa, maxb, msa, msb, reinterpret_cast<double*>(ws + p.off_part1), tol_eff,
                             smax, &s);
            if (st) return st;
        }
        if (s > smax) s = smax;
        // (2) digit planes 1..s of every part, raw sums of T1, T2, T3 at s
        if (oz::launch_digits3(va, p.la, oa, h->stream, 0, s) != hipSuccess ||
            oz::launch_digits3(vb, p.lb, ob, h->stream, 0, s) != hipSuccess)
            return OZ_ERR_HIP;
        for (int q = 0; q < 3; ++q) {
            g3[q].acc = reinterpret_cast<double*>(ws + p.off_acc[q]);
            g3[q].s = s;
            g3[q].mode = oz::kRawWrite;
            if (oz::launch_gemm(g3[q], h->stream) != hipSuccess) return OZ_ERR_HIP;
        }
        // (3) check; grow until it passes
        oz::CheckArgs c;
        std::memset(&c, 0, sizeof(c));
        c.opa = va;
        c.opb = vb;
        c.maxa = maxa;
        c.maxb = maxb;
        c.Mp = p.la.rows_pad;
        c.seed = kProbeSeed;
        c.t = reinterpret_cast<double*>(ws + p.off_t);
        c.u = reinterpret_cast<double*>(ws + p.off_u);
        c.diff = reinterpret_cast<double*>(ws + p.off_diff);
        c.ref = reinterpret_cast<double*>(ws + p.off_ref);
        c.norms = reinterpret_cast<double*>(ws + p.off_norms);
        c.part1 = reinterpret_cast<double*>(ws + p.off_part1);
        c.part2 = reinterpret_cast<double*>(ws + p.off_part2);
        c.z3 = 1;
        for (int q = 0; q < 3; ++q) {
            c.acc3[q] = g3[q].acc;
            c.EA3[q] = g3[q].EA;
            c.FB3[q] = g3[q].FB;
        }
        for (;;) {
            if (oz::launch_residual(c, h->stream) != hipSuccess) return OZ_ERR_HIP;
            double nrm[2];
            if (hipMemcpyAsync(nrm, c.norms, sizeof(nrm), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
                hipStreamSynchronize(h->stream) != hipSuccess)
                return OZ_ERR_HIP;
            eps = nrm[1] > 0.0 ? std::sqrt(nrm[0] / nrm[1]) : std::sqrt(nrm[0]);
            if (!(eps > tol_eff) || s >= smax) break;  // NaN (non-finite input) also stops
            int add = static_cast<int>(std::ceil(std::log2(eps / tol_eff) / 6.0));
            add = add < 1 ? 1 : (add > smax - s ? smax - s : add);
            // digit planes s + 1 .. s + add of every part, then the
            // anti-diagonals s + 2 .. s + add + 1 of each product, one at a time
            if (oz::launch_digits3(va, p.la, oa, h->stream, s, s + add) != hipSuccess ||
                oz::launch_digits3(vb, p.lb, ob, h->stream, s, s + add) != hipSuccess)
                return OZ_ERR_HIP;
            for (int j = 0; j < add; ++j) {
                for (int q = 0; q < 3; ++q) {
                    g3[q].s = s + 1;
                    g3[q].top = 1;
                    g3[q].mode = oz::kRawAdd;
                    if (oz::launch_gemm(g3[q], h->stream) != hipSuccess) return OZ_ERR_HIP;
                    g3[q].top = 0;
                }
                ++s;
                ++fallbacks;
            }
        }
        // (4) C = alpha ((T1 - T2) + i ((T3 - T1) - T2)) + beta C
        const double* acc3[3] = {g3[0].acc, g3[1].acc, g3[2].acc};
        const int32_t* ea3[3] = {g3[0].EA, g3[1].EA, g3[2].EA};
        const int32_t* fb3[3] = {g3[0].FB, g3[1].FB, g3[2].FB};
        if (oz::launch_finalize3(acc3, p.la.rows_pad, ea3, fb3, C, ldc, m, n, ar, ai, br, bi, beta_zero,
                                 h->stream) != hipSuccess)
            return OZ_ERR_HIP;
    }
    if (rep) {
        rep->slices_used = s;
        rep->fallbacks = fallbacks;
        rep->resid_est = eps;
        rep->zmode_used = 3;
        rep->kchunks = static_cast<int32_t>((p.la.kpad + kc - 1) / kc);
        if (hipStreamSynchronize(h->stream) != hipSuccess) return OZ_ERR_HIP;
        std::vector<int32_t> ex(static_cast<size_t>(m > n ? m : n));
        for (int q = 0; q < 3; ++q) {
            if (hipMemcpy(ex.data(), ws + p.off_ea[q], sizeof(int32_t) * m, hipMemcpyDeviceToHost) != hipSuccess)
                return OZ_ERR_HIP;
            for (int64_t i = 0; i < m; ++i)
                if (ex[i] == oz::kNonFiniteExp) rep->status = OZ_ERR_NONFINITE;
            if (hipMemcpy(ex.data(), ws + p.off_fb[q], sizeof(int32_t) * n, hipMemcpyDeviceToHost) != hipSuccess)
                return OZ_ERR_HIP;
            for (int64_t j = 0; j < n; ++j)
                if (ex[j] == oz::kNonFiniteExp) rep->status = OZ_ERR_NONFINITE;
        }
    }
    return OZ_OK;
}

// The complex form: zmode 3 asks for the 3-real-product form; with zmode 0 a
// fixed-s product takes it when every dimension is at least kAuto3mMin, and
// the 4-product form otherwise (and always for a tolerance-driven call).
// Measured on ZGEMM at s = 6 (balanced) and 7: the three products win from
// m = n = k = 2048 on (0.59 vs 0.64 ms; 3.5 vs 4.5 ms at 4096); with k up to
// 512, or m = n = k <= 1536, their three splits, T1 and T2 round trips and
// launches cost more than the quarter of INT8 work they save.
constexpr int64_t kAuto3mMin = 2048;
bool use_3m(int cplx, const oz_prec_t* prec, bool tol_mode, bool dd, int64_t m, int64_t n, int64_t k) {
    const int zmode = prec ? prec->zmode : 0;
    if (!cplx || dd) return false;
    if (zmode == 3) return true;
    return zmode == 0 && !tol_mode && m >= kAuto3mMin && n >= kAuto3mMin && k >= kAuto3mMin;
}

// c_lo != nullptr: double-double result (C the high parts, c_lo the low
// parts), alpha = 1, beta = 0, fixed s, the streaming kernel.
int gemm_common(oz_handle_t h, int cplx, char transa, char transb, int64_t m, int64_t n, int64_t k,
                const double* alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                const double* beta, double* C, int64_t ldc, const oz_prec_t* prec, oz_report_t* rep,
                double* c_lo = nullptr, const FixedWs& fixed = FixedWs()) {
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
    bool tol_mode = false;
    bool bal = false;
    double tol = 0.0;
    int smax = kDefaultSmax;
    if (prec) {
        if (prec->slices < 0 || prec->slices > OZ_MAX_SLICES) return 14;
        if (prec->zmode != 0 && prec->zmode != 3 && prec->zmode != 4) return 14;
        // 3M tolerance-driven: truncated digits (balanced growth is not incremental)
        if (cplx && prec->zmode == 3 && prec->slices == 0 && prec->digits == 1) return 14;
        if (prec->kernel < 0 || prec->kernel > 5) return 14;
        if (prec->digits != 0 && prec->digits != 1) return 14;
        bal = prec->digits == 1;
        if (prec->slices == 0) {
            tol_mode = true;
            tol = prec->tol;
            if (!(tol > 0.0)) return 14;
            if (prec->smax) smax = prec->smax;
            if (smax < 1 || smax > OZ_MAX_SLICES) return 14;
            if (bal && smax > kMaxBalancedSlices) smax = kMaxBalancedSlices;
            if (prec->sstart < 0 || prec->sstart > smax) return 14;
            if (prec->selector != 0 && prec->selector != 1) return 14;
            if (prec->selector == 1 && prec->sstart == 0 && !oz_mlp_valid(h->selector)) return OZ_ERR_ARG;
        } else {
            s = prec->slices;
        }
        kc = prec->kchunk;
        kernel = prec->kernel;
    }
    if (c_lo && (tol_mode || (cplx && prec && prec->zmode == 3))) return 14;  // fixed s, 4-product form
    // balanced digits: s <= 8, FP64 results
    if (bal && (s > kMaxBalancedSlices || c_lo)) return 14;
    const int s_plan = tol_mode ? smax : s;  // largest slice count this call may use
    if (kc < 0 || kc % 64 != 0 || (kc > 0 && kc > kchunk_bound(s_plan, bal))) return 14;
    if (kc == 0) kc = kchunk_bound(s_plan, bal);
    if (!tol_mode && s > oz::kMaxLiveSlices && kernel != 0 && kernel != 3) return 14;
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
        if (st == OZ_OK && c_lo) st = hip_status(oz::launch_scale_c(c_lo, ldc, m, n, cplx, 0.0, 0.0, 1, h->stream));
        if (st == OZ_OK && rep && hipStreamSynchronize(h->stream) != hipSuccess) st = OZ_ERR_HIP;
        return st;
    }

    if (use_3m(cplx, prec, tol_mode, c_lo != nullptr, m, n, k)) {
        // 3-real-product form: real INT32 chunks of k terms
        const int64_t kc3 = kc;  // the bound of the largest slice count the call may use
        if (!tol_mode)
            return zgemm_3m(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s, kc3, kernel, bal, rep,
                            fixed);
        if (fixed.ptr) return 14;  // the allocation-free path takes fixed slice counts
        const Tol3 t3{tol, smax, prec->sstart, prec->selector};
        return zgemm_3m(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s, kc3, kernel, bal, rep,
                        fixed, &t3);
    }
    if (fixed.ptr && tol_mode) return 14;  // the allocation-free path takes fixed slice counts
    Plan p = make_plan(cplx, m, n, k, s_plan, tol_mode);
    if (!grid_fits(p)) return OZ_ERR_UNSUPPORTED;
    p.la.bal = p.lb.bal = bal ? 1 : 0;
    char* ws = nullptr;
    st = take_ws(h, fixed, p.total, &ws);
    if (st) return st;
    auto mark = [&](oz_handle_t hh) { return fixed.ptr ? hipSuccess : ::mark(hh); };
    uint64_t* maxa = reinterpret_cast<uint64_t*>(ws + p.off_maxa);
    uint64_t* maxb = reinterpret_cast<uint64_t*>(ws + p.off_maxb);
    int32_t* EA = reinterpret_cast<int32_t*>(ws + p.off_ea);
    int32_t* FB = reinterpret_cast<int32_t*>(ws + p.off_fb);
    int8_t* SA = reinterpret_cast<int8_t*>(ws + p.off_sa);
    int8_t* SB = reinterpret_cast<int8_t*>(ws + p.off_sb);

    oz::OperandView va = view_a(transa, A, lda, m, k, cplx);
    oz::OperandView vb = view_b(transb, B, ldb, n, k, cplx);
    hipError_t e = tol_mode ? hipSuccess : mark(h);
    if (e == hipSuccess) e = oz::launch_zero_u64(maxa, static_cast<int64_t>((p.off_ea - p.off_maxa) / 8), h->stream);
    if (e == hipSuccess) e = oz::launch_scan(va, maxa, h->stream);
    if (e == hipSuccess) e = oz::launch_scan(vb, maxb, h->stream);
    // a tolerance-driven call splits its digit planes as the slice count is chosen and grown
    if (e == hipSuccess && !tol_mode) e = oz::launch_digits(va, maxa, p.la, EA, SA, h->stream);
    if (e == hipSuccess && !tol_mode) e = oz::launch_digits(vb, maxb, p.lb, FB, SB, h->stream);
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
    g.s_lay = s_plan;
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
    g.bal = bal ? 1 : 0;
    if (rep) rep->kchunks = static_cast<int32_t>((p.la.kpad + kc - 1) / kc);

    if (c_lo) {  // the GEMM launcher picks the kernel for this mode
        g.mode = oz::kFinalDD;
        g.c_lo = c_lo;
        g.tile = 0;
    }
    if (!tol_mode) {
        if (!c_lo) g.mode = oz::kFinal;
        e = mark(h);
        if (e == hipSuccess) e = oz::launch_gemm(g, h->stream);
        if (e == hipSuccess) e = mark(h);
        if (e != hipSuccess) return OZ_ERR_HIP;
    } else {
        // (1) starting s from the operand statistics, for the checked target
        const double tol_eff = tol / oz::kCheckMargin;
        double* msa = reinterpret_cast<double*>(ws + p.off_msa);
        double* msb = reinterpret_cast<double*>(ws + p.off_msb);
        if (prec->sstart > 0) {
            s = prec->sstart;
        } else if (prec->selector == 1) {
            st = oz_learned_start(h, h->selector, va, vb, maxa, maxb, msa, msb, m, n, k, cplx, tol_eff, smax,
                                  ws + p.off_sel, &s);
            if (st) return st;
        } else {
            st = rule_slices(h, va, vb, maxa, maxb, msa, msb, reinterpret_cast<double*>(ws + p.off_part1), tol_eff,
                             smax, &s, bal);
            if (st) return st;
        }
        // the learned start is trained on truncated digits; balanced digits
        // save a whole slice (2^7) only from about s = 7 on (their gain is
        // about 2^(s-1)); the residual check still guards the result
        if (bal && prec->sstart == 0 && prec->selector == 1 && s >= 7) --s;
        if (s > smax) s = smax;
        // (2) digit planes 1..s, then emulate at s into the raw FP64 sums
        if (oz::launch_digits(va, maxa, p.la, EA, SA, h->stream, 0, s) != hipSuccess ||
            oz::launch_digits(vb, maxb, p.lb, FB, SB, h->stream, 0, s) != hipSuccess)
            return OZ_ERR_HIP;
        g.acc = reinterpret_cast<double*>(ws + p.off_acc);
        g.s = s;
        // with beta = 0 the first pass also writes C, rewritten only if s grows
        g.mode = beta_zero ? oz::kRawWriteFinal : oz::kRawWrite;
        if (oz::launch_gemm(g, h->stream) != hipSuccess) return OZ_ERR_HIP;
        // (3) check; grow by one slice (new digit, new anti-diagonal) until it passes
        oz::CheckArgs c;
        std::memset(&c, 0, sizeof(c));  // z3 = 0: the raw sums of one product
        c.opa = va;
        c.opb = vb;
        c.maxa = maxa;
        c.maxb = maxb;
        c.acc = g.acc;
        c.Mp = p.la.rows_pad;
        c.EA = EA;
        c.FB = FB;
        c.seed = kProbeSeed;
        c.t = reinterpret_cast<double*>(ws + p.off_t);
        c.u = reinterpret_cast<double*>(ws + p.off_u);
        c.diff = reinterpret_cast<double*>(ws + p.off_diff);
        c.ref = reinterpret_cast<double*>(ws + p.off_ref);
        c.norms = reinterpret_cast<double*>(ws + p.off_norms);
        c.part1 = reinterpret_cast<double*>(ws + p.off_part1);
        c.part2 = reinterpret_cast<double*>(ws + p.off_part2);
        int fallbacks = 0;
        double eps = 0.0;
        for (;;) {
            if (oz::launch_residual(c, h->stream) != hipSuccess) return OZ_ERR_HIP;
            double nrm[2];
            if (hipMemcpyAsync(nrm, c.norms, sizeof(nrm), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
                hipStreamSynchronize(h->stream) != hipSuccess)
                return OZ_ERR_HIP;
            eps = nrm[1] > 0.0 ? std::sqrt(nrm[0] / nrm[1]) : std::sqrt(nrm[0]);
            if (!(eps > tol_eff) || s >= smax) break;  // NaN (non-finite input) also stops
            // slices to add before the next check: the estimate falls by at
            // least about 2^6 per slice (one for an estimate just above the target)
            int add = static_cast<int>(std::ceil(std::log2(eps / tol_eff) / 6.0));
            add = add < 1 ? 1 : (add > smax - s ? smax - s : add);
            if (bal) {
                // balanced digits depend on s: split again at s + add and
                // recompute the raw sums (no incremental growth)
                if (oz::launch_digits(va, maxa, p.la, EA, SA, h->stream, 0, s + add) != hipSuccess ||
                    oz::launch_digits(vb, maxb, p.lb, FB, SB, h->stream, 0, s + add) != hipSuccess)
                    return OZ_ERR_HIP;
                g.s = s + add;
                g.mode = beta_zero ? oz::kRawWriteFinal : oz::kRawWrite;
                if (oz::launch_gemm(g, h->stream) != hipSuccess) return OZ_ERR_HIP;
                s += add;
                fallbacks += add;
                continue;
            }
            // digit planes s + 1 .. s + add, then the anti-diagonals s + 2 ..
            // s + add + 1, one at a time (the incremental order)
            if (oz::launch_digits(va, maxa, p.la, EA, SA, h->stream, s, s + add) != hipSuccess ||
                oz::launch_digits(vb, maxb, p.lb, FB, SB, h->stream, s, s + add) != hipSuccess)
                return OZ_ERR_HIP;
            for (int j = 0; j < add; ++j) {
                g.s = s + 1;
                g.top = 1;
                g.mode = beta_zero ? oz::kRawAddFinal : oz::kRawAdd;  // with beta = 0 the growth step writes C
                if (oz::launch_gemm(g, h->stream) != hipSuccess) return OZ_ERR_HIP;
                g.top = 0;
                ++s;
                ++fallbacks;
            }
        }
        // (4) C = alpha * ldexp(acc, E + F) + beta * C (with beta = 0 the last
        // GEMM pass wrote it)
        if (!beta_zero &&
            oz::launch_finalize(g.acc, p.la.rows_pad, EA, FB, C, ldc, m, n, cplx, ar, ai, br, bi, beta_zero ? 1 : 0,
                                h->stream) != hipSuccess)
            return OZ_ERR_HIP;
        if (rep) {
            rep->slices_used = s;
            rep->fallbacks = fallbacks;
            rep->resid_est = eps;
        }
    }

    if (rep) {
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

bool oz_handle_valid(oz_handle_t h) { return valid(h); }
const std::vector<oz::TuneEntry>& oz_handle_tuning(oz_handle_t h) { return h->tune; }
int oz_handle_use_device(oz_handle_t h) { return use_device(h); }
hipStream_t oz_handle_stream(oz_handle_t h) { return h->stream; }
int oz_handle_device(oz_handle_t h) { return h->device; }
hipError_t oz_handle_mark(oz_handle_t h) { return mark(h); }
char* oz_handle_ws(oz_handle_t h, size_t bytes, int* status) {
    const int st = ensure_ws(h, bytes);
    if (status) *status = st;
    return st ? nullptr : static_cast<char*>(h->ws);
}
oz_mlp_t oz_handle_selector(oz_handle_t h) { return h->selector; }
int oz_handle_lu_stream(oz_handle_t h, hipStream_t* s2, hipEvent_t* ev) {
    if (!h->lu_stream) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return OZ_ERR_HIP;
        for (int i = 0; i < 3; ++i)
            if (hipEventCreateWithFlags(&h->lu_ev[i], hipEventDisableTiming) != hipSuccess) {
                for (int j = 0; j < i; ++j) {
                    (void)hipEventDestroy(h->lu_ev[j]);
                    h->lu_ev[j] = nullptr;
                }
                (void)hipStreamDestroy(s);
                return OZ_ERR_HIP;
            }
        h->lu_stream = s;
    }
    *s2 = h->lu_stream;
    for (int i = 0; i < 3; ++i) ev[i] = h->lu_ev[i];
    return OZ_OK;
}
char* oz_handle_lu_ws(oz_handle_t h, size_t bytes, int* status) {
    *status = OZ_OK;
    if (bytes > h->lu_ws_bytes) {
        if (h->lu_ws) {
            if (hipStreamSynchronize(h->stream) != hipSuccess ||
                (h->lu_stream && hipStreamSynchronize(h->lu_stream) != hipSuccess)) {
                *status = OZ_ERR_HIP;
                return nullptr;
            }
            (void)hipFree(h->lu_ws);
            h->lu_ws = nullptr;
            h->lu_ws_bytes = 0;
        }
        if (hipMalloc(&h->lu_ws, bytes) != hipSuccess) {
            h->lu_ws = nullptr;
            *status = OZ_ERR_ALLOC;
            return nullptr;
        }
        h->lu_ws_bytes = bytes;
    }
    return static_cast<char*>(h->lu_ws);
}
void oz_handle_set_selector(oz_handle_t h, oz_mlp_t mlp) { h->selector = mlp; }

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
    // the allocation-free entry point's scratch: its address on this device
    const int sst = scratch_setup(device, nullptr);
    if (sst) return sst;
    oz_handle_s* h = new (std::nothrow) oz_handle_s;
    if (!h) return OZ_ERR_ALLOC;
    h->magic = kMagic;
    h->device = device;
    h->stream = nullptr;
    h->ws = nullptr;
    h->ws_bytes = 0;
    h->ws_owned = true;
    h->timing = false;
    h->selector = nullptr;
    h->lu_stream = nullptr;
    h->lu_ev[0] = h->lu_ev[1] = h->lu_ev[2] = nullptr;
    h->lu_ws = nullptr;
    h->lu_ws_bytes = 0;
    *handle = h;
    return OZ_OK;
}

int oz_destroy(oz_handle_t h) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    use_device(h);
    hipStreamSynchronize(h->stream);
    if (h->ws_owned && h->ws) hipFree(h->ws);
    if (h->lu_ws) (void)hipFree(h->lu_ws);
    for (hipEvent_t ev : h->lu_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (h->lu_stream) (void)hipStreamDestroy(h->lu_stream);
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
    if (s < 0 || s > OZ_MAX_SLICES) return 14;
    const bool tol = prec && prec->slices == 0;
    const int smax = (prec && prec->smax) ? prec->smax : kDefaultSmax;
    if (tol && (smax < 1 || smax > OZ_MAX_SLICES)) return 14;
    if (use_3m(is_complex, prec, tol, false, m, n, k)) {
        *bytes = make_plan3(m, n, k, tol ? smax : s, tol).total;
        return OZ_OK;
    }
    *bytes = make_plan(is_complex ? 1 : 0, m, n, k, tol ? smax : s, tol).total;
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

int oz_gemm_noalloc(oz_handle_t h, int is_complex, char transa, char transb, int64_t m, int64_t n, int64_t k,
                    const double* alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                    const double* beta, double* C, int64_t ldc, const oz_prec_t* prec) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    if (is_complex != 0 && is_complex != 1) return OZ_ERR_ARG;
    if (prec && prec->slices == 0) return 14;  // fixed slice counts only
    int st = use_device(h);
    if (st) return st;
    FixedWs fixed;
    st = scratch_setup(h->device, &fixed.ptr);
    if (st) return st;
    fixed.bytes = kNoAllocScratchBytes;
    return gemm_common(h, is_complex, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, prec, nullptr,
                       nullptr, fixed);
}

int oz_dgemm_x2(oz_handle_t h, char transa, char transb, int64_t m, int64_t n, int64_t k, const double* A,
                int64_t lda, const double* B, int64_t ldb, double* C_hi, double* C_lo, int64_t ldc,
                const oz_prec_t* prec, oz_report_t* rep) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    if (!prec || prec->slices < 1) return 14;
    if (!C_lo || C_lo == C_hi) return 12;
    const double one[2] = {1.0, 0.0}, zero[2] = {0.0, 0.0};
    return gemm_common(h, 0, transa, transb, m, n, k, one, A, lda, B, ldb, zero, C_hi, ldc, prec, rep, C_lo);
}

int oz_zgemm_x2(oz_handle_t h, char transa, char transb, int64_t m, int64_t n, int64_t k, const double* A,
                int64_t lda, const double* B, int64_t ldb, double* C_hi, double* C_lo, int64_t ldc,
                const oz_prec_t* prec, oz_report_t* rep) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    if (!prec || prec->slices < 1) return 14;
    if (!C_lo || C_lo == C_hi) return 12;
    const double one[2] = {1.0, 0.0}, zero[2] = {0.0, 0.0};
    return gemm_common(h, 1, transa, transb, m, n, k, one, A, lda, B, ldb, zero, C_hi, ldc, prec, rep, C_lo);
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
    g.s_lay = slices;
    g.tile = kernel;
    g.diag_out = out;
    return hip_status(oz::launch_gemm(g, h->stream));
}

int oz_select_slices(oz_handle_t h, char transa, char transb, int64_t m, int64_t n, int64_t k, int is_complex,
                     const double* A, int64_t lda, const double* B, int64_t ldb, double tol, int32_t smax,
                     int32_t* s_out) {
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
    if (!(tol > 0.0) || smax < 0 || smax > OZ_MAX_SLICES || !s_out) return OZ_ERR_ARG;
    if (smax == 0) smax = kDefaultSmax;
    if (use_device(h)) return OZ_ERR_HIP;
    if (m == 0 || n == 0 || k == 0) {
        *s_out = 1;
        return OZ_OK;
    }
    const int cplx = is_complex ? 1 : 0;
    size_t o = 0;
    const size_t off_ma = o;
    o = align256(o + sizeof(uint64_t) * m);
    const size_t off_mb = o;
    o = align256(o + sizeof(uint64_t) * n);
    const size_t off_sa = o;
    o = align256(o + sizeof(double) * m);
    const size_t off_sb = o;
    o = align256(o + sizeof(double) * n);
    const size_t off_part = o;
    o = align256(o + oz::check_part_bytes(m, n, k));
    int st = ensure_ws(h, o);
    if (st) return st;
    char* ws = static_cast<char*>(h->ws);
    uint64_t* maxa = reinterpret_cast<uint64_t*>(ws + off_ma);
    uint64_t* maxb = reinterpret_cast<uint64_t*>(ws + off_mb);
    oz::OperandView va = view_a(transa, A, lda, m, k, cplx);
    oz::OperandView vb = view_b(transb, B, ldb, n, k, cplx);
    hipError_t e = oz::launch_zero_u64(maxa, static_cast<int64_t>((off_sa - off_ma) / 8), h->stream);
    if (e == hipSuccess) e = oz::launch_scan(va, maxa, h->stream);
    if (e == hipSuccess) e = oz::launch_scan(vb, maxb, h->stream);
    if (e != hipSuccess) return OZ_ERR_HIP;
    int s = 0;
    st = rule_slices(h, va, vb, maxa, maxb, reinterpret_cast<double*>(ws + off_sa),
                     reinterpret_cast<double*>(ws + off_sb), reinterpret_cast<double*>(ws + off_part), tol, smax, &s);
    if (st) return st;
    *s_out = s;
    return OZ_OK;
}

// Reads the "entries" array of the autotuner's JSON file: objects with the
// integer fields complex, n, s, tile, order (other fields are skipped).
int oz_load_tuning(oz_handle_t h, const char* path) {
    if (!valid(h)) return OZ_ERR_HANDLE;
    if (!path) {
        h->tune.clear();
        return OZ_OK;
    }
    FILE* f = std::fopen(path, "rb");
    if (!f) return OZ_ERR_ARG;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    const size_t arr = text.find("\"entries\"");
    if (arr == std::string::npos) return OZ_ERR_ARG;
    std::vector<oz::TuneEntry> out;
    size_t pos = text.find('[', arr);
    if (pos == std::string::npos) return OZ_ERR_ARG;
    auto field = [](const std::string& obj, const char* key, double* v) {
        const std::string k = std::string("\"") + key + "\"";
        const size_t at = obj.find(k);
        if (at == std::string::npos) return false;
        const size_t colon = obj.find(':', at + k.size());
        if (colon == std::string::npos) return false;
        char* end = nullptr;
        *v = std::strtod(obj.c_str() + colon + 1, &end);
        return end != obj.c_str() + colon + 1;
    };
    for (;;) {
        const size_t open = text.find('{', pos);
        const size_t close_arr = text.find(']', pos);
        if (open == std::string::npos || (close_arr != std::string::npos && close_arr < open)) break;
        const size_t close = text.find('}', open);
        if (close == std::string::npos) return OZ_ERR_ARG;
        const std::string obj = text.substr(open, close - open + 1);
        double c, n, s, t, o;
        if (!field(obj, "complex", &c) || !field(obj, "n", &n) || !field(obj, "s", &s) || !field(obj, "tile", &t) ||
            !field(obj, "order", &o))
            return OZ_ERR_ARG;
        if ((t != 1 && t != 2 && t != 4) || (o != 0 && o != 1) || s < 1 || s > oz::kMaxLiveSlices || n < 1)
            return OZ_ERR_ARG;
        out.push_back({static_cast<int>(c), static_cast<int64_t>(n), static_cast<int>(s), static_cast<int>(t),
                       static_cast<int>(o)});
        pos = close + 1;
    }
    h->tune = out;
    return OZ_OK;
}

}  // extern "C"
