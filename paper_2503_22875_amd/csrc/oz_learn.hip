// oz_learn.hip -- C ABI of the learned slice-count selection: instance
// generation, feature rows, the GPU-labelled data set, and the selection
// step used by tolerance-driven calls (see oz.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/oz.h"
#include "oz_handle.h"
#include "oz_internal.h"

namespace {

constexpr int kDefaultSmax = 12;
constexpr int kMinLearned = 2;

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

char up(char c) { return (c >= 'a' && c <= 'z') ? static_cast<char>(c - 'a' + 'A') : c; }
bool trans_ok(char c) {
    c = up(c);
    return c == 'N' || c == 'T' || c == 'C';
}

int hipst(hipError_t e) { return e == hipSuccess ? OZ_OK : OZ_ERR_HIP; }

int64_t kchunk_bound(int s) {
    int64_t kc = static_cast<int64_t>(INT32_MAX) / (static_cast<int64_t>(s) * 127 * 127);
    return kc - kc % 64;
}

// Offsets inside a selection scratch block.
struct SelLayout {
    size_t hist, fp, tols, srule, feat, y, s, total;
};
SelLayout sel_layout(int ntol) {
    SelLayout L;
    size_t o = 0;
    auto take = [&o](size_t b) {
        const size_t at = o;
        o = align256(o + b);
        return at;
    };
    L.hist = take(sizeof(unsigned long long) * 2 * oz::kHistLen);
    L.fp = take(sizeof(oz::FeatProb));
    L.tols = take(sizeof(double) * ntol);
    L.srule = take(sizeof(int32_t) * ntol);
    L.feat = take(sizeof(float) * oz::kNumFeat * ntol);
    L.y = take(sizeof(float) * ntol);
    L.s = take(sizeof(int32_t) * ntol);
    L.total = o;
    return L;
}

// Statistics and feature rows of one product, enqueued on st.  fp_host must
// stay alive until the stream has passed this point.
hipError_t features_async(hipStream_t st, const oz::OperandView& va, const oz::OperandView& vb,
                          const uint64_t* maxa, const uint64_t* maxb, double* msa, double* msb, int64_t m, int64_t n,
                          int64_t k, int cplx, int ntol, const double* tols_host, int smax, char* scratch,
                          const SelLayout& L, float* feat_dev, oz::FeatProb* fp_host) {
    unsigned long long* hist = reinterpret_cast<unsigned long long*>(scratch + L.hist);
    hipError_t e = oz::launch_zero_u64(reinterpret_cast<uint64_t*>(hist), 2 * oz::kHistLen, st);
    oz::StatSide sa{va, maxa, msa, hist}, sb{vb, maxb, msb, hist + oz::kHistLen};
    if (e == hipSuccess) e = oz::launch_stats(sa, st);
    if (e == hipSuccess) e = oz::launch_stats(sb, st);
    oz::FeatProb& fp = *fp_host;
    std::memset(&fp, 0, sizeof(fp));
    fp.msq[0] = msa;
    fp.msq[1] = msb;
    fp.hist[0] = hist;
    fp.hist[1] = hist + oz::kHistLen;
    fp.nv[0] = m;
    fp.nv[1] = n;
    fp.m = m;
    fp.n = n;
    fp.k = k;
    fp.cplx = cplx;
    fp.ntol = ntol;
    fp.tols = reinterpret_cast<const double*>(scratch + L.tols);
    fp.feat = feat_dev;
    fp.s_rule = reinterpret_cast<int32_t*>(scratch + L.srule);
    fp.smax = smax;
    if (e == hipSuccess)
        e = hipMemcpyAsync(scratch + L.tols, tols_host, sizeof(double) * ntol, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(scratch + L.fp, &fp, sizeof(fp), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = oz::launch_features(reinterpret_cast<const oz::FeatProb*>(scratch + L.fp), 1, st);
    return e;
}

// Common argument checks of the operand-taking entry points.
int check_operands(char ta, char tb, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb) {
    if (!trans_ok(ta)) return 1;
    if (!trans_ok(tb)) return 2;
    if (m < 0) return 3;
    if (n < 0) return 4;
    if (k < 0) return 5;
    const int64_t ra = up(ta) == 'N' ? m : k;
    const int64_t rb = up(tb) == 'N' ? k : n;
    if (lda < (ra > 1 ? ra : 1)) return 8;
    if (ldb < (rb > 1 ? rb : 1)) return 10;
    return OZ_OK;
}

// Scan of both operands into maxa / maxb (device scratch of m + n uint64).
hipError_t scan_both(hipStream_t st, const oz::OperandView& va, const oz::OperandView& vb, uint64_t* maxa,
                     uint64_t* maxb, int64_t m, int64_t n) {
    hipError_t e = oz::launch_zero_u64(maxa, m, st);
    if (e == hipSuccess) e = oz::launch_zero_u64(maxb, n, st);
    if (e == hipSuccess) e = oz::launch_scan(va, maxa, st);
    if (e == hipSuccess) e = oz::launch_scan(vb, maxb, st);
    return e;
}

}  // namespace

size_t oz_learned_scratch_bytes() { return sel_layout(1).total; }

int oz_learned_start(oz_handle_t h, oz_mlp_t mlp, const oz::OperandView& va, const oz::OperandView& vb,
                     const uint64_t* maxa, const uint64_t* maxb, double* msa, double* msb, int64_t m, int64_t n,
                     int64_t k, int cplx, double tol, int smax, char* scratch, int* s_out) {
    if (!oz_mlp_valid(mlp)) return OZ_ERR_ARG;
    hipStream_t st = oz_handle_stream(h);
    const SelLayout L = sel_layout(1);
    float* feat = reinterpret_cast<float*>(scratch + L.feat);
    oz::FeatProb fp;
    hipError_t e =
        features_async(st, va, vb, maxa, maxb, msa, msb, m, n, k, cplx, 1, &tol, smax, scratch, L, feat, &fp);
    int32_t* sdev = reinterpret_cast<int32_t*>(scratch + L.s);
    const int smin = smax < kMinLearned ? smax : kMinLearned;
    if (e == hipSuccess)
        e = oz_mlp_predict_device(mlp, 1, feat, reinterpret_cast<float*>(scratch + L.y), smin, smax, sdev, st);
    int32_t s = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&s, sdev, sizeof(s), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return OZ_ERR_HIP;
    *s_out = s;
    return OZ_OK;
}

extern "C" {

int oz_gen_operands(oz_handle_t h, const oz_gen_t* p, double* A, int64_t lda, double* B, int64_t ldb) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (!p || p->m < 0 || p->n < 0 || p->k < 0 || p->sig_el < 0 || p->sig_vec < 0 || p->bits < 1 || p->bits > 53 ||
        (p->family != 0 && p->family != 1) || p->zero_q < 0 || p->zero_q > (1 << 24))
        return OZ_ERR_ARG;
    if (lda < (p->m > 1 ? p->m : 1) || ldb < (p->k > 1 ? p->k : 1)) return OZ_ERR_ARG;
    if ((p->m * p->k > 0 && !A) || (p->k * p->n > 0 && !B)) return OZ_ERR_ARG;
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;
    hipStream_t st = oz_handle_stream(h);
    oz::GenSide ga{A, p->m, p->k, lda, oz::sm64_draw(p->key, 0), oz::sm64_draw(p->key, 2), 0,
                   p->sig_el, p->sig_vec, p->bits, p->family, p->zero_q};
    oz::GenSide gb{B, p->k, p->n, ldb, oz::sm64_draw(p->key, 1), oz::sm64_draw(p->key, 3), 1,
                   p->sig_el, p->sig_vec, p->bits, p->family, p->zero_q};
    hipError_t e = oz::launch_gen(ga, st);
    if (e == hipSuccess) e = oz::launch_gen(gb, st);
    return hipst(e);
}

int oz_features(oz_handle_t h, char transa, char transb, int64_t m, int64_t n, int64_t k, int is_complex,
                const double* A, int64_t lda, const double* B, int64_t ldb, int32_t ntol, const double* tols,
                int32_t smax, float* feat, int32_t* s_rule) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    int st = check_operands(transa, transb, m, n, k, lda, ldb);
    if (st) return st;
    if (ntol < 1 || !tols || !feat || smax < 0 || smax > OZ_MAX_SLICES) return OZ_ERR_ARG;
    for (int32_t t = 0; t < ntol; ++t)
        if (!(tols[t] > 0.0)) return OZ_ERR_ARG;
    if (m == 0 || n == 0 || k == 0) return OZ_ERR_ARG;  // no statistics of an empty product
    if (smax == 0) smax = kDefaultSmax;
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;
    const int cplx = is_complex ? 1 : 0;
    const SelLayout L = sel_layout(ntol);
    size_t o = align256(L.total);
    const size_t off_ma = o;
    o = align256(o + sizeof(uint64_t) * m);
    const size_t off_mb = o;
    o = align256(o + sizeof(uint64_t) * n);
    const size_t off_sa = o;
    o = align256(o + sizeof(double) * m);
    const size_t off_sb = o;
    o = align256(o + sizeof(double) * n);
    char* ws = oz_handle_ws(h, o, &st);
    if (!ws) return st;
    hipStream_t stream = oz_handle_stream(h);
    uint64_t* maxa = reinterpret_cast<uint64_t*>(ws + off_ma);
    uint64_t* maxb = reinterpret_cast<uint64_t*>(ws + off_mb);
    const oz::OperandView va = oz::operand_view(up(transa), A, lda, m, k, cplx, 1);
    const oz::OperandView vb = oz::operand_view(up(transb), B, ldb, n, k, cplx, 0);
    oz::FeatProb fp;
    hipError_t e = scan_both(stream, va, vb, maxa, maxb, m, n);
    if (e == hipSuccess)
        e = features_async(stream, va, vb, maxa, maxb, reinterpret_cast<double*>(ws + off_sa),
                           reinterpret_cast<double*>(ws + off_sb), m, n, k, cplx, ntol, tols, smax, ws, L, feat, &fp);
    std::vector<int32_t> sr(static_cast<size_t>(ntol));
    if (e == hipSuccess && s_rule)
        e = hipMemcpyAsync(sr.data(), ws + L.srule, sizeof(int32_t) * ntol, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return OZ_ERR_HIP;
    if (s_rule) std::memcpy(s_rule, sr.data(), sizeof(int32_t) * ntol);
    return OZ_OK;
}

int oz_set_selector(oz_handle_t h, oz_mlp_t mlp) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (mlp && !oz_mlp_valid(mlp)) return OZ_ERR_ARG;
    oz_handle_set_selector(h, mlp);
    return OZ_OK;
}

int oz_predict_slices(oz_handle_t h, char transa, char transb, int64_t m, int64_t n, int64_t k, int is_complex,
                      const double* A, int64_t lda, const double* B, int64_t ldb, double tol, int32_t smax,
                      int32_t* s_out) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    int st = check_operands(transa, transb, m, n, k, lda, ldb);
    if (st) return st;
    if (!(tol > 0.0) || smax < 0 || smax > OZ_MAX_SLICES || !s_out) return OZ_ERR_ARG;
    oz_mlp_t mlp = oz_handle_selector(h);
    if (!oz_mlp_valid(mlp)) return OZ_ERR_ARG;
    if (smax == 0) smax = kDefaultSmax;
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;
    if (m == 0 || n == 0 || k == 0) {
        *s_out = 1;
        return OZ_OK;
    }
    const int cplx = is_complex ? 1 : 0;
    size_t o = align256(oz_learned_scratch_bytes());
    const size_t off_ma = o;
    o = align256(o + sizeof(uint64_t) * m);
    const size_t off_mb = o;
    o = align256(o + sizeof(uint64_t) * n);
    const size_t off_sa = o;
    o = align256(o + sizeof(double) * m);
    const size_t off_sb = o;
    o = align256(o + sizeof(double) * n);
    char* ws = oz_handle_ws(h, o, &st);
    if (!ws) return st;
    hipStream_t stream = oz_handle_stream(h);
    uint64_t* maxa = reinterpret_cast<uint64_t*>(ws + off_ma);
    uint64_t* maxb = reinterpret_cast<uint64_t*>(ws + off_mb);
    const oz::OperandView va = oz::operand_view(up(transa), A, lda, m, k, cplx, 1);
    const oz::OperandView vb = oz::operand_view(up(transb), B, ldb, n, k, cplx, 0);
    if (scan_both(stream, va, vb, maxa, maxb, m, n) != hipSuccess) return OZ_ERR_HIP;
    int s = 0;
    st = oz_learned_start(h, mlp, va, vb, maxa, maxb, reinterpret_cast<double*>(ws + off_sa),
                          reinterpret_cast<double*>(ws + off_sb), m, n, k, cplx, tol, smax, ws, &s);
    if (st) return st;
    *s_out = s;
    return OZ_OK;
}

int oz_selector_dataset(oz_handle_t h, int32_t count, const oz_gen_t* params, int32_t ntol, const double* tols,
                        int32_t s_ref, int32_t smax_rule, float* X, float* y, int32_t* s_rule, double* eps) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (count < 0 || ntol < 1 || (count > 0 && (!params || !tols || !X || !y))) return OZ_ERR_ARG;
    if (s_ref < 2 || s_ref > oz::kMaxRef || smax_rule < 0 || smax_rule > OZ_MAX_SLICES) return OZ_ERR_ARG;
    if (smax_rule == 0) smax_rule = kDefaultSmax;
    const int64_t kc = kchunk_bound(s_ref);
    int64_t max_a = 0, max_b = 0, max_m = 0, max_n = 0, max_sa = 0, max_sb = 0, max_diag = 0, max_part = 0;
    for (int32_t b = 0; b < count; ++b) {
        const oz_gen_t& p = params[b];
        if (p.m < 1 || p.n < 1 || p.k < 1 || p.k > kc || p.n > 65535 || p.sig_el < 0 || p.sig_vec < 0 ||
            p.bits < 1 || p.bits > 53 || (p.family != 0 && p.family != 1) || p.zero_q < 0 || p.zero_q > (1 << 24))
            return OZ_ERR_ARG;
        for (int32_t t = 0; t < ntol; ++t)
            if (!(tols[static_cast<int64_t>(b) * ntol + t] > 0.0)) return OZ_ERR_ARG;
        const oz::SliceLayout la = oz::slice_layout(1, 0, p.m, p.k, s_ref);
        const oz::SliceLayout lb = oz::slice_layout(0, 0, p.n, p.k, s_ref);
        max_a = std::max<int64_t>(max_a, p.m * p.k);
        max_b = std::max<int64_t>(max_b, p.k * p.n);
        max_m = std::max<int64_t>(max_m, la.rows_pad);
        max_n = std::max<int64_t>(max_n, lb.rows_pad);
        max_sa = std::max<int64_t>(max_sa, static_cast<int64_t>(s_ref) * la.rows_pad * la.kpad);
        max_sb = std::max<int64_t>(max_sb, static_cast<int64_t>(s_ref) * lb.rows_pad * lb.kpad);
        max_diag = std::max<int64_t>(max_diag, static_cast<int64_t>(s_ref) * la.rows_pad * lb.rows_pad);
        max_part = std::max<int64_t>(max_part, oz::eps_partial_len(p.m, p.n));
    }
    if (count == 0) return OZ_OK;
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;
    hipStream_t st = oz_handle_stream(h);
    const int64_t rows = static_cast<int64_t>(count) * ntol;
    // one allocation for the whole run
    size_t o = 0;
    auto take = [&o](size_t b) {
        const size_t at = o;
        o = align256(o + b);
        return at;
    };
    const size_t o_A = take(sizeof(double) * max_a), o_B = take(sizeof(double) * max_b);
    const size_t o_ma = take(sizeof(uint64_t) * max_m), o_mb = take(sizeof(uint64_t) * max_n);
    const size_t o_ea = take(sizeof(int32_t) * max_m), o_fb = take(sizeof(int32_t) * max_n);
    const size_t o_sa = take(max_sa), o_sb = take(max_sb);
    const size_t o_msa = take(sizeof(double) * max_m), o_msb = take(sizeof(double) * max_n);
    const size_t o_hist = take(sizeof(unsigned long long) * 2 * oz::kHistLen);
    const size_t o_diag = take(sizeof(int32_t) * max_diag), o_part = take(sizeof(double) * max_part);
    const size_t o_eps = take(sizeof(double) * s_ref * static_cast<size_t>(count));
    const size_t o_tols = take(sizeof(double) * rows), o_srule = take(sizeof(int32_t) * rows);
    const size_t o_fp = take(sizeof(oz::FeatProb) * count);
    void* mem = nullptr;
    if (hipMalloc(&mem, o) != hipSuccess) return OZ_ERR_ALLOC;
    char* d = static_cast<char*>(mem);
    double* dA = reinterpret_cast<double*>(d + o_A);
    double* dB = reinterpret_cast<double*>(d + o_B);
    uint64_t* maxa = reinterpret_cast<uint64_t*>(d + o_ma);
    uint64_t* maxb = reinterpret_cast<uint64_t*>(d + o_mb);
    int32_t* EA = reinterpret_cast<int32_t*>(d + o_ea);
    int32_t* FB = reinterpret_cast<int32_t*>(d + o_fb);
    unsigned long long* hist = reinterpret_cast<unsigned long long*>(d + o_hist);
    double* epsd = reinterpret_cast<double*>(d + o_eps);
    std::vector<oz::FeatProb> fps(static_cast<size_t>(count));
    for (int32_t b = 0; b < count; ++b) {
        oz::FeatProb& fp = fps[b];
        std::memset(&fp, 0, sizeof(fp));
        const oz_gen_t& p = params[b];
        fp.msq[0] = reinterpret_cast<double*>(d + o_msa);
        fp.msq[1] = reinterpret_cast<double*>(d + o_msb);
        fp.hist[0] = hist;
        fp.hist[1] = hist + oz::kHistLen;
        fp.nv[0] = p.m;
        fp.nv[1] = p.n;
        fp.m = p.m;
        fp.n = p.n;
        fp.k = p.k;
        fp.ntol = ntol;
        fp.tols = reinterpret_cast<const double*>(d + o_tols) + static_cast<int64_t>(b) * ntol;
        fp.feat = X + static_cast<int64_t>(b) * ntol * oz::kNumFeat;
        fp.s_rule = reinterpret_cast<int32_t*>(d + o_srule) + static_cast<int64_t>(b) * ntol;
        fp.smax = smax_rule;
        fp.eps = epsd + static_cast<int64_t>(b) * s_ref;
        fp.s_ref = s_ref;
        fp.label = y + static_cast<int64_t>(b) * ntol;
    }
    hipError_t e = hipMemcpy(d + o_fp, fps.data(), sizeof(oz::FeatProb) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + o_tols, tols, sizeof(double) * rows, hipMemcpyHostToDevice);
    const oz::FeatProb* fpd = reinterpret_cast<const oz::FeatProb*>(d + o_fp);
    for (int32_t b = 0; b < count && e == hipSuccess; ++b) {
        const oz_gen_t& p = params[b];
        const oz::GenSide ga{dA, p.m, p.k, p.m, oz::sm64_draw(p.key, 0), oz::sm64_draw(p.key, 2), 0,
                             p.sig_el, p.sig_vec, p.bits, p.family, p.zero_q};
        const oz::GenSide gb{dB, p.k, p.n, p.k, oz::sm64_draw(p.key, 1), oz::sm64_draw(p.key, 3), 1,
                             p.sig_el, p.sig_vec, p.bits, p.family, p.zero_q};
        const oz::OperandView va = oz::operand_view('N', dA, p.m, p.m, p.k, 0, 1);
        const oz::OperandView vb = oz::operand_view('N', dB, p.k, p.n, p.k, 0, 0);
        const oz::SliceLayout la = oz::slice_layout(1, 0, p.m, p.k, s_ref);
        const oz::SliceLayout lb = oz::slice_layout(0, 0, p.n, p.k, s_ref);
        e = oz::launch_gen(ga, st);
        if (e == hipSuccess) e = oz::launch_gen(gb, st);
        if (e == hipSuccess) e = scan_both(st, va, vb, maxa, maxb, p.m, p.n);
        if (e == hipSuccess) e = oz::launch_digits(va, maxa, la, EA, reinterpret_cast<int8_t*>(d + o_sa), st);
        if (e == hipSuccess) e = oz::launch_digits(vb, maxb, lb, FB, reinterpret_cast<int8_t*>(d + o_sb), st);
        if (e == hipSuccess) e = oz::launch_zero_u64(reinterpret_cast<uint64_t*>(hist), 2 * oz::kHistLen, st);
        const oz::StatSide sa{va, maxa, reinterpret_cast<double*>(d + o_msa), hist},
            sb{vb, maxb, reinterpret_cast<double*>(d + o_msb), hist + oz::kHistLen};
        if (e == hipSuccess) e = oz::launch_stats(sa, st);
        if (e == hipSuccess) e = oz::launch_stats(sb, st);
        oz::GemmArgs g;
        std::memset(&g, 0, sizeof(g));
        g.SA = reinterpret_cast<const int8_t*>(d + o_sa);
        g.SB = reinterpret_cast<const int8_t*>(d + o_sb);
        g.EA = EA;
        g.FB = FB;
        g.Mp = la.rows_pad;
        g.Np = lb.rows_pad;
        g.kpad = la.kpad;
        g.chunk_steps = kc / oz::kStep;
        g.s = s_ref;
        g.s_lay = s_ref;
        g.diag_out = reinterpret_cast<int32_t*>(d + o_diag);
        if (e == hipSuccess) e = oz::launch_gemm(g, st);
        if (e == hipSuccess)
            e = oz::launch_eps_table(g.diag_out, la.rows_pad, lb.rows_pad, s_ref, EA, FB, maxa, maxb, p.m, p.n,
                                     reinterpret_cast<double*>(d + o_part), epsd + static_cast<int64_t>(b) * s_ref,
                                     st);
        if (e == hipSuccess) e = oz::launch_features(fpd + b, 1, st);
    }
    std::vector<int32_t> sr(static_cast<size_t>(rows));
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && s_rule)
        e = hipMemcpy(s_rule, d + o_srule, sizeof(int32_t) * rows, hipMemcpyDeviceToHost);
    if (e == hipSuccess && eps)
        e = hipMemcpy(eps, epsd, sizeof(double) * s_ref * static_cast<size_t>(count), hipMemcpyDeviceToHost);
    hipFree(mem);
    return hipst(e);
}

}  // extern "C"
