// oz_batch.hip -- batched DGEMM / ZGEMM emulation: a plan built once per batch
// (layouts, workspace offsets, work lists, descriptors uploaded), executed as
// a fixed sequence of launches on the handle's stream -- zero, batched scan,
// batched digits, one persistent GEMM launch per slice count (one for a batch
// with a single s) -- which can be captured into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/oz.h"
#include "oz_internal.h"
#include "oz_handle.h"

namespace {

constexpr uint32_t kBatchMagic = 0x6f7a6274u;  // "ozbt"

struct Group {
    int s;
    int tile;       // 1: 128 x 64, 2: 64 x 64
    int blocks;     // persistent grid
    bool multi;     // some problem spans several INT32 chunks
    int64_t nitems;
    size_t off_items;
};

struct ScaleOnly {
    double* C;
    int64_t ldc, m, n;
    int cplx;
    double br, bi;
    int beta_zero;
};

}  // namespace

struct oz_batch_s {
    uint32_t magic;
    oz_handle_t h;
    void* dev;  // descriptors + workspace, owned by the plan
    size_t dev_bytes;
    size_t off_maxbits;
    int64_t n_maxbits;
    size_t off_ops, off_scan, off_digits, off_args;
    int64_t n_scan, n_digits;
    std::vector<Group> groups;
    std::vector<ScaleOnly> scale_only;
    std::vector<int32_t> slices;  // per problem (0 for quick returns)
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

char up(char c) { return (c >= 'a' && c <= 'z') ? static_cast<char>(c - 'a' + 'A') : c; }
bool trans_ok(char c) {
    c = up(c);
    return c == 'N' || c == 'T' || c == 'C';
}

int64_t kchunk_bound(int s) {
    int64_t kc = static_cast<int64_t>(INT32_MAX) / (static_cast<int64_t>(s) * 127 * 127);
    return kc - kc % 64;
}

oz::OperandView view(char t, const double* X, int64_t ld, int64_t nv, int64_t k, int cplx, int side_a) {
    oz::OperandView v;
    v.X = X;
    const bool tr = up(t) != 'N';
    if (side_a) {
        v.sv = tr ? ld : 1;
        v.sl = tr ? 1 : ld;
    } else {
        v.sv = tr ? 1 : ld;
        v.sl = tr ? ld : 1;
    }
    v.nv = nv;
    v.k = k;
    v.cplx = cplx;
    v.conj = cplx && up(t) == 'C';
    v.side_a = side_a;
    return v;
}

}  // namespace

extern "C" {

int oz_gemm_batched_plan(oz_handle_t h, int is_complex, int32_t batch, const char* transa, const char* transb,
                         const int64_t* m, const int64_t* n, const int64_t* k, const double* alpha,
                         const double* const* A, const int64_t* lda, const double* const* B, const int64_t* ldb,
                         const double* beta, double* const* C, const int64_t* ldc, const oz_prec_t* prec,
                         const int32_t* slices, oz_batch_t* plan_out) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (!plan_out || batch < 0 || !transa || !transb || !m || !n || !k || !alpha || !A || !lda || !B || !ldb ||
        !beta || !C || !ldc)
        return OZ_ERR_ARG;
    *plan_out = nullptr;
    const int cplx = is_complex ? 1 : 0;
    const int w = cplx ? 2 : 1;
    int s_default = 7, kernel = 0;
    int64_t kc_forced = 0;
    if (prec) {
        if (prec->slices < 1 || prec->slices > oz::kMaxLiveSlices) return 14;  // fixed s per problem, s <= 8
        if (prec->kernel < 0 || prec->kernel > 2) return 14;
        s_default = prec->slices;
        kernel = prec->kernel;
        kc_forced = prec->kchunk;
    }
    // argument checks per problem (reference-BLAS positions)
    for (int32_t b = 0; b < batch; ++b) {
        if (!trans_ok(transa[b])) return 1;
        if (!trans_ok(transb[b])) return 2;
        if (m[b] < 0) return 3;
        if (n[b] < 0) return 4;
        if (k[b] < 0) return 5;
        const int64_t ra = up(transa[b]) == 'N' ? m[b] : k[b];
        const int64_t rb = up(transb[b]) == 'N' ? k[b] : n[b];
        if (lda[b] < (ra > 1 ? ra : 1)) return 8;
        if (ldb[b] < (rb > 1 ? rb : 1)) return 10;
        if (ldc[b] < (m[b] > 1 ? m[b] : 1)) return 13;
        const int sb = slices ? slices[b] : s_default;
        if (sb < 1 || sb > oz::kMaxLiveSlices) return 14;
        if (kc_forced < 0 || kc_forced % 64 != 0 || (kc_forced > 0 && kc_forced > kchunk_bound(sb))) return 14;
    }
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;

    oz_batch_s* P = new (std::nothrow) oz_batch_s;
    if (!P) return OZ_ERR_ALLOC;
    P->magic = kBatchMagic;
    P->h = h;
    P->dev = nullptr;
    P->graph = nullptr;
    P->graph_exec = nullptr;
    P->slices.assign(static_cast<size_t>(batch), 0);

    // ---- per-problem layouts and workspace offsets --------------------------
    struct Prob {
        int32_t b;
        int s;
        oz::OperandView va, vb;
        oz::SliceLayout la, lb;
        size_t off_maxa, off_maxb, off_ea, off_fb, off_sa, off_sb;
        int64_t kc;
        int64_t work;  // tiles x steps (for ordering)
    };
    std::vector<Prob> probs;
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    // maxbits of every operand first, contiguous, so one launch clears them
    int64_t n_max = 0;
    for (int32_t b = 0; b < batch; ++b) {
        const double ar = alpha[w * b], ai = cplx ? alpha[w * b + 1] : 0.0;
        const double br = beta[w * b], bi = cplx ? beta[w * b + 1] : 0.0;
        if (m[b] == 0 || n[b] == 0) continue;
        if ((ar == 0.0 && ai == 0.0) || k[b] == 0) {
            if (!(br == 1.0 && bi == 0.0))
                P->scale_only.push_back({C[b], ldc[b], m[b], n[b], cplx, br, bi, (br == 0.0 && bi == 0.0) ? 1 : 0});
            continue;
        }
        Prob q;
        q.b = b;
        q.s = slices ? slices[b] : s_default;
        q.va = view(transa[b], A[b], lda[b], m[b], k[b], cplx, 1);
        q.vb = view(transb[b], B[b], ldb[b], n[b], k[b], cplx, 0);
        q.la = oz::slice_layout(1, cplx, m[b], k[b], q.s);
        q.lb = oz::slice_layout(0, cplx, n[b], k[b], q.s);
        if (q.la.rows_pad / 64 > 65535 || q.lb.rows_pad / 64 > 65535) {
            delete P;
            return OZ_ERR_UNSUPPORTED;
        }
        q.kc = kc_forced ? kc_forced : kchunk_bound(q.s);
        q.off_maxa = static_cast<size_t>(n_max) * 8;
        n_max += m[b];
        q.off_maxb = static_cast<size_t>(n_max) * 8;
        n_max += n[b];
        probs.push_back(q);
        P->slices[b] = q.s;
    }
    P->off_maxbits = take(static_cast<size_t>(n_max) * 8);
    P->n_maxbits = n_max;
    for (Prob& q : probs) {
        q.off_maxa += P->off_maxbits;
        q.off_maxb += P->off_maxbits;
        q.off_ea = take(sizeof(int32_t) * static_cast<size_t>(q.va.nv));
        q.off_fb = take(sizeof(int32_t) * static_cast<size_t>(q.lb.rows_pad));
        q.off_sa = take(static_cast<size_t>(q.s) * q.la.rows_pad * q.la.kpad);
        q.off_sb = take(static_cast<size_t>(q.s) * q.lb.rows_pad * q.lb.kpad);
    }

    // ---- split work lists -----------------------------------------------------
    std::vector<oz::SplitOp> ops;
    std::vector<oz::BlockItem> scan_items, dig_items;
    // device addresses are known after allocation: store offsets now, patch below
    auto at = [](size_t off) { return static_cast<uintptr_t>(off); };
    for (const Prob& q : probs) {
        for (int side = 0; side < 2; ++side) {
            oz::SplitOp so;
            so.op = side == 0 ? q.va : q.vb;
            so.maxbits = reinterpret_cast<uint64_t*>(at(side == 0 ? q.off_maxa : q.off_maxb));
            so.E = reinterpret_cast<int32_t*>(at(side == 0 ? q.off_ea : q.off_fb));
            so.slices = reinterpret_cast<int8_t*>(at(side == 0 ? q.off_sa : q.off_sb));
            so.lay = side == 0 ? q.la : q.lb;
            const int32_t opi = static_cast<int32_t>(ops.size());
            ops.push_back(so);
            int64_t bx, by;
            oz::scan_blocks(so.op, &bx, &by);
            for (int64_t y = 0; y < by; ++y)
                for (int64_t x = 0; x < bx; ++x)
                    scan_items.push_back({opi, static_cast<int32_t>(x), static_cast<int32_t>(y), 0});
            oz::digits_blocks(so.op, so.lay, &bx, &by);
            for (int64_t y = 0; y < by; ++y)
                for (int64_t x = 0; x < bx; ++x)
                    dig_items.push_back({opi, static_cast<int32_t>(x), static_cast<int32_t>(y), 0});
        }
    }

    // ---- GEMM descriptors and tile lists, one group per slice count ----------
    int cus = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, oz_handle_device(h)) == hipSuccess) cus = prop.multiProcessorCount;
    }
    std::vector<oz::GemmArgs> args(probs.size());
    for (size_t i = 0; i < probs.size(); ++i) {
        const Prob& q = probs[i];
        oz::GemmArgs& g = args[i];
        std::memset(&g, 0, sizeof(g));
        g.SA = reinterpret_cast<const int8_t*>(at(q.off_sa));
        g.SB = reinterpret_cast<const int8_t*>(at(q.off_sb));
        g.EA = reinterpret_cast<const int32_t*>(at(q.off_ea));
        g.FB = reinterpret_cast<const int32_t*>(at(q.off_fb));
        g.Mp = q.la.rows_pad;
        g.Np = q.lb.rows_pad;
        g.kpad = q.la.kpad;
        g.chunk_steps = q.kc / oz::kStep;
        g.s = q.s;
        g.s_lay = q.s;
        g.cplx = cplx;
        g.mode = oz::kFinal;
        g.C = C[q.b];
        g.ldc = ldc[q.b];
        g.m = m[q.b];
        g.n = n[q.b];
        g.alpha_r = alpha[w * q.b];
        g.alpha_i = cplx ? alpha[w * q.b + 1] : 0.0;
        g.beta_r = beta[w * q.b];
        g.beta_i = cplx ? beta[w * q.b + 1] : 0.0;
        g.beta_zero = (g.beta_r == 0.0 && g.beta_i == 0.0) ? 1 : 0;
    }
    std::vector<int> svals;
    for (const Prob& q : probs)
        if (std::find(svals.begin(), svals.end(), q.s) == svals.end()) svals.push_back(q.s);
    std::sort(svals.begin(), svals.end());
    std::vector<std::vector<oz::TileItem>> group_items;
    const std::vector<oz::TuneEntry>& tune = oz_handle_tuning(h);
    // tuned choice for one problem: the entry with the same complexity and s
    // (else the nearest s) nearest in log n; -1 when there is no table
    auto tuned = [&](const oz::GemmArgs& g, int sv, int* tile, int* order) {
        int best = -1;
        double bd = 1e300;
        const double size = static_cast<double>(g.m > g.n ? g.m : g.n);
        for (size_t i = 0; i < tune.size(); ++i) {
            const oz::TuneEntry& t = tune[i];
            if (t.cplx != cplx) continue;
            const double d = std::fabs(std::log2(size / static_cast<double>(t.n))) + 4.0 * std::abs(t.s - sv);
            if (d < bd) {
                bd = d;
                best = static_cast<int>(i);
            }
        }
        if (best < 0) return false;
        *tile = tune[best].tile;
        *order = tune[best].order;
        return true;
    };
    for (int sv : svals) {
        int64_t big = 0;
        bool multi = false;
        std::vector<size_t> members;
        double vote_tile[3] = {0, 0, 0}, vote_order[2] = {0, 0};
        bool have_tune = false;
        for (size_t i = 0; i < probs.size(); ++i)
            if (probs[i].s == sv) {
                members.push_back(i);
                big += (args[i].Mp / 128) * (args[i].Np / 64);
                multi = multi || args[i].chunk_steps < args[i].kpad / oz::kStep;
                int t, od;
                if (tuned(args[i], sv, &t, &od)) {
                    const double work = static_cast<double>(args[i].Mp) * args[i].Np * args[i].kpad;
                    vote_tile[t] += work;
                    vote_order[od] += work;
                    have_tune = true;
                }
            }
        // block shape: as requested, else the tuned vote, else 128 x 64 when the
        // group has at least two such tiles per compute unit
        int tile = kernel;
        if (!tile) tile = have_tune ? (vote_tile[1] > vote_tile[2] ? 1 : 2) : (big >= 2 * cus ? 1 : 2);
        const int order = have_tune && vote_order[1] > vote_order[0] ? 1 : 0;
        const int64_t bm = tile == 1 ? 128 : 64, bn = 64;
        // problems with the most work per tile first
        std::stable_sort(members.begin(), members.end(),
                         [&](size_t a, size_t b) { return args[a].kpad > args[b].kpad; });
        auto tiles_of = [&](size_t i, std::vector<oz::TileItem>& dst) {
            for (int64_t tm = 0; tm < args[i].Mp / bm; ++tm)
                for (int64_t tn = 0; tn < args[i].Np / bn; ++tn)
                    dst.push_back({static_cast<int32_t>(i), static_cast<int32_t>(tm), static_cast<int32_t>(tn), 0});
        };
        std::vector<oz::TileItem> items;
        const int64_t per_cu = tile == 1 ? 1 : 2;  // blocks resident per compute unit
        if (order == 0) {
            for (size_t i : members) tiles_of(i, items);
        } else {
            // deal whole problems to 8 queues (least work first), then interleave
            // the queues so that item i lands on a block of XCD i % 8 (blocks of
            // a persistent grid with a multiple of 8 blocks go round-robin to
            // the XCDs); exhausted queues leave null items
            constexpr int kX = 8;
            std::vector<oz::TileItem> q[kX];
            double load[kX] = {0};
            for (size_t i : members) {
                int x = 0;
                for (int y = 1; y < kX; ++y)
                    if (load[y] < load[x]) x = y;
                tiles_of(i, q[x]);
                load[x] += static_cast<double>(args[i].Mp / bm) * (args[i].Np / bn) * args[i].kpad;
            }
            size_t longest = 0;
            for (int x = 0; x < kX; ++x) longest = std::max(longest, q[x].size());
            for (size_t j = 0; j < longest; ++j)
                for (int x = 0; x < kX; ++x) items.push_back(j < q[x].size() ? q[x][j] : oz::TileItem{-1, 0, 0, 0});
        }
        Group gr;
        gr.s = sv;
        gr.tile = tile;
        gr.multi = multi;
        gr.nitems = static_cast<int64_t>(items.size());
        int64_t blocks = std::min<int64_t>(gr.nitems, per_cu * cus);
        if (order == 1) blocks -= blocks % 8;  // keep the XCD stride
        gr.blocks = static_cast<int>(blocks > 0 ? blocks : 1);
        gr.off_items = 0;
        P->groups.push_back(gr);
        group_items.push_back(std::move(items));
    }

    // descriptors after the workspace
    P->off_ops = take(sizeof(oz::SplitOp) * ops.size());
    P->off_scan = take(sizeof(oz::BlockItem) * scan_items.size());
    P->off_digits = take(sizeof(oz::BlockItem) * dig_items.size());
    P->off_args = take(sizeof(oz::GemmArgs) * args.size());
    for (size_t gi = 0; gi < P->groups.size(); ++gi)
        P->groups[gi].off_items = take(sizeof(oz::TileItem) * group_items[gi].size());
    P->n_scan = static_cast<int64_t>(scan_items.size());
    P->n_digits = static_cast<int64_t>(dig_items.size());
    P->dev_bytes = o;
    if (o > 0 && hipMalloc(&P->dev, o) != hipSuccess) {
        delete P;
        return OZ_ERR_ALLOC;
    }
    char* dev = static_cast<char*>(P->dev);
    // patch offsets (stored as pointers from a null base) into device addresses
    auto fix = [dev](auto* p) { return reinterpret_cast<decltype(p)>(dev + reinterpret_cast<uintptr_t>(p)); };
    for (oz::SplitOp& so : ops) {
        so.maxbits = fix(so.maxbits);
        so.E = fix(so.E);
        so.slices = fix(so.slices);
    }
    for (oz::GemmArgs& g : args) {
        g.SA = fix(g.SA);
        g.SB = fix(g.SB);
        g.EA = fix(g.EA);
        g.FB = fix(g.FB);
    }
    hipError_t e = hipSuccess;
    auto up_load = [&](size_t off, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(dev + off, src, bytes, hipMemcpyHostToDevice);
    };
    up_load(P->off_ops, ops.data(), sizeof(oz::SplitOp) * ops.size());
    up_load(P->off_scan, scan_items.data(), sizeof(oz::BlockItem) * scan_items.size());
    up_load(P->off_digits, dig_items.data(), sizeof(oz::BlockItem) * dig_items.size());
    up_load(P->off_args, args.data(), sizeof(oz::GemmArgs) * args.size());
    for (size_t gi = 0; gi < P->groups.size(); ++gi)
        up_load(P->groups[gi].off_items, group_items[gi].data(), sizeof(oz::TileItem) * group_items[gi].size());
    if (e != hipSuccess) {
        hipFree(P->dev);
        delete P;
        return OZ_ERR_HIP;
    }
    *plan_out = P;
    return OZ_OK;
}

int oz_batch_execute(oz_batch_t P) {
    if (!P || P->magic != kBatchMagic) return OZ_ERR_HANDLE;
    oz_handle_t h = P->h;
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;
    hipStream_t st = oz_handle_stream(h);
    char* dev = static_cast<char*>(P->dev);
    hipError_t e = oz_handle_mark(h);  // timing: before the split launches
    for (const ScaleOnly& so : P->scale_only)
        if (e == hipSuccess) e = oz::launch_scale_c(so.C, so.ldc, so.m, so.n, so.cplx, so.br, so.bi, so.beta_zero, st);
    if (e == hipSuccess && P->n_maxbits)
        e = oz::launch_zero_u64(reinterpret_cast<uint64_t*>(dev + P->off_maxbits), P->n_maxbits, st);
    const oz::SplitOp* ops = reinterpret_cast<const oz::SplitOp*>(dev + P->off_ops);
    if (e == hipSuccess)
        e = oz::launch_scan_batched(ops, reinterpret_cast<const oz::BlockItem*>(dev + P->off_scan), P->n_scan, st);
    if (e == hipSuccess)
        e = oz::launch_digits_batched(ops, reinterpret_cast<const oz::BlockItem*>(dev + P->off_digits), P->n_digits,
                                      st);
    const oz::GemmArgs* args = reinterpret_cast<const oz::GemmArgs*>(dev + P->off_args);
    if (e == hipSuccess) e = oz_handle_mark(h);  // between split and GEMM
    for (const Group& gr : P->groups)
        if (e == hipSuccess)
            e = oz::launch_gemm_persistent(args, reinterpret_cast<const oz::TileItem*>(dev + gr.off_items), gr.nitems,
                                           gr.s, gr.tile, gr.blocks, false, gr.multi, st);
    if (e == hipSuccess) e = oz_handle_mark(h);  // after the GEMM launches
    return e == hipSuccess ? OZ_OK : OZ_ERR_HIP;
}

int oz_batch_graph_launch(oz_batch_t P) {
    if (!P || P->magic != kBatchMagic) return OZ_ERR_HANDLE;
    hipStream_t st = oz_handle_stream(P->h);
    if (st == nullptr) return OZ_ERR_ARG;  // the null stream cannot be captured
    if (oz_handle_use_device(P->h)) return OZ_ERR_HIP;
    if (!P->graph_exec) {
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return OZ_ERR_HIP;
        const int rc = oz_batch_execute(P);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        if (rc != OZ_OK || ec != hipSuccess || !g) {
            if (g) hipGraphDestroy(g);
            return rc != OZ_OK ? rc : OZ_ERR_HIP;
        }
        if (hipGraphInstantiate(&P->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(g);
            P->graph_exec = nullptr;
            return OZ_ERR_HIP;
        }
        P->graph = g;
    }
    return hipGraphLaunch(P->graph_exec, st) == hipSuccess ? OZ_OK : OZ_ERR_HIP;
}

int oz_batch_destroy(oz_batch_t P) {
    if (!P || P->magic != kBatchMagic) return OZ_ERR_HANDLE;
    oz_handle_use_device(P->h);
    hipStreamSynchronize(oz_handle_stream(P->h));
    if (P->graph_exec) hipGraphExecDestroy(P->graph_exec);
    if (P->graph) hipGraphDestroy(P->graph);
    if (P->dev) hipFree(P->dev);
    P->magic = 0;
    delete P;
    return OZ_OK;
}

int oz_batch_info(oz_batch_t P, int32_t* launches, int64_t* tiles, size_t* device_bytes, int32_t* slices) {
    if (!P || P->magic != kBatchMagic) return OZ_ERR_HANDLE;
    if (launches) *launches = static_cast<int32_t>(P->groups.size());
    if (tiles) {
        int64_t t = 0;
        for (const Group& g : P->groups) t += g.nitems;
        *tiles = t;
    }
    if (device_bytes) *device_bytes = P->dev_bytes;
    if (slices)
        for (size_t i = 0; i < P->slices.size(); ++i) slices[i] = P->slices[i];
    return OZ_OK;
}

int oz_zgemm_batched(oz_handle_t h, int32_t batch, const char* transa, const char* transb, const int64_t* m,
                     const int64_t* n, const int64_t* k, const double* alpha, const double* const* A,
                     const int64_t* lda, const double* const* B, const int64_t* ldb, const double* beta,
                     double* const* C, const int64_t* ldc, const oz_prec_t* prec, const int32_t* slices) {
    oz_batch_t P = nullptr;
    int st = oz_gemm_batched_plan(h, 1, batch, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, prec,
                                  slices, &P);
    if (st) return st;
    st = oz_batch_execute(P);
    const int st2 = oz_batch_destroy(P);
    return st ? st : st2;
}

int oz_dgemm_batched(oz_handle_t h, int32_t batch, const char* transa, const char* transb, const int64_t* m,
                     const int64_t* n, const int64_t* k, const double* alpha, const double* const* A,
                     const int64_t* lda, const double* const* B, const int64_t* ldb, const double* beta,
                     double* const* C, const int64_t* ldc, const oz_prec_t* prec, const int32_t* slices) {
    oz_batch_t P = nullptr;
    int st = oz_gemm_batched_plan(h, 0, batch, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, prec,
                                  slices, &P);
    if (st) return st;
    st = oz_batch_execute(P);
    const int st2 = oz_batch_destroy(P);
    return st ? st : st2;
}

}  // extern "C"
