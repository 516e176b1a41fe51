// oz_batch.hip -- batched DGEMM / ZGEMM emulation: a plan built once per batch
// (layouts, workspace offsets, work lists, descriptors uploaded), executed as
// a fixed sequence of launches on the handle's stream -- zero, batched scan,
// batched digits, one persistent GEMM launch per slice count (one for a batch
// with a single s) -- which can be captured into a HIP graph and replayed.
// A tolerance-driven plan instead picks each problem's starting s (rule or
// learned selector, one batched statistics pass), accumulates raw sums, and
// alternates a batched residual check with incremental growth of the failing
// problems (grouped by s) before one batched scaling pass.
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

constexpr uint64_t kProbeSeed = 0x6f7a5eedull;  // probe vector of the residual check
constexpr int kDefaultSmax = 12;

constexpr uint32_t kBatchMagic = 0x6f7a6274u;  // "ozbt"

// Launch kinds of a group: the all-diagonal tile of one s on 128 x 64 or
// 64 x 64 blocks, the streaming body, the 64 x 64 tile of mixed slice counts
// (s <= 8, each problem its own), the wide tile (9 <= s <= 14).
// kFused3 / kFused3W: fused 3-real-product tiles of complex products, s <= 6
// at two blocks per CU / s = 7, 8 at one.
constexpr int kTile128 = 1, kTile64 = 2, kStream = 3, kMixed = 4, kWide = 5, kTile128x64 = 6, kFused3 = 7,
              kFused3W = 8;

struct Group {
    int s;          // 0 for a mixed group
    int tile;       // launch kind (kTile128 ... kWide)
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
    // one-pass split of the operands with short vectors (fixed-s plans)
    size_t off_fused;
    int64_t n_fused;
    // 3-real-product plans: the three-part split lists
    bool z3;
    size_t off_ops3, off_scan3, off_digits3;
    int64_t n_scan3, n_digits3;
    std::vector<Group> groups;
    std::vector<ScaleOnly> scale_only;
    std::vector<int32_t> slices;  // per problem (0 for quick returns)
    hipGraph_t graph;
    // second stream for the one-wave-per-SIMD launches (s > 8), forked from
    // and joined back into the handle's stream, so they fill the tail of the
    // mixed-s launch instead of running after it
    hipStream_t aux;
    hipEvent_t ev_fork, ev_join;
    hipGraphExec_t graph_exec;
    // ---- tolerance-driven plans ----
    bool tol_mode;
    double tol;
    int smax, sstart, selector, kernel, cplx, cus;
    std::vector<int32_t> prob_b;          // plan problem -> batch index
    std::vector<double> tols;             // tolerance per plan problem
    std::vector<oz::GemmArgs> host_args;  // raw-write descriptors (host copies)
    // host copies of the tile lists uploaded by the GEMM rounds of the current
    // execution (each read by its asynchronous upload; cleared once the
    // execution has synchronised after its last upload)
    std::vector<std::vector<oz::TileItem>> round_lists;
    size_t off_args_add;                  // raw-add descriptors
    size_t off_stat_sides, off_stat_items, off_hist, off_fp, off_feat, off_y, off_s, off_tols;
    int64_t n_stat_items, n_hist;
    size_t off_check, off_active, off_norms, off_wt, off_gv, off_row, off_final, off_final_items, off_dyn;
    size_t off_prange;  // digit-plane range per operand of a split round
    int64_t n_wt, n_gv, n_row, n_final, dyn_cap;
    // host copies of the check work lists, and room for the lists of one
    // round compacted to its open problems
    std::vector<oz::BlockItem> wt_items, gv_items, row_items;
    size_t off_check_dyn;
    std::vector<int32_t> s_cur, fallbacks;
    std::vector<double> resid;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

char up(char c) { return (c >= 'a' && c <= 'z') ? static_cast<char>(c - 'a' + 'A') : c; }
bool trans_ok(char c) {
    c = up(c);
    return c == 'N' || c == 'T' || c == 'C';
}

// terms per INT32 chunk: s products of digits up to 127 (truncated) or 128
// (balanced) in magnitude on one anti-diagonal
int64_t kchunk_bound(int s, bool bal) {
    const int64_t dmax = bal ? 128 : 127;
    int64_t kc = static_cast<int64_t>(INT32_MAX) / (static_cast<int64_t>(s) * dmax * dmax);
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

// One persistent launch over the tiles of `members` (indices into args), all
// with slice count sv (sv = 0: a mixed group, each problem at its own
// args[i].s): launch kind as requested (kTile128, kTile64, kTile128x64 --
// which falls back to kTile64 unless sv <= 6 and every problem is one INT32
// chunk -- or kStream, kMixed, kWide), else the tuned vote, else 128 x 64 when
// the group has at least two such tiles per compute unit; tile order 0
// (problems with the most work per tile first) or 1 (whole problems dealt to
// per-XCD queues) as tuned.  Tiles that hold only padding rows or columns of
// the slice layout are left out.
void build_group(const std::vector<oz::GemmArgs>& args, std::vector<size_t> members, int sv, int kernel, int cplx,
                 int cus, const std::vector<oz::TuneEntry>& tune, Group* out, std::vector<oz::TileItem>* out_items) {
    // tuned choice for one problem: the entry with the same complexity and s
    // (else the nearest s) nearest in log n; false when there is no table
    auto tuned = [&](const oz::GemmArgs& g, int* tile, int* order) {
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
    int64_t big = 0;
    bool multi = false;
    double vote_tile[5] = {0, 0, 0, 0, 0}, vote_order[2] = {0, 0};  // tiles 1, 2, 4
    bool have_tune = false;
    for (size_t i : members) {
        big += (args[i].Mp / 128) * (args[i].Np / 64);
        multi = multi || args[i].chunk_steps < args[i].kpad / oz::kStep;
        int t, od;
        if (tuned(args[i], &t, &od)) {
            const double work = static_cast<double>(args[i].Mp) * args[i].Np * args[i].kpad;
            vote_tile[t] += work;
            vote_order[od] += work;
            have_tune = true;
        }
    }
    int tile = kernel;
    if (!tile && have_tune) {
        tile = vote_tile[1] > vote_tile[2] ? 1 : 2;
        if (vote_tile[4] > vote_tile[tile]) tile = kTile128x64;
    }
    if (!tile) tile = big >= 2 * cus ? 1 : 2;
    // the two-tile 128 x 64 block holds one s <= 6 and a single INT32 chunk
    if (tile == kTile128x64 && (sv < 1 || sv > 6 || multi)) tile = kTile64;
    const int order = have_tune && vote_order[1] > vote_order[0] ? 1 : 0;
    // a mixed-s launch runs the problems with s <= 6 and one INT32 chunk on
    // 128 x 64 two-tile blocks, the others on 64 x 64 blocks
    auto two_tile = [&](size_t i) {
        return tile == kMixed && args[i].s <= 6 && args[i].chunk_steps >= args[i].kpad / oz::kStep;
    };
    auto bm_of = [&](size_t i) -> int64_t {
        return (tile == kTile128 || tile == kTile128x64 || two_tile(i)) ? 128 : 64;
    };
    const int64_t bn = 64;
    // work of one tile: slice pairs times steps, times its 64-row blocks
    auto tile_work = [&](size_t i) {
        const int64_t si = args[i].s;
        return static_cast<double>(si * (si + 1) / 2) * static_cast<double>(args[i].kpad) *
               static_cast<double>(bm_of(i) / 64);
    };
    std::stable_sort(members.begin(), members.end(), [&](size_t a, size_t b) { return tile_work(a) > tile_work(b); });
    // tiles holding valid C' rows and columns only (rows of a complex two-row
    // operand: 16 complex rows span 32 rows of C'); the padding of the slice
    // layout is never computed
    auto tiles_m = [&](size_t i) {
        const int64_t rows = args[i].cplx ? 2 * oz::round_up(args[i].m, 16) : args[i].m, bm = bm_of(i);
        return std::min<int64_t>((rows + bm - 1) / bm, args[i].Mp / bm);
    };
    auto tiles_n = [&](size_t i) { return std::min<int64_t>((args[i].n + bn - 1) / bn, args[i].Np / bn); };
    auto tiles_of = [&](size_t i, std::vector<oz::TileItem>& dst) {
        const int32_t sflag = static_cast<int32_t>(args[i].s) | (two_tile(i) ? oz::kTwoTileItem : 0);
        for (int64_t tm = 0; tm < tiles_m(i); ++tm)
            for (int64_t tn = 0; tn < tiles_n(i); ++tn)
                dst.push_back({static_cast<int32_t>(i), static_cast<int32_t>(tm), static_cast<int32_t>(tn), sflag});
    };
    std::vector<oz::TileItem>& items = *out_items;
    items.clear();
    const int64_t per_cu = (tile == kTile128 || tile == kWide || tile == kFused3W) ? 1 : 2;  // blocks per CU
    if (order == 0) {
        for (size_t i : members) tiles_of(i, items);
    } else {
        // deal whole problems to 8 queues (least work first), then interleave
        // the queues so that item i lands on a block of XCD i % 8 (blocks of a
        // persistent grid with a multiple of 8 blocks go round-robin to the
        // XCDs); exhausted queues leave null items
        constexpr int kX = 8;
        std::vector<oz::TileItem> q[kX];
        double load[kX] = {0};
        for (size_t i : members) {
            int x = 0;
            for (int y = 1; y < kX; ++y)
                if (load[y] < load[x]) x = y;
            tiles_of(i, q[x]);
            load[x] += static_cast<double>(tiles_m(i)) * tiles_n(i) * tile_work(i);
        }
        size_t longest = 0;
        for (int x = 0; x < kX; ++x) longest = std::max(longest, q[x].size());
        for (size_t j = 0; j < longest; ++j)
            for (int x = 0; x < kX; ++x) items.push_back(j < q[x].size() ? q[x][j] : oz::TileItem{-1, 0, 0, 0});
    }
    Group& gr = *out;
    gr.s = sv;
    gr.tile = tile;
    gr.multi = multi;
    gr.nitems = static_cast<int64_t>(items.size());
    int64_t blocks = std::min<int64_t>(gr.nitems, per_cu * cus);
    if (order == 1) blocks -= blocks % 8;  // keep the XCD stride
    gr.blocks = static_cast<int>(blocks > 0 ? blocks : 1);
    gr.off_items = 0;
}

// Launch of one group (any kind) over its tile list.
hipError_t launch_group(const Group& gr, const oz::GemmArgs* dargs, const oz::TileItem* items, bool top,
                        hipStream_t st) {
    switch (gr.tile) {
        case kStream: return oz::launch_gemm_stream_persistent(dargs, items, gr.nitems, gr.s, top, gr.blocks, st);
        case kMixed: return oz::launch_gemm_persistent_mixed(dargs, items, gr.nitems, gr.blocks, top, gr.multi, st);
        case kWide:
            return oz::launch_gemm_wide_persistent(dargs, items, gr.nitems, gr.blocks, top, gr.multi, gr.s, st);
        case kFused3: return oz::launch_gemm_persistent_3m(dargs, items, gr.nitems, gr.blocks, false, st);
        case kFused3W: return oz::launch_gemm_persistent_3m(dargs, items, gr.nitems, gr.blocks, true, st);
        default:
            return oz::launch_gemm_persistent(dargs, items, gr.nitems, gr.s, gr.tile == kTile128x64 ? 4 : gr.tile,
                                              gr.blocks, top, gr.multi, st);
    }
}

// Every group of a round: the one-wave-per-SIMD groups (wide, streaming and
// fused s = 7, 8) on the plan's second stream, the others on st, when there
// are both kinds.
// items_of(gr) gives the device address of a group's tile list.
template <class ItemsOf>
hipError_t launch_groups(oz_batch_t P, const std::vector<Group>& groups, const oz::GemmArgs* dargs, ItemsOf items_of,
                         bool top, hipStream_t st) {
    auto one_wave = [](const Group& gr) { return gr.tile == kWide || gr.tile == kStream || gr.tile == kFused3W; };
    bool narrow = false, wide = false;
    for (const Group& gr : groups) {
        if (one_wave(gr)) wide = true;
        else narrow = true;
    }
    const bool fork = narrow && wide;
    hipError_t e = hipSuccess;
    if (fork) {
        e = hipEventRecord(P->ev_fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(P->aux, P->ev_fork, 0);
    }
    for (const Group& gr : groups)
        if (e == hipSuccess && one_wave(gr)) e = launch_group(gr, dargs, items_of(gr), top, fork ? P->aux : st);
    for (const Group& gr : groups)
        if (e == hipSuccess && !one_wave(gr)) e = launch_group(gr, dargs, items_of(gr), top, st);
    if (fork) {
        if (e == hipSuccess) e = hipEventRecord(P->ev_join, P->aux);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, P->ev_join, 0);
    }
    return e;
}

// Groups of one GEMM round over `members` (slice counts s_of(i)): every
// problem with s <= 8 in one mixed 64 x 64 launch (or, with a single such s,
// the tuned block shape for it), every problem with s in 9..14 in one or two
// wide launches (several INT32 chunks at s >= 13 excepted), one streaming
// launch per remaining s.
template <class SOf>
void round_groups(const std::vector<oz::GemmArgs>& args, const std::vector<size_t>& members, SOf s_of, int kernel,
                  int cplx, int cus, const std::vector<oz::TuneEntry>& tune, std::vector<Group>* groups,
                  std::vector<std::vector<oz::TileItem>>* items) {
    auto multi_of = [&](size_t i) { return args[i].chunk_steps < args[i].kpad / oz::kStep; };
    // a wide launch with several INT32 chunks holds s <= 12 only (register budget)
    bool wide_multi = false;
    for (size_t i : members) {
        const int s = s_of(i);
        if (s > oz::kMaxLiveSlices && s <= 12 && multi_of(i)) wide_multi = true;
    }
    std::vector<size_t> low, wide, streamed;
    std::vector<int> lowvals, streamvals;
    for (size_t i : members) {
        const int s = s_of(i);
        if (s <= oz::kMaxLiveSlices) {
            low.push_back(i);
            if (std::find(lowvals.begin(), lowvals.end(), s) == lowvals.end()) lowvals.push_back(s);
        } else if (s <= (wide_multi ? 12 : oz::kMaxWideSlices) && !(s >= 13 && multi_of(i))) {
            wide.push_back(i);
        } else {
            streamed.push_back(i);
            if (std::find(streamvals.begin(), streamvals.end(), s) == streamvals.end()) streamvals.push_back(s);
        }
    }
    auto add = [&](const std::vector<size_t>& mem, int sv, int kind) {
        Group gr;
        std::vector<oz::TileItem> it;
        build_group(args, mem, sv, kind, cplx, cus, tune, &gr, &it);
        groups->push_back(gr);
        items->push_back(std::move(it));
    };
    // the longest tiles first: their launches run beside the others (second
    // stream), one per slice range that the wide kernel holds without spills
    // (group s = the range's top: 9..12 and 13..14 with one INT32 chunk, 9..11
    // and 12 with several)
    const int wide_lo_top = wide_multi ? 11 : 12;
    std::vector<size_t> wide_lo, wide_hi;
    for (size_t i : wide) (s_of(i) <= wide_lo_top ? wide_lo : wide_hi).push_back(i);
    if (!wide_lo.empty()) add(wide_lo, wide_lo_top, kWide);
    if (!wide_hi.empty()) add(wide_hi, wide_multi ? 12 : oz::kMaxWideSlices, kWide);
    std::sort(streamvals.begin(), streamvals.end());
    for (int sv : streamvals) {
        std::vector<size_t> mem;
        for (size_t i : streamed)
            if (s_of(i) == sv) mem.push_back(i);
        add(mem, sv, kStream);
    }
    if (lowvals.size() == 1) add(low, lowvals[0], kernel);
    else if (lowvals.size() > 1) add(low, 0, kMixed);
}


}  // namespace

extern "C" {

int oz_gemm_batched_plan(oz_handle_t h, int is_complex, int32_t batch, const char* transa, const char* transb,
                         const int64_t* m, const int64_t* n, const int64_t* k, const double* alpha,
                         const double* const* A, const int64_t* lda, const double* const* B, const int64_t* ldb,
                         const double* beta, double* const* C, const int64_t* ldc, const oz_prec_t* prec,
                         const int32_t* slices, const double* tols, oz_batch_t* plan_out) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (!plan_out || batch < 0 || !transa || !transb || !m || !n || !k || !alpha || !A || !lda || !B || !ldb ||
        !beta || !C || !ldc)
        return OZ_ERR_ARG;
    *plan_out = nullptr;
    const int cplx = is_complex ? 1 : 0;
    const int w = cplx ? 2 : 1;
    int s_default = 7, kernel = 0;
    int64_t kc_forced = 0;
    bool tol_mode = false, bal = false;
    double tol = 0.0;
    int smax = kDefaultSmax, sstart = 0, selector = 0;
    if (prec) {
        if (prec->kernel < 0 || prec->kernel > 4 || prec->kernel == 3 || prec->digits < 0 || prec->digits > 1)
            return 14;
        if (prec->zmode != 0 && prec->zmode != 3 && prec->zmode != 4) return 14;
        if (prec->slices == 0) {
            // tolerance-driven: s per problem chosen at execution
            tol_mode = true;
            tol = prec->tol;
            if (prec->smax) smax = prec->smax;
            sstart = prec->sstart;
            selector = prec->selector;
            // balanced digits: fixed slice counts only (the batched growth adds planes one at a time)
            if (!(tol > 0.0) || smax < 1 || smax > OZ_MAX_SLICES || sstart < 0 || sstart > smax ||
                (selector != 0 && selector != 1) || slices || prec->digits)
                return 14;
            if (selector == 1 && sstart == 0 && !oz_mlp_valid(oz_handle_selector(h))) return OZ_ERR_ARG;
            s_default = smax;  // digit planes held for growth
            if (tols)
                for (int32_t b = 0; b < batch; ++b)
                    if (!(tols[b] > 0.0)) return 14;
        } else {
            if (prec->slices < 1 || prec->slices > oz::kMaxWideSlices) return 14;  // fixed s per problem, s <= 14
            s_default = prec->slices;
        }
        kernel = prec->kernel == 4 ? kTile128x64 : prec->kernel;
        kc_forced = prec->kchunk;
        bal = prec->digits == 1;
    }
    if (tols && !tol_mode) return 14;  // per-problem tolerances: tolerance-driven plans only
    // 3-real-product form: complex products with fixed slice counts up to 8
    const bool z3 = cplx && prec && prec->zmode == 3;
    if (z3 && tol_mode) return 14;
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
        if (sb < 1 || sb > (tol_mode ? OZ_MAX_SLICES : oz::kMaxWideSlices)) return 14;
        if ((bal || z3) && sb > oz::kMaxLiveSlices) return 14;  // balanced digits, 3 products: s <= 8
        if (kc_forced < 0 || kc_forced % 64 != 0 || (kc_forced > 0 && kc_forced > kchunk_bound(sb, bal))) return 14;
    }
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;

    oz_batch_s* P = new (std::nothrow) oz_batch_s;
    if (!P) return OZ_ERR_ALLOC;
    P->magic = kBatchMagic;
    P->h = h;
    P->dev = nullptr;
    P->graph = nullptr;
    P->graph_exec = nullptr;
    P->aux = nullptr;
    P->ev_fork = P->ev_join = nullptr;
    if (hipStreamCreateWithFlags(&P->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming) != hipSuccess) {
        if (P->aux) (void)hipStreamDestroy(P->aux);
        if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
        delete P;
        return OZ_ERR_HIP;
    }
    P->slices.assign(static_cast<size_t>(batch), 0);
    P->tol_mode = tol_mode;
    P->tol = tol;
    P->smax = smax;
    P->sstart = sstart;
    P->selector = selector;
    P->kernel = kernel;
    P->cplx = cplx;
    P->n_stat_items = P->n_hist = P->n_wt = P->n_gv = P->n_row = P->n_final = P->dyn_cap = 0;
    P->z3 = z3;
    P->off_fused = 0;
    P->n_fused = 0;
    P->off_ops3 = P->off_scan3 = P->off_digits3 = 0;
    P->n_scan3 = P->n_digits3 = 0;

    // ---- per-problem layouts and workspace offsets --------------------------
    struct Prob {
        int32_t b;
        int s;
        oz::OperandView va, vb;
        oz::SliceLayout la, lb;  // 3-real-product form: the real layout of each part
        size_t off_maxa, off_maxb, off_ea, off_fb, off_sa, off_sb;
        // 3-real-product form: part q (real, imaginary, sum) of each side
        size_t off3_maxa[3], off3_maxb[3], off3_ea[3], off3_fb[3], off3_sa[3], off3_sb[3];
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
        q.la = oz::slice_layout(1, z3 ? 0 : cplx, m[b], k[b], q.s);
        q.lb = oz::slice_layout(0, z3 ? 0 : cplx, n[b], k[b], q.s);
        q.la.bal = q.lb.bal = bal ? 1 : 0;
        if (q.la.rows_pad / 64 > 65535 || q.lb.rows_pad / 64 > 65535) {
            delete P;
            return OZ_ERR_UNSUPPORTED;
        }
        q.kc = kc_forced ? kc_forced : kchunk_bound(q.s, bal);
        q.off_maxa = static_cast<size_t>(n_max) * 8;
        n_max += m[b];
        q.off_maxb = static_cast<size_t>(n_max) * 8;
        n_max += n[b];
        if (z3) {
            // part 0 reuses the offsets above; parts 1, 2 follow
            q.off3_maxa[0] = q.off_maxa;
            q.off3_maxb[0] = q.off_maxb;
            for (int pq = 1; pq < 3; ++pq) {
                q.off3_maxa[pq] = static_cast<size_t>(n_max) * 8;
                n_max += m[b];
                q.off3_maxb[pq] = static_cast<size_t>(n_max) * 8;
                n_max += n[b];
            }
        }
        probs.push_back(q);
        P->prob_b.push_back(b);
        P->tols.push_back(tols ? tols[b] : tol);
        P->slices[b] = tol_mode ? 0 : q.s;
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
        if (z3) {
            q.off3_ea[0] = q.off_ea;
            q.off3_fb[0] = q.off_fb;
            q.off3_sa[0] = q.off_sa;
            q.off3_sb[0] = q.off_sb;
            q.off3_maxa[0] = q.off_maxa;
            q.off3_maxb[0] = q.off_maxb;
            for (int pq = 1; pq < 3; ++pq) {
                q.off3_maxa[pq] += P->off_maxbits;
                q.off3_maxb[pq] += P->off_maxbits;
                q.off3_ea[pq] = take(sizeof(int32_t) * static_cast<size_t>(q.va.nv));
                q.off3_fb[pq] = take(sizeof(int32_t) * static_cast<size_t>(q.lb.rows_pad));
                q.off3_sa[pq] = take(static_cast<size_t>(q.s) * q.la.rows_pad * q.la.kpad);
                q.off3_sb[pq] = take(static_cast<size_t>(q.s) * q.lb.rows_pad * q.lb.kpad);
            }
        }
    }
    // tolerance-driven buffers per problem: raw sums, statistics, check vectors
    struct TolOff {
        size_t acc, msa, msb, t, u, diff, ref;
    };
    std::vector<TolOff> toff(tol_mode ? probs.size() : 0);
    const size_t nprob = probs.size();
    if (tol_mode) {
        for (size_t i = 0; i < nprob; ++i) {
            const Prob& q = probs[i];
            const int64_t mm = q.va.nv, nn = q.vb.nv, kk = q.va.k;
            TolOff& t = toff[i];
            t.acc = take(sizeof(double) * static_cast<size_t>(q.la.rows_pad) * q.lb.rows_pad);
            t.msa = take(sizeof(double) * mm);
            t.msb = take(sizeof(double) * nn);
            t.t = take(sizeof(double) * nn);
            t.u = take(sizeof(double) * 4 * kk);
            t.diff = take(sizeof(double) * 2 * mm);
            t.ref = take(sizeof(double) * 2 * mm);
        }
        P->off_norms = take(sizeof(double) * 2 * nprob);
        P->n_hist = static_cast<int64_t>(2 * oz::kHistLen * nprob);
        P->off_hist = take(sizeof(unsigned long long) * P->n_hist);
        P->off_feat = take(sizeof(float) * oz::kNumFeat * nprob);
        P->off_y = take(sizeof(float) * nprob);
        P->off_s = take(sizeof(int32_t) * nprob);
        P->off_tols = take(sizeof(double) * nprob);
        P->off_active = take(sizeof(int32_t) * nprob);
        P->off_prange = take(sizeof(int32_t) * 4 * nprob);
    }

    // ---- split work lists -----------------------------------------------------
    std::vector<oz::SplitOp> ops;
    std::vector<oz::BlockItem> scan_items, dig_items, fused_items;
    std::vector<oz::Split3Op> ops3;
    std::vector<oz::BlockItem> scan3_items, dig3_items;
    // device addresses are known after allocation: store offsets now, patch below
    auto at = [](size_t off) { return static_cast<uintptr_t>(off); };
    for (const Prob& q : probs) {
        if (z3) {
            for (int side = 0; side < 2; ++side) {
                oz::Split3Op so;
                so.op = side == 0 ? q.va : q.vb;
                so.lay = side == 0 ? q.la : q.lb;
                for (int pq = 0; pq < 3; ++pq) {
                    so.o.maxbits[pq] = reinterpret_cast<uint64_t*>(at(side == 0 ? q.off3_maxa[pq] : q.off3_maxb[pq]));
                    so.o.E[pq] = reinterpret_cast<int32_t*>(at(side == 0 ? q.off3_ea[pq] : q.off3_fb[pq]));
                    so.o.slices[pq] = reinterpret_cast<int8_t*>(at(side == 0 ? q.off3_sa[pq] : q.off3_sb[pq]));
                }
                const int32_t opi = static_cast<int32_t>(ops3.size());
                ops3.push_back(so);
                int64_t bx, by;
                oz::scan_blocks(so.op, &bx, &by);
                for (int64_t y = 0; y < by; ++y)
                    for (int64_t x = 0; x < bx; ++x)
                        scan3_items.push_back({opi, static_cast<int32_t>(x), static_cast<int32_t>(y), 0});
                oz::digits3_blocks(so.lay, &bx, &by);
                for (int64_t y = 0; y < by; ++y)
                    for (int64_t x = 0; x < bx; ++x)
                        dig3_items.push_back({opi, static_cast<int32_t>(x), static_cast<int32_t>(y), 0});
            }
            continue;
        }
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
            if (!tol_mode && oz::split_fusable(so.op)) {
                // short vectors: one pass reads the operand once
                oz::fused_split_blocks(so.op, &by);
                for (int64_t y = 0; y < by; ++y) fused_items.push_back({opi, 0, static_cast<int32_t>(y), 0});
                continue;
            }
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
    P->cus = cus;
    std::vector<oz::GemmArgs> args(probs.size());
    for (size_t i = 0; i < probs.size(); ++i) {
        const Prob& q = probs[i];
        oz::GemmArgs& g = args[i];
        std::memset(&g, 0, sizeof(g));
        // 3-real-product form: this descriptor is T3's (the sum parts), whose
        // scales also mark non-finite input; T1 and T2 follow below
        g.SA = reinterpret_cast<const int8_t*>(at(z3 ? q.off3_sa[2] : q.off_sa));
        g.SB = reinterpret_cast<const int8_t*>(at(z3 ? q.off3_sb[2] : q.off_sb));
        g.EA = reinterpret_cast<const int32_t*>(at(z3 ? q.off3_ea[2] : q.off_ea));
        g.FB = reinterpret_cast<const int32_t*>(at(z3 ? q.off3_fb[2] : q.off_fb));
        g.Mp = q.la.rows_pad;
        g.Np = q.lb.rows_pad;
        g.kpad = q.la.kpad;
        g.chunk_steps = q.kc / oz::kStep;
        g.s = q.s;
        g.s_lay = q.s;
        g.cplx = z3 ? 0 : cplx;
        g.bal = q.la.bal;
        // tolerance-driven: raw sums for the check; with beta = 0 also C, which
        // is then rewritten only for problems whose slice count grows
        g.mode = tol_mode ? oz::kRawWrite : oz::kFinal;
        g.acc = tol_mode ? reinterpret_cast<double*>(at(toff[i].acc)) : nullptr;
        g.C = C[q.b];
        g.ldc = ldc[q.b];
        g.m = m[q.b];
        g.n = n[q.b];
        g.alpha_r = alpha[w * q.b];
        g.alpha_i = cplx ? alpha[w * q.b + 1] : 0.0;
        g.beta_r = beta[w * q.b];
        g.beta_i = cplx ? beta[w * q.b + 1] : 0.0;
        g.beta_zero = (g.beta_r == 0.0 && g.beta_i == 0.0) ? 1 : 0;
        if (tol_mode && g.beta_zero) g.mode = oz::kRawWriteFinal;
    }
    // device descriptors: one per problem, or (3-real-product form) T1, T2, T3
    // of each problem in turn
    std::vector<oz::GemmArgs> dargs_host;
    if (z3) {
        for (size_t i = 0; i < probs.size(); ++i) {
            const Prob& q = probs[i];
            for (int pq = 0; pq < 3; ++pq) {
                oz::GemmArgs g = args[i];
                g.SA = reinterpret_cast<const int8_t*>(at(q.off3_sa[pq]));
                g.SB = reinterpret_cast<const int8_t*>(at(q.off3_sb[pq]));
                g.EA = reinterpret_cast<const int32_t*>(at(q.off3_ea[pq]));
                g.FB = reinterpret_cast<const int32_t*>(at(q.off3_fb[pq]));
                dargs_host.push_back(g);
            }
        }
    }
    std::vector<std::vector<oz::TileItem>> group_items;
    if (z3) {
        // fused tiles: s <= 6 at two blocks per CU, s = 7, 8 at one (second stream)
        std::vector<size_t> lo, hi;
        for (size_t i = 0; i < probs.size(); ++i) (probs[i].s <= 6 ? lo : hi).push_back(3 * i);
        for (int pass = 0; pass < 2; ++pass) {
            const std::vector<size_t>& mem = pass == 0 ? hi : lo;
            if (mem.empty()) continue;
            Group gr;
            std::vector<oz::TileItem> it;
            build_group(dargs_host, mem, 0, pass == 0 ? kFused3W : kFused3, cplx, cus, oz_handle_tuning(h), &gr, &it);
            P->groups.push_back(gr);
            group_items.push_back(std::move(it));
        }
    } else if (!tol_mode) {
        std::vector<size_t> members(probs.size());
        for (size_t i = 0; i < probs.size(); ++i) members[i] = i;
        round_groups(args, members, [&](size_t i) { return probs[i].s; }, kernel, cplx, cus, oz_handle_tuning(h),
                     &P->groups, &group_items);
    }
    // descriptors after the workspace
    P->off_ops = take(sizeof(oz::SplitOp) * ops.size());
    P->off_scan = take(sizeof(oz::BlockItem) * scan_items.size());
    P->off_digits = take(sizeof(oz::BlockItem) * dig_items.size());
    P->off_fused = take(sizeof(oz::BlockItem) * fused_items.size());
    P->n_fused = static_cast<int64_t>(fused_items.size());
    P->off_args = take(sizeof(oz::GemmArgs) * (z3 ? dargs_host.size() : args.size()));
    if (z3) {
        P->off_ops3 = take(sizeof(oz::Split3Op) * ops3.size());
        P->off_scan3 = take(sizeof(oz::BlockItem) * scan3_items.size());
        P->off_digits3 = take(sizeof(oz::BlockItem) * dig3_items.size());
        P->n_scan3 = static_cast<int64_t>(scan3_items.size());
        P->n_digits3 = static_cast<int64_t>(dig3_items.size());
    }
    for (size_t gi = 0; gi < P->groups.size(); ++gi)
        P->groups[gi].off_items = take(sizeof(oz::TileItem) * group_items[gi].size());
    P->n_scan = static_cast<int64_t>(scan_items.size());
    P->n_digits = static_cast<int64_t>(dig_items.size());
    std::vector<oz::StatSide> stat_sides;
    std::vector<oz::BlockItem> stat_items, wt_items, gv_items, row_items, fin_items;
    std::vector<oz::FeatProb> fps;
    std::vector<oz::CheckArgs> checks;
    std::vector<oz::FinalArgs> finals;
    std::vector<oz::GemmArgs> args_add;
    if (tol_mode) {
        int64_t tiles = 0;
        for (size_t i = 0; i < nprob; ++i) {
            const Prob& q = probs[i];
            const TolOff& t = toff[i];
            const int64_t mm = q.va.nv, nn = q.vb.nv, kk = q.va.k;
            unsigned long long* hist =
                reinterpret_cast<unsigned long long*>(at(P->off_hist)) + 2 * oz::kHistLen * i;
            double* msa = reinterpret_cast<double*>(at(t.msa));
            double* msb = reinterpret_cast<double*>(at(t.msb));
            for (int side = 0; side < 2; ++side) {
                const int32_t si = static_cast<int32_t>(stat_sides.size());
                oz::StatSide ss{side == 0 ? q.va : q.vb,
                                reinterpret_cast<const uint64_t*>(at(side == 0 ? q.off_maxa : q.off_maxb)),
                                side == 0 ? msa : msb, hist + side * oz::kHistLen};
                stat_sides.push_back(ss);
                int64_t nb;
                oz::stat_blocks(ss.op, &nb);
                for (int64_t y = 0; y < nb; ++y) stat_items.push_back({si, 0, static_cast<int32_t>(y), 0});
            }
            oz::FeatProb fp;
            std::memset(&fp, 0, sizeof(fp));
            fp.msq[0] = msa;
            fp.msq[1] = msb;
            fp.hist[0] = hist;
            fp.hist[1] = hist + oz::kHistLen;
            fp.nv[0] = mm;
            fp.nv[1] = nn;
            fp.m = mm;
            fp.n = nn;
            fp.k = kk;
            fp.cplx = cplx;
            fp.ntol = 1;
            fp.tols = reinterpret_cast<const double*>(at(P->off_tols)) + i;
            fp.feat = reinterpret_cast<float*>(at(P->off_feat)) + oz::kNumFeat * i;
            fp.s_rule = reinterpret_cast<int32_t*>(at(P->off_s)) + i;
            fp.smax = smax;
            fps.push_back(fp);
            oz::CheckArgs c;
            std::memset(&c, 0, sizeof(c));
            c.opa = q.va;
            c.opb = q.vb;
            c.maxa = reinterpret_cast<const uint64_t*>(at(q.off_maxa));
            c.maxb = reinterpret_cast<const uint64_t*>(at(q.off_maxb));
            c.acc = args[i].acc;
            c.Mp = q.la.rows_pad;
            c.EA = args[i].EA;
            c.FB = args[i].FB;
            c.seed = kProbeSeed;
            c.t = reinterpret_cast<double*>(at(t.t));
            c.u = reinterpret_cast<double*>(at(t.u));
            c.diff = reinterpret_cast<double*>(at(t.diff));
            c.ref = reinterpret_cast<double*>(at(t.ref));
            c.norms = reinterpret_cast<double*>(at(P->off_norms)) + 2 * i;
            checks.push_back(c);
            const int32_t pi = static_cast<int32_t>(i);
            for (int64_t x = 0; x < (nn + 255) / 256; ++x) wt_items.push_back({pi, static_cast<int32_t>(x), 0, 0});
            for (int64_t x = 0; x < (kk + 63) / 64; ++x) gv_items.push_back({pi, static_cast<int32_t>(x), 0, 0});
            for (int64_t x = 0; x < (mm + 63) / 64; ++x) row_items.push_back({pi, static_cast<int32_t>(x), 0, 0});
            for (int64_t x = 0; x < (mm + 255) / 256; ++x) fin_items.push_back({pi, static_cast<int32_t>(x), 0, 0});
            const oz::GemmArgs& g = args[i];
            finals.push_back({g.acc, g.Mp, g.EA, g.FB, g.C, g.ldc, g.m, g.n, cplx, g.alpha_r, g.alpha_i, g.beta_r,
                              g.beta_i, g.beta_zero});
            oz::GemmArgs ga = g;
            ga.mode = g.beta_zero ? oz::kRawAddFinal : oz::kRawAdd;  // beta = 0: growth writes C
            args_add.push_back(ga);
            tiles += (g.Mp / 64) * (g.Np / 64);
        }
        // dynamic tile lists of one growth round: every problem at most once,
        // plus the null items of the per-XCD queues (at most 8 per problem)
        P->dyn_cap = tiles + 8 * static_cast<int64_t>(nprob) + 8;
        P->off_args_add = take(sizeof(oz::GemmArgs) * nprob);
        P->off_stat_sides = take(sizeof(oz::StatSide) * stat_sides.size());
        P->off_stat_items = take(sizeof(oz::BlockItem) * stat_items.size());
        P->off_fp = take(sizeof(oz::FeatProb) * nprob);
        P->off_check = take(sizeof(oz::CheckArgs) * nprob);
        P->off_wt = take(sizeof(oz::BlockItem) * wt_items.size());
        P->off_check_dyn = take(sizeof(oz::BlockItem) * (wt_items.size() + gv_items.size() + row_items.size()));
        P->off_gv = take(sizeof(oz::BlockItem) * gv_items.size());
        P->off_row = take(sizeof(oz::BlockItem) * row_items.size());
        P->off_final = take(sizeof(oz::FinalArgs) * nprob);
        P->off_final_items = take(sizeof(oz::BlockItem) * fin_items.size());
        P->off_dyn = take(sizeof(oz::TileItem) * P->dyn_cap);
        P->n_stat_items = static_cast<int64_t>(stat_items.size());
        P->n_wt = static_cast<int64_t>(wt_items.size());
        P->n_gv = static_cast<int64_t>(gv_items.size());
        P->n_row = static_cast<int64_t>(row_items.size());
        P->wt_items = wt_items;
        P->gv_items = gv_items;
        P->row_items = row_items;
        P->n_final = static_cast<int64_t>(fin_items.size());
    }
    P->s_cur.assign(nprob, 0);
    P->fallbacks.assign(nprob, 0);
    P->resid.assign(nprob, 0.0);
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
    for (auto* list : {&args, &dargs_host})
        for (oz::GemmArgs& g : *list) {
            g.SA = fix(g.SA);
            g.SB = fix(g.SB);
            g.EA = fix(g.EA);
            g.FB = fix(g.FB);
            if (g.acc) g.acc = fix(g.acc);
        }
    for (oz::Split3Op& so : ops3)
        for (int pq = 0; pq < 3; ++pq) {
            so.o.maxbits[pq] = fix(so.o.maxbits[pq]);
            so.o.E[pq] = fix(so.o.E[pq]);
            so.o.slices[pq] = fix(so.o.slices[pq]);
        }
    for (oz::GemmArgs& g : args_add) {
        g.SA = fix(g.SA);
        g.SB = fix(g.SB);
        g.EA = fix(g.EA);
        g.FB = fix(g.FB);
        g.acc = fix(g.acc);
    }
    for (oz::StatSide& ss : stat_sides) {
        ss.maxbits = fix(ss.maxbits);
        ss.msq = fix(ss.msq);
        ss.hist = fix(ss.hist);
    }
    for (oz::FeatProb& fp : fps) {
        fp.msq[0] = fix(fp.msq[0]);
        fp.msq[1] = fix(fp.msq[1]);
        fp.hist[0] = fix(fp.hist[0]);
        fp.hist[1] = fix(fp.hist[1]);
        fp.tols = fix(fp.tols);
        fp.feat = fix(fp.feat);
        fp.s_rule = fix(fp.s_rule);
    }
    for (oz::CheckArgs& c : checks) {
        c.maxa = fix(c.maxa);
        c.maxb = fix(c.maxb);
        c.acc = fix(c.acc);
        c.EA = fix(c.EA);
        c.FB = fix(c.FB);
        c.t = fix(c.t);
        c.u = fix(c.u);
        c.diff = fix(c.diff);
        c.ref = fix(c.ref);
        c.norms = fix(c.norms);
    }
    for (oz::FinalArgs& f : finals) {
        f.acc = fix(f.acc);
        f.EA = fix(f.EA);
        f.FB = fix(f.FB);
    }
    P->host_args = args;
    hipError_t e = hipSuccess;
    auto up_load = [&](size_t off, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(dev + off, src, bytes, hipMemcpyHostToDevice);
    };
    up_load(P->off_ops, ops.data(), sizeof(oz::SplitOp) * ops.size());
    up_load(P->off_scan, scan_items.data(), sizeof(oz::BlockItem) * scan_items.size());
    up_load(P->off_digits, dig_items.data(), sizeof(oz::BlockItem) * dig_items.size());
    up_load(P->off_fused, fused_items.data(), sizeof(oz::BlockItem) * fused_items.size());
    if (z3) {
        up_load(P->off_args, dargs_host.data(), sizeof(oz::GemmArgs) * dargs_host.size());
        up_load(P->off_ops3, ops3.data(), sizeof(oz::Split3Op) * ops3.size());
        up_load(P->off_scan3, scan3_items.data(), sizeof(oz::BlockItem) * scan3_items.size());
        up_load(P->off_digits3, dig3_items.data(), sizeof(oz::BlockItem) * dig3_items.size());
    } else {
        up_load(P->off_args, args.data(), sizeof(oz::GemmArgs) * args.size());
    }
    for (size_t gi = 0; gi < P->groups.size(); ++gi)
        up_load(P->groups[gi].off_items, group_items[gi].data(), sizeof(oz::TileItem) * group_items[gi].size());
    if (tol_mode) {
        up_load(P->off_args_add, args_add.data(), sizeof(oz::GemmArgs) * nprob);
        up_load(P->off_stat_sides, stat_sides.data(), sizeof(oz::StatSide) * stat_sides.size());
        up_load(P->off_stat_items, stat_items.data(), sizeof(oz::BlockItem) * stat_items.size());
        up_load(P->off_fp, fps.data(), sizeof(oz::FeatProb) * nprob);
        up_load(P->off_check, checks.data(), sizeof(oz::CheckArgs) * nprob);
        up_load(P->off_wt, wt_items.data(), sizeof(oz::BlockItem) * wt_items.size());
        up_load(P->off_gv, gv_items.data(), sizeof(oz::BlockItem) * gv_items.size());
        up_load(P->off_row, row_items.data(), sizeof(oz::BlockItem) * row_items.size());
        up_load(P->off_final, finals.data(), sizeof(oz::FinalArgs) * nprob);
        up_load(P->off_final_items, fin_items.data(), sizeof(oz::BlockItem) * fin_items.size());
        // the selection (features, rule) targets the checked tolerance
        std::vector<double> tol_eff(P->tols);
        for (double& t : tol_eff) t /= oz::kCheckMargin;
        up_load(P->off_tols, tol_eff.data(), sizeof(double) * nprob);
    }
    if (e != hipSuccess) {
        hipFree(P->dev);
        delete P;
        return OZ_ERR_HIP;
    }
    *plan_out = P;
    return OZ_OK;
}

}  // extern "C"

namespace {

// One round of GEMM work of a tolerance-driven plan: every listed problem at
// its current slice count, raw-write (first round) or only the new
// anti-diagonal added to the raw sums (growth), in the launches of
// round_groups.
int tol_round(oz_batch_t P, const std::vector<size_t>& members, bool growth, hipStream_t st) {
    char* dev = static_cast<char*>(P->dev);
    const oz::GemmArgs* dargs =
        reinterpret_cast<const oz::GemmArgs*>(dev + (growth ? P->off_args_add : P->off_args));
    // the descriptors on the device carry the planned s: the round's s is set per problem below
    std::vector<oz::GemmArgs> cur(P->host_args);
    for (size_t i : members) cur[i].s = P->s_cur[i];
    std::vector<Group> groups;
    std::vector<std::vector<oz::TileItem>> gitems;
    round_groups(cur, members, [&](size_t i) { return P->s_cur[i]; }, P->kernel == 1 ? 1 : 0, P->cplx, P->cus,
                 oz_handle_tuning(P->h), &groups, &gitems);
    // the host list lives in the plan until the execution ends (moving the
    // outer vector keeps every list's storage): the copy needs no wait of its
    // own, and the GEMM launches queue behind the split
    P->round_lists.emplace_back();
    std::vector<oz::TileItem>& all = P->round_lists.back();
    for (size_t g = 0; g < groups.size(); ++g) {
        groups[g].off_items = all.size();
        all.insert(all.end(), gitems[g].begin(), gitems[g].end());
    }
    if (groups.empty()) return OZ_OK;
    if (static_cast<int64_t>(all.size()) > P->dyn_cap) return OZ_ERR_ALLOC;
    oz::TileItem* ditems = reinterpret_cast<oz::TileItem*>(dev + P->off_dyn);
    if (hipMemcpyAsync(ditems, all.data(), sizeof(oz::TileItem) * all.size(), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return OZ_ERR_HIP;
    // off_items: index into the round's tile list
    return launch_groups(P, groups, dargs, [&](const Group& gr) { return ditems + gr.off_items; }, growth, st) ==
                   hipSuccess
               ? OZ_OK
               : OZ_ERR_HIP;
}

int execute_tol(oz_batch_t P) {
    oz_handle_t h = P->h;
    hipStream_t st = oz_handle_stream(h);
    // lists left by an execution that stopped on an error: their uploads may
    // still read them
    if (!P->round_lists.empty()) {
        if (hipStreamSynchronize(st) != hipSuccess) return OZ_ERR_HIP;
        P->round_lists.clear();
    }
    char* dev = static_cast<char*>(P->dev);
    const size_t nprob = P->prob_b.size();
    hipError_t e = hipSuccess;
    for (const ScaleOnly& so : P->scale_only)
        if (e == hipSuccess) e = oz::launch_scale_c(so.C, so.ldc, so.m, so.n, so.cplx, so.br, so.bi, so.beta_zero, st);
    if (e == hipSuccess && P->n_maxbits)
        e = oz::launch_zero_u64(reinterpret_cast<uint64_t*>(dev + P->off_maxbits), P->n_maxbits, st);
    const oz::SplitOp* ops = reinterpret_cast<const oz::SplitOp*>(dev + P->off_ops);
    if (e == hipSuccess)
        e = oz::launch_scan_batched(ops, reinterpret_cast<const oz::BlockItem*>(dev + P->off_scan), P->n_scan, st);
    if (e != hipSuccess) return OZ_ERR_HIP;
    if (nprob == 0) return OZ_OK;
    // digit planes [lo, hi) of both operands of every problem (2 ops per problem)
    std::vector<int32_t> prange(4 * nprob, 0);
    int32_t* dprange = reinterpret_cast<int32_t*>(dev + P->off_prange);
    auto split_round = [&]() {
        hipError_t r = hipMemcpyAsync(dprange, prange.data(), sizeof(int32_t) * prange.size(), hipMemcpyHostToDevice,
                                      st);
        if (r == hipSuccess)
            r = oz::launch_digits_batched(ops, reinterpret_cast<const oz::BlockItem*>(dev + P->off_digits),
                                          P->n_digits, st, dprange);
        return r;
    };
    // (1) starting slice counts
    std::vector<int32_t> s0(nprob, P->sstart);
    if (P->sstart == 0) {
        int32_t* sdev = reinterpret_cast<int32_t*>(dev + P->off_s);
        e = oz::launch_zero_u64(reinterpret_cast<uint64_t*>(dev + P->off_hist), P->n_hist, st);
        if (e == hipSuccess)
            e = oz::launch_stats_batched(reinterpret_cast<const oz::StatSide*>(dev + P->off_stat_sides),
                                         reinterpret_cast<const oz::BlockItem*>(dev + P->off_stat_items),
                                         P->n_stat_items, st);
        if (e == hipSuccess)
            e = oz::launch_features(reinterpret_cast<const oz::FeatProb*>(dev + P->off_fp),
                                    static_cast<int64_t>(nprob), st);
        if (e == hipSuccess && P->selector == 1) {
            oz_mlp_t mlp = oz_handle_selector(h);
            if (!oz_mlp_valid(mlp)) return OZ_ERR_ARG;
            e = oz_mlp_predict_device(mlp, static_cast<int64_t>(nprob), reinterpret_cast<float*>(dev + P->off_feat),
                                      reinterpret_cast<float*>(dev + P->off_y), P->smax < 2 ? P->smax : 2, P->smax,
                                      sdev, st);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(s0.data(), sdev, sizeof(int32_t) * nprob, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return OZ_ERR_HIP;
    }
    std::vector<size_t> members(nprob);
    for (size_t i = 0; i < nprob; ++i) {
        P->s_cur[i] = s0[i];
        P->fallbacks[i] = 0;
        P->resid[i] = 0.0;
        members[i] = i;
        for (int side = 0; side < 2; ++side) {
            prange[4 * i + 2 * side] = 0;
            prange[4 * i + 2 * side + 1] = s0[i];
        }
    }
    // (2) digit planes 1..s and raw sums at the starting s (the round waits
    // for its uploads, so prange may change afterwards)
    if (split_round() != hipSuccess) return OZ_ERR_HIP;
    int rc = tol_round(P, members, false, st);
    if (rc) return rc;
    // (3) check the active problems; grow the failing ones by one slice
    std::vector<int32_t> active(nprob, 1);
    std::vector<int> target_s(nprob, 0);
    std::vector<double> norms(2 * nprob);
    const oz::CheckArgs* checks = reinterpret_cast<const oz::CheckArgs*>(dev + P->off_check);
    int32_t* dactive = reinterpret_cast<int32_t*>(dev + P->off_active);
    std::vector<oz::BlockItem> citems;
    oz::BlockItem* dcitems = reinterpret_cast<oz::BlockItem*>(dev + P->off_check_dyn);
    for (bool first = true;; first = false) {
        e = hipMemcpyAsync(dactive, active.data(), sizeof(int32_t) * nprob, hipMemcpyHostToDevice, st);
        // the first round checks every problem (the planned lists); later
        // rounds only the open ones (lists compacted on the host)
        const oz::BlockItem *wt = reinterpret_cast<const oz::BlockItem*>(dev + P->off_wt),
                            *gv = reinterpret_cast<const oz::BlockItem*>(dev + P->off_gv),
                            *rw = reinterpret_cast<const oz::BlockItem*>(dev + P->off_row);
        int64_t nwt = P->n_wt, ngv = P->n_gv, nrw = P->n_row;
        if (!first) {
            citems.clear();
            for (const auto* lst : {&P->wt_items, &P->gv_items, &P->row_items}) {
                for (const oz::BlockItem& it : *lst)
                    if (active[it.op]) citems.push_back(it);
                if (lst == &P->wt_items) nwt = static_cast<int64_t>(citems.size());
                else if (lst == &P->gv_items) ngv = static_cast<int64_t>(citems.size()) - nwt;
                else nrw = static_cast<int64_t>(citems.size()) - nwt - ngv;
            }
            if (e == hipSuccess && !citems.empty())
                e = hipMemcpyAsync(dcitems, citems.data(), sizeof(oz::BlockItem) * citems.size(),
                                   hipMemcpyHostToDevice, st);
            wt = dcitems;
            gv = dcitems + nwt;
            rw = dcitems + nwt + ngv;
        }
        if (e == hipSuccess)
            e = oz::launch_residual_batched(checks, static_cast<int64_t>(nprob), dactive, wt, nwt, gv, ngv, rw, nrw,
                                            st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(norms.data(), dev + P->off_norms, sizeof(double) * 2 * nprob, hipMemcpyDeviceToHost,
                               st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return OZ_ERR_HIP;
        std::vector<size_t> grow;
        for (size_t i = 0; i < nprob; ++i) {
            if (!active[i]) continue;
            const double n0 = norms[2 * i], n1 = norms[2 * i + 1];
            const double eps = n1 > 0.0 ? std::sqrt(n0 / n1) : std::sqrt(n0);
            P->resid[i] = eps;
            const double target = P->tols[i] / oz::kCheckMargin;
            if (!(eps > target) || P->s_cur[i] >= P->smax) {  // NaN also stops
                active[i] = 0;
                continue;
            }
            // slices to add before the next check: the estimate falls by at
            // least about 2^6 per slice, so ceil(log2(eps / target) / 6)
            // (one for an estimate just above the target)
            int add = static_cast<int>(std::ceil(std::log2(eps / target) / 6.0));
            add = add < 1 ? 1 : add;
            const int room = P->smax - P->s_cur[i];
            grow.push_back(i);
            target_s[i] = P->s_cur[i] + (add < room ? add : room);
        }
        if (grow.empty()) break;
        // the new digit planes of the growing problems only
        std::fill(prange.begin(), prange.end(), 0);
        int steps = 0;
        for (size_t i : grow) {
            for (int side = 0; side < 2; ++side) {
                prange[4 * i + 2 * side] = P->s_cur[i];
                prange[4 * i + 2 * side + 1] = target_s[i];
            }
            steps = std::max(steps, target_s[i] - P->s_cur[i]);
        }
        if (split_round() != hipSuccess) return OZ_ERR_HIP;
        // one anti-diagonal at a time, each problem up to its target (the
        // order of the single call's growth, without the checks in between)
        for (int j = 0; j < steps; ++j) {
            std::vector<size_t> step_members;
            for (size_t i : grow)
                if (P->s_cur[i] < target_s[i]) {
                    ++P->s_cur[i];
                    ++P->fallbacks[i];
                    step_members.push_back(i);
                }
            rc = tol_round(P, step_members, true, st);
            if (rc) return rc;
        }
    }
    // (4) C = alpha * ldexp(acc, E + F) + beta * C for the problems with
    // beta != 0 (with beta = 0 every GEMM pass, first or growth, writes C)
    bool any = false;
    for (size_t i = 0; i < nprob; ++i) {
        active[i] = P->host_args[i].mode != oz::kRawWriteFinal ? 1 : 0;  // beta != 0
        any = any || active[i];
    }
    e = hipSuccess;
    if (any) {
        // the flags of the last check round may still be in use: the stream orders the copy after it
        e = hipMemcpyAsync(dactive, active.data(), sizeof(int32_t) * nprob, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = oz::launch_finalize_batched(reinterpret_cast<const oz::FinalArgs*>(dev + P->off_final), dactive,
                                            reinterpret_cast<const oz::BlockItem*>(dev + P->off_final_items),
                                            P->n_final, st);
        // the host flags must outlive the copy
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    for (size_t i = 0; i < nprob; ++i) P->slices[P->prob_b[i]] = P->s_cur[i];
    // every upload was followed by a synchronising read of the residual check
    if (e == hipSuccess) P->round_lists.clear();
    return e == hipSuccess ? OZ_OK : OZ_ERR_HIP;
}

}  // namespace

extern "C" {

int oz_batch_execute(oz_batch_t P) {
    if (!P || P->magic != kBatchMagic) return OZ_ERR_HANDLE;
    oz_handle_t h = P->h;
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;
    if (P->tol_mode) return execute_tol(P);
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
    if (e == hipSuccess)
        e = oz::launch_split_fused_batched(ops, reinterpret_cast<const oz::BlockItem*>(dev + P->off_fused),
                                           P->n_fused, st);
    if (P->z3) {
        const oz::Split3Op* ops3 = reinterpret_cast<const oz::Split3Op*>(dev + P->off_ops3);
        if (e == hipSuccess)
            e = oz::launch_scan3_batched(ops3, reinterpret_cast<const oz::BlockItem*>(dev + P->off_scan3),
                                         P->n_scan3, st);
        if (e == hipSuccess)
            e = oz::launch_digits3_batched(ops3, reinterpret_cast<const oz::BlockItem*>(dev + P->off_digits3),
                                           P->n_digits3, st);
    }
    const oz::GemmArgs* args = reinterpret_cast<const oz::GemmArgs*>(dev + P->off_args);
    if (e == hipSuccess) e = oz_handle_mark(h);  // between split and GEMM
    if (e == hipSuccess)
        e = launch_groups(  // off_items: byte offset into the plan's allocation
            P, P->groups, args,
            [&](const Group& gr) { return reinterpret_cast<const oz::TileItem*>(dev + gr.off_items); }, false, st);
    if (e == hipSuccess) e = oz_handle_mark(h);  // after the GEMM launches
    return e == hipSuccess ? OZ_OK : OZ_ERR_HIP;
}

int oz_batch_graph_launch(oz_batch_t P) {
    if (!P || P->magic != kBatchMagic) return OZ_ERR_HANDLE;
    if (P->tol_mode) return OZ_ERR_ARG;  // host decisions between launches: not capturable
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
    if (P->aux) (void)hipStreamDestroy(P->aux);
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    P->magic = 0;
    delete P;
    return OZ_OK;
}

int oz_batch_report(oz_batch_t P, oz_report_t* reps) {
    if (!P || P->magic != kBatchMagic) return OZ_ERR_HANDLE;
    if (!reps) return OZ_ERR_ARG;
    for (size_t b = 0; b < P->slices.size(); ++b) {
        std::memset(&reps[b], 0, sizeof(oz_report_t));
        reps[b].slices_used = P->slices[b];
        reps[b].zmode_used = P->cplx ? (P->z3 ? 3 : 4) : 0;
    }
    for (size_t i = 0; i < P->prob_b.size(); ++i) {
        oz_report_t& r = reps[P->prob_b[i]];
        r.fallbacks = P->fallbacks[i];
        r.resid_est = P->resid[i];
        const oz::GemmArgs& g = P->host_args[i];
        r.kchunks = static_cast<int32_t>((g.kpad / oz::kStep + g.chunk_steps - 1) / g.chunk_steps);
    }
    // scale exponents marking non-finite input
    std::vector<int32_t> ea, fb;
    for (size_t i = 0; i < P->host_args.size(); ++i) {
        const oz::GemmArgs& g = P->host_args[i];
        ea.resize(static_cast<size_t>(g.m));
        fb.resize(static_cast<size_t>(g.n));
        if (hipStreamSynchronize(oz_handle_stream(P->h)) != hipSuccess ||
            hipMemcpy(ea.data(), g.EA, sizeof(int32_t) * g.m, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(fb.data(), g.FB, sizeof(int32_t) * g.n, hipMemcpyDeviceToHost) != hipSuccess)
            return OZ_ERR_HIP;
        bool bad = false;
        for (int32_t x : ea) bad = bad || x == oz::kNonFiniteExp;
        for (int32_t x : fb) bad = bad || x == oz::kNonFiniteExp;
        if (bad) reps[P->prob_b[i]].status = OZ_ERR_NONFINITE;
    }
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
                                  slices, nullptr, &P);
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
                                  slices, nullptr, &P);
    if (st) return st;
    st = oz_batch_execute(P);
    const int st2 = oz_batch_destroy(P);
    return st ? st : st2;
}

}  // extern "C"
