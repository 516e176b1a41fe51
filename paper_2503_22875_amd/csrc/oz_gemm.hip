// oz_gemm.hip -- INT8 slice-pair products on CDNA4 matrix cores with the
// FP64 rescale-accumulate epilogue fused (paper Sec. 2.2: INT8 matrix units
// with INT32 accumulation, result accumulated at higher precision).
//
// A block computes a BM x BN tile of C' = A' * B' (A', B' the slice buffers
// of oz_split) with WMW x WNW waves, each owning a 32 x 32 sub-tile and one
// v_mfma_i32_32x32x32_i8 per slice pair and 32-term step.
//
// All-diagonal form: every step stages the s slices of both operands in LDS
// once and runs all s(s+1)/2 pairs (p, q) with p + q <= s + 1, accumulating
// pair (p, q) into the INT32 register tile of its anti-diagonal d = p + q.
// Loading s slices for s(s+1)/2 products gives (s+1)/2 times the arithmetic
// intensity of streaming one pair at a time, and no INT32 partial ever
// leaves the registers.  Per INT32 chunk (kchunk terms, sized so that
// s * kchunk * 127^2 <= 2^31 - 1) the s diagonal tiles are folded into an
// FP64 tile, from d = s+1 down to 2, each times 2^(-7d) (exact; 2^(2-8d) for
// balanced digits).  The final
// epilogue applies 2^(E_i + F_j) with ldexp and alpha/beta.
//
// LDS stages (a ring of NST): for each operand, 16-term half h, slice p:
// 64 rows x 16 bytes, a contiguous 1 KiB run in the global slice layout,
// moved by global_load_lds_dwordx4 (global memory straight into LDS, one wave
// per run, 16 bytes per lane, no staging registers).  Each MFMA operand read
// (32 lanes x 16 consecutive bytes) is free of bank conflicts.  The copy of
// step ks + NST - 1 is in flight while the MFMAs of step ks run, so NST - 1
// steps of MFMA work cover the memory latency.
#include <type_traits>

#include "oz_internal.h"

namespace oz {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void global_cvoid;

// Exponent of the weight of anti-diagonal d: 2^(-7d) for truncated digits,
// 2^(2-8d) for balanced ones.  Every term S_d * 2^e is exact (ldexp of an
// INT32 value far from the FP64 range limits).
__device__ __forceinline__ int diag_exp(int d, int bal) { return bal ? 2 - 8 * d : -7 * d; }

// Fold the live INT32 diagonal tiles into the FP64 tile, from the top
// (d = DD + 2 = S + 1) down to d = DLO + 2; acc[i] holds diagonal DLO + i.
template <int ND, int DLO, int DD>
__device__ __forceinline__ void fold_diags(double (&acc64)[16], v16i (&acc)[ND], int bal) {
    const int e = diag_exp(DD + 2, bal);
#pragma unroll
    for (int r = 0; r < 16; ++r) acc64[r] = acc64[r] + ldexp(static_cast<double>(acc[DD - DLO][r]), e);
    if constexpr (DD > DLO) fold_diags<ND, DLO, DD - 1>(acc64, acc, bal);
}

// The same fold into a double-double (hi, lo): each term, exact in FP64, is
// added by dd_add_exact (defined below).
__device__ __forceinline__ void dd_add_exact(double& hi, double& lo, double x);
template <int ND, int DLO, int DD>
__device__ __forceinline__ void fold_diags_dd(double (&hi)[16], double (&lo)[16], v16i (&acc)[ND], int bal) {
    const int e = diag_exp(DD + 2, bal);
#pragma unroll
    for (int r = 0; r < 16; ++r) dd_add_exact(hi[r], lo[r], ldexp(static_cast<double>(acc[DD - DLO][r]), e));
    if constexpr (DD > DLO) fold_diags_dd<ND, DLO, DD - 1>(hi, lo, acc, bal);
}

// Tile order: the hardware hands consecutive blocks to the 8 XCDs in turn,
// and each XCD has its own L2.  Block b is given the tile t = start(x) + b/8 of
// a contiguous range per XCD x = b % 8, and inside that range tiles run in
// groups of kGroupM tile rows, column by column, so the blocks resident on one
// XCD at a time share a few row slices of A' and column slices of B'.
constexpr int kXcds = 8;
constexpr int kGroupM = 8;

__device__ __forceinline__ void tile_of_block(int64_t b, int64_t tiles_m, int64_t tiles_n, int64_t& tm,
                                              int64_t& tn) {
    const int64_t T = tiles_m * tiles_n;
    const int64_t x = b % kXcds, r = b / kXcds;
    const int64_t q = T / kXcds, rr = T % kXcds;
    const int64_t t = x * q + (x < rr ? x : rr) + r;
    const int64_t per_group = static_cast<int64_t>(kGroupM) * tiles_n;
    const int64_t grp = t / per_group, in = t % per_group;
    const int64_t gm0 = grp * kGroupM;
    const int64_t gh = (tiles_m - gm0) < kGroupM ? (tiles_m - gm0) : kGroupM;
    tm = gm0 + in % gh;
    tn = in / gh;
}

// Wait until at most N vector-memory operations of this wave are in flight
// (loads and stores retire in issue order on this architecture).
template <int N>
__device__ __forceinline__ void wait_vm() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Workgroup barrier of the copy ring.  __syncthreads() carries a release
// fence, which waits for every outstanding global->LDS copy (vmcnt(0)) and
// would drain the copies just issued for later stages; here the wait_vm
// before the barrier decides which copies must have landed.  The memory
// clobbers keep the compiler from moving LDS accesses across the barrier, so
// every LDS read of a buffer is issued before the barrier that precedes its
// refill; the compiler may still wait for the last reads, and issue the MFMAs
// they feed, after it.  The refill is issued only after the barrier and writes
// LDS when its global data returns, a round trip through L2 at the least
// (hundreds of cycles), while the reads already issued are at most a few
// 1 KiB wave reads per wave queued at the CU's LDS (128 B per clock).  An
// lgkmcnt(0) wait before the barrier measured 1% slower on the default product.
__device__ __forceinline__ void ring_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Final epilogue of one wave's 32 x 32 sub-tile whose first row of C' is
// row0: v = ldexp(acc64, E_i + F_j), then alpha/beta (two rounded products
// and one rounded add per part, no fused multiply-add), or NaN where the row
// or column scale marks Inf/NaN input.  Register r holds C' row
// row0 + 8*(r/4) + 4*half + r%4 of column col.
__device__ __forceinline__ void store_tile(const GemmArgs& g, const double (&acc64)[16], int64_t row0, int half,
                                           int64_t col) {
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    if (g.mode == kCombine3M) {
        // this product is T3 of the 3-real-product form; one entry per register
        if (col >= g.n) return;
        const int32_t f = g.FB[col];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t i = row0 + 8 * (r >> 2) + 4 * half + (r & 3);
            if (i >= g.m) continue;
            const int32_t e = g.EA[i];
            const double t3 = (e == kNonFiniteExp || f == kNonFiniteExp) ? nan : ldexp(acc64[r], e + f);
            const double t1 = g.t1[i + col * g.ldt], t2 = g.t2[i + col * g.ldt];
            const double cr = t1 - t2;
            const double ci = (t3 - t1) - t2;
            double* c = g.C + 2 * (i + col * g.ldc);
            double outr = g.alpha_r * cr - g.alpha_i * ci;
            double outi = g.alpha_r * ci + g.alpha_i * cr;
            if (!g.beta_zero) {
                const double c0 = c[0], c1 = c[1];
                outr = outr + (g.beta_r * c0 - g.beta_i * c1);
                outi = outi + (g.beta_r * c1 + g.beta_i * c0);
            }
            c[0] = outr;
            c[1] = outi;
        }
        return;
    }
    if (g.mode != kFinal) {
        // raw tile sums in C' space (every padded row and column is stored)
#pragma unroll
        for (int r = 0; r < 16; ++r) g.acc[col * g.Mp + row0 + 8 * (r >> 2) + 4 * half + (r & 3)] = acc64[r];
        if (g.mode != kRawWriteFinal && g.mode != kRawAddFinal) return;
    }
    if (col >= g.n) return;
    const int32_t f = g.FB[col];
    if (!g.cplx) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t i = row0 + 8 * (r >> 2) + 4 * half + (r & 3);
            if (i >= g.m) continue;
            const int32_t e = g.EA[i];
            double* c = g.C + i + col * g.ldc;
            double out;
            if (e == kNonFiniteExp || f == kNonFiniteExp) {
                out = nan;
            } else {
                const double v = ldexp(acc64[r], e + f);
                out = g.alpha_r * v;
                if (!g.beta_zero) out = out + g.beta_r * (*c);
            }
            *c = out;
        }
    } else {
        // 32 C' rows = 16 complex rows; register r (r%8 < 4) holds the real part
        // and r + 4 the imaginary part of complex row row0/2 + 8*(r/8) + 4*half + r%4
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if ((r & 4) != 0) continue;
            const int64_t ci = row0 / 2 + 8 * (r >> 3) + 4 * half + (r & 3);
            if (ci >= g.m) continue;
            const int32_t e = g.EA[ci];
            double* c = g.C + 2 * (ci + col * g.ldc);
            double outr, outi;
            if (e == kNonFiniteExp || f == kNonFiniteExp) {
                outr = outi = nan;
            } else {
                const double vr = ldexp(acc64[r], e + f);
                const double vi = ldexp(acc64[r + 4], e + f);
                outr = g.alpha_r * vr - g.alpha_i * vi;
                outi = g.alpha_r * vi + g.alpha_i * vr;
                if (!g.beta_zero) {
                    const double cr = c[0], cim = c[1];
                    outr = outr + (g.beta_r * cr - g.beta_i * cim);
                    outi = outi + (g.beta_r * cim + g.beta_i * cr);
                }
            }
            c[0] = outr;
            c[1] = outi;
        }
    }
}

// (hi, lo) + x for an exactly representable x (a diagonal sum times a power
// of two): TwoSum of hi and x, its error added to lo, then renormalised by a
// fast TwoSum.  Exact while the running sum spans fewer than about 100 bits.
__device__ __forceinline__ void dd_add_exact(double& hi, double& lo, double x) {
    const double s = hi + x;
    const double bb = s - hi;
    const double err = (hi - (s - bb)) + (x - bb);
    const double t = lo + err;
    hi = s + t;
    lo = t - (hi - s);
}

// Epilogue of kFinalDD: C = ldexp(hi, E_i + F_j), c_lo = ldexp(lo, E_i + F_j)
// (NaN in both where a scale marks Inf/NaN input); layout as store_tile.
__device__ __forceinline__ void store_tile_dd(const GemmArgs& g, const double (&hi)[16], const double (&lo)[16],
                                              int64_t row0, int half, int64_t col) {
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    if (col >= g.n) return;
    const int32_t f = g.FB[col];
    if (!g.cplx) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t i = row0 + 8 * (r >> 2) + 4 * half + (r & 3);
            if (i >= g.m) continue;
            const int32_t e = g.EA[i];
            const bool bad = e == kNonFiniteExp || f == kNonFiniteExp;
            g.C[i + col * g.ldc] = bad ? nan : ldexp(hi[r], e + f);
            g.c_lo[i + col * g.ldc] = bad ? nan : ldexp(lo[r], e + f);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if ((r & 4) != 0) continue;
            const int64_t ci = row0 / 2 + 8 * (r >> 3) + 4 * half + (r & 3);
            if (ci >= g.m) continue;
            const int32_t e = g.EA[ci];
            const bool bad = e == kNonFiniteExp || f == kNonFiniteExp;
            double* ch = g.C + 2 * (ci + col * g.ldc);
            double* cl = g.c_lo + 2 * (ci + col * g.ldc);
            ch[0] = bad ? nan : ldexp(hi[r], e + f);
            ch[1] = bad ? nan : ldexp(hi[r + 4], e + f);
            cl[0] = bad ? nan : ldexp(lo[r], e + f);
            cl[1] = bad ? nan : ldexp(lo[r + 4], e + f);
        }
    }
}

// TM: 32-row MFMA tiles per wave along M (1 or 2).  With TM = 2 a wave owns
// a 64 x 32 sub-tile and every B fragment read from LDS feeds two MFMAs, so
// the block reads 3s instead of 4s fragments per 2 s(s+1)/2 products and the
// ring carries fewer bytes per MFMA.
template <int S, int WMW, int WNW, int NST, int TM = 1>
struct TileCfg {
    static constexpr int BM = 32 * WMW * TM, BN = 32 * WNW;
    static constexpr int NW = WMW * WNW;                     // waves per block
    static constexpr int RA = 2 * S * (BM / 64);             // 1 KiB runs of A per stage
    static constexpr int RB = 2 * S * (BN / 64);             // 1 KiB runs of B per stage
    static constexpr int R = RA + RB;
    static constexpr int A_CHUNKS = RA * 64;                 // 16-byte chunks
    static constexpr int STAGE = R * 64;
    static constexpr int RHI = (R + NW - 1) / NW;            // runs of waves w < R % NW (all if 0)
    static constexpr int RLO = R / NW;                       // runs of the other waves (may be 0)
    static_assert(BM % 64 == 0 && BN % 64 == 0, "block sides are multiples of 64");
};

// TOP: only the anti-diagonal d = S + 1 (pairs p + q = S + 1), the growth
// step S-1 -> S of a tolerance-driven call; otherwise all d = 2 .. S+1.
// One BM x BN tile (tile row tm, tile column tn) of the product described by g,
// staged through the caller's LDS ring lds[NST][STAGE].
// XD: fold into a double-double and write C_hi / C_lo (kFinalDD).
// OUT: hand the folded FP64 tile sums (before the scales) to the caller in
// out[16] instead of running the epilogue (one 32-row tile per wave, FP64 sums).
template <int S, int WMW, int WNW, int NST, bool TOP, bool DIAG, bool MULTI, bool XD = false, int TM = 1,
          bool OUT = false>
__device__ __forceinline__ void tile_body(const GemmArgs& g, int64_t tm, int64_t tn,
                                          v4i (*lds)[TileCfg<S, WMW, WNW, NST, TM>::STAGE], double* out = nullptr) {
    using T = TileCfg<S, WMW, WNW, NST, TM>;
    constexpr int DLO = TOP ? S - 1 : 0;  // lowest live diagonal index (d - 2)
    constexpr int ND = S - DLO;           // live INT32 diagonal tiles
    // two sub-tiles per wave keep twice the INT32 tiles live: not with the
    // chunked FP64 sums, the double-double fold or the diagonal export
    static_assert(TM == 1 || (TM == 2 && !MULTI && !XD && !DIAG), "TM = 2: single-chunk FP64 results only");
    static_assert(!OUT || (TM == 1 && !XD && !DIAG && !TOP), "OUT: one tile per wave, all diagonals, FP64 sums");

    // the wave index is uniform: kept in a scalar register, the copy addresses
    // below are scalar arithmetic off the vector pipe
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WNW, wn = wave % WNW;
    const int half = lane >> 5, row = lane & 31;
    const v4i* SA = reinterpret_cast<const v4i*>(g.SA);
    const v4i* SB = reinterpret_cast<const v4i*>(g.SB);
    const int64_t nsteps = g.kpad / kStep;

    // Stage of step ks -> LDS buffer: run j (< R) of the stage is moved by wave
    // j % NW.  A run j < RA is (h*S + p) = j / (BM/64), 64-row block j % (BM/64);
    // a B run likewise.  LDS holds A as [h*S + p][BM rows] and B as
    // [h*S + p][BN cols], 16 bytes each.  LDS plane hp = h*S + p of step ks
    // comes from global plane (2*ks + h)*s_lay + p: stages are issued in step
    // order, so each run keeps a uniform source pointer that advances by
    // 2*s_lay planes per issue.
    const v4i* run_src[T::RHI];
    const int64_t adv_a = 2 * g.s_lay * g.Mp, adv_b = 2 * g.s_lay * g.Np;  // per issue, A runs / B runs
#pragma unroll
    for (int i = 0; i < T::RHI; ++i) {
        const int j = wave + T::NW * i;  // wave-uniform
        run_src[i] = SA;
        if (j >= T::R) continue;
        if (j < T::RA) {
            const int hp = j / (T::BM / 64), rb = j % (T::BM / 64);
            run_src[i] = SA + (static_cast<int64_t>(hp / S) * g.s_lay + hp % S) * g.Mp + tm * T::BM + rb * 64;
        } else {
            const int jb = j - T::RA;
            const int hp = jb / (T::BN / 64), cb = jb % (T::BN / 64);
            run_src[i] = SB + (static_cast<int64_t>(hp / S) * g.s_lay + hp % S) * g.Np + tn * T::BN + cb * 64;
        }
    }
    auto issue = [&](int buf) {
#pragma unroll
        for (int i = 0; i < T::RHI; ++i) {
            const int j = wave + T::NW * i;  // wave-uniform
            if (j >= T::R) break;
            __builtin_amdgcn_global_load_lds((global_cvoid*)(run_src[i] + lane), (lds_void*)(&lds[buf][j * 64]), 16,
                                             0, 0);
            run_src[i] += j < T::RA ? adv_a : adv_b;
        }
    };
    // all but the newest stage's copies of this wave have landed
    // Wait until the oldest stage in flight has landed while the `younger`
    // (0 .. NST-2) stages issued after it may still fly; copies retire in
    // issue order, and each stage is RHI or RLO copies of this wave.
    auto wait_stage = [&](int64_t younger) {
        const bool hi = T::R % T::NW == 0 || wave < T::R % T::NW;
        if (NST > 3 && younger >= 2) {
            if (hi) wait_vm<(NST > 3 ? 2 : 0) * T::RHI>();
            else wait_vm<(NST > 3 ? 2 : 0) * T::RLO>();
        } else if (NST > 2 && younger >= 1) {
            if (hi) wait_vm<T::RHI>();
            else wait_vm<T::RLO>();
        } else {
            wait_vm<0>();
        }
    };

    v16i acc[TM][ND];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][d][r] = 0;

    // first C' row of the wave's sub-tile i
    const int64_t row0 = tm * T::BM + wm * 32 * TM;
    const int64_t col = tn * T::BN + wn * 32 + row;
    // FP64 tile: 0, or the raw sums of the previous slice count (kRawAdd)
    auto init64 = [&](double (&a64)[16], int64_t r0) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            a64[r] = (!OUT && (g.mode == kRawAdd || g.mode == kRawAddFinal))
                         ? g.acc[col * g.Mp + r0 + 8 * (r >> 2) + 4 * half + (r & 3)]
                         : 0.0;
    };
    double acc64[16];
    double lo64[XD ? 16 : 1];
    if constexpr (MULTI) init64(acc64, row0);
    if constexpr (XD)
#pragma unroll
        for (int r = 0; r < 16; ++r) lo64[r] = 0.0;

    // prologue: stages 0 .. NST-2 in flight; stage 0 landed, the others may fly
#pragma unroll
    for (int st = 0; st < NST - 1; ++st)
        if (st < nsteps) issue(st);
    wait_stage((nsteps - 1 < NST - 2) ? nsteps - 1 : NST - 2);
    __syncthreads();

    int64_t chunk_pos = 0, chunk = 0;
    // one step on ring buffer BUF (a compile-time index, so that every LDS
    // read is a fixed register plus an immediate offset)
    auto step = [&](int64_t ks, auto bufc) {
        constexpr int BUF = decltype(bufc)::value;
        const bool more = ks + NST - 1 < nsteps;
        if (more) issue((BUF + NST - 1) % NST);
        const v4i* L = lds[BUF];
        v4i bq[S];
#pragma unroll
        for (int q = 0; q < S; ++q) bq[q] = L[T::A_CHUNKS + (half * S + q) * T::BN + wn * 32 + row];
#pragma unroll
        for (int p = 0; p < S; ++p) {
            v4i a[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = L[(half * S + p) * T::BM + (wm * TM + i) * 32 + row];
#pragma unroll
            for (int q = (DLO > p ? DLO - p : 0); q < S - p; ++q)
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    acc[i][p + q - DLO] =
                        __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], bq[q], acc[i][p + q - DLO], 0, 0, 0);
        }
        if constexpr (MULTI || DIAG) {
            if (++chunk_pos == g.chunk_steps || ks + 1 == nsteps) {
                if constexpr (DIAG) {
#pragma unroll
                    for (int d = 0; d < ND; ++d)
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            g.diag_out[((chunk * S + d + DLO) * g.Np + col) * g.Mp + row0 + 8 * (r >> 2) +
                                       4 * half + (r & 3)] = acc[0][d][r];
                } else if constexpr (XD) {
                    fold_diags_dd<ND, DLO, S - 1>(acc64, lo64, acc[0], g.bal);
                } else {
                    fold_diags<ND, DLO, S - 1>(acc64, acc[0], g.bal);
                }
#pragma unroll
                for (int d = 0; d < ND; ++d)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[0][d][r] = 0;
                chunk_pos = 0;
                ++chunk;
            }
        }
        // the stage of step ks + 1 must have landed before the barrier; the
        // stages issued after it (up to ks + NST - 1) may still fly
        {
            const int64_t after = nsteps - ks - 2;  // stages that exist after ks + 1
            wait_stage(after < NST - 2 ? (after > 0 ? after : 0) : NST - 2);
        }
        ring_barrier();
    };
    static_assert(NST >= 2 && NST <= 4, "ring of 2 to 4 stages");
    for (int64_t ks = 0; ks < nsteps; ks += NST) {
        step(ks, std::integral_constant<int, 0>{});
        if (ks + 1 < nsteps) step(ks + 1, std::integral_constant<int, 1>{});
        if constexpr (NST >= 3)
            if (ks + 2 < nsteps) step(ks + 2, std::integral_constant<int, 2>{});
        if constexpr (NST >= 4)
            if (ks + 3 < nsteps) step(ks + 3, std::integral_constant<int, 3>{});
    }
    if constexpr (DIAG) return;
    if constexpr (OUT) {
        if constexpr (!MULTI) {
            init64(acc64, row0);
            fold_diags<ND, DLO, S - 1>(acc64, acc[0], g.bal);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) out[r] = acc64[r];
        return;
    }
    if constexpr (MULTI || XD) {
        if constexpr (!MULTI) {
            init64(acc64, row0);
            fold_diags_dd<ND, DLO, S - 1>(acc64, lo64, acc[0], g.bal);
        }
        if constexpr (XD)
            store_tile_dd(g, acc64, lo64, row0, half, col);
        else
            store_tile(g, acc64, row0, half, col);
    } else {
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            init64(acc64, row0 + 32 * i);
            fold_diags<ND, DLO, S - 1>(acc64, acc[i], g.bal);
            store_tile(g, acc64, row0 + 32 * i, half, col);
        }
    }
}

template <int S, int WMW, int WNW, int NST, bool TOP, bool DIAG, bool MULTI, int TM = 1>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * WMW * WNW, 64 * WMW * WNW),
                          amdgpu_waves_per_eu(2, 2))) void gemm_kernel(GemmArgs g) {
    using T = TileCfg<S, WMW, WNW, NST, TM>;
    __shared__ v4i lds[NST][T::STAGE];
    int64_t tm, tn;
    tile_of_block(blockIdx.x, g.Mp / T::BM, g.Np / T::BN, tm, tn);
    tile_body<S, WMW, WNW, NST, TOP, DIAG, MULTI, false, TM>(g, tm, tn, lds);
}

// Wide form for 9 <= s <= kMaxWideSlices: the same tile body on a 64 x 64
// block with a 2-stage ring at one wave per SIMD, which gives each wave the
// 512 registers that s INT32 diagonal tiles need (one block per CU).
template <int S, bool TOP, bool DIAG, bool MULTI, bool XD>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1))) void gemm_wide_kernel(
    GemmArgs g) {
    using T = TileCfg<S, 2, 2, 2>;
    __shared__ v4i lds[2][T::STAGE];
    int64_t tm, tn;
    tile_of_block(blockIdx.x, g.Mp / T::BM, g.Np / T::BN, tm, tn);
    tile_body<S, 2, 2, 2, TOP, DIAG, MULTI, XD>(g, tm, tn, lds);
}

// Tile list walk of a persistent block: tiles b, b + gridDim.x, ...; the next
// item is loaded while the current tile runs, so its load is off the path
// between tiles.  Padding items (problem -1) are skipped.
template <class F>
__device__ __forceinline__ void for_each_item(const TileItem* __restrict__ items, int64_t nitems, F&& f) {
    int64_t it = blockIdx.x;
    if (it >= nitems) return;
    TileItem ti = items[it];
    for (; it < nitems; it += gridDim.x) {
        const int64_t nx = it + gridDim.x;
        const TileItem next = nx < nitems ? items[nx] : TileItem{-1, 0, 0, 0};
        if (ti.prob >= 0) f(ti);  // uniform over the block
        ti = next;
    }
}

// Persistent form for a batch: block b takes tiles b, b + gridDim.x, ... of the
// tile list; a tile names its problem (a GemmArgs in device memory) and its
// tile row and column (problem -1: a padding item, skipped).  Every problem of
// one launch has the same s; MULTI is
// set when any problem of the launch spans more than one INT32 chunk.
template <int S, int WMW, int WNW, int NST, bool TOP, bool MULTI, int TM = 1>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * WMW * WNW, 64 * WMW * WNW),
                          amdgpu_waves_per_eu(2, 2))) void gemm_persistent_kernel(const GemmArgs* __restrict__ probs,
                                                                                  const TileItem* __restrict__ items,
                                                                                  int64_t nitems) {
    using T = TileCfg<S, WMW, WNW, NST, TM>;
    __shared__ v4i lds[NST][T::STAGE];
    for_each_item(items, nitems, [&](const TileItem& ti) {
        tile_body<S, WMW, WNW, NST, TOP, false, MULTI, false, TM>(probs[ti.prob], ti.tm, ti.tn, lds);
        __syncthreads();  // the next tile refills the LDS ring
    });
}

// Persistent form over tiles of problems with different slice counts (all
// s <= kMaxLiveSlices): each tile runs the 64 x 64 all-diagonal body of its own
// problem's s, so one launch covers a whole round of a heterogeneous batch
// instead of one launch (and one tail) per slice count.  The 2-stage LDS ring
// is sized for the largest s; a tile of smaller s uses a prefix of it.
template <int S, bool TOP, bool MULTI>
__device__ __forceinline__ void mixed_tile(const GemmArgs& g, const TileItem& ti, v4i* lds) {
    using T = TileCfg<S, 2, 2, 2>;
    tile_body<S, 2, 2, 2, TOP, false, MULTI>(g, ti.tm, ti.tn, reinterpret_cast<v4i(*)[T::STAGE]>(lds));
}

// Every tile takes the chunked body (the FP64 fold at each chunk end, for one
// chunk once after the last step -- the same additions in the same order as
// the fold after the loop): with the fold after the loop the s = 7, 8 bodies of
// this one function spilled about 110 registers to scratch (measured: the
// tolerance-driven batches ran 3% faster without the spills).
// A tile item whose s carries kTwoTileItem is a 128 x 64 tile of two-tile
// waves (s <= 6, one INT32 chunk): half the tiles of the 64 x 64 form, and
// each B fragment read from LDS feeds two MFMAs.
template <int S, bool TOP>
__device__ __forceinline__ void mixed_tile2(const GemmArgs& g, const TileItem& ti, v4i* lds) {
    using T = TileCfg<S, 2, 2, 2, 2>;
    tile_body<S, 2, 2, 2, TOP, false, false, false, 2>(g, ti.tm, ti.tn, reinterpret_cast<v4i(*)[T::STAGE]>(lds));
}

template <bool TOP, bool MULTI>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2))) void
gemm_persistent_mixed_kernel(const GemmArgs* __restrict__ probs, const TileItem* __restrict__ items, int64_t nitems) {
    constexpr int kLds1 = 2 * TileCfg<kMaxLiveSlices, 2, 2, 2>::STAGE, kLds2 = 2 * TileCfg<6, 2, 2, 2, 2>::STAGE;
    __shared__ v4i lds[kLds1 > kLds2 ? kLds1 : kLds2];
    for_each_item(items, nitems, [&](const TileItem& ti) {
        const GemmArgs& g = probs[ti.prob];
        if (ti.s & kTwoTileItem) {
            switch (ti.s & ~kTwoTileItem) {  // uniform over the block
                case 1: mixed_tile2<1, TOP>(g, ti, lds); break;
                case 2: mixed_tile2<2, TOP>(g, ti, lds); break;
                case 3: mixed_tile2<3, TOP>(g, ti, lds); break;
                case 4: mixed_tile2<4, TOP>(g, ti, lds); break;
                case 5: mixed_tile2<5, TOP>(g, ti, lds); break;
                default: mixed_tile2<6, TOP>(g, ti, lds); break;
            }
            __syncthreads();  // the next tile refills the LDS ring
            return;
        }
        switch (ti.s) {  // the tile's slice count, uniform over the block
            case 1: mixed_tile<1, TOP, true>(g, ti, lds); break;
            case 2: mixed_tile<2, TOP, true>(g, ti, lds); break;
            case 3: mixed_tile<3, TOP, true>(g, ti, lds); break;
            case 4: mixed_tile<4, TOP, true>(g, ti, lds); break;
            case 5: mixed_tile<5, TOP, true>(g, ti, lds); break;
            case 6: mixed_tile<6, TOP, true>(g, ti, lds); break;
            case 7: mixed_tile<7, TOP, true>(g, ti, lds); break;
            default: mixed_tile<8, TOP, true>(g, ti, lds); break;
        }
        __syncthreads();  // the next tile refills the LDS ring
    });
}

// Persistent form of the wide all-diagonal tile (9 <= s <= kMaxWideSlices, one
// wave per SIMD), for batched problems above the 2-waves-per-SIMD budget; like
// the mixed form, each tile runs at its own problem's s, within the launch's
// range LO..HI.  The ranges are what one function holds without spilling
// (measured): 9..12 and 13..14 with one INT32 chunk, 9..11 and 12 with several
// (several chunks at s >= 13 take the streaming body).  A single instance over
// 9..14 spilled 63 registers to scratch.
template <int K, int HI, bool TOP, bool MULTI>
__device__ __forceinline__ void wide_tile(int s, const GemmArgs& g, const TileItem& ti, v4i* lds) {
    if constexpr (K < HI) {
        if (s == K) mixed_tile<K, TOP, MULTI>(g, ti, lds);
        else wide_tile<K + 1, HI, TOP, MULTI>(s, g, ti, lds);
    } else {
        mixed_tile<HI, TOP, MULTI>(g, ti, lds);
    }
}

template <bool TOP, bool MULTI, int LO, int HI>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1))) void
gemm_wide_persistent_kernel(const GemmArgs* __restrict__ probs, const TileItem* __restrict__ items, int64_t nitems) {
    __shared__ v4i lds[2 * TileCfg<HI, 2, 2, 2>::STAGE];
    for_each_item(items, nitems, [&](const TileItem& ti) {
        wide_tile<LO, HI, TOP, MULTI>(ti.s, probs[ti.prob], ti, lds);  // ti.s uniform over the block
        __syncthreads();
    });
}

// Fused 3-real-product tile of a complex product (s <= kMaxLiveSlices, each
// tile its own s): the three real products T1 = Ar Br, T2 = Ai Bi and
// T3 = (Ar + Ai)(Br + Bi) of one 64 x 64 tile run back to back through the same
// LDS ring, T1 and T2 kept in registers as scaled FP64 values, and the
// epilogue forms Cr = T1 - T2, Ci = (T3 - T1) - T2 and alpha, beta -- the
// bits of three separate launches with the combine in the last one, without
// writing T1 and T2 to memory.  g3[0..2] describe T1, T2, T3 (real products
// over the real slice layouts; C, alpha, beta in g3[2]).
__device__ __forceinline__ double scaled_part(const GemmArgs& g, double v, int64_t i, int64_t col) {
    const int32_t e = g.EA[i], f = g.FB[col];
    return (e == kNonFiniteExp || f == kNonFiniteExp) ? __longlong_as_double(0x7ff8000000000000ll)
                                                      : ldexp(v, e + f);
}

// The chunked body folds the INT32 tiles into the FP64 tile at every chunk end
// (for one chunk: once, after the last step), which keeps fewer registers live
// at the end than a fold after the loop.
template <int S>
__device__ __forceinline__ void fused3_tile(const GemmArgs* g3, const TileItem& ti, v4i* lds) {
    using T = TileCfg<S, 2, 2, 2>;
    auto L = reinterpret_cast<v4i(*)[T::STAGE]>(lds);
    double t1[16], t2[16], t3[16];
    tile_body<S, 2, 2, 2, false, false, true, false, 1, true>(g3[0], ti.tm, ti.tn, L, t1);
    __syncthreads();  // the next product refills the ring
    tile_body<S, 2, 2, 2, false, false, true, false, 1, true>(g3[1], ti.tm, ti.tn, L, t2);
    __syncthreads();
    tile_body<S, 2, 2, 2, false, false, true, false, 1, true>(g3[2], ti.tm, ti.tn, L, t3);
    const GemmArgs& g = g3[2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int64_t row0 = ti.tm * 64 + (wave >> 1) * 32;
    const int64_t col = ti.tn * 64 + (wave & 1) * 32 + (lane & 31);
    if (col >= g.n) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t i = row0 + 8 * (r >> 2) + 4 * half + (r & 3);
        if (i >= g.m) continue;
        const double T1 = scaled_part(g3[0], t1[r], i, col), T2 = scaled_part(g3[1], t2[r], i, col);
        const double T3 = scaled_part(g, t3[r], i, col);
        const double cr = T1 - T2;
        const double ci = (T3 - T1) - T2;
        double* c = g.C + 2 * (i + col * g.ldc);
        double outr = g.alpha_r * cr - g.alpha_i * ci;
        double outi = g.alpha_r * ci + g.alpha_i * cr;
        if (!g.beta_zero) {
            const double c0 = c[0], c1 = c[1];
            outr = outr + (g.beta_r * c0 - g.beta_i * c1);
            outi = outi + (g.beta_r * c1 + g.beta_i * c0);
        }
        c[0] = outr;
        c[1] = outi;
    }
}

// Persistent form over fused 3-product tiles (item.prob indexes the first of
// the problem's three descriptors; each tile at its own s).  HI = 6: s = 1..6
// at two waves per SIMD; HI = 8: s = 7, 8, whose INT32 tiles plus T1 and T2
// need the registers of one wave per SIMD (one block per CU).
template <int HI>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(HI <= 6 ? 2 : 1, HI <= 6 ? 2 : 1)))
void gemm_persistent_3m_kernel(const GemmArgs* __restrict__ probs, const TileItem* __restrict__ items,
                               int64_t nitems) {
    __shared__ v4i lds[2 * TileCfg<HI, 2, 2, 2>::STAGE];
    for_each_item(items, nitems, [&](const TileItem& ti) {
        const GemmArgs* g3 = probs + ti.prob;
        if constexpr (HI <= 6) {
            switch (ti.s) {  // uniform over the block
                case 1: fused3_tile<1>(g3, ti, lds); break;
                case 2: fused3_tile<2>(g3, ti, lds); break;
                case 3: fused3_tile<3>(g3, ti, lds); break;
                case 4: fused3_tile<4>(g3, ti, lds); break;
                case 5: fused3_tile<5>(g3, ti, lds); break;
                default: fused3_tile<6>(g3, ti, lds); break;
            }
        } else {
            if (ti.s == 7) fused3_tile<7>(g3, ti, lds);
            else fused3_tile<8>(g3, ti, lds);
        }
        __syncthreads();  // the next tile refills the LDS ring
    });
}

// Streaming form for any s (used above the all-diagonal kernel's register
// budget, s > kMaxLiveSlices): one INT32 tile, one anti-diagonal at a time.
// For each INT32 chunk and each d = s+1 down to 2, the pairs (p, d-p) of that
// diagonal are streamed step by step (one A slice and one B slice, 4 KiB per
// stage, double buffered) into the INT32 tile, which is then folded into the
// FP64 tile -- the same order as the all-diagonal kernel, hence the same bits.
// 64 x 64 block tile, 4 waves.
template <bool DIAG>
__device__ __forceinline__ void stream_body(const GemmArgs& g, int s, int top, int64_t tm, int64_t tn,
                                            v4i (*lds)[256]) {
    // lds: [A: h*64 + row | B: 128 + h*64 + col]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int half = lane >> 5, row = lane & 31;
    const v4i* SA = reinterpret_cast<const v4i*>(g.SA);
    const v4i* SB = reinterpret_cast<const v4i*>(g.SB);
    const int64_t nsteps = g.kpad / kStep;
    const int64_t row0 = tm * 64 + wm * 32;
    const int64_t col = tn * 64 + wn * 32 + row;

    // wave 0/1: A half 0/1 of slice p; wave 2/3: B half 0/1 of slice q
    auto issue = [&](int64_t ks, int p, int q, int buf) {
        const int h = wave & 1;
        const v4i* src = (wave < 2) ? SA + ((2 * ks + h) * g.s_lay + (p - 1)) * g.Mp + tm * 64 + lane
                                    : SB + ((2 * ks + h) * g.s_lay + (q - 1)) * g.Np + tn * 64 + lane;
        __builtin_amdgcn_global_load_lds((global_cvoid*)(src), (lds_void*)(&lds[buf][wave * 64]), 16, 0, 0);
    };

    double acc64[16], lo64[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc64[r] = (g.mode == kRawAdd || g.mode == kRawAddFinal)
                       ? g.acc[col * g.Mp + row0 + 8 * (r >> 2) + 4 * half + (r & 3)]
                       : 0.0;
        lo64[r] = 0.0;
    }
    const bool dd = g.mode == kFinalDD;
    const int64_t nchunks = (nsteps + g.chunk_steps - 1) / g.chunk_steps;
    const int dmin = top ? s + 1 : 2;
    for (int64_t c = 0; c < nchunks; ++c) {
        const int64_t k0 = c * g.chunk_steps;
        const int64_t k1 = (k0 + g.chunk_steps < nsteps) ? k0 + g.chunk_steps : nsteps;
        for (int d = s + 1; d >= dmin; --d) {
            const int plo = (d - s > 1) ? d - s : 1;
            const int phi = (d - 1 < s) ? d - 1 : s;
            const int np = phi - plo + 1;
            const int64_t items = static_cast<int64_t>(np) * (k1 - k0);
            v16i acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0;
            issue(k0, plo, d - plo, 0);
            wait_vm<0>();
            __syncthreads();
            for (int64_t it = 0; it < items; ++it) {
                const int buf = static_cast<int>(it & 1);
                if (it + 1 < items) {
                    const int p1 = plo + static_cast<int>((it + 1) % np);
                    issue(k0 + (it + 1) / np, p1, d - p1, buf ^ 1);
                }
                const v4i a = lds[buf][half * 64 + wm * 32 + row];
                const v4i b = lds[buf][128 + half * 64 + wn * 32 + row];
                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc, 0, 0, 0);
                wait_vm<0>();
                __syncthreads();
            }
            if constexpr (DIAG) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    g.diag_out[((c * s + (d - 2)) * g.Np + col) * g.Mp + row0 + 8 * (r >> 2) + 4 * half + (r & 3)] =
                        acc[r];
            } else if (dd) {
                const double sc = ldexp(1.0, diag_exp(d, g.bal));  // exact power of two
#pragma unroll
                for (int r = 0; r < 16; ++r) dd_add_exact(acc64[r], lo64[r], static_cast<double>(acc[r]) * sc);
            } else {
                const double sc = ldexp(1.0, diag_exp(d, g.bal));  // exact power of two
#pragma unroll
                for (int r = 0; r < 16; ++r) acc64[r] = acc64[r] + static_cast<double>(acc[r]) * sc;
            }
        }
    }
    if constexpr (DIAG) return;
    if (dd)
        store_tile_dd(g, acc64, lo64, row0, half, col);
    else
        store_tile(g, acc64, row0, half, col);
}

template <bool DIAG>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256))) void gemm_stream_kernel(GemmArgs g) {
    __shared__ v4i lds[2][256];
    int64_t tm, tn;
    tile_of_block(blockIdx.x, g.Mp / 64, g.Np / 64, tm, tn);
    stream_body<DIAG>(g, g.s, g.top, tm, tn, lds);
}

// Batched streaming form: a persistent grid walking 64 x 64 tiles of many
// problems, all at slice count s (top: only the anti-diagonal s + 1).
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256))) void gemm_stream_persistent_kernel(
    const GemmArgs* __restrict__ probs, const TileItem* __restrict__ items, int64_t nitems, int s, int top) {
    __shared__ v4i lds[2][256];
    for_each_item(items, nitems, [&](const TileItem& ti) {
        stream_body<false>(probs[ti.prob], s, top, ti.tm, ti.tn, lds);
        __syncthreads();
    });
}

__global__ void scale_c_kernel(double* C, int64_t ldc, int64_t m, int64_t n, int cplx, double br, double bi,
                               int beta_zero) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        if (!cplx) {
            double* c = C + i + j * ldc;
            *c = beta_zero ? 0.0 : br * (*c);
        } else {
            double* c = C + 2 * (i + j * ldc);
            if (beta_zero) {
                c[0] = 0.0;
                c[1] = 0.0;
            } else {
                const double cr = c[0], cim = c[1];
                c[0] = br * cr - bi * cim;
                c[1] = br * cim + bi * cr;
            }
        }
    }
}

template <int S, int WMW, int WNW, int NST>
hipError_t launch_cfg(const GemmArgs& g, hipStream_t st) {
    using T = TileCfg<S, WMW, WNW, NST>;
    const int64_t blocks = (g.Np / T::BN) * (g.Mp / T::BM);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(blocks)), block(64 * T::NW);
    const bool multi = g.chunk_steps < g.kpad / kStep;
    if (g.diag_out && !g.top)
        hipLaunchKernelGGL((gemm_kernel<S, WMW, WNW, NST, false, true, true>), grid, block, 0, st, g);
    else if (g.diag_out)
        hipLaunchKernelGGL((gemm_kernel<S, WMW, WNW, NST, true, true, true>), grid, block, 0, st, g);
    else if (g.top && multi)
        hipLaunchKernelGGL((gemm_kernel<S, WMW, WNW, NST, true, false, true>), grid, block, 0, st, g);
    else if (g.top)
        hipLaunchKernelGGL((gemm_kernel<S, WMW, WNW, NST, true, false, false>), grid, block, 0, st, g);
    else if (multi)
        hipLaunchKernelGGL((gemm_kernel<S, WMW, WNW, NST, false, false, true>), grid, block, 0, st, g);
    else
        hipLaunchKernelGGL((gemm_kernel<S, WMW, WNW, NST, false, false, false>), grid, block, 0, st, g);
    return hipGetLastError();
}

template <int S, int WMW, int WNW, int NST>
hipError_t launch_persistent_cfg(const GemmArgs* probs, const TileItem* items, int64_t nitems, int blocks, bool top,
                                 bool multi, hipStream_t st) {
    using T = TileCfg<S, WMW, WNW, NST>;
    dim3 grid(static_cast<unsigned>(blocks)), block(64 * T::NW);
#define OZ_PERSIST(TOPV, MULTIV)                                                                              \
    hipLaunchKernelGGL((gemm_persistent_kernel<S, WMW, WNW, NST, TOPV, MULTIV>), grid, block, 0, st, probs, \
                       items, nitems)
    if (top && multi) OZ_PERSIST(true, true);
    else if (top) OZ_PERSIST(true, false);
    else if (multi) OZ_PERSIST(false, true);
    else OZ_PERSIST(false, false);
#undef OZ_PERSIST
    return hipGetLastError();
}

// Ring depth of the 64 x 64 block of a single product: as deep as two blocks
// per CU allow in the 160 KiB of LDS (4 s KiB per stage), so that the copies
// of short steps (small s) get more than one step to land.  The persistent
// batch kernel keeps 2 stages: its tiles have few steps, and a deeper
// prologue costs more there than it hides (measured on the 512-problem batch).
constexpr int ring64(int s) { return s <= 4 ? 4 : (s <= 6 ? 3 : 2); }

template <int S>
hipError_t launch_persistent_s(const GemmArgs* probs, const TileItem* items, int64_t nitems, int blocks, int tile,
                               bool top, bool multi, hipStream_t st) {
    if (tile == 4) {
        // 128 x 64 blocks of two-tile waves: s <= 6, one INT32 chunk per problem
        if constexpr (S <= 6) {
            if (multi) return hipErrorInvalidValue;
            dim3 grid(static_cast<unsigned>(blocks)), block(256);
            if (top)
                hipLaunchKernelGGL((gemm_persistent_kernel<S, 2, 2, 2, true, false, 2>), grid, block, 0, st, probs,
                                   items, nitems);
            else
                hipLaunchKernelGGL((gemm_persistent_kernel<S, 2, 2, 2, false, false, 2>), grid, block, 0, st, probs,
                                   items, nitems);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (tile == 1) return launch_persistent_cfg<S, 4, 2, 3>(probs, items, nitems, blocks, top, multi, st);
    return launch_persistent_cfg<S, 2, 2, 2>(probs, items, nitems, blocks, top, multi, st);
}

// Blocks of two 32-row tiles per wave (single INT32 chunk, FP64 result):
// 128 x 64 with 4 waves, the ring as deep as two blocks per CU allow (6 s KiB
// per stage), or 128 x 128 with 8 waves (one block per CU, 8 s KiB per stage).
constexpr int ring128x64(int s) { return s <= 4 ? 3 : 2; }
constexpr int ring128x128(int s) { return s <= 6 ? 3 : 2; }

template <int S, int WMW, int WNW, int NST>
hipError_t launch_cfg_tm2(const GemmArgs& g, hipStream_t st) {
    using T = TileCfg<S, WMW, WNW, NST, 2>;
    const int64_t blocks = (g.Np / T::BN) * (g.Mp / T::BM);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(blocks)), block(64 * T::NW);
    if (g.top)
        hipLaunchKernelGGL((gemm_kernel<S, WMW, WNW, NST, true, false, false, 2>), grid, block, 0, st, g);
    else
        hipLaunchKernelGGL((gemm_kernel<S, WMW, WNW, NST, false, false, false, 2>), grid, block, 0, st, g);
    return hipGetLastError();
}

// Tiles of the 128 x 64 two-tile block from which it is the default: two
// blocks on every compute unit of the chip (smaller products keep the 64 x 64
// block, which has twice the tiles).
constexpr int64_t kTm2MinTiles = 512;

// Block shape by default: for s <= 6 with one INT32 chunk and at least
// kTm2MinTiles tiles, the 128 x 64 block of two-tile waves (tile 4; measured
// 8% faster than 64 x 64 on the ZGEMM n = 4096, s = 6 products); otherwise
// 64 x 64 with 4 waves of one tile each.  In both, two blocks share a CU, each
// with its own barrier, so the two waves on a SIMD drift apart and one keeps
// the matrix pipe busy while the other waits on LDS or the barrier (measured
// faster than one 128 x 64 block of 8 one-tile waves per CU -- tile 1, 3-stage
// ring -- from n = 1024 to 4096, and than the 128 x 128 block of 8 two-tile
// waves, tile 5).
template <int S>
hipError_t launch_s(const GemmArgs& g, hipStream_t st) {
    // two 32-row tiles per wave fit the 256 registers of two waves per SIMD
    // up to s = 6 (2 s INT32 tiles of 16 registers plus s B fragments)
    if constexpr (S <= 6) {
        const bool single = g.chunk_steps >= g.kpad / kStep && !g.diag_out;
        const bool big = (g.Mp / 128) * (g.Np / 64) >= kTm2MinTiles;
        if ((g.tile == 4 || (g.tile == 0 && big)) && single) return launch_cfg_tm2<S, 2, 2, ring128x64(S)>(g, st);
        if (g.tile == 5 && single) return launch_cfg_tm2<S, 2, 4, ring128x128(S)>(g, st);
    }
    if (g.tile == 1) return launch_cfg<S, 4, 2, 3>(g, st);
    return launch_cfg<S, 2, 2, ring64(S)>(g, st);
}

hipError_t launch_stream(const GemmArgs& g, hipStream_t st);

// Combinations whose INT32 tiles plus the FP64 (or double-double) chunk sums
// would spill registers go to the streaming kernel instead: several INT32
// chunks with s >= 13 (s >= 12 for a double-double result), and the chunked
// diagonal export with s = 14.
template <int S>
hipError_t launch_wide(const GemmArgs& g, hipStream_t st) {
    using T = TileCfg<S, 2, 2, 2>;
    const int64_t blocks = (g.Np / T::BN) * (g.Mp / T::BM);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(blocks)), block(256);
    const bool multi = g.chunk_steps < g.kpad / kStep;
#define OZ_WIDE(TOPV, DIAGV, MULTIV, XDV) \
    hipLaunchKernelGGL((gemm_wide_kernel<S, TOPV, DIAGV, MULTIV, XDV>), grid, block, 0, st, g)
    if (g.mode == kFinalDD) {
        if (!multi) {
            OZ_WIDE(false, false, false, true);
        } else {
            if constexpr (S <= 11) OZ_WIDE(false, false, true, true);
            else return launch_stream(g, st);
        }
    } else if (g.diag_out && !g.top) {
        if constexpr (S <= 13) OZ_WIDE(false, true, true, false);
        else return launch_stream(g, st);
    } else if (g.diag_out) {
        OZ_WIDE(true, true, true, false);
    } else if (g.top && multi) {
        OZ_WIDE(true, false, true, false);
    } else if (g.top) {
        OZ_WIDE(true, false, false, false);
    } else if (multi) {
        if constexpr (S <= 12) OZ_WIDE(false, false, true, false);
        else return launch_stream(g, st);
    } else {
        OZ_WIDE(false, false, false, false);
    }
#undef OZ_WIDE
    return hipGetLastError();
}

// Double-double results for s <= 8: the wide form as well (its XD variants only).
template <int S>
hipError_t launch_wide_xd(const GemmArgs& g, hipStream_t st) {
    using T = TileCfg<S, 2, 2, 2>;
    const int64_t blocks = (g.Np / T::BN) * (g.Mp / T::BM);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(blocks)), block(256);
    if (g.chunk_steps < g.kpad / kStep)
        hipLaunchKernelGGL((gemm_wide_kernel<S, false, false, true, true>), grid, block, 0, st, g);
    else
        hipLaunchKernelGGL((gemm_wide_kernel<S, false, false, false, true>), grid, block, 0, st, g);
    return hipGetLastError();
}

hipError_t launch_stream(const GemmArgs& g, hipStream_t st) {
    const int64_t blocks = (g.Np / 64) * (g.Mp / 64);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(blocks));
    if (g.diag_out)
        hipLaunchKernelGGL((gemm_stream_kernel<true>), grid, dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((gemm_stream_kernel<false>), grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& g, hipStream_t st) {
    if (g.s < 1 || g.s > 18 || g.s_lay < g.s) return hipErrorInvalidValue;
    const bool raw = g.mode == kRawWrite || g.mode == kRawAdd || g.mode == kRawWriteFinal || g.mode == kRawAddFinal;
    if (raw && g.acc == nullptr) return hipErrorInvalidValue;
    if (g.mode == kCombine3M && (g.t1 == nullptr || g.t2 == nullptr || g.cplx)) return hipErrorInvalidValue;
    if (g.mode == kFinalDD && (g.c_lo == nullptr || g.top)) return hipErrorInvalidValue;
    if (g.tile == 3) return launch_stream(g, st);
    if (g.mode == kFinalDD && g.s <= kMaxLiveSlices) {
        switch (g.s) {
            case 1: return launch_wide_xd<1>(g, st);
            case 2: return launch_wide_xd<2>(g, st);
            case 3: return launch_wide_xd<3>(g, st);
            case 4: return launch_wide_xd<4>(g, st);
            case 5: return launch_wide_xd<5>(g, st);
            case 6: return launch_wide_xd<6>(g, st);
            case 7: return launch_wide_xd<7>(g, st);
            default: return launch_wide_xd<8>(g, st);
        }
    }
    switch (g.s) {
        case 1: return launch_s<1>(g, st);
        case 2: return launch_s<2>(g, st);
        case 3: return launch_s<3>(g, st);
        case 4: return launch_s<4>(g, st);
        case 5: return launch_s<5>(g, st);
        case 6: return launch_s<6>(g, st);
        case 7: return launch_s<7>(g, st);
        case 8: return launch_s<8>(g, st);
        case 9: return launch_wide<9>(g, st);
        case 10: return launch_wide<10>(g, st);
        case 11: return launch_wide<11>(g, st);
        case 12: return launch_wide<12>(g, st);
        case 13: return launch_wide<13>(g, st);
        case 14: return launch_wide<14>(g, st);
        default: return launch_stream(g, st);
    }
}

hipError_t launch_gemm_persistent(const GemmArgs* probs, const TileItem* items, int64_t nitems, int s, int tile,
                                  int blocks, bool top, bool multi, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (blocks <= 0 || (tile != 1 && tile != 2 && tile != 4)) return hipErrorInvalidValue;
    switch (s) {
        case 1: return launch_persistent_s<1>(probs, items, nitems, blocks, tile, top, multi, st);
        case 2: return launch_persistent_s<2>(probs, items, nitems, blocks, tile, top, multi, st);
        case 3: return launch_persistent_s<3>(probs, items, nitems, blocks, tile, top, multi, st);
        case 4: return launch_persistent_s<4>(probs, items, nitems, blocks, tile, top, multi, st);
        case 5: return launch_persistent_s<5>(probs, items, nitems, blocks, tile, top, multi, st);
        case 6: return launch_persistent_s<6>(probs, items, nitems, blocks, tile, top, multi, st);
        case 7: return launch_persistent_s<7>(probs, items, nitems, blocks, tile, top, multi, st);
        case 8: return launch_persistent_s<8>(probs, items, nitems, blocks, tile, top, multi, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_persistent_mixed(const GemmArgs* probs, const TileItem* items, int64_t nitems, int blocks,
                                        bool top, bool multi, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (blocks <= 0) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(blocks)), block(256);
#define OZ_MIXED(TOPV, MULTIV) \
    hipLaunchKernelGGL((gemm_persistent_mixed_kernel<TOPV, MULTIV>), grid, block, 0, st, probs, items, nitems)
    (void)multi;  // every tile takes the chunked body
    if (top) OZ_MIXED(true, true);
    else OZ_MIXED(false, true);
#undef OZ_MIXED
    return hipGetLastError();
}

hipError_t launch_gemm_persistent_3m(const GemmArgs* probs, const TileItem* items, int64_t nitems, int blocks,
                                     bool high, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (blocks <= 0) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(blocks)), block(256);
    if (high)
        hipLaunchKernelGGL((gemm_persistent_3m_kernel<8>), grid, block, 0, st, probs, items, nitems);
    else
        hipLaunchKernelGGL((gemm_persistent_3m_kernel<6>), grid, block, 0, st, probs, items, nitems);
    return hipGetLastError();
}

hipError_t launch_gemm_wide_persistent(const GemmArgs* probs, const TileItem* items, int64_t nitems, int blocks,
                                       bool top, bool multi, int s_hi, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (blocks <= 0) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(blocks)), block(256);
#define OZ_WIDEP(TOPV, MULTIV, LO, HI) \
    hipLaunchKernelGGL((gemm_wide_persistent_kernel<TOPV, MULTIV, LO, HI>), grid, block, 0, st, probs, items, nitems)
#define OZ_WIDEP_RANGES(TOPV)                         \
    if (multi && s_hi == 11) OZ_WIDEP(TOPV, true, 9, 11); \
    else if (multi && s_hi == 12) OZ_WIDEP(TOPV, true, 12, 12); \
    else if (!multi && (s_hi == 11 || s_hi == 12)) OZ_WIDEP(TOPV, false, 9, 12); \
    else if (!multi && s_hi == 14) OZ_WIDEP(TOPV, false, 13, 14); \
    else return hipErrorInvalidValue;
    if (top) {
        OZ_WIDEP_RANGES(true)
    } else {
        OZ_WIDEP_RANGES(false)
    }
#undef OZ_WIDEP_RANGES
#undef OZ_WIDEP
    return hipGetLastError();
}

hipError_t launch_gemm_stream_persistent(const GemmArgs* probs, const TileItem* items, int64_t nitems, int s,
                                         bool top, int blocks, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (blocks <= 0 || s < 1 || s > 18) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemm_stream_persistent_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, probs,
                       items, nitems, s, top ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_scale_c(double* C, int64_t ldc, int64_t m, int64_t n, int cplx, double br, double bi,
                          int beta_zero, hipStream_t st) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>(n < 65535 ? n : 65535));
    hipLaunchKernelGGL(scale_c_kernel, grid, dim3(256), 0, st, C, ldc, m, n, cplx, br, bi, beta_zero);
    return hipGetLastError();
}

}  // namespace oz
