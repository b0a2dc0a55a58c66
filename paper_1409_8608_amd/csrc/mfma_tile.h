// Matrix-core contraction kernel for gfx950 (FP64 v_mfma_f64_16x16x4f64, FP32
// v_mfma_f32_16x16x4f32).  It runs the fused direct contraction (one launch,
// GEMM view M x N x K with arbitrary strides) and the gemm-shaped family
// members (batch = parallel loops, sequential passes = in-launch contracted
// loops, each pass reading and writing C).
//
// Operand staging: a BM x BK tile of A and a BK x BN tile of B go global ->
// registers -> LDS, double-buffered, one barrier per K tile.  Each tile is
// loaded with lanes along whichever index is contiguous in memory (M or K for
// A, N or K for B).  In LDS every row (one m of A, one n of B) holds its BK = 16
// contracted positions contiguously, in 16-byte chunks permuted per row so
// that fragment reads hit distinct banks.  Within a tile, lane group g = lane
// / 16 takes positions 4g .. 4g+3 in the four MFMA steps (both operands alike,
// so every position still meets its partner): a lane reads its fragment for
// all four steps with one (FP32) or two (FP64) 16-byte reads.  K is walked through a table of (A, B)
// offset pairs built by the planner in a blocked order in which A's and B's
// contiguous contracted indices both form runs; that handles any number of
// contracted indices and permuted strides with one kernel.
//
// The MFMA "row" operand is B (rows = n) and the "column" operand is A
// (columns = m), so each accumulator register holds 16 consecutive m of one n
// in 16 consecutive lanes:
// with C's unit stride along m the epilogue stores whole 128-byte (FP64) rows.
//
// Split-BF16 form (X3, batches): the same staging reads FP64 (or FP32)
// operands; a first sweep over K finds each row's (A) and column's (B)
// largest binary exponent e, so that the scaled values x = v 2^-e lie in
// (-2, 2).  Each staged value is then split into three BF16 terms by
// round-to-nearest-even at 8 significant bits (t1 = rn(x), t2 = rn(x - t1),
// t3 = rn(x - t1 - t2)) on its way to LDS, and the tile multiplies the six
// term products with p + q <= 4 on v_mfma_f32_16x16x16_bf16: the leading
// product in one FP32 accumulator, the other five in a second.  The epilogue
// adds the two in FP64 and unscales, C = alpha 2^(eA + eB) (big + small) +
// beta C.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "devutil.h"
#include "gett.h"

namespace tc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Accumulator layout of the 16x16x4 forms: lane l, register q holds column
// l % 16 of row 4*(l/16) + q for FP32, but row (l/16) + 4*q for FP64.
template <> struct Mfma<double> {
    typedef d4 acc_t;
    static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
    static __device__ __forceinline__ acc_t mac(double rowop, double colop, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(rowop, colop, c, 0, 0, 0);
    }
};
template <> struct Mfma<float> {
    typedef f4 acc_t;
    static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
    static __device__ __forceinline__ acc_t mac(float rowop, float colop, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(rowop, colop, c, 0, 0, 0);
    }
};

// LDS layout of a staged tile: row r holds positions 0..15 in 16-byte chunks;
// chunk c sits at c ^ f(r).  Chosen with an LDS read-pattern probe on MI355X
// for the fragment reads (16 consecutive rows per lane group, one chunk per
// group for FP32, two for FP64): both run as fast as a linear read, where the
// unpermuted rows take 1.5x (FP32) and 2.7x (FP64).
template <typename T> struct TileLds;
template <> struct TileLds<float> {
    static constexpr int CE = 4;   // elements per 16-byte chunk
    static __device__ __forceinline__ int swz(int r, int c) { return c ^ ((r >> 1) & 3); }
};
template <> struct TileLds<double> {
    static constexpr int CE = 2;
    static __device__ __forceinline__ int swz(int r, int c) { return c ^ ((((r >> 1) & 3) << 1) | ((r >> 3) & 1)); }
};
// element (row, k) of a staged tile with BK = 16
template <typename T>
__device__ __forceinline__ int tile_at(int r, int k) {
    constexpr int CE = TileLds<T>::CE;
    return r * 16 + TileLds<T>::swz(r, k / CE) * CE + (k % CE);
}

__device__ __forceinline__ int64_t dm(int64_t& rem, int64_t ext) {
    if ((uint64_t)rem <= 0xffffffffull && (uint64_t)ext <= 0xffffffffull) {
        uint32_t r = (uint32_t)rem, e = (uint32_t)ext;
        uint32_t q = r / e;
        rem = q;
        return (int64_t)(r - q * e);
    }
    int64_t q = rem / ext, m = rem - q * ext;
    rem = q;
    return m;
}


// s_waitcnt immediate that waits for LDS/scalar-memory traffic only (gfx9
// encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8; a field at its
// maximum does not wait).
constexpr int kWaitLgkm0 = 15 | (3 << 14) | (7 << 4);

// Block barrier for LDS hand-offs: this wave's LDS traffic is complete, then
// s_barrier.  Unlike __syncthreads it does not wait for outstanding global
// loads and stores, which stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// How a thread stages an operand tile: lanes along the free index (M-major),
// along K one element at a time, or along K in 16-byte chunks.
enum { LD_MMAJ = 0, LD_KSCAL = 1, LD_KVEC = 2 };

// offset of linear index `i` within a dimension group, for tensor slot 0 (A),
// 1 (B) or 2 (C)
template <int SLOT>
__device__ __forceinline__ int64_t group_off(const GtDims& g, int64_t i) {
    int64_t off = 0;
    for (int d = 0; d < g.n; ++d) {
        int64_t r = dm(i, g.d[d].ext);
        off += r * (SLOT == 0 ? g.d[d].sA : SLOT == 1 ? g.d[d].sB : g.d[d].sC);
    }
    return off;
}

// Tiles are handed to XCDs in contiguous ranges: the hardware deals blocks
// round-robin over the 8 XCDs, so block b runs on XCD b % 8.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t total) {
    const int64_t X = 8;
    int64_t xcd = b % X, idx = b / X;
    int64_t per = total / X, rem = total % X;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// One BM x BN output tile (all passes) of the contraction described by `a`,
// with the operand pointers and scalars given separately (a batch keeps them
// apart from the static descriptors).  Called by a whole block.
// ---- split-BF16 helpers (X3 tiles) ----
typedef short xs4 __attribute__((ext_vector_type(4)));

// 2^k for k in [-1074, 1023] (subnormal below -1022)
__device__ __forceinline__ double pow2d(int k) {
    const uint64_t u = k >= -1022 ? (uint64_t)(k + 1023) << 52 : 1ull << (k + 1074);
    return __longlong_as_double((long long)u);
}

// floor(log2 |x|) of a normal x (zero and subnormals give -1023, which the
// scale clamps to -1022)
__device__ __forceinline__ int expo2(double x) {
    return (int)(((uint64_t)__double_as_longlong(x) >> 52) & 0x7ff) - 1023;
}

// BF16 pattern of a value with at most 8 significant bits (exact in FP32)
__device__ __forceinline__ uint16_t bf16_of(double t) {
    return (uint16_t)(__float_as_uint((float)t) >> 16);
}

// Element (row, k) of one term plane of a staged X3 tile (16 positions per
// row, 8-byte units permuted by (row >> 2) & 3 so that the 16 rows one
// fragment read touches fall on distinct banks).
__device__ __forceinline__ int xtile_at(int r, int k) {
    return r * 16 + ((((k >> 2) ^ (r >> 2)) & 3) << 2) + (k & 3);
}

template <typename T, int BM, int BN, int BK, int AMODE, int BMODE, bool SPLIT = false, bool DEEP = true,
          bool X3 = false, int NW = 4>
__device__ __forceinline__ void mfma_tile(const MfmaArgs& a, const void* Ap, const void* Bp, void* Cp,
                                          double alpha_d, double beta_d, int64_t tile, int64_t slice) {
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr int NT = 64 * NW;                             // threads per block
    constexpr int EA = BM * BK / NT, EB = BN * BK / NT;     // elements per thread per tile
    constexpr bool A_KMAJ = AMODE != LD_MMAJ, B_KMAJ = BMODE != LD_MMAJ;
    constexpr bool AV = AMODE == LD_KVEC, BV = BMODE == LD_KVEC;
    constexpr int VEC = 16 / (int)sizeof(T), CPR = BK / VEC;  // chunk width, chunks per row
    constexpr int CA = EA / VEC, CB = EB / VEC;              // chunks per thread (vector loads)
    typedef T vT __attribute__((ext_vector_type(VEC)));
    static_assert((!AV || EA % VEC == 0) && (!BV || EB % VEC == 0) && NT % CPR == 0, "vector staging shape");
    // four waves, 2 x 2 over the tile, or 1 x 4 along n for tiles of 32 rows;
    // eight waves (two per SIMD), 2 x 4, or 4 x 2 for tiles of 256 rows
    static_assert(NW == 4 || (NW == 8 && BM >= 64), "eight waves take tiles of at least 64 rows");
    constexpr int WM = (NW == 8 && BM >= 256) ? 4 : BM >= 64 ? 2 : 1, WN = NW / WM;
    constexpr int FM = BM / WM / 16, FN = BN / WN / 16;    // 16x16 blocks per wave
    static_assert(EA >= 1 && EB >= 1, "tile too small for the block's threads");
    static_assert(BM % (NT / BK) == 0 && BN % (NT / BK) == 0, "M/N-major staging needs whole row groups");
    static_assert(BK == 16, "the LDS layout holds 16 positions per row");
    static_assert(!X3 || (!AV && !BV && !SPLIT), "X3 tiles stage element by element and do not split K");
    __shared__ __attribute__((aligned(16))) T As[X3 ? 1 : 2][X3 ? 1 : BM * BK];
    __shared__ __attribute__((aligned(16))) T Bs[X3 ? 1 : 2][X3 ? 1 : BN * BK];
    // X3: three BF16 term planes per operand and buffer, and the per-row
    // (per-column) exponents and scales
    __shared__ __attribute__((aligned(16))) uint16_t Xa[X3 ? 2 : 1][X3 ? 3 * BM * BK : 1];
    __shared__ __attribute__((aligned(16))) uint16_t Xb[X3 ? 2 : 1][X3 ? 3 * BN * BK : 1];
    __shared__ int sEA[X3 ? BM : 1], sEB[X3 ? BN : 1];
    __shared__ double sSA[X3 ? BM : 1], sSB[X3 ? BN : 1];

    const gmem<T>* __restrict__ Ag = (const gmem<T>*)Ap;
    const gmem<T>* __restrict__ Bg = (const gmem<T>*)Bp;
    gmem<T>* Cg = (gmem<T>*)Cp;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int wm = wid % WM, wn = wid / WM;

    int64_t rest = tile;
    const int64_t mt = dm(rest, a.mt);
    const int64_t nt = dm(rest, a.nt);
    const int64_t bt = rest;
    const int64_t m_base = mt * BM, n_base = nt * BN;

    int64_t bA = 0, bB = 0, bC = 0;
    {
        int64_t r = bt;
        for (int d = 0; d < a.batch.n; ++d) {
            int64_t q = dm(r, a.batch.d[d].ext);
            bA += q * a.batch.d[d].sA;
            bB += q * a.batch.d[d].sB;
            bC += q * a.batch.d[d].sC;
        }
    }

    // per-block offset tables: A/C offsets of the tile's rows (m) and B/C
    // offsets of its columns (n); -1 marks rows/columns past the edge
    __shared__ int64_t sAm[BM], sCm[BM], sBn[BN], sCn[BN];
    for (int i = tid; i < BM; i += NT) {
        int64_t m = m_base + i;
        bool ok = m < a.M;
        sAm[i] = ok ? group_off<0>(a.m, m) : -1;
        sCm[i] = ok ? group_off<2>(a.m, m) : -1;
    }
    for (int i = tid; i < BN; i += NT) {
        int64_t n = n_base + i;
        bool ok = n < a.N;
        sBn[i] = ok ? group_off<1>(a.n, n) : -1;
        sCn[i] = ok ? group_off<2>(a.n, n) : -1;
    }
    if constexpr (X3) {
        for (int i = tid; i < BM; i += NT) sEA[i] = -1023;
        for (int i = tid; i < BN; i += NT) sEB[i] = -1023;
    }
    lds_barrier();

    const T alpha = (T)alpha_d, beta = (T)beta_d;
    // this block's K tiles: all of them, or one slice when K is split
    int64_t kt_count = a.Kpad / BK, k_first = 0;
    if constexpr (SPLIT) {
        if (a.kslices > 1) {
            k_first = slice * a.kslice_tiles;
            kt_count = std::max<int64_t>(0, std::min<int64_t>(a.kslice_tiles, kt_count - k_first));
        }
    } else {
        (void)slice;
    }
    // alpha = 0 reads neither A nor B: no K tiles, so the epilogue writes
    // beta * C (zeros without reading C when beta = 0)
    const int64_t ktiles = alpha_d == 0.0 ? 0 : kt_count;
    const gmem<int64_t>* ktab0 = (const gmem<int64_t>*)(SPLIT ? a.ktab + 2 * k_first * BK : a.ktab);
    constexpr int RT = NT / BK;

    // X3 with a single K tile (at most 16 summed positions): sweep 1's
    // operand values and masks, which the staging step then takes instead of
    // loading the same tile again
    T xa[X3 ? EA : 1], xb[X3 ? EB : 1];
    uint32_t xmA = 0, xmB = 0;
    if constexpr (X3) {
        // Sweep 1: the largest exponent of each of the tile's rows of A and
        // columns of B over all of K (a thread's element slots keep their row
        // from tile to tile), then the scales 2^-e.  X3 tiles take one pass.
        int ea[EA], eb[EB];
#pragma unroll
        for (int e = 0; e < EA; ++e) ea[e] = -1023;
#pragma unroll
        for (int e = 0; e < EB; ++e) eb[e] = -1023;
        // each tile's K-table entries are requested one tile ahead, before
        // the operands of the tile in hand
        const int ia = 2 * (A_KMAJ ? tid % BK : tid / RT), ib = 2 * (B_KMAJ ? tid % BK : tid / RT) + 1;
        int64_t ka = ktiles > 0 ? ktab0[ia] : 0, kb = ktiles > 0 ? ktab0[ib] : 0;
        for (int64_t kt = 0; kt < ktiles; ++kt) {
            const gmem<int64_t>* kt1 = ktab0 + 2 * std::min<int64_t>(kt + 1, ktiles - 1) * BK;
            const int64_t na = kt1[ia], nb = kt1[ib];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int e = 0; e < EA; ++e) {
                const int idx = tid + NT * e;
                const int64_t om = sAm[A_KMAJ ? idx / BK : tid % RT + RT * e];
                const bool ok = (om >= 0) & (ka >= 0);
                xa[e] = Ag[bA + (ok ? om + ka : 0)];
                if (ok) ea[e] = max(ea[e], expo2((double)xa[e]));
                xmA = (xmA & ~(1u << e)) | ((uint32_t)ok << e);
            }
#pragma unroll
            for (int e = 0; e < EB; ++e) {
                const int idx = tid + NT * e;
                const int64_t on = sBn[B_KMAJ ? idx / BK : tid % RT + RT * e];
                const bool ok = (on >= 0) & (kb >= 0);
                xb[e] = Bg[bB + (ok ? on + kb : 0)];
                if (ok) eb[e] = max(eb[e], expo2((double)xb[e]));
                xmB = (xmB & ~(1u << e)) | ((uint32_t)ok << e);
            }
            ka = na;
            kb = nb;
        }
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            const int idx = tid + NT * e;
            atomicMax(&sEA[A_KMAJ ? idx / BK : tid % RT + RT * e], ea[e]);
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            const int idx = tid + NT * e;
            atomicMax(&sEB[B_KMAJ ? idx / BK : tid % RT + RT * e], eb[e]);
        }
        lds_barrier();
        for (int i = tid; i < BM; i += NT) {
            sEA[i] = min(max(sEA[i], -1022), 1023);
            sSA[i] = pow2d(-sEA[i]);
        }
        for (int i = tid; i < BN; i += NT) {
            sEB[i] = min(max(sEB[i], -1022), 1023);
            sSB[i] = pow2d(-sEB[i]);
        }
        lds_barrier();
    }

    int64_t pctr[GT_MAXD];
    for (int d = 0; d < a.pass.n; ++d) pctr[d] = 0;
    int64_t pA = 0, pB = 0;

    for (int64_t pass = 0; pass < a.npass; ++pass) {
        // X3: big (the leading term product) and small (the other five)
        acc_t acc[X3 ? 1 : FN][X3 ? 1 : FM];
        f4 big[X3 ? FN : 1][X3 ? FM : 1], small[X3 ? FN : 1][X3 ? FM : 1];
        if constexpr (X3) {
#pragma unroll
            for (int i = 0; i < FN; ++i)
#pragma unroll
                for (int j = 0; j < FM; ++j) big[i][j] = small[i][j] = f4{0, 0, 0, 0};
        } else {
#pragma unroll
            for (int i = 0; i < FN; ++i)
#pragma unroll
                for (int j = 0; j < FM; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
        }

        // Register slots for operand tiles in flight: tile kt + NS - 1 is
        // loaded while tile kt is multiplied, so a load has NS - 1 tiles of
        // MFMA time to arrive.  FP32 keeps two tiles in flight (its MFMAs take
        // half as long per tile as FP64's); FP64 two with eight waves per
        // block (C4 FP64 66.3% -> 70.2% of peak against one), one with four
        // (its registers are all taken).
        constexpr int NS = (DEEP && !X3 && (sizeof(T) == 4 || NW == 8)) ? 3 : 2;
        T ra[NS - 1][EA], rb[NS - 1][EB];
        vT va[NS - 1][CA], vb[NS - 1][CB];
        uint32_t okA[NS - 1], okB[NS - 1];
        // K-table entries of a tile are fetched one step before its operands
        // (two table slots, tile t in slot t % 2), and in each step before the
        // operand loads: waiting for a table then never waits for operand
        // loads still in flight.  In K-major loading a thread always handles
        // the same k of a tile (one entry); in M/N-major loading EA/EB.
        // Every thread handles one K position per tile: tid % BK along K
        // (K-major) or tid / RT with RT = NT / BK threads on consecutive
        // rows (M/N-major, rows tid % RT + RT * e), so one table entry each.
        constexpr int TA = 1, TB = 1;
        int64_t tA[2][TA], tB[2][TB];
        auto tload = [&](int64_t kt, auto ts_c) {
            constexpr int ts = decltype(ts_c)::value;
            const gmem<int64_t>* kt0 = ktab0 + 2 * kt * BK;
#pragma unroll
            for (int e = 0; e < TA; ++e)
                tA[ts][e] = kt0[2 * (AV ? VEC * (tid % CPR) : A_KMAJ ? tid % BK : tid / RT)];
#pragma unroll
            for (int e = 0; e < TB; ++e)
                tB[ts][e] = kt0[2 * (BV ? VEC * (tid % CPR) : B_KMAJ ? tid % BK : tid / RT) + 1];
        };
        // Operand loads with clamped addresses (element (batch, pass, 0, 0) is
        // always valid), so no branch sits around a load.  The raw values stay
        // in registers with a validity mask; padding is zeroed only when the
        // tile is written to LDS, so the loads stay in flight until then.
        auto gload = [&](auto slot_c, auto ts_c, bool live) {
            constexpr int sl = decltype(slot_c)::value, ts = decltype(ts_c)::value;
            uint32_t ma = 0, mb = 0;
            if constexpr (AV) {
                // 16-byte chunks: chunk q = row q / CPR, positions VEC * (q % CPR) ..
#pragma unroll
                for (int e = 0; e < CA; ++e) {
                    const int64_t om = sAm[(tid + NT * e) / CPR];
                    const bool ok = (om >= 0) & (tA[ts][0] >= 0) & live;
                    va[sl][e] = *(const gmem<vT>*)(Ag + bA + pA + (ok ? om + tA[ts][0] : 0));
                    ma |= (uint32_t)ok << e;
                }
            } else {
#pragma unroll
                for (int e = 0; e < EA; ++e) {
                    const int idx = tid + NT * e;
                    const int64_t om = sAm[A_KMAJ ? idx / BK : tid % RT + RT * e];
                    const int64_t ko = tA[ts][0];
                    const bool ok = (om >= 0) & (ko >= 0) & live;
                    ra[sl][e] = Ag[bA + pA + (ok ? om + ko : 0)];
                    ma |= (uint32_t)ok << e;
                }
            }
            if constexpr (BV) {
#pragma unroll
                for (int e = 0; e < CB; ++e) {
                    const int64_t on = sBn[(tid + NT * e) / CPR];
                    const bool ok = (on >= 0) & (tB[ts][0] >= 0) & live;
                    vb[sl][e] = *(const gmem<vT>*)(Bg + bB + pB + (ok ? on + tB[ts][0] : 0));
                    mb |= (uint32_t)ok << e;
                }
            } else {
#pragma unroll
                for (int e = 0; e < EB; ++e) {
                    const int idx = tid + NT * e;
                    const int64_t on = sBn[B_KMAJ ? idx / BK : tid % RT + RT * e];
                    const int64_t ko = tB[ts][0];
                    const bool ok = (on >= 0) & (ko >= 0) & live;
                    rb[sl][e] = Bg[bB + pB + (ok ? on + ko : 0)];
                    mb |= (uint32_t)ok << e;
                }
            }
            okA[sl] = ma;
            okB[sl] = mb;
        };
        auto sstore = [&](int buf, auto slot_c) {
            constexpr int sl = decltype(slot_c)::value;
            if constexpr (X3) {
                // scale, split into three terms (round-to-nearest-even at 8
                // significant bits), one plane per term
                auto put = [&](uint16_t* plane, int rows, int r, int k, double x) {
                    const double t1 = rn8(x), r1 = x - t1;
                    const double t2 = rn8(r1), t3 = rn8(r1 - t2);
                    const int at = xtile_at(r, k);
                    plane[at] = bf16_of(t1);
                    plane[rows * BK + at] = bf16_of(t2);
                    plane[2 * rows * BK + at] = bf16_of(t3);
                };
#pragma unroll
                for (int e = 0; e < EA; ++e) {
                    const int idx = tid + NT * e;
                    const int r = A_KMAJ ? idx / BK : tid % RT + RT * e, k = A_KMAJ ? idx % BK : tid / RT;
                    const double x = (okA[sl] >> e) & 1 ? (double)ra[sl][e] * sSA[r] : 0.0;
                    put(Xa[buf], BM, r, k, x);
                }
#pragma unroll
                for (int e = 0; e < EB; ++e) {
                    const int idx = tid + NT * e;
                    const int r = B_KMAJ ? idx / BK : tid % RT + RT * e, k = B_KMAJ ? idx % BK : tid / RT;
                    const double x = (okB[sl] >> e) & 1 ? (double)rb[sl][e] * sSB[r] : 0.0;
                    put(Xb[buf], BN, r, k, x);
                }
                return;
            }
            if constexpr (AV) {
#pragma unroll
                for (int e = 0; e < CA; ++e) {
                    const int q = tid + NT * e;
                    *(vT*)&As[buf][tile_at<T>(q / CPR, VEC * (q % CPR))] = (okA[sl] >> e) & 1 ? va[sl][e] : vT(0);
                }
            } else {
#pragma unroll
                for (int e = 0; e < EA; ++e) {
                    const int idx = tid + NT * e;
                    As[buf][tile_at<T>(A_KMAJ ? idx / BK : tid % RT + RT * e, A_KMAJ ? idx % BK : tid / RT)] =
                        (okA[sl] >> e) & 1 ? ra[sl][e] : (T)0;
                }
            }
            if constexpr (BV) {
#pragma unroll
                for (int e = 0; e < CB; ++e) {
                    const int q = tid + NT * e;
                    *(vT*)&Bs[buf][tile_at<T>(q / CPR, VEC * (q % CPR))] = (okB[sl] >> e) & 1 ? vb[sl][e] : vT(0);
                }
            } else {
#pragma unroll
                for (int e = 0; e < EB; ++e) {
                    const int idx = tid + NT * e;
                    Bs[buf][tile_at<T>(B_KMAJ ? idx / BK : tid % RT + RT * e, B_KMAJ ? idx % BK : tid / RT)] =
                        (okB[sl] >> e) & 1 ? rb[sl][e] : (T)0;
                }
            }
        };
        auto compute = [&](int buf) {
            // this lane's positions 4g .. 4g+3 of each fragment row, g = lane / 16
            typedef T v4 __attribute__((ext_vector_type(4)));
            constexpr int CE = TileLds<T>::CE;
            const int g = lane >> 4, r16 = lane & 15;
            if constexpr (X3) {
                auto xfrag = [&](const uint16_t* plane, int row) -> xs4 {
                    return *(const xs4*)(plane + row * 16 + (((g ^ (row >> 2)) & 3) << 2));
                };
                xs4 fb[3][FN];
#pragma unroll
                for (int i = 0; i < FN; ++i)
#pragma unroll
                    for (int t = 0; t < 3; ++t) fb[t][i] = xfrag(Xb[buf] + t * BN * BK, wn * (BN / WN) + i * 16 + r16);
#pragma unroll
                for (int j = 0; j < FM; ++j) {
                    xs4 fa[3];
#pragma unroll
                    for (int t = 0; t < 3; ++t) fa[t] = xfrag(Xa[buf] + t * BM * BK, wm * (BM / WM) + j * 16 + r16);
#pragma unroll
                    for (int i = 0; i < FN; ++i) {
                        big[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fb[0][i], fa[0], big[i][j], 0, 0, 0);
                        f4 sm = small[i][j];
                        sm = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fb[0][i], fa[1], sm, 0, 0, 0);
                        sm = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fb[1][i], fa[0], sm, 0, 0, 0);
                        sm = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fb[0][i], fa[2], sm, 0, 0, 0);
                        sm = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fb[2][i], fa[0], sm, 0, 0, 0);
                        sm = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fb[1][i], fa[1], sm, 0, 0, 0);
                        small[i][j] = sm;
                    }
                }
            } else {
                auto frag = [&](const T* tile, int row) -> v4 {
                    v4 v;
#pragma unroll
                    for (int h = 0; h < 4 / CE; ++h) {
                        typedef T vc __attribute__((ext_vector_type(CE)));
                        const vc c = *(const vc*)(tile + row * 16 + TileLds<T>::swz(row, (4 * g) / CE + h) * CE);
#pragma unroll
                        for (int q = 0; q < CE; ++q) v[h * CE + q] = c[q];
                    }
                    return v;
                };
                v4 fb[FN];
#pragma unroll
                for (int i = 0; i < FN; ++i) fb[i] = frag(Bs[buf], wn * (BN / WN) + i * 16 + r16);
#pragma unroll
                for (int j = 0; j < FM; ++j) {
                    const v4 fa = frag(As[buf], wm * (BM / WM) + j * 16 + r16);
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                        for (int i = 0; i < FN; ++i) acc[i][j] = Mfma<T>::mac(fb[i][s4], fa[s4], acc[i][j]);
                }
            }
        };
        typedef std::integral_constant<int, 0> S0;
        typedef std::integral_constant<int, 1> S1;
        typedef std::integral_constant<int, NS - 2> SL;   // slot 1 (FP32) or 0 (FP64)

        // prologue: tile 0 to LDS, tiles 1 .. NS-2 in registers, table of the
        // next tile to load
        if (ktiles > 0) {
            const int64_t last = ktiles - 1;
            // Loads leave the prologue in the order a step leaves them (the
            // table of tile NS - 1, then the operands of tile 1 for FP32), so
            // the wait counts at the loop entry match the steady state.
            if (X3 && ktiles == 1) {
                // the tile sweep 1 loaded (same table entries, same masks)
#pragma unroll
                for (int e = 0; e < EA; ++e) ra[0][e] = xa[e];
#pragma unroll
                for (int e = 0; e < EB; ++e) rb[0][e] = xb[e];
                okA[0] = xmA;
                okB[0] = xmB;
            } else {
                tload(0, S0{});
                gload(S0{}, S0{}, true);
            }
            sstore(0, S0{});
            tload(std::min<int64_t>(1, last), S1{});
            if (NS == 3) {
                tload(std::min<int64_t>(2, last), S0{});
                gload(SL{}, S1{}, ktiles > 1);
            }
            lds_barrier();
            // One K tile: load tile kt + NS - 1 into the slot that tile kt + 1
            // does not use, multiply tile kt, store tile kt + 1 from its slot.
            // The loads are issued on every step (past the last tile all
            // lanes read element 0 and the values are dropped) and the barrier
            // waits for LDS traffic only, so the compiler's wait counting
            // keeps the loads of later tiles in flight across steps.
            // Step parity p = kt % 2 is a compile-time constant (steps come
            // in pairs), so every slot index below is too.
            auto step = [&](int64_t kt, auto p_c) {
                constexpr int p = decltype(p_c)::value;
                tload(std::min<int64_t>(kt + NS, last), std::integral_constant<int, (p + NS) % 2>{});
                // FP64: the table loads must stay ahead of the operand loads
                // (the next step's table wait would otherwise wait for them)
                if constexpr (NS == 2) __builtin_amdgcn_sched_barrier(0);
                gload(std::integral_constant<int, NS == 3 ? p : 0>{}, std::integral_constant<int, (p + NS - 1) % 2>{},
                      kt + NS - 1 < ktiles);
                // FP64: keep the loads ahead of the MFMAs (under its register
                // pressure the scheduler sinks them next to their LDS stores,
                // leaving no time to arrive); FP32 spreads them among the
                // MFMAs by itself, which measures faster
                if constexpr (NS == 2) __builtin_amdgcn_sched_barrier(0);
                compute(p);
                // FP64: the store of the next tile (and its wait for the
                // loads) stays after the MFMAs
                if constexpr (NS == 2) __builtin_amdgcn_sched_barrier(0);
                if (kt + 1 < ktiles) sstore(p ^ 1, std::integral_constant<int, NS == 3 ? 1 - p : 0>{});
                lds_barrier();
            };
            // operand slots: tile t in slot t % 2 (FP32), slot 0 (FP64)
            int64_t kt = 0;
            for (; kt + 1 < ktiles; kt += 2) {
                step(kt, S0{});
                step(kt + 1, S1{});
            }
            if (kt < ktiles) step(kt, S0{});
        }

        if constexpr (X3) {
            // lane holds D[n = 4 (lane / 16) + q][m = lane % 16] of each block
#pragma unroll
            for (int i = 0; i < FN; ++i) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int nl = wn * (BN / WN) + i * 16 + 4 * (lane >> 4) + q;
                    const int64_t cn = sCn[nl];
                    if (cn < 0) continue;
                    const int en = sEB[nl];
#pragma unroll
                    for (int j = 0; j < FM; ++j) {
                        const int ml = wm * (BM / WM) + j * 16 + (lane & 15);
                        const int64_t cm = sCm[ml];
                        if (cm < 0) continue;
                        gmem<T>* cp = Cg + bC + cn + cm;
                        double v = alpha_d * ldexp((double)big[i][j][q] + (double)small[i][j][q], sEA[ml] + en);
                        if (beta_d != 0.0) v += beta_d * (double)(*cp);
                        *cp = (T)v;
                    }
                }
            }
        } else {
            // epilogue: lane holds D[n = row(lane, q)][m = lane % 16] of each block
            if constexpr (SPLIT) if (a.kslices > 1) {
                // split K: raw partial tile to the workspace (rows and columns past
                // the edge hold zeros and are never read)
                gmem<T>* wsp = (gmem<T>*)a.ws + (slice * a.ntiles + tile) * (int64_t)(BM * BN);
#pragma unroll
                for (int i = 0; i < FN; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int j = 0; j < FM; ++j)
                            wsp[(wn * (BN / WN) + i * 16 + Mfma<T>::row(lane, q)) * BM + wm * (BM / WM) + j * 16 +
                                (lane & 15)] = acc[i][j][q];
                continue;   // a split launch has one pass
            }
#pragma unroll
            for (int i = 0; i < FN; ++i) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t cn = sCn[wn * (BN / WN) + i * 16 + Mfma<T>::row(lane, q)];
                    if (cn < 0) continue;
#pragma unroll
                    for (int j = 0; j < FM; ++j) {
                        const int64_t cm = sCm[wm * (BM / WM) + j * 16 + (lane & 15)];
                        if (cm < 0) continue;
                        gmem<T>* cp = Cg + bC + cn + cm;
                        T v = alpha * acc[i][j][q];
                        if (a.mode == 1) v = *cp + v;
                        else if (beta_d != 0.0) v += beta * (*cp);
                        *cp = v;
                    }
                }
            }
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        // next pass (innermost pass loop fastest)
        for (int d = a.pass.n - 1; d >= 0; --d) {
            pA += a.pass.d[d].sA;
            pB += a.pass.d[d].sB;
            if (++pctr[d] < a.pass.d[d].ext) break;
            pA -= a.pass.d[d].sA * a.pass.d[d].ext;
            pB -= a.pass.d[d].sB * a.pass.d[d].ext;
            pctr[d] = 0;
        }
    }
}

// Persistent form for batches.  A group's work list of (contraction, tile)
// items is cut into eight ranges, one per XCD, each holding whole
// contractions, so that the tiles of one contraction run on one XCD and share
// its L2.  Block b runs on XCD b % 8 (the hardware deals blocks round-robin)
// and takes runs of `chunk` consecutive items off its range's counter; when
// its range is exhausted it takes items from the other ranges in turn, and it
// exits once all eight counters have passed their ranges' ends.  Claiming a
// run per atomic keeps the counters from serialising the many small tiles of
// a large batch.  xstart: the nine range offsets (xstart[8] = list length);
// counter: eight counters, zero at launch.  X3: the split-BF16 tiles.  NW:
// waves per block.
template <typename T, int BM, int BN, int BK, int AMODE, int BMODE, bool X3 = false, int NW = 4>
__global__ __launch_bounds__(64 * NW) void k_mfma_batch(const MfmaArgs* __restrict__ items,
                                                      const BatchPtrs* __restrict__ ptrs,
                                                      const int2* __restrict__ work, const int* __restrict__ xstart,
                                                      int chunk, int* counter) {
    __shared__ int s_w;
    const int x0 = blockIdx.x % 8;
    for (int d = 0; d < 8; ++d) {
        const int x = (x0 + d) & 7;
        const int lo = xstart[x], n = xstart[x + 1] - lo;
        for (;;) {
            if (threadIdx.x == 0) s_w = atomicAdd(counter + x, chunk);
            lds_barrier();
            const int w0 = s_w;
            lds_barrier();   // every thread has read s_w before thread 0 claims again
            if (w0 >= n) break;
            const int w1 = min(w0 + chunk, n);
            for (int w = w0; w < w1; ++w) {
                const int2 wi = work[lo + w];
                const BatchPtrs& pt = ptrs[wi.x];
                // batch tiles have short K: one step of loads in flight (the
                // two-deep prefetch costs registers these kernels do not have)
                mfma_tile<T, BM, BN, BK, AMODE, BMODE, false, false, X3, NW>(items[wi.x], pt.A, pt.B, pt.C,
                                                                              pt.alpha, pt.beta, wi.y, 0);
                lds_barrier();   // the tile's LDS tables are reused by the next item
            }
        }
    }
}

}  // namespace tc
