// Split-precision contraction on BF16 matrix cores (gfx950
// v_mfma_f32_16x16x32_bf16).
//
// 1. k_split2 (both operands in one launch; k_split_long past 8192
//    positions): one block per slice (one row m of A's GEMM view, or one
//    column n of B's), reading the slice once.  FP64 absmax over the slice ->
//    exponent e = floor(log2(max)); the
//    scaled values x = v * 2^-e (exact) are split into three BF16 terms by
//    round-to-nearest-even, t1 = rn(x), t2 = rn(x - t1), t3 = rn(x - t1 - t2),
//    in the K order of the plan's offset table.  The terms are written as
//    ready-made LDS images: for every 128-row tile and 32-wide K stage, one
//    contiguous 24 KB block [term][row][four 16-byte chunks], the chunks of
//    each row permuted by xswz so that fragment reads hit distinct banks.
// 2. k_x3: C tile = sum over the six term products t_A,p t_B,q with p+q <= 4
//    (ablations: the three with p+q <= 3, or all nine).
//    Stages are copied HBM -> LDS by the DMA form of the global load (no
//    registers in between), double-buffered.  The leading product t_A1 t_B1
//    and the five small products accumulate in two FP32 accumulators over all
//    of K (FP32 accumulation, as an FP32 matrix product would); the epilogue
//    adds the two partials in FP64, which is exact, and unscales:
//    C = alpha * 2^(eA + eB) * (big + small) + beta * C.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "devutil.h"
#include "launch.h"
#include "plan.h"

namespace tc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int SPLIT_BK = 32;      // contracted positions per stage (one 16x16x32 MFMA step)
constexpr int XR = 128;           // rows per stage image (panel row tile)
constexpr int XSTAGE = 3 * XR * SPLIT_BK * 2;   // bytes of one stage image (24 KB)
constexpr int XPIECE = 1024;      // bytes one wave copies per DMA instruction (64 lanes x 16 B)
// Product tile: 256 (m) x 128 (n) per block of eight waves, two per SIMD, each
// wave 64 x 64.  Measured on MI355X at 4096^2 x 4096 against 128 x 128 tiles
// with eight 64 x 32 waves: a quarter fewer staged bytes and a third fewer
// fragment reads per flop.
constexpr int XBM = 2 * XR, XBN = XR;
constexpr int XWAVES = 8;

// Physical 16-byte chunk of logical chunk c (k = 8c .. 8c+7) of row r inside a
// stage image.  Rows are 64 bytes, so the 16 rows one fragment read touches
// (rows 16b .. 16b+15 in lanes 0-15, the same rows one chunk further in each
// next 16 lanes) would fall on few banks.  Measured on MI355X with a
// read-pattern probe: permuting chunk c of row r by (r >> 1) & 3 makes that
// read as fast as a linear 1 KB read; other permutations tried (r & 3,
// (r >> 2) & 3, ((r >> 1) ^ (r >> 3)) & 3, 80-byte padded rows) took 1.55x as
// long.
__host__ __device__ __forceinline__ int xswz(int r, int c) { return c ^ ((r >> 1) & 3); }

// Round-to-nearest-even to an 8-bit significand, unbounded exponent (the
// values stay far inside BF16's range after the per-slice scaling).
__device__ __forceinline__ double rn_bf16(double x) { return rn8(x); }

__device__ __forceinline__ uint16_t bf16_bits(double t) {
    // t has at most 8 significant bits and a float exponent: exact in FP32,
    // and its FP32 pattern has zero low 16 bits
    float f = (float)t;
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ int64_t grp_off(const GtDims& g, int64_t i, int slot) {
    int64_t off = 0;
    for (int d = 0; d < g.n; ++d) {
        int64_t e = g.d[d].ext;
        int64_t q = i / e, r = i - q * e;
        off += r * (slot == 0 ? g.d[d].sA : slot == 1 ? g.d[d].sB : g.d[d].sC);
        i = q;
    }
    return off;
}

struct SplitArgs {
    const void* X;
    // batches: X, and whether to run at all (alpha != 0), come from the
    // member's staged pointers at run time (X unused)
    const BatchPtrs* bp;
    GtDims rows;          // the side's free dims (slot selects the stride)
    int slot;             // 0: A side (sA); 1: B side (sB)
    const int64_t* koff;  // Kp element offsets of the side's operand, -1 for padding
    int64_t nrows, Kp;
    int64_t Kt;           // positions with table entries (a multiple of 32); Kt .. Kp are zero
                          // terms that the zeroed workspace already holds
    uint16_t* panels;     // stage images, see xswz
    int32_t* exps;
};

// Element offset of (term, row, k) in a side's stage images.
__host__ __device__ __forceinline__ int64_t panel_off(int64_t row, int64_t k, int term, int64_t Kp) {
    const int64_t rt = row / XR, kt = k / SPLIT_BK;
    const int rr = (int)(row % XR), kk = (int)(k % SPLIT_BK);
    return ((rt * (Kp / SPLIT_BK) + kt) * 3 + term) * (int64_t)(XR * SPLIT_BK) + rr * SPLIT_BK +
           xswz(rr, kk >> 3) * 8 + (kk & 7);
}

// Block b runs on XCD b % 8; give each XCD a contiguous range of items.
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t total) {
    const int64_t X = 8;
    int64_t xcd = b % X, idx = b / X;
    int64_t per = total / X, rem = total % X;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pack2(double lo, double hi) {
    return (uint32_t)bf16_bits(lo) | ((uint32_t)bf16_bits(hi) << 16);
}

// BF16 terms for any K: two passes over the slice, the second re-reading it
// (from cache); one block per slice.
template <typename T>
__global__ __launch_bounds__(256) void k_split_long(SplitArgs a) {
    __shared__ double red[4];
    if (a.bp && a.bp->alpha == 0.0) return;   // a batch member with alpha = 0 reads neither input
    const gmem<T>* X = (const gmem<T>*)(a.bp ? (a.slot == 0 ? a.bp->A : a.bp->B) : a.X);
    const gmem<int64_t>* koff = (const gmem<int64_t>*)a.koff;
    const int64_t row = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t base = grp_off(a.rows, row, a.slot);
    double amax = 0.0;
    for (int64_t k = tid; k < a.Kt; k += 256) {
        const int64_t o = koff[k];
        const double v = o >= 0 ? (double)X[base + o] : 0.0;
        amax = fmax(amax, fabs(v));
    }
    for (int s = 32; s > 0; s >>= 1) amax = fmax(amax, __shfl_xor(amax, s));
    if ((tid & 63) == 0) red[tid >> 6] = amax;
    __syncthreads();
    amax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int e = 0;
    if (amax > 0.0) {
        int E;
        frexp(amax, &E);
        e = E - 1;
    }
    if (tid == 0) ((gmem<int32_t>*)a.exps)[row] = e;
    constexpr int64_t TS = XR * SPLIT_BK;
    for (int64_t k = tid; k < a.Kt; k += 256) {
        const int64_t o = koff[k];
        const double x = o >= 0 ? ldexp((double)X[base + o], -e) : 0.0;
        const double r1 = rn_bf16(x);
        const double rest = x - r1;
        const double r2 = rn_bf16(rest);
        const double r3 = rn_bf16(rest - r2);
        gmem<uint16_t>* t = (gmem<uint16_t>*)a.panels + panel_off(row, k, 0, a.Kp);
        t[0] = bf16_bits(r1);
        t[TS] = bf16_bits(r2);
        t[2 * TS] = bf16_bits(r3);
    }
}

// Both operands' split in one launch (up to 8192 positions per slice): blocks
// 0 .. nrows(A) - 1 take A's slices, the rest B's (one slice per block, the
// slices handed to XCDs in contiguous ranges: neighbouring slices share
// stage-image cache lines, which then fill in one L2).  A side reads its
// slice in one of three ways:
//   mode 0: every chunk of eight positions is eight consecutive aligned
//     elements; consecutive threads load consecutive 16-byte pieces (two FP64
//     or four FP32 positions), so a wave's load covers whole chunks, and each
//     thread stores its piece's terms (4 or 8 bytes per term);
//   mode 1: within a chunk the valid positions are a prefix, at offsets o0 +
//     e * cstride (one table entry per chunk: o0 * 16 + count); a thread takes
//     a chunk, without a table entry per position;
//   mode 2: one table entry per position.
struct SplitSide {
    const void* X;
    GtDims rows;
    int slot;
    int mode;
    const int64_t* koff;
    const int64_t* cinfo;   // mode 1: per chunk o0 * 16 + count
    int64_t cstride;        // mode 1: element stride between a chunk's positions
    int64_t nrows;
    uint16_t* panels;
    int32_t* exps;
};

struct Split2Args {
    SplitSide s[2];
    const BatchPtrs* bp;
    int64_t Kp, Kt;
};

template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_split2(Split2Args a) {
    __shared__ double red[4];
    if (a.bp && a.bp->alpha == 0.0) return;   // a batch member with alpha = 0 reads neither input
    const int64_t nA = a.s[0].nrows;
    const int64_t item = xcd_item(blockIdx.x, nA + a.s[1].nrows);
    const int side = item < nA ? 0 : 1;
    const SplitSide& S = a.s[side];
    const int64_t row = side == 0 ? item : item - nA;
    const gmem<T>* X = (const gmem<T>*)(a.bp ? (S.slot == 0 ? a.bp->A : a.bp->B) : S.X);
    const gmem<int64_t>* koff = (const gmem<int64_t>*)S.koff;
    const gmem<int64_t>* cinfo = (const gmem<int64_t>*)S.cinfo;
    gmem<uint16_t>* panels = (gmem<uint16_t>*)S.panels;
    const int tid = threadIdx.x;
    const int64_t base = grp_off(S.rows, row, S.slot);
    const int64_t nch = a.Kt / 8;
    constexpr int W = 16 / (int)sizeof(T), P = 8 / W;   // elements per 16-byte piece, pieces per chunk
    typedef T vW __attribute__((ext_vector_type(W)));
    double v[CPT * 8];
    double amax = 0.0;
    const int mode = S.mode;
    if (mode == 0) {
#pragma unroll
        for (int q = 0; q < CPT * P; ++q) {
            const int64_t pc = tid + 256 * q, ch = pc / P;
            const bool in = ch < nch;
            const int64_t o = koff[8 * (in ? ch : 0)];
            const bool ok = in && o >= 0;
            const vW t = *(const gmem<vW>*)(X + base + (ok ? o + W * (pc % P) : 0));
#pragma unroll
            for (int w = 0; w < W; ++w) {
                v[q * W + w] = ok ? (double)t[w] : 0.0;
                amax = fmax(amax, fabs(v[q * W + w]));
            }
        }
    } else if (mode == 1) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int64_t ch = tid + 256 * c;
            const int64_t info = ch < nch ? cinfo[ch] : 0;
            const int64_t o0 = info >> 4;
            const int cnt = (int)(info & 15);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool ok = e < cnt;
                const double x = (double)X[base + (ok ? o0 + e * S.cstride : 0)];
                v[c * 8 + e] = ok ? x : 0.0;
                amax = fmax(amax, fabs(v[c * 8 + e]));
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int64_t ch = tid + 256 * c;
            const bool in = ch < nch;
            const gmem<int64_t>* ko = koff + 8 * (in ? ch : 0);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t o = ko[e];
                const bool ok = in && o >= 0;
                const double x = (double)X[base + (ok ? o : 0)];
                v[c * 8 + e] = ok ? x : 0.0;
                amax = fmax(amax, fabs(v[c * 8 + e]));
            }
        }
    }
    for (int s = 32; s > 0; s >>= 1) amax = fmax(amax, __shfl_xor(amax, s));
    if ((tid & 63) == 0) red[tid >> 6] = amax;
    __syncthreads();
    amax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int e = 0;
    if (amax > 0.0) {
        int E;
        frexp(amax, &E);
        e = E - 1;
    }
    if (tid == 0) ((gmem<int32_t>*)S.exps)[row] = e;
    constexpr int64_t TS = XR * SPLIT_BK;   // elements between the terms of one stage image
    if (mode == 0) {
#pragma unroll
        for (int q = 0; q < CPT * P; ++q) {
            const int64_t pc = tid + 256 * q, ch = pc / P;
            if (ch >= nch) break;
            uint32_t w1[W / 2], w2[W / 2], w3[W / 2];
#pragma unroll
            for (int h = 0; h < W / 2; ++h) {
                double t1[2], t2[2], t3[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const double x = ldexp(v[q * W + 2 * h + u], -e);
                    t1[u] = rn_bf16(x);
                    const double rest = x - t1[u];
                    t2[u] = rn_bf16(rest);
                    t3[u] = rn_bf16(rest - t2[u]);
                }
                w1[h] = pack2(t1[0], t1[1]);
                w2[h] = pack2(t2[0], t2[1]);
                w3[h] = pack2(t3[0], t3[1]);
            }
            gmem<uint16_t>* out = panels + panel_off(row, 8 * ch + W * (pc % P), 0, a.Kp);
            if constexpr (W == 2) {
                *(gmem<uint32_t>*)out = w1[0];
                *(gmem<uint32_t>*)(out + TS) = w2[0];
                *(gmem<uint32_t>*)(out + 2 * TS) = w3[0];
            } else {
                *(gmem<u32x2>*)out = u32x2{w1[0], w1[1]};
                *(gmem<u32x2>*)(out + TS) = u32x2{w2[0], w2[1]};
                *(gmem<u32x2>*)(out + 2 * TS) = u32x2{w3[0], w3[1]};
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int64_t ch = tid + 256 * c;
            if (ch >= nch) break;
            double t1[8], t2[8], t3[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double x = ldexp(v[c * 8 + q], -e);
                t1[q] = rn_bf16(x);
                const double rest = x - t1[q];
                t2[q] = rn_bf16(rest);
                t3[q] = rn_bf16(rest - t2[q]);
            }
            gmem<u32x4>* out = (gmem<u32x4>*)(panels + panel_off(row, 8 * ch, 0, a.Kp));
            out[0] = u32x4{pack2(t1[0], t1[1]), pack2(t1[2], t1[3]), pack2(t1[4], t1[5]), pack2(t1[6], t1[7])};
            out[TS / 8] = u32x4{pack2(t2[0], t2[1]), pack2(t2[2], t2[3]), pack2(t2[4], t2[5]), pack2(t2[6], t2[7])};
            out[2 * TS / 8] =
                u32x4{pack2(t3[0], t3[1]), pack2(t3[2], t3[3]), pack2(t3[4], t3[5]), pack2(t3[6], t3[7])};
        }
    }
}

// ---------------------------------------------------------------------------
// FP8 (OCP E4M3) form.  Term p is stored scaled by 2^(4(p-1)) so that it stays
// in E4M3's normal range; the product kernel undoes the scale through the
// matrix instruction's per-operand E8M0 scales.  Stage images hold 64 K
// positions of one byte: [term][128 rows][four 16-byte chunks], the chunks of
// row r permuted by (r >> 3) & 3 (the fragment reads take 32 consecutive rows
// per half-wave; an LDS read-pattern probe on MI355X found this permutation as
// fast as a linear read, where (r >> 1) & 3 took 1.55x and no permutation 2.9x).
constexpr int F8_BK = 64;

__host__ __device__ __forceinline__ int xswz8(int r, int c) { return c ^ ((r >> 3) & 3); }

__host__ __device__ __forceinline__ int64_t panel_off8(int64_t row, int64_t k, int term, int64_t Kp) {
    const int64_t rt = row / XR, kt = k / F8_BK;
    const int rr = (int)(row % XR), kk = (int)(k % F8_BK);
    return ((rt * (Kp / F8_BK) + kt) * 3 + term) * (int64_t)(XR * F8_BK) + rr * F8_BK +
           xswz8(rr, kk >> 4) * 16 + (kk & 15);
}

// Round to nearest even on the E4M3 grid: 4 significant bits, spacing 2^-9
// below the smallest normal 2^-6, saturating at +-448.
__device__ __forceinline__ double rn_e4m3(double x) {
    if (x == 0.0) return x;
    int E;
    frexp(x, &E);
    const int lead = E - 1 > -6 ? E - 1 : -6;
    const double q = ldexp(rint(ldexp(x, -(lead - 3))), lead - 3);
    return fmin(fmax(q, -448.0), 448.0);
}

// E4M3 code of a value already on the grid: sign, 4-bit exponent (bias 7),
// 3-bit fraction; exponent 0 holds the subnormals m * 2^-9.
__device__ __forceinline__ uint32_t e4m3_code(double q) {
    const uint32_t sgn = q < 0.0 ? 0x80u : 0u;
    const double a = fabs(q);
    if (a == 0.0) return sgn;
    int E;
    const double m = frexp(a, &E);
    const int e = E - 1 + 7;
    if (e >= 1) return sgn | ((uint32_t)e << 3) | (uint32_t)((m * 2.0 - 1.0) * 8.0);
    return sgn | (uint32_t)(a * 512.0);
}

__device__ __forceinline__ uint32_t pack4_e4m3(const double* t) {
    return e4m3_code(t[0]) | (e4m3_code(t[1]) << 8) | (e4m3_code(t[2]) << 16) | (e4m3_code(t[3]) << 24);
}

// One block per slice, like k_split; a thread owns chunks of sixteen positions
// (one 16-byte chunk of each term image).
template <typename T, int CPT, bool VEC>
__global__ __launch_bounds__(256) void k_split8(SplitArgs a) {
    __shared__ double red[4];
    if (a.bp && a.bp->alpha == 0.0) return;   // a batch member with alpha = 0 reads neither input
    const gmem<T>* X = (const gmem<T>*)(a.bp ? (a.slot == 0 ? a.bp->A : a.bp->B) : a.X);
    const gmem<int64_t>* koff = (const gmem<int64_t>*)a.koff;
    const int64_t row = xcd_item(blockIdx.x, a.nrows);
    const int tid = threadIdx.x;
    const int64_t base = grp_off(a.rows, row, a.slot);
    const int64_t nch = a.Kt / 16;
    double v[CPT][16];
    double amax = 0.0;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t ch = tid + 256 * c;
        const bool in = ch < nch;
        const gmem<int64_t>* ko = koff + 16 * (in ? ch : 0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (VEC) {
                typedef T v16 __attribute__((ext_vector_type(16 / sizeof(T))));
                constexpr int W = 16 / sizeof(T);
                const int64_t o = ko[8 * h];
                const bool ok = in && o >= 0;
                const gmem<v16>* p = (const gmem<v16>*)(X + base + (ok ? o : 0));
#pragma unroll
                for (int q = 0; q < 8 / W; ++q) {
                    const v16 t = p[q];
#pragma unroll
                    for (int w = 0; w < W; ++w) v[c][8 * h + q * W + w] = ok ? (double)t[w] : 0.0;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int64_t o = ko[8 * h + e];
                    const bool ok = in && o >= 0;
                    const double x = (double)X[base + (ok ? o : 0)];
                    v[c][8 * h + e] = ok ? x : 0.0;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) amax = fmax(amax, fabs(v[c][e]));
    }
    for (int s = 32; s > 0; s >>= 1) amax = fmax(amax, __shfl_xor(amax, s));
    if ((tid & 63) == 0) red[tid >> 6] = amax;
    __syncthreads();
    amax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int e = 0;
    if (amax > 0.0) {
        int E;
        frexp(amax, &E);
        e = E - 1;
    }
    if (tid == 0) ((gmem<int32_t>*)a.exps)[row] = e;
    constexpr int64_t TS = XR * F8_BK;   // bytes between the terms of one stage image
    gmem<uint8_t>* pan = (gmem<uint8_t>*)a.panels;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t ch = tid + 256 * c;
        if (ch >= nch) break;
        double t1[16], t2[16], t3[16];   // t2, t3 as stored: scaled by 2^4 and 2^8
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const double x = ldexp(v[c][q], -e);
            t1[q] = rn_e4m3(x);
            const double r1 = x - t1[q];
            t2[q] = rn_e4m3(ldexp(r1, 4));
            t3[q] = rn_e4m3(ldexp(r1 - ldexp(t2[q], -4), 8));
        }
        gmem<u32x4>* out = (gmem<u32x4>*)(pan + panel_off8(row, 16 * ch, 0, a.Kp));
        out[0] = u32x4{pack4_e4m3(t1), pack4_e4m3(t1 + 4), pack4_e4m3(t1 + 8), pack4_e4m3(t1 + 12)};
        out[TS / 16] = u32x4{pack4_e4m3(t2), pack4_e4m3(t2 + 4), pack4_e4m3(t2 + 8), pack4_e4m3(t2 + 12)};
        out[2 * TS / 16] = u32x4{pack4_e4m3(t3), pack4_e4m3(t3 + 4), pack4_e4m3(t3 + 8), pack4_e4m3(t3 + 12)};
    }
}

struct X3Args {
    const BatchPtrs* bp;  // batches: C, alpha and beta from the member's staged entry (C, alpha, beta unused)
    const uint16_t* tA;   // stage images of A's terms (panel_off layout)
    const uint16_t* tB;   // stage images of B's terms
    const int32_t* eA;
    const int32_t* eB;
    void* C;
    GtDims m, n;          // C offsets (sC)
    int64_t M, N, Kp, mt, nt, ntiles;
    double alpha, beta;
};


typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt immediates (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8); a field at its maximum does not wait.
constexpr int wait_vm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
constexpr int kWaitLgkm0 = 15 | (3 << 14) | (7 << 4);

// One block = eight waves on a 256 (m) x 128 (n) tile; wave (wm, wn) owns
// 64 m x 64 n, four by four blocks of 16 x 16.  A stage (32 K positions of all
// three terms: two stage images of A, one of B, 72 KB) arrives in LDS by DMA
// while the previous stage is multiplied; each wave copies six 1 KB pieces of
// A and three of B per stage.  Work per stage and wave: 96 MFMAs against 24
// fragment reads of 16 bytes per lane.  NP: term products kept (6: p+q <= 4;
// ablations 3: p+q <= 3, and 9: all).
template <typename T, int NP = 6>
__global__ __launch_bounds__(64 * XWAVES) void k_x3(X3Args a) {
    static_assert(NP == 3 || NP == 6 || NP == 9, "3, 6 or 9 term products");
    constexpr int NVA = 2 * XSTAGE / 16, NVB = XSTAGE / 16;   // uint4 per A / B stage
    constexpr int PA = 2 * XSTAGE / XPIECE / XWAVES;          // DMA pieces per wave: 6 of A
    constexpr int PB = XSTAGE / XPIECE / XWAVES;              // and 3 of B
    constexpr int NT = 64 * XWAVES;
    static_assert(PB * XWAVES * XPIECE == XSTAGE && PA == 2 * PB, "stage pieces");
    // One array per buffer: every DMA and every fragment read names its
    // buffer statically.
    __shared__ uint4 sA0[NVA], sA1[NVA], sB0[NVB], sB1[NVB];
    __shared__ int64_t sCm[XBM], sCn[XBN];
    __shared__ int32_t sEm[XBM], sEn[XBN];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar DMA bases
    const int wm = wid & 3, wn = wid >> 2;
    // tile order: contiguous per XCD, then groups of eight m-tiles sweeping n,
    // so the blocks resident on one XCD share stage images in its L2
    const int64_t L = xcd_item(blockIdx.x, a.ntiles);
    constexpr int64_t GM = 8;
    const int64_t g = L / (GM * a.nt), first = g * GM;
    const int64_t gm = a.mt - first < GM ? a.mt - first : GM;
    const int64_t r = L - g * GM * a.nt;
    const int64_t mt = first + r % gm, nt = r / gm;
    const int64_t m_base = mt * XBM, n_base = nt * XBN;
    for (int i = tid; i < XBM; i += NT) {
        const int64_t m = m_base + i;
        sCm[i] = m < a.M ? grp_off(a.m, m, 2) : -1;
        sEm[i] = m < a.M ? a.eA[m] : 0;
    }
    for (int i = tid; i < XBN; i += NT) {
        const int64_t n = n_base + i;
        sCn[i] = n < a.N ? grp_off(a.n, n, 2) : -1;
        sEn[i] = n < a.N ? a.eB[n] : 0;
    }
    __syncthreads();

    const double alpha = a.bp ? a.bp->alpha : a.alpha, beta_d = a.bp ? a.bp->beta : a.beta;
    // alpha = 0 (a batch member): no stage is loaded; the epilogue writes beta * C
    const int64_t ktiles = alpha == 0.0 ? 0 : a.Kp / SPLIT_BK;
    // A's stage kt: the images of row tiles 2 mt and 2 mt + 1; B's: row tile nt
    const char* gA = (const char*)a.tA + 2 * mt * ktiles * XSTAGE;
    const char* gB = (const char*)a.tB + nt * ktiles * XSTAGE;
    const uint32_t loff = (uint32_t)lane * 16u;
    auto dma = [&](int64_t kt, uint4* sa, uint4* sb) {
#pragma unroll
        for (int e = 0; e < PA; ++e) {
            const int piece = wid + XWAVES * e;                     // 0 .. 47
            const int img = e < PA / 2 ? 0 : 1;                     // pieces 0-23: row tile 2 mt
            const char* src = gA + (img * ktiles + kt) * XSTAGE + (piece - img * (XSTAGE / XPIECE)) * XPIECE;
            __builtin_amdgcn_global_load_lds(src + loff, (lds_void_t*)(sa + piece * 64), 16, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < PB; ++e) {
            const int piece = wid + XWAVES * e;                     // 0 .. 23
            __builtin_amdgcn_global_load_lds(gB + kt * XSTAGE + piece * XPIECE + loff,
                                             (lds_void_t*)(sb + piece * 64), 16, 0, 0);
        }
    };

    // fragment: this lane's 8 consecutive k (logical chunk lane/16) of one row
    const int r16 = lane & 15, ch = lane >> 4;
    auto frag = [&](const uint4* st, int term, int row) -> bf8 {
        const uint4 v = st[(term * XR + row) * 4 + xswz(row, ch)];
        return __builtin_bit_cast(bf8, v);
    };
    // this wave's m rows lie in image wm / 2 of the A stage
    const int aimg = (wm >> 1) * (NVA / 2), arow = (wm & 1) * 64;

    f4 big[4][4], small[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            big[i][j] = f4{0, 0, 0, 0};
            small[i][j] = f4{0, 0, 0, 0};
        }

    // The MFMA row operand is the B side (n), so a lane holds
    // D[n = 4*(lane/16) + q][m = lane % 16].
    auto mma = [&](f4 (&acc)[4][4], const bf8 (&fb)[4], const bf8 (&fa)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[i], fa[j], acc[i][j], 0, 0, 0);
    };
    auto load_b = [&](const uint4* sb, int t, bf8 (&fb)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) fb[i] = frag(sb, t, wn * 64 + i * 16 + r16);
    };
    auto load_a = [&](const uint4* sa, int t, bf8 (&fa)[4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) fa[j] = frag(sa + aimg, t, arow + j * 16 + r16);
    };
    // Each group's fragments are requested before the previous group's MFMAs
    // are issued, so the LDS latency runs under matrix work; sched_barrier(0)
    // holds this order (the scheduler would otherwise hoist every read of the
    // step and run out of registers).
    auto compute = [&](const uint4* sa, const uint4* sb) {
        bf8 b1[4], b2[4], b3[4], a1[4], a2[4], a3[4];
        if constexpr (NP == 3) {
            // t_A1 t_B1, then t_A1 t_B2 and t_A2 t_B1
            load_b(sb, 0, b1);
            load_a(sa, 0, a1);
            load_b(sb, 1, b2);
            __builtin_amdgcn_sched_barrier(0);
            mma(big, b1, a1);
            __builtin_amdgcn_sched_barrier(0);
            load_a(sa, 1, a2);
            __builtin_amdgcn_sched_barrier(0);
            mma(small, b2, a1);
            mma(small, b1, a2);
            __builtin_amdgcn_sched_barrier(0);
            return;
        }
        load_b(sb, 0, b1);
        load_a(sa, 0, a1);
        load_b(sb, 2, b3);
        __builtin_amdgcn_sched_barrier(0);
        load_b(sb, 1, b2);
        __builtin_amdgcn_sched_barrier(0);
        mma(big, b1, a1);      // t_A1 t_B1
        mma(small, b3, a1);    // t_A1 t_B3
        __builtin_amdgcn_sched_barrier(0);
        load_a(sa, 1, a2);
        __builtin_amdgcn_sched_barrier(0);
        mma(small, b2, a1);    // t_A1 t_B2
        __builtin_amdgcn_sched_barrier(0);
        load_a(sa, 2, a3);
        __builtin_amdgcn_sched_barrier(0);
        mma(small, b1, a2);    // t_A2 t_B1
        mma(small, b2, a2);    // t_A2 t_B2
        __builtin_amdgcn_sched_barrier(0);
        mma(small, b1, a3);    // t_A3 t_B1
        if constexpr (NP == 9) {
            mma(small, b3, a2);    // t_A2 t_B3
            mma(small, b2, a3);    // t_A3 t_B2
            mma(small, b3, a3);    // t_A3 t_B3
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    // Stage kt sits in (sa, sb); stage kt + 1 goes into (na, nb), which every
    // wave finished reading in the previous step.  ktiles is even (the host
    // pads K) and every step issues its DMA -- past the end it reloads the
    // last stage into the buffer nobody reads again -- so the loop body has no
    // conditional DMA and names every buffer statically.
    auto step = [&](int64_t kt, const uint4* sa, const uint4* sb, uint4* na, uint4* nb) {
        __builtin_amdgcn_s_waitcnt(wait_vm(0));    // stage kt landed
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);    // this wave's reads of the previous stage are done
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        dma(kt + 1 < ktiles ? kt + 1 : ktiles - 1, na, nb);
        compute(sa, sb);
    };
    if (ktiles > 0) dma(0, sA0, sB0);
    for (int64_t kt = 0; kt < ktiles; kt += 2) {
        step(kt, sA0, sB0, sA1, sB1);
        step(kt + 1, sA1, sB1, sA0, sB0);
    }
    __builtin_amdgcn_s_waitcnt(wait_vm(0));   // the trailing reload lands before the block exits

    gmem<T>* C = (gmem<T>*)(a.bp ? a.bp->C : a.C);
    const T beta = (T)beta_d;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int nl = wn * 64 + i * 16 + 4 * (lane >> 4) + q;
            const int64_t cn = sCn[nl];
            if (cn < 0) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ml = wm * 64 + j * 16 + (lane & 15);
                const int64_t cm = sCm[ml];
                if (cm < 0) continue;
                // the two FP32 partials add exactly in FP64
                const double v = alpha * ldexp((double)big[i][j][q] + (double)small[i][j][q], sEm[ml] + sEn[nl]);
                gmem<T>* cp = C + cn + cm;
                T out = (T)v;
                if (beta_d != 0.0) out += beta * (*cp);
                *cp = out;
            }
        }
}

typedef int i8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

// E8M0 scale of term p (0-based): the stored term is 2^(4p) times the true one.
constexpr int kScale[3] = {127, 123, 119};

// FP8 product kernel: the block and stage structure of k_x3 (256 x 128 tile,
// eight waves of 64 x 64, double-buffered DMA stages of 72 KB) with 64 K
// positions per stage and v_mfma_scale_f32_32x32x64_f8f6f4: a wave holds two
// by two blocks of 32 x 32.  Operand lane l supplies row l % 32 and the 32
// bytes of K half l / 32; the accumulator holds D[8 (q/4) + 4 (l/32) + q % 4]
// [l % 32] (both checked with an exact one-wave probe on MI355X).  The
// instruction's per-operand E8M0 scales undo the terms' 2^(4(p-1)), so the five
// small products share one FP32 accumulator.  Work per stage and wave: 24
// MFMAs of 64 x 32 x 32 x 2 flops against 24 fragment reads of 16 bytes.
template <typename T>
__global__ __launch_bounds__(64 * XWAVES) void k_x3_8(X3Args a) {
    constexpr int NVA = 2 * XSTAGE / 16, NVB = XSTAGE / 16;
    constexpr int PA = 2 * XSTAGE / XPIECE / XWAVES, PB = XSTAGE / XPIECE / XWAVES;
    constexpr int NT = 64 * XWAVES;
    __shared__ uint4 sA0[NVA], sA1[NVA], sB0[NVB], sB1[NVB];
    __shared__ int64_t sCm[XBM], sCn[XBN];
    __shared__ int32_t sEm[XBM], sEn[XBN];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wid & 3, wn = wid >> 2;
    const int64_t L = xcd_item(blockIdx.x, a.ntiles);
    constexpr int64_t GM = 8;
    const int64_t g = L / (GM * a.nt), first = g * GM;
    const int64_t gm = a.mt - first < GM ? a.mt - first : GM;
    const int64_t r = L - g * GM * a.nt;
    const int64_t mt = first + r % gm, nt = r / gm;
    const int64_t m_base = mt * XBM, n_base = nt * XBN;
    for (int i = tid; i < XBM; i += NT) {
        const int64_t m = m_base + i;
        sCm[i] = m < a.M ? grp_off(a.m, m, 2) : -1;
        sEm[i] = m < a.M ? a.eA[m] : 0;
    }
    for (int i = tid; i < XBN; i += NT) {
        const int64_t n = n_base + i;
        sCn[i] = n < a.N ? grp_off(a.n, n, 2) : -1;
        sEn[i] = n < a.N ? a.eB[n] : 0;
    }
    __syncthreads();

    const double alpha = a.bp ? a.bp->alpha : a.alpha, beta_d = a.bp ? a.bp->beta : a.beta;
    const int64_t ktiles = alpha == 0.0 ? 0 : a.Kp / F8_BK;
    const char* gA = (const char*)a.tA + 2 * mt * ktiles * XSTAGE;
    const char* gB = (const char*)a.tB + nt * ktiles * XSTAGE;
    const uint32_t loff = (uint32_t)lane * 16u;
    auto dma = [&](int64_t kt, uint4* sa, uint4* sb) {
#pragma unroll
        for (int e = 0; e < PA; ++e) {
            const int piece = wid + XWAVES * e;
            const int img = e < PA / 2 ? 0 : 1;
            const char* src = gA + (img * ktiles + kt) * XSTAGE + (piece - img * (XSTAGE / XPIECE)) * XPIECE;
            __builtin_amdgcn_global_load_lds(src + loff, (lds_void_t*)(sa + piece * 64), 16, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < PB; ++e) {
            const int piece = wid + XWAVES * e;
            __builtin_amdgcn_global_load_lds(gB + kt * XSTAGE + piece * XPIECE + loff,
                                             (lds_void_t*)(sb + piece * 64), 16, 0, 0);
        }
    };

    const int r32 = lane & 31, hk = lane >> 5;
    auto frag = [&](const uint4* st, int term, int row) -> i8v {
        const uint4* rp = st + (term * XR + row) * 4;
        const uint4 lo = rp[xswz8(row, 2 * hk)], hi = rp[xswz8(row, 2 * hk + 1)];
        i8v v;
        v[0] = (int)lo.x; v[1] = (int)lo.y; v[2] = (int)lo.z; v[3] = (int)lo.w;
        v[4] = (int)hi.x; v[5] = (int)hi.y; v[6] = (int)hi.z; v[7] = (int)hi.w;
        return v;
    };
    const int aimg = (wm >> 1) * (NVA / 2), arow = (wm & 1) * 64;

    f16v big[2][2], small[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            big[i][j] = f16v{};
            small[i][j] = f16v{};
        }
    // first operand: the B side (n), second: the A side (m)
    auto mma = [&](f16v (&acc)[2][2], const i8v (&fb)[2], const i8v (&fa)[2], int sb, int sa) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fb[i], fa[j], acc[i][j], 0, 0, 0, sb, 0, sa);
    };
    auto load_b = [&](const uint4* sb, int t, i8v (&fb)[2]) {
#pragma unroll
        for (int i = 0; i < 2; ++i) fb[i] = frag(sb, t, wn * 64 + i * 32 + r32);
    };
    auto load_a = [&](const uint4* sa, int t, i8v (&fa)[2]) {
#pragma unroll
        for (int j = 0; j < 2; ++j) fa[j] = frag(sa + aimg, t, arow + j * 32 + r32);
    };
    auto compute = [&](const uint4* sa, const uint4* sb) {
        i8v b1[2], b2[2], b3[2], a1[2], a2[2], a3[2];
        load_b(sb, 0, b1);
        load_a(sa, 0, a1);
        load_b(sb, 2, b3);
        __builtin_amdgcn_sched_barrier(0);
        load_b(sb, 1, b2);
        __builtin_amdgcn_sched_barrier(0);
        mma(big, b1, a1, kScale[0], kScale[0]);      // t_A1 t_B1
        mma(small, b3, a1, kScale[2], kScale[0]);    // t_A1 t_B3
        __builtin_amdgcn_sched_barrier(0);
        load_a(sa, 1, a2);
        __builtin_amdgcn_sched_barrier(0);
        mma(small, b2, a1, kScale[1], kScale[0]);    // t_A1 t_B2
        __builtin_amdgcn_sched_barrier(0);
        load_a(sa, 2, a3);
        __builtin_amdgcn_sched_barrier(0);
        mma(small, b1, a2, kScale[0], kScale[1]);    // t_A2 t_B1
        mma(small, b2, a2, kScale[1], kScale[1]);    // t_A2 t_B2
        __builtin_amdgcn_sched_barrier(0);
        mma(small, b1, a3, kScale[0], kScale[2]);    // t_A3 t_B1
        __builtin_amdgcn_sched_barrier(0);
    };
    auto step = [&](int64_t kt, const uint4* sa, const uint4* sb, uint4* na, uint4* nb) {
        __builtin_amdgcn_s_waitcnt(wait_vm(0));
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        dma(kt + 1 < ktiles ? kt + 1 : ktiles - 1, na, nb);
        compute(sa, sb);
    };
    if (ktiles > 0) dma(0, sA0, sB0);
    for (int64_t kt = 0; kt < ktiles; kt += 2) {
        step(kt, sA0, sB0, sA1, sB1);
        step(kt + 1, sA1, sB1, sA0, sB0);
    }
    __builtin_amdgcn_s_waitcnt(wait_vm(0));

    gmem<T>* C = (gmem<T>*)(a.bp ? a.bp->C : a.C);
    const T beta = (T)beta_d;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int nl = wn * 64 + i * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
            const int64_t cn = sCn[nl];
            if (cn < 0) continue;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int ml = wm * 64 + j * 32 + (lane & 31);
                const int64_t cm = sCm[ml];
                if (cm < 0) continue;
                const double v = alpha * ldexp((double)big[i][j][q] + (double)small[i][j][q], sEm[ml] + sEn[nl]);
                gmem<T>* cp = C + cn + cm;
                T out = (T)v;
                if (beta_d != 0.0) out += beta * (*cp);
                *cp = out;
            }
        }
}

// ---------------------------------------------------------------------------
// Workspace layout inside p->d_split: K offsets of A | of B | terms A | terms B |
// exps A | exps B
// | chunk tables of A | of B (affine chunks, BF16 form)
enum { L_KOA = 0, L_KOB, L_TA, L_TB, L_EA, L_EB, L_KP, L_RA, L_RB, L_KT, L_VA, L_VB,
       L_CIA, L_CIB, L_CSA, L_CSB, L_AFA, L_AFB };

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

tc_status prepare_split(tc_plan_s* p) {
    if (p->d_split) return TC_OK;
    if (allocation_forbidden()) return fail_unprepared();
    const bool fp8 = p->spec.compute == TC_FP8X3;
    const int SB = fp8 ? F8_BK : SPLIT_BK;   // K positions per product-kernel stage
    const int64_t tb = fp8 ? 1 : 2;          // bytes per term element
    const GemmView& gv = p->gv;
    // 8 x 8 blocks: a k_split thread's chunk of eight positions is a run of
    // eight along A's contiguous index, and the eight chunks of a block read
    // eight consecutive elements along B's in every load
    std::vector<int64_t> tab = build_ktab(gv.k, 2 * SPLIT_BK, 8);
    // padded to a whole number of two-stage turns of the product kernel's
    // buffer rotation; the padding positions (-1) hold zero terms
    const int64_t Kt = (int64_t)tab.size() / 2;
    const int64_t Kp = round_up(Kt, 2 * SB);
    std::vector<int64_t> ko[2] = {std::vector<int64_t>(Kp, -1), std::vector<int64_t>(Kp, -1)};
    for (int64_t k = 0; k < Kt; ++k) {
        ko[0][k] = tab[2 * k];
        ko[1][k] = tab[2 * k + 1];
    }
    int64_t RA = round_up(std::max<int64_t>(1, gv.M), XBM), RB = round_up(std::max<int64_t>(1, gv.N), XBN);
    int64_t off = 0;
    int64_t* L = p->split_layout;
    L[L_KOA] = off;  off += round_up(Kp * 8, 256);
    L[L_KOB] = off;  off += round_up(Kp * 8, 256);
    L[L_TA] = off;   off += round_up(3 * RA * Kp * tb, 256);
    L[L_TB] = off;   off += round_up(3 * RB * Kp * tb, 256);
    L[L_EA] = off;   off += round_up(RA * 4, 256);
    L[L_EB] = off;   off += round_up(RB * 4, 256);
    L[L_CIA] = off;  off += round_up(std::max<int64_t>(1, Kt / 8) * 8, 256);
    L[L_CIB] = off;  off += round_up(std::max<int64_t>(1, Kt / 8) * 8, 256);
    L[L_KP] = Kp; L[L_RA] = RA; L[L_RB] = RB; L[L_KT] = Kt;
    // Chunk-vector reads for a side: every chunk of eight positions is eight
    // consecutive elements (or eight padding entries), starting at an element
    // offset that, with every row offset, keeps 16-byte alignment (the operand
    // pointer's own alignment is checked per call).
    const int64_t W = 16 / p->spec.elem_bytes();
    for (int side = 0; side < 2; ++side) {
        bool vec = Kt > 0;
        for (int64_t c = 0; vec && c < Kt / 8; ++c) {
            const int64_t o0 = ko[side][8 * c];
            for (int e = 1; vec && e < 8; ++e) {
                const int64_t o = ko[side][8 * c + e];
                vec = o0 < 0 ? o < 0 : o == o0 + e;
            }
            vec = vec && (o0 < 0 || o0 % W == 0);
        }
        const std::vector<GtDim>& g = side == 0 ? gv.m : gv.n;
        for (const GtDim& d : g) vec = vec && (side == 0 ? d.sA : d.sB) % W == 0;
        L[side == 0 ? L_VA : L_VB] = vec ? 1 : 0;
    }
    // Affine chunks: in every chunk of eight positions the valid entries are a
    // prefix at offsets o0 + e * s, with one s for the whole side.
    std::vector<int64_t> cinfo[2];
    for (int side = 0; side < 2; ++side) {
        bool aff = Kt > 0 && !fp8;
        int64_t stride = 0;
        cinfo[side].assign((size_t)std::max<int64_t>(1, Kt / 8), 0);
        for (int64_t c = 0; aff && c < Kt / 8; ++c) {
            const int64_t* k = ko[side].data() + 8 * c;
            int cnt = 0;
            while (cnt < 8 && k[cnt] >= 0) ++cnt;
            for (int e = cnt; aff && e < 8; ++e) aff = k[e] < 0;
            if (cnt >= 2) {
                if (stride == 0) stride = k[1] - k[0];
                for (int e = 1; aff && e < cnt; ++e) aff = k[e] == k[0] + e * stride;
            }
            aff = aff && (cnt == 0 || (k[0] >= 0 && k[0] < (INT64_C(1) << 58)));
            cinfo[side][c] = cnt == 0 ? 0 : k[0] * 16 + cnt;
        }
        L[side == 0 ? L_AFA : L_AFB] = aff ? 1 : 0;
        L[side == 0 ? L_CSA : L_CSB] = stride;
    }
    hipError_t e = hipMalloc(&p->d_split, (size_t)std::max<int64_t>(off, 256));
    if (e != hipSuccess) {
        p->d_split = nullptr;
        return fail(TC_E_NOMEM, std::string("hipMalloc split workspace: ") + hipGetErrorString(e));
    }
    p->split_bytes = off;
    // zero everything once: padded rows of the stage images stay zero
    e = hipMemset(p->d_split, 0, (size_t)off);
    for (int side = 0; side < 2 && e == hipSuccess && Kp > 0; ++side)
        e = hipMemcpy((char*)p->d_split + L[side == 0 ? L_KOA : L_KOB], ko[side].data(), (size_t)(Kp * 8),
                      hipMemcpyHostToDevice);
    for (int side = 0; side < 2 && e == hipSuccess && Kt > 0; ++side)
        e = hipMemcpy((char*)p->d_split + L[side == 0 ? L_CIA : L_CIB], cinfo[side].data(),
                      cinfo[side].size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "split workspace set-up");
    return TC_OK;
}

// BF16 terms of slices longer than k_split2 takes (more than 8192 positions).
template <typename T>
static void launch_split_long(const SplitArgs& s, dim3 grid, dim3 blk, hipStream_t st) {
    hipLaunchKernelGGL(k_split_long<T>, grid, blk, 0, st, s);
}

// FP8 terms for up to 8192 contracted positions (k_split8 keeps a slice in
// registers; longer slices are refused by run_split).
template <typename T>
static void launch_split8(const SplitArgs& s, int64_t nch, bool vec, dim3 grid, dim3 blk, hipStream_t st) {
    const int cpt = nch <= 256 ? 1 : 2;
    if (vec) {
        if (cpt == 1) hipLaunchKernelGGL((k_split8<T, 1, true>), grid, blk, 0, st, s);
        else hipLaunchKernelGGL((k_split8<T, 2, true>), grid, blk, 0, st, s);
    } else {
        if (cpt == 1) hipLaunchKernelGGL((k_split8<T, 1, false>), grid, blk, 0, st, s);
        else hipLaunchKernelGGL((k_split8<T, 2, false>), grid, blk, 0, st, s);
    }
}

// The split form's launches: the two split passes and the product.  With `bp`
// (a batch member) the operands, alpha and beta are read from the member's
// staged entry when the kernels run, and the split passes take element loads
// (the pointers' alignment is not known ahead).
static tc_status launch_split_form(tc_plan_s* p, const void* A, const void* B, void* C, double alpha,
                                   double beta, const BatchPtrs* bp, hipStream_t st);

tc_status run_split(tc_plan_s* p, const void* A, const void* B, void* C, double alpha, double beta,
                    hipStream_t st) {
    return launch_split_form(p, A, B, C, alpha, beta, nullptr, st);
}

int64_t split_positions(const tc_plan_s* p) { return p->d_split ? p->split_layout[L_KT] : 0; }

tc_status run_split_batched(tc_plan_s* p, const BatchPtrs* bp, hipStream_t st) {
    return launch_split_form(p, nullptr, nullptr, nullptr, 0.0, 0.0, bp, st);
}

static tc_status launch_split_form(tc_plan_s* p, const void* A, const void* B, void* C, double alpha,
                                   double beta, const BatchPtrs* bp, hipStream_t st) {
    const GemmView& gv = p->gv;
    const bool f64 = p->spec.dtype == TC_F64;
    const bool fp8 = p->spec.compute == TC_FP8X3;
    if (fp8 && p->split_layout[L_KT] > 8192)
        return fail(TC_E_UNSUPPORTED, "FP8 split form takes at most 8192 contracted positions");
    const int64_t* L = p->split_layout;
    char* w = (char*)p->d_split;
    const int64_t Kp = L[L_KP], RA = L[L_RA], RB = L[L_RB];
    uint16_t* tA = (uint16_t*)(w + L[L_TA]);
    uint16_t* tB = (uint16_t*)(w + L[L_TB]);
    int32_t* eA = (int32_t*)(w + L[L_EA]);
    int32_t* eB = (int32_t*)(w + L[L_EB]);
    hipError_t e;
    if (!fp8 && L[L_KT] > 0 && L[L_KT] / 8 <= 1024) {
        // both sides in one launch
        Split2Args s2{};
        s2.bp = bp;
        s2.Kp = Kp;
        s2.Kt = L[L_KT];
        for (int side = 0; side < 2; ++side) {
            SplitSide& S = s2.s[side];
            S.X = side == 0 ? A : B;
            const std::vector<GtDim>& g = side == 0 ? gv.m : gv.n;
            S.rows.n = (int)g.size();
            for (int d = 0; d < S.rows.n; ++d) S.rows.d[d] = g[d];
            S.slot = side;
            S.koff = (const int64_t*)(w + L[side == 0 ? L_KOA : L_KOB]);
            S.cinfo = (const int64_t*)(w + L[side == 0 ? L_CIA : L_CIB]);
            S.cstride = L[side == 0 ? L_CSA : L_CSB];
            S.nrows = std::max<int64_t>(0, side == 0 ? gv.M : gv.N);
            S.panels = side == 0 ? tA : tB;
            S.exps = side == 0 ? eA : eB;
            const bool vec = !bp && L[side == 0 ? L_VA : L_VB] != 0 && ((uintptr_t)S.X) % 16 == 0;
            S.mode = vec ? 0 : L[side == 0 ? L_AFA : L_AFB] ? 1 : 2;
        }
        const int64_t blocks = s2.s[0].nrows + s2.s[1].nrows;
        if (blocks > 0x7fffffff) return fail(TC_E_EXTENT, "too many slices for one launch");
        if (blocks > 0) {
            const int64_t nch = s2.Kt / 8;
            const int cpt = nch <= 256 ? 1 : nch <= 512 ? 2 : 4;
            const dim3 grid((unsigned)blocks), blk(256);
            if (f64) {
                if (cpt == 1) hipLaunchKernelGGL((k_split2<double, 1>), grid, blk, 0, st, s2);
                else if (cpt == 2) hipLaunchKernelGGL((k_split2<double, 2>), grid, blk, 0, st, s2);
                else hipLaunchKernelGGL((k_split2<double, 4>), grid, blk, 0, st, s2);
            } else {
                if (cpt == 1) hipLaunchKernelGGL((k_split2<float, 1>), grid, blk, 0, st, s2);
                else if (cpt == 2) hipLaunchKernelGGL((k_split2<float, 2>), grid, blk, 0, st, s2);
                else hipLaunchKernelGGL((k_split2<float, 4>), grid, blk, 0, st, s2);
            }
            e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "split kernel launch");
        }
    }
    for (int side = 0; side < 2; ++side) {
        if (!fp8 && L[L_KT] > 0 && L[L_KT] / 8 <= 1024) break;   // done above
        SplitArgs s{};
        s.X = side == 0 ? A : B;
        s.bp = bp;
        const std::vector<GtDim>& g = side == 0 ? gv.m : gv.n;
        s.rows.n = (int)g.size();
        for (int d = 0; d < s.rows.n; ++d) s.rows.d[d] = g[d];
        s.slot = side;
        s.koff = (const int64_t*)(w + L[side == 0 ? L_KOA : L_KOB]);
        s.nrows = side == 0 ? gv.M : gv.N;
        s.Kp = Kp;
        s.Kt = L[L_KT];
        s.panels = side == 0 ? tA : tB;
        s.exps = side == 0 ? eA : eB;
        if (s.nrows <= 0 || L[L_KT] == 0) continue;   // no K: the exponents stay 0, the terms empty
        if (s.nrows > 0x7fffffff) return fail(TC_E_EXTENT, "too many slices for one launch");
        const dim3 grid((unsigned)s.nrows), blk(256);
        const bool vec = !bp && L[side == 0 ? L_VA : L_VB] != 0 && ((uintptr_t)s.X) % 16 == 0;
        if (fp8) {
            const int64_t nch = s.Kt / 16;   // chunks of sixteen positions (Kt is a multiple of 64)
            if (f64) launch_split8<double>(s, nch, vec, grid, blk, st);
            else launch_split8<float>(s, nch, vec, grid, blk, st);
        } else {
            if (f64) launch_split_long<double>(s, grid, blk, st);
            else launch_split_long<float>(s, grid, blk, st);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "split kernel launch");
    }
    X3Args x{};
    x.bp = bp;
    x.tA = tA; x.tB = tB;
    x.eA = eA; x.eB = eB;
    x.C = C;
    x.m.n = (int)gv.m.size();
    for (int d = 0; d < x.m.n; ++d) x.m.d[d] = gv.m[d];
    x.n.n = (int)gv.n.size();
    for (int d = 0; d < x.n.n; ++d) x.n.d[d] = gv.n[d];
    x.M = gv.M; x.N = gv.N; x.Kp = Kp;
    x.mt = RA / XBM; x.nt = RB / XBN;
    x.ntiles = x.mt * x.nt;
    x.alpha = alpha; x.beta = beta;
    if (x.ntiles > 0x7fffffff) return fail(TC_E_EXTENT, "too many output tiles for one launch");
    const dim3 xg((unsigned)x.ntiles), xb(64 * XWAVES);
    if (fp8) {
        if (f64) hipLaunchKernelGGL(k_x3_8<double>, xg, xb, 0, st, x);
        else hipLaunchKernelGGL(k_x3_8<float>, xg, xb, 0, st, x);
    } else if (p->split_products == 3) {
        if (f64) hipLaunchKernelGGL((k_x3<double, 3>), xg, xb, 0, st, x);
        else hipLaunchKernelGGL((k_x3<float, 3>), xg, xb, 0, st, x);
    } else if (p->split_products == 9) {
        if (f64) hipLaunchKernelGGL((k_x3<double, 9>), xg, xb, 0, st, x);
        else hipLaunchKernelGGL((k_x3<float, 9>), xg, xb, 0, st, x);
    } else {
        if (f64) hipLaunchKernelGGL(k_x3<double>, xg, xb, 0, st, x);
        else hipLaunchKernelGGL(k_x3<float>, xg, xb, 0, st, x);
    }
    e = hipGetLastError();
    return e == hipSuccess ? TC_OK : hip_fail(e, "split product kernel launch");
}

}  // namespace tc

extern "C" tc_status tc_set_split_products(tc_plan_t p, int products) {
    using namespace tc;
    if (!p) return fail(TC_E_NULL, "plan is NULL");
    if (p->spec.compute != TC_BF16X3) return fail(TC_E_UNSUPPORTED, "term-product count applies to TC_BF16X3 plans");
    if (products != 3 && products != 6 && products != 9)
        return fail(TC_E_UNSUPPORTED, "term products: 3 (p+q <= 3), 6 (p+q <= 4) or 9 (all)");
    p->split_products = products;
    if (p->real) p->real->split_products = products;
    return TC_OK;
}

extern "C" tc_status tc_split_terms(tc_plan_t p, int side, void* terms, int32_t* exps, int64_t* rows,
                                    int64_t* kp) {
    using namespace tc;
    if (!p || !rows || !kp) return fail(TC_E_NULL, "NULL argument");
    if (p->real) return tc_split_terms(p->real, side, terms, exps, rows, kp);   // complex: the embedded operands
    if (p->spec.compute == TC_NATIVE) return fail(TC_E_UNSUPPORTED, "plan has no split precision");
    if (!p->d_split) return fail(TC_E_UNSUPPORTED, "no split computed yet: run tc_contract first");
    if (side != 0 && side != 1) return fail(TC_E_VARIANT, "side must be 0 (A) or 1 (B)");
    const int64_t* L = p->split_layout;
    const int64_t Kp = L[L_KP];
    const int64_t R = side == 0 ? L[L_RA] : L[L_RB];
    const int64_t n = side == 0 ? p->gv.M : p->gv.N;
    *rows = n;
    *kp = Kp;
    if (!terms && !exps) return TC_OK;
    char* w = (char*)p->d_split;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronize");
    if (terms) {
        // the device keeps stage images; hand back [term][row][Kp]
        const bool fp8 = p->spec.compute == TC_FP8X3;
        const int64_t elems = 3 * R * Kp, tb = fp8 ? 1 : 2;
        std::vector<uint8_t> img((size_t)(elems * tb));
        e = hipMemcpy(img.data(), w + L[side == 0 ? L_TA : L_TB], (size_t)(elems * tb), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "copy split terms");
        for (int t = 0; t < 3; ++t)
            for (int64_t r = 0; r < n; ++r)
                for (int64_t k = 0; k < Kp; ++k) {
                    const int64_t o = (t * n + r) * Kp + k;
                    if (fp8) ((uint8_t*)terms)[o] = img[(size_t)panel_off8(r, k, t, Kp)];
                    else ((uint16_t*)terms)[o] = ((const uint16_t*)img.data())[(size_t)panel_off(r, k, t, Kp)];
                }
    }
    if (exps) {
        e = hipMemcpy(exps, w + L[side == 0 ? L_EA : L_EB], (size_t)(n * 4), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "copy split exponents");
    }
    return TC_OK;
}
