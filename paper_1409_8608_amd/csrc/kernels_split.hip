// Split-precision contraction on BF16 matrix cores (gfx950
// v_mfma_f32_16x16x32_bf16).
//
// 1. k_split: one block per slice (one row m of A's GEMM view, or one column n
//    of B's).  FP64 absmax over the slice -> exponent e = floor(log2(max)); the
//    scaled values x = v * 2^-e (exact) are split into three BF16 terms by
//    round-to-nearest-even, t1 = rn(x), t2 = rn(x - t1), t3 = rn(x - t1 - t2),
//    and packed K-contiguous ([term][row][Kp], Kp a multiple of 32) in the
//    K order of the plan's offset table.
// 2. k_x3: C tile = sum over the six term products t_A,p t_B,q with p+q <= 4.
//    The leading product and the five small ones accumulate in two FP32
//    accumulators over K chunks of 256; after each chunk both are added into an
//    FP64 running sum with Neumaier compensation.  Epilogue:
//    C = alpha * 2^(eA + eB) * (sum + comp) + beta * C.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "launch.h"
#include "plan.h"

namespace tc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int SPLIT_BK = 32;      // contracted positions per MFMA (16x16x32)
constexpr int SPLIT_CHUNK = 256;  // FP32 accumulation length before the FP64 fold
constexpr int XBM = 64, XBN = 128;

// Round-to-nearest-even to an 8-bit significand, unbounded exponent (the
// values stay far inside BF16's range after the per-slice scaling).
__device__ __forceinline__ double rn_bf16(double x) {
    int E;
    double m = frexp(x, &E);
    return ldexp(rint(ldexp(m, 8)), E - 8);
}

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
    GtDims rows;          // the side's free dims (slot selects the stride)
    int slot;             // 0: A side (sA, table column 0); 1: B side (sB, column 1)
    const int64_t* ktab;  // Kp pairs
    int64_t nrows, Kp, row_stride;   // packed row stride (elements)
    uint16_t* terms;      // [3][rows_padded][Kp]
    int64_t term_stride;  // elements between terms
    int32_t* exps;
};

template <typename T>
__global__ __launch_bounds__(256) void k_split(SplitArgs a) {
    __shared__ double red[4];
    const T* X = (const T*)a.X;
    const int64_t row = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t base = grp_off(a.rows, row, a.slot);
    double amax = 0.0;
    for (int64_t k = tid; k < a.Kp; k += 256) {
        int64_t o = a.ktab[2 * k + a.slot];
        double v = o >= 0 ? (double)X[base + o] : 0.0;
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
    if (tid == 0) a.exps[row] = e;
    uint16_t* t1 = a.terms + row * a.row_stride;
    uint16_t* t2 = t1 + a.term_stride;
    uint16_t* t3 = t2 + a.term_stride;
    for (int64_t k = tid; k < a.Kp; k += 256) {
        int64_t o = a.ktab[2 * k + a.slot];
        double x = o >= 0 ? ldexp((double)X[base + o], -e) : 0.0;
        double r1 = rn_bf16(x);
        double rest = x - r1;
        double r2 = rn_bf16(rest);
        double r3 = rn_bf16(rest - r2);
        t1[k] = bf16_bits(r1);
        t2[k] = bf16_bits(r2);
        t3[k] = bf16_bits(r3);
    }
}

struct X3Args {
    const uint16_t* tA;   // [3][rowsA][Kp]
    const uint16_t* tB;   // [3][rowsB][Kp]
    int64_t tsA, tsB;     // term strides (elements)
    const int32_t* eA;
    const int32_t* eB;
    void* C;
    GtDims m, n;          // C offsets (sC)
    int64_t M, N, Kp, mt, nt, ntiles;
    double alpha, beta;
};

__device__ __forceinline__ int64_t xcd_tile3(int64_t b, int64_t total) {
    const int64_t X = 8;
    int64_t xcd = b % X, idx = b / X;
    int64_t per = total / X, rem = total % X;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

template <typename T>
__global__ __launch_bounds__(256) void k_x3(X3Args a) {
    constexpr int BK = SPLIT_BK;
    constexpr int LDR = BK + 8;                  // padded row (bf16 elements): 80 bytes
    constexpr int FM = XBM / 32, FN = XBN / 32;  // 16x16 blocks per wave (wave tile 32 x 64)
    __shared__ uint16_t sA[2][3][XBM][LDR];
    __shared__ uint16_t sB[2][3][XBN][LDR];
    __shared__ int64_t sCm[XBM], sCn[XBN];
    __shared__ int32_t sEm[XBM], sEn[XBN];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid & 1, wn = wid >> 1;
    const int64_t tile = xcd_tile3(blockIdx.x, a.ntiles);
    const int64_t mt = tile % a.mt, nt = tile / a.mt;
    const int64_t m_base = mt * XBM, n_base = nt * XBN;
    for (int i = tid; i < XBM; i += 256) {
        int64_t m = m_base + i;
        sCm[i] = m < a.M ? grp_off(a.m, m, 2) : -1;
        sEm[i] = m < a.M ? a.eA[m] : 0;
    }
    for (int i = tid; i < XBN; i += 256) {
        int64_t n = n_base + i;
        sCn[i] = n < a.N ? grp_off(a.n, n, 2) : -1;
        sEn[i] = n < a.N ? a.eB[n] : 0;
    }

    // global -> LDS: 16-byte pieces, four per row and term
    constexpr int PA = 3 * XBM * 4 / 256, PB = 3 * XBN * 4 / 256;
    uint4 ra[PA], rb[PB];
    auto gload = [&](int64_t kt) {
#pragma unroll
        for (int e = 0; e < PA; ++e) {
            int idx = tid + 256 * e;
            int piece = idx & 3, row = (idx >> 2) % XBM, term = (idx >> 2) / XBM;
            const uint16_t* src = a.tA + term * a.tsA + (m_base + row) * a.Kp + kt * BK + piece * 8;
            ra[e] = *(const uint4*)src;
        }
#pragma unroll
        for (int e = 0; e < PB; ++e) {
            int idx = tid + 256 * e;
            int piece = idx & 3, row = (idx >> 2) % XBN, term = (idx >> 2) / XBN;
            const uint16_t* src = a.tB + term * a.tsB + (n_base + row) * a.Kp + kt * BK + piece * 8;
            rb[e] = *(const uint4*)src;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int e = 0; e < PA; ++e) {
            int idx = tid + 256 * e;
            int piece = idx & 3, row = (idx >> 2) % XBM, term = (idx >> 2) / XBM;
            *(uint4*)&sA[buf][term][row][piece * 8] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < PB; ++e) {
            int idx = tid + 256 * e;
            int piece = idx & 3, row = (idx >> 2) % XBN, term = (idx >> 2) / XBN;
            *(uint4*)&sB[buf][term][row][piece * 8] = rb[e];
        }
    };

    f4 big[FN][FM], small[FN][FM];
    double sum[FN][FM][4], comp[FN][FM][4];
#pragma unroll
    for (int i = 0; i < FN; ++i)
#pragma unroll
        for (int j = 0; j < FM; ++j) {
            big[i][j] = f4{0, 0, 0, 0};
            small[i][j] = f4{0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[i][j][q] = comp[i][j][q] = 0.0;
        }
    auto fold = [&]() {
#pragma unroll
        for (int i = 0; i < FN; ++i)
#pragma unroll
            for (int j = 0; j < FM; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // Neumaier: add the two chunk partials into (sum, comp)
                    double parts[2] = {(double)small[i][j][q], (double)big[i][j][q]};
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        double s = sum[i][j][q], x = parts[p], t = s + x;
                        comp[i][j][q] += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
                        sum[i][j][q] = t;
                    }
                    big[i][j][q] = 0.f;
                    small[i][j][q] = 0.f;
                }
    };

    const int64_t ktiles = a.Kp / BK;
    const int per_chunk = SPLIT_CHUNK / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int64_t kt = 0; kt < ktiles; ++kt) {
        const int buf = (int)(kt & 1);
        if (kt + 1 < ktiles) gload(kt + 1);
        // fragments: lane holds 8 consecutive k of row (lane % 16) at k offset 8*(lane/16)
        bf8 fa[3][FM], fb[3][FN];
        const int r16 = lane & 15, k8 = (lane >> 4) * 8;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
#pragma unroll
            for (int j = 0; j < FM; ++j)
                fa[t][j] = *(const bf8*)&sA[buf][t][wm * (XBM / 2) + j * 16 + r16][k8];
#pragma unroll
            for (int i = 0; i < FN; ++i)
                fb[t][i] = *(const bf8*)&sB[buf][t][wn * (XBN / 2) + i * 16 + r16][k8];
        }
        // five small products first, then the leading one; row operand = B side (n)
#pragma unroll
        for (int pq = 0; pq < 5; ++pq) {
            const int p = pq == 0 ? 0 : pq == 1 ? 1 : pq == 2 ? 0 : pq == 3 ? 2 : 1;   // A term
            const int q = pq == 0 ? 1 : pq == 1 ? 0 : pq == 2 ? 2 : pq == 3 ? 0 : 1;   // B term
#pragma unroll
            for (int i = 0; i < FN; ++i)
#pragma unroll
                for (int j = 0; j < FM; ++j)
                    small[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[q][i], fa[p][j], small[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < FN; ++i)
#pragma unroll
            for (int j = 0; j < FM; ++j)
                big[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[0][i], fa[0][j], big[i][j], 0, 0, 0);
        if ((kt + 1) % per_chunk == 0 || kt + 1 == ktiles) fold();
        if (kt + 1 < ktiles) sstore(buf ^ 1);
        __syncthreads();
    }

    // epilogue: lane holds D[n = 4*(lane/16) + q][m = lane % 16] of each block
    T* C = (T*)a.C;
    const T beta = (T)a.beta;
#pragma unroll
    for (int i = 0; i < FN; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int nl = wn * (XBN / 2) + i * 16 + 4 * (lane >> 4) + q;
            const int64_t cn = sCn[nl];
            if (cn < 0) continue;
#pragma unroll
            for (int j = 0; j < FM; ++j) {
                const int ml = wm * (XBM / 2) + j * 16 + (lane & 15);
                const int64_t cm = sCm[ml];
                if (cm < 0) continue;
                double v = a.alpha * ldexp(sum[i][j][q] + comp[i][j][q], sEm[ml] + sEn[nl]);
                T* cp = C + cn + cm;
                T out = (T)v;
                if (a.beta != 0.0) out += beta * (*cp);
                *cp = out;
            }
        }
}

// ---------------------------------------------------------------------------
// Workspace layout inside p->d_split: ktab | terms A | terms B | exps A | exps B
enum { L_KTAB = 0, L_TA, L_TB, L_EA, L_EB, L_KP, L_RA, L_RB };

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

tc_status prepare_split(tc_plan_s* p) {
    if (p->d_split) return TC_OK;
    if (p->spec.compute == TC_FP8X3) return fail(TC_E_UNSUPPORTED, "FP8 split terms are not built on the GPU");
    const GemmView& gv = p->gv;
    std::vector<int64_t> tab = build_ktab(gv.k, SPLIT_BK);
    int64_t Kp = (int64_t)tab.size() / 2;
    int64_t RA = round_up(std::max<int64_t>(1, gv.M), XBM), RB = round_up(std::max<int64_t>(1, gv.N), XBN);
    int64_t off = 0;
    int64_t* L = p->split_layout;
    L[L_KTAB] = off; off += round_up((int64_t)tab.size() * 8, 256);
    L[L_TA] = off;   off += round_up(3 * RA * Kp * 2, 256);
    L[L_TB] = off;   off += round_up(3 * RB * Kp * 2, 256);
    L[L_EA] = off;   off += round_up(RA * 4, 256);
    L[L_EB] = off;   off += round_up(RB * 4, 256);
    L[L_KP] = Kp; L[L_RA] = RA; L[L_RB] = RB;
    hipError_t e = hipMalloc(&p->d_split, (size_t)std::max<int64_t>(off, 256));
    if (e != hipSuccess) {
        p->d_split = nullptr;
        return fail(TC_E_NOMEM, std::string("hipMalloc split workspace: ") + hipGetErrorString(e));
    }
    p->split_bytes = off;
    // zero everything once: padded rows of the term buffers stay zero
    e = hipMemset(p->d_split, 0, (size_t)off);
    if (e == hipSuccess && !tab.empty())
        e = hipMemcpy((char*)p->d_split + L[L_KTAB], tab.data(), tab.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "split workspace set-up");
    return TC_OK;
}

tc_status run_split(tc_plan_s* p, const void* A, const void* B, void* C, double alpha, double beta,
                    hipStream_t st) {
    const GemmView& gv = p->gv;
    const bool f64 = p->spec.dtype == TC_F64;
    const int64_t* L = p->split_layout;
    char* w = (char*)p->d_split;
    const int64_t Kp = L[L_KP], RA = L[L_RA], RB = L[L_RB];
    uint16_t* tA = (uint16_t*)(w + L[L_TA]);
    uint16_t* tB = (uint16_t*)(w + L[L_TB]);
    int32_t* eA = (int32_t*)(w + L[L_EA]);
    int32_t* eB = (int32_t*)(w + L[L_EB]);
    const int64_t* ktab = (const int64_t*)(w + L[L_KTAB]);
    hipError_t e;
    for (int side = 0; side < 2; ++side) {
        SplitArgs s{};
        s.X = side == 0 ? A : B;
        const std::vector<GtDim>& g = side == 0 ? gv.m : gv.n;
        s.rows.n = (int)g.size();
        for (int d = 0; d < s.rows.n; ++d) s.rows.d[d] = g[d];
        s.slot = side;
        s.ktab = ktab;
        s.nrows = side == 0 ? gv.M : gv.N;
        s.Kp = Kp;
        s.row_stride = Kp;
        s.terms = side == 0 ? tA : tB;
        s.term_stride = (side == 0 ? RA : RB) * Kp;
        s.exps = side == 0 ? eA : eB;
        if (s.nrows <= 0) continue;
        if (f64) hipLaunchKernelGGL(k_split<double>, dim3((unsigned)s.nrows), dim3(256), 0, st, s);
        else hipLaunchKernelGGL(k_split<float>, dim3((unsigned)s.nrows), dim3(256), 0, st, s);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "split kernel launch");
    }
    X3Args x{};
    x.tA = tA; x.tB = tB;
    x.tsA = RA * Kp; x.tsB = RB * Kp;
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
    if (f64) hipLaunchKernelGGL(k_x3<double>, dim3((unsigned)x.ntiles), dim3(256), 0, st, x);
    else hipLaunchKernelGGL(k_x3<float>, dim3((unsigned)x.ntiles), dim3(256), 0, st, x);
    e = hipGetLastError();
    return e == hipSuccess ? TC_OK : hip_fail(e, "split product kernel launch");
}

}  // namespace tc

extern "C" tc_status tc_split_terms(tc_plan_t p, int side, void* terms, int32_t* exps, int64_t* rows,
                                    int64_t* kp) {
    using namespace tc;
    if (!p || !rows || !kp) return fail(TC_E_NULL, "NULL argument");
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
    if (terms)
        for (int t = 0; t < 3; ++t) {
            e = hipMemcpy((char*)terms + t * n * Kp * 2, w + L[side == 0 ? L_TA : L_TB] + t * R * Kp * 2,
                          (size_t)(n * Kp * 2), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "copy split terms");
        }
    if (exps) {
        e = hipMemcpy(exps, w + L[side == 0 ? L_EA : L_EB], (size_t)(n * 4), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "copy split exponents");
    }
    return TC_OK;
}
