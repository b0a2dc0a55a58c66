// HBM-bound kernels: the fused small-K streaming contraction, the SIMT bodies
// of the dot/axpy/gemv/ger family members, strided copies, the C := beta*C
// prologue and the cache-touch kernel used by the micro-benchmarks.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "devutil.h"
#include "launch.h"

namespace tc {

// ---------------------------------------------------------------------------
// Fused streaming kernel for small contracted extents, K <= KT.
//
// C is written along its unit-stride M dimension; each thread owns VEC
// consecutive m and loads their A rows (VEC x K) into registers, then
// computes R columns n of C (R * rpb columns per block, rpb = 256 / tpr rows
// of threads) and retires.  Measured on MI355X, a one-shot grid whose blocks
// each write a few KB and exit streams writes markedly faster than persistent
// blocks walking long column ranges: the blocks in flight then cover one
// compact window of C.  Stores are 16-byte non-temporal vector stores.  Work per
// output: 2K flops, one store; A comes from L2 after its first touch.
template <typename T, int KT, int VEC, int R>
__global__ __launch_bounds__(256) void k_stream(const T* __restrict__ A, const T* __restrict__ B,
                                                T* __restrict__ C, StreamArgs a) {
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    const int tid = threadIdx.x;
    const int tpr = a.tpr;
    const int rpb = 256 / tpr;
    const int64_t span = (int64_t)tpr * VEC;
    const int64_t mblocks = (a.M + span - 1) / span;
    const int64_t mb = blockIdx.x % mblocks;
    const int64_t nb = blockIdx.x / mblocks;
    const int64_t m0 = mb * span + (int64_t)(tid % tpr) * VEC;
    const bool full = (m0 + VEC <= a.M);
    const T alpha = (T)a.alpha, beta = (T)a.beta;

    // A rows of the thread's m, clamped to the last valid m (always a legal
    // address) and selected to zero past the edge: no branch around a load.
    T av[VEC][KT];
    const bool avec = full && a.sAm == 1;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        if (k < a.K) {                                   // uniform
            const T* ap = A + a.kA[k];
            if (avec && ((uintptr_t)(ap + m0)) % (sizeof(T) * VEC) == 0) {
                vec_t t = *(const vec_t*)(ap + m0);
#pragma unroll
                for (int v = 0; v < VEC; ++v) av[v][k] = t[v];
            } else {
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const int64_t m = min(m0 + v, a.M - 1);
                    const T x = ap[m * a.sAm];
                    av[v][k] = (m0 + v < a.M) ? x : (T)0;
                }
            }
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) av[v][k] = (T)0;
        }
    }

    const int64_t n_first = nb * (int64_t)(R * rpb) + tid / tpr;
    T bv[R][KT];
    int64_t offC[R];
    bool nok[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int64_t n = n_first + (int64_t)q * rpb;
        nok[q] = n < a.N;
        const int64_t nn = nok[q] ? n : 0;
        int64_t offB = 0, oc = 0;
        if (a.n.n == 1) {
            offB = nn * a.n.d[0].sB;
            oc = nn * a.n.d[0].sC;
        } else {
            int64_t rem = nn;
            for (int d = 0; d < a.n.n; ++d) {
                int64_t r = divmod(rem, a.n.d[d].ext);
                offB += r * a.n.d[d].sB;
                oc += r * a.n.d[d].sC;
            }
        }
        offC[q] = oc;
#pragma unroll
        for (int k = 0; k < KT; ++k) bv[q][k] = (k < a.K) ? B[offB + a.kB[k]] : (T)0;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        T out[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            T acc = 0;
#pragma unroll
            for (int k = 0; k < KT; ++k) acc += av[v][k] * bv[q][k];
            out[v] = alpha * acc;
        }
        if (!nok[q]) continue;
        T* cp = C + offC[q] + m0;
        if (a.beta != 0.0) {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                if (m0 + v < a.M) out[v] += beta * cp[v];
        }
        if (full && (((uintptr_t)cp) % (sizeof(T) * VEC) == 0)) {
            vec_t val;
#pragma unroll
            for (int v = 0; v < VEC; ++v) val[v] = out[v];
            __builtin_nontemporal_store(val, (vec_t*)cp);
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                if (m0 + v < a.M) cp[v] = out[v];
        }
    }
}

// Straight-line form of k_stream for unit-stride, vector-aligned A and C.
// Each wave covers 64 * VEC consecutive m of one column n: the column index is
// wave-uniform (readfirstlane; a compile-time zero when one block spans
// TPR = 256 threads), so everything that depends on n -- the N-dimension
// decomposition, the B loads, the column guard -- runs on the scalar unit.
// All R columns' B values are requested before the first FMA, so the block
// waits for one round of scalar loads, not R; the vector path is a fixed
// sequence of A loads, FMAs and one 16-byte non-temporal store per column.
// TPR threads (64, 128 or 256) share one M span of TPR * VEC elements; the
// host covers the largest multiple of 64 * VEC in M with this kernel and
// hands the remainder to k_stream.
template <typename T, int KT, int VEC, int R, int TPR, bool BETA>
__global__ __launch_bounds__(256) void k_stream_wave(const T* __restrict__ A, const T* __restrict__ B,
                                                     T* __restrict__ C, StreamArgs a) {
    static_assert(TPR >= 64 && TPR <= 256, "a wave must lie inside one column");
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    constexpr int RPB = 256 / TPR;
    constexpr int SPAN = TPR * VEC;
    const int tid = threadIdx.x;
    const uint32_t mblocks = (uint32_t)(a.M / SPAN);
    const uint32_t mb = blockIdx.x % mblocks;
    const uint32_t nb = blockIdx.x / mblocks;
    const int row = TPR == 256 ? 0 : __builtin_amdgcn_readfirstlane(tid / TPR);
    const int64_t m0 = (int64_t)mb * SPAN + (tid % TPR) * VEC;
    const T alpha = (T)a.alpha;

    int64_t offB[R], offC[R];
    bool ok[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int64_t n = ((int64_t)nb * R + q) * RPB + row;
        ok[q] = n < a.N;
        const int64_t nn = ok[q] ? n : a.N - 1;
        if (a.n.n == 1) {
            offB[q] = nn * a.n.d[0].sB;
            offC[q] = nn * a.n.d[0].sC;
        } else {
            int64_t rem = nn, ob = 0, oc = 0;
            for (int d = 0; d < a.n.n; ++d) {
                int64_t r = divmod(rem, a.n.d[d].ext);
                ob += r * a.n.d[d].sB;
                oc += r * a.n.d[d].sC;
            }
            offB[q] = ob;
            offC[q] = oc;
        }
    }
    // kA/kB entries K..KT-1 repeat entry K-1 (the host pads them): every load
    // is in bounds and unconditional, and the padded terms are zeroed by
    // selects, not branches.
    T bv[R][KT];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            const T x = B[offB[q] + a.kB[k]];
            bv[q][k] = (k < a.K) ? x : (T)0;
        }
    T av[VEC][KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        const vec_t t = *(const vec_t*)(A + a.kA[k] + m0);
#pragma unroll
        for (int v = 0; v < VEC; ++v) av[v][k] = (k < a.K) ? t[v] : (T)0;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (!ok[q]) break;   // columns grow with q: the rest are past N too
        vec_t val;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            T acc = 0;
#pragma unroll
            for (int k = 0; k < KT; ++k) acc += av[v][k] * bv[q][k];
            val[v] = alpha * acc;
        }
        vec_t* cp = (vec_t*)(C + offC[q] + m0);
        if (BETA) {
            const vec_t old = *cp;
            const T beta = (T)a.beta;
#pragma unroll
            for (int v = 0; v < VEC; ++v) val[v] += beta * old[v];
        }
        __builtin_nontemporal_store(val, cp);
    }
}

static int next_pow2(int64_t x) {
    int p = 1;
    while (p < x && p < 256) p <<= 1;
    return p;
}

// Threads per M span of k_stream_wave.  Measured on MI355X at n^3 outputs,
// n = 384..1024: one wave per span streams as fast as or faster than 128 or
// 256 threads per span, and it covers every M that is a multiple of 64 * VEC.
constexpr int kWaveTpr = 64;

// columns per thread row: four for K <= 8, fewer for larger K (registers)
static int stream_r(int K) { return K <= 8 ? 4 : K <= 16 ? 2 : 1; }

// columns per wave of k_stream_wave, measured at a = b = c = 1024 (FP64):
// four for up to 4 positions (eight: 2-3% slower), eight for 5..8 (1.339 ms
// against 1.378 ms with four), four for 9..16 (2.61 ms against 3.06 ms with
// two), one beyond; more columns per wave read each wave's A rows once for
// more stores
static int wave_r(int K) { return K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 4 : 1; }

void stream_shape(bool f64, StreamArgs& a) {
    const int VEC = f64 ? 2 : 4;
    int64_t lanes = (a.M + VEC - 1) / VEC;
    a.tpr = next_pow2(std::max<int64_t>(1, lanes));
    a.rows_per_block = (int64_t)stream_r(a.K) * (256 / a.tpr);
}

int64_t stream_grid(bool f64, const StreamArgs& a) {
    const int VEC = f64 ? 2 : 4;
    int64_t span = (int64_t)a.tpr * VEC;
    int64_t mblocks = (a.M + span - 1) / span;
    int64_t nchunks = (a.N + a.rows_per_block - 1) / a.rows_per_block;
    return mblocks * nchunks;
}

template <typename T, int VEC, bool BETA>
static void launch_wave(const T* A, const T* B, T* C, const StreamArgs& w, unsigned grid, hipStream_t st) {
    dim3 g(grid), b(256);
    if (w.K <= 4) hipLaunchKernelGGL((k_stream_wave<T, 4, VEC, 4, kWaveTpr, BETA>), g, b, 0, st, A, B, C, w);
    else if (w.K <= 8) hipLaunchKernelGGL((k_stream_wave<T, 8, VEC, 8, kWaveTpr, BETA>), g, b, 0, st, A, B, C, w);
    else if (w.K <= 16) hipLaunchKernelGGL((k_stream_wave<T, 16, VEC, 4, kWaveTpr, BETA>), g, b, 0, st, A, B, C, w);
    else hipLaunchKernelGGL((k_stream_wave<T, 32, VEC, 1, kWaveTpr, BETA>), g, b, 0, st, A, B, C, w);
}

// The largest multiple of one wave span (64 * VEC) in M goes to k_stream_wave
// when A is unit-stride along M and every A row and C column it touches is
// 16-byte aligned; k_stream covers the rest of M (and everything else).
template <typename T, int VEC>
static hipError_t stream_dispatch(StreamArgs& a, hipStream_t st) {
    if (a.M <= 0 || a.N <= 0) return hipSuccess;
    const T* A = (const T*)a.A;
    const T* B = (const T*)a.B;
    T* C = (T*)a.C;
    constexpr int64_t span = (int64_t)kWaveTpr * VEC;
    bool wave = a.sAm == 1 && ((uintptr_t)A) % (sizeof(T) * VEC) == 0 && ((uintptr_t)C) % (sizeof(T) * VEC) == 0;
    for (int d = 0; wave && d < a.n.n; ++d) wave = a.n.d[d].sC % VEC == 0;
    for (int k = 0; wave && k < a.K; ++k) wave = a.kA[k] % VEC == 0;
    const int64_t mbulk = wave ? a.M / span * span : 0;
    if (mbulk > 0) {
        StreamArgs w = a;
        w.M = mbulk;
        for (int k = w.K; k < GT_SMALLK_MAX; ++k) {
            w.kA[k] = w.kA[w.K - 1];
            w.kB[k] = w.kB[w.K - 1];
        }
        const int64_t cols = (int64_t)(256 / kWaveTpr) * wave_r(a.K);
        const int64_t grid = (mbulk / span) * ((a.N + cols - 1) / cols);
        if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
        if (a.beta != 0.0) launch_wave<T, VEC, true>(A, B, C, w, (unsigned)grid, st);
        else launch_wave<T, VEC, false>(A, B, C, w, (unsigned)grid, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || mbulk == a.M) return e;
    }
    StreamArgs t = a;
    t.A = A + mbulk;   // mbulk > 0 only where A is unit-stride along M
    t.C = C + mbulk;
    t.M = a.M - mbulk;
    stream_shape(sizeof(T) == 8, t);
    const int64_t grid = stream_grid(sizeof(T) == 8, t);
    if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
    dim3 g((unsigned)grid), b(256);
    const T* At = (const T*)t.A;
    T* Ct = (T*)t.C;
    if (t.K <= 4) hipLaunchKernelGGL((k_stream<T, 4, VEC, 4>), g, b, 0, st, At, B, Ct, t);
    else if (t.K <= 8) hipLaunchKernelGGL((k_stream<T, 8, VEC, 4>), g, b, 0, st, At, B, Ct, t);
    else if (t.K <= 16) hipLaunchKernelGGL((k_stream<T, 16, VEC, 2>), g, b, 0, st, At, B, Ct, t);
    else hipLaunchKernelGGL((k_stream<T, 32, VEC, 1>), g, b, 0, st, At, B, Ct, t);
    return hipGetLastError();
}

hipError_t launch_stream(bool f64, StreamArgs& a, hipStream_t st) {
    if (a.K > GT_SMALLK_MAX || a.K < 1) return hipErrorInvalidValue;
    return f64 ? stream_dispatch<double, 2>(a, st) : stream_dispatch<float, 4>(a, st);
}

// ---------------------------------------------------------------------------
// SIMT body of a family member: one thread per output element of one kernel
// invocation (kernel-internal free indices fastest, then the parallel loops,
// innermost first).  The in-launch contracted loops run in order; every
// iteration is one invocation: C is read, the kernel's sum over its kept
// contracted index is added (times alpha) and C is written back.
template <typename T>
__global__ __launch_bounds__(256) void k_simt(SimtArgs a) {
    const T* __restrict__ A = (const T*)a.A;
    const T* __restrict__ B = (const T*)a.B;
    T* C = (T*)a.C;
    const T alpha = (T)a.alpha;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.total; idx += stride) {
        int64_t rem = idx, oA = 0, oB = 0, oC = 0;
        for (int d = 0; d < a.out.n; ++d) {
            int64_t r = divmod(rem, a.out.d[d].ext);
            oA += r * a.out.d[d].sA;
            oB += r * a.out.d[d].sB;
            oC += r * a.out.d[d].sC;
        }
        int64_t ctr[GT_MAXD];
        for (int d = 0; d < a.pass.n; ++d) ctr[d] = 0;
        int64_t pA = 0, pB = 0;
        for (int64_t p = 0; p < a.npass; ++p) {
            T acc = 0;
            const T* ap = A + oA + pA;
            const T* bp = B + oB + pB;
            for (int64_t k = 0; k < a.kb.ext; ++k) acc += ap[k * a.kb.sA] * bp[k * a.kb.sB];
            T c = C[oC];
            C[oC] = c + alpha * acc;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);   // next invocation re-reads C
            for (int d = a.pass.n - 1; d >= 0; --d) {  // innermost pass loop fastest
                pA += a.pass.d[d].sA;
                pB += a.pass.d[d].sB;
                if (++ctr[d] < a.pass.d[d].ext) break;
                pA -= a.pass.d[d].sA * a.pass.d[d].ext;
                pB -= a.pass.d[d].sB * a.pass.d[d].ext;
                ctr[d] = 0;
            }
        }
    }
}

// The same body with G lanes per output element, for long kernels (dot or
// gemv rows of many elements) with few outputs per launch: the lanes of a
// group take every G-th term of the kernel's sum, an xor-shuffle tree adds the
// G partial sums, and the group's first lane updates C.  Invocations of one
// output still run in order.
template <typename T, int G>
__global__ __launch_bounds__(256) void k_simt_group(SimtArgs a) {
    const T* __restrict__ A = (const T*)a.A;
    const T* __restrict__ B = (const T*)a.B;
    T* C = (T*)a.C;
    const T alpha = (T)a.alpha;
    const int l = threadIdx.x % G;
    const int64_t gstride = (int64_t)gridDim.x * (blockDim.x / G);
    for (int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; idx < a.total; idx += gstride) {
        int64_t rem = idx, oA = 0, oB = 0, oC = 0;
        for (int d = 0; d < a.out.n; ++d) {
            int64_t r = divmod(rem, a.out.d[d].ext);
            oA += r * a.out.d[d].sA;
            oB += r * a.out.d[d].sB;
            oC += r * a.out.d[d].sC;
        }
        int64_t ctr[GT_MAXD];
        for (int d = 0; d < a.pass.n; ++d) ctr[d] = 0;
        int64_t pA = 0, pB = 0;
        for (int64_t p = 0; p < a.npass; ++p) {
            T acc = 0;
            const T* ap = A + oA + pA;
            const T* bp = B + oB + pB;
            for (int64_t k = l; k < a.kb.ext; k += G) acc += ap[k * a.kb.sA] * bp[k * a.kb.sB];
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
            if (l == 0) {
                T c = C[oC];
                C[oC] = c + alpha * acc;
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);   // next invocation re-reads C
            for (int d = a.pass.n - 1; d >= 0; --d) {  // innermost pass loop fastest
                pA += a.pass.d[d].sA;
                pB += a.pass.d[d].sB;
                if (++ctr[d] < a.pass.d[d].ext) break;
                pA -= a.pass.d[d].sA * a.pass.d[d].ext;
                pB -= a.pass.d[d].sB * a.pass.d[d].ext;
                ctr[d] = 0;
            }
        }
    }
}

static unsigned grid_for(int64_t total, int64_t cap = 65536) {
    int64_t g = (total + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Lanes per output: one while the outputs alone fill the device (about 2^18
// threads), else as many as the kernel length uses (8 or 64).
int simt_group(int64_t total, int64_t klen) {
    if (total >= (1 << 18) || klen < 16) return 1;
    return (klen >= 128 && total * 64 <= (1LL << 22)) ? 64 : 8;
}

hipError_t launch_simt(bool f64, SimtArgs& a, hipStream_t st) {
    if (a.total <= 0 || a.npass <= 0) return hipSuccess;
    const int G = simt_group(a.total, a.kb.ext);
    dim3 g(grid_for(a.total * G, 1 << 20)), b(256);
    if (G == 64) {
        if (f64) hipLaunchKernelGGL((k_simt_group<double, 64>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_simt_group<float, 64>), g, b, 0, st, a);
    } else if (G == 8) {
        if (f64) hipLaunchKernelGGL((k_simt_group<double, 8>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_simt_group<float, 8>), g, b, 0, st, a);
    } else {
        if (f64) hipLaunchKernelGGL(k_simt<double>, g, b, 0, st, a);
        else hipLaunchKernelGGL(k_simt<float>, g, b, 0, st, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_copy(CopyArgs a) {
    const T* __restrict__ src = (const T*)a.src;
    T* __restrict__ dst = (T*)a.dst;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.total; idx += stride) {
        int64_t rem = idx, os = 0, od = 0;
        for (int d = 0; d < a.dims.n; ++d) {
            int64_t r = divmod(rem, a.dims.d[d].ext);
            os += r * a.dims.d[d].sA;
            od += r * a.dims.d[d].sC;
        }
        dst[od] = src[os];
    }
}

hipError_t launch_copy(bool f64, CopyArgs& a, hipStream_t st) {
    if (a.total <= 0) return hipSuccess;
    dim3 g(grid_for(a.total, 1 << 20)), b(256);
    if (f64) hipLaunchKernelGGL(k_copy<double>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_copy<float>, g, b, 0, st, a);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_scale(ScaleArgs a) {
    T* C = (T*)a.C;
    const T beta = (T)a.beta;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.total; idx += stride) {
        int64_t rem = idx, oc = 0;
        for (int d = 0; d < a.dims.n; ++d) oc += divmod(rem, a.dims.d[d].ext) * a.dims.d[d].sC;
        C[oc] = (a.beta == 0.0) ? (T)0 : beta * C[oc];
    }
}

hipError_t launch_scale(bool f64, ScaleArgs& a, hipStream_t st) {
    if (a.total <= 0) return hipSuccess;
    dim3 g(grid_for(a.total, 1 << 20)), b(256);
    if (f64) hipLaunchKernelGGL(k_scale<double>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_scale<float>, g, b, 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_touch(const float4* __restrict__ p, int64_t n4, float* sink) {
    float s = 0.f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        float4 v = p[i];
        s += v.x + v.y + v.z + v.w;
    }
    if (s == 1234.5678f) sink[0] = s;   // keeps the loads; practically never taken
}

hipError_t launch_touch(const void* p, int64_t bytes, float* sink, hipStream_t st) {
    int64_t n4 = bytes / 16;
    if (n4 <= 0) return hipSuccess;
    dim3 g(grid_for(n4, 8192)), b(256);
    hipLaunchKernelGGL(k_touch, g, b, 0, st, (const float4*)p, n4, sink);
    return hipGetLastError();
}

}  // namespace tc
