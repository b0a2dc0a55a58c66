// HBM-bound kernels: the fused small-K streaming contraction, the SIMT bodies
// of the dot/axpy/gemv/ger family members, strided copies, the C := beta*C
// prologue and the cache-touch kernel used by the micro-benchmarks.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"

namespace tc {

// rem := rem / ext, returns rem % ext; 32-bit arithmetic when it fits
__device__ __forceinline__ int64_t divmod(int64_t& rem, int64_t ext) {
    if ((uint64_t)rem <= 0xffffffffull && (uint64_t)ext <= 0xffffffffull) {
        uint32_t r = (uint32_t)rem, e = (uint32_t)ext;
        uint32_t q = r / e;
        rem = q;
        return (int64_t)(r - q * e);
    }
    int64_t q = rem / ext;
    int64_t m = rem - q * ext;
    rem = q;
    return m;
}

// ---------------------------------------------------------------------------
// Fused streaming kernel, K <= KT.  Each thread owns VEC consecutive elements
// of C's unit-stride M dimension and keeps their A rows (VEC x K) in
// registers.  A block walks a range of N columns in chunks of R = 256/KT: the
// block first stages B[:, n] of the chunk's columns and their C offsets in LDS
// (one element per thread, generic strides decoded once), then every thread
// computes its VEC outputs of each column from broadcast LDS reads and writes
// them with one vector store.  Work per output: 2K flops and one 8-byte
// (FP64) store; A and B are read once.
template <typename T, int KT, int VEC>
__global__ __launch_bounds__(256) void k_stream(const T* __restrict__ A, const T* __restrict__ B,
                                                T* __restrict__ C, StreamArgs a) {
    constexpr int R = 256 / KT;
    __shared__ T Bs[R][KT];
    __shared__ int64_t Cs[R];
    const int tid = threadIdx.x;
    const int tpr = a.tpr;
    const int rpb = 256 / tpr;
    const int64_t span = (int64_t)tpr * VEC;
    const int64_t mblocks = (a.M + span - 1) / span;
    const int64_t mb = blockIdx.x % mblocks;
    const int64_t nb = blockIdx.x / mblocks;
    const int64_t m0 = mb * span + (int64_t)(tid % tpr) * VEC;
    const T alpha = (T)a.alpha, beta = (T)a.beta;

    T av[VEC][KT];
#pragma unroll
    for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int k = 0; k < KT; ++k)
            av[v][k] = (k < a.K && m0 + v < a.M) ? A[(m0 + v) * a.sAm + a.kA[k]] : (T)0;

    const int64_t n_lo = nb * a.rows_per_block;
    const int64_t n_hi = min(a.N, n_lo + a.rows_per_block);
    const bool full = (m0 + VEC <= a.M);
    const int lr = tid / tpr;
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    for (int64_t n0 = n_lo; n0 < n_hi; n0 += R) {
        {   // stage the chunk: thread (r, k) loads B[k, n0 + r]
            const int r = tid / KT, k = tid % KT;
            const int64_t n = n0 + r;
            T v = 0;
            if (n < n_hi) {
                int64_t offB = 0, offC = 0;
                if (a.n.n == 1) {
                    offB = n * a.n.d[0].sB;
                    offC = n * a.n.d[0].sC;
                } else {
                    int64_t rem = n;
                    for (int d = 0; d < a.n.n; ++d) {
                        int64_t q = divmod(rem, a.n.d[d].ext);
                        offB += q * a.n.d[d].sB;
                        offC += q * a.n.d[d].sC;
                    }
                }
                if (k < a.K) v = B[offB + a.kB[k]];
                if (k == 0) Cs[r] = offC;
            }
            Bs[r][k] = v;
        }
        __syncthreads();
        const int rows = (int)min<int64_t>(R, n_hi - n0);
#pragma unroll 2
        for (int r = lr; r < rows; r += rpb) {
            T out[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                T acc = 0;
#pragma unroll
                for (int k = 0; k < KT; ++k) acc += av[v][k] * Bs[r][k];
                out[v] = alpha * acc;
            }
            T* cp = C + Cs[r] + m0;
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
        __syncthreads();
    }
}

static int next_pow2(int64_t x) {
    int p = 1;
    while (p < x && p < 256) p <<= 1;
    return p;
}

void stream_shape(bool f64, StreamArgs& a) {
    const int VEC = f64 ? 2 : 4;
    int64_t lanes = (a.M + VEC - 1) / VEC;
    a.tpr = next_pow2(std::max<int64_t>(1, lanes));
    int rpb = 256 / a.tpr;
    int64_t span = (int64_t)a.tpr * VEC;
    int64_t mblocks = (a.M + span - 1) / span;
    int64_t row_groups = (a.N + rpb - 1) / rpb;
    const int64_t target = 8192;
    int64_t per = std::max<int64_t>(1, (row_groups * mblocks + target - 1) / target);
    a.rows_per_block = per * rpb;
}

int64_t stream_grid(bool f64, const StreamArgs& a) {
    const int VEC = f64 ? 2 : 4;
    int64_t span = (int64_t)a.tpr * VEC;
    int64_t mblocks = (a.M + span - 1) / span;
    int64_t nchunks = (a.N + a.rows_per_block - 1) / a.rows_per_block;
    return mblocks * nchunks;
}

template <typename T, int VEC>
static hipError_t stream_dispatch(StreamArgs& a, hipStream_t st) {
    int64_t grid = stream_grid(sizeof(T) == 8, a);
    if (grid <= 0) return hipSuccess;
    if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
    dim3 g((unsigned)grid), b(256);
    const T* A = (const T*)a.A;
    const T* B = (const T*)a.B;
    T* C = (T*)a.C;
    if (a.K <= 4) hipLaunchKernelGGL((k_stream<T, 4, VEC>), g, b, 0, st, A, B, C, a);
    else if (a.K <= 8) hipLaunchKernelGGL((k_stream<T, 8, VEC>), g, b, 0, st, A, B, C, a);
    else if (a.K <= 16) hipLaunchKernelGGL((k_stream<T, 16, VEC>), g, b, 0, st, A, B, C, a);
    else hipLaunchKernelGGL((k_stream<T, 32, VEC>), g, b, 0, st, A, B, C, a);
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

static unsigned grid_for(int64_t total, int64_t cap = 65536) {
    int64_t g = (total + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

hipError_t launch_simt(bool f64, SimtArgs& a, hipStream_t st) {
    if (a.total <= 0 || a.npass <= 0) return hipSuccess;
    dim3 g(grid_for(a.total, 1 << 20)), b(256);
    if (f64) hipLaunchKernelGGL(k_simt<double>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_simt<float>, g, b, 0, st, a);
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
