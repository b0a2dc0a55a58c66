// Host-side launchers of the HIP kernels.  All launches are asynchronous on
// the given stream and return hipSuccess or the launch error.
#pragma once

#include <hip/hip_runtime.h>

#include "gett.h"

namespace tc {

// Fused contraction for small contracted extents (K <= GT_SMALLK_MAX): C is
// streamed along its unit-stride M dimension, A's rows stay in registers.
hipError_t launch_stream(bool f64, StreamArgs& a, hipStream_t st);
// Choose threads-per-row and rows-per-block for the streaming kernel.
void stream_shape(bool f64, StreamArgs& a);
int64_t stream_grid(bool f64, const StreamArgs& a);

// Family-member bodies with dot/axpy/gemv/ger kernels: one thread per output
// element of one invocation.
hipError_t launch_simt(bool f64, SimtArgs& a, hipStream_t st);

// Matrix-core contraction (gemm-shaped members and the fused kernel).
hipError_t launch_mfma(bool f64, MfmaArgs& a, hipStream_t st);
void mfma_tiles(bool f64, MfmaArgs& a);
int mfma_bk(bool f64);
bool mfma_a_first(bool f64, int64_t M, int64_t N, int64_t K);
// ws_cap: largest workspace the caller can give (bytes)
int64_t mfma_split_plan(bool f64, int64_t M, int64_t N, int64_t Kpad, int64_t* slice_tiles, int64_t* ws_bytes,
                        int64_t ws_cap = 64LL << 20);

// Batches: tile shape 0 = 128x128, 1 = 64x64, 2 = 32x128; persistent kernel over a work
// list of (contraction, tile) pairs in eight per-XCD ranges (xstart: nine
// offsets), taken off eight atomic counters.
void mfma_tiles_shape(int shape, MfmaArgs& a);
bool mfma_kmajor_a(const MfmaArgs& a);
bool mfma_kmajor_b(const MfmaArgs& a);
hipError_t launch_mfma_batch(bool f64, int shape, bool ak, bool bk, const MfmaArgs* items, const BatchPtrs* ptrs,
                             const int2* work, const int* xstart, int nwork, int* counter, int grid, hipStream_t st);
int mfma_batch_occupancy(bool f64, int shape, bool ak, bool bk);
hipError_t launch_mfma_shape(bool f64, int shape, MfmaArgs& a, hipStream_t st);
// The same for split-BF16 tiles (FP64 or FP32 storage; one pass, no split K).
hipError_t launch_x3_batch(bool f64, int shape, bool ak, bool bk, const MfmaArgs* items, const BatchPtrs* ptrs,
                           const int2* work, const int* xstart, int nwork, int* counter, int grid, hipStream_t st);
int x3_batch_occupancy(bool f64, int shape, bool ak, bool bk);
hipError_t launch_x3_shape(bool f64, int shape, MfmaArgs& a, hipStream_t st);

// Strided copy (copy statements of the family) and C := beta*C prologue.
hipError_t launch_copy(bool f64, CopyArgs& a, hipStream_t st);
hipError_t launch_scale(bool f64, ScaleArgs& a, hipStream_t st);

// Cache set-up for micro-benchmarks: read `n` elements at `p` (touch) and
// accumulate into a sink so the reads are not removed.
hipError_t launch_touch(const void* p, int64_t bytes, float* sink, hipStream_t st);

}  // namespace tc
