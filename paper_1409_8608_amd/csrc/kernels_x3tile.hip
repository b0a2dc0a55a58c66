// Split-BF16 tile kernels for batches (the X3 form of the tile in
// mfma_tile.h): the persistent kernel over a group's work list, and a
// one-shot launch of one member's tiles that the batch tuner times.  Both
// stage element by element (batch members' K tables are not checked for
// chunk contiguity) and take one pass.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"
#include "mfma_tile.h"

namespace tc {

namespace {

constexpr int kXBK = 16;

// waves per block: eight (two per SIMD) for the 128 x 128 tiles, whose four-wave
// form takes all 256 VGPRs
template <int BM>
constexpr int x3_nw() { return BM == 128 ? 8 : 4; }

template <typename T, int BM, int BN, int AMODE, int BMODE>
__global__ __launch_bounds__(64 * x3_nw<BM>()) void k_mfma_x3(MfmaArgs a) {
    const int64_t t = xcd_tile(blockIdx.x, a.ntiles);
    mfma_tile<T, BM, BN, kXBK, AMODE, BMODE, false, false, true, x3_nw<BM>()>(a, a.A, a.B, a.C, a.alpha, a.beta, t, 0);
}

template <typename T, int BM, int BN>
hipError_t one_shot(const MfmaArgs& a, bool ak, bool bk, hipStream_t st) {
    if (a.ntiles <= 0) return hipSuccess;
    if (a.ntiles > 0x7fffffff) return hipErrorInvalidConfiguration;
    dim3 g((unsigned)a.ntiles), b(64 * x3_nw<BM>());
    if (ak && bk) hipLaunchKernelGGL((k_mfma_x3<T, BM, BN, 1, 1>), g, b, 0, st, a);
    else if (ak) hipLaunchKernelGGL((k_mfma_x3<T, BM, BN, 1, 0>), g, b, 0, st, a);
    else if (bk) hipLaunchKernelGGL((k_mfma_x3<T, BM, BN, 0, 1>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_mfma_x3<T, BM, BN, 0, 0>), g, b, 0, st, a);
    return hipGetLastError();
}

template <typename T, int BM, int BN>
hipError_t persistent(bool ak, bool bk, const MfmaArgs* items, const BatchPtrs* ptrs, const int2* work,
                      const int* xstart, int nwork, int* counter, int grid, hipStream_t st) {
    constexpr int NW = x3_nw<BM>();
    dim3 g(grid), b(64 * NW);
    // runs of up to 16 items when the list is long (as the native batch kernel)
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(16, (int64_t)nwork / ((int64_t)grid * 64)));
    if (ak && bk)
        hipLaunchKernelGGL((k_mfma_batch<T, BM, BN, kXBK, 1, 1, true, NW>), g, b, 0, st, items, ptrs, work, xstart, chunk, counter);
    else if (ak)
        hipLaunchKernelGGL((k_mfma_batch<T, BM, BN, kXBK, 1, 0, true, NW>), g, b, 0, st, items, ptrs, work, xstart, chunk, counter);
    else if (bk)
        hipLaunchKernelGGL((k_mfma_batch<T, BM, BN, kXBK, 0, 1, true, NW>), g, b, 0, st, items, ptrs, work, xstart, chunk, counter);
    else
        hipLaunchKernelGGL((k_mfma_batch<T, BM, BN, kXBK, 0, 0, true, NW>), g, b, 0, st, items, ptrs, work, xstart, chunk, counter);
    return hipGetLastError();
}

template <typename T, int BM, int BN>
int occupancy(bool ak, bool bk) {
    constexpr int NW = x3_nw<BM>();
    int n = 0;
    hipError_t e;
    if (ak && bk) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_batch<T, BM, BN, kXBK, 1, 1, true, NW>, 64 * NW, 0);
    else if (ak) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_batch<T, BM, BN, kXBK, 1, 0, true, NW>, 64 * NW, 0);
    else if (bk) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_batch<T, BM, BN, kXBK, 0, 1, true, NW>, 64 * NW, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_batch<T, BM, BN, kXBK, 0, 0, true, NW>, 64 * NW, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

hipError_t launch_x3_shape(bool f64, int shape, MfmaArgs& a, hipStream_t st) {
    if (a.npass != 1 || a.kslices > 1) return hipErrorInvalidValue;
    mfma_tiles_shape(shape, a);
    const bool ak = mfma_kmajor_a(a), bk = mfma_kmajor_b(a);
    if (f64)
        return shape == 0   ? one_shot<double, 128, 128>(a, ak, bk, st)
               : shape == 1 ? one_shot<double, 64, 64>(a, ak, bk, st)
                            : one_shot<double, 32, 128>(a, ak, bk, st);
    return shape == 0   ? one_shot<float, 128, 128>(a, ak, bk, st)
           : shape == 1 ? one_shot<float, 64, 64>(a, ak, bk, st)
                        : one_shot<float, 32, 128>(a, ak, bk, st);
}

hipError_t launch_x3_batch(bool f64, int shape, bool ak, bool bk, const MfmaArgs* items, const BatchPtrs* ptrs,
                           const int2* work, const int* xstart, int nwork, int* counter, int grid, hipStream_t st) {
    if (nwork <= 0) return hipSuccess;
    if (f64)
        return shape == 0   ? persistent<double, 128, 128>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st)
               : shape == 1 ? persistent<double, 64, 64>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st)
                            : persistent<double, 32, 128>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st);
    return shape == 0   ? persistent<float, 128, 128>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st)
           : shape == 1 ? persistent<float, 64, 64>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st)
                        : persistent<float, 32, 128>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st);
}

int x3_batch_occupancy(bool f64, int shape, bool ak, bool bk) {
    if (f64)
        return shape == 0 ? occupancy<double, 128, 128>(ak, bk)
                          : shape == 1 ? occupancy<double, 64, 64>(ak, bk) : occupancy<double, 32, 128>(ak, bk);
    return shape == 0 ? occupancy<float, 128, 128>(ak, bk)
                      : shape == 1 ? occupancy<float, 64, 64>(ak, bk) : occupancy<float, 32, 128>(ak, bk);
}

}  // namespace tc
