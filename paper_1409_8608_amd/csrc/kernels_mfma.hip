// Launchers of the matrix-core tile kernels (the tile itself is in
// mfma_tile.h): one-shot and split-K launches of the fused view and the
// gemm-shaped members, and the persistent form for batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "launch.h"
#include "mfma_tile.h"

namespace tc {

// SPLIT: the launch may split K (the split path costs registers, so launches
// that never split use the kernel without it).
// NW: waves per block (4, or 8 = two per SIMD).
template <typename T, int BM, int BN, int BK, int AMODE, int BMODE, bool SPLIT, int NW>
__global__ __launch_bounds__(64 * NW) void k_mfma(MfmaArgs a) {
    const int64_t S = SPLIT && a.kslices > 1 ? a.kslices : 1;
    const int64_t t = xcd_tile(blockIdx.x, a.ntiles * S);
    mfma_tile<T, BM, BN, BK, AMODE, BMODE, SPLIT, true, false, NW>(a, a.A, a.B, a.C, a.alpha, a.beta, t % a.ntiles,
                                                                   t / a.ntiles);
}

// Split-K reduction: output (m, n) is the sum of its slices' partials, in
// slice order, then C = alpha * sum + beta * C.
template <typename T, int BM, int BN>
__global__ __launch_bounds__(256) void k_splitk_reduce(MfmaArgs a) {
    const T alpha = (T)a.alpha, beta = (T)a.beta;
    const T* __restrict__ ws = (const T*)a.ws;
    T* C = (T*)a.C;
    const int64_t total = a.M * a.N, sstride = a.ntiles * (int64_t)(BM * BN);
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = idx % a.M, n = idx / a.M;
        const int64_t tile = (n / BN) * a.mt + m / BM;
        const T* p = ws + tile * (int64_t)(BM * BN) + (n % BN) * BM + m % BM;
        T sum = 0;
        for (int64_t s = 0; s < a.kslices; ++s) sum += p[s * sstride];
        T* cp = C + group_off<2>(a.m, m) + group_off<2>(a.n, n);
        T v = alpha * sum;
        if (a.beta != 0.0) v += beta * (*cp);
        *cp = v;
    }
}


// Tile shape of the one-shot launches (eight waves per block): 128 x 128 x 16,
// each wave 64 x 32; FP32 with at least 2048 summed positions 256 x 128 x 16,
// each wave 64 x 64, which halves the barriers and stagings per MFMA (FP32
// MFMAs take half as long as FP64's).  Measured on MI355X: 4096^2 x 4096 FP32
// 1.690 -> 1.395 ms with the wide tile; 256^3 x 1024 0.374 -> 0.446 ms, so short
// contractions keep 128 x 128.
constexpr int kBK = 16;
constexpr int kBMW = 256;   // rows of the wide FP32 tile
static bool wide_tile(bool f64, int64_t kpad) { return !f64 && kpad >= 2048; }
static int64_t tile_m(bool f64, int64_t kpad) { return wide_tile(f64, kpad) ? kBMW : 128; }
constexpr int64_t kTileN = 128;

int mfma_bk(bool) { return kBK; }

void mfma_tiles(bool f64, MfmaArgs& a) {
    const int64_t bm = tile_m(f64, a.Kpad);
    a.mt = (a.M + bm - 1) / bm;
    a.nt = (a.N + kTileN - 1) / kTileN;
    a.ntiles = a.mt * a.nt * a.nbatch;
}

// K-table walk for a fused M x N launch.  Tiles are dealt to the 8 XCDs in
// contiguous ranges with m tiles fastest, so the blocks resident on one XCD
// (at most about 64) span min(mt, R) m tiles and R / mt n tiles.  The operand
// with more distinct rows in that set walks its contiguous contracted index
// fastest (its cache lines are reused on consecutive K tiles); the other
// reuses its lines every 4 tiles (super-blocks of 4 blocks).
bool mfma_a_first(bool f64, int64_t M, int64_t N, int64_t K) {
    const int64_t bm = tile_m(f64, K), bn = kTileN;
    const int64_t mt = (M + bm - 1) / bm, nt = (N + bn - 1) / bn;
    const int64_t R = std::max<int64_t>(1, std::min<int64_t>((mt * nt + 7) / 8, 64));
    return std::min(mt, R) * bm > (R + mt - 1) / mt * bn;
}

// Lanes go along K for an operand whose free group is not unit-stride.
static bool k_major(const GtDims& g, int slot) {
    if (g.n == 0) return true;
    int64_t s = slot == 0 ? g.d[0].sA : g.d[0].sB;
    return s != 1;
}

// every offset of the group is a multiple of v elements
static bool group_aligned(const GtDims& g, int slot, int64_t v) {
    for (int d = 0; d < g.n; ++d) {
        int64_t s = slot == 0 ? g.d[d].sA : g.d[d].sB;
        if (g.d[d].ext > 1 && s % v != 0) return false;
    }
    return true;
}

// Load mode of operand `slot` (0 = A over the M group, 1 = B over N):
// 16-byte chunk loads when lanes run along K, the K table's chunks are
// contiguous and aligned (flag from the planner), every row, batch and pass
// offset is a multiple of the chunk and the base pointer is 16-byte aligned.
static int load_mode(const MfmaArgs& a, bool f64, int slot) {
    const GtDims& g = slot == 0 ? a.m : a.n;
    if (!k_major(g, slot)) return LD_MMAJ;
    const int64_t v = f64 ? 2 : 4;
    const void* base = slot == 0 ? a.A : a.B;
    bool vec = ((a.kvec >> slot) & 1) && group_aligned(g, slot, v) && group_aligned(a.batch, slot, v) &&
               group_aligned(a.pass, slot, v) && ((uintptr_t)base % 16 == 0);
    return vec ? LD_KVEC : LD_KSCAL;
}

// Chunk loads need a whole number of 16-byte chunks per thread; a tile side
// too small for that stages element by element.
template <typename T, int ROWS, int NT>
constexpr int fit_mode(int m) {
    return (m == LD_KVEC && (ROWS * kBK / NT) % (16 / (int)sizeof(T)) != 0) ? LD_KSCAL : m;
}

// Waves per block of the one-shot 128 x 128 launches: eight, two per SIMD, so
// that one wave's MFMAs run while the other waits at a step barrier or issues
// its loads (with four, one wave per SIMD, the matrix pipe idled whenever the
// wave did anything else).
constexpr int kNW = 8;

template <typename T, int BM, int BN, bool SPLIT = false, int NW = 4>
static hipError_t tile_dispatch(const MfmaArgs& a, int am, int bm, hipStream_t st) {
    const int64_t S = SPLIT && a.kslices > 1 ? a.kslices : 1;
    if (a.ntiles <= 0) return hipSuccess;
    if (a.ntiles * S > 0x7fffffff) return hipErrorInvalidConfiguration;
    dim3 g((unsigned)(a.ntiles * S)), b(64 * NW);
    constexpr int NT = 64 * NW;
    constexpr int A0 = fit_mode<T, BM, NT>(0), A1 = fit_mode<T, BM, NT>(1), A2 = fit_mode<T, BM, NT>(2);
    constexpr int B0 = fit_mode<T, BN, NT>(0), B1 = fit_mode<T, BN, NT>(1), B2 = fit_mode<T, BN, NT>(2);
    switch (am * 3 + bm) {
        case 0: hipLaunchKernelGGL((k_mfma<T, BM, BN, kBK, A0, B0, SPLIT, NW>), g, b, 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_mfma<T, BM, BN, kBK, A0, B1, SPLIT, NW>), g, b, 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_mfma<T, BM, BN, kBK, A0, B2, SPLIT, NW>), g, b, 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_mfma<T, BM, BN, kBK, A1, B0, SPLIT, NW>), g, b, 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_mfma<T, BM, BN, kBK, A1, B1, SPLIT, NW>), g, b, 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_mfma<T, BM, BN, kBK, A1, B2, SPLIT, NW>), g, b, 0, st, a); break;
        case 6: hipLaunchKernelGGL((k_mfma<T, BM, BN, kBK, A2, B0, SPLIT, NW>), g, b, 0, st, a); break;
        case 7: hipLaunchKernelGGL((k_mfma<T, BM, BN, kBK, A2, B1, SPLIT, NW>), g, b, 0, st, a); break;
        default: hipLaunchKernelGGL((k_mfma<T, BM, BN, kBK, A2, B2, SPLIT, NW>), g, b, 0, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_mfma(bool f64, MfmaArgs& a, hipStream_t st) {
    int am = load_mode(a, f64, 0), bm = load_mode(a, f64, 1);
    if (a.kslices <= 1)
        return f64 ? tile_dispatch<double, 128, 128, false, kNW>(a, am, bm, st)
               : wide_tile(f64, a.Kpad) ? tile_dispatch<float, kBMW, 128, false, kNW>(a, am, bm, st)
                                        : tile_dispatch<float, 128, 128, false, kNW>(a, am, bm, st);
    hipError_t e = f64 ? tile_dispatch<double, 128, 128, true, kNW>(a, am, bm, st)
                   : wide_tile(f64, a.Kpad) ? tile_dispatch<float, kBMW, 128, true, kNW>(a, am, bm, st)
                                            : tile_dispatch<float, 128, 128, true, kNW>(a, am, bm, st);
    if (e != hipSuccess || a.ntiles <= 0) return e;
    if (a.nbatch != 1 || a.npass != 1 || a.mode != 0 || !a.ws) return hipErrorInvalidValue;
    const int64_t total = a.M * a.N;
    dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536))), b(256);
    if (f64) hipLaunchKernelGGL((k_splitk_reduce<double, 128, 128>), g, b, 0, st, a);
    else if (wide_tile(f64, a.Kpad)) hipLaunchKernelGGL((k_splitk_reduce<float, kBMW, 128>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_splitk_reduce<float, 128, 128>), g, b, 0, st, a);
    return hipGetLastError();
}

// Split-K choice for a fused M x N x Kpad launch (one batch, one pass): none
// while the output tiles fill about two waves of resident blocks, or when K is
// short; else enough slices of at least 8 K tiles to fill them, with the
// workspace (slices x tiles x tile elements) at most ws_cap bytes.
// Returns the slice count and sets the tiles per slice and the workspace bytes.
int64_t mfma_split_plan(bool f64, int64_t M, int64_t N, int64_t Kpad, int64_t* slice_tiles, int64_t* ws_bytes,
                        int64_t ws_cap) {
    const int64_t bm = tile_m(f64, Kpad), bn = kTileN;
    const int64_t ntiles = ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
    const int64_t ktiles = Kpad / kBK;
    // resident blocks of the eight-wave tile kernels on 256 CUs: one per CU,
    // two for the FP32 128 x 128 form
    const int64_t fill = (f64 || bm == kBMW) ? 256 : 512;
    const int64_t esize = f64 ? 8 : 4;
    *slice_tiles = ktiles;
    *ws_bytes = 0;
    if (ntiles <= 0 || ntiles >= fill || ktiles < 16) return 1;
    int64_t S = std::min<int64_t>((2 * fill + ntiles - 1) / ntiles, ktiles / 8);
    S = std::min<int64_t>(S, ws_cap / (ntiles * bm * bn * esize));
    if (S < 2) return 1;
    const int64_t per = (ktiles + S - 1) / S;
    S = (ktiles + per - 1) / per;
    *slice_tiles = per;
    *ws_bytes = S * ntiles * bm * bn * esize;
    return S;
}

// ---------------------------------------------------------------------------
// Batches: tile shapes 0 = 128x128, 1 = 64x64, 2 = 32x128 (m x n; for
// contractions with few rows).  Batch members use the scalar load modes
// (their K tables are not checked for chunk contiguity).
static void shape_dims(int shape, int& bm, int& bn) {
    bm = shape == 0 ? 128 : shape == 1 ? 64 : 32;
    bn = shape == 0 ? 128 : shape == 1 ? 64 : 128;
}

void mfma_tiles_shape(int shape, MfmaArgs& a) {
    int bm, bn;
    shape_dims(shape, bm, bn);
    a.mt = (a.M + bm - 1) / bm;
    a.nt = (a.N + bn - 1) / bn;
    a.ntiles = a.mt * a.nt * a.nbatch;
}

bool mfma_kmajor_a(const MfmaArgs& a) { return k_major(a.m, 0); }
bool mfma_kmajor_b(const MfmaArgs& a) { return k_major(a.n, 1); }

// Waves per block of the persistent kernel's 128 x 128 tiles (the FP64 form
// needs all 256 VGPRs with four; see kNW).
constexpr int kBNW = 8;

template <int BM>
constexpr int batch_nw() { return BM == 128 ? kBNW : 4; }

template <typename T, int BM, int BN>
static hipError_t batch_dispatch(bool ak, bool bk, const MfmaArgs* items, const BatchPtrs* ptrs, const int2* work,
                                 const int* xstart, int nwork, int* counter, int grid, hipStream_t st) {
    constexpr int NW = batch_nw<BM>();
    dim3 g(grid), b(64 * NW);
    // runs of up to 16 items when the list is long (at least about 64 runs
    // per block); short lists of costly tiles keep single items for balance
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(16, (int64_t)nwork / ((int64_t)grid * 64)));
    if (ak && bk) hipLaunchKernelGGL((k_mfma_batch<T, BM, BN, kBK, 1, 1, false, NW>), g, b, 0, st, items, ptrs, work, xstart, chunk, counter);
    else if (ak) hipLaunchKernelGGL((k_mfma_batch<T, BM, BN, kBK, 1, 0, false, NW>), g, b, 0, st, items, ptrs, work, xstart, chunk, counter);
    else if (bk) hipLaunchKernelGGL((k_mfma_batch<T, BM, BN, kBK, 0, 1, false, NW>), g, b, 0, st, items, ptrs, work, xstart, chunk, counter);
    else hipLaunchKernelGGL((k_mfma_batch<T, BM, BN, kBK, 0, 0, false, NW>), g, b, 0, st, items, ptrs, work, xstart, chunk, counter);
    return hipGetLastError();
}

hipError_t launch_mfma_batch(bool f64, int shape, bool ak, bool bk, const MfmaArgs* items, const BatchPtrs* ptrs,
                             const int2* work, const int* xstart, int nwork, int* counter, int grid, hipStream_t st) {
    if (nwork <= 0) return hipSuccess;
    if (f64)
        return shape == 0   ? batch_dispatch<double, 128, 128>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st)
               : shape == 1 ? batch_dispatch<double, 64, 64>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st)
                            : batch_dispatch<double, 32, 128>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st);
    return shape == 0   ? batch_dispatch<float, 128, 128>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st)
           : shape == 1 ? batch_dispatch<float, 64, 64>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st)
                        : batch_dispatch<float, 32, 128>(ak, bk, items, ptrs, work, xstart, nwork, counter, grid, st);
}

// Resident blocks per CU of the persistent kernel (occupancy query).
template <typename T, int BM, int BN>
static int occ_of(bool ak, bool bk) {
    constexpr int NW = batch_nw<BM>();
    int n = 0;
    hipError_t e;
    if (ak && bk) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_batch<T, BM, BN, kBK, 1, 1, false, NW>, 64 * NW, 0);
    else if (ak) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_batch<T, BM, BN, kBK, 1, 0, false, NW>, 64 * NW, 0);
    else if (bk) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_batch<T, BM, BN, kBK, 0, 1, false, NW>, 64 * NW, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_batch<T, BM, BN, kBK, 0, 0, false, NW>, 64 * NW, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

int mfma_batch_occupancy(bool f64, int shape, bool ak, bool bk) {
    if (f64)
        return shape == 0 ? occ_of<double, 128, 128>(ak, bk)
                          : shape == 1 ? occ_of<double, 64, 64>(ak, bk) : occ_of<double, 32, 128>(ak, bk);
    return shape == 0 ? occ_of<float, 128, 128>(ak, bk)
                      : shape == 1 ? occ_of<float, 64, 64>(ak, bk) : occ_of<float, 32, 128>(ak, bk);
}

// One-shot launch with a chosen tile shape (used to time tuning candidates),
// with the persistent batch kernel's waves per block.
hipError_t launch_mfma_shape(bool f64, int shape, MfmaArgs& a, hipStream_t st) {
    mfma_tiles_shape(shape, a);
    int am = load_mode(a, f64, 0), bm = load_mode(a, f64, 1);
    if (shape == 0)
        return f64 ? tile_dispatch<double, 128, 128, false, kBNW>(a, am, bm, st)
                   : tile_dispatch<float, 128, 128, false, kBNW>(a, am, bm, st);
    if (shape == 1)
        return f64 ? tile_dispatch<double, 64, 64>(a, am, bm, st) : tile_dispatch<float, 64, 64>(a, am, bm, st);
    return f64 ? tile_dispatch<double, 32, 128>(a, am, bm, st) : tile_dispatch<float, 32, 128>(a, am, bm, st);
}

}  // namespace tc
