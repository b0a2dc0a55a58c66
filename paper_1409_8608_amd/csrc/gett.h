// Plain-old-data launch descriptors shared by the host planner and the HIP
// kernels.  Offsets and strides are in elements.
#pragma once

#include <cstdint>

#define GT_MAXD 8
#define GT_SMALLK_MAX 32

// One loop or tensor dimension: its extent and its stride in A, B and C
// (0 where the tensor does not depend on it).  Copy and scale kernels use sA as
// the source stride and sC as the destination stride.
struct GtDim {
    int64_t ext;
    int64_t sA, sB, sC;
};

struct GtDims {
    int n;
    GtDim d[GT_MAXD];
};

// Body launch of one family member.
//   out:  output dimensions, first fastest.  For the SIMT kernels these are the
//         kernel's kept free indices (C's axis order) followed by the parallel
//         loops, innermost loop first.  For the matrix-core kernel the first
//         `nm` entries form M, the next `nn` form N and the rest are the batch.
//   kb:   the kernel's kept contracted index (ext 1 and strides 0 if none).
//   pass: contracted loops that run sequentially inside the launch, outermost
//         first; each iteration is one kernel invocation that reads and writes C.
struct GtDesc {
    GtDims out;
    GtDim kb;
    GtDims pass;
    int nm, nn;
    int64_t offA, offB, offC;
};

struct SimtArgs {
    const void* A;
    const void* B;
    void* C;
    GtDims out;
    GtDim kb;
    GtDims pass;
    int64_t total;      // product of out extents
    int64_t npass;      // product of pass extents
    double alpha;
};

struct StreamArgs {     // fused kernel for small contracted extents
    const void* A;
    const void* B;
    void* C;
    int64_t M, N;       // M: one dimension, unit stride in C
    int64_t sAm;        // A stride along M
    GtDims n;           // N dimensions (sB, sC), first fastest
    int K;
    int64_t kA[GT_SMALLK_MAX], kB[GT_SMALLK_MAX];
    double alpha, beta;
    int tpr;            // threads per N row (power of two)
    int64_t rows_per_block;
};

struct MfmaArgs {
    const void* A;
    const void* B;
    void* C;
    GtDims m;           // M dims: sA, sC
    GtDims n;           // N dims: sB, sC
    GtDims batch;       // batch dims: sA, sB, sC
    GtDims pass;        // pass dims (sequential, C re-read each pass): sA, sB
    const int64_t* ktab;  // Kpad pairs (offA, offB); (-1, -1) marks zero padding
    int64_t M, N, Kpad, nbatch, npass;
    int64_t mt, nt, ntiles;   // tile counts
    double alpha, beta;
    int mode;           // 0: C = alpha*acc + beta*C; 1: per pass C += alpha*acc
    int kvec;           // bit 0 (A), bit 1 (B): every 16-byte chunk of K-table
                        // positions is contiguous and aligned in that operand
    // split K (fused launches with few output tiles): kslices > 1 slices of
    // kslice_tiles K tiles each; every (slice, tile) block writes its raw
    // accumulators to ws, [slice][tile][n][m], and a reduction kernel forms C
    void* ws;
    int64_t kslices, kslice_tiles;
};

// Per-call operands of one batch member.
struct BatchPtrs {
    const void* A;
    const void* B;
    void* C;
    double alpha, beta;
};

struct CopyArgs {
    const void* src;
    void* dst;
    GtDims dims;        // sA = source stride, sC = destination stride
    int64_t total;
};

struct ScaleArgs {
    void* C;
    GtDims dims;        // sC
    int64_t total;
    double beta;
};

// Complex operand -> real 2x2 blocks (times alpha).  For each complex element y
// of the source, with t = alpha * y, the destination holds t_re at its offset,
// -t_im one re/im step of the other operand further (s_in), t_im one re/im step
// of C further (s_out) and t_re at both steps.
struct ZExpandArgs {
    const void* src;
    void* dst;
    GtDims dims;        // sA = source stride (complex elements), sC = destination stride (reals)
    int64_t total;
    int64_t s_in, s_out;
    double alpha_re, alpha_im;
};

// C := beta * C for complex C (beta == 0 writes zeros without reading C).
struct ZScaleArgs {
    void* C;
    GtDims dims;        // sC, complex elements
    int64_t total;
    double beta_re, beta_im;
};
