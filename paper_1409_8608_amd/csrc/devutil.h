// Small device helpers shared by the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tc {

// Global-memory view of a pointer.  Where a kernel reads its pointers from
// memory (a batch's device table, an argument struct indexed at run time) the
// compiler cannot tell the address space and issues flat loads and stores;
// those also count against the LDS wait counter, so every LDS barrier would
// wait for all memory operations in flight.  Every operand, table and
// workspace the kernels touch is device memory.
template <typename T> using gmem = T __attribute__((address_space(1)));

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

// Round-to-nearest-even to 8 significant bits with an unbounded exponent
// (the value 2^E rint(m 2^8) for x = m 2^E, 1/2 <= |m| < 1), on the FP64 bit
// pattern: the 45 low fraction bits are dropped after adding half an ulp of
// the kept part (less one when its last bit is 0, so that ties go to even); a
// carry moves into the exponent, as it should.  A subnormal x is scaled by 2^64
// first (exact) and the result scaled back (exact: its lowest bit is not below
// x's).  Zero keeps its sign.
__device__ __forceinline__ double rn8(double x) {
    const bool sub = __builtin_fabs(x) < 0x1p-1022;
    uint64_t u = (uint64_t)__double_as_longlong(sub ? x * 0x1p64 : x);
    u += 0xFFFFFFFFFFFull + ((u >> 45) & 1);
    u &= ~0x1FFFFFFFFFFFull;
    const double r = __longlong_as_double((long long)u);
    return sub ? r * 0x1p-64 : r;
}

}  // namespace tc
