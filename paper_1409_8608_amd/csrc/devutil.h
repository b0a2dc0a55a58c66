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

}  // namespace tc
