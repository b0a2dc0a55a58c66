// tc_contract_noalloc: the fused contraction for callers that cannot allocate
// device memory (code under graph capture, tight serving loops).  Every device
// buffer the call needs beyond A, B and C -- the matrix-core kernel's K table
// and its split-K partial tiles -- lives in one file-scope device array,
// `scratch`, which each GPU holds from the library's load to the end of the
// process.  Calls on one GPU share it and keep the last call's contents: calls
// that overlap on one GPU (streams with no ordering between them) race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "launch.h"
#include "plan.h"

using namespace tc;

static __device__ __align__(256) unsigned char scratch[TC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

// Device address of the array on the current device, looked up once per
// device with that device current.  The array's name in host code is only a
// host-side handle, so kernels and copies take this address instead.
tc_status scratch_on_current(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(TC_E_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return TC_OK;
}

constexpr int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

}  // namespace

extern "C" tc_status tc_contract_noalloc(tc_plan_t p, const void* A, const void* B, void* C, double alpha,
                                         double beta, void* stream) {
    bool runs = false;
    tc_status st = validate_call(p, A, B, C, alpha, 0.0, 0.0, &runs);
    if (st || !runs) return st;
    const Spec& s = p->spec;
    if (s.is_complex()) return fail(TC_E_UNSUPPORTED, "tc_contract_noalloc takes real plans");
    if (s.compute != TC_NATIVE) return fail(TC_E_UNSUPPORTED, "tc_contract_noalloc runs the native compute mode");
    if (p->selected != TC_VARIANT_FUSED)
        return fail(TC_E_UNSUPPORTED, "tc_contract_noalloc runs the fused kernel: select TC_VARIANT_FUSED");
    hipStream_t hs = (hipStream_t)stream;
    const bool f64 = s.dtype == TC_F64;
    int64_t K = 1;
    for (char ch : s.summed()) K *= s.e(ch);
    if (alpha == 0.0 || K == 0) {
        if (beta == 1.0) return TC_OK;
        ScaleArgs sa = scale_args(s, C, beta);
        hipError_t e = launch_scale(f64, sa, hs);
        return e == hipSuccess ? TC_OK : hip_fail(e, "scale kernel launch");
    }
    const GemmView& gv = p->gv;
    if (gv.swapped) std::swap(A, B);
    if (use_stream_kernel(s, gv)) return launch_fused_stream(p, A, B, C, alpha, beta, hs);

    // Matrix-core tiles: the K table (16 bytes per padded position) first,
    // then the split-K partial tiles, each 256-byte aligned.  The table's
    // padding only adds positions, so K alone already rules out tables that
    // cannot fit.
    if (K > TC_NOALLOC_SCRATCH_BYTES / 16)
        return fail(TC_E_UNSUPPORTED, "contracted extent " + std::to_string(K) +
                                          " needs a K table beyond the no-allocation scratch of " +
                                          std::to_string((long long)TC_NOALLOC_SCRATCH_BYTES) + " bytes");
    const int BK = mfma_bk(f64);
    if (p->h_ktab.empty()) {
        p->h_ktab = build_ktab(gv.k, BK, 4, mfma_a_first(f64, gv.M, gv.N, gv.K), 4);
        p->h_kvec = ktab_vec_flags(p->h_ktab, f64 ? 2 : 4);
    }
    const int64_t tab_bytes = (int64_t)(p->h_ktab.size() * sizeof(int64_t));
    const int64_t ws_off = align256(tab_bytes);
    if (ws_off > TC_NOALLOC_SCRATCH_BYTES)
        return fail(TC_E_UNSUPPORTED, "K table of " + std::to_string(tab_bytes) +
                                          " bytes exceeds the no-allocation scratch of " +
                                          std::to_string((long long)TC_NOALLOC_SCRATCH_BYTES) + " bytes");
    const int64_t kpad = (int64_t)p->h_ktab.size() / 2;
    int64_t slice_tiles = 0, ws_bytes = 0, kslices = 1;
    if (gv.b.empty())
        kslices = mfma_split_plan(f64, gv.M, gv.N, kpad, &slice_tiles, &ws_bytes,
                                  std::min<int64_t>(64LL << 20, TC_NOALLOC_SCRATCH_BYTES - ws_off));
    void* base = nullptr;
    st = scratch_on_current(&base);
    if (st) return st;
    hipError_t e = hipMemcpyAsync(base, p->h_ktab.data(), (size_t)tab_bytes, hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "K table copy to scratch");
    return launch_fused_mfma(p, A, B, C, alpha, beta, (const int64_t*)base, kpad, p->h_kvec,
                             (char*)base + ws_off, kslices, slice_tiles, hs);
}
