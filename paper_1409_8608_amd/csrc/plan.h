// The plan object behind tc_plan_t and the internal entry points that use it.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "tc_internal.h"

struct tc_plan_s {
    tc::Spec spec;
    tc::GemmView gv;
    // The algorithm family and each member's GPU schedule are built on first
    // use: a plan that only runs the fused kernel (a batch member, say) never
    // pays for enumerating up to a few hundred members.
    std::vector<tc::Variant>& fam() {
        build_family();
        return fam_;
    }
    std::vector<tc::VariantPlan>& vplans() {
        build_family();
        return vplans_;
    }
    void build_family() {
        if (family_built_) return;
        fam_ = tc::enumerate_family(spec);
        vplans_.reserve(fam_.size());
        for (auto& v : fam_) vplans_.push_back(tc::plan_variant(spec, v));
        family_built_ = true;
    }
    // caller's cache precondition: elements of other data accessed between an
    // operand's previous use and this run (A, B, C), added at the walk's root
    int64_t root_gap[3] = {0, 0, 0};
    int selected = TC_VARIANT_FUSED;
    int predicted_best = TC_VARIANT_FUSED;
    bool have_prediction = false;

    // device workspace (allocated by prepare, freed by destroy)
    void* d_ktab = nullptr;          // fused matrix-core K table
    bool ktab_ready = false;         // d_ktab (and the split-K workspace) set up
    int64_t ktab_cap = 0, kpad = 0;
    int kvec = 0;                    // chunk flags of d_ktab (MfmaArgs::kvec)
    void* d_splitk = nullptr;        // split-K partial tiles of the fused kernel
    int64_t splitk_cap = 0, kslices = 1, kslice_tiles = 0;
    void* d_var_ktab = nullptr;      // K table of the selected gemm member
    int64_t var_ktab_cap = 0, var_kpad = 0;
    int var_kvec = 0;
    int var_ktab_for = -1;
    void* d_temp[3] = {nullptr, nullptr, nullptr};   // copy temporaries of A, B and C
    int64_t temp_cap[3] = {0, 0, 0};
    // complex storage: the contraction runs as the real plan `real` over an
    // embedded form in which operand `zside` is expanded into 2x2 real blocks
    tc_plan_s* real = nullptr;
    int zside = -1;
    GtDims zdims{};                  // expanded operand: sA source stride (complex elements),
                                     // sC destination stride (reals)
    int64_t zelems = 0;              // its complex elements
    int64_t zs_in = 0, zs_out = 0;   // destination strides of the two re/im indices
    void* d_zexp = nullptr;          // the expanded operand
    int64_t zexp_cap = 0;
    int zvec = 0;                    // complex streaming kernel's widest lane form (0: not used); gv complex
    // host copy of the fused K table, for the no-allocation entry point
    std::vector<int64_t> h_ktab;
    int h_kvec = 0;
    // split-precision buffers (one allocation)
    int split_products = 6;          // BF16 term products kept: 6 (p+q <= 4), or 3 / 9 (ablations)
    void* d_split = nullptr;
    int64_t split_bytes = 0;
    int64_t split_layout[24] = {0};

private:
    std::vector<tc::Variant> fam_;
    std::vector<tc::VariantPlan> vplans_;
    bool family_built_ = false;
};

namespace tc {
extern thread_local std::string g_last_error;
tc_status fail(tc_status s, const std::string& msg);
tc_status ensure_device_buffer(void** p, int64_t* cap, int64_t bytes);
// tc_contract never allocates: while it checks a plan's workspace, every step
// of prepare_plan that would allocate or upload fails instead (fail_unprepared)
bool allocation_forbidden();
tc_status fail_unprepared();
struct NoAllocScope {
    bool saved;
    NoAllocScope();
    ~NoAllocScope();
};
// Is a HIP device visible to this process?  (Looked up once.)  Plans built
// with one allocate their workspace at once; without one they stay host-only.
bool device_visible();
tc_status hip_fail(hipError_t e, const char* what);

std::vector<int64_t> build_ktab(const std::vector<GtDim>& kd, int BK, int bA = 4, bool a_first = false, int G = 0);
int ktab_vec_flags(const std::vector<int64_t>& tab, int v);
bool use_stream_kernel(const Spec& s, const GemmView& gv);
// Shape part of the streaming kernel's arguments (M, N, K tables, threads per
// row) for a plan that use_stream_kernel accepts; pointers and scalars unset.
StreamArgs stream_args(const GemmView& gv, bool f64);
tc_status prepare_plan(tc_plan_s* p);
tc_status contract_dispatch(tc_plan_s* p, const void* A, const void* B, void* C, double alpha, double beta,
                            hipStream_t st);
tc_status validate_call(const tc_plan_s* p, const void* A, const void* B, const void* C, double alpha_re,
                        double alpha_im, double beta_im, bool* runs);
// Fused launches with A and B in GEMM-view order (swapped already).
tc_status launch_fused_stream(const tc_plan_s* p, const void* A, const void* B, void* C, double alpha, double beta,
                              hipStream_t st);
tc_status launch_fused_mfma(const tc_plan_s* p, const void* A, const void* B, void* C, double alpha, double beta,
                            const int64_t* ktab, int64_t kpad, int kvec, void* ws, int64_t kslices,
                            int64_t kslice_tiles, hipStream_t st);
tc_status run_variant(tc_plan_s* p, int v, const void* A, const void* B, void* C, double alpha, double beta,
                      hipStream_t st);

// split precision (kernels_split.hip)
tc_status prepare_split(tc_plan_s* p);
tc_status run_split(tc_plan_s* p, const void* A, const void* B, void* C, double alpha, double beta,
                    hipStream_t st);
// The same launches for a batch member whose operands (GEMM-view order),
// alpha and beta are read from its staged entry `bp` when the kernels run.
tc_status run_split_batched(tc_plan_s* p, const BatchPtrs* bp, hipStream_t st);
// contracted positions of a split plan's term tables (0 before its workspace exists)
int64_t split_positions(const tc_plan_s* p);
void release_plan_device(tc_plan_s* p);

// complex storage (complex.hip)
tc_status build_complex(tc_plan_s* p);
tc_status prepare_complex(tc_plan_s* p);
tc_status run_complex(tc_plan_s* p, const void* A, const void* B, void* C, double alpha_re, double alpha_im,
                      double beta_re, double beta_im, hipStream_t st);
}  // namespace tc
