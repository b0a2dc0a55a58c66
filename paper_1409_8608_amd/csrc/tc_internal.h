// Internal declarations of libtc: host-side planning (spec, family, schedule,
// symbolic prediction) shared by the C ABI and the kernel launchers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tc.h"
#include "gett.h"

namespace tc {

// Error carrier: every internal routine returns a status and fills `msg`.
struct Err {
    tc_status st = TC_OK;
    std::string msg;
    tc_status set(tc_status s, std::string m) { st = s; msg = std::move(m); return s; }
};

// ---------------------------------------------------------------------------
// Contraction spec (Section 1): operand letters and the role of every index.
struct Spec {
    std::string a, b, c;            // letters of A, B and C in axis order
    std::string contracted;         // in A's axis order
    std::string free_a, free_b;     // in C's axis order
    // index classes outside the paper's definition (no family members; the
    // fused kernel only): batch indices in A, B and C (C's order) and trace
    // indices in one input only (that input's order)
    std::string batch, trace_a, trace_b;
    std::string base;               // C's letters, then the summed ones
    // bound per letter (index by letter - 'a'); stride 0 where the operand lacks it
    int64_t ext[26] = {0};
    int64_t sA[26] = {0}, sB[26] = {0}, sC[26] = {0};
    bool inA[26] = {false}, inB[26] = {false}, inC[26] = {false};
    tc_dtype dtype = TC_F64;
    tc_compute compute = TC_NATIVE;
    int64_t nA = 0, nB = 0, nC = 0;       // element counts (products of extents)
    int64_t spanA = 0, spanB = 0, spanC = 0; // 1 + largest element offset (0 if empty)

    int64_t e(char ch) const { return ext[ch - 'a']; }
    int64_t stride(int tensor, char ch) const {
        int k = ch - 'a';
        return tensor == 0 ? sA[k] : tensor == 1 ? sB[k] : sC[k];
    }
    const std::string& letters(int tensor) const { return tensor == 0 ? a : tensor == 1 ? b : c; }
    int64_t flops() const;                 // 2 * product of all extents
    // indices summed over: contracted, then trace indices of A and of B
    std::string summed() const { return contracted + trace_a + trace_b; }
    bool general() const { return !batch.empty() || !trace_a.empty() || !trace_b.empty(); }
    // bytes per element (a complex element holds its real and imaginary part)
    int elem_bytes() const { return dtype == TC_C128 ? 16 : dtype == TC_F64 || dtype == TC_C64 ? 8 : 4; }
    bool is_complex() const { return dtype == TC_C128 || dtype == TC_C64; }
};

tc_status parse_spec(const char* text, Spec& s, Err& err);
tc_status bind_spec(Spec& s, const char* index_chars, const int64_t* extents, int n_index,
                    const int64_t* stA, const int64_t* stB, const int64_t* stC, Err& err);

// ---------------------------------------------------------------------------
// Family member (Section 2).
struct Operand {
    int tensor;                       // 0 A, 1 B, 2 C
    std::string letters;
    std::vector<bool> fixed;          // per axis: sliced (fixed by a loop)
};

struct Variant {
    int number = 0;                   // paper numbering, from 1
    int kernel = 0;                   // TC_KERNEL_*
    std::string kept;                 // kernel indices
    std::string loops;                // sliced indices, outermost first
    std::vector<std::pair<int, int>> copies;   // (tensor, loop level; -1 = before all loops)
    std::string name;
    Operand ops[3];
    int n_hoisted = 0;                // leading contracted loops -> launch passes
};

std::vector<Variant> enumerate_family(const Spec& s);

// ---------------------------------------------------------------------------
// Symbolic prediction (Section 3).
struct SetupItem { int kind; int tensor; int64_t size; };   // kind 0 op, 1 remote
struct BenchClass {
    std::string label;
    double weight = 0;
    std::vector<SetupItem> setup;
    int start = -1;                    // -1 steady/fail; else first-iteration loop position
    std::vector<bool> prefetched;      // per operand: prefetch emulation used
};

int64_t region_size(const Spec& s, const Operand& op, const std::string& joined);
// root_gap: elements of other data accessed between the operand's previous use
// and this run, added when the walk reaches the root (0: the paper's assumption)
int64_t access_distance(const Spec& s, const Variant& v, int tensor, int start = -1, int64_t root_gap = 0);
int prefetch_kind(const Spec& s, const Variant& v, int tensor, int line_elems);  // 0 none, 1 line, 2 stream
std::vector<BenchClass> bench_classes(const Spec& s, const Variant& v, int stage,
                                      double cache_elems, int line_elems, const int64_t* root_gaps = nullptr);

// ---------------------------------------------------------------------------
// GPU schedules.
//
// A fused plan is a GEMM view: M = free indices of A, N = free indices of B,
// K = contracted indices.  Dimensions of a group that are laid out as one
// (stride[d+1] == stride[d] * ext[d] in every operand holding them) are merged.
struct GemmView {
    std::vector<GtDim> m, n, k;       // each group, unit-C-stride dim first where possible
    std::vector<GtDim> b;             // batch indices (sA, sB, sC)
    bool swapped = false;             // A and B exchanged so that C's unit stride is in M
    int64_t M = 1, N = 1, K = 1;
};
GemmView gemm_view(const Spec& s);
// Drop extent-1 dims and merge dims that continue each other in A, B and C.
void merge_group(std::vector<GtDim>& g);
// C's dimensions (sC), extent-1 ones dropped and contiguous ones merged.
std::vector<GtDim> c_dims(const Spec& s);
// Arguments of the C := beta * C kernel over all of C.
inline ScaleArgs scale_args(const Spec& s, void* C, double beta) {
    ScaleArgs sa{};
    sa.C = C;
    sa.beta = beta;
    sa.total = 1;
    for (const GtDim& d : c_dims(s)) {
        sa.dims.d[sa.dims.n++] = d;
        sa.total *= d.ext;
    }
    return sa;
}

// Launch sequence of one family member.
struct CopyStep {
    int tensor;                        // 0 A, 1 B
    int level;
    GtDims dims;                       // slice axes then slot axes; src = operand, dst = temp
    int64_t slice_elems = 0, slots = 1;
    int hoist_depth = 0;               // hoisted loops the copy's source offset depends on
};
struct VariantPlan {
    GtDesc body;                       // body launch (hoisted-loop offsets added per pass)
    std::vector<GtDim> hoisted;        // hoisted loops (outermost first): strides into A, B, C
    std::vector<CopyStep> copies;      // copies of A and B slices
    // copy of C's slices (Section 2: a copy "prior and/or after" the call):
    // per pass, C -> temp before the body and temp -> C after it; dims as
    // for the copy in (sA = C's stride, sC = the temp's)
    std::vector<CopyStep> c_copies;
    int64_t temp_elems[3] = {0, 0, 0}; // temp buffer sizes for A, B and C copies
    bool mfma = false;                 // gemm body on matrix cores
    int n_body_dims = 0;               // leading out dims that are the kernel's own free indices
    // a C copy with a contracted loop at or outside its level inside the free
    // loops: its in/out copies would interleave with the sequential passes of
    // the body launch, which this schedule does not do
    bool needs_c_copy = false;
    int64_t launches = 0;
};
VariantPlan plan_variant(const Spec& s, const Variant& v);

}  // namespace tc
