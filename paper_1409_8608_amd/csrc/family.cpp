// The algorithm family (Section 2) and its mapping to GPU launches.
//
// Table 1: the kernel keeps 1 contracted index (dot, gemv, gemm) or none (axpy,
// ger), and 0, 1 or 1+1 free indices; every other index is sliced into a loop,
// and all loop orders are generated.  Matrix operands of gemv, ger and gemm
// without a unit-stride kept axis are copied first, inside the innermost loop
// their slice depends on; the name carries an apostrophe after that loop.
#include <algorithm>
#include <numeric>

#include "tc_internal.h"

namespace tc {

static bool has(const std::string& s, char ch) { return s.find(ch) != std::string::npos; }

static const char* kKernelNames[5] = {"dot", "axpy", "gemv", "ger", "gemm"};

// Kept index sets of one kernel, in legend order (kept free indices in C's
// order, the kept contracted index in A's order innermost).
static std::vector<std::string> kept_sets(const Spec& s, int kernel) {
    std::vector<std::string> out;
    switch (kernel) {
        case TC_KERNEL_DOT:
            for (char k : s.contracted) out.push_back(std::string(1, k));
            break;
        case TC_KERNEL_AXPY:
            for (char f : s.c) out.push_back(std::string(1, f));
            break;
        case TC_KERNEL_GEMV:
            for (char f : s.c)
                for (char k : s.contracted) out.push_back(std::string{f, k});
            break;
        case TC_KERNEL_GER:
            for (char fa : s.free_a)
                for (char fb : s.free_b) out.push_back(std::string{fa, fb});
            break;
        case TC_KERNEL_GEMM:
            for (char fa : s.free_a)
                for (char fb : s.free_b)
                    for (char k : s.contracted) out.push_back(std::string{fa, fb, k});
            break;
    }
    return out;
}

std::vector<Variant> enumerate_family(const Spec& s) {
    std::vector<Variant> fam;
    if (s.general()) return fam;   // Table 1 covers contracted and free indices only
    if (s.is_complex()) return fam;  // complex plans run the fused kernel only
    // n letters give up to (n - 1)! loop orders per kernel; beyond 7 letters the
    // family is left to the fused kernel (a member's launch describes at most
    // GT_MAXD loops)
    if (s.base.size() > 7) return fam;
    int number = 0;
    for (int kernel = 0; kernel < 5; ++kernel) {
        for (const std::string& kept : kept_sets(s, kernel)) {
            // sliced indices in base order; next_permutation walks the loop
            // orders lexicographically over that order
            std::vector<int> rank;
            for (size_t p = 0; p < s.base.size(); ++p)
                if (!has(kept, s.base[p])) rank.push_back((int)p);
            do {
                Variant v;
                v.number = ++number;
                v.kernel = kernel;
                v.kept = kept;
                for (int r : rank) v.loops += s.base[r];
                for (int t = 0; t < 3; ++t) {
                    Operand& op = v.ops[t];
                    op.tensor = t;
                    op.letters = s.letters(t);
                    op.fixed.clear();
                    int n_kept = 0;
                    bool unit_kept = false;
                    for (char ch : op.letters) {
                        bool f = !has(kept, ch);
                        op.fixed.push_back(f);
                        if (!f) {
                            ++n_kept;
                            if (s.stride(t, ch) == 1) unit_kept = true;
                        }
                    }
                    if (n_kept == 2 && !unit_kept) {
                        int level = -1;
                        for (size_t ax = 0; ax < op.letters.size(); ++ax)
                            if (op.fixed[ax]) level = std::max(level, (int)v.loops.find(op.letters[ax]));
                        v.copies.push_back({t, level});
                    }
                }
                std::string name;
                for (auto& c : v.copies)
                    if (c.second == -1) name += '\'';
                for (size_t p = 0; p < v.loops.size(); ++p) {
                    name += v.loops[p];
                    for (auto& c : v.copies)
                        if (c.second == (int)p) name += '\'';
                }
                v.name = name + "-" + kKernelNames[kernel];
                while (v.n_hoisted < (int)v.loops.size() && has(s.contracted, v.loops[v.n_hoisted]))
                    ++v.n_hoisted;
                fam.push_back(std::move(v));
            } while (std::next_permutation(rank.begin(), rank.end()));
        }
    }
    return fam;
}

// ---------------------------------------------------------------------------
// GPU schedule of a member.
//
// * The leading contracted loops (those outside every free loop) become
//   separate launch passes: each pass covers the whole rest of the nest.
// * The remaining free loops become parallel output dimensions of one launch,
//   ordered innermost loop first, after the kernel's own free indices, so the
//   loop order decides which invocations are neighbours on the device.
// * The remaining contracted loops run sequentially inside the launch; each of
//   their iterations is one kernel invocation that reads and writes C.
// * A copy runs as its own launch before the body: it writes one slot per
//   execution of the copy statement within a pass (the loops at or outside
//   its level, hoisted loops excluded), and the body reads its slot.
VariantPlan plan_variant(const Spec& s, const Variant& v) {
    VariantPlan vp;
    GtDesc& d = vp.body;
    d = GtDesc{};
    auto dim = [&](char ch) {
        int k = ch - 'a';
        return GtDim{s.ext[k], s.sA[k], s.sB[k], s.sC[k]};
    };
    int L = (int)v.loops.size();
    int H = v.n_hoisted;
    for (int p = 0; p < H; ++p) vp.hoisted.push_back(dim(v.loops[p]));

    // temp layout of each copied operand: kept axes compact in operand order,
    // then one slot axis per non-hoisted loop at or outside the copy level
    int64_t tstride[3][26];
    bool copied[3] = {false, false, false};
    for (auto& c : v.copies) {
        if (c.first == 2) {
            for (int p = H; p <= c.second; ++p)
                if (has(s.contracted, v.loops[p])) vp.needs_c_copy = true;
            if (vp.needs_c_copy) continue;
        }
        int t = c.first;
        copied[t] = true;
        for (int k = 0; k < 26; ++k) tstride[t][k] = 0;
        CopyStep cs;
        cs.tensor = t;
        cs.level = c.second;
        cs.dims.n = 0;
        int64_t run = 1;
        const Operand& op = v.ops[t];
        for (size_t ax = 0; ax < op.letters.size(); ++ax) {
            if (op.fixed[ax]) continue;
            char ch = op.letters[ax];
            tstride[t][ch - 'a'] = run;
            cs.dims.d[cs.dims.n++] = GtDim{s.e(ch), s.stride(t, ch), 0, run};
            run *= s.e(ch);
        }
        cs.slice_elems = run;
        for (int p = H; p <= c.second; ++p) {
            char ch = v.loops[p];
            tstride[t][ch - 'a'] = run;
            // the slot axis walks the source only along indices the slice has
            int64_t src = has(op.letters, ch) ? s.stride(t, ch) : 0;
            cs.dims.d[cs.dims.n++] = GtDim{s.e(ch), src, 0, run};
            run *= s.e(ch);
        }
        cs.slots = run / std::max<int64_t>(1, cs.slice_elems);
        if (cs.slice_elems == 0) cs.slots = 0;
        cs.hoist_depth = std::min(H, c.second + 1);
        vp.temp_elems[t] = run;
        (t == 2 ? vp.c_copies : vp.copies).push_back(cs);
    }
    auto sa = [&](char ch) { return copied[0] ? tstride[0][ch - 'a'] : s.sA[ch - 'a']; };
    auto sb = [&](char ch) { return copied[1] ? tstride[1][ch - 'a'] : s.sB[ch - 'a']; };
    auto sc = [&](char ch) { return copied[2] ? tstride[2][ch - 'a'] : s.sC[ch - 'a']; };
    auto gd = [&](char ch) { return GtDim{s.e(ch), sa(ch), sb(ch), sc(ch)}; };

    vp.mfma = (v.kernel == TC_KERNEL_GEMM);
    d.out.n = 0;
    d.nm = d.nn = 0;
    if (vp.mfma) {
        // M = kept free index of A, N = kept free index of B
        for (char ch : v.kept)
            if (has(s.free_a, ch)) { d.out.d[d.out.n++] = gd(ch); d.nm = 1; }
        for (char ch : v.kept)
            if (has(s.free_b, ch)) { d.out.d[d.out.n++] = gd(ch); d.nn = 1; }
    } else {
        for (char ch : s.c)
            if (has(v.kept, ch)) d.out.d[d.out.n++] = gd(ch);
        vp.n_body_dims = d.out.n;
    }
    for (int p = L - 1; p >= H; --p)
        if (!has(s.contracted, v.loops[p])) d.out.d[d.out.n++] = gd(v.loops[p]);
    d.kb = GtDim{1, 0, 0, 0};
    for (char ch : v.kept)
        if (has(s.contracted, ch)) d.kb = gd(ch);
    d.pass.n = 0;
    for (int p = H; p < L; ++p)
        if (has(s.contracted, v.loops[p])) d.pass.d[d.pass.n++] = gd(v.loops[p]);
    d.offA = d.offB = d.offC = 0;

    int64_t passes = 1;
    for (auto& h : vp.hoisted) passes *= h.ext;
    int64_t copy_launches = 0;
    for (auto& cs : vp.copies) {
        int64_t n = 1;
        for (int p = 0; p < cs.hoist_depth; ++p) n *= vp.hoisted[p].ext;
        copy_launches += n;
    }
    copy_launches += 2 * passes * (int64_t)vp.c_copies.size();   // C in and out around every body launch
    vp.launches = 1 + passes + copy_launches;   // C prologue, bodies, copies
    return vp;
}

}  // namespace tc
