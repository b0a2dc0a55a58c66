// Symbolic half of the performance model (Section 3): access distances
// (Section 3.2), setup lists with the 5/4-cache cut, prefetching (Section 3.3),
// prefetch failures (Section 3.4) and first-iteration classes (Section 3.5).
#include <algorithm>
#include <cmath>

#include "tc_internal.h"

namespace tc {

static bool has(const std::string& s, char ch) { return s.find(ch) != std::string::npos; }

// Elements of operand `op` once joined (made ':') along every loop in `joined`.
int64_t region_size(const Spec& s, const Operand& op, const std::string& joined) {
    int64_t n = 1;
    for (size_t ax = 0; ax < op.letters.size(); ++ax)
        if (!op.fixed[ax] || has(joined, op.letters[ax])) n *= s.e(op.letters[ax]);
    return n;
}

static bool depends(const Operand& op, char loop, const std::string& joined) {
    for (size_t ax = 0; ax < op.letters.size(); ++ax)
        if (op.fixed[ax] && op.letters[ax] == loop && !has(joined, loop)) return true;
    return false;
}

// The walk over the member's program (Section 3.2: the back-traversal covers
// any combination of loops and kernels).  The program of a member: its loops
// in order; at the head of the body of loop position l (-1: before all loops)
// the copies the member takes at level l (X~ := X[slice]), then the next loop
// (the kernel in the innermost body), then the copies of C back (X[slice] :=
// X~).  The kernel works on the buffer X~ of a copied operand, which no loop
// changes.  Regions are numbered 0..2 (A, B, C) and 3..5 (their buffers).
namespace {

struct Reg {
    int id;                            // 0..2 operand, 3..5 the buffer of operand id - 3
    const Operand* op;                 // the operand (its letters; a buffer keeps the kept axes)
    std::string joined;                // loops it is joined along
};

bool copied(const Variant& v, int t) {
    for (auto& c : v.copies)
        if (c.first == t) return true;
    return false;
}

int64_t reg_size(const Spec& s, const Reg& r) {
    if (r.id < 3) return region_size(s, *r.op, r.joined);
    int64_t n = 1;                     // a buffer: the slice's kept axes
    for (size_t ax = 0; ax < r.op->letters.size(); ++ax)
        if (!r.op->fixed[ax]) n *= s.e(r.op->letters[ax]);
    return n;
}

bool reg_varies(const Reg& r, char loop) {
    if (r.id >= 3) return false;       // one buffer for every iteration
    for (size_t ax = 0; ax < r.op->letters.size(); ++ax)
        if (r.op->fixed[ax] && r.op->letters[ax] == loop && !has(r.joined, loop)) return true;
    return false;
}

// The set M: per region id, the loops it is joined along (a region merged
// with another of its tensor is joined along the loops either is joined along:
// their union for the nested regions a walk meets).
struct RegionSet {
    bool in[6] = {false, false, false, false, false, false};
    std::string joined[6];
    void add(int id, const std::string& j) {
        if (!in[id]) {
            in[id] = true;
            joined[id] = j;
        } else {
            for (char ch : j)
                if (!has(joined[id], ch)) joined[id] += ch;
        }
    }
    int64_t size(const Spec& s, const Variant& v) const {
        int64_t n = 0;
        for (int id = 0; id < 6; ++id)
            if (in[id]) n += reg_size(s, Reg{id, &v.ops[id % 3], joined[id]});
        return n;
    }
};

// Regions of the copies at level l: copy-ins at the head of the body, copy-outs
// (of C) at its end.
void copy_regions(const Variant& v, int l, bool outs, std::vector<int>& ids) {
    for (auto& c : v.copies)
        if (c.second == l && (!outs || c.first == 2)) {
            ids.push_back(c.first);
            ids.push_back(c.first + 3);
        }
}

// Every region the body at level l and everything inside it access, joined
// along `joined` (which holds the loops from l + 1 inward, and l itself when
// the whole loop is meant).
void add_body(const Variant& v, int l, const std::string& joined, RegionSet& M) {
    const int L = (int)v.loops.size();
    for (int q = l; q < L; ++q) {
        std::vector<int> ids;
        copy_regions(v, q, false, ids);
        for (int id : ids) M.add(id, joined);
    }
    for (int t = 0; t < 3; ++t) M.add(copied(v, t) ? t + 3 : t, joined);
}

}  // namespace

// Access distance of kernel operand `tensor` (a copied operand: its buffer).
// The walk starts at the kernel, or, for a first-iteration class, at loop
// position `start` with M holding that loop's whole body joined along it and
// the loops inside it (Section 3.5).  Case 1: the operand does not change
// across the loop -> the statements after the current position in that body
// (previous iteration) are walked back from its end, and the walk stops.
// Case 2: it does -> the whole loop, joined along it, goes into M, and the
// walk goes up.  An earlier statement of a body that touches the operand's
// tensor stops the walk.  Case 3: the root -> the caller's root gap is added:
// the paper assumes the contraction runs again and again with nothing in
// between, a caller who knows the surrounding program states what is accessed
// in between.
int64_t access_distance(const Spec& s, const Variant& v, int tensor, int start, int64_t root_gap) {
    const int L = (int)v.loops.size();
    RegionSet M;
    Reg op{copied(v, tensor) ? tensor + 3 : tensor, &v.ops[tensor], ""};
    int level = L - 1;                 // body holding the current node
    if (start >= 0) {
        std::string inner = v.loops.substr(start);
        add_body(v, start, inner, M);
        op.joined = inner;
        level = start - 1;
    }
    auto touches = [&](int id) { return id == op.id; };   // a statement on the operand's tensor
    for (;;) {
        // earlier statements of this body: its copy-ins (the current node
        // follows them)
        {
            std::vector<int> ids;
            copy_regions(v, level, false, ids);
            for (int q = (int)ids.size() / 2 - 1; q >= 0; --q) {
                if (touches(ids[2 * q]) || touches(ids[2 * q + 1])) return M.size(s, v);
                M.add(ids[2 * q], "");
                M.add(ids[2 * q + 1], "");
            }
        }
        if (level < 0) return M.size(s, v) + root_gap;   // case 3
        const char loop = v.loops[level];
        if (!reg_varies(op, loop)) {       // case 1: the tail of the previous iteration
            std::vector<int> ids;
            copy_regions(v, level, true, ids);
            for (int q = (int)ids.size() / 2 - 1; q >= 0; --q) {
                if (touches(ids[2 * q]) || touches(ids[2 * q + 1])) break;
                M.add(ids[2 * q], "");
                M.add(ids[2 * q + 1], "");
            }
            return M.size(s, v);
        }
        add_body(v, level, v.loops.substr(level), M);    // case 2
        op.joined += loop;
        --level;
    }
}

// 1: the innermost loop indexes the operand's first axis (cache-line sharing);
// 2: it indexes the second axis while the first is whole or within one line.
int prefetch_kind(const Spec& s, const Variant& v, int tensor, int line_elems) {
    if (v.loops.empty()) return 0;
    char inner = v.loops.back();
    const Operand& op = v.ops[tensor];
    if (!depends(op, inner, "")) return 0;
    if (!op.letters.empty() && op.letters[0] == inner) return 1;
    if (op.letters.size() >= 2 && op.letters[1] == inner) {
        bool whole = !op.fixed[0];
        bool small = op.fixed[0] || s.e(op.letters[0]) <= line_elems;
        if (whole || small) return 2;
    }
    return 0;
}

static int64_t one_line_size(const Spec& s, const Operand& op, int line_elems) {
    int64_t n = 1;
    for (size_t ax = 0; ax < op.letters.size(); ++ax) {
        int64_t e = op.fixed[ax] ? 1 : s.e(op.letters[ax]);
        if (ax == 0) e = std::min<int64_t>(e, line_elems);
        n *= e;
    }
    return n;
}

struct Item { int tensor; int64_t size, dist; };

// Operands by decreasing distance, each followed by the remote region that
// makes the sizes to its right add up to its distance; cut from the front to
// 5/4 of the cache.  An operands-only list is empty (the repetitions already
// touch every operand).
static std::vector<SetupItem> setup_list(std::vector<Item> items, double cache_elems) {
    std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.dist > y.dist; });
    std::vector<SetupItem> seq;
    for (size_t k = 0; k < items.size(); ++k) {
        seq.push_back({0, items[k].tensor, items[k].size});
        int64_t r = (k + 1 < items.size()) ? items[k].dist - items[k + 1].dist - items[k + 1].size
                                           : items[k].dist;
        if (r > 0) seq.push_back({1, -1, r});
    }
    double limit = 1.25 * cache_elems;
    double total = 0;
    for (auto& e : seq) total += (double)e.size;
    if (total > limit) {
        std::vector<SetupItem> kept;
        double acc = 0;
        for (auto it = seq.rbegin(); it != seq.rend(); ++it) {
            if (acc + (double)it->size <= limit) {
                kept.push_back(*it);
                acc += (double)it->size;
            } else {
                int64_t rest = (int64_t)std::floor(limit - acc);
                if (rest > 0) kept.push_back({1, -1, rest});
                break;
            }
        }
        std::reverse(kept.begin(), kept.end());
        seq = kept;
    }
    bool only_ops = std::all_of(seq.begin(), seq.end(), [](const SetupItem& e) { return e.kind == 0; });
    if (only_ops) seq.clear();
    return seq;
}

std::vector<BenchClass> bench_classes(const Spec& s, const Variant& v, int stage,
                                      double cache_elems, int line_elems, const int64_t* root_gaps) {
    const int64_t gap0[3] = {0, 0, 0};
    const int64_t* gap = root_gaps ? root_gaps : gap0;
    std::vector<BenchClass> out;
    if (stage <= 1) {
        BenchClass c;
        c.label = "steady";
        c.weight = 1.0;
        c.prefetched.assign(3, false);
        out.push_back(c);
        return out;
    }
    int64_t size[3], dist[3];
    int kind[3];
    for (int t = 0; t < 3; ++t) {
        size[t] = region_size(s, v.ops[t], "");
        dist[t] = access_distance(s, v, t, -1, gap[t]);
        // the kernel reads a copied operand from its buffer, which no loop changes
        kind[t] = stage >= 3 && !copied(v, t) ? prefetch_kind(s, v, t, line_elems) : 0;
    }
    // Operands in the order of the access-distance list (ties: A, B, C); the
    // prefetch distances of Section 3.3 are folded into that list, so equal
    // distances keep it (its example lists C[a,:,c], A[a,:], B[:,:,c]).
    int order[3] = {0, 1, 2};
    std::stable_sort(order, order + 3, [&](int x, int y) { return dist[x] > dist[y]; });
    auto steady_with = [&](const bool pf[3]) {
        std::vector<Item> items;
        for (int q = 0; q < 3; ++q) {
            const int t = order[q];
            items.push_back(pf[t] ? Item{t, one_line_size(s, v.ops[t], line_elems), 0}
                                  : Item{t, size[t], dist[t]});
        }
        return setup_list(items, cache_elems);
    };
    const int L = (int)v.loops.size();
    double inner_first = (stage >= 5 && L > 0) ? 1.0 / (double)s.e(v.loops[L - 1]) : 0.0;
    double steady_share = 1.0 - inner_first;
    bool pf_all[3], pf_stream[3];
    bool any_line = false;
    for (int t = 0; t < 3; ++t) {
        pf_all[t] = kind[t] != 0;
        pf_stream[t] = kind[t] == 2;
        any_line = any_line || kind[t] == 1;
    }
    if (stage >= 4 && any_line) {
        double period = (double)line_elems;
        BenchClass st{"steady", steady_share * (period - 1) / period, steady_with(pf_all), -1,
                      std::vector<bool>(pf_all, pf_all + 3)};
        BenchClass fl{"fail", steady_share / period, steady_with(pf_stream), -1,
                      std::vector<bool>(pf_stream, pf_stream + 3)};
        out.push_back(st);
        out.push_back(fl);
    } else {
        out.push_back(BenchClass{"steady", steady_share, steady_with(pf_all), -1,
                                 std::vector<bool>(pf_all, pf_all + 3)});
    }
    if (stage >= 5 && L > 0) {
        // share of invocations at which loops[k..] are all in their first iteration
        std::vector<double> first(L);
        for (int k = 0; k < L; ++k) {
            double f = 1.0;
            for (int m = k; m < L; ++m) f /= (double)s.e(v.loops[m]);
            first[k] = f;
        }
        std::vector<int> own;
        for (int k = L - 1; k >= 0; --k)
            if (k == L - 1 || first[k] > 0.01) own.push_back(k);
        for (size_t q = 0; q < own.size(); ++q) {
            int k = own[q];
            double share = first[k] - (q + 1 < own.size() ? first[own[q + 1]] : 0.0);
            std::vector<Item> items;
            for (int t = 0; t < 3; ++t) items.push_back(Item{t, size[t], access_distance(s, v, t, k, gap[t])});
            BenchClass c{std::string("first@") + v.loops[k], share, setup_list(items, cache_elems), k,
                         std::vector<bool>(3, false)};
            out.push_back(c);
        }
    }
    return out;
}

}  // namespace tc
