// Contraction spec: parsing, index roles and binding of extents and strides
// (Section 1, "Tensor Notation"), and the GEMM view of a contraction.
#include <algorithm>
#include <climits>
#include <cstring>

#include "tc_internal.h"

namespace tc {

static bool has(const std::string& s, char ch) { return s.find(ch) != std::string::npos; }

int64_t Spec::flops() const {
    int64_t n = 2;
    for (char ch : base) n *= ext[ch - 'a'];
    return n;
}

// "out=inA,inB": lowercase letters only, no letter twice in one operand; a
// letter is contracted (both inputs, not C) or free (one input and C), the
// paper's two classes, or, read as the same sum over every index absent from
// C, batch (both inputs and C) or trace (one input only).
tc_status parse_spec(const char* text, Spec& s, Err& err) {
    if (!text) return err.set(TC_E_NULL, "spec is NULL");
    std::string t(text);
    size_t eq = t.find('=');
    if (eq == std::string::npos || t.find('=', eq + 1) != std::string::npos)
        return err.set(TC_E_SPEC, "spec needs exactly one '=': " + t);
    size_t comma = t.find(',', eq + 1);
    if (comma == std::string::npos || t.find(',', comma + 1) != std::string::npos)
        return err.set(TC_E_SPEC, "spec needs exactly one ',' after '=': " + t);
    s.c = t.substr(0, eq);
    s.a = t.substr(eq + 1, comma - eq - 1);
    s.b = t.substr(comma + 1);
    for (const std::string* op : {&s.a, &s.b, &s.c}) {
        if (op->size() > 16) return err.set(TC_E_SPEC, "operand with more than 16 indices");
        for (size_t p = 0; p < op->size(); ++p) {
            char ch = (*op)[p];
            if (ch < 'a' || ch > 'z') return err.set(TC_E_SPEC, std::string("index must be a-z: '") + ch + "'");
            if (op->find(ch, p + 1) != std::string::npos)
                return err.set(TC_E_SPEC, std::string("index repeated within one operand: ") + ch);
        }
    }
    s.contracted.clear(); s.free_a.clear(); s.free_b.clear();
    s.batch.clear(); s.trace_a.clear(); s.trace_b.clear();
    for (char ch : s.a) {
        bool inB = has(s.b, ch), inC = has(s.c, ch);
        if (!inB && !inC) s.trace_a += ch;          // summed, B constant along it
        else if (inB && !inC) s.contracted += ch;
    }
    for (char ch : s.b)
        if (!has(s.a, ch) && !has(s.c, ch)) s.trace_b += ch;
    for (char ch : s.c) {
        bool inA = has(s.a, ch), inB = has(s.b, ch);
        if (!inA && !inB) return err.set(TC_E_SPEC, std::string("output index in no input: ") + ch);
        if (inA && inB) s.batch += ch;
        else if (inA) s.free_a += ch;
        else s.free_b += ch;
    }
    s.base = s.c + s.summed();
    return TC_OK;
}

static bool mul_ok(int64_t a, int64_t b, int64_t& out) {
    if (a == 0 || b == 0) { out = 0; return true; }
    if (a > INT64_MAX / b) return false;
    out = a * b;
    return true;
}

tc_status bind_spec(Spec& s, const char* index_chars, const int64_t* extents, int n_index,
                    const int64_t* stA, const int64_t* stB, const int64_t* stC, Err& err) {
    if (n_index < 0 || (n_index > 0 && (!index_chars || !extents)))
        return err.set(TC_E_NULL, "index_chars/extents missing");
    bool seen[26] = {false};
    for (int t = 0; t < n_index; ++t) {
        char ch = index_chars[t];
        if (ch < 'a' || ch > 'z') return err.set(TC_E_EXTENT, std::string("bad index letter '") + ch + "'");
        if (seen[ch - 'a']) return err.set(TC_E_EXTENT, std::string("index given twice: ") + ch);
        if (!has(s.base, ch)) return err.set(TC_E_EXTENT, std::string("index not in the spec: ") + ch);
        if (extents[t] < 0) return err.set(TC_E_EXTENT, std::string("negative extent for ") + ch);
        seen[ch - 'a'] = true;
        s.ext[ch - 'a'] = extents[t];
    }
    for (char ch : s.base)
        if (!seen[ch - 'a']) return err.set(TC_E_EXTENT, std::string("no extent for index ") + ch);

    const std::string* ops[3] = {&s.a, &s.b, &s.c};
    const int64_t* given[3] = {stA, stB, stC};
    int64_t* dst[3] = {s.sA, s.sB, s.sC};
    bool* in[3] = {s.inA, s.inB, s.inC};
    int64_t* counts[3] = {&s.nA, &s.nB, &s.nC};
    int64_t* spans[3] = {&s.spanA, &s.spanB, &s.spanC};
    for (int t = 0; t < 3; ++t) {
        int64_t run = 1, n = 1, last = 0;
        bool overflow = false;
        for (size_t p = 0; p < ops[t]->size(); ++p) {
            char ch = (*ops[t])[p];
            int64_t e = s.ext[ch - 'a'];
            int64_t st = given[t] ? given[t][p] : run;
            if (given[t] && t < 2 && st < 0) return err.set(TC_E_STRIDE, "negative input stride");
            if (given[t] && t == 2 && st <= 0) return err.set(TC_E_STRIDE, "C strides must be positive");
            dst[t][ch - 'a'] = st;
            in[t][ch - 'a'] = true;
            if (!mul_ok(n, e, n)) overflow = true;
            if (!given[t] && !mul_ok(run, e, run)) overflow = true;
            if (e > 0) {
                int64_t reach;
                if (!mul_ok(e - 1, st, reach) || last > INT64_MAX - reach) overflow = true;
                else last += reach;
            }
        }
        if (overflow) return err.set(TC_E_EXTENT, "element count or offset overflows int64");
        *counts[t] = n;
        *spans[t] = n == 0 ? 0 : last + 1;
    }
    // C must not overlap itself: sorted by stride, every stride must clear the
    // extent of everything below it (a sufficient condition for a one-to-one map).
    std::vector<std::pair<int64_t, int64_t>> cd;
    for (char ch : s.c)
        if (s.ext[ch - 'a'] > 1) cd.push_back({s.sC[ch - 'a'], s.ext[ch - 'a']});
    std::sort(cd.begin(), cd.end());
    int64_t reach = 1;
    if (s.nC > 0)
        for (auto& p : cd) {
            if (p.first < reach) return err.set(TC_E_STRIDE, "C strides overlap (C would alias itself)");
            reach = p.first * p.second;
        }
    return TC_OK;
}

// ---------------------------------------------------------------------------
// GEMM view.
void merge_group(std::vector<GtDim>& g) {
    // drop extent-1 dims (they add nothing), then merge d+1 into d when it
    // continues d in every tensor
    std::vector<GtDim> out;
    for (auto& d : g)
        if (d.ext != 1) out.push_back(d);
    bool changed = true;
    while (changed && out.size() > 1) {
        changed = false;
        for (size_t i = 0; i < out.size() && !changed; ++i)
            for (size_t j = 0; j < out.size() && !changed; ++j) {
                if (i == j) continue;
                GtDim& x = out[i];
                GtDim& y = out[j];
                auto cont = [&](int64_t sx, int64_t sy) { return sy == sx * x.ext; };
                if (cont(x.sA, y.sA) && cont(x.sB, y.sB) && cont(x.sC, y.sC)) {
                    x.ext *= y.ext;
                    out.erase(out.begin() + j);
                    changed = true;
                }
            }
    }
    if (out.empty() && !g.empty()) out.push_back(GtDim{1, 0, 0, 0});
    g = out;
}

std::vector<GtDim> c_dims(const Spec& s) {
    std::vector<GtDim> g;
    for (char ch : s.c) g.push_back(GtDim{s.e(ch), 0, 0, s.sC[ch - 'a']});
    merge_group(g);
    if (g.empty()) g.push_back(GtDim{1, 0, 0, 0});
    return g;
}

GemmView gemm_view(const Spec& s) {
    GemmView v;
    // Put C's unit-stride index in M; if it belongs to B, swap the roles of A
    // and B (the contraction is symmetric in its inputs).
    char unit = 0;
    for (char ch : s.c)
        if (s.sC[ch - 'a'] == 1 && s.ext[ch - 'a'] > 1) { unit = ch; break; }
    v.swapped = unit && has(s.free_b, unit);
    const std::string& fm = v.swapped ? s.free_b : s.free_a;
    const std::string& fn = v.swapped ? s.free_a : s.free_b;
    auto sa = [&](char ch) { return v.swapped ? s.sB[ch - 'a'] : s.sA[ch - 'a']; };
    auto sb = [&](char ch) { return v.swapped ? s.sA[ch - 'a'] : s.sB[ch - 'a']; };
    for (char ch : fm) v.m.push_back(GtDim{s.e(ch), sa(ch), 0, s.sC[ch - 'a']});
    for (char ch : fn) v.n.push_back(GtDim{s.e(ch), 0, sb(ch), s.sC[ch - 'a']});
    // trace indices are contracted dimensions with stride 0 in the operand
    // that lacks them (its value is reused along them)
    for (char ch : s.summed()) v.k.push_back(GtDim{s.e(ch), sa(ch), sb(ch), 0});
    for (char ch : s.batch) v.b.push_back(GtDim{s.e(ch), sa(ch), sb(ch), s.sC[ch - 'a']});
    auto by_c = [](const GtDim& x, const GtDim& y) { return x.sC < y.sC; };
    std::stable_sort(v.m.begin(), v.m.end(), by_c);
    std::stable_sort(v.n.begin(), v.n.end(), by_c);
    merge_group(v.m);
    merge_group(v.n);
    merge_group(v.k);
    // no summed index (an outer product): one K position, offset 0 in both
    if (v.k.empty()) v.k.push_back(GtDim{1, 0, 0, 0});
    merge_group(v.b);
    if (v.b.size() == 1 && v.b[0].ext == 1) v.b.clear();
    std::stable_sort(v.m.begin(), v.m.end(), by_c);
    std::stable_sort(v.n.begin(), v.n.end(), by_c);
    v.M = v.N = v.K = 1;
    for (auto& d : v.m) v.M *= d.ext;
    for (auto& d : v.n) v.N *= d.ext;
    for (auto& d : v.k) v.K *= d.ext;
    if (s.free_a.empty() && !v.swapped) v.M = 1;
    return v;
}

}  // namespace tc
