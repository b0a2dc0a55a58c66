// Host-only fuzz of the planner, built by the CPU test suite with address and
// undefined-behaviour checks: random specs (half valid by construction with
// free, contracted, batch and trace indices, half arbitrary and mostly
// invalid), extents (zero and negative ones too) and strides, through parsing,
// binding, the GEMM view, the family, each member's schedule and the symbolic
// prediction with and without root gaps.  Usage: host_fuzz <seed> <iterations>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>
#include "../paper_1409_8608_amd/csrc/tc_internal.h"
using namespace tc;
int main(int argc, char** argv) {
    std::mt19937_64 rng(argc > 1 ? atoll(argv[1]) : 1);
    auto U = [&](int n) { return (int)(rng() % (uint64_t)n); };
    long ok = 0, fam = 0;
    const long iters = argc > 2 ? atol(argv[2]) : 20000;
    for (long it = 0; it < iters; ++it) {
        std::string alpha = "abcdefghijklmnopqrstuvwxyz";
        int nl = 1 + U(9);
        std::string pool = alpha.substr(U(26 - nl), nl);
        auto word = [&](int maxlen) {
            std::string w;
            int L = U(maxlen + 1);
            for (int q = 0; q < L; ++q) w += pool[U(pool.size())];
            if (U(50) == 0) w += "A";
            return w;
        };
        std::string text = word(6) + (U(40) ? "=" : "") + word(6) + (U(40) ? "," : "") + word(6);
        if (U(100) == 0) text += ",x";
        if (U(4)) {   // valid by construction: free, contracted, batch and trace classes
            std::string L = "abcdefgijklmst";
            std::shuffle(L.begin(), L.end(), rng);
            int n[6] = {U(3), U(3), U(4), U(2), U(2), U(2)};
            std::string g[6];
            int at = 0;
            for (int q = 0; q < 6; ++q) { g[q] = L.substr(at, n[q]); at += n[q]; }
            std::string a = g[0] + g[2] + g[3] + g[4], b = g[1] + g[2] + g[3] + g[5], c = g[0] + g[1] + g[3];
            std::shuffle(a.begin(), a.end(), rng);
            std::shuffle(b.begin(), b.end(), rng);
            std::shuffle(c.begin(), c.end(), rng);
            text = c + "=" + a + "," + b;
        }
        Spec s;
        Err err;
        if (parse_spec(text.c_str(), s, err)) continue;
        std::string chars;
        std::vector<int64_t> ext;
        for (char ch : s.base)
            if (chars.find(ch) == std::string::npos) { chars += ch; ext.push_back(U(20) == 0 ? -1 : U(5)); }
        if (U(30) == 0 && !chars.empty()) { chars.pop_back(); ext.pop_back(); }
        std::vector<int64_t> st[3];
        const int64_t* sp[3] = {nullptr, nullptr, nullptr};
        for (int t = 0; t < 3; ++t) {
            if (U(2)) continue;
            for (size_t q = 0; q < s.letters(t).size(); ++q) st[t].push_back(U(10) == 0 ? -1 : U(40));
            sp[t] = st[t].data();
        }
        if (bind_spec(s, chars.c_str(), ext.data(), (int)chars.size(), sp[0], sp[1], sp[2], err)) continue;
        ++ok;
        GemmView gv = gemm_view(s);
        std::vector<GtDim> cd = c_dims(s);
        (void)cd;
        if (gv.m.size() > GT_MAXD || gv.n.size() > GT_MAXD || gv.k.size() > GT_MAXD || gv.b.size() > GT_MAXD) continue;
        std::vector<Variant> f = enumerate_family(s);
        fam += (long)f.size();
        for (size_t v = 0; v < f.size() && v < 40; ++v) {
            VariantPlan vp = plan_variant(s, f[v]);
            (void)vp;
            for (int t = 0; t < 3; ++t) (void)access_distance(s, f[v], t, -1, U(3) ? 0 : 1000);
            int64_t gaps[3] = {0, 5, 100000};
            for (int stage = 1; stage <= 5; ++stage) (void)bench_classes(s, f[v], stage, 1000.0, 16, U(2) ? gaps : nullptr);
        }
    }
    printf("bound %ld, members %ld\n", ok, fam);
    return 0;
}
