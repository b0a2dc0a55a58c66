// Batches: many independent contractions in one HIP graph.
//
// Every contraction of a batch runs as matrix-core tiles in a persistent
// kernel.  Its candidates are (loop/kernel variant x tile shape): the fused
// GEMM view, or a gemm member of the paper's family (Section 2) whose loops
// are all free indices, so that they become batch dimensions of the tile
// kernel -- for C_abc = A_ai B_ibc, c-gemm and b-gemm -- each with the tile
// shapes 128x128, 64x64 and 32x128 (m x n).  tc_batch_create picks the fused
// view with a default shape (or the tuning cache's choice for a contraction
// seen before), writes one static descriptor per contraction to device memory,
// builds work lists of (contraction, tile) pairs, one per (storage type, tile
// shape, operand layout) group, cut into eight ranges of whole contractions
// balanced by estimated cost (contracted length x tile area x tiles), one per
// XCD so that a contraction's tiles share one L2, each range longest tiles
// first, and captures a graph: a staging
// kernel that copies the call's pointers and scalars from pinned host memory,
// a kernel that zeroes the work counters (no memset nodes), and one persistent
// kernel per group whose blocks take tiles off their XCD's range counter (and
// then off the other ranges' counters), the
// groups spread over up to four graph branches.  tc_batch_contract only writes
// the staging buffer and replays the graph.
//
// Split-precision members: a TC_BF16X3 plan runs as split-BF16 tiles of the
// same persistent kernel (FP64 or FP32 operands split into three BF16 terms
// in the tile, with per-row and per-column power-of-two scales found by a
// first sweep over K; its candidates are the fused view with the three
// shapes), in groups of its own.  A TC_FP8X3 plan runs its plan's own
// launches (split passes and scaled FP8 products) in a graph branch.
//
// tc_batch_tune chooses each contraction's candidate the way Section 3
// predicts a family member: micro-benchmarks of the kernel, run after the
// cache set-up the member meets, composed by invocation counts.  In a batch a
// member's operands were last touched a whole replay ago, so every walk
// reaches the root with a gap of the batch's other data, beyond 5/4 of the
// device cache: the set-up is one remote region of 5/4 of the cache (every
// operand cold).  One micro-benchmark per (storage, shape, contracted-length
// bucket, operand layouts, C layout) times a representative launch after that
// set-up (median of ten); a candidate's estimate is its tile count times the
// per-tile share of the device.  The top_k candidates by estimate are then
// timed alone, each after the same set-up, and the fastest is picked.  Whole
// batches are timed with those picks, with the estimate's first choices and
// with the previous choices, and the fastest set is kept (and put in the
// tuning cache).  tc_batch_score times every candidate of a seeded sample of
// members alone, the same way, and reports how often the estimate's first
// choice, the top_k pick, the kept choice and the untuned default fall within
// 5% of the measured best (and are the best), with their geometric-mean
// regret.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "launch.h"
#include "plan.h"

using namespace tc;

namespace {

// One way to run a batch member: a loop/kernel variant (the fused view or a
// gemm member) with a tile shape.
struct Cand {
    int variant;        // TC_VARIANT_FUSED or a family member index
    int shape;          // 0: 128x128, 1: 64x64, 2: 32x128
    int64_t tab_off;    // its K table in the batch's table array
    int64_t kpad;
    bool swap;          // A and B exchange places in the tile kernel
};

struct BatchGroup {
    bool f64;
    bool x3;            // split-BF16 tiles
    int shape;
    bool ak, bk;
    std::vector<int2> work;   // eight per-XCD ranges of whole contractions
    int xstart[9] = {0};      // range offsets
    int2* d_work = nullptr;   // the list, then the nine offsets
    int grid = 1;
};

constexpr int kShapes = 3;
constexpr int BATCH_BK = 16;
constexpr double kCacheBytes = 256.0 * 1024 * 1024;   // the device's last-level cache

// Tuning cache: a contraction's kept candidate (variant, shape) by its plan
// signature, for the batches a process builds later.
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune_cache;

std::string signature(const tc_plan_s* p) {
    const Spec& s = p->spec;
    std::string k = std::to_string((int)s.dtype) + "/" + std::to_string((int)s.compute) + "|" + s.a + "," + s.b +
                    "=" + s.c + "|";
    for (char ch : s.base) k += std::to_string(s.e(ch)) + ",";
    for (int t = 0; t < 3; ++t) {
        k += "|";
        for (char ch : s.letters(t)) k += std::to_string(s.stride(t, ch)) + ",";
    }
    return k;
}

}  // namespace

struct tc_batch_s {
    std::vector<tc_plan_s*> plans;
    std::vector<char> split;                // member runs the split-FP8 form (its plan's own launches)
    std::vector<char> x3;                   // member runs split-BF16 tiles
    std::vector<std::vector<Cand>> cands;   // per member (none for a split-FP8 member)
    std::vector<int> choice;                // index into cands[c]
    std::vector<int> deflt;                 // the untuned default's index
    std::vector<std::vector<double>> est;   // seed estimates (seconds), filled by tuning
    std::vector<int> topk;                  // the tuner's pick among the top_k timed alone (-1: none)
    std::vector<MfmaArgs> items;            // static descriptors of the chosen candidates
    std::vector<BatchGroup> groups;
    MfmaArgs* d_items = nullptr;
    BatchPtrs* d_ptrs = nullptr;
    BatchPtrs* h_ptrs = nullptr;     // pinned
    int* d_counters = nullptr;
    int64_t* d_ktab = nullptr;       // all K tables, concatenated
    hipStream_t cap = nullptr;
    hipStream_t side[3] = {nullptr, nullptr, nullptr};   // capture branches (default priority)
    hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
    double hit_rate = -1.0;          // within-5% rate of the tuned choice in the last score
};

namespace tc {

__global__ void k_stage(const BatchPtrs* __restrict__ src, BatchPtrs* __restrict__ dst, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_zero(int* c, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0;
}

static void free_groups(tc_batch_s* b) {
    for (auto& g : b->groups)
        if (g.d_work) (void)hipFree(g.d_work);
    b->groups.clear();
    if (b->d_counters) (void)hipFree(b->d_counters);
    b->d_counters = nullptr;
}

static void drop_graph(tc_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

static int default_shape(const MfmaArgs& a) { return a.M <= 32 ? 2 : (a.M <= 64 || a.N <= 64) ? 1 : 0; }

// A family member the tile kernel runs as one item: a gemm whose loops are all
// free indices (they become batch dimensions), with no copies.
static bool batchable_member(const VariantPlan& vp) {
    return vp.mfma && vp.copies.empty() && vp.hoisted.empty() && vp.body.pass.n == 0 && !vp.needs_c_copy;
}

// The static descriptor of candidate `cd` of member `c` (pointers unset).
static MfmaArgs make_item(const tc_batch_s* b, int c, const Cand& cd) {
    tc_plan_s* p = b->plans[c];
    MfmaArgs a{};
    if (b->split[c]) return a;            // no tiles: the split-FP8 form runs its own launches
    if (cd.variant == TC_VARIANT_FUSED) {
        const GemmView& gv = p->gv;
        a.m.n = (int)gv.m.size();
        for (int d = 0; d < a.m.n; ++d) a.m.d[d] = gv.m[d];
        a.n.n = (int)gv.n.size();
        for (int d = 0; d < a.n.n; ++d) a.n.d[d] = gv.n[d];
        a.batch.n = (int)gv.b.size();
        a.nbatch = 1;
        for (int d = 0; d < a.batch.n; ++d) {
            a.batch.d[d] = gv.b[d];
            a.nbatch *= gv.b[d].ext;
        }
        a.M = gv.M;
        a.N = gv.N;
    } else {
        // the member's body (Section 2 loop nest on the device): M and N the
        // kernel's kept free indices, its loops the batch dimensions
        const GtDesc& d = p->vplans()[cd.variant].body;
        a.m.n = d.nm;
        if (d.nm) a.m.d[0] = d.out.d[0];
        a.n.n = d.nn;
        if (d.nn) a.n.d[0] = d.out.d[d.nm];
        a.batch.n = 0;
        a.nbatch = 1;
        for (int q = d.nm + d.nn; q < d.out.n; ++q) {
            a.batch.d[a.batch.n++] = d.out.d[q];
            a.nbatch *= d.out.d[q].ext;
        }
        a.M = d.nm ? d.out.d[0].ext : 1;
        a.N = d.nn ? d.out.d[d.nm].ext : 1;
    }
    a.pass.n = 0;
    a.npass = 1;
    a.ktab = b->d_ktab + cd.tab_off;
    a.Kpad = cd.kpad;
    a.mode = 0;
    mfma_tiles_shape(cd.shape, a);
    return a;
}

// work lists per group, longest tiles first
static tc_status build_groups(tc_batch_s* b) {
    free_groups(b);
    const int n = (int)b->plans.size();
    b->items.resize(n);
    for (int c = 0; c < n; ++c) b->items[c] = b->split[c] ? MfmaArgs{} : make_item(b, c, b->cands[c][b->choice[c]]);
    std::map<int, int> gid;   // key -> group index
    std::vector<std::vector<int>> gmembers;   // members of each group
    int ncu = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    for (int c = 0; c < n; ++c) {
        if (b->split[c]) continue;
        MfmaArgs& a = b->items[c];
        const bool f64 = b->plans[c]->spec.dtype == TC_F64;
        const bool x3 = b->x3[c];
        const bool ak = mfma_kmajor_a(a), bk = mfma_kmajor_b(a);
        const int sh = b->cands[c][b->choice[c]].shape;
        const int key = (x3 ? 32 : 0) | (f64 ? 16 : 0) | (sh << 2) | (ak ? 2 : 0) | (bk ? 1 : 0);   // sh in 0..3
        if (!gid.count(key)) {
            gid[key] = (int)b->groups.size();
            BatchGroup g;
            g.f64 = f64;
            g.x3 = x3;
            g.shape = sh;
            g.ak = ak;
            g.bk = bk;
            b->groups.push_back(g);
            gmembers.emplace_back();
        }
        gmembers[gid[key]].push_back(c);
    }
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        BatchGroup& g = b->groups[gi];
        // Members go whole to the XCD with the least estimated work so far,
        // largest members first (cost of a tile: contracted length x tile
        // area); each range then lists its members longest tiles first, a
        // member's tiles together.
        auto tile_cost = [&](int c) {
            const int sh = b->cands[c][b->choice[c]].shape;
            return b->items[c].Kpad * (sh == 0 ? 128 * 128 : sh == 1 ? 64 * 64 : 32 * 128);
        };
        std::vector<int> ms = gmembers[gi];
        std::stable_sort(ms.begin(), ms.end(), [&](int x, int y) {
            return tile_cost(x) * b->items[x].ntiles > tile_cost(y) * b->items[y].ntiles;
        });
        std::vector<int> xm[8];
        int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int c : ms) {
            const int x = (int)(std::min_element(load, load + 8) - load);
            xm[x].push_back(c);
            load[x] += tile_cost(c) * b->items[c].ntiles;
        }
        for (int x = 0; x < 8; ++x) {
            std::stable_sort(xm[x].begin(), xm[x].end(), [&](int p, int q) { return tile_cost(p) > tile_cost(q); });
            g.xstart[x] = (int)g.work.size();
            for (int c : xm[x])
                for (int64_t t = 0; t < b->items[c].ntiles; ++t) g.work.push_back(int2{c, (int)t});
        }
        g.xstart[8] = (int)g.work.size();
        const size_t list_bytes = sizeof(int2) * g.work.size();
        hipError_t e = hipMalloc(&g.d_work, list_bytes + sizeof(g.xstart));
        if (e != hipSuccess) return fail(TC_E_NOMEM, "hipMalloc batch work list");
        e = hipMemcpy(g.d_work, g.work.data(), list_bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((char*)g.d_work + list_bytes, g.xstart, sizeof(g.xstart), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload batch work list");
        int occ = g.x3 ? x3_batch_occupancy(g.f64, g.shape, g.ak, g.bk) : mfma_batch_occupancy(g.f64, g.shape, g.ak, g.bk);
        g.grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)g.work.size(), (int64_t)occ * ncu));
    }
    hipError_t e = hipMalloc(&b->d_counters, sizeof(int) * 8 * std::max<size_t>(1, b->groups.size()));
    if (e != hipSuccess) return fail(TC_E_NOMEM, "hipMalloc batch counters");
    e = hipMemcpy(b->d_items, b->items.data(), sizeof(MfmaArgs) * b->items.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload batch descriptors");
    return TC_OK;
}

static tc_status capture(tc_batch_s* b) {
    drop_graph(b);
    const int n = (int)b->items.size();
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    hipLaunchKernelGGL(k_stage, dim3((n + 255) / 256), dim3(256), 0, b->cap, b->h_ptrs, b->d_ptrs, n);
    const int ncount = 8 * (int)b->groups.size();   // eight per-XCD counters per group
    hipLaunchKernelGGL(k_zero, dim3(std::max(1, (ncount + 63) / 64)), dim3(64), 0, b->cap, b->d_counters, ncount);
    // the groups (and the split-FP8 members) are independent: up to four
    // branches of the graph, so that one group's tail overlaps the next group's
    // blocks
    std::vector<int> splits;
    for (int c = 0; c < n; ++c)
        if (b->split[c]) splits.push_back(c);
    const size_t jobs = b->groups.size() + splits.size();
    const int nb = (int)std::min<size_t>(4, jobs);
    if (nb > 1 && e == hipSuccess) e = hipEventRecord(b->fork, b->cap);
    for (int q = 1; q < nb && e == hipSuccess; ++q) e = hipStreamWaitEvent(b->side[q - 1], b->fork, 0);
    tc_status st = TC_OK;
    for (size_t j = 0; j < jobs && e == hipSuccess && !st; ++j) {
        const int q = (int)(j % nb);
        hipStream_t sq = q == 0 ? b->cap : b->side[q - 1];
        if (j < b->groups.size()) {
            BatchGroup& g = b->groups[j];
            const int* xs = (const int*)((const char*)g.d_work + sizeof(int2) * g.work.size());
            hipError_t le = (g.x3 ? launch_x3_batch : launch_mfma_batch)(g.f64, g.shape, g.ak, g.bk, b->d_items,
                                                                         b->d_ptrs, g.d_work, xs, (int)g.work.size(),
                                                                         b->d_counters + 8 * j, g.grid, sq);
            if (le != hipSuccess) e = le;
        } else {
            const int c = splits[j - b->groups.size()];
            st = run_split_batched(b->plans[c], b->d_ptrs + c, sq);
        }
    }
    for (int q = 1; q < nb && e == hipSuccess && !st; ++q) {
        e = hipEventRecord(b->join[q - 1], b->side[q - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->join[q - 1], 0);
    }
    if (st) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(b->cap, &g);
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(e != hipSuccess ? e : e2, "capture batch graph");
    }
    b->graph = graph;
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "instantiate batch graph");
    return TC_OK;
}

static tc_status rebuild(tc_batch_s* b) {
    drop_graph(b);
    tc_status st = build_groups(b);
    return st ? st : capture(b);
}

// Timing of single members' candidates after the batch's cache set-up (every
// operand cold: a remote region of 5/4 of the device cache is touched first).
struct Timer {
    tc_batch_s* b;
    hipStream_t st;
    void* scratch = nullptr;
    float* sink = nullptr;
    int64_t scratch_bytes = 0;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int ncu = 256;

    tc_status open() {
        st = b->cap;
        scratch_bytes = (int64_t)(1.25 * kCacheBytes) + (1 << 20);
        if (hipMalloc(&scratch, (size_t)scratch_bytes) != hipSuccess) return fail(TC_E_NOMEM, "tuning scratch");
        if (hipMalloc(&sink, 256) != hipSuccess) return fail(TC_E_NOMEM, "tuning scratch");
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return fail(TC_E_HIP, "events");
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            ncu = prop.multiProcessorCount;
        return TC_OK;
    }
    ~Timer() {
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
        if (scratch) (void)hipFree(scratch);
        if (sink) (void)hipFree(sink);
    }
    // the previous call gave this member all three operands (an alpha = 0
    // member may have left A and B out: it is not timed)
    bool usable(int c) const { return !b->split[c] && b->h_ptrs[c].A && b->h_ptrs[c].B && b->h_ptrs[c].C; }
    MfmaArgs item(int c, const Cand& cd) {
        MfmaArgs a = make_item(b, c, cd);
        const BatchPtrs& pt = b->h_ptrs[c];
        a.A = cd.swap ? pt.B : pt.A;
        a.B = cd.swap ? pt.A : pt.B;
        a.C = pt.C;
        a.alpha = pt.alpha == 0.0 ? 1.0 : pt.alpha;
        a.beta = 0.0;
        return a;
    }
    // median of `reps` timings (seconds) of candidate cd of member c, one warm-up first
    hipError_t time(int c, const Cand& cd, int reps, double* out) {
        MfmaArgs a = item(c, cd);
        const bool f64 = b->plans[c]->spec.dtype == TC_F64;
        std::vector<float> ts;
        for (int r = 0; r <= reps; ++r) {
            hipError_t e = launch_touch(scratch, scratch_bytes, sink, st);
            if (e == hipSuccess) e = hipEventRecord(t0, st);
            if (e == hipSuccess) e = (b->x3[c] ? launch_x3_shape : launch_mfma_shape)(f64, cd.shape, a, st);
            if (e == hipSuccess) e = hipEventRecord(t1, st);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e != hipSuccess) return e;
            if (r > 0) ts.push_back(ms);
        }
        std::sort(ts.begin(), ts.end());
        *out = ts[ts.size() / 2] * 1e-3;
        return hipSuccess;
    }
};

static int kbucket(int64_t kpad) {
    int bkt = 0;
    while ((16LL << bkt) < kpad && bkt < 12) ++bkt;
    return bkt;
}

// micro-benchmark key of a candidate: storage, shape, contracted-length
// bucket, operand layouts, C unit-stride along m
static std::string bench_key(const tc_batch_s* b, int c, const Cand& cd, const MfmaArgs& a) {
    const bool cm1 = a.m.n > 0 && a.m.d[0].sC == 1;
    return std::to_string((int)b->plans[c]->spec.dtype) + (b->x3[c] ? "x/" : "/") + std::to_string(cd.shape) + "/" +
           std::to_string(kbucket(cd.kpad)) + "/" + std::to_string((int)mfma_kmajor_a(a)) +
           std::to_string((int)mfma_kmajor_b(a)) + std::to_string((int)cm1);
}

// Seed estimates of every candidate (see the file comment).
static tc_status seed_estimates(tc_batch_s* b, Timer& tm) {
    const int n = (int)b->plans.size();
    std::map<std::string, std::pair<int64_t, std::pair<int, int>>> rep;   // key -> (tiles, (member, cand))
    for (int c = 0; c < n; ++c)
        for (int j = 0; j < (int)b->cands[c].size() && tm.usable(c); ++j) {
            const MfmaArgs a = make_item(b, c, b->cands[c][j]);
            const std::string key = bench_key(b, c, b->cands[c][j], a);
            auto it = rep.find(key);
            if (it == rep.end() || it->second.first < a.ntiles) rep[key] = {a.ntiles, {c, j}};
        }
    std::map<std::string, double> per_tile;
    for (auto& kv : rep) {
        const int c = kv.second.second.first, j = kv.second.second.second;
        const Cand& cd = b->cands[c][j];
        const MfmaArgs a = make_item(b, c, cd);
        const bool f64 = b->plans[c]->spec.dtype == TC_F64;
        double t;
        hipError_t e = tm.time(c, cd, 10, &t);            // Section 3: median of ten
        if (e != hipSuccess) return hip_fail(e, "tuning micro-benchmark");
        const int64_t wave = (int64_t)(b->x3[c] ? x3_batch_occupancy : mfma_batch_occupancy)(
                                 f64, cd.shape, mfma_kmajor_a(a), mfma_kmajor_b(a)) * tm.ncu;
        per_tile[kv.first] = t / (double)std::max<int64_t>(a.ntiles, wave);
    }
    b->est.assign(n, {});
    for (int c = 0; c < n; ++c)
        for (const Cand& cd : b->cands[c]) {
            const MfmaArgs a = make_item(b, c, cd);
            b->est[c].push_back(per_tile[bench_key(b, c, cd, a)] * (double)a.ntiles);
        }
    return TC_OK;
}

static int argmin(const std::vector<double>& v) {
    return (int)(std::min_element(v.begin(), v.end()) - v.begin());
}

}  // namespace tc

extern "C" {

tc_status tc_batch_create(tc_batch_t* out, const tc_plan_t* plans, int n) {
    if (!out) return fail(TC_E_NULL, "out is NULL");
    *out = nullptr;
    if (n < 0 || (n > 0 && !plans)) return fail(TC_E_NULL, "plans is NULL");
    tc_batch_s* b = new (std::nothrow) tc_batch_s();
    if (!b) return fail(TC_E_NOMEM, "host allocation");
    std::vector<int64_t> tab_all;
    for (int c = 0; c < n; ++c) {
        tc_plan_s* p = plans[c];
        if (!p) {
            delete b;
            return fail(TC_E_NULL, "a plan is NULL");
        }
        if (p->spec.is_complex()) {
            delete b;
            return fail(TC_E_UNSUPPORTED, "batches take real plans");
        }
        if (p->spec.nC == 0 || p->gv.K == 0) {
            delete b;
            return fail(TC_E_UNSUPPORTED, "batch members need a non-empty C and contracted extent");
        }
        if (p->spec.compute == TC_BF16X3 && p->split_products != 6) {
            delete b;
            return fail(TC_E_UNSUPPORTED, "batch split-BF16 tiles keep six term products");
        }
        b->plans.push_back(p);
        b->x3.push_back(p->spec.compute == TC_BF16X3);
        if (p->spec.compute == TC_FP8X3) {
            // the split-FP8 form (per-slice scaled FP8 terms on matrix cores)
            // runs its plan's own launches in the graph, on the plan's
            // workspace: a plan can be one such member only
            for (int q = 0; q < c; ++q)
                if (plans[q] == p) {
                    delete b;
                    return fail(TC_E_UNSUPPORTED, "a split-FP8 plan is listed twice (its workspace is per plan)");
                }
            if (!p->d_split) {
                delete b;
                return fail(TC_E_UNSUPPORTED, "split-FP8 member without its workspace (plan built with no GPU)");
            }
            if (split_positions(p) > 8192) {
                delete b;
                return fail(TC_E_UNSUPPORTED, "FP8 split form takes at most 8192 contracted positions");
            }
            b->split.push_back(1);
            b->cands.emplace_back();
            continue;
        }
        b->split.push_back(0);
        std::vector<Cand> cs;
        auto add_variant = [&](int v, const std::vector<GtDim>& kd, bool swap) {
            std::vector<int64_t> tab = build_ktab(kd, BATCH_BK);
            const int64_t off = (int64_t)tab_all.size();
            tab_all.insert(tab_all.end(), tab.begin(), tab.end());
            for (int sh = 0; sh < kShapes; ++sh) cs.push_back(Cand{v, sh, off, (int64_t)tab.size() / 2, swap});
        };
        add_variant(TC_VARIANT_FUSED, p->gv.k, p->gv.swapped);
        // gemm members keep the one contracted index: only specs with a single
        // contracted index (and no batch or trace index) have members whose
        // loops are all free (split-BF16 members: the fused view only)
        if (p->spec.contracted.size() == 1 && !p->spec.general() && !b->x3.back()) {
            for (int v = 0; v < (int)p->fam().size(); ++v) {
                const VariantPlan& vp = p->vplans()[v];
                if (batchable_member(vp)) add_variant(v, {vp.body.kb}, false);
            }
        }
        b->cands.push_back(cs);
    }
    hipError_t e = hipMalloc(&b->d_ktab, sizeof(int64_t) * std::max<size_t>(1, tab_all.size()));
    if (e == hipSuccess && !tab_all.empty())
        e = hipMemcpy(b->d_ktab, tab_all.data(), sizeof(int64_t) * tab_all.size(), hipMemcpyHostToDevice);
    // default: the fused view with the default shape, or the tuning cache's choice
    for (int c = 0; c < n && e == hipSuccess; ++c) {
        if (b->split[c]) {
            b->deflt.push_back(-1);
            b->choice.push_back(-1);
            continue;
        }
        int d = 0;
        const MfmaArgs a0 = make_item(b, c, b->cands[c][0]);
        for (int j = 0; j < (int)b->cands[c].size(); ++j)
            if (b->cands[c][j].variant == TC_VARIANT_FUSED && b->cands[c][j].shape == default_shape(a0)) d = j;
        b->deflt.push_back(d);
        int ch = d;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(signature(b->plans[c]));
        if (it != g_tune_cache.end())
            for (int j = 0; j < (int)b->cands[c].size(); ++j)
                if (b->cands[c][j].variant == it->second.first && b->cands[c][j].shape == it->second.second) ch = j;
        b->choice.push_back(ch);
    }
    if (e == hipSuccess) e = hipMalloc(&b->d_items, sizeof(MfmaArgs) * std::max(1, n));
    if (e == hipSuccess) e = hipMalloc(&b->d_ptrs, sizeof(BatchPtrs) * std::max(1, n));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_ptrs, sizeof(BatchPtrs) * std::max(1, n), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    for (int q = 0; q < 3 && e == hipSuccess; ++q) e = hipStreamCreateWithFlags(&b->side[q], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int q = 0; q < 3 && e == hipSuccess; ++q) e = hipEventCreateWithFlags(&b->join[q], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        tc_batch_destroy(b);
        return fail(TC_E_NOMEM, std::string("batch set-up: ") + hipGetErrorString(e));
    }
    std::memset(b->h_ptrs, 0, sizeof(BatchPtrs) * std::max(1, n));
    tc_status st = rebuild(b);          // the graph reads the call's pointers from pinned staging
    if (st) {
        tc_batch_destroy(b);
        return st;
    }
    *out = b;
    return TC_OK;
}

tc_status tc_batch_destroy(tc_batch_t b) {
    if (!b) return TC_OK;
    if (b->launched) (void)hipEventSynchronize(b->done);
    drop_graph(b);
    free_groups(b);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_ptrs) (void)hipFree(b->d_ptrs);
    if (b->h_ptrs) (void)hipHostFree(b->h_ptrs);
    if (b->d_ktab) (void)hipFree(b->d_ktab);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int q = 0; q < 3; ++q) {
        if (b->side[q]) (void)hipStreamDestroy(b->side[q]);
        if (b->join[q]) (void)hipEventDestroy(b->join[q]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->done) (void)hipEventDestroy(b->done);
    delete b;
    return TC_OK;
}

tc_status tc_batch_contract(tc_batch_t b, const void* const* A, const void* const* B, void* const* C,
                            const double* alpha, const double* beta, void* stream) {
    if (!b) return fail(TC_E_NULL, "batch is NULL");
    const int n = (int)b->items.size();
    if (n == 0) return TC_OK;
    if (!A || !B || !C || !alpha || !beta) return fail(TC_E_NULL, "NULL argument array");
    for (int c = 0; c < n; ++c) {
        const Spec& s = b->plans[c]->spec;
        if (!C[c]) return fail(TC_E_NULL, "NULL C in batch member " + std::to_string(c));
        if (alpha[c] == 0.0) continue;            // A and B are not read
        if (!A[c] || !B[c]) return fail(TC_E_NULL, "NULL A or B in batch member " + std::to_string(c));
        const int es = s.elem_bytes();
        auto ov = [&](const void* x, int64_t sx, const void* y, int64_t sy) {
            uintptr_t x0 = (uintptr_t)x, x1 = x0 + (uintptr_t)(sx * es), y0 = (uintptr_t)y, y1 = y0 + (uintptr_t)(sy * es);
            return x0 < y1 && y0 < x1;
        };
        if (ov(C[c], s.spanC, A[c], s.spanA) || ov(C[c], s.spanC, B[c], s.spanB))
            return fail(TC_E_ALIAS, "C overlaps A or B in batch member " + std::to_string(c));
    }
    if (b->launched) {
        hipError_t e = hipEventSynchronize(b->done);   // the staging buffer is read by the previous replay
        if (e != hipSuccess) return hip_fail(e, "wait for previous batch");
    }
    for (int c = 0; c < n; ++c) {
        // each member's operands in its kernels' order (the split-FP8 form and the
        // fused view take A and B in GEMM-view order)
        const bool sw = b->split[c] ? b->plans[c]->gv.swapped : b->cands[c][b->choice[c]].swap;
        b->h_ptrs[c].A = sw ? B[c] : A[c];
        b->h_ptrs[c].B = sw ? A[c] : B[c];
        b->h_ptrs[c].C = C[c];
        b->h_ptrs[c].alpha = alpha[c];
        b->h_ptrs[c].beta = beta[c];
    }
    if (!b->exec) return fail(TC_E_UNSUPPORTED, "batch graph missing (an earlier tc_batch_tune failed)");
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch batch graph");
    e = hipEventRecord(b->done, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "record batch event");
    b->launched = true;
    return TC_OK;
}

// Candidate choice (see the file comment).  Uses the operands of the previous
// tc_batch_contract call, which must have been made.
tc_status tc_batch_tune(tc_batch_t b, int top_k) {
    if (!b) return fail(TC_E_NULL, "batch is NULL");
    if (!b->launched) return fail(TC_E_UNSUPPORTED, "call tc_batch_contract once before tuning");
    if (top_k < 1) top_k = 1;
    hipError_t e = hipEventSynchronize(b->done);
    if (e != hipSuccess) return hip_fail(e, "synchronize");
    const int n = (int)b->plans.size();
    // the tuned members' staging entries: the previous call's pointers (in
    // candidate-independent order) and alpha; C := alpha * contract(A, B)
    auto swapped = [&](int c) { return !b->split[c] && b->cands[c][b->choice[c]].swap; };
    for (int c = 0; c < n; ++c)
        if (swapped(c)) std::swap(b->h_ptrs[c].A, b->h_ptrs[c].B);
    Timer tm{b, nullptr};
    tc_status st = tm.open();
    if (!st) st = seed_estimates(b, tm);
    // whole-batch time of a configuration: graph replays with beta = 0
    auto time_graph = [&](double* out) -> tc_status {
        for (int c = 0; c < n; ++c) {
            b->h_ptrs[c].beta = 0.0;
            if (b->h_ptrs[c].alpha == 0.0) b->h_ptrs[c].alpha = 1.0;
        }
        // staging holds the pointers in A, B order; the graph wants each
        // member's kernel order
        std::vector<BatchPtrs> keep(b->h_ptrs, b->h_ptrs + n);
        for (int c = 0; c < n; ++c)
            if (swapped(c)) std::swap(b->h_ptrs[c].A, b->h_ptrs[c].B);
        hipError_t err = hipGraphLaunch(b->exec, tm.st);   // warm-up
        if (err == hipSuccess) err = hipEventRecord(tm.t0, tm.st);
        for (int r = 0; r < 5 && err == hipSuccess; ++r) err = hipGraphLaunch(b->exec, tm.st);
        if (err == hipSuccess) err = hipEventRecord(tm.t1, tm.st);
        if (err == hipSuccess) err = hipEventSynchronize(tm.t1);
        float ms = 0;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, tm.t0, tm.t1);
        std::copy(keep.begin(), keep.end(), b->h_ptrs);
        if (err != hipSuccess) return hip_fail(err, "batch timing replays");
        *out = ms / 5.0;
        return TC_OK;
    };
    double before_ms = 0.0;
    if (!st) st = time_graph(&before_ms);
    const std::vector<int> old_choice = b->choice;
    std::vector<int> seed_choice = b->choice, iso_choice = b->choice;
    b->topk.assign(n, -1);
    for (int c = 0; c < n && !st; ++c) {
        if (!tm.usable(c)) continue;
        std::vector<int> order(b->cands[c].size());
        for (int j = 0; j < (int)order.size(); ++j) order[j] = j;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->est[c][x] < b->est[c][y]; });
        seed_choice[c] = order[0];
        double best_t = INFINITY;
        int best = order[0];
        for (int q = 0; q < (int)order.size() && q < top_k; ++q) {
            double t;
            e = tm.time(c, b->cands[c][order[q]], 3, &t);
            if (e != hipSuccess) {
                st = hip_fail(e, "tuning launches");
                break;
            }
            if (t < best_t) {
                best_t = t;
                best = order[q];
            }
        }
        iso_choice[c] = best;
        b->topk[c] = best;
    }
    // A member timed alone runs on an idle device, where small tiles win by
    // parallelism; inside the batch the device is full and a tile's share of
    // it counts, which the estimate models (tile count x per-tile share).  So
    // the whole batch is timed with the picks among the top_k, with the
    // estimate's first choices, and with the previous choices, and a new
    // configuration replaces the kept one only if it beats two timings of it
    // (replay times drift by a few percent, as much as a change gains or
    // loses).
    auto use = [&](const std::vector<int>& ch) {
        b->choice = ch;
        return rebuild(b);
    };
    std::vector<int> kept = old_choice;
    double kept_ms = before_ms;
    for (const std::vector<int>* cfg : {&iso_choice, &seed_choice}) {
        if (st || *cfg == kept) continue;
        double new_ms = 0.0, again_ms = 0.0;
        st = use(*cfg);
        if (!st) st = time_graph(&new_ms);
        if (st || new_ms >= kept_ms) continue;
        st = use(kept);
        if (!st) st = time_graph(&again_ms);
        if (!st && new_ms < again_ms) {
            kept = *cfg;
            kept_ms = new_ms;
        }
    }
    if (!st) st = use(kept);
    // staging back in each kept choice's kernel order
    for (int c = 0; c < n; ++c)
        if (swapped(c)) std::swap(b->h_ptrs[c].A, b->h_ptrs[c].B);
    if (!st) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (int c = 0; c < n; ++c)
            if (!b->split[c])
                g_tune_cache[signature(b->plans[c])] = {b->cands[c][b->choice[c]].variant,
                                                        b->cands[c][b->choice[c]].shape};
    }
    return st;
}

tc_status tc_batch_score(tc_batch_t b, int sample, uint64_t seed, tc_tune_score* out) {
    if (!b || !out) return fail(TC_E_NULL, "NULL argument");
    if (!b->launched) return fail(TC_E_UNSUPPORTED, "call tc_batch_contract once before scoring");
    std::memset(out, 0, sizeof(*out));
    hipError_t e = hipEventSynchronize(b->done);
    if (e != hipSuccess) return hip_fail(e, "synchronize");
    const int n = (int)b->plans.size();
    if (n == 0 || sample <= 0) return TC_OK;
    Timer tm{b, nullptr};
    tc_status st = tm.open();
    // the staging entries in A, B order for the timer
    auto swapped = [&](int c) { return !b->split[c] && b->cands[c][b->choice[c]].swap; };
    for (int c = 0; c < n; ++c)
        if (swapped(c)) std::swap(b->h_ptrs[c].A, b->h_ptrs[c].B);
    if (!st && b->est.empty()) st = seed_estimates(b, tm);
    std::vector<int> members;
    for (int c = 0; c < n; ++c)
        if (tm.usable(c)) members.push_back(c);
    std::mt19937_64 rng(seed);
    std::shuffle(members.begin(), members.end(), rng);
    members.resize(std::min((int)members.size(), sample));
    if (members.empty()) st = fail(TC_E_UNSUPPORTED, "no member with all three operands to time");
    double lr[4] = {0, 0, 0, 0};
    int hit[4] = {0, 0, 0, 0}, top[4] = {0, 0, 0, 0}, best_member = 0, n_cand = 0;
    for (int c : members) {
        if (st) break;
        std::vector<double> t(b->cands[c].size());
        for (size_t j = 0; j < t.size(); ++j) {
            e = tm.time(c, b->cands[c][j], 5, &t[j]);
            if (e != hipSuccess) {
                st = hip_fail(e, "scoring launches");
                break;
            }
        }
        if (st) break;
        n_cand += (int)t.size();
        const int best = argmin(t);
        if (b->cands[c][best].variant != TC_VARIANT_FUSED) ++best_member;
        const int pick[4] = {argmin(b->est[c]), b->choice[c], b->deflt[c],
                             b->topk.empty() || b->topk[c] < 0 ? argmin(b->est[c]) : b->topk[c]};
        for (int q = 0; q < 4; ++q) {
            const double r = t[pick[q]] / t[best];
            lr[q] += std::log(r);
            if (r <= 1.05) ++hit[q];
            if (pick[q] == best) ++top[q];
        }
    }
    for (int c = 0; c < n; ++c)
        if (swapped(c)) std::swap(b->h_ptrs[c].A, b->h_ptrs[c].B);
    if (st) return st;
    const double m = (double)members.size();
    out->n_sampled = (int)members.size();
    out->candidates_mean = n_cand / m;
    out->within5_seed = hit[0] / m;
    out->argmin_seed = top[0] / m;
    out->regret_seed = std::exp(lr[0] / m);
    out->within5_tuned = hit[1] / m;
    out->argmin_tuned = top[1] / m;
    out->regret_tuned = std::exp(lr[1] / m);
    out->within5_default = hit[2] / m;
    out->argmin_default = top[2] / m;
    out->regret_default = std::exp(lr[2] / m);
    out->within5_topk = hit[3] / m;
    out->argmin_topk = top[3] / m;
    out->regret_topk = std::exp(lr[3] / m);
    out->member_best_share = best_member / m;
    b->hit_rate = out->within5_tuned;
    return TC_OK;
}

tc_status tc_batch_info(tc_batch_t b, int* n_members, int64_t* n_tiles, int* n_groups, double* tune_hit_rate) {
    if (!b) return fail(TC_E_NULL, "batch is NULL");
    int64_t tiles = 0;
    for (auto& g : b->groups) tiles += (int64_t)g.work.size();
    if (n_members) *n_members = (int)b->plans.size();
    if (n_tiles) *n_tiles = tiles;
    if (n_groups) *n_groups = (int)b->groups.size();
    if (tune_hit_rate) *tune_hit_rate = b->hit_rate;
    return TC_OK;
}

tc_status tc_batch_set_choice(tc_batch_t b, int member, int variant, int shape) {
    if (!b) return fail(TC_E_NULL, "batch is NULL");
    if (member < 0 || member >= (int)b->plans.size()) return fail(TC_E_VARIANT, "member out of range");
    if (b->split[member]) return fail(TC_E_VARIANT, "a split-FP8 member has no tile candidates");
    int j = -1;
    for (int q = 0; q < (int)b->cands[member].size(); ++q)
        if (b->cands[member][q].variant == variant && b->cands[member][q].shape == shape) j = q;
    if (j < 0) return fail(TC_E_VARIANT, "not a candidate of this member (a gemm member whose loops are all free "
                                          "indices, or the fused view, with shape 0..2)");
    if (b->launched) {
        hipError_t e = hipEventSynchronize(b->done);
        if (e != hipSuccess) return hip_fail(e, "synchronize");
    }
    // the staged pointers follow the member's kernel order
    if (b->cands[member][b->choice[member]].swap != b->cands[member][j].swap)
        std::swap(b->h_ptrs[member].A, b->h_ptrs[member].B);
    b->choice[member] = j;
    return rebuild(b);
}

tc_status tc_batch_choice(tc_batch_t b, int member, int* variant, int* shape, int* n_candidates) {
    if (!b) return fail(TC_E_NULL, "batch is NULL");
    if (member < 0 || member >= (int)b->plans.size()) return fail(TC_E_VARIANT, "member out of range");
    if (b->split[member]) {                   // the split-FP8 form: its own launches
        if (variant) *variant = TC_VARIANT_FUSED;
        if (shape) *shape = -1;
        if (n_candidates) *n_candidates = 0;
        return TC_OK;
    }
    const Cand& cd = b->cands[member][b->choice[member]];
    if (variant) *variant = cd.variant;
    if (shape) *shape = cd.shape;
    if (n_candidates) *n_candidates = (int)b->cands[member].size();
    return TC_OK;
}

}  // extern "C"
