// Batches: many independent contractions in one HIP graph.
//
// tc_batch_create turns every contraction into matrix-core tiles of a chosen
// shape (128x128, 64x64 or 32x128 outputs), writes one static descriptor per
// contraction to device memory and builds work lists of (contraction, tile)
// pairs, one per (storage type, tile shape, operand layout) group, ordered
// longest-first by the estimated cost of a tile (contracted length x tile
// area).  tc_batch_create (and tc_batch_tune after a change of shapes)
// captures a graph: a staging kernel that copies the call's pointers and
// scalars from pinned host memory, a kernel that zeroes the work counters (no
// memset nodes), and one persistent kernel per group whose blocks take tiles
// off the group's counter, the groups spread over up to four graph branches.
// tc_batch_contract only writes the staging buffer and replays the graph.
//
// tc_batch_tune chooses each contraction's tile shape.  Seed: micro-benchmarks
// time one full wave of tiles for each shape and contracted-length bucket, and
// a contraction's estimate is its tile count times the per-tile share of that
// wave (cost composed from kernel micro-benchmarks, as in Section 3).  The
// top_k candidates by estimate are then timed on the device, one contraction
// at a time, and the fastest is kept; the share of contractions where the
// estimate's first choice was within 5% of the measured best is recorded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "launch.h"
#include "plan.h"

using namespace tc;

struct BatchGroup {
    bool f64;
    int shape;
    bool ak, bk;
    std::vector<int2> work;
    int2* d_work = nullptr;
    int grid = 1;
};

struct tc_batch_s {
    std::vector<tc_plan_s*> plans;
    std::vector<MfmaArgs> items;     // static descriptors (pointers filled per call)
    std::vector<int> shape;          // tile shape per contraction
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
    double hit_rate = -1.0;
    int n_tuned = 0;
};

namespace tc {

constexpr int BATCH_BK = 16;

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

// work lists per group, longest tiles first
static tc_status build_groups(tc_batch_s* b) {
    free_groups(b);
    std::map<int, int> gid;   // key -> group index
    std::vector<std::vector<std::pair<int64_t, int2>>> lists;
    int ncu = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    for (int c = 0; c < (int)b->items.size(); ++c) {
        MfmaArgs& a = b->items[c];
        const bool f64 = b->plans[c]->spec.dtype == TC_F64;
        const bool ak = mfma_kmajor_a(a), bk = mfma_kmajor_b(a);
        const int sh = b->shape[c];
        mfma_tiles_shape(sh, a);
        const int key = (f64 ? 16 : 0) | (sh << 2) | (ak ? 2 : 0) | (bk ? 1 : 0);   // sh in 0..3
        if (!gid.count(key)) {
            gid[key] = (int)b->groups.size();
            BatchGroup g;
            g.f64 = f64;
            g.shape = sh;
            g.ak = ak;
            g.bk = bk;
            b->groups.push_back(g);
            lists.emplace_back();
        }
        const int64_t cost = a.Kpad * (sh == 0 ? 128 * 128 : sh == 1 ? 64 * 64 : 32 * 128);
        for (int64_t t = 0; t < a.ntiles; ++t) lists[gid[key]].push_back({cost, int2{c, (int)t}});
    }
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        auto& L = lists[gi];
        std::stable_sort(L.begin(), L.end(), [](const std::pair<int64_t, int2>& x, const std::pair<int64_t, int2>& y) {
            return x.first > y.first;
        });
        BatchGroup& g = b->groups[gi];
        for (auto& e : L) g.work.push_back(e.second);
        hipError_t e = hipMalloc(&g.d_work, sizeof(int2) * std::max<size_t>(1, g.work.size()));
        if (e != hipSuccess) return fail(TC_E_NOMEM, "hipMalloc batch work list");
        e = hipMemcpy(g.d_work, g.work.data(), sizeof(int2) * g.work.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload batch work list");
        int occ = mfma_batch_occupancy(g.f64, g.shape, g.ak, g.bk);
        g.grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)g.work.size(), (int64_t)occ * ncu));
    }
    hipError_t e = hipMalloc(&b->d_counters, sizeof(int) * std::max<size_t>(1, b->groups.size()));
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
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, b->cap, b->d_counters, (int)b->groups.size());
    // the groups are independent: up to four branches of the graph, so that one
    // group's tail overlaps the next group's blocks
    const int nb = (int)std::min<size_t>(4, b->groups.size());
    if (nb > 1 && e == hipSuccess) e = hipEventRecord(b->fork, b->cap);
    for (int q = 1; q < nb && e == hipSuccess; ++q) e = hipStreamWaitEvent(b->side[q - 1], b->fork, 0);
    for (size_t gi = 0; gi < b->groups.size() && e == hipSuccess; ++gi) {
        BatchGroup& g = b->groups[gi];
        const int q = (int)(gi % nb);
        hipStream_t st = q == 0 ? b->cap : b->side[q - 1];
        hipError_t le = launch_mfma_batch(g.f64, g.shape, g.ak, g.bk, b->d_items, b->d_ptrs, g.d_work,
                                          (int)g.work.size(), b->d_counters + gi, g.grid, st);
        if (le != hipSuccess) e = le;
    }
    for (int q = 1; q < nb && e == hipSuccess; ++q) {
        e = hipEventRecord(b->join[q - 1], b->side[q - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->join[q - 1], 0);
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

constexpr int kShapes = 3;   // tile shapes 128x128, 64x64, 32x128

static int default_shape(const MfmaArgs& a) { return a.M <= 32 ? 2 : (a.M <= 64 || a.N <= 64) ? 1 : 0; }

}  // namespace tc

extern "C" {

tc_status tc_batch_create(tc_batch_t* out, const tc_plan_t* plans, int n) {
    if (!out) return fail(TC_E_NULL, "out is NULL");
    *out = nullptr;
    if (n < 0 || (n > 0 && !plans)) return fail(TC_E_NULL, "plans is NULL");
    tc_batch_s* b = new (std::nothrow) tc_batch_s();
    if (!b) return fail(TC_E_NOMEM, "host allocation");
    std::vector<int64_t> tab_all;
    std::vector<int64_t> tab_off;
    for (int c = 0; c < n; ++c) {
        tc_plan_s* p = plans[c];
        if (!p) {
            delete b;
            return fail(TC_E_NULL, "a plan is NULL");
        }
        if (p->spec.compute != TC_NATIVE) {
            delete b;
            return fail(TC_E_UNSUPPORTED, "batches run the native compute mode");
        }
        if (p->spec.is_complex()) {
            delete b;
            return fail(TC_E_UNSUPPORTED, "batches take real plans");
        }
        if (p->spec.nC == 0 || p->gv.K == 0) {
            delete b;
            return fail(TC_E_UNSUPPORTED, "batch members need a non-empty C and contracted extent");
        }
        const GemmView& gv = p->gv;
        std::vector<int64_t> tab = build_ktab(gv.k, BATCH_BK);
        tab_off.push_back((int64_t)tab_all.size());
        tab_all.insert(tab_all.end(), tab.begin(), tab.end());
        MfmaArgs a{};
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
        a.pass.n = 0;
        a.M = gv.M;
        a.N = gv.N;
        a.Kpad = (int64_t)tab.size() / 2;
        a.npass = 1;
        a.mode = 0;
        b->items.push_back(a);
        b->plans.push_back(p);
        b->shape.push_back(default_shape(a));
    }
    hipError_t e = hipMalloc(&b->d_ktab, sizeof(int64_t) * std::max<size_t>(1, tab_all.size()));
    if (e == hipSuccess && !tab_all.empty())
        e = hipMemcpy(b->d_ktab, tab_all.data(), sizeof(int64_t) * tab_all.size(), hipMemcpyHostToDevice);
    for (int c = 0; c < n; ++c) b->items[c].ktab = b->d_ktab + tab_off[c];
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
    tc_status st = build_groups(b);
    if (!st) st = capture(b);          // the graph reads the call's pointers from pinned staging
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
        const bool sw = b->plans[c]->gv.swapped;
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

// Tile-shape tuning (see the file comment).  Uses the operands of the previous
// tc_batch_contract call, which must have been made.
tc_status tc_batch_tune(tc_batch_t b, int top_k) {
    if (!b) return fail(TC_E_NULL, "batch is NULL");
    if (!b->launched) return fail(TC_E_UNSUPPORTED, "call tc_batch_contract once before tuning");
    if (top_k < 1) top_k = 1;
    hipError_t e = hipEventSynchronize(b->done);
    if (e != hipSuccess) return hip_fail(e, "synchronize");
    const int n = (int)b->items.size();
    hipStream_t st = b->cap;
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return fail(TC_E_HIP, "events");
    // Whole-batch time of the current configuration: graph replays with the
    // previous call's operands and beta = 0 (C := alpha * contract(A, B)).
    auto time_graph = [&](double* out) -> tc_status {
        for (int c = 0; c < n; ++c) b->h_ptrs[c].beta = 0.0;
        if (!b->exec) {
            tc_status cs = capture(b);
            if (cs) return cs;
        }
        hipError_t err = hipGraphLaunch(b->exec, st);   // warm-up
        if (err == hipSuccess) err = hipEventRecord(t0, st);
        for (int r = 0; r < 5 && err == hipSuccess; ++r) err = hipGraphLaunch(b->exec, st);
        if (err == hipSuccess) err = hipEventRecord(t1, st);
        if (err == hipSuccess) err = hipEventSynchronize(t1);
        float ms = 0;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, t0, t1);
        if (err != hipSuccess) return hip_fail(err, "batch timing replays");
        *out = ms / 5.0;
        return TC_OK;
    };
    double before_ms = 0.0;
    {
        tc_status ts = time_graph(&before_ms);
        if (ts) {
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            return ts;
        }
    }
    const std::vector<int> old_shape = b->shape;
    auto time_one = [&](int c, int sh, double* out) -> hipError_t {
        MfmaArgs a = b->items[c];
        a.A = b->h_ptrs[c].A;
        a.B = b->h_ptrs[c].B;
        a.C = b->h_ptrs[c].C;
        a.alpha = b->h_ptrs[c].alpha;
        a.beta = 0.0;
        mfma_tiles_shape(sh, a);
        const bool f64 = b->plans[c]->spec.dtype == TC_F64;
        std::vector<float> ts;
        for (int r = 0; r < 4; ++r) {
            hipError_t err = hipEventRecord(t0, st);
            if (err == hipSuccess) err = launch_mfma_shape(f64, sh, a, st);
            if (err == hipSuccess) err = hipEventRecord(t1, st);
            if (err == hipSuccess) err = hipEventSynchronize(t1);
            float ms = 0;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, t0, t1);
            if (err != hipSuccess) return err;
            if (r > 0) ts.push_back(ms);
        }
        std::sort(ts.begin(), ts.end());
        *out = ts[ts.size() / 2] * 1e-3;
        return hipSuccess;
    };
    // seed: per (storage, shape, K bucket) the time of one tile, measured on the
    // batch's own member with the most tiles in that bucket, divided by its tile
    // count (a wave's worth of tiles shares the device)
    std::map<std::string, double> tile_cost;
    auto bucket = [](int64_t kpad) {
        int bkt = 0;
        while ((16LL << bkt) < kpad && bkt < 12) ++bkt;
        return bkt;
    };
    std::map<std::string, std::pair<int64_t, int>> rep;   // key -> (tiles, member)
    for (int c = 0; c < n; ++c)
        for (int sh = 0; sh < kShapes; ++sh) {
            MfmaArgs a = b->items[c];
            mfma_tiles_shape(sh, a);
            std::string key = std::to_string(b->plans[c]->spec.dtype) + "/" + std::to_string(sh) + "/" +
                              std::to_string(bucket(a.Kpad));
            if (!rep.count(key) || rep[key].first < a.ntiles) rep[key] = {a.ntiles, c};
        }
    for (auto& kv : rep) {
        int sh = kv.first[2] - '0';
        double t;
        e = time_one(kv.second.second, sh, &t);
        if (e != hipSuccess) break;
        tile_cost[kv.first] = t / (double)std::max<int64_t>(1, kv.second.first);
    }
    int hits = 0;
    for (int c = 0; c < n && e == hipSuccess; ++c) {
        std::vector<std::pair<double, int>> cand;
        for (int sh = 0; sh < kShapes; ++sh) {
            MfmaArgs a = b->items[c];
            mfma_tiles_shape(sh, a);
            std::string key = std::to_string(b->plans[c]->spec.dtype) + "/" + std::to_string(sh) + "/" +
                              std::to_string(bucket(a.Kpad));
            cand.push_back({tile_cost[key] * (double)a.ntiles, sh});
        }
        std::sort(cand.begin(), cand.end());
        int seed_pick = cand[0].second;
        double best_t = INFINITY;
        int best = seed_pick;
        std::vector<double> meas(kShapes, INFINITY);
        for (int q = 0; q < (int)cand.size() && q < std::max(top_k, 2); ++q) {
            double t;
            e = time_one(c, cand[q].second, &t);
            if (e != hipSuccess) break;
            meas[cand[q].second] = t;
            if (q < top_k && t < best_t) {
                best_t = t;
                best = cand[q].second;
            }
        }
        double truly_best = *std::min_element(meas.begin(), meas.end());
        if (meas[seed_pick] <= 1.05 * truly_best) ++hits;
        b->shape[c] = best;
    }
    if (e != hipSuccess) {
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        return hip_fail(e, "tuning launches");
    }
    b->hit_rate = n ? (double)hits / n : 1.0;
    b->n_tuned = n;
    // Members timed alone favour small tiles (more parallelism on an idle
    // device); inside the batch that need not hold, so the whole batch is
    // timed with the new shapes and the previous ones are kept unless the new
    // ones are faster than both timings of the previous ones (replay times
    // drift by a few percent, as much as a change of shapes gains or loses).
    const std::vector<int> new_shape = b->shape;
    auto use = [&](const std::vector<int>& shp) {
        b->shape = shp;
        drop_graph(b);
        tc_status r = build_groups(b);
        return r ? r : capture(b);
    };
    tc_status ts = use(new_shape);
    double after_ms = 0.0;
    if (!ts) ts = time_graph(&after_ms);
    if (!ts && after_ms < before_ms) {
        double again_ms = 0.0;
        ts = use(old_shape);
        if (!ts) ts = time_graph(&again_ms);
        if (!ts && after_ms < again_ms) ts = use(new_shape);
    } else if (!ts) {
        ts = use(old_shape);
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return ts;
}

tc_status tc_batch_info(tc_batch_t b, int* n_members, int64_t* n_tiles, int* n_groups, double* tune_hit_rate) {
    if (!b) return fail(TC_E_NULL, "batch is NULL");
    int64_t tiles = 0;
    for (auto& g : b->groups) tiles += (int64_t)g.work.size();
    if (n_members) *n_members = (int)b->items.size();
    if (n_tiles) *n_tiles = tiles;
    if (n_groups) *n_groups = (int)b->groups.size();
    if (tune_hit_rate) *tune_hit_rate = b->hit_rate;
    return TC_OK;
}

}  // extern "C"
