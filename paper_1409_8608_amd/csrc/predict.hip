// Measured half of the performance model (Section 3): micro-benchmarks of one
// family member's kernel under the cache precondition of each benchmark class,
// composed into a predicted run time.
//
// Reading for the GPU.  A member's kernel invocations run many at a time, so a
// micro-benchmark times one launch of the member's body over a SAMPLE of its
// invocations (the first ones in schedule order, enough to fill the device:
// about 2^19 outputs worth for one-thread-per-output bodies, 2^25 for
// matrix-core bodies, or the whole launch if smaller), preceded by the class's
// setup list: operand
// regions are touched in list order and every remote region is a distinct
// piece of a scratch buffer, so after the setup the caches hold what the
// setup list says.  Ten repetitions, median (Sections 3.1, 3.2).  A class's
// time is the median scaled from the sample's invocations to the class's
// share of all invocations (Sections 3.4, 3.5); the classes are summed.  The
// member's copy launches and the C := beta*C launch are timed the same way (one
// launch each, scaled by their count).  Cache parameters: the 256 MB
// last-level (Infinity) cache, 128-byte lines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "launch.h"
#include "plan.h"

namespace tc {

static const double kCacheBytes = 256.0 * 1024 * 1024;
static const int kLineBytes = 128;
static const int kReps = 10;

struct PredCtx {
    tc_plan_s* p;
    void* A = nullptr;
    void* B = nullptr;
    void* C = nullptr;
    void* scratch = nullptr;
    int64_t scratch_bytes = 0;
    float* sink = nullptr;
    hipStream_t st = nullptr;
    std::map<std::string, double> cache;   // benchmark key -> median seconds
    int n_measured = 0;
};

static tc_status dev_alloc(void** p, int64_t bytes) {
    hipError_t e = hipMalloc(p, (size_t)std::max<int64_t>(bytes, 256));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(TC_E_NOMEM, std::string("hipMalloc (prediction buffers): ") + hipGetErrorString(e));
    }
    e = hipMemset(*p, 0, (size_t)std::max<int64_t>(bytes, 256));
    return e == hipSuccess ? TC_OK : hip_fail(e, "hipMemset");
}

// Sample of a member's body launch: the body's own dimensions stay whole, the
// parallel loops are cut (innermost first) to about `target` outputs.  Returns
// the fraction of one launch's invocations the sample covers.
static double sample_desc(const VariantPlan& vp, GtDesc& d, int64_t target) {
    d = vp.body;
    // leading out dims that belong to the kernel call itself
    const int nk = vp.mfma ? d.nm + d.nn : vp.n_body_dims;
    int64_t per_inv = 1;
    for (int q = 0; q < nk; ++q) per_inv *= d.out.d[q].ext;
    int64_t inv_total = 1;
    for (int q = nk; q < d.out.n; ++q) inv_total *= d.out.d[q].ext;
    const int64_t want = std::max<int64_t>(1, target / std::max<int64_t>(1, per_inv));
    int64_t inv = 1;
    for (int q = nk; q < d.out.n; ++q) {
        const int64_t e = d.out.d[q].ext;
        if (inv * e <= want) {
            inv *= e;
        } else {
            const int64_t keep = std::max<int64_t>(1, want / inv);
            d.out.d[q].ext = keep;
            inv *= keep;
            for (int r = q + 1; r < d.out.n; ++r) d.out.d[r].ext = 1;
            break;
        }
    }
    return inv_total > 0 ? (double)inv / (double)inv_total : 1.0;
}

static hipError_t launch_body(PredCtx& c, const VariantPlan& vp, const GtDesc& d, const void* A, const void* B) {
    tc_plan_s* p = c.p;
    bool f64 = p->spec.dtype == TC_F64;
    // a member that copies C runs its body on C's temporary
    void* Cb = vp.c_copies.empty() ? c.C : p->d_temp[2];
    if (vp.mfma) {
        MfmaArgs a{};
        a.A = A; a.B = B; a.C = Cb;
        a.m.n = d.nm;
        if (d.nm) a.m.d[0] = d.out.d[0];
        a.n.n = d.nn;
        if (d.nn) a.n.d[0] = d.out.d[d.nm];
        a.nbatch = 1;
        for (int q = d.nm + d.nn; q < d.out.n; ++q) {
            a.batch.d[a.batch.n++] = d.out.d[q];
            a.nbatch *= d.out.d[q].ext;
        }
        a.pass = d.pass;
        a.npass = 1;
        for (int q = 0; q < d.pass.n; ++q) a.npass *= d.pass.d[q].ext;
        a.ktab = (const int64_t*)p->d_var_ktab;
        a.M = d.nm ? d.out.d[0].ext : 1;
        a.N = d.nn ? d.out.d[d.nm].ext : 1;
        a.Kpad = p->var_kpad;
        a.kvec = p->var_kvec;
        a.alpha = 1.0; a.beta = 1.0;
        a.mode = 1;
        mfma_tiles(f64, a);
        return launch_mfma(f64, a, c.st);
    }
    SimtArgs a{};
    a.A = A; a.B = B; a.C = Cb;
    a.out = d.out;
    a.kb = d.kb;
    a.pass = d.pass;
    a.total = 1;
    for (int q = 0; q < d.out.n; ++q) a.total *= d.out.d[q].ext;
    a.npass = 1;
    for (int q = 0; q < d.pass.n; ++q) a.npass *= d.pass.d[q].ext;
    a.alpha = 1.0;
    return launch_simt(f64, a, c.st);
}

// setup list -> touch launches (operands at their base, remote regions from
// consecutive pieces of the scratch buffer)
static hipError_t run_setup(PredCtx& c, const std::vector<SetupItem>& setup, const void* opA, const void* opB) {
    int es = c.p->spec.elem_bytes();
    int64_t roff = 0;
    for (const SetupItem& it : setup) {
        int64_t bytes = it.size * es;
        const void* ptr;
        if (it.kind == 0) {
            ptr = it.tensor == 0 ? opA : it.tensor == 1 ? opB : c.C;
            int64_t span = (it.tensor == 0 ? c.p->spec.spanA : it.tensor == 1 ? c.p->spec.spanB : c.p->spec.spanC) * es;
            bytes = std::min(bytes, std::max<int64_t>(span, 16));
        } else {
            bytes = std::min(bytes, c.scratch_bytes);
            if (roff + bytes > c.scratch_bytes) roff = 0;
            ptr = (const char*)c.scratch + roff;
            roff += (bytes + 255) / 256 * 256;
        }
        hipError_t e = launch_touch(ptr, bytes, c.sink, c.st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// median over kReps of {setup; timed launch}
template <typename F>
static tc_status time_median(PredCtx& c, const std::vector<SetupItem>& setup, const void* opA, const void* opB,
                             F launch, double* out) {
    std::vector<hipEvent_t> ev(2 * (kReps + 1));
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(TC_E_HIP, "hipEventCreate");
    hipError_t err = hipSuccess;
    for (int r = 0; r <= kReps && err == hipSuccess; ++r) {   // r = 0 warms up
        err = run_setup(c, setup, opA, opB);
        if (err == hipSuccess) err = hipEventRecord(ev[2 * r], c.st);
        if (err == hipSuccess) err = launch();
        if (err == hipSuccess) err = hipEventRecord(ev[2 * r + 1], c.st);
    }
    if (err == hipSuccess) err = hipStreamSynchronize(c.st);
    std::vector<double> t;
    for (int r = 1; r <= kReps && err == hipSuccess; ++r) {
        float ms = 0;
        err = hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]);
        t.push_back(ms * 1e-3);
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (err != hipSuccess) return hip_fail(err, "micro-benchmark");
    std::sort(t.begin(), t.end());
    *out = 0.5 * (t[kReps / 2 - 1] + t[kReps / 2]);
    ++c.n_measured;
    return TC_OK;
}

static std::string key_of(int v, const GtDesc& d, const std::vector<SetupItem>& setup, bool mfma) {
    std::string k = std::to_string(mfma) + "|" + std::to_string(d.out.n) + ":";
    for (int q = 0; q < d.out.n; ++q)
        k += std::to_string(d.out.d[q].ext) + "," + std::to_string(d.out.d[q].sA) + "," +
             std::to_string(d.out.d[q].sB) + "," + std::to_string(d.out.d[q].sC) + ";";
    k += "|" + std::to_string(d.kb.ext) + "," + std::to_string(d.kb.sA) + "," + std::to_string(d.kb.sB);
    k += "|";
    for (int q = 0; q < d.pass.n; ++q)
        k += std::to_string(d.pass.d[q].ext) + "," + std::to_string(d.pass.d[q].sA) + "," +
             std::to_string(d.pass.d[q].sB) + ";";
    k += "|";
    for (auto& it : setup) k += std::to_string(it.kind) + "," + std::to_string(it.tensor) + "," + std::to_string(it.size) + ";";
    (void)v;
    return k;
}

static tc_status predict_variant(PredCtx& c, int v, tc_prediction* out) {
    tc_plan_s* p = c.p;
    const Spec& s = p->spec;
    const Variant& var = p->fam()[v];
    VariantPlan& vp = p->vplans()[v];
    auto t0 = std::chrono::steady_clock::now();
    int measured0 = c.n_measured;
    std::memset(out, 0, sizeof(*out));
    out->variant = v;
    if (vp.needs_c_copy) {
        for (int st = 0; st < 5; ++st) out->stage_s[st] = INFINITY;
        out->predicted_s = INFINITY;
        return TC_OK;
    }
    // workspace of this member (copy temporaries, K table of a gemm body)
    int saved = p->selected;
    p->selected = v;
    tc_status stt = prepare_plan(p);
    p->selected = saved;
    if (stt) return stt;
    bool copied[2] = {false, false};
    for (auto& cs : vp.copies) copied[cs.tensor] = true;
    const void* opA = copied[0] ? p->d_temp[0] : c.A;
    const void* opB = copied[1] ? p->d_temp[1] : c.B;

    GtDesc d;
    // The sample must fill the device, or scaling it up overstates the time:
    // 2^19 outputs are 2048 blocks of the one-thread-per-output bodies, and
    // 2^25 outputs about 2048 tiles of 128 x 128 for matrix-core bodies.
    const int64_t target = vp.mfma ? ((int64_t)1 << 25) : ((int64_t)1 << 19);
    double frac = sample_desc(vp, d, target);
    int64_t hoisted = 1;
    for (auto& h : vp.hoisted) hoisted *= h.ext;
    // sample share of all invocations
    const double launches_equiv = (double)hoisted / frac;   // sample -> whole member

    // fixed costs: copies (one launch each per pass group) and the beta prologue
    double fixed = 0.0;
    bool f64 = s.dtype == TC_F64;
    for (auto& cs : vp.copies) {
        int64_t n = 1;
        for (int q = 0; q < cs.hoist_depth; ++q) n *= vp.hoisted[q].ext;
        std::string key = "copy|" + std::to_string(cs.tensor) + "|" + std::to_string(cs.slice_elems) + "|" +
                          std::to_string(cs.slots);
        for (int q = 0; q < cs.dims.n; ++q)
            key += "," + std::to_string(cs.dims.d[q].ext) + ":" + std::to_string(cs.dims.d[q].sA);
        double t;
        auto it = c.cache.find(key);
        if (it != c.cache.end()) {
            t = it->second;
        } else {
            CopyArgs ca{};
            ca.src = cs.tensor == 0 ? c.A : c.B;
            ca.dst = p->d_temp[cs.tensor];
            ca.dims = cs.dims;
            ca.total = cs.slice_elems * cs.slots;
            stt = time_median(c, {}, opA, opB, [&]() { return launch_copy(f64, ca, c.st); }, &t);
            if (stt) return stt;
            c.cache[key] = t;
        }
        fixed += t * (double)n;
    }
    // C's copies in and out around every body launch (one of each per pass)
    for (auto& cs : vp.c_copies) {
        std::string key = "ccopy|" + std::to_string(cs.slice_elems) + "|" + std::to_string(cs.slots);
        for (int q = 0; q < cs.dims.n; ++q)
            key += "," + std::to_string(cs.dims.d[q].ext) + ":" + std::to_string(cs.dims.d[q].sA);
        double t;
        auto it = c.cache.find(key);
        if (it != c.cache.end()) {
            t = it->second;
        } else {
            CopyArgs ca{};
            ca.src = c.C;
            ca.dst = p->d_temp[2];
            ca.dims = cs.dims;
            ca.total = cs.slice_elems * cs.slots;
            stt = time_median(c, {}, opA, opB, [&]() { return launch_copy(f64, ca, c.st); }, &t);
            if (stt) return stt;
            c.cache[key] = t;
        }
        int64_t passes = 1;
        for (auto& h : vp.hoisted) passes *= h.ext;
        fixed += 2.0 * t * (double)passes;
    }
    {
        std::string key = "scale";
        double t;
        auto it = c.cache.find(key);
        if (it != c.cache.end()) {
            t = it->second;
        } else {
            ScaleArgs sa = scale_args(s, c.C, 0.0);
            stt = time_median(c, {}, opA, opB, [&]() { return launch_scale(f64, sa, c.st); }, &t);
            if (stt) return stt;
            c.cache[key] = t;
        }
        fixed += t;
    }

    const double cache_elems = kCacheBytes / s.elem_bytes();
    const int line_elems = kLineBytes / s.elem_bytes();
    for (int stage = 1; stage <= 5; ++stage) {
        std::vector<BenchClass> cls = bench_classes(s, var, stage, cache_elems, line_elems, p->root_gap);
        double total = fixed;
        for (const BenchClass& bc : cls) {
            if (bc.weight <= 0) continue;
            std::string key = key_of(v, d, bc.setup, vp.mfma);
            double t;
            auto it = c.cache.find(key);
            if (it != c.cache.end()) {
                t = it->second;
            } else {
                stt = time_median(c, bc.setup, opA, opB, [&]() { return launch_body(c, vp, d, opA, opB); }, &t);
                if (stt) return stt;
                c.cache[key] = t;
            }
            total += bc.weight * t * launches_equiv;
        }
        out->stage_s[stage - 1] = total;
    }
    out->predicted_s = out->stage_s[4];
    out->n_bench = c.n_measured - measured0;
    out->bench_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return TC_OK;
}

// The fused kernel is one launch, not a loop nest of calls: its "prediction"
// is its own median over ten launches.
static tc_status predict_fused(PredCtx& c, tc_prediction* out) {
    tc_plan_s* p = c.p;
    std::memset(out, 0, sizeof(*out));
    out->variant = TC_VARIANT_FUSED;
    auto t0 = std::chrono::steady_clock::now();
    int saved = p->selected;
    p->selected = TC_VARIANT_FUSED;
    tc_status stt = prepare_plan(p);
    if (!stt) {
        double t;
        stt = time_median(c, {}, c.A, c.B, [&]() -> hipError_t {
            tc_status r = contract_dispatch(p, c.A, c.B, c.C, 1.0, 0.0, c.st);
            return r == TC_OK ? hipSuccess : hipErrorLaunchFailure;
        }, &t);
        if (!stt)
            for (int s = 0; s < 5; ++s) out->stage_s[s] = t;
        out->predicted_s = stt ? INFINITY : t;
    }
    p->selected = saved;
    out->n_bench = 1;
    out->bench_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return stt;
}

}  // namespace tc

extern "C" tc_status tc_predict(tc_plan_t p, tc_prediction* out, int capacity, int* n_out) {
    using namespace tc;
    if (!p || !n_out) return fail(TC_E_NULL, "NULL argument");
    const int count = (int)p->fam().size() + 1;
    *n_out = count;
    if (capacity < count || !out) return fail(TC_E_CAPACITY, "capacity too small");
    if (p->spec.compute != TC_NATIVE) return fail(TC_E_UNSUPPORTED, "prediction covers the native compute mode");
    if (p->spec.nC == 0) return fail(TC_E_UNSUPPORTED, "empty contraction");
    PredCtx c;
    c.p = p;
    int es = p->spec.elem_bytes();
    tc_status st = TC_OK;
    if (!st) st = dev_alloc(&c.A, std::max<int64_t>(1, p->spec.spanA) * es);
    if (!st) st = dev_alloc(&c.B, std::max<int64_t>(1, p->spec.spanB) * es);
    if (!st) st = dev_alloc(&c.C, std::max<int64_t>(1, p->spec.spanC) * es);
    c.scratch_bytes = (int64_t)(1.25 * kCacheBytes) + (1 << 20);
    if (!st) st = dev_alloc(&c.scratch, c.scratch_bytes);
    if (!st) st = dev_alloc((void**)&c.sink, 256);
    if (!st && hipStreamCreate(&c.st) != hipSuccess) st = fail(TC_E_HIP, "hipStreamCreate");
    int best = -1;
    double best_t = INFINITY;
    for (int v = 0; v < (int)p->fam().size() && !st; ++v) {
        st = predict_variant(c, v, &out[v]);
        if (!st && out[v].predicted_s < best_t) {
            best_t = out[v].predicted_s;
            best = v;
        }
    }
    if (!st) st = predict_fused(c, &out[count - 1]);
    if (!st) {
        if (out[count - 1].predicted_s < best_t) best = TC_VARIANT_FUSED;
        p->predicted_best = best;
        p->have_prediction = true;
        // a plan that selects the predicted member gets that member's workspace now
        if (p->selected == TC_VARIANT_PREDICTED) st = prepare_plan(p);
    }
    if (c.st) (void)hipStreamDestroy(c.st);
    for (void* b : {c.A, c.B, c.C, c.scratch, (void*)c.sink})
        if (b) (void)hipFree(b);
    return st;
}
