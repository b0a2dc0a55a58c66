// The C ABI: plans, dispatch of tc_contract to the fused kernels or to a family
// member's launch sequence, and the host-only queries of the performance model.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "launch.h"
#include "plan.h"

using namespace tc;

namespace tc {
thread_local std::string g_last_error;

tc_status fail(tc_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

tc_status hip_fail(hipError_t e, const char* what) {
    return fail(TC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Blocked K order for the matrix-core kernels.  Tiles of BK contracted
// positions are rectangles, bA positions along the contracted index that is
// contiguous in A (dA) by BK / bA along the one contiguous in B (dB), so both
// operands read runs.  Blocks are walked with one of dA, dB fastest
// (`a_first`), in super-blocks of G blocks along each of them (G = 0: the
// whole extent), then the other contracted indices in order: an operand whose
// contiguous index walks fastest reuses each cache line on consecutive tiles,
// the other one every G tiles.  Positions are (offA, offB) pairs; a tile that
// is not full is padded with (-1, -1) entries (zero contributions).
std::vector<int64_t> build_ktab(const std::vector<GtDim>& kd, int BK, int bA, bool a_first, int G) {
    std::vector<int64_t> tab;
    int nd = (int)kd.size();
    int64_t K = 1;
    for (auto& d : kd) K *= d.ext;
    if (nd == 0 || K == 0) return tab;
    int dA = -1, dB = -1;
    for (int d = 0; d < nd; ++d) {
        if (dA < 0 && kd[d].sA == 1 && kd[d].ext > 1) dA = d;
        if (dB < 0 && kd[d].sB == 1 && kd[d].ext > 1) dB = d;
    }
    std::vector<int64_t> bs(nd, 1);
    if (dA >= 0 && dB >= 0 && dA != dB) {
        bs[dA] = std::min<int64_t>(kd[dA].ext, bA);
        bs[dB] = std::min<int64_t>(kd[dB].ext, BK / bs[dA]);
    } else {
        int d = dA >= 0 ? dA : dB >= 0 ? dB : 0;
        bs[d] = std::min<int64_t>(kd[d].ext, BK);
    }
    std::vector<int64_t> nblk(nd);
    for (int d = 0; d < nd; ++d) nblk[d] = (kd[d].ext + bs[d] - 1) / bs[d];
    // Walk digits: (dim, weight, range).  Block index along d = sum of its
    // digits times weights; a combination past nblk[d] is skipped.
    struct Digit { int d; int64_t w, n; };
    std::vector<Digit> dig;
    int f = a_first ? dA : dB, s = a_first ? dB : dA;
    if (s == f) s = -1;
    auto gsz = [&](int d) { return G > 0 ? std::min<int64_t>(G, nblk[d]) : nblk[d]; };
    if (f >= 0) dig.push_back({f, 1, gsz(f)});
    if (s >= 0) dig.push_back({s, 1, gsz(s)});
    if (f >= 0) dig.push_back({f, gsz(f), (nblk[f] + gsz(f) - 1) / gsz(f)});
    if (s >= 0) dig.push_back({s, gsz(s), (nblk[s] + gsz(s) - 1) / gsz(s)});
    for (int d = 0; d < nd; ++d)
        if (d != dA && d != dB) dig.push_back({d, 1, nblk[d]});
    // points inside a block: dA fastest, then dB, then the others
    std::vector<int> inner;
    if (dA >= 0) inner.push_back(dA);
    if (dB >= 0 && dB != dA) inner.push_back(dB);
    for (int d = 0; d < nd; ++d)
        if (d != dA && d != dB) inner.push_back(d);
    std::vector<int64_t> dv(dig.size(), 0), bi(nd);
    while (true) {
        std::fill(bi.begin(), bi.end(), 0);
        for (size_t q = 0; q < dig.size(); ++q) bi[dig[q].d] += dv[q] * dig[q].w;
        bool inside = true;
        for (int d = 0; d < nd; ++d)
            if (bi[d] >= nblk[d]) inside = false;
        if (inside) {
            std::vector<int64_t> li(nd, 0);
            int cnt = 0;
            while (true) {
                bool ok = true;
                int64_t oa = 0, ob = 0;
                for (int d = 0; d < nd; ++d) {
                    int64_t x = bi[d] * bs[d] + li[d];
                    if (x >= kd[d].ext) ok = false;
                    oa += x * kd[d].sA;
                    ob += x * kd[d].sB;
                }
                if (ok) {
                    tab.push_back(oa);
                    tab.push_back(ob);
                    ++cnt;
                }
                int q = 0;
                for (; q < (int)inner.size(); ++q) {
                    int d = inner[q];
                    if (++li[d] < bs[d]) break;
                    li[d] = 0;
                }
                if (q == (int)inner.size()) break;
            }
            for (; cnt % BK != 0 || cnt == 0; ++cnt) {
                tab.push_back(-1);
                tab.push_back(-1);
            }
        }
        size_t q = 0;
        for (; q < dig.size(); ++q) {
            if (++dv[q] < dig[q].n) break;
            dv[q] = 0;
        }
        if (q == dig.size()) break;
    }
    return tab;
}

// Bit t set when every run of v table positions starting at a multiple of v
// is, for operand t (0 = A, 1 = B), either all padding or v consecutive
// offsets starting at a multiple of v: the matrix-core kernels may then stage
// that operand's K-major tiles in 16-byte chunks.
int ktab_vec_flags(const std::vector<int64_t>& tab, int v) {
    const int64_t n = (int64_t)tab.size() / 2;
    if (n == 0 || n % v != 0) return 0;
    int flags = 0;
    for (int t = 0; t < 2; ++t) {
        bool ok = true;
        for (int64_t p = 0; ok && p < n; p += v) {
            const int64_t o0 = tab[2 * p + t];
            for (int j = 1; j < v && ok; ++j) {
                const int64_t o = tab[2 * (p + j) + t];
                ok = o0 < 0 ? o < 0 : o == o0 + j;
            }
            if (o0 >= 0 && o0 % v != 0) ok = false;
        }
        if (ok) flags |= 1 << t;
    }
    return flags;
}

}  // namespace tc

// ---------------------------------------------------------------------------
namespace tc {
static thread_local bool g_no_alloc = false;
bool allocation_forbidden() { return g_no_alloc; }
NoAllocScope::NoAllocScope() : saved(g_no_alloc) { g_no_alloc = true; }
NoAllocScope::~NoAllocScope() { g_no_alloc = saved; }
tc_status fail_unprepared() {
    return fail(TC_E_UNSUPPORTED, "the plan's device workspace for the selected variant is not allocated "
                                  "(no GPU was visible when the plan was built or the variant selected): "
                                  "call tc_plan_prepare");
}

bool device_visible() {
    static const bool visible = [] {
        int n = 0;
        return hipGetDeviceCount(&n) == hipSuccess && n > 0;
    }();
    return visible;
}

tc_status ensure_device_buffer(void** p, int64_t* cap, int64_t bytes) {
    if (bytes <= *cap) return TC_OK;
    if (g_no_alloc) return fail_unprepared();
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc(p, (size_t)std::max<int64_t>(bytes, 256));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(TC_E_NOMEM, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
    }
    *cap = std::max<int64_t>(bytes, 256);
    return TC_OK;
}
}  // namespace tc
using tc::ensure_device_buffer;

static tc_status upload(void** p, int64_t* cap, const std::vector<int64_t>& v) {
    if (allocation_forbidden()) return fail_unprepared();
    int64_t bytes = (int64_t)(v.size() * sizeof(int64_t));
    tc_status s = ensure_device_buffer(p, cap, bytes);
    if (s) return s;
    if (bytes) {
        hipError_t e = hipMemcpy(*p, v.data(), (size_t)bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy K table");
    }
    return TC_OK;
}

namespace tc {

StreamArgs stream_args(const GemmView& gv, bool f64) {
    StreamArgs a{};
    a.M = gv.m[0].ext;
    a.sAm = gv.m[0].sA;
    a.N = gv.N;
    a.n.n = (int)gv.n.size();
    for (int d = 0; d < a.n.n; ++d) a.n.d[d] = gv.n[d];
    // contracted positions in odometer order (first index fastest)
    a.K = (int)gv.K;
    std::vector<int64_t> idx(gv.k.size(), 0);
    for (int k = 0; k < a.K; ++k) {
        int64_t oa = 0, ob = 0;
        for (size_t d = 0; d < gv.k.size(); ++d) {
            oa += idx[d] * gv.k[d].sA;
            ob += idx[d] * gv.k[d].sB;
        }
        a.kA[k] = oa;
        a.kB[k] = ob;
        for (size_t d = 0; d < gv.k.size(); ++d) {
            if (++idx[d] < gv.k[d].ext) break;
            idx[d] = 0;
        }
    }
    stream_shape(f64, a);
    return a;
}

// The streaming kernel runs contractions whose C is unit-stride along one free
// index of an input, with at most 8 summed positions, or 9..16 where M is a
// whole number of wave spans with A unit-stride along it (the straight-line
// wave kernel then covers all of M).  Matrix-core tiles take the rest.
// Measured on MI355X: over 504 small-K contractions with M log-uniform in
// 8..256, the general streaming kernel took 2.3 ms against 4.1 ms for up to 8
// positions and 16.6 ms against 8.6 ms for 9..32; at a = b = c = 1024 the wave
// kernel took 2.49-2.61 ms against 3.33 ms for 12..16 positions (FP64) and
// 7.8-8.2 ms against 4.0 ms for 24..32 (FP32: 6.6-7.1 against 1.9).
bool use_stream_kernel(const Spec& s, const GemmView& gv) {
    if (gv.K < 1 || gv.K > 16 || gv.m.size() != 1 || gv.m[0].sC != 1 || !gv.b.empty()) return false;
    if (gv.K <= 8) return true;
    const int64_t span = 64 * (s.dtype == TC_F64 ? 2 : 4);
    return gv.m[0].sA == 1 && gv.M % span == 0;
}

tc_status prepare_plan(tc_plan_s* p) {
    if (p->real) return prepare_complex(p);
    const Spec& s = p->spec;
    bool f64 = s.dtype == TC_F64;
    int BK = mfma_bk(f64);
    if (p->selected == TC_VARIANT_FUSED || p->selected == TC_VARIANT_PREDICTED) {
        if (!use_stream_kernel(s, p->gv) && !p->ktab_ready) {
            std::vector<int64_t> tab = build_ktab(p->gv.k, BK, 4, mfma_a_first(f64, p->gv.M, p->gv.N, p->gv.K), 4);
            p->kpad = (int64_t)tab.size() / 2;
            p->kvec = ktab_vec_flags(tab, f64 ? 2 : 4);
            tc_status st = upload(&p->d_ktab, &p->ktab_cap, tab);
            if (st) return st;
            int64_t ws = 0;
            p->kslices = s.compute == TC_NATIVE && p->gv.b.empty()
                             ? mfma_split_plan(f64, p->gv.M, p->gv.N, p->kpad, &p->kslice_tiles, &ws)
                             : 1;
            if (p->kslices > 1) {
                st = ensure_device_buffer(&p->d_splitk, &p->splitk_cap, ws);
                if (st) return st;
            }
            p->ktab_ready = true;
        }
        if (s.compute != TC_NATIVE) {
            tc_status st = prepare_split(p);
            if (st) return st;
        }
    }
    if (p->selected == TC_VARIANT_PREDICTED && !p->have_prediction)
        return fail(TC_E_VARIANT, "the prediction behind TC_VARIANT_PREDICTED was cleared (root gaps changed): "
                                  "call tc_predict again or select a variant");
    int v = p->selected == TC_VARIANT_PREDICTED ? p->predicted_best : p->selected;
    if (v >= 0) {
        VariantPlan& vp = p->vplans()[v];
        if (vp.needs_c_copy)
            return fail(TC_E_UNSUPPORTED, "member copies C with a contracted loop at or outside the copy inside "
                                          "its free loops: not run on the GPU");
        for (int t = 0; t < 3; ++t) {
            tc_status st = ensure_device_buffer(&p->d_temp[t], &p->temp_cap[t], vp.temp_elems[t] * s.elem_bytes());
            if (st) return st;
        }
        if (vp.mfma && p->var_ktab_for != v) {
            std::vector<GtDim> kd;
            if (vp.body.kb.ext != 1 || vp.body.kb.sA != 0 || vp.body.kb.sB != 0) kd.push_back(vp.body.kb);
            else kd.push_back(GtDim{1, 0, 0, 0});
            std::vector<int64_t> tab = build_ktab(kd, BK);
            p->var_kpad = (int64_t)tab.size() / 2;
            p->var_kvec = ktab_vec_flags(tab, f64 ? 2 : 4);
            tc_status st = upload(&p->d_var_ktab, &p->var_ktab_cap, tab);
            if (st) return st;
            p->var_ktab_for = v;
        }
    }
    return TC_OK;
}

static const char* ptr_add(const void* p, int64_t elems, int esize) {
    return (const char*)p + elems * esize;
}

// The fused direct contraction on the streaming kernel (few summed positions;
// the K offsets travel in the launch arguments).  A and B in GEMM-view order.
tc_status launch_fused_stream(const tc_plan_s* p, const void* A, const void* B, void* C, double alpha, double beta,
                              hipStream_t st) {
    StreamArgs a = stream_args(p->gv, p->spec.dtype == TC_F64);
    a.A = A; a.B = B; a.C = C;
    a.alpha = alpha;
    a.beta = beta;
    hipError_t e = launch_stream(p->spec.dtype == TC_F64, a, st);
    return e == hipSuccess ? TC_OK : hip_fail(e, "stream kernel launch");
}

// The fused direct contraction on matrix-core tiles, with the K table and the
// split-K partial tiles given by the caller (the plan's workspace, or the
// no-allocation entry point's scratch).  A and B are in GEMM-view order.
tc_status launch_fused_mfma(const tc_plan_s* p, const void* A, const void* B, void* C, double alpha, double beta,
                            const int64_t* ktab, int64_t kpad, int kvec, void* ws, int64_t kslices,
                            int64_t kslice_tiles, hipStream_t st) {
    const GemmView& gv = p->gv;
    const bool f64 = p->spec.dtype == TC_F64;
    MfmaArgs a{};
    a.A = A; a.B = B; a.C = C;
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
    a.ktab = ktab;
    a.kvec = kvec;
    if (kslices > 1) {
        a.ws = ws;
        a.kslices = kslices;
        a.kslice_tiles = kslice_tiles;
    }
    a.M = gv.M; a.N = gv.N; a.Kpad = kpad;
    a.npass = 1;
    a.alpha = alpha; a.beta = beta;
    a.mode = 0;
    mfma_tiles(f64, a);
    hipError_t e = launch_mfma(f64, a, st);
    return e == hipSuccess ? TC_OK : hip_fail(e, "mfma kernel launch");
}

// The fused direct contraction: one launch (two with split K).
static tc_status run_fused(tc_plan_s* p, const void* A, const void* B, void* C, double alpha,
                           double beta, hipStream_t st) {
    const Spec& s = p->spec;
    const GemmView& gv = p->gv;
    if (gv.swapped) std::swap(A, B);
    if (s.compute != TC_NATIVE) return run_split(p, A, B, C, alpha, beta, st);
    if (use_stream_kernel(s, gv)) return launch_fused_stream(p, A, B, C, alpha, beta, st);
    return launch_fused_mfma(p, A, B, C, alpha, beta, (const int64_t*)p->d_ktab, p->kpad, p->kvec, p->d_splitk,
                             p->kslices, p->kslice_tiles, st);
}

tc_status run_variant(tc_plan_s* p, int v, const void* A, const void* B, void* C, double alpha,
                      double beta, hipStream_t st) {
    const Spec& s = p->spec;
    const VariantPlan& vp = p->vplans()[v];
    bool f64 = s.dtype == TC_F64;
    int es = s.elem_bytes();
    hipError_t e;
    // C := beta*C, then every invocation adds alpha*(kernel result)
    if (beta != 1.0) {
        ScaleArgs sa = scale_args(s, C, beta);
        e = launch_scale(f64, sa, st);
        if (e != hipSuccess) return hip_fail(e, "scale kernel launch");
    }
    const void* X[2] = {A, B};
    bool copied[2] = {false, false};
    for (auto& cs : vp.copies) copied[cs.tensor] = true;
    const int H = (int)vp.hoisted.size();
    std::vector<int64_t> h(H, 0);
    int64_t total_passes = 1;
    for (auto& d : vp.hoisted) total_passes *= d.ext;
    for (int64_t pass = 0; pass < total_passes; ++pass) {
        int64_t hA = 0, hB = 0, hC = 0;
        for (int q = 0; q < H; ++q) {
            hA += h[q] * vp.hoisted[q].sA;
            hB += h[q] * vp.hoisted[q].sB;
            hC += h[q] * vp.hoisted[q].sC;
        }
        for (auto& cs : vp.copies) {
            bool due = true;
            for (int q = cs.hoist_depth; q < H; ++q)
                if (h[q] != 0) due = false;
            if (!due) continue;
            int64_t src = 0;
            for (int q = 0; q < cs.hoist_depth; ++q)
                src += h[q] * (cs.tensor == 0 ? vp.hoisted[q].sA : vp.hoisted[q].sB);
            CopyArgs ca{};
            ca.src = ptr_add(X[cs.tensor], src, es);
            ca.dst = p->d_temp[cs.tensor];
            ca.dims = cs.dims;
            ca.total = cs.slice_elems * cs.slots;
            e = launch_copy(f64, ca, st);
            if (e != hipSuccess) return hip_fail(e, "copy kernel launch");
        }
        const void* a_ptr = copied[0] ? p->d_temp[0] : ptr_add(A, hA, es);
        const void* b_ptr = copied[1] ? p->d_temp[1] : ptr_add(B, hB, es);
        void* c_dst = (void*)ptr_add(C, hC, es);
        // C's slices into their temporary before the body, back after it
        for (auto& cs : vp.c_copies) {
            CopyArgs ca{};
            ca.src = c_dst;
            ca.dst = p->d_temp[2];
            ca.dims = cs.dims;
            ca.total = cs.slice_elems * cs.slots;
            e = launch_copy(f64, ca, st);
            if (e != hipSuccess) return hip_fail(e, "copy kernel launch (C in)");
        }
        void* c_ptr = vp.c_copies.empty() ? c_dst : p->d_temp[2];
        const GtDesc& d = vp.body;
        if (vp.mfma) {
            MfmaArgs a{};
            a.A = a_ptr; a.B = b_ptr; a.C = c_ptr;
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
            a.pass = d.pass;
            a.npass = 1;
            for (int q = 0; q < d.pass.n; ++q) a.npass *= d.pass.d[q].ext;
            a.ktab = (const int64_t*)p->d_var_ktab;
            a.M = d.nm ? d.out.d[0].ext : 1;
            a.N = d.nn ? d.out.d[d.nm].ext : 1;
            a.Kpad = p->var_kpad;
            a.kvec = p->var_kvec;
            a.alpha = alpha; a.beta = 1.0;
            a.mode = 1;
            mfma_tiles(f64, a);
            e = launch_mfma(f64, a, st);
            if (e != hipSuccess) return hip_fail(e, "mfma body launch");
        } else {
            SimtArgs a{};
            a.A = a_ptr; a.B = b_ptr; a.C = c_ptr;
            a.out = d.out;
            a.kb = d.kb;
            a.pass = d.pass;
            a.total = 1;
            for (int q = 0; q < d.out.n; ++q) a.total *= d.out.d[q].ext;
            a.npass = 1;
            for (int q = 0; q < d.pass.n; ++q) a.npass *= d.pass.d[q].ext;
            a.alpha = alpha;
            e = launch_simt(f64, a, st);
            if (e != hipSuccess) return hip_fail(e, "simt body launch");
        }
        for (auto& cs : vp.c_copies) {
            CopyArgs ca{};
            ca.src = p->d_temp[2];
            ca.dst = c_dst;
            ca.dims = cs.dims;
            for (int q = 0; q < ca.dims.n; ++q) std::swap(ca.dims.d[q].sA, ca.dims.d[q].sC);
            ca.total = cs.slice_elems * cs.slots;
            e = launch_copy(f64, ca, st);
            if (e != hipSuccess) return hip_fail(e, "copy kernel launch (C out)");
        }
        for (int q = H - 1; q >= 0; --q) {
            if (++h[q] < vp.hoisted[q].ext) break;
            h[q] = 0;
        }
    }
    return TC_OK;
}

tc_status contract_dispatch(tc_plan_s* p, const void* A, const void* B, void* C, double alpha, double beta,
                            hipStream_t st) {
    if (p->real) return run_complex(p, A, B, C, alpha, 0.0, beta, 0.0, st);
    const Spec& s = p->spec;
    bool f64 = s.dtype == TC_F64;
    int64_t K = 1;
    for (char ch : s.summed()) K *= s.e(ch);
    if (s.nC == 0) return TC_OK;
    if (alpha == 0.0 || K == 0) {
        if (beta == 1.0) return TC_OK;
        ScaleArgs sa = scale_args(s, C, beta);
        hipError_t e = launch_scale(f64, sa, st);
        return e == hipSuccess ? TC_OK : hip_fail(e, "scale kernel launch");
    }
    int v = p->selected == TC_VARIANT_PREDICTED ? p->predicted_best : p->selected;
    if (v < 0) return run_fused(p, A, B, C, alpha, beta, st);
    if (s.compute != TC_NATIVE) return fail(TC_E_UNSUPPORTED, "split precision runs in the fused kernel only");
    return run_variant(p, v, A, B, C, alpha, beta, st);
}

}  // namespace tc

namespace tc {
// Checks of a contraction call made before any device work: NULL pointers and
// aliasing of C with an input that is read.  Sets *runs to false when the call
// has nothing to compute (an empty C).
tc_status validate_call(const tc_plan_s* p, const void* A, const void* B, const void* C, double alpha_re,
                        double alpha_im, double beta_im, bool* runs) {
    if (!p) return fail(TC_E_NULL, "plan is NULL");
    const Spec& s = p->spec;
    if (!s.is_complex() && (alpha_im != 0.0 || beta_im != 0.0))
        return fail(TC_E_UNSUPPORTED, "complex alpha or beta on a real plan");
    int64_t K = 1;
    for (char ch : s.summed()) K *= s.e(ch);
    bool reads_inputs = (alpha_re != 0.0 || alpha_im != 0.0) && K > 0 && s.nC > 0;
    if (s.nC > 0 && !C) return fail(TC_E_NULL, "C is NULL");
    if (reads_inputs && ((s.nA > 0 && !A) || (s.nB > 0 && !B))) return fail(TC_E_NULL, "A or B is NULL");
    int es = s.elem_bytes();
    auto overlap = [&](const void* x, int64_t span_x, const void* y, int64_t span_y) {
        if (!x || !y || span_x == 0 || span_y == 0) return false;
        uintptr_t x0 = (uintptr_t)x, x1 = x0 + (uintptr_t)(span_x * es);
        uintptr_t y0 = (uintptr_t)y, y1 = y0 + (uintptr_t)(span_y * es);
        return x0 < y1 && y0 < x1;
    };
    if (reads_inputs && (overlap(C, s.spanC, A, s.spanA) || overlap(C, s.spanC, B, s.spanB)))
        return fail(TC_E_ALIAS, "C overlaps A or B");
    *runs = s.nC > 0;
    return TC_OK;
}
}  // namespace tc

// ===========================================================================
extern "C" {

tc_status tc_plan(tc_plan_t* out, const char* spec, const char* index_chars, const int64_t* extents,
                  int n_index, const int64_t* strides_A, const int64_t* strides_B,
                  const int64_t* strides_C, tc_dtype dtype, tc_compute compute) {
    if (!out) return fail(TC_E_NULL, "out is NULL");
    *out = nullptr;
    if (dtype != TC_F64 && dtype != TC_F32 && dtype != TC_C128 && dtype != TC_C64)
        return fail(TC_E_DTYPE, "dtype must be TC_F64, TC_F32, TC_C128 or TC_C64");
    if (compute != TC_NATIVE && compute != TC_BF16X3 && compute != TC_FP8X3)
        return fail(TC_E_DTYPE, "unknown compute mode");
    tc_plan_s* p = new (std::nothrow) tc_plan_s();
    if (!p) return fail(TC_E_NOMEM, "host allocation");
    Err err;
    p->spec.dtype = dtype;
    p->spec.compute = compute;
    if (parse_spec(spec, p->spec, err) ||
        bind_spec(p->spec, index_chars, extents, n_index, strides_A, strides_B, strides_C, err)) {
        delete p;
        return fail(err.st, err.msg);
    }
    if (compute != TC_NATIVE && p->spec.general()) {
        delete p;
        return fail(TC_E_UNSUPPORTED, "split precision needs contracted and free indices only");
    }
    if (p->spec.is_complex()) {
        tc_status st = build_complex(p);
        if (!st && device_visible()) st = prepare_plan(p);
        if (st) {
            tc_plan_destroy(p);
            return st;
        }
        *out = p;
        return TC_OK;
    }
    p->gv = gemm_view(p->spec);
    const GemmView& gv = p->gv;
    if ((int)gv.m.size() > GT_MAXD || (int)gv.n.size() > GT_MAXD || (int)gv.b.size() > GT_MAXD ||
        (int)gv.k.size() > GT_MAXD || (int)c_dims(p->spec).size() > GT_MAXD) {
        delete p;
        return fail(TC_E_UNSUPPORTED, "more than 8 dimension groups (after merging contiguous ones) "
                                      "in M, N, K, the batch indices or C");
    }
    if (device_visible()) {
        tc_status st = prepare_plan(p);
        if (st) {
            tc_plan_destroy(p);
            return st;
        }
    }
    *out = p;
    return TC_OK;
}

tc_status tc_plan_destroy(tc_plan_t p) {
    if (!p) return TC_OK;
    if (p->real) tc_plan_destroy(p->real);
    release_plan_device(p);
    delete p;
    return TC_OK;
}

tc_status tc_variant_count(tc_plan_t p, int* n) {
    if (!p || !n) return fail(TC_E_NULL, "NULL argument");
    *n = (int)p->fam().size();
    return TC_OK;
}

tc_status tc_variant_get(tc_plan_t p, int variant, tc_variant_info* out) {
    if (!p || !out) return fail(TC_E_NULL, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    if (variant == TC_VARIANT_FUSED) {
        std::snprintf(out->name, sizeof(out->name), "fused");
        out->number = 0;
        out->kernel = TC_KERNEL_FUSED;
        out->launches = 1;
        out->invocations = 1;
        out->runs_on_gpu = 1;
        return TC_OK;
    }
    if (variant < 0 || variant >= (int)p->fam().size()) return fail(TC_E_VARIANT, "variant out of range");
    const Variant& v = p->fam()[variant];
    std::snprintf(out->name, sizeof(out->name), "%s", v.name.c_str());
    out->number = v.number;
    out->kernel = v.kernel;
    std::snprintf(out->kept, sizeof(out->kept), "%s", v.kept.c_str());
    std::snprintf(out->loops, sizeof(out->loops), "%s", v.loops.c_str());
    out->n_copies = (int)std::min<size_t>(4, v.copies.size());
    for (int c = 0; c < out->n_copies; ++c) {
        out->copy_tensor[c] = "ABC"[v.copies[c].first];
        out->copy_level[c] = v.copies[c].second;
    }
    out->n_hoisted = v.n_hoisted;
    out->launches = p->vplans()[variant].launches;
    out->runs_on_gpu = p->vplans()[variant].needs_c_copy ? 0 : 1;
    int64_t inv = 1;
    for (char ch : v.loops) inv *= p->spec.e(ch);
    out->invocations = inv;
    return TC_OK;
}

tc_status tc_set_variant(tc_plan_t p, int variant) {
    if (!p) return fail(TC_E_NULL, "plan is NULL");
    if (variant == TC_VARIANT_PREDICTED) {
        if (p->predicted_best < -2 || !p->have_prediction)
            return fail(TC_E_VARIANT, "no prediction yet: call tc_predict first");
    } else if (variant != TC_VARIANT_FUSED && (variant < 0 || variant >= (int)p->fam().size())) {
        return fail(TC_E_VARIANT, "variant out of range");
    }
    if (variant >= 0 && p->spec.compute != TC_NATIVE)
        return fail(TC_E_UNSUPPORTED, "split precision runs in the fused kernel only");
    const int previous = p->selected;
    p->selected = variant;
    // a member that would copy C has no GPU schedule: tc_contract refuses it
    const bool runnable = variant < 0 || !p->vplans()[variant].needs_c_copy;
    if (runnable && device_visible()) {
        tc_status st = prepare_plan(p);
        if (st) {
            p->selected = previous;
            return st;
        }
    }
    return TC_OK;
}

tc_status tc_plan_prepare(tc_plan_t p) {
    if (!p) return fail(TC_E_NULL, "plan is NULL");
    return prepare_plan(p);
}

tc_status tc_plan_workspace(tc_plan_t p, int64_t* bytes) {
    if (!p || !bytes) return fail(TC_E_NULL, "NULL argument");
    *bytes = p->ktab_cap + p->var_ktab_cap + p->temp_cap[0] + p->temp_cap[1] + p->temp_cap[2] + p->split_bytes +
             p->splitk_cap +
             p->zexp_cap;
    if (p->real) {
        int64_t inner = 0;
        tc_plan_workspace(p->real, &inner);
        *bytes += inner;
    }
    return TC_OK;
}


static tc_status contract_entry(tc_plan_t p, const void* A, const void* B, void* C, double alpha_re,
                                double alpha_im, double beta_re, double beta_im, void* stream) {
    bool runs = false;
    tc_status st = validate_call(p, A, B, C, alpha_re, alpha_im, beta_im, &runs);
    if (st || !runs) return st;
    if (std::getenv("TC_FAULT") && std::strcmp(std::getenv("TC_FAULT"), "launch") == 0)
        return fail(TC_E_HIP, "injected launch failure (TC_FAULT=launch)");
    {
        NoAllocScope no_alloc;          // every buffer was allocated by tc_plan / tc_set_variant
        st = prepare_plan(p);
    }
    if (st) return st;
    if (p->real) return run_complex(p, A, B, C, alpha_re, alpha_im, beta_re, beta_im, (hipStream_t)stream);
    return contract_dispatch(p, A, B, C, alpha_re, beta_re, (hipStream_t)stream);
}

tc_status tc_contract(tc_plan_t p, const void* A, const void* B, void* C, double alpha, double beta,
                      void* stream) {
    return contract_entry(p, A, B, C, alpha, 0.0, beta, 0.0, stream);
}

tc_status tc_contract_complex(tc_plan_t p, const void* A, const void* B, void* C, double alpha_re,
                              double alpha_im, double beta_re, double beta_im, void* stream) {
    return contract_entry(p, A, B, C, alpha_re, alpha_im, beta_re, beta_im, stream);
}

tc_status tc_access_distance(tc_plan_t p, int variant, int tensor, int64_t* out) {
    if (!p || !out) return fail(TC_E_NULL, "NULL argument");
    if (variant < 0 || variant >= (int)p->fam().size()) return fail(TC_E_VARIANT, "variant out of range");
    if (tensor < 0 || tensor > 2) return fail(TC_E_VARIANT, "tensor must be 0, 1 or 2");
    *out = access_distance(p->spec, p->fam()[variant], tensor, -1, p->root_gap[tensor]);
    return TC_OK;
}

tc_status tc_bench_classes(tc_plan_t p, int variant, int stage, double cache_elems, int line_elems,
                           tc_bench_class* out, int capacity, int* n_out) {
    if (!p || !n_out) return fail(TC_E_NULL, "NULL argument");
    if (variant < 0 || variant >= (int)p->fam().size()) return fail(TC_E_VARIANT, "variant out of range");
    if (stage < 1 || stage > 5 || line_elems < 1 || !(cache_elems > 0))
        return fail(TC_E_UNSUPPORTED, "stage must be 1..5, line and cache positive");
    std::vector<BenchClass> cls =
        bench_classes(p->spec, p->fam()[variant], stage, cache_elems, line_elems, p->root_gap);
    *n_out = (int)cls.size();
    if ((int)cls.size() > capacity || (capacity > 0 && !out)) return fail(TC_E_CAPACITY, "capacity too small");
    for (size_t c = 0; c < cls.size(); ++c) {
        tc_bench_class& o = out[c];
        std::memset(&o, 0, sizeof(o));
        std::snprintf(o.label, sizeof(o.label), "%s", cls[c].label.c_str());
        o.weight = cls[c].weight;
        o.n_items = (int)std::min<size_t>(TC_MAX_SETUP, cls[c].setup.size());
        for (int k = 0; k < o.n_items; ++k) {
            o.items[k].kind = cls[c].setup[k].kind;
            o.items[k].tensor = cls[c].setup[k].tensor;
            o.items[k].size = cls[c].setup[k].size;
        }
    }
    return TC_OK;
}

tc_status tc_set_root_gap(tc_plan_t p, const int64_t* gap) {
    if (!p) return fail(TC_E_NULL, "plan is NULL");
    for (int t = 0; t < 3; ++t)
        if (gap && gap[t] < 0) return fail(TC_E_EXTENT, "root gaps must be >= 0");
    for (int t = 0; t < 3; ++t) p->root_gap[t] = gap ? gap[t] : 0;
    p->have_prediction = false;     // an earlier prediction assumed other gaps
    return TC_OK;
}

tc_status tc_chain_root_gaps(const tc_plan_t* plans, const int* ids, int n) {
    if (n < 0 || (n > 0 && (!plans || !ids))) return fail(TC_E_NULL, "plans or ids is NULL");
    for (int j = 0; j < n; ++j)
        if (!plans[j]) return fail(TC_E_NULL, "a plan is NULL");
    // bytes of every tensor id (the largest operand that names it)
    std::map<int, int64_t> bytes;
    for (int j = 0; j < n; ++j) {
        const Spec& s = plans[j]->spec;
        const int64_t cnt[3] = {s.nA, s.nB, s.nC};
        for (int t = 0; t < 3; ++t) {
            int64_t b = cnt[t] * s.elem_bytes();
            int64_t& have = bytes[ids[3 * j + t]];
            have = std::max(have, b);
        }
    }
    auto uses = [&](int k, int id) { return ids[3 * k] == id || ids[3 * k + 1] == id || ids[3 * k + 2] == id; };
    for (int j = 0; j < n; ++j) {
        int64_t gap[3];
        for (int t = 0; t < 3; ++t) {
            const int id = ids[3 * j + t];
            std::set<int> seen;   // tensors the contractions run since `id` was last used access
            for (int back = 1; back <= n; ++back) {
                const int k = ((j - back) % n + n) % n;
                if (k == j || uses(k, id)) break;
                for (int q = 0; q < 3; ++q) seen.insert(ids[3 * k + q]);
            }
            int64_t b = 0;
            for (int x : seen)
                if (!uses(j, x)) b += bytes[x];
            gap[t] = b / plans[j]->spec.elem_bytes();
        }
        tc_status st = tc_set_root_gap(plans[j], gap);
        if (st) return st;
    }
    return TC_OK;
}

const char* tc_status_str(tc_status s) {
    switch (s) {
        case TC_OK: return "TC_OK";
        case TC_E_SPEC: return "TC_E_SPEC";
        case TC_E_EXTENT: return "TC_E_EXTENT";
        case TC_E_STRIDE: return "TC_E_STRIDE";
        case TC_E_DTYPE: return "TC_E_DTYPE";
        case TC_E_ALIAS: return "TC_E_ALIAS";
        case TC_E_NULL: return "TC_E_NULL";
        case TC_E_VARIANT: return "TC_E_VARIANT";
        case TC_E_HIP: return "TC_E_HIP";
        case TC_E_NOMEM: return "TC_E_NOMEM";
        case TC_E_UNSUPPORTED: return "TC_E_UNSUPPORTED";
        case TC_E_CAPACITY: return "TC_E_CAPACITY";
    }
    return "TC_E_UNKNOWN";
}

const char* tc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
