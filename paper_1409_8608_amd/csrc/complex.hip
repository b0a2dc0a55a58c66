// Complex contractions (storage TC_C128 / TC_C64) run as real contractions on
// an embedded form.
//
// With a complex number stored as the pair (re, im), the product x y is the
// real matrix-vector product
//     [ (xy)_re ]   [ y_re  -y_im ] [ x_re ]
//     [ (xy)_im ] = [ y_im   y_re ] [ x_im ]
// so once one operand (Y) is written out as those 2x2 blocks, the complex sum
// of Section 1 over the summed indices is a real contraction with two more
// indices: a summed one running over the re/im pair of the other operand (X,
// unit stride in X's own storage) and a free one running over the re/im pair
// of C (unit stride in C).  X and C are read in place with their strides
// doubled (in reals); Y -- the operand with fewer elements -- is expanded once
// per call into plan workspace with alpha folded in.  Every real kernel
// (streaming, matrix core, split K) then applies unchanged, and the flop count
// is that of the complex sum: four real products per complex one.
#include <algorithm>
#include <cstring>
#include <string>

#include "plan.h"

namespace tc {

static bool has(const std::string& s, char ch) { return s.find(ch) != std::string::npos; }

static int64_t grid_for(int64_t n, int64_t cap) {
    return std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

template <typename T>
__global__ __launch_bounds__(256) void k_zexpand(ZExpandArgs a) {
    const T* __restrict__ src = (const T*)a.src;
    T* __restrict__ dst = (T*)a.dst;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.total; idx += stride) {
        int64_t rem = idx, os = 0, od = 0;
        for (int d = 0; d < a.dims.n; ++d) {
            const int64_t q = rem % a.dims.d[d].ext;
            rem /= a.dims.d[d].ext;
            os += q * a.dims.d[d].sA;
            od += q * a.dims.d[d].sC;
        }
        const double yr = (double)src[2 * os], yi = (double)src[2 * os + 1];
        double tr = a.alpha_re * yr, ti = a.alpha_re * yi;
        if (a.alpha_im != 0.0) {
            tr -= a.alpha_im * yi;
            ti += a.alpha_im * yr;
        }
        dst[od] = (T)tr;
        dst[od + a.s_in] = (T)-ti;
        dst[od + a.s_out] = (T)ti;
        dst[od + a.s_in + a.s_out] = (T)tr;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zscale(ZScaleArgs a) {
    T* __restrict__ C = (T*)a.C;
    const T br = (T)a.beta_re, bi = (T)a.beta_im;
    const bool zero = a.beta_re == 0.0 && a.beta_im == 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.total; idx += stride) {
        int64_t rem = idx, oc = 0;
        for (int d = 0; d < a.dims.n; ++d) {
            oc += (rem % a.dims.d[d].ext) * a.dims.d[d].sC;
            rem /= a.dims.d[d].ext;
        }
        T re = 0, im = 0;
        if (!zero) {
            const T cr = C[2 * oc], ci = C[2 * oc + 1];
            re = br * cr - bi * ci;
            im = br * ci + bi * cr;
        }
        C[2 * oc] = re;
        C[2 * oc + 1] = im;
    }
}

// ---------------------------------------------------------------------------
tc_status build_complex(tc_plan_s* p) {
    const Spec& s = p->spec;
    for (const std::string* op : {&s.a, &s.b, &s.c})
        if (op->size() >= 16) return fail(TC_E_UNSUPPORTED, "complex plans take at most 15 indices per operand");
    // two letters the spec does not use: zi runs over X's re/im pair, zo over C's
    char zi = 0, zo = 0;
    for (char ch = 'a'; ch <= 'z' && !zo; ++ch) {
        if (has(s.base, ch)) continue;
        if (!zi) zi = ch;
        else zo = ch;
    }
    if (!zo) return fail(TC_E_UNSUPPORTED, "a complex plan needs two index letters its spec does not use");

    const int y = s.nA <= s.nB ? 0 : 1;   // the expanded operand
    const std::string& ylet = s.letters(y);
    const std::string& xlet = s.letters(1 - y);
    // Y's layout in workspace: Y's own index order with zo in front of its first
    // index of C and zi in front of its first contracted index, so that the two
    // new indices sit where they continue the original layout
    std::string yexp;
    bool put_o = false, put_i = false;
    for (char ch : ylet) {
        if (!put_o && has(s.c, ch)) { yexp += zo; put_o = true; }
        if (!put_i && has(s.contracted, ch)) { yexp += zi; put_i = true; }
        yexp += ch;
    }
    if (!put_i) yexp = std::string(1, zi) + yexp;
    if (!put_o) yexp = std::string(1, zo) + yexp;

    auto ext = [&](char ch) -> int64_t { return ch == zi || ch == zo ? 2 : s.e(ch); };
    int64_t st_exp[26] = {0};
    int64_t run = 1;
    for (char ch : yexp) {
        st_exp[ch - 'a'] = run;
        run *= ext(ch);
    }
    std::vector<int64_t> stY, stX, stC;
    for (char ch : yexp) stY.push_back(st_exp[ch - 'a']);
    stX.push_back(1);
    for (char ch : xlet) stX.push_back(2 * s.stride(1 - y, ch));
    stC.push_back(1);
    // an empty C has zero Fortran strides after its zero extent; it is never
    // written, and the real plan wants positive C strides
    for (char ch : s.c) stC.push_back(std::max<int64_t>(1, 2 * s.stride(2, ch)));

    const std::string xexp = std::string(1, zi) + xlet;
    const std::string cexp = std::string(1, zo) + s.c;
    const std::string spec = cexp + "=" + (y == 0 ? yexp + "," + xexp : xexp + "," + yexp);
    std::string chars = s.base;
    chars += zi;
    chars += zo;
    std::vector<int64_t> exts;
    for (char ch : chars) exts.push_back(ext(ch));
    const tc_dtype rdt = s.dtype == TC_C128 ? TC_F64 : TC_F32;
    tc_status st = tc_plan(&p->real, spec.c_str(), chars.c_str(), exts.data(), (int)chars.size(),
                           y == 0 ? stY.data() : stX.data(), y == 0 ? stX.data() : stY.data(), stC.data(), rdt,
                           TC_NATIVE);
    if (st) return st;

    std::vector<GtDim> g;
    for (char ch : ylet) g.push_back(GtDim{s.e(ch), s.stride(y, ch), 0, st_exp[ch - 'a']});
    merge_group(g);
    if ((int)g.size() > GT_MAXD) return fail(TC_E_UNSUPPORTED, "more than 8 dimension groups in an operand");
    p->zdims.n = (int)g.size();
    for (size_t d = 0; d < g.size(); ++d) p->zdims.d[d] = g[d];
    p->zside = y;
    p->zelems = y == 0 ? s.nA : s.nB;
    p->zs_in = st_exp[zi - 'a'];
    p->zs_out = st_exp[zo - 'a'];
    return TC_OK;
}

tc_status prepare_complex(tc_plan_s* p) {
    const int rb = p->spec.dtype == TC_C128 ? 8 : 4;
    tc_status st = ensure_device_buffer(&p->d_zexp, &p->zexp_cap, 4 * p->zelems * rb);
    if (st) return st;
    return prepare_plan(p->real);
}

tc_status run_complex(tc_plan_s* p, const void* A, const void* B, void* C, double alpha_re, double alpha_im,
                      double beta_re, double beta_im, hipStream_t st) {
    const Spec& s = p->spec;
    const bool f64 = s.dtype == TC_C128;
    if (s.nC == 0) return TC_OK;
    int64_t K = 1;
    for (char ch : s.summed()) K *= s.e(ch);
    const bool no_product = (alpha_re == 0.0 && alpha_im == 0.0) || K == 0;
    double inner_beta = beta_re;
    if (no_product || beta_im != 0.0) {
        // C := beta * C here; the real contraction (if any) then adds to it
        if (!(beta_re == 1.0 && beta_im == 0.0)) {
            ZScaleArgs a{};
            a.C = C;
            a.beta_re = beta_re;
            a.beta_im = beta_im;
            a.total = 1;
            for (const GtDim& d : c_dims(s)) {
                a.dims.d[a.dims.n++] = d;
                a.total *= d.ext;
            }
            dim3 g(grid_for(a.total, 1 << 20)), b(256);
            if (f64) hipLaunchKernelGGL(k_zscale<double>, g, b, 0, st, a);
            else hipLaunchKernelGGL(k_zscale<float>, g, b, 0, st, a);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "complex scale kernel launch");
        }
        if (no_product) return TC_OK;
        inner_beta = 1.0;
    }
    tc_status stt = prepare_complex(p);
    if (stt) return stt;
    ZExpandArgs a{};
    a.src = p->zside == 0 ? A : B;
    a.dst = p->d_zexp;
    a.dims = p->zdims;
    a.total = p->zelems;
    a.s_in = p->zs_in;
    a.s_out = p->zs_out;
    a.alpha_re = alpha_re;
    a.alpha_im = alpha_im;
    dim3 g(grid_for(a.total, 1 << 20)), b(256);
    if (f64) hipLaunchKernelGGL(k_zexpand<double>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_zexpand<float>, g, b, 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "complex expansion kernel launch");
    const void* Ain = p->zside == 0 ? p->d_zexp : A;
    const void* Bin = p->zside == 0 ? B : p->d_zexp;
    return contract_dispatch(p->real, Ain, Bin, C, 1.0, inner_beta, st);
}

}  // namespace tc
