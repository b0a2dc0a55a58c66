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
// is that of the complex sum: four real products per complex one.  The
// split-precision forms apply the same way, to the embedded real operands.
#include <algorithm>
#include <cstring>
#include <string>

#include "devutil.h"
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

// Streaming kernel for few summed positions on complex data (the complex form
// of the real streaming kernel).  The embedding above doubles the summed length
// and stores each element of the expanded operand twice, which for a streamed
// C multiplies the on-chip reads per byte of C; here the operands stay complex.
// A block is four waves, one C column each (R columns per wave).  Along C's
// unit-stride M dimension a lane owns W chunks of 16 bytes (CPC complex
// elements each), 64 chunks apart, so every load and store instruction of a
// wave covers 1 KB of contiguous memory; it keeps A's K values for them in
// registers and reuses them for all R columns.  kA/kB (complex-element offsets)
// are padded by the host to KT entries repeating the last one; padded terms are
// zeroed by selects.
template <typename T, int KT, int W, int R, bool BETA>
__global__ __launch_bounds__(256) void k_zstream_wave(const T* __restrict__ A, const T* __restrict__ B,
                                                      T* __restrict__ C, StreamArgs a, double alpha_im,
                                                      double beta_im) {
    constexpr int CPC = 8 / (int)sizeof(T);          // complex elements per 16-byte chunk
    constexpr int VEC = W * CPC;                      // complex elements per lane
    typedef T vec_t __attribute__((ext_vector_type(2 * CPC)));
    constexpr int SPAN = 64 * VEC;
    const int tid = threadIdx.x;
    const uint32_t mblocks = (uint32_t)(a.M / SPAN);
    const uint32_t mb = blockIdx.x % mblocks;
    const uint32_t nb = blockIdx.x / mblocks;
    const int row = __builtin_amdgcn_readfirstlane(tid / 64);
    const int64_t m0 = (int64_t)mb * SPAN + (tid % 64) * CPC;   // chunk w starts at m0 + 64 CPC w

    int64_t offB[R], offC[R];
    bool ok[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int64_t n = ((int64_t)nb * R + q) * 4 + row;
        ok[q] = n < a.N;
        const int64_t nn = ok[q] ? n : a.N - 1;
        if (a.n.n == 1) {
            offB[q] = nn * a.n.d[0].sB;
            offC[q] = nn * a.n.d[0].sC;
        } else {
            int64_t rem = nn, ob = 0, oc = 0;
            for (int d = 0; d < a.n.n; ++d) {
                const int64_t r = divmod(rem, a.n.d[d].ext);
                ob += r * a.n.d[d].sB;
                oc += r * a.n.d[d].sC;
            }
            offB[q] = ob;
            offC[q] = oc;
        }
    }
    T br[R][KT], bi[R][KT];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            const T* bp = B + 2 * (offB[q] + a.kB[k]);
            const T xr = bp[0], xi = bp[1];
            br[q][k] = (k < a.K) ? xr : (T)0;
            bi[q][k] = (k < a.K) ? xi : (T)0;
        }
    T ar[VEC][KT], ai[VEC][KT];
#pragma unroll
    for (int k = 0; k < KT; ++k)
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const vec_t t = *(const vec_t*)(A + 2 * (a.kA[k] + m0 + 64 * CPC * w));
#pragma unroll
            for (int c = 0; c < CPC; ++c) {
                ar[w * CPC + c][k] = (k < a.K) ? t[2 * c] : (T)0;
                ai[w * CPC + c][k] = (k < a.K) ? t[2 * c + 1] : (T)0;
            }
        }
    const T alr = (T)a.alpha, ali = (T)alpha_im;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (!ok[q]) break;   // columns grow with q: the rest are past N too
#pragma unroll
        for (int w = 0; w < W; ++w) {
            vec_t val;
#pragma unroll
            for (int c = 0; c < CPC; ++c) {
                const int v = w * CPC + c;
                T sr = 0, si = 0;
#pragma unroll
                for (int k = 0; k < KT; ++k) {   // four fused multiply-adds per complex term
                    sr += ar[v][k] * br[q][k];
                    sr -= ai[v][k] * bi[q][k];
                    si += ar[v][k] * bi[q][k];
                    si += ai[v][k] * br[q][k];
                }
                val[2 * c] = alr * sr - ali * si;
                val[2 * c + 1] = alr * si + ali * sr;
            }
            vec_t* cp = (vec_t*)(C + 2 * (offC[q] + m0 + 64 * CPC * w));
            if (BETA) {
                const vec_t old = *cp;
                const T bre = (T)a.beta, bim = (T)beta_im;
#pragma unroll
                for (int c = 0; c < CPC; ++c) {
                    val[2 * c] += bre * old[2 * c] - bim * old[2 * c + 1];
                    val[2 * c + 1] += bre * old[2 * c + 1] + bim * old[2 * c];
                }
            }
            __builtin_nontemporal_store(val, cp);
        }
    }
}

template <typename T, int W, bool BETA>
static void launch_zstream(const StreamArgs& w, double alpha_im, double beta_im, unsigned grid, hipStream_t st) {
    const T* A = (const T*)w.A;
    const T* B = (const T*)w.B;
    T* C = (T*)w.C;
    dim3 g(grid), b(256);
    if (w.K <= 4)
        hipLaunchKernelGGL((k_zstream_wave<T, 4, W, 4, BETA>), g, b, 0, st, A, B, C, w, alpha_im, beta_im);
    else
        hipLaunchKernelGGL((k_zstream_wave<T, 8, W, 4, BETA>), g, b, 0, st, A, B, C, w, alpha_im, beta_im);
}

// Complex elements per lane: a wide form (two 16-byte chunks, twice the
// outputs per B value read) and a narrow one (one chunk).
static int zvec_narrow(bool f64) { return f64 ? 1 : 2; }

// The complex streaming kernel takes a plan whose complex GEMM view has at most
// 8 summed positions (beyond that the embedding on matrix-core tiles is faster:
// at a = b = c = 1024 with 12 or 16 positions 8.05 ms against 8.9-9.4 ms for
// c128, 3.75 against 4.1-4.5 ms for c64), one M dimension with unit stride in C and in A (after
// the swap that puts C's unit stride in M), no batch indices, M a whole number
// of wave spans (64 VEC), and every N stride of C and K stride of A a multiple
// of a chunk's complex elements.  Returns the widest VEC that fits, 0 if none;
// the call then also needs A and C to start on 16 bytes.
static int zstream_vec(const tc_plan_s* p) {
    const GemmView& gv = p->gv;
    const bool f64 = p->spec.dtype == TC_C128;
    const int cpc = zvec_narrow(f64);
    if (gv.K < 1 || gv.K > 8 || gv.m.size() != 1 || !gv.b.empty()) return 0;
    if ((int)gv.n.size() > GT_MAXD || (int)gv.k.size() > GT_MAXD) return 0;   // launch descriptor sizes
    if (gv.m[0].sC != 1 || gv.m[0].sA != 1) return 0;
    for (const GtDim& d : gv.n)
        if (d.sC % cpc != 0) return 0;
    for (const GtDim& d : gv.k)
        if (d.sA % cpc != 0) return 0;
    if (gv.M % (128 * cpc) == 0) return 2 * cpc;
    return gv.M % (64 * cpc) == 0 ? cpc : 0;
}

// Runs the streaming kernel if the pointers allow; *ran is false otherwise.
static tc_status run_zstream(tc_plan_s* p, const void* A, const void* B, void* C, double alpha_re,
                             double alpha_im, double beta_re, double beta_im, hipStream_t st, bool* ran) {
    const GemmView& gv = p->gv;
    const bool f64 = p->spec.dtype == TC_C128;
    *ran = false;
    if (gv.swapped) std::swap(A, B);
    const int vec = p->zvec;
    // every access is one 16-byte chunk: A and C must start on 16 bytes
    if (((uintptr_t)A) % 16 != 0 || ((uintptr_t)C) % 16 != 0) return TC_OK;
    StreamArgs w{};
    w.A = A; w.B = B; w.C = C;
    w.M = gv.M;
    w.sAm = 1;
    w.N = gv.N;
    w.n.n = (int)gv.n.size();
    for (int d = 0; d < w.n.n; ++d) w.n.d[d] = gv.n[d];
    w.K = (int)gv.K;
    std::vector<int64_t> idx(gv.k.size(), 0);
    for (int k = 0; k < w.K; ++k) {
        int64_t oa = 0, ob = 0;
        for (size_t d = 0; d < gv.k.size(); ++d) {
            oa += idx[d] * gv.k[d].sA;
            ob += idx[d] * gv.k[d].sB;
        }
        w.kA[k] = oa;
        w.kB[k] = ob;
        for (size_t d = 0; d < gv.k.size(); ++d) {
            if (++idx[d] < gv.k[d].ext) break;
            idx[d] = 0;
        }
    }
    for (int k = w.K; k < GT_SMALLK_MAX; ++k) {
        w.kA[k] = w.kA[w.K - 1];
        w.kB[k] = w.kB[w.K - 1];
    }
    w.alpha = alpha_re;
    w.beta = beta_re;
    const int64_t cols = 4 * 4;   // four waves of four columns (R = 4 in every launch above)
    const int64_t grid = (gv.M / (64 * vec)) * ((gv.N + cols - 1) / cols);
    if (grid > 0x7fffffff) return TC_OK;
    const bool beta = beta_re != 0.0 || beta_im != 0.0;
    const unsigned g = (unsigned)grid;
    const bool wide = vec > zvec_narrow(f64);
    if (f64 && wide) {
        if (beta) launch_zstream<double, 2, true>(w, alpha_im, beta_im, g, st);
        else launch_zstream<double, 2, false>(w, alpha_im, beta_im, g, st);
    } else if (f64) {
        if (beta) launch_zstream<double, 1, true>(w, alpha_im, beta_im, g, st);
        else launch_zstream<double, 1, false>(w, alpha_im, beta_im, g, st);
    } else if (wide) {
        if (beta) launch_zstream<float, 2, true>(w, alpha_im, beta_im, g, st);
        else launch_zstream<float, 2, false>(w, alpha_im, beta_im, g, st);
    } else {
        if (beta) launch_zstream<float, 1, true>(w, alpha_im, beta_im, g, st);
        else launch_zstream<float, 1, false>(w, alpha_im, beta_im, g, st);
    }
    *ran = true;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? TC_OK : hip_fail(e, "complex streaming kernel launch");
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
                           s.compute);
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
    // the complex GEMM view (strides in complex elements) for the streaming kernel
    p->gv = gemm_view(s);
    // the split-precision forms run on the embedded real plan only
    p->zvec = s.compute == TC_NATIVE ? zstream_vec(p) : 0;
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
    if (!no_product && p->zvec) {
        bool ran = false;
        tc_status r = run_zstream(p, A, B, C, alpha_re, alpha_im, beta_re, beta_im, st, &ran);
        if (r || ran) return r;
    }
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

    if (!p->d_zexp) return fail_unprepared();
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
