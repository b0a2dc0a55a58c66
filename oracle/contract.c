/*
 * Plain FP64 loop-nest tensor contraction -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the oracle: a slow, obviously correct CPU implementation of the
 * contraction defined in Section 1 ("Tensor Notation") of Peise, Fabregat-Traver
 * and Bientinesi, "On the Performance Prediction of BLAS-based Tensor
 * Contractions" (arXiv 1409.8608).  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the GPU
 * library: it has its own spec parser and its own loops.
 *
 * Definition (Section 1): for every free multi-index f of C,
 *     C[f] = alpha * sum_{k over all contracted indices} A[f_A, k] * B[f_B, k]
 *            + beta * C_in[f]
 * Contracted indices appear in both inputs and not in C; free indices appear in
 * exactly one input and in C.  Two index classes the paper does not define are
 * read as the same sum over every index absent from C: a batch index (in A, B
 * and C) is a free index of both inputs, so each of its values is an ordinary
 * contraction of slices; a trace index (in one input only) is summed with the
 * other input constant along it.  Element (x_1..x_d) of an operand X lives at
 * X + sum_m x_m * stride_m (element units).  The paper assumes Fortran order
 * (first index stride 1); explicit strides generalise that.  The paper's
 * algorithms accumulate into C ("+="); alpha/beta are the BLAS reading of that,
 * with the paper's own runs being alpha = 1, beta = 0.
 *   beta == 0  -> C_in is not read.
 *   alpha == 0 -> A and B are not read.
 *
 * Fixed summation order: the outer odometer runs over C's indices with C's first
 * index fastest; the inner odometer runs over the summed indices (those not in
 * C) in the order they appear in A's spec, then B's indices that are in neither
 * A nor C, first fastest; the accumulator starts at 0.0.
 * Build with -O2 -ffp-contract=off and without fast-math so the products and sums
 * are rounded exactly as written.
 *
 * oracle_contract_z is the same definition over complex numbers (storage as C99
 * double complex: real part, then imaginary part), each product written out as
 * (xr yr - xi yi) + i (xr yi + xi yr) and summed in the same order.
 *
 * oracle_contract_par is oracle_contract with C's outermost index spread over
 * host threads (OpenMP): every output element is summed by one thread in the
 * same order, so its results equal the serial ones bit for bit.  Only the
 * CPU-baseline timing uses it.
 *
 * mode 1 ("Dot2") accumulates with an error-free TwoSum/TwoProduct pair
 * (Ogita, Rump, Oishi, "Accurate sum and dot product", SIAM J. Sci. Comput.
 * 26(6), 2005, Algorithm 5.3), giving a result as if computed in twice the
 * working precision; it is used to measure GPU error floors free of oracle noise.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define OR_MAXIDX 16

enum { OR_OK = 0, OR_E_SPEC = 1, OR_E_EXTENT = 2, OR_E_NULL = 3 };

typedef struct {
    char a[OR_MAXIDX + 1], b[OR_MAXIDX + 1], c[OR_MAXIDX + 1];
    int na, nb, nc;
} or_spec;

/* "abc=ai,ibc" -> three index strings.  Whitespace is not allowed. */
static int or_parse(const char* s, or_spec* p) {
    const char* eq = strchr(s, '=');
    if (!eq) return OR_E_SPEC;
    const char* comma = strchr(eq + 1, ',');
    if (!comma) return OR_E_SPEC;
    p->nc = (int)(eq - s);
    p->na = (int)(comma - eq - 1);
    p->nb = (int)strlen(comma + 1);
    if (p->nc > OR_MAXIDX || p->na > OR_MAXIDX || p->nb > OR_MAXIDX) return OR_E_SPEC;
    memcpy(p->c, s, (size_t)p->nc);          p->c[p->nc] = 0;
    memcpy(p->a, eq + 1, (size_t)p->na);     p->a[p->na] = 0;
    memcpy(p->b, comma + 1, (size_t)p->nb);  p->b[p->nb] = 0;
    const char* all[3] = {p->a, p->b, p->c};
    for (int t = 0; t < 3; ++t)
        for (const char* q = all[t]; *q; ++q) {
            if (*q < 'a' || *q > 'z') return OR_E_SPEC;
            if (strchr(q + 1, *q)) return OR_E_SPEC;     /* repeated in one operand */
        }
    /* every index of C must come from an input; any index of an input is allowed:
     * contracted (A and B), free (one input and C), batch (A, B and C) or trace
     * (one input only) */
    for (const char* q = p->c; *q; ++q)
        if (!strchr(p->a, *q) && !strchr(p->b, *q)) return OR_E_SPEC;
    return OR_OK;
}

static int pos(const char* s, char ch) {
    const char* q = strchr(s, ch);
    return q ? (int)(q - s) : -1;
}

static int64_t extent_of(char ch, const char* idx_chars, const int64_t* extents, int n_idx) {
    for (int t = 0; t < n_idx; ++t)
        if (idx_chars[t] == ch) return extents[t];
    return -1;
}

/* Everything the loops need: parsed spec, per-operand extents and strides,
 * and the summed indices. */
typedef struct {
    or_spec p;
    int64_t extC[OR_MAXIDX];
    int64_t sA[OR_MAXIDX], sB[OR_MAXIDX], sC[OR_MAXIDX];
    char kidx[2 * OR_MAXIDX + 1];
    int nk;
    int64_t kext[2 * OR_MAXIDX];
    int64_t nC, nK;
} or_plan;

/* Strides are in each operand's own spec order; a NULL stride array means
 * Fortran-contiguous for that operand. */
static int or_setup(const char* spec, const char* idx_chars, const int64_t* extents, int n_idx,
                    const int64_t* strides_A, const int64_t* strides_B, const int64_t* strides_C,
                    or_plan* q) {
    or_spec* p = &q->p;
    int rc = or_parse(spec, p);
    if (rc) return rc;
    const char* names[3] = {p->a, p->b, p->c};
    int64_t* strs[3] = {q->sA, q->sB, q->sC};
    const int64_t* given[3] = {strides_A, strides_B, strides_C};
    int lens[3] = {p->na, p->nb, p->nc};
    for (int t = 0; t < 3; ++t) {
        int64_t run = 1;
        for (int m = 0; m < lens[t]; ++m) {
            int64_t e = extent_of(names[t][m], idx_chars, extents, n_idx);
            if (e < 0) return OR_E_EXTENT;
            if (t == 2) q->extC[m] = e;
            strs[t][m] = given[t] ? given[t][m] : run;
            run *= e;
        }
    }
    /* summed indices (not in C): A's in A's order, then B's own */
    q->nk = 0;
    for (int m = 0; m < p->na; ++m)
        if (pos(p->c, p->a[m]) < 0) q->kidx[q->nk++] = p->a[m];
    for (int m = 0; m < p->nb; ++m)
        if (pos(p->c, p->b[m]) < 0 && pos(p->a, p->b[m]) < 0) q->kidx[q->nk++] = p->b[m];
    q->kidx[q->nk] = 0;
    for (int k = 0; k < q->nk; ++k) q->kext[k] = extent_of(q->kidx[k], idx_chars, extents, n_idx);
    q->nC = 1;
    q->nK = 1;
    for (int m = 0; m < p->nc; ++m) q->nC *= q->extC[m];
    for (int k = 0; k < q->nk; ++k) q->nK *= q->kext[k];
    return OR_OK;
}

/* Offsets of C[ci] and of the free parts of A and B. */
static void or_free_offsets(const or_plan* q, const int64_t* ci, int64_t* offC, int64_t* offA, int64_t* offB) {
    const or_spec* p = &q->p;
    *offC = *offA = *offB = 0;
    for (int m = 0; m < p->nc; ++m) {
        *offC += ci[m] * q->sC[m];
        int pa = pos(p->a, p->c[m]), pb = pos(p->b, p->c[m]);
        if (pa >= 0) *offA += ci[m] * q->sA[pa];
        if (pb >= 0) *offB += ci[m] * q->sB[pb];
    }
}

/* Add the summed part of the offsets at summed position ki. */
static void or_sum_offsets(const or_plan* q, const int64_t* ki, int64_t* oa, int64_t* ob) {
    const or_spec* p = &q->p;
    for (int k = 0; k < q->nk; ++k) {
        int pa = pos(p->a, q->kidx[k]), pb = pos(p->b, q->kidx[k]);
        if (pa >= 0) *oa += ki[k] * q->sA[pa];   /* a trace index of B leaves A fixed */
        if (pb >= 0) *ob += ki[k] * q->sB[pb];
    }
}

/* Odometer step, first index fastest. */
static void or_step(int64_t* idx, const int64_t* ext, int n) {
    for (int m = 0; m < n; ++m) {
        if (++idx[m] < ext[m]) return;
        idx[m] = 0;
    }
}

/* Elements f0 .. f0 + count - 1 of C in the fixed order, ci holding the
 * multi-index of f0. */
static void or_run(const or_plan* pq, int64_t* ci, int64_t count,
                   const double* A, const double* B, double* C, double alpha, double beta, int mode) {
    const or_plan q = *pq;
    int64_t ki[2 * OR_MAXIDX];
    for (int64_t f = 0; f < count; ++f) {
        int64_t offC, offA, offB;
        or_free_offsets(&q, ci, &offC, &offA, &offB);
        double acc = 0.0, comp = 0.0;
        if (alpha != 0.0) {
            memset(ki, 0, sizeof ki);
            for (int64_t k = 0; k < q.nK; ++k) {
                int64_t oa = offA, ob = offB;
                or_sum_offsets(&q, ki, &oa, &ob);
                double x = A[oa], y = B[ob];
                if (mode == 1) {
                    /* TwoProduct via fma, TwoSum (Knuth) */
                    double prod = x * y;
                    double perr = fma(x, y, -prod);
                    double s = acc + prod;
                    double bb = s - acc;
                    double serr = (acc - (s - bb)) + (prod - bb);
                    acc = s;
                    comp += perr + serr;
                } else {
                    acc += x * y;
                }
                or_step(ki, q.kext, q.nk);
            }
            if (mode == 1) acc = acc + comp;
        }
        double out = alpha * acc;
        if (beta != 0.0) out += beta * C[offC];
        C[offC] = out;
        or_step(ci, q.extC, q.p.nc);
    }
}

static int or_check(const char* spec, const char* idx_chars, const int64_t* extents, int n_idx,
                    const int64_t* strides_A, const int64_t* strides_B, const int64_t* strides_C,
                    const double* A, const double* B, const double* C, double alpha, or_plan* q) {
    int rc = or_setup(spec, idx_chars, extents, n_idx, strides_A, strides_B, strides_C, q);
    if (rc) return rc;
    if (q->nC == 0) return OR_OK;
    if (!C) return OR_E_NULL;
    if (alpha != 0.0 && q->nK > 0 && (!A || !B)) return OR_E_NULL;
    return OR_OK;
}

/* Returns 0 on success. */
int oracle_contract(const char* spec, const char* idx_chars, const int64_t* extents, int n_idx,
                    const double* A, const int64_t* strides_A,
                    const double* B, const int64_t* strides_B,
                    double* C, const int64_t* strides_C,
                    double alpha, double beta, int mode) {
    or_plan q;
    int rc = or_check(spec, idx_chars, extents, n_idx, strides_A, strides_B, strides_C, A, B, C, alpha, &q);
    if (rc || q.nC == 0) return rc;
    int64_t ci[OR_MAXIDX];
    memset(ci, 0, sizeof ci);
    or_run(&q, ci, q.nC, A, B, C, alpha, beta, mode);
    return OR_OK;
}

/* The same, C's outermost (last) index spread over `threads` host threads. */
int oracle_contract_par(const char* spec, const char* idx_chars, const int64_t* extents, int n_idx,
                        const double* A, const int64_t* strides_A,
                        const double* B, const int64_t* strides_B,
                        double* C, const int64_t* strides_C,
                        double alpha, double beta, int threads) {
    or_plan q;
    int rc = or_check(spec, idx_chars, extents, n_idx, strides_A, strides_B, strides_C, A, B, C, alpha, &q);
    if (rc || q.nC == 0) return rc;
    const int last = q.p.nc - 1;
    const int64_t outer = last >= 0 ? q.extC[last] : 1;
    const int64_t per = q.nC / outer;          /* elements per value of the outermost index */
    int64_t o;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
    for (o = 0; o < outer; ++o) {
        int64_t ci[OR_MAXIDX];
        memset(ci, 0, sizeof ci);
        if (last >= 0) ci[last] = o;
        or_run(&q, ci, per, A, B, C, alpha, beta, 0);
    }
    return OR_OK;
}

/* Complex operands: each element is two doubles (real, imaginary); strides
 * count complex elements.  alpha and beta are (re, im) pairs.  beta == 0 does
 * not read C; alpha == 0 does not read A or B. */
int oracle_contract_z(const char* spec, const char* idx_chars, const int64_t* extents, int n_idx,
                      const double* A, const int64_t* strides_A,
                      const double* B, const int64_t* strides_B,
                      double* C, const int64_t* strides_C,
                      double alpha_re, double alpha_im, double beta_re, double beta_im) {
    or_plan q;
    int rc = or_setup(spec, idx_chars, extents, n_idx, strides_A, strides_B, strides_C, &q);
    if (rc) return rc;
    if (q.nC == 0) return OR_OK;
    if (!C) return OR_E_NULL;
    int use_ab = alpha_re != 0.0 || alpha_im != 0.0;
    int use_c = beta_re != 0.0 || beta_im != 0.0;
    if (use_ab && q.nK > 0 && (!A || !B)) return OR_E_NULL;

    int64_t ci[OR_MAXIDX], ki[2 * OR_MAXIDX];
    memset(ci, 0, sizeof ci);
    for (int64_t f = 0; f < q.nC; ++f) {
        int64_t offC, offA, offB;
        or_free_offsets(&q, ci, &offC, &offA, &offB);
        double acc_re = 0.0, acc_im = 0.0;
        if (use_ab) {
            memset(ki, 0, sizeof ki);
            for (int64_t k = 0; k < q.nK; ++k) {
                int64_t oa = offA, ob = offB;
                or_sum_offsets(&q, ki, &oa, &ob);
                double xr = A[2 * oa], xi = A[2 * oa + 1];
                double yr = B[2 * ob], yi = B[2 * ob + 1];
                acc_re += xr * yr - xi * yi;
                acc_im += xr * yi + xi * yr;
                or_step(ki, q.kext, q.nk);
            }
        }
        double out_re = alpha_re * acc_re - alpha_im * acc_im;
        double out_im = alpha_re * acc_im + alpha_im * acc_re;
        if (use_c) {
            double cr = C[2 * offC], cim = C[2 * offC + 1];
            out_re += beta_re * cr - beta_im * cim;
            out_im += beta_re * cim + beta_im * cr;
        }
        C[2 * offC] = out_re;
        C[2 * offC + 1] = out_im;
        or_step(ci, q.extC, q.p.nc);
    }
    return OR_OK;
}
