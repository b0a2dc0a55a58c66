/*
 * tc.h -- C ABI of the MI355X tensor-contraction library (libtc.so).
 *
 * The library computes dense two-operand tensor contractions written in
 * Einstein notation (Peise, Fabregat-Traver, Bientinesi, "On the Performance
 * Prediction of BLAS-based Tensor Contractions", arXiv 1409.8608, Section 1,
 * "Tensor Notation"):
 *
 *     C[f] = alpha * sum_k A[f_A, k] * B[f_B, k] + beta * C[f]
 *
 * where the contracted indices k appear in both inputs and not in C, and the
 * free indices f appear in exactly one input and in C.  Every member of the
 * paper's algorithm family (Section 2: loop nests over sliced indices around a
 * dot, axpy, gemv, ger or gemm call, with copies where a matrix slice lacks a
 * contiguous dimension) runs on the GPU, plus one fused direct-contraction
 * kernel.  The paper's micro-benchmark performance model (Section 3) predicts
 * which member is fastest.
 *
 * Conventions for every entry point
 *   - All functions return a tc_status; no C++ exception crosses the ABI.
 *     tc_last_error() returns a thread-local detail string for the last
 *     failing call on the calling thread.
 *   - Arguments are validated before any device work, so a failing call leaves
 *     C untouched.
 *   - Tensor pointers (A, B, C) are DEVICE pointers (e.g. torch data_ptr()).
 *     They are borrowed: the caller keeps them alive until the stream work has
 *     completed.  `stream` is a hipStream_t passed as void*; NULL is the null
 *     stream.  Asynchronous device faults surface at the caller's next sync.
 *   - Strides are in ELEMENTS, one per axis in the operand's spec order.  A NULL
 *     stride array means Fortran order (first axis stride 1), the paper's
 *     storage.  Input strides must be >= 0 (0 broadcasts); C strides must be
 *     > 0 and C must not overlap itself.
 *   - A plan must not be used by two host threads at once; distinct plans are
 *     independent.  Calls on one plan reuse its device workspace (copy
 *     temporaries, split-precision terms, split-K partial tiles): two calls on
 *     one plan on streams with no ordering between them race; give each
 *     concurrent stream its own plan.
 */
#ifndef TC_H
#define TC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tc_plan_s* tc_plan_t;     /* opaque, owned by the caller until tc_plan_destroy */
typedef struct tc_batch_s* tc_batch_t;   /* opaque, owned by the caller until tc_batch_destroy */

/* Storage type of A, B and C.  TC_C128 / TC_C64 are complex: each element is
 * its real part followed by its imaginary part (the layout of C99 double
 * complex / float complex), and strides count complex elements.  A complex
 * contraction runs as a real one in the matching real precision: one operand
 * (the one with fewer elements) is written once per call into plan workspace as
 * real 2x2 blocks [re -im; im re], scaled by alpha, which adds a summed index
 * over the other operand's (re, im) pair and a free index over C's; that
 * operand and C are read in place.  Complex plans have no family members,
 * cannot join a batch and need two letters the spec does not use
 * (TC_E_UNSUPPORTED otherwise).  With TC_BF16X3 / TC_FP8X3 the split forms
 * run on the embedded real operands, and tc_split_terms reports those. */
typedef enum { TC_F64 = 0, TC_F32 = 1, TC_C128 = 2, TC_C64 = 3 } tc_dtype;

/* Arithmetic path.  TC_NATIVE computes in the storage type.  TC_BF16X3 splits
 * each power-of-two scaled slice into three BF16 terms and forms the six
 * products of order <= 4 on BF16 matrix cores with FP32 accumulation (the
 * leading product and the five smaller ones in two sums, added exactly in FP64
 * at the end).  TC_FP8X3 does the same with OCP E4M3 terms, term p scaled by
 * 2^(4(p-1)) to stay in E4M3's normal range, on FP8 matrix cores whose operand
 * scales undo that factor; at most 8192 contracted positions. */
typedef enum { TC_NATIVE = 0, TC_BF16X3 = 1, TC_FP8X3 = 2 } tc_compute;

typedef enum {
    TC_OK = 0,
    TC_E_SPEC,         /* malformed spec (repeated letter, C index in no input, ...) */
    TC_E_EXTENT,       /* missing/negative extent, or element count overflow */
    TC_E_STRIDE,       /* negative input stride, non-positive or self-overlapping C stride */
    TC_E_DTYPE,        /* unknown dtype or dtype/compute pair */
    TC_E_ALIAS,        /* C's address range overlaps A's or B's */
    TC_E_NULL,         /* NULL pointer where a non-empty tensor or output is needed */
    TC_E_VARIANT,      /* variant index out of range */
    TC_E_HIP,          /* a HIP runtime call or kernel launch failed */
    TC_E_NOMEM,        /* device workspace allocation failed */
    TC_E_UNSUPPORTED,  /* valid request this build does not execute (reason in tc_last_error) */
    TC_E_CAPACITY      /* output array too small; *n_out holds the size needed */
} tc_status;

/* Kernel of a family member (Section 2 kernel list); TC_KERNEL_FUSED is the
 * library's own direct-contraction kernel (not a paper algorithm). */
enum { TC_KERNEL_DOT = 0, TC_KERNEL_AXPY = 1, TC_KERNEL_GEMV = 2, TC_KERNEL_GER = 3,
       TC_KERNEL_GEMM = 4, TC_KERNEL_FUSED = 5 };

#define TC_VARIANT_FUSED (-2)      /* the fused direct-contraction kernel */
#define TC_VARIANT_PREDICTED (-1)  /* the fastest member according to tc_predict */

/* One family member.  `number` follows the paper's legend numbering (kernel-
 * major: dot, axpy, gemv, ger, gemm), starting at 1.  `name` is the paper's
 * name, e.g. "ca-gemv" or "i'c-gemm" (Section 2, footnote on names). */
typedef struct {
    char    name[40];
    int     number;
    int     kernel;                /* TC_KERNEL_* */
    char    kept[8];               /* kept (kernel) index letters, NUL-terminated */
    char    loops[16];             /* sliced index letters, outermost loop first */
    int     n_copies;
    char    copy_tensor[4];        /* 'A', 'B' or 'C' for each copy */
    int     copy_level[4];         /* loop position the copy runs in; -1 before all loops */
    /* GPU schedule (how the loop nest maps to launches): */
    int     n_hoisted;             /* leading contracted loops run as separate launch passes */
    int64_t launches;              /* kernel launches per contraction, copies and prologue included */
    int64_t invocations;           /* kernel calls of the paper's loop nest (product of loop extents) */
    int     runs_on_gpu;           /* 0: tc_contract refuses the member (a copy of C with a contracted
                                      loop at or outside it among the free loops) */
} tc_variant_info;

/* One entry of a micro-benchmark setup list (Section 3.2): an access to a kernel
 * operand, or to a remote region of `size` elements. */
typedef struct {
    int     kind;                  /* 0 = operand, 1 = remote region */
    int     tensor;                /* 0 = A, 1 = B, 2 = C (operand entries), -1 for remote */
    int64_t size;                  /* elements */
} tc_setup_item;

#define TC_MAX_SETUP 16
/* One benchmark class of a prediction (Sections 3.4, 3.5): steady state,
 * prefetch failure or first iteration of a loop, with its share of the kernel
 * invocations and its setup list. */
typedef struct {
    char          label[16];       /* "steady", "fail", "first@<loop>" */
    double        weight;          /* share of all kernel invocations, sums to 1 */
    int           n_items;
    tc_setup_item items[TC_MAX_SETUP];
} tc_bench_class;

/* Result of tc_predict for one variant. */
typedef struct {
    int    variant;                /* 0-based index into the plan's family, or TC_VARIANT_FUSED */
    double predicted_s;            /* stage-5 prediction (all refinements) */
    double stage_s[5];             /* predictions of stages 1..5 (Section 3.1 .. 3.5) */
    double bench_s;                /* time spent measuring this variant's micro-benchmarks */
    int    n_bench;                /* distinct micro-benchmarks it used */
} tc_prediction;

/* --- plans ---------------------------------------------------------------- */

/* Build a plan: parse `spec` ("abc=ai,ibc"), classify indices (Section 1),
 * bind extents and strides, enumerate the algorithm family (Section 2,
 * Table 1 x loop orders) and map each member to a GPU schedule.  When a GPU is
 * visible, the plan then allocates on the current device every buffer the
 * fused kernel needs (K table, split-K partial tiles, split-precision terms,
 * complex expansion), so that tc_contract never allocates; a plan built where
 * no GPU is visible is host-only (queries and the symbolic model) until
 * tc_plan_prepare.
 *   Index classes: contracted (both inputs, not C) and free (one input and C)
 *   as in Section 1; also batch (A, B and C) and trace (one input only),
 *   computed as the same sum over every index absent from C.  Specs with
 *   batch or trace indices have no family members (fused kernel only) and
 *   no split-precision forms (TC_E_UNSUPPORTED).  Specs with more than 7
 *   distinct letters have no family members either (n letters give up to
 *   (n - 1)! loop orders per kernel).
 *   Each of M (free indices of one input), N, K, the batch indices and C may
 *   hold at most 8 dimension groups once indices that continue each other in
 *   memory are merged; more is TC_E_UNSUPPORTED.
 *   index_chars/extents: n_index letters and their extents (every letter of
 *                        the spec must be given; extra letters are an error).
 *   strides_X: element strides in X's spec order, or NULL for Fortran order.
 * Errors: TC_E_SPEC, TC_E_EXTENT, TC_E_STRIDE, TC_E_DTYPE, TC_E_NULL,
 * TC_E_UNSUPPORTED. */
tc_status tc_plan(tc_plan_t* out, const char* spec,
                  const char* index_chars, const int64_t* extents, int n_index,
                  const int64_t* strides_A, const int64_t* strides_B, const int64_t* strides_C,
                  tc_dtype dtype, tc_compute compute);

/* Free a plan and its device workspace.  NULL is accepted.  (Lifetime of the
 * plan object; no passage.) */
tc_status tc_plan_destroy(tc_plan_t plan);

/* Number of members of the plan's algorithm family (Section 2: Table 1's
 * kernels x every loop order of the other indices; 36 for "abc=ai,ibc",
 * Section 3's case study). */
tc_status tc_variant_count(tc_plan_t plan, int* n);

/* Describe member `variant` (0-based) or TC_VARIANT_FUSED: the paper's name
 * and number (Section 2, footnote on names; Figure 2/4/5 legends), kernel,
 * loops and copies, and its GPU schedule. */
tc_status tc_variant_get(tc_plan_t plan, int variant, tc_variant_info* out);

/* Select which algorithm tc_contract runs: a 0-based member of the family
 * (Section 2), TC_VARIANT_FUSED (default), or TC_VARIANT_PREDICTED, the one
 * Section 3's prediction ranks fastest (requires a prior tc_predict; changing
 * the root gaps clears the prediction, and tc_contract then returns
 * TC_E_VARIANT until tc_predict runs again).  When a GPU is visible the
 * selected member's buffers (copy temporaries, K table) are allocated here.
 * Errors: TC_E_VARIANT, TC_E_UNSUPPORTED, TC_E_NOMEM, TC_E_HIP. */
tc_status tc_set_variant(tc_plan_t plan, int variant);

/* Allocate every device buffer the selected variant needs on the current
 * device: temporaries of the copies of Section 2 (the operands marked ' in a
 * member's name), K tables, split-K partial tiles, split-precision terms.
 * tc_plan and tc_set_variant do this themselves when a GPU is visible; call it
 * for a plan built without one.  Idempotent.  Errors: TC_E_NOMEM, TC_E_HIP. */
tc_status tc_plan_prepare(tc_plan_t plan);

/* Bytes of device workspace the plan holds now (the buffers tc_plan_prepare
 * lists; no passage). */
tc_status tc_plan_workspace(tc_plan_t plan, int64_t* bytes);

/* Run the contraction (Section 1's definition; the kernels of Section 2
 * accumulate, read here as alpha and beta) with the selected variant on
 * `stream`:
 *     C = alpha * contract(A, B) + beta * C
 * alpha/beta are rounded to the storage type.  beta == 0: C is not read.
 * alpha == 0: A and B are not read.  Asynchronous; returns after the launches.
 * Never allocates: a plan without its device workspace (built with no GPU
 * visible) gives TC_E_UNSUPPORTED, so calls can be captured in a HIP graph.
 * Errors: TC_E_NULL, TC_E_ALIAS, TC_E_VARIANT, TC_E_UNSUPPORTED, TC_E_HIP. */
tc_status tc_contract(tc_plan_t plan, const void* A, const void* B, void* C,
                      double alpha, double beta, void* stream);

/* tc_contract with complex alpha and beta, (re, im) each; rounded to the plan's
 * real precision as in tc_contract.  alpha == 0 (both parts): A and B are not
 * read.  beta == 0: C is not read.  On a real plan both imaginary parts must be
 * zero (TC_E_UNSUPPORTED otherwise).  Errors as tc_contract. */
tc_status tc_contract_complex(tc_plan_t plan, const void* A, const void* B, void* C,
                              double alpha_re, double alpha_im, double beta_re, double beta_im, void* stream);

/* Term products kept by a TC_BF16X3 plan (the library's split-precision
 * form; not in the paper): 6 (every t_A,p t_B,q with p + q <= 4, the default),
 * or, as ablations, 3 (p + q <= 3: about 2^-16 of |A||B| dropped) or 9 (all).
 * Host only; takes effect at the next tc_contract.  A batch takes only plans
 * with 6.  Errors: TC_E_NULL, TC_E_UNSUPPORTED (not a TC_BF16X3 plan, or a
 * count other than 3, 6, 9). */
tc_status tc_set_split_products(tc_plan_t plan, int products);

/* Copy the split terms of the last tc_contract of a TC_BF16X3 or TC_FP8X3
 * plan to host memory, for bit-exact checks of the quantisation (the
 * library's split-precision form; not in the paper).  side 0 = A,
 * 1 = B.  The GEMM view of the plan orders rows by the free indices of that
 * side (first fastest) and columns by the plan's K order.  terms: 3 * rows * kp
 * elements, term-major, row-major: BF16 bit patterns (uint16) for TC_BF16X3,
 * E4M3 codes (uint8, term p stored times 2^(4(p-1))) for TC_FP8X3.  exps: rows
 * power-of-two exponents.
 * With both pointers NULL only *rows and *kp are filled.  Synchronises the
 * device.  Errors: TC_E_UNSUPPORTED (no split yet), TC_E_VARIANT (bad side). */
tc_status tc_split_terms(tc_plan_t plan, int side, void* terms, int32_t* exps, int64_t* rows, int64_t* kp);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tc_contract
 * with the fused kernel, whose device buffers beyond A, B and C (the
 * matrix-core kernel's table of contracted positions, 16 bytes per position,
 * and its split-K partial tiles) live in a static device array of
 * TC_NOALLOC_SCRATCH_BYTES that each GPU holds from the library's load to the
 * end of the process.  The call makes no device allocation of any kind (and
 * does not touch the plan's own workspace); the table is copied host to device
 * on `stream` (hipMemcpyAsync) before the launch.  Every call on one GPU shares
 * that GPU's array and overwrites it: calls that overlap on one GPU (streams
 * with no ordering between them) race, so order them on one stream.  Same
 * semantics and checks as tc_contract.  Needs a real plan, the native compute
 * mode and the fused kernel selected (the default); the streaming kernel (few
 * summed positions) needs no scratch.  A split-K choice is limited to what fits
 * in the array beside the table (fewer slices, down to none).
 * Errors: as tc_contract; TC_E_UNSUPPORTED for a complex or split-precision
 * plan, a member variant selected, or a table of contracted positions larger
 * than the array (more than TC_NOALLOC_SCRATCH_BYTES / 16 positions). */
#define TC_NOALLOC_SCRATCH_BYTES (64LL << 20)
tc_status tc_contract_noalloc(tc_plan_t plan, const void* A, const void* B, void* C,
                              double alpha, double beta, void* stream);

/* --- performance prediction (Section 3) ----------------------------------- */

/* Access distance, in elements, of kernel operand `tensor` (0 = A, 1 = B,
 * 2 = C) of member `variant` (Section 3.2).  Host only. */
tc_status tc_access_distance(tc_plan_t plan, int variant, int tensor, int64_t* out);

/* Benchmark classes of member `variant` at prediction stage `stage` (1 = repeated
 * execution, 2 = access distances, 3 = prefetching, 4 = prefetch failures,
 * 5 = first iterations separate), for a cache of `cache_elems` elements and a
 * line of `line_elems` elements.  Host only.  Errors: TC_E_CAPACITY. */
tc_status tc_bench_classes(tc_plan_t plan, int variant, int stage, double cache_elems,
                           int line_elems, tc_bench_class* out, int capacity, int* n_out);

/* Cache precondition of the prediction (Section 3.2, the walk's third case).
 * When the back-traversal of an operand reaches the algorithm's root, the paper
 * assumes the contraction runs again and again with nothing in between, since
 * it cannot know the surrounding program.  gap[t] (t = 0 A, 1 B, 2 C) states
 * what the caller's program does: the number of elements (of the plan's storage
 * type) of other data it accesses between the previous use of operand t and
 * this contraction.  It is added to the access distance at the root, in
 * tc_access_distance, tc_bench_classes and tc_predict.  NULL or all zero is the
 * paper's assumption (the default); a gap of 5/4 of the cache or more makes
 * the operand cold.  Clears an earlier prediction.  Host only.
 * Errors: TC_E_NULL, TC_E_EXTENT (negative gap). */
tc_status tc_set_root_gap(tc_plan_t plan, const int64_t* gap);

/* Root gaps for a chain of n contractions that a program runs in this order,
 * again and again (for instance T = A B, then D = T E).  ids holds 3 * n tensor
 * ids, A, B and C of each plan; equal ids name the same tensor.  For operand t
 * of plan j the gap is the total size of the distinct tensors accessed by the
 * plans run since that tensor was last used (by an earlier plan of the chain,
 * or else by plan j's own previous run), leaving out plan j's own tensors,
 * which the walk counts already; sizes are element counts times element bytes,
 * converted to plan j's elements.  Calls tc_set_root_gap on every plan; a plan
 * listed more than once keeps the gaps of its last position.
 * Host only.  Errors: TC_E_NULL. */
tc_status tc_chain_root_gaps(const tc_plan_t* plans, const int* ids, int n);

/* Predict the run time of every member (and the fused kernel, last) on the
 * current device: for each member's benchmark classes, run the GPU
 * micro-benchmark (setup accesses, then the member's kernel on a sample of its
 * invocations, 10 repetitions, median) and weight and sum the medians.
 * Micro-benchmarks shared by several members run once.  Needs scratch device
 * memory of up to a few hundred MB, freed on return.  Synchronous.
 * Errors: TC_E_CAPACITY (*n_out = count + 1), TC_E_HIP, TC_E_NOMEM. */
tc_status tc_predict(tc_plan_t plan, tc_prediction* out, int capacity, int* n_out);

/* --- batches ----------------------------------------------------------------- */

/* Build a batch of n independent contractions (not in the paper: many
 * contractions in one launch; its tuner is seeded as Section 3 predicts).
 * Plans stay owned by the caller and must outlive the batch; each needs real
 * storage, a non-empty C and a contracted extent > 0.  Every native or
 * TC_BF16X3 contraction becomes matrix-core tiles (128x128 outputs, 64x64 when
 * M or N is at most 64, 32x128 when M is at most 32); a TC_BF16X3 member's
 * tiles split its operands into three per-row / per-column scaled BF16 terms
 * and multiply six term products on BF16 matrix cores (the split-precision
 * form of tc_contract, with the scales and terms formed inside the tile).
 * Work lists of (contraction, tile) pairs, longest tiles first, go to device
 * memory once, and the HIP graph that tc_batch_contract replays is captured
 * here: pointer staging from pinned host memory, counter reset, one
 * persistent kernel per group on up to four graph branches.  A TC_FP8X3
 * member runs its plan's own split and product launches in a branch, on the
 * plan's workspace: such a plan may appear once per batch and needs at most
 * 8192 contracted positions (TC_E_UNSUPPORTED otherwise).
 * Errors: TC_E_NULL, TC_E_UNSUPPORTED, TC_E_NOMEM, TC_E_HIP. */
tc_status tc_batch_create(tc_batch_t* out, const tc_plan_t* plans, int n);

/* Choose each member's candidate -- a loop/kernel variant (the fused GEMM
 * view, or a gemm member of the paper's family whose loops are all free
 * indices, Section 2) with a tile shape (128x128, 64x64, 32x128) -- the way
 * Section 3 predicts a member: micro-benchmarks of the tile kernel run after
 * the cache set-up a batch member meets (its operands cold: a remote region
 * of 5/4 of the device cache), median of ten, composed by tile counts into an
 * estimate per candidate.  The best `top_k` candidates by estimate are timed
 * on the device one member at a time (after the same set-up) and the fastest
 * picked.  The whole batch is then timed (graph replays) with those picks,
 * with the estimate's first choices and with the previous choices; a new set
 * replaces the kept one only if it beats two timings of it.  The kept choices
 * go to a process-wide tuning cache that later batches start from, and the
 * graph is captured again.  Uses --
 * and overwrites C with alpha * contract(A, B) of -- the operands of the
 * previous tc_batch_contract, which must have been made (members whose A or B
 * was NULL keep their choice).  Synchronous; allocates tuning scratch. */
tc_status tc_batch_tune(tc_batch_t batch, int top_k);

/* Run all contractions (each Section 1's definition, as in tc_contract):
 * C_t = alpha_t * contract(A_t, B_t) + beta_t * C_t.  A, B, C, alpha, beta are
 * host arrays of n entries (device pointers for the tensors, borrowed as in
 * tc_contract).  alpha_t == 0: A_t and B_t are not read (and may be NULL);
 * beta_t == 0: C_t is not read.  Writes the pointers and scalars to the
 * batch's pinned staging buffer and replays the graph captured by
 * tc_batch_create (or tc_batch_tune) on `stream`; allocates nothing.  The call
 * waits for the previous replay of this batch before restaging pointers.
 * Errors: TC_E_NULL, TC_E_ALIAS, TC_E_UNSUPPORTED, TC_E_HIP. */
tc_status tc_batch_contract(tc_batch_t batch, const void* const* A, const void* const* B,
                            void* const* C, const double* alpha, const double* beta, void* stream);

/* Scores of the tuner against exhaustive measurement (the paper's goal of
 * picking the fastest algorithm, Section 1 and the conclusions): for a seeded
 * sample of members, every candidate is timed alone after the batch's cache
 * set-up (median of five), and four choices are compared with the measured
 * best: the estimate's first choice, tc_batch_tune's pick among its top_k
 * timed alone, the choice it kept after timing whole batches, and the untuned
 * default (fused view, default shape).  A choice "hits" when it
 * measures within 5% of the best (several candidates can be about equally
 * fast); "argmin" counts exact picks of the fastest; the regret is the
 * geometric mean of time(choice) / time(best). */
typedef struct {
    int    n_sampled;
    double candidates_mean;        /* candidates (variant x shape) per sampled member */
    double within5_seed, argmin_seed, regret_seed;
    double within5_tuned, argmin_tuned, regret_tuned;
    double within5_default, argmin_default, regret_default;
    double member_best_share;      /* sampled members whose fastest candidate is a family member */
    double within5_topk, argmin_topk, regret_topk;   /* tc_batch_tune's pick among its top_k timed alone */
} tc_tune_score;

/* Score the current choices on `sample` members drawn with `seed` (see
 * tc_tune_score).  Uses -- and overwrites C of -- the previous
 * tc_batch_contract's operands, as tc_batch_tune does.  Synchronous.
 * Errors: TC_E_NULL, TC_E_UNSUPPORTED, TC_E_NOMEM, TC_E_HIP. */
tc_status tc_batch_score(tc_batch_t batch, int sample, uint64_t seed, tc_tune_score* out);

/* The candidate member `member` runs with: its variant (TC_VARIANT_FUSED or a
 * 0-based family member of its plan), tile shape (0: 128x128, 1: 64x64,
 * 2: 32x128) and how many candidates it has (a TC_BF16X3 member: the fused
 * view with three shapes; a TC_FP8X3 member: TC_VARIANT_FUSED, shape -1 and
 * no candidates).  Any output pointer may be NULL. */
tc_status tc_batch_choice(tc_batch_t batch, int member, int* variant, int* shape, int* n_candidates);

/* Make member `member` run candidate (variant, shape) -- variant
 * TC_VARIANT_FUSED or a family member of its plan that is a candidate (see
 * tc_batch_tune), shape 0..2 -- and capture the graph again.  Allocates
 * (work lists).  A TC_FP8X3 member has no candidates (TC_E_VARIANT).
 * Errors: TC_E_NULL, TC_E_VARIANT, TC_E_NOMEM, TC_E_HIP. */
tc_status tc_batch_set_choice(tc_batch_t batch, int member, int variant, int shape);

/* Members, work items (tiles), persistent-kernel groups and the within-5%
 * rate of the tuned choices in the last tc_batch_score (-1 before one).
 * Any pointer may be NULL. */
tc_status tc_batch_info(tc_batch_t batch, int* n_members, int64_t* n_tiles, int* n_groups, double* tune_hit_rate);

/* Free a batch (its graph, work lists and staging buffers).  NULL is
 * accepted.  (Lifetime of the batch object; no passage.) */
tc_status tc_batch_destroy(tc_batch_t batch);

/* --- errors (library conventions; no passage) ------------------------------- */
const char* tc_status_str(tc_status s);
const char* tc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TC_H */
