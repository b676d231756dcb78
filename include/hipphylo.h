/*
 * hipphylo - phylogenetic log-likelihoods and branch-length gradients on AMD Instinct MI355X.
 *
 * C ABI of the library.  The calls follow the paper's statement of the problem
 * (BEAGLE 4.1, Introduction and Key Improvements): a client sets tip states and
 * pattern weights, sets the eigensystem of the rate matrix, the category rates
 * and the stationary frequencies, updates the cached transition-probability
 * matrices P(t) = V exp(diag(lam) r t) V^-1 (Discussion: matrices come from an
 * eigendecomposition and are cached across patterns), updates post-order
 * partial likelihoods over an operation list (Felsenstein's pruning, cited in
 * the Introduction), integrates the root, and runs the pre-order traversal
 * whose partials give the gradient with respect to every branch length as a
 * pre . Q . post sandwich in one linear-time pass (Algorithmic advances;
 * Discussion).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns an int: HP_OK (0) or a negative HP_ERR_* code.  No C++
 *    exception crosses this boundary.  hp_last_error() returns the message of
 *    the most recent failure on an instance.
 *  - Node/buffer numbering: tips are 0..n_tips-1.  Post-order partial buffers
 *    are addressed as n_tips..n_tips+n_partials-1 (so a tree's internal node v
 *    can use post buffer v); pre-order partial buffers are 0..n_partials-1.
 *  - Partials are stored on the device as [category][pattern][state] with the
 *    pattern count padded (to a multiple of 128 for n_states <= 4, 192 for
 *    4 < n_states <= 64, none above)
 *    and the state count padded
 *    (hp_query HP_Q_STATE_PAD, HP_Q_PATTERN_PAD); padding patterns carry weight
 *    0 and an unknown state at every tip, so they contribute exactly nothing.
 *  - Device memory: the library never allocates device memory.  The caller
 *    sizes a workspace with hp_workspace_bytes, allocates it (any allocator) and
 *    passes it to hp_create; it must outlive the instance.  Host arrays passed to
 *    any call are borrowed for the duration of the call only (per-call arguments such
 *    as operation lists and branch lengths are copied into pinned staging before the
 *    call returns; the device copy is stream-ordered, so those calls do not wait for
 *    the device).
 *  - Streams: all device work is ordered on the instance's HIP stream
 *    (hp_set_stream).  Calls that return results in host memory synchronise that
 *    stream; the *_device variants only enqueue.
 *  - An instance is not thread-safe.  Distinct instances on distinct streams do
 *    not affect each other, and results are bitwise reproducible (all pattern
 *    sums are fixed-order two-stage FP64 reductions, no floating-point atomics).
 */
#ifndef HIPPHYLO_H
#define HIPPHYLO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
#define HP_OK               0
#define HP_ERR_ARG         -1  /* NULL pointer, bad count or malformed descriptor            */
#define HP_ERR_INDEX       -2  /* buffer, matrix, eigen, tip or gradient index out of range    */
#define HP_ERR_VALUE       -3  /* NaN/Inf/negative branch length or weight, state > S,
                                  frequencies not summing to 1 within 1e-9                    */
#define HP_ERR_UNSUPPORTED -4  /* state-count / precision / category-count combination        */
#define HP_ERR_WORKSPACE   -5  /* workspace missing, misaligned or smaller than required       */
#define HP_ERR_STATE       -6  /* a required input (eigensystem, tree, ...) was never set      */
#define HP_ERR_DEVICE      -7  /* a HIP runtime error; hp_last_error() carries its string      */
#define HP_ERR_NUMERIC     -8  /* a site likelihood was 0 or not finite (lnL written as -inf) */

/* ---------------------------------------------------------------- precisions */
#define HP_PREC_F64   0  /* partials and arithmetic in FP64                                    */
#define HP_PREC_F32   1  /* partials and arithmetic in FP32 (the plain single-precision form)  */
#define HP_PREC_BF16  2  /* partials stored in BF16, partials x P(t) on MFMA, FP32 accumulation */
#define HP_PREC_F16   3  /* partials stored in FP16, partials x P(t) on MFMA, FP32 accumulation */
#define HP_PREC_BF16X3 4 /* partials stored in FP32, partials x P(t) on the BF16 MFMA with both
                            operands split into hi + lo BF16 parts (three products per step:
                            hi.hi + hi.lo + lo.hi, ~2^-17 relative), FP32 accumulation     */

/* ---------------------------------------------------------------- rescaling policies
 * Rescaling multiplies a node's partials for one pattern by 2^-e, e being the
 * binary exponent of their maximum over categories and states, so the maximum
 * lands in [0.5, 1).  This is exact in binary floating point; the exponents of
 * post-order partials are accumulated per pattern in int32 and added back as
 * e * ln 2 at the root, those of pre-order partials cancel in the gradient. */
#define HP_SCALE_NONE          0  /* never rescale (FP64 on small trees)                     */
#define HP_SCALE_EVERY_NODE    1  /* rescale every post- and pre-order partial                */
#define HP_SCALE_EVERY_K_LEVELS 2 /* post: rescale a node once k internal nodes have been
                                     combined without rescaling along some path below it
                                     (every root-to-tip path is rescaled at least every k
                                     levels); pre: every node                               */

typedef struct hp_desc {
    int32_t n_tips;        /* N >= 2                                                    */
    int32_t n_patterns;    /* P >= 1                                                    */
    int32_t n_states;      /* S in [2, 64]                                              */
    int32_t n_categories;  /* K in [1, 8]                                               */
    int32_t n_partials;    /* post-order partial buffers (>= N-1 for hp_set_tree)       */
    int32_t n_matrices;    /* transition-matrix slots (>= 2N-2 for hp_set_tree)         */
    int32_t n_eigen;       /* eigensystem / frequency slots, >= 1                       */
    int32_t precision;     /* HP_PREC_*                                                 */
    int32_t scaling;       /* HP_SCALE_*                                                */
    int32_t scale_period;  /* k for HP_SCALE_EVERY_K_LEVELS (>= 1), ignored otherwise    */
    int32_t device;        /* HIP device ordinal the workspace lives on                 */
    int32_t n_pre_partials;/* pre-order partial buffers; 0 means n_partials.  hp_set_tree
                              reuses them as the pre-order walk frees them and needs only
                              hp_plan_pre_buffers() of them (about the tree's height), so
                              a whole-tree instance can size its workspace with that      */
    int32_t flags;         /* HP_FLAG_* bits (0: none)                                   */
} hp_desc;

/* Cache Q . post during the post-order traversal (Discussion: the product of the rate matrix
 * and the post-order partial at each node is cached in the post-order pass, so that the
 * gradient's sandwich needs S partial values instead of the S x S rate matrix).  For
 * 4 < n_states <= 64 (HP_ERR_UNSUPPORTED otherwise).  Every hp_update_post then also writes
 * w_v = Q post_v (Q of eigen slot 0, which must be set first) beside each destination
 * buffer, and hp_update_matrices also forms the tip columns (Q P_k(t))[:, s]; hp_pre_gradients
 * [_device] with eigen_idx 0 take each numerator as (P_c^T v_c) . w_c for an internal child and
 * v_c . (Q P_c)[:, s] for a tip, instead of forming Q P_c post_c.  The workspace grows by one
 * more post-order buffer (in the compute type: FP64, else FP32) per buffer and one tip table per
 * matrix slot.  Whole-tree calls do
 * not use the cache. */
#define HP_FLAG_QPOST_CACHE 1

typedef struct hp_instance hp_instance;

/* Post-order operation: dest = (P[mat1] child1) * (P[mat2] child2) per category and pattern.
 * child < n_tips reads that tip's states; otherwise it names a post buffer.  dest is a
 * post buffer index (>= n_tips).  rescale: 1 to rescale dest (its exponent joins the
 * cumulative exponent that every post buffer carries for its subtree), 0 not to. */
typedef struct hp_post_op {
    int32_t dest, child1, mat1, child2, mat2, rescale;
} hp_post_op;

/* Pre-order operation for one parent with two children.  parent_pre < 0 means the parent
 * is the root (its pre-order partial is the frequency vector); otherwise it names a pre
 * buffer.  childX_post names the child's post buffer or tip; matX the matrix of the edge
 * above the child; childX_pre the pre buffer that receives the child's pre-order partial
 * (< 0: not stored, e.g. for tips); gradX the slot of out_grad receiving the derivative of
 * lnL with respect to that edge's length (< 0: not computed).  Gradient slots must be
 * distinct within one list. */
typedef struct hp_pre_op {
    int32_t parent_pre;
    int32_t child1_post, mat1, child1_pre, grad1;
    int32_t child2_post, mat2, child2_pre, grad2;
} hp_pre_op;

/* ---------------------------------------------------------------- lifecycle */

/* Bytes of device workspace an instance with this descriptor needs (256-byte aligned): the
 * partial-likelihood buffers, transition matrices and model of one data set, the library
 * being an instance per data set or alignment block (Introduction; Benchmarks on NVIDIA and
 * AMD GPUs, one instance per device on a block of patterns). */
int hp_workspace_bytes(const hp_desc* desc, size_t* out_bytes);

/* (Introduction: the library is created per data set and then driven call by call.)
 * Create an instance on desc->device using the caller's workspace (device pointer,
 * 256-byte aligned, at least hp_workspace_bytes).  hip_stream may be NULL (the null
 * stream) or a hipStream_t.  Tip states start as "unknown", pattern weights as 1, the
 * category rates as 1 and the category weights as 1/K. */
int hp_create(const hp_desc* desc, void* dev_workspace, size_t workspace_bytes,
              void* hip_stream, hp_instance** out);
/* Release the instance (its host-side state; the caller frees the workspace). */
int hp_destroy(hp_instance* inst);
/* The stream all device work of the instance is ordered on (the library runs on a device
 * beside its client; Introduction).  Work already issued on the previous stream is completed
 * before the switch. */
int hp_set_stream(hp_instance* inst, void* hip_stream);

/* (Library plumbing, not from the paper.)  Copy the message of the last failed call on inst
 * (or of hp_create if inst is NULL)
 * into buf (always NUL-terminated when len > 0). */
int hp_last_error(const hp_instance* inst, char* buf, size_t len);

#define HP_Q_STATE_PAD      1
#define HP_Q_PATTERN_PAD    2
#define HP_Q_ELEMENT_BYTES  3
#define HP_Q_BLOCKS         4  /* pattern tiles (workgroups) one traversal launches   */
#define HP_Q_RUNTIME_VERSION 5 /* hipRuntimeGetVersion() of the runtime in use        */
#define HP_Q_TILE           6  /* patterns per traversal workgroup.  For n_states <= 4 it is
                                  64 or 128, chosen by hp_create from the device's occupancy
                                  so that the launch fills whole rounds of resident
                                  workgroups (environment HIPPHYLO_SMALL_PPL=1|2 forces
                                  64 or 128 patterns per workgroup); 16 otherwise        */
int hp_query(const hp_instance* inst, int what, int64_t* out);

/* ---------------------------------------------------------------- data */

/* The observed sequence data whose likelihood is computed (Introduction; Scaling by number
 * of taxa and site patterns: data are unique site patterns at the tips).
 * Tip states for one tip: states[n_patterns] with values 0..S-1, or S for unknown
 * (all-ones partial).  on_device != 0: states is a device pointer (copied stream-ordered,
 * not validated); otherwise a host pointer (validated, copied before return). */
int hp_set_tip_states(hp_instance* inst, int tip, const uint8_t* states, int on_device);
/* Pattern weights c_p >= 0 (host, FP64, n_patterns values; non-integers allowed): the count
 * of each unique site pattern, lnL = sum_p c_p l_p (Scaling by number of taxa and site
 * patterns). */
int hp_set_pattern_weights(hp_instance* inst, const double* weights);
/* Stationary frequencies of slot idx (host, FP64, S values, > 0, summing to 1 +- 1e-9): the
 * distribution at the root of the CTMC substitution model (Algorithmic advances). */
int hp_set_frequencies(hp_instance* inst, int idx, const double* pi);
/* Rate-category rates r_k >= 0 (host FP64, K values), shared by every matrix and slot: rate
 * heterogeneity across sites, each category a scaled copy of the CTMC (Discussion: the
 * matrices of a substitution model are cached and reused across patterns). */
int hp_set_category_rates(hp_instance* inst, const double* rates);
/* (The mixture over rate categories, as for the rates above.)
 * Category weights w_k >= 0 of slot idx (host FP64, K values; n_eigen slots, each 1/K at
 * creation).  The whole-tree calls use slot 0; the root and gradient calls name theirs. */
int hp_set_category_weights(hp_instance* inst, int idx, const double* weights);
/* (Discussion: transition matrices come from a numerical eigendecomposition of the rate
 * matrix.)  Eigensystem of slot idx: row-major S x S V and Vinv with Q = V diag(lam) Vinv
 * (host FP64).
 * The library also forms Q itself in FP64, for the gradient. */
int hp_set_eigen(hp_instance* inst, int idx, const double* V, const double* Vinv,
                 const double* lam);

/* ---------------------------------------------------------------- transition matrices */

/* (Discussion: the transition-probability matrices are formed from the eigendecomposition
 * and cached for reuse across patterns.)
 * For i < count: matrix slot mat_idx[i] <- P_k(t[i]) = V diag(exp(lam r_k t[i])) Vinv for
 * every category k, computed in FP64 and stored in the instance precision.  t: host FP64,
 * finite and >= 0 (HP_ERR_VALUE otherwise). */
int hp_update_matrices(hp_instance* inst, int eigen_idx, const int32_t* mat_idx,
                       const double* t, int count);

/* ---------------------------------------------------------------- traversals */

/* Post-order partial updates (Felsenstein's pruning, the post-order traversal; Introduction
 * and Algorithmic advances), in list order (children must be computed before use). */
int hp_update_post(hp_instance* inst, const hp_post_op* ops, int count);

/* Root integration (the likelihood at the root of Felsenstein's pruning; Introduction) of
 * post buffer root_buf with frequency slot freq_idx and category-weight slot catw_idx:
 *   l_p = ln(sum_k w_k sum_x pi_x post[k,p,x]) + E_p ln 2 ,  lnL = sum_p c_p l_p  (FP64),
 * E_p being the cumulative rescaling exponent the buffer carries for its subtree (every
 * post buffer holds its own, in place of separate scale buffers).
 * Blocking: writes *out_lnl and, if out_site_lnl != NULL, n_patterns values (host).
 * Returns HP_ERR_NUMERIC (and lnL = -inf) if some weighted site likelihood is 0 or
 * not finite. */
int hp_root_lnl(hp_instance* inst, int root_buf, int freq_idx, int catw_idx, double* out_lnl,
                double* out_site_lnl);
/* The same, stream-ordered into device memory: d_lnl (1 FP64) and, if d_site_lnl != NULL,
 * n_patterns FP64 site log-likelihoods.  Nothing waits for the device; a zero site
 * likelihood makes lnL -inf and raises the status word read by hp_status (HP_ERR_NUMERIC). */
int hp_root_lnl_device(hp_instance* inst, int root_buf, int freq_idx, int catw_idx, double* d_lnl,
                       double* d_site_lnl);

/* Pre-order partial updates (no gradients), in list order (parents before children):
 * pre_c = P_c^T (pre_n o P_s post_s) for child c of n with sibling s, pre_root = pi (the
 * pre-order traversal that complements the post-order one; Key Improvements, Algorithmic
 * advances).  Rescaled per pattern when the instance rescales; those exponents cancel in
 * the gradient and are not kept. */
int hp_update_pre(hp_instance* inst, const hp_pre_op* ops, int count, int freq_idx);

/* Pre-order partial updates fused with the branch-length gradients (the sandwich of a
 * pre-order partial, the rate matrix and a post-order partial, evaluated for every branch
 * in one pre-order traversal; Key Improvements, Algorithmic advances; Discussion) of the
 * model whose rate matrix comes from eigen slot eigen_idx, with category-weight slot
 * catw_idx: for every child c with gradX >= 0,
 *   out_grad[gradX] = sum_p c_p [sum_k w_k r_k pre_c^T Q post_c] / [sum_k w_k pre_c^T post_c]
 * Blocking; out_grad is host memory of n_grad FP64 values, slots not named by the list
 * are set to 0. */
int hp_pre_gradients(hp_instance* inst, const hp_pre_op* ops, int count, int freq_idx,
                     int catw_idx, int eigen_idx, double* out_grad, int n_grad);

/* Stream-ordered form of hp_pre_gradients: d_grad is device memory of n_grad FP64 values
 * and the list's gradients are added to it (slots the list does not name gain +0), so the
 * batches of one backward pass accumulate into one vector.  Nothing waits for the device;
 * the operation list is copied before return. */
int hp_pre_gradients_device(hp_instance* inst, const hp_pre_op* ops, int count, int freq_idx,
                            int catw_idx, int eigen_idx, double* d_grad, int n_grad);

/* A list mixing post-order and pre-order operations, taken in order in one launch, with the
 * pre-order operations' branch gradients added into d_grad as by hp_pre_gradients_device: a
 * backward pass that recomputes post-order partials right before the pre-order operations
 * that read them, so that only some post-order partials need be kept between the passes
 * (the pre-order traversal of Algorithmic advances; Discussion: caching strategies during
 * the post- and pre-order traversals).  ops: count entries of 10 int32 each: a kind (0: a
 * post-order operation, fields hp_post_op; 1: a pre-order operation, fields hp_pre_op) and
 * its fields, unused trailing fields ignored; validated as those operations are, gradient
 * slots distinct over the list.  n_states <= 64 (HP_ERR_UNSUPPORTED on the eigensystem path).
 * Stream-ordered; the list is copied before return. */
int hp_traverse_gradients_device(hp_instance* inst, const int32_t* ops, int count, int freq_idx,
                                 int catw_idx, int eigen_idx, double* d_grad, int n_grad);

/* ---------------------------------------------------------------- whole-tree evaluation */

/* (The post- and pre-order traversals of one tree; Algorithmic advances.)
 * Fix the tree used by hp_evaluate*: children[2N-1][2] (row-major int32) in the standard
 * numbering (tips 0..N-1, internal N..2N-2, root 2N-2; tips have -1 children).  Internal
 * node v uses post buffer v and pre buffer v-N; branch c (the edge above node c) uses
 * matrix slot c and gradient slot c.  Builds and uploads the operation lists and the
 * rescaling plan once. */
int hp_set_tree(hp_instance* inst, const int32_t* children);

/* (The traversal orders of Algorithmic advances, as operation lists.)
 * Host-only: the operation lists hp_set_tree builds for a children table, for inspection or
 * for driving the operation-level calls.  out_post_ops receives N-1 hp_post_op (post-order,
 * children first, with the rescale flags of the given policy) and out_pre_ops N-1 hp_pre_op
 * (parents first).  Touches no device; the error message is read with hp_last_error(NULL). */
int hp_plan_tree(int n_tips, const int32_t* children, int scaling, int scale_period,
                 int32_t* out_post_ops, int32_t* out_pre_ops);

/* (Discussion: caching strategies during the post- and pre-order traversals.)
 * Host-only: the number of pre-order buffers hp_set_tree's operation lists use for this
 * tree.  A pre-order partial lives from its parent's operation to its own, and the list
 * visits the tree depth-first, so buffers are handed out from a free list and the count is
 * bounded by the tree's height + 1 (the whole-tree lists need it in n_pre_partials). */
int hp_plan_pre_buffers(int n_tips, const int32_t* children, int* out_count);

/* The likelihood and its gradient with respect to every branch length in one post-order and
 * one pre-order traversal (Algorithmic advances: linear in the number of tips; Scaling by
 * number of taxa and site patterns: the lnL + gradient evaluation the HMC runs time).
 * One full evaluation on the tree of hp_set_tree with model slot 0: transition matrices
 * for all 2N-2 branches from t (FP64, 2N-2 values, indexed by node), post-order partials,
 * root integration, and, if want_grad, pre-order partials and all 2N-2 branch gradients.
 * Host pointers; blocking.  grad may be NULL when want_grad == 0.  A small 4-state problem
 * with gradients (at most 64 taxa and 64 workgroups of 64 patterns, its matrices fitting one
 * workgroup's LDS) runs as one kernel launch that takes t by value; each workgroup writes its
 * pattern sums and then its own status word to pinned host memory, and the call returns once
 * every workgroup's word has arrived, after adding the sums on the host in the fixed order of
 * the reduction kernel (bitwise equal to the three-launch form).  It leaves no partials or
 * matrices in the workspace and neither reads nor clears the device status word. */
int hp_evaluate(hp_instance* inst, const double* t, int want_grad, double* out_lnl,
                double* out_grad);

/* (As hp_evaluate; Algorithmic advances.)
 * The same evaluation, fully stream-ordered: d_t (2N-2 FP64 branch lengths), d_out
 * (1 + 2N-2 FP64: lnL then gradients) are device pointers; nothing is synchronised.
 * Branch lengths are validated on the device: a negative or non-finite length makes the
 * output NaN and raises the status word read by hp_status (HP_ERR_VALUE). */
int hp_evaluate_device(hp_instance* inst, const double* d_t, int want_grad, double* d_out);

/* For callers that cannot allocate device memory or host staging at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the evaluation
 * of hp_evaluate_device with its reduction scratch - the per-workgroup FP64 partial sums of
 * lnL and of every gradient that a second kernel adds up in a fixed order - taken from a
 * static device array of the library (16 MiB on each GPU the library runs on, held until
 * the process ends) instead of the instance's workspace.  Same arguments, same kernels and
 * bitwise the same results as hp_evaluate_device; stream-ordered, nothing is allocated or
 * synchronised.  Evaluations needing more than 16 MiB of rows ((1 + 2N-2) x the launch's
 * workgroups x 8 bytes with gradients, 8 bytes per workgroup without) are rejected with
 * HP_ERR_WORKSPACE before anything is enqueued; more than 64 states is HP_ERR_UNSUPPORTED.
 * Every call on one GPU shares that GPU's array: calls whose work overlaps on the device
 * (other streams, other host threads) race and must be serialised by the caller. */
int hp_evaluate_device_noalloc(hp_instance* inst, const double* d_t, int want_grad, double* d_out);

/* (The pre-order traversal with the gradient sandwich; Algorithmic advances, Discussion.)
 * Pre-order partials and all 2N-2 branch gradients of the tree of hp_set_tree from the
 * post-order partials and transition matrices left by the preceding
 * hp_evaluate_device(want_grad = 0) on this instance (the "store" form of a backward pass:
 * nothing from the forward pass is recomputed).  d_grad: device pointer, 2N-2 FP64 values
 * indexed by node.  Stream-ordered; the caller must not have changed the partials or the
 * matrices in between (the library cannot detect it). */
int hp_gradients_device(hp_instance* inst, double* d_grad);

/* Approximate gradient of lnL with respect to every entry Q_ij of the rate matrix of model
 * slot 0, for random-effects substitution models (Key Improvements, Algorithmic advances:
 * the gradient with respect to the rate-matrix entries, with the derivative of each matrix
 * exponential taken to first order).  With dP_k(t)/dQ_ij ~= r_k t E_ij P_k(t) (E_ij: the
 * matrix unit at (i, j)), each branch c contributes through its own matrix:
 *     G_ij = sum_c t_c sum_p c_p [sum_k w_k r_k (top_c)_i (u_c)_j] / [sum_k w_k top_c . u_c]
 * with u_c = P_k(t_c) post_c and top_c = pre_n o (P_k(t_s) post_s), n the parent and s the
 * sibling of c.  Every entry is treated as free, the diagonal included; the client applies
 * the chain rule to its model's parameters (and to the rate normalisation, if any).
 * One whole-tree evaluation as hp_evaluate with want_grad = 1, plus G: out_lnl (1),
 * out_grad (2N-2, by node) and out_rate_grad (S*S, row-major), host pointers, blocking.
 * For n_states > 4 the products that form G run on the matrix cores (BF16 operands on the
 * BF16/FP16 paths); FP64 with n_states > 32 and n_categories > 4 is HP_ERR_UNSUPPORTED. */
int hp_evaluate_rate_gradient(hp_instance* inst, const double* t, double* out_lnl, double* out_grad,
                              double* out_rate_grad);
/* The same, stream-ordered on device pointers: d_t (2N-2 FP64) and d_out (1 + 2N-2 + S*S FP64:
 * lnL, branch gradients, G row-major).  Nothing is synchronised; errors via hp_status. */
int hp_evaluate_rate_gradient_device(hp_instance* inst, const double* d_t, double* d_out);

/* ---------------------------------------------------------------- batched evaluation
 * Whole-tree evaluations of up to HP_MAX_BATCH instances in one launch per kernel (matrix
 * assembly, traversal, reduction), for serving many clients (Benchmarks on NVIDIA and AMD
 * GPUs: independent instances evaluate independent blocks of patterns at once).  The instances must share
 * device, precision, state padding, category count and tile (HP_Q_TILE), must each have had hp_set_tree and
 * model slot 0 set, and may each appear only once; their trees, pattern counts and models
 * may differ.  d_t[i] (2N_i-2 FP64) and d_out[i] (1 + 2N_i-2 FP64 with gradients, else 1)
 * are device pointers.  Work is enqueued on hip_stream (not on the instances' streams) and
 * nothing is synchronised; each instance's device status is checked with hp_status.
 * Results are bitwise identical to hp_evaluate_device of each instance alone.  Errors are
 * read with hp_last_error(NULL). */
#define HP_MAX_BATCH 32
int hp_batch_evaluate_device(hp_instance* const* insts, const double* const* d_t,
                             double* const* d_out, int n, int want_grad, void* hip_stream);

/* (Library plumbing, not from the paper.)
 * Synchronise the stream and return (then clear) the device-side status of work enqueued
 * since the last call: HP_OK, HP_ERR_VALUE or HP_ERR_NUMERIC. */
int hp_status(hp_instance* inst);

/* ---------------------------------------------------------------- kernel timing
 * The paper measures the time spent inside the library.  While enabled, every kernel an
 * instance launches is bracketed by HIP events on its stream (a few microseconds of
 * overhead per launch).  hp_profile_read synchronises the stream and returns, per kernel
 * class, the summed milliseconds and launch counts since the last read, then resets them. */
#define HP_KERNEL_PMAT       0  /* transition-matrix assembly                          */
#define HP_KERNEL_TRAVERSAL  1  /* post-/pre-order partials, root and gradient sums    */
#define HP_KERNEL_REDUCE     2  /* second stage of the pattern reductions              */
#define HP_KERNEL_CLASSES    3
int hp_profile(hp_instance* inst, int enable);
int hp_profile_read(hp_instance* inst, double* out_ms, int64_t* out_count);

#ifdef __cplusplus
}
#endif

#endif /* HIPPHYLO_H */
