/*
 * fmm.h -- C-ABI of the MI355X (gfx950) fast multipole library for 3D Laplace
 * potentials and forces, after Yokota & Barba, "Hierarchical N-body
 * simulations with auto-tuning for heterogeneous systems" (arXiv 1108.5815).
 *
 * What is computed (paper: introduction; "Results", Laplace potential and
 * force): for N particles with positions x_i and charges q_i,
 *     phi_i = sum_{j != i, x_j != x_i} q_j / |x_i - x_j|
 *     E_i   = -grad phi_i = sum_{j != i, x_j != x_i} q_j (x_i - x_j) / |x_i - x_j|^3
 * approximated by a hierarchical method: adaptive octree (cells hold at most
 * ncrit particles), dual tree traversal with the acceptance criterion
 * theta = (r_t + r_s)/R ("Dual tree traversal"; "Results"), and spherical
 * harmonic expansions of order p (degrees 0..p) for the far field, with
 * particle-particle sums for the near field.
 *
 * Conventions shared by every entry point
 *  - A context owns every internal device buffer and is bound to one device
 *    and one HIP stream.  All device work is enqueued on that stream.
 *  - Pointers named "device" must be device (or managed) memory readable by
 *    the context's device; pointers named "host" are ordinary host memory.
 *  - Arrays are structure-of-arrays, one value per particle, in the caller's
 *    particle order, contiguous, of the element type named by the dtype
 *    argument (FMM_F32 = float, FMM_F64 = double).
 *  - Every call returns an fmm_status and never aborts.  On error the context
 *    stays valid; fmm_last_error() returns a message owned by the context,
 *    valid until the next call on it.  A context is not thread-safe; distinct
 *    contexts are independent.
 */
#ifndef FMM_H_
#define FMM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_ctx_s *fmm_ctx;

typedef enum {
    FMM_OK = 0,
    FMM_ERR_INVALID_ARG = 1,   /* bad size, pointer, parameter or non-finite input */
    FMM_ERR_OUT_OF_MEMORY = 2, /* a device allocation failed */
    FMM_ERR_DEVICE = 3,        /* a HIP call or kernel launch failed */
    FMM_ERR_STATE = 4,         /* call made out of order (e.g. evaluate before traverse) */
    FMM_ERR_UNSUPPORTED = 5    /* valid request this build does not implement */
} fmm_status;

/* Choice of interaction for each accepted cell pair ("Kernel pre-calculation";
 * "Results"): the FMM always converts multipoles into local expansions
 * (cell-cell, M2L); the treecode always evaluates multipoles at the target
 * particles (cell-particle, M2P); the hybrid picks, per pair, the kind of
 * smallest modelled time among M2L, M2P and particle-particle (P2P). */
typedef enum {
    FMM_POLICY_FMM = 0,
    FMM_POLICY_TREECODE = 1,
    FMM_POLICY_HYBRID_TIMED = 2, /* unit costs from fmm_tune() or fmm_set_costs() */
    FMM_POLICY_HYBRID_MLP = 3    /* learned cost model, with the timed unit costs (when set) as its
                                    fallback: they decide the pairs whose two least predicted costs
                                    lie within 1/8 (log2 units) of each other, and every pair when
                                    no model is loaded */
} fmm_policy;

typedef enum {
    FMM_PREC_FP32 = 0,       /* FP32 kernels, FP64 per-target final sum */
    FMM_PREC_SPLIT_BF16 = 1  /* as FP32, but same-level M2L as BF16 products on the
                                matrix cores with FP32 accumulation, graded by multipole
                                degree: hi*hi + hi*lo + lo*hi for coefficient index
                                k < 32, hi*hi + hi*lo below 48, hi*hi above; p <= 12 */
} fmm_precision;
/* There is no FP64 evaluation form: FP64 inputs and outputs are accepted
 * (FMM_F64), the quantisation and the per-target final sum are FP64, and the
 * expansion and particle-particle arithmetic is FP32.  Its rounding (about
 * 1e-7 relative) bounds the attainable accuracy: orders whose truncation
 * error lies below that gain nothing.  Any other precision value gives
 * FMM_ERR_INVALID_ARG. */

typedef enum { FMM_F32 = 0, FMM_F64 = 1 } fmm_dtype;

/* Expansion family of the far field (paper: "Hybrid treecode/FMM
 * algorithm": spherical-harmonic kernels with the ability to switch to
 * Cartesian expansions when the required accuracy is low; "Introduction to
 * treecodes & FMM": treecodes use Taylor series in Cartesian coordinates,
 * typically p = 3).  Spherical: Greengard-Rokhlin harmonics, (p+1)^2
 * coefficients, any p <= FMM_P_MAX.  Cartesian: Taylor coefficients of
 * 1/|x - y| in multi-indices |k| <= p, (p+1)(p+2)(p+3)/6 coefficients,
 * p <= 6, M2L truncated at |m| + |k| <= p.  Auto: Cartesian for the orders
 * up to a given one (the low-accuracy range), spherical above. */
typedef enum {
    FMM_EXPANSION_SPHERICAL = 0,
    FMM_EXPANSION_CARTESIAN = 1,
    FMM_EXPANSION_AUTO = 2
} fmm_expansion;

enum { FMM_LIST_M2L = 0, FMM_LIST_M2P = 1, FMM_LIST_P2P = 2 };

/* Largest supported expansion order. */
#define FMM_P_MAX 16

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the handle. */
fmm_status fmm_create(fmm_ctx *out, int device, void *hip_stream);

/* Release every buffer of the context.  NULL is accepted. */
void fmm_destroy(fmm_ctx ctx);

/* Message of the last failed call on ctx ("" if none). */
const char *fmm_last_error(fmm_ctx ctx);

/* Re-bind the context to another stream of the same device. */
fmm_status fmm_set_stream(fmm_ctx ctx, void *hip_stream);

/*
 * Device-memory hook for the context's internal buffers (tree, lists,
 * expansions, tables, work space).  alloc(bytes, user) returns device memory
 * of the context's device aligned to at least 256 bytes, or NULL on failure;
 * free_fn(ptr, user) releases it.  The context calls both from the thread
 * that makes the fmm_* call, and synchronises its stream before freeing.
 * Passing alloc = free_fn = NULL restores hipMalloc / hipFree.  Buffers
 * already held keep the routine that allocated them and are released by it.
 * A NULL return turns the call that needed the memory into
 * FMM_ERR_OUT_OF_MEMORY; the context stays valid and a later call may retry.
 * Setting only one of the two routines gives FMM_ERR_INVALID_ARG.
 */
typedef void *(*fmm_alloc_fn)(size_t bytes, void *user);
typedef void (*fmm_free_fn)(void *ptr, void *user);
fmm_status fmm_set_allocator(fmm_ctx ctx, fmm_alloc_fn alloc, fmm_free_fn free_fn, void *user);

/*
 * Tree build (paper: "Hierarchical N-body algorithms", clustering into a
 * hierarchy of cells; "Results", N_crit is the maximum number of particles
 * per cell).
 *   n            number of particles, 0 <= n < 2^31 (n = 0 is a no-op)
 *   dtype        element type of x, y, z, q
 *   x, y, z, q   device arrays of n values; read during the call and copied
 *                into the context (Morton-sorted), so they may be reused or
 *                freed once the context's stream has passed this call
 *   ncrit        leaf capacity, >= 1: a cell holding more than ncrit particles
 *                splits into its non-empty octants (not below level 21)
 * The bounding cube is anchored at the minimum corner with side equal to the
 * largest extent; coordinates are quantised to 21 bits per axis in FP64 and
 * interleaved into 63-bit Morton keys (x lowest).  Particles are sorted by
 * (key, original index).  Non-finite coordinates give FMM_ERR_INVALID_ARG.
 * Synchronises the stream once per tree level.
 */
fmm_status fmm_build_tree(fmm_ctx ctx, int64_t n, int dtype, const void *x, const void *y,
                          const void *z, const void *q, int32_t ncrit);

/*
 * Targets that differ from the sources (paper: "Dual tree traversal": the
 * traversal pairs a target tree with a source tree, and the method also
 * handles targets and sources that are not the same particles).  Builds a
 * target tree over (tx, ty, tz) and a source tree over (sx, sy, sz) with
 * charges q, both inside one bounding cube (that of all the points, as
 * fmm_build_tree would give it), each sorted and split as fmm_build_tree
 * does.  fmm_traverse then starts from the pair (target root, source root),
 * so every list pairs a target-tree cell with a source-tree cell, and
 * fmm_evaluate writes the potential and field at the n_targets targets due to
 * all sources (a source at the same point as a target is skipped).
 *   n_targets, n_sources  >= 0, sum < 2^31 (either may be 0)
 *   tx, ty, tz            device arrays of n_targets values
 *   sx, sy, sz, q         device arrays of n_sources values
 * Copies the inputs into the context (they may be reused once the stream
 * has passed the call).  Introspection reports the two trees as a forest:
 * the target root is cell 0 and the source root cell 1 (when both sets are
 * non-empty); keys and permutation cover the targets then the sources.
 * Errors as fmm_build_tree.
 */
fmm_status fmm_build_tree_ts(fmm_ctx ctx, int dtype, int64_t n_targets, const void *tx, const void *ty,
                             const void *tz, int64_t n_sources, const void *sx, const void *sy, const void *sz,
                             const void *q, int32_t ncrit);

/*
 * Dual tree traversal (paper: "Dual tree traversal"; "Results" for the
 * criterion): from the root pair, the larger cell of each pair is split
 * (both when of equal size); a new pair is accepted when
 * (r_t + r_s)^2 <= theta^2 R^2 with r the half side of each cube and R the
 * distance between cube centres; a pair of leaves that is not accepted is a
 * particle-particle interaction; any other pair is split again.  Accepted
 * pairs get M2L, M2P or P2P by `policy`.
 *   p      expansion order, 0 <= p <= FMM_P_MAX (degrees 0..p)
 *   theta  in (0, 1)
 * Requires a built tree.  Synchronises the stream once per traversal level.
 */
fmm_status fmm_traverse(fmm_ctx ctx, int32_t p, double theta, int32_t policy);

/*
 * Evaluation (paper: "Hierarchical N-body algorithms" for the upward and
 * downward passes of the FMM and the treecode; "Hybrid treecode/FMM
 * algorithm" and "Results" for the cell-cell, cell-particle and
 * particle-particle interactions of the lists): P2M at leaves, M2M upward,
 * M2L / M2P / P2P over the lists, L2L downward, L2P at leaves, and the
 * per-target sum, written in the caller's original particle order.
 *   precision  an fmm_precision
 *   out_dtype  element type of the outputs (FMM_F32 or FMM_F64)
 *   phi, ex, ey, ez  device arrays of n values (caller-owned); E = -grad phi;
 *              n_targets values after fmm_build_tree_ts; may be NULL when
 *              that count is zero, else NULL is FMM_ERR_INVALID_ARG
 * Requires a completed traversal.  Asynchronous on the context stream.
 */
fmm_status fmm_evaluate(fmm_ctx ctx, int32_t precision, int32_t out_dtype, void *phi, void *ex,
                        void *ey, void *ez);

/*
 * fmm_evaluate for callers that cannot allocate device memory: code under
 * stream (graph) capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, kernels and results (bit for bit) as
 * fmm_evaluate, but every work buffer of the evaluation (expansions,
 * near-field partials, GEMM and class partials, flags) lies in one fixed
 * work area of FMM_NOALLOC_SCRATCH_BYTES per device, which the library holds
 * from its first context on that device until the process ends; the call
 * makes no device or host allocation.  The tree, lists and operator tables
 * come from the context (fmm_build_tree / fmm_traverse, which do allocate).
 * Every kernel runs in order on the context stream (no second stream).
 * The area is shared by every context and call on the device and keeps the
 * last call's contents: calls that overlap on one device race, so callers
 * must order them (one stream, or events).  fmm_get_expansions does not see
 * this call's expansions.  An evaluation needing more work space than the
 * area (at most 33 bytes per particle plus 4 (G + 3) K bytes per cell, with
 * K = (p+1)^2 rounded up to a multiple of 32 and G = 8 slot groups at
 * theta = 0.5, 16 at theta = 0.4: roughly 290k uniform particles at p = 10,
 * theta = 0.5, ncrit = 64) gives FMM_ERR_INVALID_ARG with the sizes in the
 * message; other errors as fmm_evaluate.
 */
#define FMM_NOALLOC_SCRATCH_BYTES (64u << 20)
fmm_status fmm_evaluate_noalloc(fmm_ctx ctx, int32_t precision, int32_t out_dtype, void *phi, void *ex,
                                void *ey, void *ez);

/*
 * Batches of independent problems of uneven size (many instances evaluated
 * together so that each phase is one pass over all of them):
 * instance k owns particles [offsets[k], offsets[k+1]) of x, y, z, q and no
 * interaction crosses instances.  Each instance gets its own bounding cube,
 * Morton keys and root exactly as fmm_build_tree would give it alone, so its
 * cells, lists and results are those of a build of that instance by itself.
 * fmm_traverse and fmm_evaluate then work on the whole forest.
 *   n_inst        >= 1
 *   offsets_host  n_inst + 1 non-decreasing values, offsets[0] = 0,
 *                 offsets[n_inst] = total particles < 2^31; empty instances
 *                 are allowed
 * Other arguments and errors as fmm_build_tree.  Introspection then reports
 * the forest: cells of all instances (the roots first, in instance order),
 * keys sorted by (instance, key, original index), lists over all instances.
 */
fmm_status fmm_build_tree_batch(fmm_ctx ctx, int32_t n_inst, const int64_t *offsets_host, int dtype,
                                const void *x, const void *y, const void *z, const void *q, int32_t ncrit);

/* fmm_build_tree_batch, fmm_traverse and fmm_evaluate in one call; outputs
 * are device arrays of offsets[n_inst] values in the input order. */
fmm_status fmm_evaluate_batch(fmm_ctx ctx, int32_t n_inst, const int64_t *offsets_host, int dtype,
                              const void *x, const void *y, const void *z, const void *q, int32_t ncrit,
                              int32_t p, double theta, int32_t policy, int32_t precision, int32_t out_dtype,
                              void *phi, void *ex, void *ey, void *ez);

/*
 * Expansion family of the following traversals (and their evaluations):
 * FMM_EXPANSION_SPHERICAL (the default), FMM_EXPANSION_CARTESIAN (then
 * fmm_traverse gives FMM_ERR_UNSUPPORTED for p > 6), or FMM_EXPANSION_AUTO,
 * which takes the Cartesian family when p <= auto_cartesian_max_p (in
 * [-1, 6]; -1 never; ignored for the other two) and the spherical one
 * otherwise.  The family is fixed at fmm_traverse; fmm_get_expansion
 * reports the family of the last traversal.  Both families give the method
 * its usual accuracy at a given (p, theta); the Cartesian M2L truncation
 * (|m| + |k| <= p) is somewhat looser than the spherical one.
 */
fmm_status fmm_set_expansion(fmm_ctx ctx, int32_t expansion, int32_t auto_cartesian_max_p);
fmm_status fmm_get_expansion(fmm_ctx ctx, int32_t *family);

/*
 * M2L of the accepted cell pairs outside the batched same-level GEMM (mixed
 * levels, or same-level pairs whose parents were at different levels): the
 * paper chooses between translation schemes per pair ("Dual tree
 * traversal": rotation-based or plane-wave translations; "Introduction to
 * treecodes & FMM": fast translations cost p^4 or less instead of p^6).
 *   FMM_M2L_CLASS_DENSE    (default) pairs grouped by (level difference,
 *                          offset) into classes, one operator per class and
 *                          matrix-core products per class; pairs outside the
 *                          class key one by one with the dense O(p^4) kernel
 *   FMM_M2L_CLASS_ROTATION as above, the pairs outside the key by rotation
 *   FMM_M2L_PAIR_DENSE     every such pair one by one, dense
 *   FMM_M2L_PAIR_ROTATION  every such pair one by one by rotation: the
 *                          multipole rotated to the offset's axis, translated
 *                          along it (orders m decouple), rotated back, O(p^3)
 * The Cartesian family always takes the class products and its dense
 * per-pair kernel.  Results differ by rounding only.  fmm_autotune times the
 * four on the current lists and keeps the fastest.  Setting it after a
 * traversal regroups that traversal's pairs.
 */
enum {
    FMM_M2L_CLASS_DENSE = 0,
    FMM_M2L_CLASS_ROTATION = 1,
    FMM_M2L_PAIR_DENSE = 2,
    FMM_M2L_PAIR_ROTATION = 3
};
fmm_status fmm_set_m2l_kernel(fmm_ctx ctx, int32_t kind);
fmm_status fmm_get_m2l_kernel(fmm_ctx ctx, int32_t *kind);

/*
 * Unit costs of the timed hybrid (paper: "Kernel pre-calculation"): the
 * modelled time of an accepted pair is c_m2l for M2L, c_m2p * n_t for M2P and
 * (c_p2p * n_t) * n_s for P2P (n_t, n_s = particles of the target and source
 * cell, FP64); the least wins, ties go to M2L, then M2P.  All > 0.
 */
fmm_status fmm_set_costs(fmm_ctx ctx, double c_m2l, double c_m2p, double c_p2p);
fmm_status fmm_get_costs(fmm_ctx ctx, double *costs3_host);

/*
 * Kernel pre-calculation (paper: "Kernel pre-calculation"): time the M2L, M2P
 * and P2P kernels on artificial coordinates, charges and expansions at order
 * p and store the unit costs used by FMM_POLICY_HYBRID_TIMED.  Needs no tree.
 */
fmm_status fmm_tune(fmm_ctx ctx, int32_t p, int32_t precision);

/* ---------------- learned cost model (FMM_POLICY_HYBRID_MLP) ----------------
 * A 6 -> 64 -> 64 -> 3 ReLU perceptron (FP32, FMM_MLP_PARAMS weights laid out
 * W1[64][6], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]) predicts log2 of
 * the time in ns that an accepted cell pair costs as M2L, M2P or P2P; the
 * traversal picks the least.  Pair features: log2(r_t/r_s)/2, log2(n_t)/8,
 * log2(n_s)/8, p/10, ((r_t+r_s)/R)/theta, theta.  This replaces the fixed
 * unit costs of the kernel pre-calculation ("Kernel pre-calculation"), which
 * on GPUs mispredict because kernel time is not proportional to problem size
 * ("Results").  The network is evaluated once per (p, theta, weights) over a
 * quantised feature grid (level difference in [-4, 4], log2 counts in
 * quarter steps, 4 bins of the distance ratio) that the traversal reads. */
#define FMM_MLP_PARAMS 4803

/* Generate timing records with the library's own kernels on artificial
 * clustered particle sets (homogeneous leaves of 2..128 particles; a
 * two-level set for mixed-level M2L; target and source trees with 4x fewer
 * or more particles per source leaf for P2P off the diagonal; the rest of
 * the feature grid from how each kind's work scales),
 * then train on the GPU with the library's forward/backward/Adam kernels
 * (full batch, `epochs` steps, step 3e-2 decayed by a cosine to 1/20 of it,
 * weights initialised from `seed`).  Enables
 * FMM_POLICY_HYBRID_MLP.  The timings are taken with the M2L kernel of
 * `precision` (FMM_PREC_FP32 or FMM_PREC_SPLIT_BF16), which evaluations using
 * the model should then use.  *final_loss (may be NULL) receives the mean
 * squared error of the log2 times.  Needs no tree; leaves the context's tree
 * intact. */
fmm_status fmm_costmodel_train(fmm_ctx ctx, int32_t p, double theta, int32_t precision, int32_t epochs,
                               uint64_t seed, double *final_loss);

/* Train on caller-given records (host arrays): features[n_rec][6],
 * kinds[n_rec] in {0 M2L, 1 M2P, 2 P2P}, targets[n_rec] = log2 ns; Adam
 * with step lr at the first epoch, decayed by a cosine to lr / 20. */
fmm_status fmm_costmodel_fit(fmm_ctx ctx, int32_t n_rec, const float *features, const int32_t *kinds,
                             const float *targets, int32_t epochs, double lr, uint64_t seed,
                             double *final_loss);

/* The records of the last fmm_costmodel_train (host arrays of cap entries;
 * *count receives the number available). */
fmm_status fmm_costmodel_records(fmm_ctx ctx, int32_t cap, int32_t *count, float *features, int32_t *kinds,
                                 float *targets);

/* Weights in and out (host arrays of FMM_MLP_PARAMS floats). */
fmm_status fmm_costmodel_get_weights(fmm_ctx ctx, float *weights);
fmm_status fmm_costmodel_set_weights(fmm_ctx ctx, const float *weights);

/* One evaluation of the training kernels: mean squared error (*loss) of
 * log2 times and its gradient (grad[FMM_MLP_PARAMS]) for the given weights
 * and records (all host arrays). */
fmm_status fmm_costmodel_loss_grad(fmm_ctx ctx, const float *weights, int32_t n_rec, const float *features,
                                   const int32_t *kinds, const float *targets, float *loss, float *grad);

/*
 * Persist the cost model: a versioned text file holding the weights (exact,
 * as hexadecimal floats), the order, theta and precision it was trained for
 * (-1 where unknown, e.g. after fmm_costmodel_set_weights), the name of the
 * device whose kernel timings trained it, the final training loss, the
 * timed unit costs (if set) and the tile shapes, schedule, M2L kernel kind
 * (fmm_set_m2l_kernel) and M2L tile width (fmm_set_m2l_tile) in use.  This keeps the learned choices of a device fixed across processes, where
 * retraining on fresh timings would give slightly different choices.
 * save: FMM_ERR_STATE without a model, FMM_ERR_DEVICE if the file cannot be
 * written.  load(path, p, precision): the file must come from a device of
 * the same name and, unless the argument is -1, have been trained for that
 * order and precision; otherwise FMM_ERR_INVALID_ARG (also for a missing,
 * unreadable or malformed file, or another format version) and the context
 * keeps its model.  On success the weights, unit costs (when the file has
 * them), tile shapes, schedule, M2L kernel kind and tile width (when the
 * file has them) replace the context's.
 */
fmm_status fmm_costmodel_save(fmm_ctx ctx, const char *path);
fmm_status fmm_costmodel_load(fmm_ctx ctx, const char *path, int32_t p, int32_t precision);

/* The choice table the traversal reads for (p, theta): 9 x 81 x 81 x 4
 * entries (level difference + 4, quarter-octave bucket of n_t, of n_s,
 * distance-ratio bin), each 0 M2L, 1 M2P or 2 P2P; host array.  With unit
 * costs set, an entry whose two least predictions (log2 ns) differ by less
 * than 1/8 holds the timed choice at the bucket's counts n = 2^(bucket/4)
 * (c_m2l, c_m2p n_t, (c_p2p n_t) n_s in FP64; least wins, ties to M2L, then
 * M2P). */
#define FMM_MLP_TABLE (9 * 81 * 81 * 4)
fmm_status fmm_costmodel_table(fmm_ctx ctx, int32_t p, double theta, uint8_t *table);

/* ---------------- introspection (host outputs, for checking) ---------------- */

/* Counts after the last build/traverse.  Any pointer may be NULL. */
fmm_status fmm_get_sizes(fmm_ctx ctx, int64_t *n_cells, int64_t *n_m2l, int64_t *n_m2p,
                         int64_t *n_p2p);

/* M2L pairs after the last traversal, split into those converted by the
 * batched same-level GEMM (matrix cores) and those converted one by one
 * (mixed levels or offsets outside the per-octant tables).  NULL allowed. */
fmm_status fmm_get_m2l_split(fmm_ctx ctx, int64_t *n_batched, int64_t *n_general);

/*
 * Same-level M2L batching for (p, theta), needing no context or device: the
 * number of accepted same-level offsets per octant class (*slots: the slot
 * count of each target's GEMM row, 189 at theta = 0.5, 567 at 0.4; it grows
 * as theta^-3) and whether the batched matrix-core GEMM is used (*batched:
 * 1 if p has a matrix-core tiling and *slots <= 4096, else 0; all cell-cell
 * pairs then go through the class-batched path).  Either pointer may be NULL.
 */
fmm_status fmm_m2l_slots(int32_t p, double theta, int32_t *slots, int32_t *batched);

/* Shape of the batched same-level M2L after the last traversal: the number
 * of GEMM tiles (targets of one octant class, 64 or 128 per tile), tiles x
 * slots per class, and the slots actually multiplied (those used by at least
 * one target of the tile).  NULL allowed. */
fmm_status fmm_get_gemm_shape(fmm_ctx ctx, int64_t *tiles, int64_t *slots, int64_t *active_slots);

/* Work of the last traversal's lists: particle pairs of the P2P list
 * (sum of n_t * n_s, self pairs included) and target particles of the M2P
 * list (sum of n_t).  Either pointer may be NULL. */
fmm_status fmm_get_work(fmm_ctx ctx, int64_t *p2p_particle_pairs, int64_t *m2p_targets);

/* Bounding cube: lo3_host[3] minimum corner, side_host[1] side (of instance
 * 0 after a batch build). */
fmm_status fmm_get_bbox(fmm_ctx ctx, double *lo3_host, double *side_host);

/* Bounding cubes of the first n_inst instances of the last build:
 * lo_side_host[4k .. 4k+2] minimum corner, [4k+3] side; an empty instance
 * reports (0, 0, 0, 1).  n_inst must not exceed the built count. */
fmm_status fmm_get_bboxes(fmm_ctx ctx, int32_t n_inst, double *lo_side_host);

/* Sorted Morton keys and permutation (perm[k] = original index of the k-th
 * sorted particle); host arrays of n entries. */
fmm_status fmm_get_keys(fmm_ctx ctx, uint64_t *sorted_keys_host, int32_t *perm_host);

/* Cells in breadth-first (level, key) order; host arrays of n_cells entries
 * (centre_h: 3 per cell, half-grid units of side/2^22; radius_h: half side in
 * the same units).  Any pointer may be NULL. */
fmm_status fmm_get_cells(fmm_ctx ctx, int32_t *level, uint64_t *prefix, int32_t *begin,
                         int32_t *end, int32_t *parent, int32_t *first_child, int32_t *nchild,
                         int32_t *centre_h, int32_t *radius_h);

/* Interaction list `kind` (FMM_LIST_*) as (target cell, source cell) pairs,
 * grouped by target in increasing order; host arrays of the list's size. */
fmm_status fmm_get_list(fmm_ctx ctx, int32_t kind, int32_t *tgt_host, int32_t *src_host);

/* Consistency checks on host copies of the context's state (a debugging
 * aid, synchronous, O(n + cells + pairs)): the particle permutation and key
 * order, every cell's particle range, parent, level and children (which
 * must partition it), the leaf count, every list pair's cell indices, the
 * per-target grouping and offsets of the cell-particle and particle-particle
 * lists, and the GEMM gather table.  FMM_OK, or FMM_ERR_STATE with the first
 * violation in fmm_last_error (also without a tree). */
fmm_status fmm_validate(fmm_ctx ctx);

/* Scaled expansions after fmm_evaluate: per cell (p+1)^2 reals, degree n at
 * offset n*n as [Re c_n^0, Re c_n^1, Im c_n^1, ..., Re c_n^n, Im c_n^n], in
 * the Greengard-Rokhlin normalisation, multipoles divided by r^n and locals
 * multiplied by r^(n+1) (r = cell half side).  Host arrays n_cells*(p+1)^2.
 * Cartesian family: per cell (p+1)(p+2)(p+3)/6 reals, multi-index
 * (k1, k2, k3) at n(n+1)(n+2)/6 + (n-k1)(n-k1+1)/2 + k3 (n = |k|), the
 * multipole M_k = sum q (s - x)^k divided by r^|k| and the local L_m (phi =
 * sum L_m (x - t)^m) multiplied by r^(|m|+1). */
fmm_status fmm_get_expansions(fmm_ctx ctx, float *multipole_host, float *local_host);

/* Milliseconds of the phases of the last build/traverse/evaluate (recorded
 * only while timing is enabled), in the order: bbox+keys, sort, tree,
 * traverse, lists, p2m+m2m, m2l (batched GEMM phase: multipole split, GEMM,
 * group sum), m2l (general pairs), l2l, p2p, far+final, and last the
 * batched M2L GEMM kernel alone (0 when it did not run).  Writes
 * min(cap, 12) values; returns their count in *count. */
fmm_status fmm_get_timings(fmm_ctx ctx, double *ms_host, int32_t cap, int32_t *count);

/* Enable (1) or disable (0) per-phase timing events (adds synchronisation).
 * With overlap on, the P2P entry is the kernel's own duration on the second
 * stream; the phases then add up to more than the evaluation. */
fmm_status fmm_set_timing(fmm_ctx ctx, int32_t enabled);

/* Schedule of the near field: 0 runs every kernel in order on the context
 * stream; 1 runs P2P on a second stream of the context (default priority)
 * forked at the start of fmm_evaluate; 2 (the default) forks it after the
 * upward pass, so that it overlaps the M2L and L2L kernels.  The second
 * stream joins back into the context stream before the final sum.  Results
 * are identical under every schedule. */
fmm_status fmm_set_overlap(fmm_ctx ctx, int32_t schedule);

/*
 * Autotuner for tile shapes and schedule, on the context's current tree and
 * lists (e.g. the batch about to be evaluated repeatedly).  Leaves fall in
 * four size classes (at most 8, 16, 32 or more particles); for each class it
 * times the P2P kernel's tile shapes (`reps` launches each, events on the
 * context stream) and keeps the fastest: 1, 2 or 4 targets per lane with
 * every operation on the vector ALUs, or -1, -2, -4: that many targets per
 * lane with the sums over sources on the matrix cores (FP32 rank-1 updates
 * on v_mfma_f32_4x4x1f32; the vector ALUs form only 1/r and 1/r^3); if the lists
 * hold M2L pairs outside the same-level GEMM (spherical family) it times
 * fmm_evaluate under the four kinds of fmm_set_m2l_kernel and keeps the
 * fastest; then it times fmm_evaluate at `precision` under each tile width
 * of the M2L GEMM (where it has two, fmm_set_m2l_tile) and each of the three
 * schedules of fmm_set_overlap, and keeps the fastest pair.  The schedule and the M2L tile width do not change results; the
 * P2P tile shape and the M2L kind change how sums are split into FP32
 * partials, so results move by rounding only (each choice is itself
 * deterministic).
 * Requires a completed traversal.  Default before tuning: 4 targets per lane,
 * schedule 2.
 */
fmm_status fmm_autotune(fmm_ctx ctx, int32_t precision, int32_t reps);

/* Targets per tile of the same-level M2L GEMM (one octant class per tile):
 * 64 or 128 where the coefficient storage width is 128 (spherical p = 10),
 * 0 = the width's default (64); other widths have one tiling and ignore it.
 * Takes effect at the next fmm_traverse (fmm_autotune also rebuilds the
 * current tables when it picks a width).  Wider tiles load each translation
 * operator once for more targets.  get: the width of the current tables
 * (after a traversal with GEMM pairs), else the one asked for.  Any other
 * value is FMM_ERR_INVALID_ARG. */
fmm_status fmm_set_m2l_tile(fmm_ctx ctx, int32_t cols);
fmm_status fmm_get_m2l_tile(fmm_ctx ctx, int32_t *cols);

/* The tile shapes in use (p2p_tpl[4], host) and the schedule (*overlap, as
 * fmm_set_overlap);
 * either pointer may be NULL.  fmm_set_tile_config sets the shapes (each 1,
 * 2 or 4 targets per lane on the vector ALUs, or -1, -2, -4 for the
 * matrix-core form); any other value is FMM_ERR_INVALID_ARG and leaves the
 * shapes unchanged. */
fmm_status fmm_get_tile_config(fmm_ctx ctx, int32_t *p2p_tpl, int32_t *overlap);
fmm_status fmm_set_tile_config(fmm_ctx ctx, const int32_t *p2p_tpl);

#ifdef __cplusplus
}
#endif

#endif /* FMM_H_ */
