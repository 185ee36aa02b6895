/*
 * fmm.h - C interface of the MI355X (gfx950) dual-tree-traversal fast
 * multipole method for the 3-D Laplace kernel.
 *
 * Method: R. Yokota, "An FMM Based on Dual Tree Traversal for Many-core
 * Architectures" (arXiv:1209.3516).  A Morton-key octree with at most ncrit
 * bodies per leaf (section 3.3), interaction lists from a dual tree traversal
 * under the multipole acceptance criterion theta (section 3.2; section 3.3,
 * Algorithms 3 and 4), Cartesian Taylor expansions (section 3.1, Table 2), and
 * the P2M, M2M, M2L, P2P, L2L and L2P kernels.
 *
 * Quantities (the paper states no formulas; these are the textbook ones):
 *   phi_i  = sum_{j : |x_j - x_i| > 0} q_j / |x_j - x_i|
 *   grad_i = d phi / d x (x_i) = sum_j q_j (x_j - x_i) / |x_j - x_i|^3
 * No 1/(4 pi) factor and no softening.  Order p keeps multipole and local
 * terms of total degree 0..p-1, p(p+1)(p+2)/6 coefficients per cell.
 *
 * Conventions for every function:
 *  - Return 0 (FMM_OK) or a negative fmm_status; nothing aborts or exits.
 *    fmm_last_error() gives a message for the last failure on this thread.
 *  - Arguments are checked before any GPU call, so FMM_EINVAL cases never
 *    touch the device.
 *  - Host pointers are borrowed for the duration of the call only.
 *  - "Device" pointers are HIP device allocations of the caller (for example
 *    torch tensors); they are read or written asynchronously on the given
 *    HIP stream (hipStream_t passed as void*; NULL = the null stream).  The
 *    call returns after enqueueing; the caller synchronises.
 *  - Handles (fmm_tree, fmm_lists) own host memory and, once a device call
 *    has been made, device memory; a handle is used from one host thread and
 *    one stream at a time.
 *  - Environment: FMM_LOG=1 prints tree and list statistics to stderr (host
 *    calls only).  FMM_FAULT_INJECT=alloc:K makes the K-th allocation
 *    checkpoint of a tree build or traversal fail (FMM_ENOMEM, nothing
 *    leaked); FMM_FAULT_INJECT=launch:K makes the K-th kernel launch of each
 *    evaluation report FMM_EDEVICE instead of launching.  For tests.
 */
#ifndef PAPER_1209_3516_AMD_FMM_H
#define PAPER_1209_3516_AMD_FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fmm_status {
  FMM_OK = 0,
  FMM_EINVAL = -1,  /* bad argument (NaN position, theta outside (0,1), p out of range...) */
  FMM_ENOMEM = -2,  /* host or device allocation failed */
  FMM_EDEVICE = -3, /* a HIP call failed; fmm_last_error() holds hipGetErrorString */
  FMM_ESTATE = -4   /* handles that do not belong together (lists of another tree) */
};

enum fmm_precision {
  FMM_MIXED = 0, /* P2P, M2L, P2M, L2P in FP32; P2P sums Kahan-compensated */
  FMM_FP64 = 1   /* every kernel in FP64, plain sums */
};

enum fmm_traverse_flags {
  FMM_MAC_FIRST = 0u, /* test the MAC before the leaf test (default) */
  FMM_LEAF_FIRST = 1u /* leaf test first, as printed in Algorithm 4 */
};

enum fmm_list_kind { FMM_P2P = 0, FMM_M2L = 1, FMM_M2P = 2 };

/* Flags of fmm_tree_build_ex. */
enum fmm_tree_flags {
  FMM_TREE_BOX_CENTRES = 1u /* expansion centres at the centres of the Morton cubes */
};
enum { FMM_MAX_M2P = 64 }; /* largest m2p_max of fmm_traverse_hybrid */

enum fmm_eval_flags {
  FMM_EVAL_TIMING = 1, /* record per-phase device times (fmm_last_timings) */
  FMM_EVAL_KEEP_STAGES = 2, /* keep a copy of the locals after M2L (fmm_copy_expansions) */
  FMM_EVAL_SERIAL = 4, /* run P2P on the caller's stream instead of overlapping it with the
                          upward pass, M2L and L2L on a second (library-owned) stream */
  FMM_EVAL_M2L_MFMA = 8, /* M2L batched by translation vector on the matrix cores; needs a
                           tree built with FMM_TREE_BOX_CENTRES and FMM_MIXED precision */
  FMM_EVAL_MUTUAL_P2P = 16 /* mutual P2P: each unordered pair of P2P leaves is evaluated
                              once, for the bodies of both (section 2: the mutual interaction
                              of falcON that exaFMM inherits).  FMM_MIXED only; every leaf
                              must hold at most 64 bodies (FMM_EINVAL otherwise, on the
                              first evaluation, which builds its plan from the host copy of
                              the lists).  Applies where the sources are charges alone:
                              fmm_evaluate and the pass of fmm_evaluate_backward without v;
                              the other passes run one-sided.  Not with
                              fmm_evaluate_range or fmm_evaluate_noalloc (FMM_EINVAL) */
};

/* Phases reported by fmm_last_timings, in this order.  Without FMM_EVAL_SERIAL
 * the P2P phase overlaps P2M..L2L, so the phases then sum to more than the total. */
enum fmm_phase {
  FMM_PHASE_GATHER = 0, /* charges into Morton order */
  FMM_PHASE_P2P = 1,    /* near field */
  FMM_PHASE_P2M = 2,
  FMM_PHASE_M2M = 3,
  FMM_PHASE_M2L = 4, /* M2L, and M2P for hybrid lists */
  FMM_PHASE_L2L = 5,
  FMM_PHASE_L2P = 6, /* L2P + near/far combine + scatter to user order */
  FMM_PHASE_TOTAL = 7,
  FMM_NUM_PHASES = 8
};

#define FMM_MAX_P 8
#define FMM_MAX_LEVEL 21

typedef struct fmm_tree fmm_tree;
typedef struct fmm_lists fmm_lists;

typedef struct fmm_eval_opts {
  int p;               /* expansion order, 1..FMM_MAX_P (degrees 0..p-1) */
  int precision;       /* enum fmm_precision */
  int fp64_top_levels; /* FMM_MIXED only: multipoles/locals of cells at level <= this are
                          kept and translated (M2M, L2L) in FP64; -1 = automatic
                          (3 when p >= 8, otherwise none); -2 = none */
  int flags;           /* enum fmm_eval_flags */
} fmm_eval_opts;

/* Read-only view of a tree (library-owned host arrays, valid until the tree is freed). */
typedef struct fmm_tree_view_t {
  int64_t n;         /* bodies */
  int64_t n_cells;   /* cells, numbered breadth first (children contiguous) */
  int64_t n_leaves;
  int32_t max_level; /* deepest level (root = 0) */
  int32_t fp32_exact; /* 1 if every position is exactly representable in FP32 */
  const int32_t *perm;        /* [n]  Morton position -> user index */
  const uint64_t *keys;       /* [n]  63-bit Morton keys in Morton order */
  const int32_t *level;       /* [n_cells] */
  const int32_t *parent;      /* [n_cells] -1 for the root */
  const int32_t *child_begin; /* [n_cells] first child (0 for a leaf) */
  const int32_t *n_child;     /* [n_cells] 0 for a leaf */
  const int64_t *body_begin;  /* [n_cells] first body (Morton position) */
  const int64_t *n_body;      /* [n_cells] */
  const double *center;       /* [n_cells][3] expansion centre: middle of the cell's tight bounding box */
  const double *radius;       /* [n_cells] largest centre-to-body distance */
} fmm_tree_view_t;

typedef struct fmm_lists_stats_t {
  int64_t p2p_entries; /* leaf pairs in the P2P list */
  int64_t m2l_entries; /* cell pairs in the M2L list */
  int64_t p2p_pairs;   /* body-body interactions: sum over entries n_A*n_B, minus n_A for (A,A) */
  int64_t p2p_work_items; /* GPU work items of the P2P kernel (one wave each) */
  int64_t p2p_max_row_sources; /* largest number of source bodies of one target leaf */
  int64_t m2p_entries; /* cell pairs in the M2P list (hybrid lists; else 0) */
} fmm_lists_stats_t;

/*
 * Build the octree (section 3.3: Morton keys, ncrit bodies per leaf).
 *   xyz   host, n x 3 row-major FP64 positions in user order; finite.
 *   n     >= 0 (0 gives an empty tree whose evaluation is a no-op).
 *   ncrit >= 1: a cell with more than ncrit bodies is split (up to level 21).
 * Root cube: centre (lo+hi)/2, half-width max_d (hi_d-lo_d)/2.  Keys use 21 bits
 * per axis (x in the lowest bit of each triplet); bodies are sorted stably by key.
 * Cells with more than ncrit bodies get one child per non-empty octant.
 * Host only: no GPU is touched.  *out is owned by the caller until fmm_tree_free.
 */
int fmm_tree_build(const double *xyz, int64_t n, int ncrit, fmm_tree **out);

/*
 * fmm_tree_build with options.  flags: 0 (the same tree as fmm_tree_build) or
 * FMM_TREE_BOX_CENTRES: every cell's expansion centre is the geometric centre
 * of its cube in the Morton subdivision of the root cube (the geometric
 * centre of the paper's Table 3), (c_d - h) + (i_d + 1/2) 2h / 2^L for a
 * level-L cell with integer coordinates i, instead of the middle of its
 * bodies' bounding box; the radius stays the largest centre-to-body distance.
 * Translation vectors between such centres are multiples of half a cube
 * side, so they repeat across the tree (what the MFMA M2L of
 * FMM_EVAL_M2L_MFMA batches over).  Other arguments and errors as
 * fmm_tree_build; FMM_EINVAL for unknown flags.  Host only.
 */
int fmm_tree_build_ex(const double *xyz, int64_t n, int ncrit, unsigned flags, fmm_tree **out);

/*
 * The same tree built on the GPU (bounding-box reduction, Morton keys with
 * the same FP64 expression and no FMA contraction, stable radix sort of
 * (key, index), level-by-level octant split, per-cell bounding box and
 * radius): identical bit for bit to fmm_tree_build's.
 *   xyz_dev device, n x 3 row-major FP64 positions in user order.
 * Uses the current device and `stream` (synchronised).  The tree keeps its
 * device arrays for the evaluation and a host copy for views and the host
 * traversal.  FMM_EINVAL for non-finite positions, else as fmm_tree_build.
 */
int fmm_tree_build_gpu(const void *xyz_dev, int64_t n, int ncrit, fmm_tree **out, void *stream);

/*
 * Replace the positions (host, n x 3, user order) while keeping the structure
 * (keys, cells, centres, radii) frozen - used for finite-difference checks of
 * the gradient, which differentiate the method with its tree held fixed.
 * Host only; device copies are refreshed by the next evaluation.
 */
int fmm_tree_set_positions(fmm_tree *t, const double *xyz);

int fmm_tree_view(const fmm_tree *t, fmm_tree_view_t *v);
void fmm_tree_free(fmm_tree *t);

/*
 * Dual tree traversal (section 3.3, Algorithms 3 and 4) from (root, root).
 * MAC (section 3.2): (A, B) is well separated iff
 *   (theta*theta) * ((dx*dx + dy*dy) + dz*dz) > (B_A + B_B)^2   (FP64, strict),
 * d the distance between expansion centres, B the cell radii; 0 < theta < 1.
 * Not separated: both leaves -> P2P; a self pair (A, A) splits into all pairs
 * of children; otherwise the cell with the larger radius is split (equal radii:
 * the lower-numbered one), never a leaf.  The lists are symmetric.
 * flags: FMM_MAC_FIRST (default) or FMM_LEAF_FIRST.
 * Output: two CSR lists (P2P, M2L), one row per target cell, sources ascending,
 * and the work plan of the P2P kernel (targets in groups of at most 64 per
 * leaf, sources in chunks of contiguous runs), which the first evaluation
 * uploads.  FMM_EINVAL when that plan would hold 2^31 or more runs, work
 * items or partial sums (it indexes them with 32-bit integers; the
 * environment variable FMM_PLAN_LIMIT=K lowers the limit, for tests).
 * Host only: no GPU is touched.
 */
int fmm_traverse(const fmm_tree *t, double theta, unsigned flags, fmm_lists **out);

/*
 * Treecode/FMM hybrid lists: the traversal of fmm_traverse, except that an
 * accepted pair (A, B) whose target A is a leaf of at most m2p_max bodies goes
 * to a third list, M2P, instead of M2L: B's multipole is then evaluated
 * directly at A's bodies (the treecode's kernel, Algorithm 1; the M2L/M2P
 * choice of the auto-tuned hybrid codes that section 2 of the paper
 * describes).  The P2P list and the union of M2L and M2P equal fmm_traverse's.
 *   m2p_max  0..FMM_MAX_M2P; 0 gives fmm_traverse's lists.
 * M2P uses derivatives of 1/r up to degree p (its gradient keeps one more
 * degree than L2P's).  The far-field operator is then no longer symmetric, so
 * fmm_evaluate_backward returns FMM_ESTATE and fmm_evaluate_range FMM_EINVAL
 * for such lists.  Host only, like fmm_traverse.
 */
int fmm_traverse_hybrid(const fmm_tree *t, double theta, unsigned flags, int m2p_max,
                        fmm_lists **out);

/*
 * The same traversal on the GPU (level-synchronous frontier of cell pairs,
 * same FP64 MAC without FMA contraction, canonical order by a 64-bit radix
 * sort): the lists are identical bit for bit to fmm_traverse's.  Uses the
 * current device and `stream` (hipStream_t or NULL) and synchronises it.
 * The lists stay on the device, and the P2P work plan of fmm_evaluate is
 * built there too (the same plan the host builds from the same lists), so
 * the first evaluation uploads nothing.  The host copy of the lists is made
 * by the first fmm_lists_view on the handle (a blocking copy; do not call it
 * concurrently with other calls on the same handle).  Errors as
 * fmm_traverse, plus FMM_EDEVICE, and FMM_EINVAL when a list or one level of
 * the traversal would hold 2^31 or more cell pairs (the device sort counts in
 * 32 bits; fmm_traverse has no such limit).
 */
int fmm_traverse_gpu(const fmm_tree *t, double theta, unsigned flags, fmm_lists **out,
                     void *stream);

/* CSR view of one list (library-owned host arrays, valid until fmm_lists_free).
 * kind FMM_P2P, FMM_M2L or FMM_M2P (empty unless the lists are hybrid).
 * nrows = number of cells; row_ptr[nrows+1] int64; col[nnz] int32.  For lists
 * from fmm_traverse_gpu the first call copies them to the host (FMM_EDEVICE
 * or FMM_ENOMEM if that fails). */
int fmm_lists_view(const fmm_lists *l, int kind, const int64_t **row_ptr, const int32_t **col,
                   int64_t *nrows, int64_t *nnz);
int fmm_lists_stats(const fmm_lists *l, fmm_lists_stats_t *s);
void fmm_lists_free(fmm_lists *l);

/*
 * Counts of the work plan FMM_EVAL_MUTUAL_P2P evaluates these lists with
 * (section 2: falcON's mutual interaction), built on the host and not kept:
 *   out[0] work items, out[1] runs (one source leaf B > A each),
 *   out[2] body pairs of the leaf pairs A < B (each evaluated once, for both
 *          bodies), out[3] ordered body pairs i != j within one leaf
 *          (evaluated one-sided), out[4] partial-sum slots of the sums the
 *          bodies of each leaf B receive from its leaves A < B.
 * For symmetric lists 2 out[2] + out[3] is fmm_lists_stats' p2p_pairs.
 * out: caller-owned int64[5].  Lists from fmm_traverse_gpu are first copied
 * to the host (as by fmm_lists_view).  FMM_EINVAL with a message, as the
 * first evaluation with the flag: leaves of more than 64 bodies, lists that
 * are not symmetric, counts that need more than 32-bit offsets.
 */
int fmm_mutual_plan_stats(const fmm_tree *t, const fmm_lists *l, int64_t *out);

/*
 * The order in which an evaluation over all targets dispatches its P2P and
 * M2L work on the GPU (scheduling only: it changes no result, and the
 * method does not define it), copied to the host.  Work-groups go to the
 * GPU's eight XCDs in turn (work-group w to XCD w mod 8).  Both orders cut
 * their units, in plan order, into eight contiguous ranges of about equal
 * work (range x: the units whose work midpoints fall in the x-th eighth of
 * the total), range x for XCD x, and take each range by decreasing rank,
 * ties in plan order; *len = 8 m, m the units of the largest range, and
 * out[8 j + x] is the j-th unit of range x, or -1 past its end (work-group w
 * takes unit out[w]; every unit occurs once).
 *   kind FMM_P2P: the units are the P2P work items (one per group of at
 *     most 64 targets of a leaf and chunk of its sources); work and rank
 *     are both the item's estimated cost (its staged source batches, the
 *     steps over each lane's targets, the merge of its source streams).
 *   kind FMM_M2L: the units are the cells; a row's work is one pass per 64
 *     entries, plus one, and its rank is its length.
 * The lists must be on the device (after fmm_traverse_gpu or a first
 * evaluation; FMM_ESTATE otherwise).  out: caller-owned int32[cap], or NULL
 * to get *len only; FMM_EINVAL for another kind, a NULL len, or cap < *len.
 */
int fmm_dispatch_order(const fmm_lists *l, int kind, int32_t *out, int64_t cap, int64_t *len);

/*
 * Forward evaluation on one GPU: the evaluation phase of the method, i.e. the
 * kernels the paper names (section 3.3 and the list of kernels timed with
 * Table 4): P2M on every leaf and M2M up the tree (upward pass), M2L over the
 * M2L list and P2P over the P2P list (the pairs the dual tree traversal of
 * Algorithms 3 and 4 produced), L2L down the tree and L2P at every body, with
 * the near (P2P) and far (L2P) fields added per body.  The expansions are the
 * Cartesian Taylor series of section 3.1 (Table 2) truncated at total degree
 * p - 1, so an accepted pair's error falls as theta^p (section 3.2).  P2P is
 * the direct sum of section 3.4 (potential and gradient of q_j / r).
 *   q_dev    device, [n] charges in user order (float for FMM_MIXED, double for FMM_FP64)
 *   phi_dev  device, [n] potentials out (same dtype)
 *   grad_dev device, [n][3] gradients out (same dtype), or NULL
 *   stream   hipStream_t or NULL.
 * l must come from fmm_traverse(t, ...) (else FMM_ESTATE).  The first call on a
 * (tree, lists, p, precision) uploads the tree, lists and work plan and
 * allocates device scratch (hipMalloc); later calls reuse them.  No float
 * atomics: repeated calls give bitwise identical results.  Unless
 * FMM_EVAL_SERIAL is set, the near field (P2P) runs on a second stream owned
 * by the lists handle, forked from and joined back into `stream` with events,
 * so it overlaps the far field; all outputs are complete when `stream` is.
 */
int fmm_evaluate(const fmm_tree *t, const fmm_lists *l, const fmm_eval_opts *o, const void *q_dev,
                 void *phi_dev, void *grad_dev, void *stream);

/*
 * fmm_evaluate for callers that cannot allocate device memory: code under
 * stream capture, tight serving loops, harnesses that forbid allocation.
 * Computes exactly what fmm_evaluate computes (the same kernels; results
 * identical bit for bit) with every device buffer of the evaluation
 * (multipoles, locals, FP64 top levels, P2P partial sums) taken from one
 * fixed array of FMM_NOALLOC_SCRATCH_BYTES of device memory that the library
 * holds on each GPU it runs on until the process ends.  The call makes no
 * hipMalloc, hipFree, stream or event; the near field runs on `stream`
 * (as with FMM_EVAL_SERIAL).
 *   t, l, o, q_dev, phi_dev, grad_dev, stream  as fmm_evaluate; o->flags may
 *            hold only FMM_EVAL_SERIAL.
 * Preconditions: the tree, lists and work plan are already on the current
 * device for o->precision (one fmm_evaluate with the same precision on this
 * device puts them there, as do fmm_tree_build_gpu + fmm_traverse_gpu
 * followed by such a call); otherwise FMM_ESTATE.
 * Errors: FMM_EINVAL when the evaluation needs more than
 * FMM_NOALLOC_SCRATCH_BYTES (the message gives both sizes; 10^6 uniform
 * bodies at p = 4 need about 41 MB), for FMM_EVAL_TIMING or
 * FMM_EVAL_KEEP_STAGES, and for hybrid (M2P) lists; the argument errors of
 * fmm_evaluate.  Every buffer of the array is written before it is read
 * within one call, so nothing needs clearing between calls.  All calls on
 * one GPU share its array: calls that overlap in time on one GPU (two host
 * threads, or two streams not ordered by events) race and give undefined
 * results.  fmm_copy_expansions and fmm_last_timings keep describing the
 * last fmm_evaluate.
 */
#define FMM_NOALLOC_SCRATCH_BYTES (128ull << 20)
int fmm_evaluate_noalloc(const fmm_tree *t, const fmm_lists *l, const fmm_eval_opts *o,
                         const void *q_dev, void *phi_dev, void *grad_dev, void *stream);
/* Size of that array in bytes (FMM_NOALLOC_SCRATCH_BYTES). */
size_t fmm_noalloc_scratch_bytes(void);

/*
 * Evaluation for the targets of one range of leaves in Morton order: the
 * share of one GPU when the target bodies are split into contiguous Morton
 * ranges (the partition of a global Morton order with work weights that
 * section 2 of the paper describes for distributed trees).
 *   body_begin, body_end  Morton positions, 0 <= body_begin <= body_end <= n,
 *                         each the first body of a leaf or n (else FMM_EINVAL);
 *                         an empty range is a no-op.
 *   q_dev, phi_dev, grad_dev, stream  as fmm_evaluate (user order, full length n).
 * Writes phi and grad only for the bodies of the range (user index perm[b],
 * see fmm_tree_view); other entries are left unchanged.  P2P, M2L, L2L and
 * L2P run only for the cells that hold bodies of the range; P2M and M2M run
 * for the whole tree (on several GPUs: local subtrees plus an exchange of
 * multipoles).  The values written are bit for bit those of fmm_evaluate.
 */
int fmm_evaluate_range(const fmm_tree *t, const fmm_lists *l, const fmm_eval_opts *o,
                       int64_t body_begin, int64_t body_end, const void *q_dev, void *phi_dev,
                       void *grad_dev, void *stream);

/*
 * Split the target leaves, in Morton order, into n_parts contiguous ranges of
 * about equal work for fmm_evaluate_range: a leaf weighs its P2P body pairs
 * plus m2l_weight times its M2L entries, where the entries of a cell's row are
 * shared among its bodies and passed down to the leaves below it.
 *   bounds  host, [n_parts + 1] out: bounds[0] = 0, bounds[n_parts] = n,
 *           non-decreasing, every bound a leaf boundary (ranges may be empty).
 * Host only; for lists from fmm_traverse_gpu it makes their host copy.
 */
int fmm_partition_targets(const fmm_tree *t, const fmm_lists *l, int n_parts, double m2l_weight,
                          int64_t *bounds);

/*
 * Backward of L = sum_i w_i phi_i + sum_i v_i . grad_i for the forward above,
 * with the tree, lists, centres and radii held fixed.  (The paper evaluates
 * the forward only; this is the adjoint of the discrete method of sections
 * 3.1 to 3.4 with the traversal's output frozen.)  The method is linear in
 * q and its far-field operator is symmetric (the lists are symmetric), so
 *   dL/dq_j = Phi_j           Phi: potential of charges w plus dipoles -v
 *                             (a dipole s at x_j has potential s.(x_j - y)/|x_j - y|^3)
 *   dL/dx_i = w_i grad_i[q] + q_i grad Phi_i + H_i[q] v_i
 * where H[q] is the Hessian of the charge field (second derivatives of the
 * local expansion plus the near-field Hessian of 1/r).  With v = NULL (a loss
 * on the potential only) this is one evaluation with charges w plus an
 * elementwise combine; with v it is two evaluations (charges w + dipoles -v,
 * and charges q with Hessian-vector outputs) plus the combine.
 *   q_dev       device [n]: the forward's charges (required when dx_dev != NULL)
 *   grad_q_dev  device [n][3]: grad[q] from the forward (required when dx_dev != NULL)
 *   w_dev       device [n]: dL/dphi (required; zeros for a loss on the gradient only)
 *   v_dev       device [n][3]: dL/dgrad, or NULL
 *   dq_dev      device [n] out, or NULL;  dx_dev device [n][3] out, or NULL
 * Same dtype/stream rules as fmm_evaluate.
 */
int fmm_evaluate_backward(const fmm_tree *t, const fmm_lists *l, const fmm_eval_opts *o,
                          const void *q_dev, const void *grad_q_dev, const void *w_dev,
                          const void *v_dev, void *dq_dev, void *dx_dev, void *stream);

/*
 * Direct O(N) sum per target in FP64 on the GPU (zero-distance pairs skipped),
 * the reference the method approximates; used to report accuracy as the
 * relative L2 error against direct summation (the error measure of Table 4
 * and section 3.5).
 *   xyz_dev     device, double [n][3] positions (user order)
 *   q_dev       device, double [n] charges
 *   targets_dev device, int64 [m] target indices in [0, n)
 *   phi_dev     device, double [m]; grad_dev device, double [m][3] or NULL
 */
int fmm_direct(const void *xyz_dev, const void *q_dev, int64_t n, const int64_t *targets_dev,
               int64_t m, void *phi_dev, void *grad_dev, void *stream);

/*
 * Per-phase device times (milliseconds, enum fmm_phase order) of the last
 * evaluation on these lists (fmm_evaluate, fmm_evaluate_range or
 * fmm_evaluate_backward's passes), which must have been called with
 * FMM_EVAL_TIMING (FMM_ESTATE otherwise).  Waits for that evaluation to
 * finish.  ms must hold FMM_NUM_PHASES doubles.
 */
int fmm_last_timings(const fmm_lists *l, double *ms);

/*
 * Mean per-phase device times (milliseconds, enum fmm_phase order) over the
 * last n evaluations on these lists, all called with FMM_EVAL_TIMING one
 * after another (an evaluation without the flag starts the count again);
 * the events of the last FMM_TIMING_HISTORY timed evaluations are held, so a
 * run of evaluations can be timed without waiting between them and read
 * afterwards.  Waits for the newest to finish.  ms must hold FMM_NUM_PHASES
 * doubles.  FMM_EINVAL unless 1 <= n <= FMM_TIMING_HISTORY; FMM_ESTATE if
 * fewer than n such evaluations are held.
 */
#define FMM_TIMING_HISTORY 64
int fmm_mean_timings(const fmm_lists *l, int n, double *ms);

/* Message for the last failure on the calling thread ("" if none). */
const char *fmm_last_error(void);

/* Number of expansion coefficients p(p+1)(p+2)/6, or -1 for p out of range. */
int fmm_num_terms(int p);

/*
 * Copy a device-side expansion array of the last evaluation into host memory,
 * for staged parity checks: kind 0 = multipoles M after the upward pass,
 * 1 = locals after M2L (before L2L), 2 = locals after L2L.  dst: host double
 * [n_cells][fmm_num_terms(p)], coefficient t having exponents exps[t] as given
 * by fmm_term_exponents (int32 [T][3]).  Synchronises the device.  kind 1
 * requires the last evaluation to have been called with FMM_EVAL_KEEP_STAGES.
 */
int fmm_copy_expansions(const fmm_lists *l, int kind, double *dst);
int fmm_term_exponents(int p, int32_t *exps);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_1209_3516_AMD_FMM_H */
