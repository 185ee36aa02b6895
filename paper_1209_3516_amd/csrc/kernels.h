// Host-side launchers of the gfx950 kernels (implemented in p2p.hip, far.hip,
// misc.hip, tree_gpu.hip and plan_gpu.hip).
// Plain pointers and sizes only; every launcher enqueues on `stream`
// (a hipStream_t) and returns the hipError_t of the launch as an int.
#pragma once

#include <cstdint>
#include <string>

#include "fmm_internal.h"

namespace fmmlib {
namespace dev {

// Expansion coefficients per cell are stored with a row stride padded to a
// multiple of 4 (16-byte rows for FP32).
inline int terms(int p) { return p * (p + 1) * (p + 2) / 6; }
inline int stride(int p) { return (terms(p) + 3) & ~3; }
// Multipoles folded for M2L keep the p^2 terms of z exponent <= 1.
inline int rstride(int p) { return (p * p + 3) & ~3; }

// bodies: [n] float4/double4 (x, y, z, q) in Morton order.
int gather_charges(bool fp64, int64_t n, const int32_t *perm, const void *q_user, void *bodies,
                   void *stream);

// What a P2P/L2P pass computes (see p2p.hip): charges -> (phi, grad);
// charges + dipoles -> (phi, grad); charges with per-target vectors v ->
// Hessian of the charge field applied to v.
enum EvalMode { kCharges = 0, kDipoles = 1, kHessVec = 2 };

// vec: [n] float4/double4 per-body dipoles (kDipoles) or per-target vectors
// (kHessVec), Morton order; unused for kCharges.
// four_waves: in FP32 charges mode, the kernel held to four waves per SIMD
// (else the general one, three waves); the caller picks it by whether the
// far field's M2L waves, running beside P2P, fit in what its waves leave.
// order: NULL (n_items work-groups; work-group w takes item xcd_remap(w), so
// that each XCD works on an equal-count contiguous range of the
// Morton-ordered items), or the n_order entries of the dispatch_orders order
// of the n_items items (n_order work-groups; work-group w takes item
// order[w], none if it is -1).
int p2p(bool fp64, int mode, bool mask_all, bool four_waves, int64_t n_items,
        const P2PItem *items, const int32_t *order, int64_t n_order, const int32_t *run_body,
        const int32_t *run_prefix, const void *bodies, const void *vec, void *part_s,
        void *part_c, void *stream);

// Sources the P2P kernels stage through LDS per batch.
constexpr int kP2PStageBatch = 384;

// Mutual P2P over the items of a P2PMutualPlan (FP32 charges): target sums to
// (part_s, part_c) at each item's out_off, source sums to part_m at the runs'
// run_dst.  bodies: [n] float4 (x, y, z, q), Morton order.
int p2p_mutual(bool mask_all, int64_t n_items, const P2PItem *items, const int32_t *run_body,
               const int32_t *run_prefix, const int32_t *run_dst, const void *bodies,
               void *part_s, void *part_c, void *part_m, void *stream);

// out[i] = sign * v[perm[i]] as a 4-vector (w = 0); v is user order [n][3].
int gather_vectors(bool fp64, int64_t n, const int32_t *perm, const void *v_user, double sign,
                   void *out, void *stream);

// geo: [n_cells] double4 (centre x, y, z, radius).
// dipoles: [n] 4-vectors in Morton order, or NULL for charges only.
// n_bodies: bodies of the tree (the mean leaf size picks the lane layout).
int p2m(int p, bool fp64, int64_t n_leaves, const int32_t *leaf_cell, const int32_t *cell_body_begin,
        const int32_t *cell_n_body, const double *geo, const void *bodies, const void *dipoles,
        void *M, double *M64, int64_t n_top, int64_t n_bodies, void *stream);

// Parents are the cells [c0, c1) of one level; leaves among them are skipped.
// child_fp64: children's multipoles are read from M64 (else from M).
// out_fp64: the parent is accumulated in FP64 into M64 and copied to M.
int m2m(int p, bool fp64, int64_t c0, int64_t c1, const int32_t *child_begin,
        const int32_t *n_child, const double *geo, void *M, double *M64, bool child_fp64,
        bool out_fp64, void *stream);

// Mr[c] (stride rstride(p)): the multipole of cell c folded onto its terms
// of z exponent <= 1, which is all that M2L needs of it (G = 1/r is
// harmonic).  Cells [0, n_cells).
int fold_multipoles(int p, bool fp64, int64_t n_cells, const void *M, void *Mr, void *stream);

// Batched M2L of box-centred trees (m2l_mfma.hip).  m2l_offsets: FP32
// derivative rows dtab[n_off][terms(p)] of the vectors off[n_off][3].
// m2l_mfma: the tiles [tile0, tile1) of the plan (FP32 multipoles Mr with
// stride rstride(p), locals L with stride stride(p)); every cell of those
// tiles gets its M2L locals written.
int m2l_offsets(int p, int64_t n_off, const double *off, float *dtab, void *stream);
int m2l_mfma(int p, int64_t tile0, int64_t tile1, const int32_t *tile_cells,
             const int64_t *tile_group_begin, const int32_t *group_offset,
             const int32_t *group_src, const float *dtab, const float *Mr, float *L,
             void *stream);

// Target cells [r0, r1) from the folded multipoles Mr; acc_fp64: the row
// accumulates in FP64 into L64, else into L (FP32 in mixed mode).
// order: NULL (r1 - r0 work-groups; work-group w takes cell r0 + xcd_remap(w)),
// or, when r1 is the number of cells, the n_order entries of the
// dispatch_orders M2L order of all cells (n_order work-groups; work-group w
// takes cell order[w], none if it is -1 or below r0).
int m2l(int p, bool fp64, int64_t r0, int64_t r1, const int64_t *ptr,
        const int32_t *col, const double *geo, const void *Mr, void *L, double *L64,
        bool acc_fp64, const int32_t *order, int64_t n_order, void *stream);

// (dispatch_orders, declared with DevicePlan below, builds the orders.)

// Children are the cells [c0, c1) of one level.
int l2l(int p, bool fp64, int64_t c0, int64_t c1, const int32_t *parent, const double *geo,
        void *L, double *L64, bool parent_fp64, bool child_fp64, void *stream);

int copy_top_locals(int p, int64_t n_top, const double *L64, float *L, void *stream);

// Source-side sums of the mutual P2P (FP32 only): body k of compact leaf a
// adds part_m[leaf_mbase[a] + j * n_body + k], j < leaf_nlow[a] (float4).
// part_m NULL: none.
struct MutualSlots {
  const void *part_m = nullptr;
  const int32_t *leaf_mbase = nullptr, *leaf_nlow = nullptr;
};

// kHessVec: tvec holds the per-target vectors (Morton order) and grad receives
// H v; phi is not written.
// Bodies [i0, i1) (Morton positions).  m2p_in: [n] (phi, grad) from m2p(),
// added to the far field, or NULL.
int l2p_combine(int p, bool fp64, int mode, int64_t i0, int64_t i1, const int32_t *body_leaf,
                const int32_t *leaf_cell, const int32_t *leaf_pbase, const int32_t *leaf_nchunk,
                const int32_t *cell_body_begin, const int32_t *cell_n_body, const double *geo,
                const void *L, const void *bodies, const void *tvec, const void *part_s,
                const void *part_c, MutualSlots ms, const void *m2p_in, const int32_t *perm,
                void *phi, void *grad, void *stream);

// M2P for the target leaves rows[0..n_rows) (each at most 64 bodies) over the
// M2P CSR list: out[b] = (phi, grad) of body b (Morton order) from the
// multipoles of the row's source cells.
int m2p(int p, bool fp64, int64_t n_rows, const int32_t *rows, const int64_t *ptr,
        const int32_t *col, const int32_t *cell_body_begin, const int32_t *cell_n_body,
        const double *geo, const void *M, const void *bodies, void *out, void *stream);

// dx = w * grad_q + q * grad_w (+ hv if not NULL), user order.
int backward_combine(bool fp64, int64_t n, const void *q, const void *w, const void *grad_q,
                     const void *grad_w, const void *hv, void *dx, void *stream);

// Interaction lists on the device (CSR, rows = target cells, sources
// ascending).  Pointers are hipMalloc'd by dual_traverse_gpu; the caller frees.
struct DeviceLists {
  int64_t n_rows = 0, p2p_nnz = 0, m2l_nnz = 0;
  int64_t *p2p_ptr = nullptr, *m2l_ptr = nullptr;
  int32_t *p2p_col = nullptr, *m2l_col = nullptr;
};

// Dual tree traversal on the GPU with the rules of the host traversal.
// geo: [n_cells] double4 (centre, radius); synchronises `stream`.
// Returns kTraverseTooLarge (no HIP error) when a frontier or a list would
// reach 2^31 entries (the device sort and scans count in 32 bits).
constexpr int kTraverseTooLarge = -2;
int dual_traverse_gpu(int64_t n_cells, const double *geo, const int32_t *child_begin,
                      const int32_t *n_child, double theta, bool leaf_first, void *stream,
                      DeviceLists &out);

// A tree built on the device: arrays hipMalloc'd by build_tree_gpu (caller
// frees); geo [n_cells] double4 (centre, radius); pos [n][3] Morton order.
struct DeviceTree {
  int64_t n = 0, n_cells = 0;
  int32_t *perm = nullptr, *body_begin = nullptr, *n_body = nullptr, *child_begin = nullptr,
          *n_child = nullptr, *parent = nullptr;
  double *geo = nullptr, *pos = nullptr;
  uint64_t *keys = nullptr;
};

// Tree build on the GPU with the rules of build_tree; fills `t` (host copy of
// the cell arrays; perm, keys and pos are left empty) and `out` (device
// arrays, including the Morton-ordered positions and keys).  xyz: device [n][3] FP64, user order.  Returns 0,
// a hipError_t, or -1 with `err` set for non-finite positions.
int build_tree_gpu(const double *xyz, int64_t n, int ncrit, void *stream, DeviceTree &out,
                   TreeData &t, std::string &err);

// Scratch of the tree build, traversal and plan builder comes from the
// device's default stream-ordered pool, which keeps up to this many freed
// bytes for reuse instead of returning them to the driver.
constexpr uint64_t kPoolKeepBytes = 16ull << 30;
int keep_pool_memory();

// Tree builds, traversals and plan builds run on one library-owned
// non-blocking stream per device (default priority), made to wait for the
// caller's stream `user` by an event; those calls synchronise it before they
// return.  Scratch from the pool is then allocated and returned on it rather
// than on the legacy null stream, whose stream-ordered frees synchronise.
constexpr int kMaxDevices = 64;
// The traversal keeps up to this much of its scratch on each device for the
// next traversal instead of freeing it (a traversal of 10^7 bodies at
// theta = 0.3 needs about 10 GB; a device has 288 GB).
constexpr size_t kKeepScratchBytes = size_t(16) << 30;
int build_stream(void *user, void **out);  // *out: the hipStream_t

// P2P work plan on the device (the layout of P2PPlan, see plan.cpp).
struct PlanLayouts {
  int32_t cfg[65];  // tgt_cfg bits (n_tgt | R << 8 | L << 16 | K << 24) for n_tgt = 0..64
};
struct DevicePlan {
  P2PItem *items = nullptr;
  // Dispatch order of the items for a P2P launch over all of them (see
  // dispatch_orders; order_len entries), or NULL.
  int32_t *order = nullptr;
  int64_t order_len = 0;
  int32_t *run_body = nullptr, *run_prefix = nullptr;
  int32_t *leaf_cell = nullptr, *leaf_pbase = nullptr, *leaf_nchunk = nullptr,
          *body_leaf = nullptr;
  int64_t n_items = 0, n_runs = 0, n_leaves = 0, n_partials = 0;
  int64_t max_row_sources = 0, p2p_pairs = 0;
  void release();
};

// Build the P2P work plan from device CSR P2P lists and the device tree
// arrays; the result is the plan build_p2p_plan makes, entry for entry.
// Synchronises `stream`.  Returns 0 or a hipError_t (on error `out` is empty).
int build_p2p_plan_gpu(int64_t n, int64_t n_cells, int64_t n_leaves, const int32_t *n_child,
                       const int32_t *body_begin, const int32_t *n_body, const int64_t *p2p_ptr,
                       const int32_t *p2p_col, const PlanLayouts &layouts, void *stream,
                       DevicePlan &out);

// The dispatch orders of a launch over all of the plan's P2P items and of
// one over all n_cells M2L rows (CSR row pointers m2l_ptr), replacing
// plan.order / plan.order_len and *m2l_order / *m2l_len (device arrays the
// caller frees with hipFree).  Work-groups go to the eight XCDs in turn
// (work-group w to XCD w mod 8), and contiguous ranges of units differ
// widely in work, so each order cuts its units, in plan order, into eight
// contiguous ranges of about equal estimated work, range x going to XCD x:
// its units keep their neighbourhood, and with it the reuse of sources
// (bodies, multipoles) in that XCD's L2.  Within a range the units go by
// decreasing rank (ties in plan order), so that the long ones start first
// and the short ones fill the end of the launch.  The order has 8 m
// entries, m the units of the largest range: entry 8 j + x is the j-th unit
// of range x, or -1 past its end.
//   P2P item: work and rank are its estimated cost (the wave's VALU work:
//     its staged batches, the steps over its lanes' targets, the stream
//     merge, and a fixed part).  (By this estimate the equal-count ranges
//     that xcd_remap gives the XCDs differ in cost by up to 2.7x on a
//     Plummer sphere of 10^6 bodies.)
//   M2L row: its work is one pass per 64 entries plus one; its rank, its
//     length.  (Cells are numbered breadth first, and the upper levels'
//     rows are the longest.)
// The items, their partial-sum slots and every result are unchanged.
// Synchronises the library's build stream (waiting for `stream` first).
// Returns 0 or a hipError_t (then no order is set).
int dispatch_orders(DevicePlan &plan, const int64_t *m2l_ptr, int64_t n_cells,
                    int32_t **m2l_order, int64_t *m2l_len, void *stream);

// pos: device [n][3] FP64 (Morton order) -> out: device [n] double4 (fp64)
// or float4 (rounded to nearest), (x, y, z, 0).
int pack_positions(bool fp64, int64_t n, const double *pos, void *out, void *stream);

int direct_sum(const double *xyz, const double *q, int64_t n, const int64_t *targets, int64_t m,
               double *phi, double *grad, void *stream);

}  // namespace dev
}  // namespace fmmlib
