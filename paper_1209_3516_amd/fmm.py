"""Python binding of libfmm.so, the gfx950 dual-tree-traversal Laplace FMM.

Argument marshalling only: every step of the method runs in the library
(host C++ for the tree and the traversal, HIP kernels for the evaluation).
torch supplies device memory and streams.  If the library is not built, every
entry point raises; there is no fallback.

    tree  = Tree(xyz_float64_numpy, ncrit)          # Morton octree (host)
    lists = Lists(tree, theta)                       # dual tree traversal (host)
    phi, grad = evaluate(tree, lists, q_cuda, p)     # one GPU evaluation
    phi = potential(x_cuda, q_cuda, tree, lists, p)  # differentiable in q and x
"""
import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfmm.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE, FMM_ESTATE = 0, -1, -2, -3, -4
FMM_MIXED, FMM_FP64 = 0, 1
FMM_MAC_FIRST, FMM_LEAF_FIRST = 0, 1
FMM_P2P, FMM_M2L, FMM_M2P = 0, 1, 2
FMM_EVAL_TIMING, FMM_EVAL_KEEP_STAGES, FMM_EVAL_SERIAL = 1, 2, 4
FMM_TREE_BOX_CENTRES = 1
FMM_EVAL_M2L_MFMA = 8
FMM_EVAL_MUTUAL_P2P = 16
PHASES = ("gather", "p2p", "p2m", "m2m", "m2l", "l2l", "l2p", "total")

_STATUS = {FMM_EINVAL: "EINVAL", FMM_ENOMEM: "ENOMEM", FMM_EDEVICE: "EDEVICE",
           FMM_ESTATE: "ESTATE"}


class FMMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_STATUS.get(code, code), msg))
        self.code = code


class _EvalOpts(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("precision", ctypes.c_int),
                ("fp64_top_levels", ctypes.c_int), ("flags", ctypes.c_int)]


class _TreeView(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_cells", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("max_level", ctypes.c_int32), ("fp32_exact", ctypes.c_int32),
                ("perm", ctypes.c_void_p), ("keys", ctypes.c_void_p), ("level", ctypes.c_void_p),
                ("parent", ctypes.c_void_p), ("child_begin", ctypes.c_void_p),
                ("n_child", ctypes.c_void_p), ("body_begin", ctypes.c_void_p),
                ("n_body", ctypes.c_void_p), ("center", ctypes.c_void_p),
                ("radius", ctypes.c_void_p)]


class _ListStats(ctypes.Structure):
    _fields_ = [("p2p_entries", ctypes.c_int64), ("m2l_entries", ctypes.c_int64),
                ("p2p_pairs", ctypes.c_int64), ("p2p_work_items", ctypes.c_int64),
                ("p2p_max_row_sources", ctypes.c_int64), ("m2p_entries", ctypes.c_int64)]


EXPORTS = ("fmm_tree_build", "fmm_tree_build_ex", "fmm_tree_set_positions", "fmm_tree_view", "fmm_tree_free",
           "fmm_traverse", "fmm_lists_view", "fmm_lists_stats", "fmm_lists_free",
           "fmm_evaluate", "fmm_evaluate_backward", "fmm_direct", "fmm_last_timings", "fmm_mean_timings",
           "fmm_last_error", "fmm_num_terms", "fmm_copy_expansions", "fmm_term_exponents",
           "fmm_traverse_gpu", "fmm_tree_build_gpu", "fmm_evaluate_range",
           "fmm_partition_targets", "fmm_traverse_hybrid", "fmm_evaluate_noalloc",
           "fmm_noalloc_scratch_bytes", "fmm_mutual_plan_stats", "fmm_dispatch_order")

_lib = None


def lib():
    """Load libfmm.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfmm.so is not built (%s); run paper_1209_3516_amd/build_lib.py"
                           % LIB_PATH)
    import torch  # noqa: F401  (its HIP runtime must be the one libfmm binds to)
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint,
                              ctypes.c_double)
    sig = {
        "fmm_tree_build": ([vp, i64, i32, ctypes.POINTER(vp)], i32),
        "fmm_tree_build_ex": ([vp, i64, i32, u32, ctypes.POINTER(vp)], i32),
        "fmm_tree_set_positions": ([vp, vp], i32),
        "fmm_tree_view": ([vp, ctypes.POINTER(_TreeView)], i32),
        "fmm_tree_free": ([vp], None),
        "fmm_traverse": ([vp, dbl, u32, ctypes.POINTER(vp)], i32),
        "fmm_traverse_gpu": ([vp, dbl, u32, ctypes.POINTER(vp), vp], i32),
        "fmm_traverse_hybrid": ([vp, dbl, u32, i32, ctypes.POINTER(vp)], i32),
        "fmm_tree_build_gpu": ([vp, i64, i32, ctypes.POINTER(vp), vp], i32),
        "fmm_lists_view": ([vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                            ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
        "fmm_lists_stats": ([vp, ctypes.POINTER(_ListStats)], i32),
        "fmm_mutual_plan_stats": ([vp, vp, vp], i32),
        "fmm_dispatch_order": ([vp, i32, vp, i64, ctypes.POINTER(i64)], i32),
        "fmm_lists_free": ([vp], None),
        "fmm_evaluate": ([vp, vp, ctypes.POINTER(_EvalOpts), vp, vp, vp, vp], i32),
        "fmm_evaluate_noalloc": ([vp, vp, ctypes.POINTER(_EvalOpts), vp, vp, vp, vp], i32),
        "fmm_noalloc_scratch_bytes": ([], ctypes.c_size_t),
        "fmm_evaluate_range": ([vp, vp, ctypes.POINTER(_EvalOpts), i64, i64, vp, vp, vp, vp],
                               i32),
        "fmm_partition_targets": ([vp, vp, i32, dbl, vp], i32),
        "fmm_evaluate_backward": ([vp, vp, ctypes.POINTER(_EvalOpts), vp, vp, vp, vp, vp, vp,
                                   vp], i32),
        "fmm_direct": ([vp, vp, i64, vp, i64, vp, vp, vp], i32),
        "fmm_last_timings": ([vp, ctypes.POINTER(dbl)], i32),
        "fmm_mean_timings": ([vp, i32, ctypes.POINTER(dbl)], i32),
        "fmm_last_error": ([], ctypes.c_char_p),
        "fmm_num_terms": ([i32], i32),
        "fmm_copy_expansions": ([vp, i32, vp], i32),
        "fmm_term_exponents": ([i32, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc):
    if rc != FMM_OK:
        raise FMMError(rc, lib().fmm_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _t_ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def num_terms(p):
    return lib().fmm_num_terms(int(p))


def term_exponents(p):
    e = np.zeros((num_terms(p), 3), np.int32)
    _check(lib().fmm_term_exponents(int(p), _np_ptr(e)))
    return e


class Tree:
    """Morton octree with at most ncrit bodies per leaf, built on the host.
    box_centres=True: expansion centres at the centres of the Morton cubes."""

    def __init__(self, xyz, ncrit, box_centres=False):
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        self.n = xyz.shape[0]
        self.ncrit = int(ncrit)
        h = ctypes.c_void_p()
        _check(lib().fmm_tree_build_ex(_np_ptr(xyz), self.n, self.ncrit,
                                       FMM_TREE_BOX_CENTRES if box_centres else 0,
                                       ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_device(cls, xyz, ncrit):
        """Build the tree on the GPU from a CUDA float64 tensor [n, 3] (user
        order); identical to Tree(xyz.cpu().numpy(), ncrit)."""
        _check_tensor(xyz, xyz.shape[0], xyz.dtype, "xyz", 3)
        import torch
        if xyz.dtype != torch.float64:
            raise ValueError("xyz must be float64")
        self = cls.__new__(cls)
        self.n = xyz.shape[0]
        self.ncrit = int(ncrit)
        h = ctypes.c_void_p()
        _check(lib().fmm_tree_build_gpu(_t_ptr(xyz), self.n, self.ncrit, ctypes.byref(h),
                                        _stream()))
        self._h = h
        return self

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fmm_tree_free(self._h)
            self._h = None

    def _view(self):
        v = _TreeView()
        _check(lib().fmm_tree_view(self._h, ctypes.byref(v)))
        return v

    @property
    def n_cells(self):
        return self._view().n_cells

    @property
    def max_level(self):
        return self._view().max_level

    def view(self):
        """Copies of the tree arrays as numpy arrays."""
        v = self._view()
        n, nc = v.n, v.n_cells

        def arr(ptr, dtype, count, shape=None):
            if count == 0:
                return np.zeros(shape or (0,), dtype)
            buf = (ctypes.c_byte * (count * np.dtype(dtype).itemsize)).from_address(ptr)
            a = np.frombuffer(buf, dtype=dtype, count=count).copy()
            return a.reshape(shape) if shape else a

        return dict(n=n, n_cells=nc, n_leaves=v.n_leaves, max_level=v.max_level,
                    fp32_exact=bool(v.fp32_exact),
                    perm=arr(v.perm, np.int32, n), keys=arr(v.keys, np.uint64, n),
                    level=arr(v.level, np.int32, nc), parent=arr(v.parent, np.int32, nc),
                    child_begin=arr(v.child_begin, np.int32, nc),
                    n_child=arr(v.n_child, np.int32, nc),
                    body_begin=arr(v.body_begin, np.int64, nc),
                    n_body=arr(v.n_body, np.int64, nc),
                    center=arr(v.center, np.float64, 3 * nc, (nc, 3)),
                    radius=arr(v.radius, np.float64, nc))

    def set_positions(self, xyz):
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        if xyz.shape[0] != self.n:
            raise ValueError("set_positions: wrong number of bodies")
        _check(lib().fmm_tree_set_positions(self._h, _np_ptr(xyz)))


class Lists:
    """P2P and M2L interaction lists from the dual tree traversal, on the host
    or (device=True) on the GPU; both give identical lists.  m2p_max > 0: the
    treecode/FMM hybrid (host only), accepted pairs whose target is a leaf of
    at most m2p_max bodies go to an M2P list."""

    def __init__(self, tree, theta, leaf_first=False, device=False, m2p_max=0):
        h = ctypes.c_void_p()
        flags = FMM_LEAF_FIRST if leaf_first else FMM_MAC_FIRST
        if m2p_max:
            if device:
                raise ValueError("hybrid (M2P) lists are built on the host only")
            _check(lib().fmm_traverse_hybrid(tree._h, float(theta), flags, int(m2p_max),
                                             ctypes.byref(h)))
        elif device:
            _check(lib().fmm_traverse_gpu(tree._h, float(theta), flags, ctypes.byref(h),
                                          _stream()))
        else:
            _check(lib().fmm_traverse(tree._h, float(theta), flags, ctypes.byref(h)))
        self._h = h
        self.tree = tree
        self.theta = float(theta)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fmm_lists_free(self._h)
            self._h = None

    def csr(self, kind):
        ptr, col = ctypes.c_void_p(), ctypes.c_void_p()
        nrows, nnz = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fmm_lists_view(self._h, int(kind), ctypes.byref(ptr), ctypes.byref(col),
                                    ctypes.byref(nrows), ctypes.byref(nnz)))
        p = np.frombuffer((ctypes.c_int64 * (nrows.value + 1)).from_address(ptr.value),
                          dtype=np.int64).copy()
        c = (np.frombuffer((ctypes.c_int32 * nnz.value).from_address(col.value),
                           dtype=np.int32).copy() if nnz.value else np.zeros(0, np.int32))
        return p, c

    def stats(self):
        s = _ListStats()
        _check(lib().fmm_lists_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _ListStats._fields_}

    def mutual_plan_stats(self):
        """Counts of the mutual P2P's work plan (fmm_mutual_plan_stats)."""
        out = np.zeros(5, dtype=np.int64)
        _check(lib().fmm_mutual_plan_stats(self.tree._h, self._h, _np_ptr(out)))
        keys = ("items", "runs", "upper_pairs", "self_pairs", "source_slots")
        return dict(zip(keys, (int(v) for v in out)))

    def dispatch_order(self, kind):
        """The GPU dispatch order of a full evaluation's P2P work items
        (kind FMM_P2P) or M2L cells (FMM_M2L, with -1 padding), as int32
        (fmm_dispatch_order)."""
        n = ctypes.c_int64()
        _check(lib().fmm_dispatch_order(self._h, int(kind), None, 0, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        _check(lib().fmm_dispatch_order(self._h, int(kind), _np_ptr(out), int(out.size),
                                        ctypes.byref(n)))
        return out[:n.value]


def _opts(p, precision, flags=0, fp64_top_levels=-1):
    prec = {"mixed": FMM_MIXED, "fp64": FMM_FP64}[precision]
    return _EvalOpts(int(p), prec, int(fp64_top_levels), int(flags))


def _dtype(precision):
    import torch
    return torch.float64 if precision == "fp64" else torch.float32


def _check_tensor(t, n, dtype, name, cols=None):
    shape = (n,) if cols is None else (n, cols)
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
        raise ValueError("%s must be a contiguous %s CUDA tensor of shape %s" % (name, dtype, shape))


def evaluate(tree, lists, q, p, precision="mixed", grad=True, timing=False, keep_stages=False,
             fp64_top_levels=-1, out=None, serial=False, body_range=None, m2l_mfma=False,
             mutual_p2p=False):
    """One FMM evaluation.  q: CUDA tensor [n] (float32 for "mixed", float64 for
    "fp64"), user order.  Returns (phi [n], grad [n,3] or None).  serial=True
    keeps the near field on the caller's stream (no overlap with the far field).
    body_range=(b0, b1): only the targets at Morton positions [b0, b1) (leaf
    boundaries, e.g. from partition()); other output entries are not written.
    m2l_mfma=True: M2L batched by translation vector on the matrix cores
    (trees built with box_centres=True, mixed precision).  mutual_p2p=True:
    each unordered pair of P2P leaves evaluated once for both (mixed
    precision, leaves of at most 64 bodies, all targets)."""
    import torch
    dt = _dtype(precision)
    _check_tensor(q, tree.n, dt, "q")
    if out is None:
        phi = torch.empty(tree.n, dtype=dt, device=q.device)
        g = torch.empty(tree.n, 3, dtype=dt, device=q.device) if grad else None
    else:
        phi, g = out
    flags = ((FMM_EVAL_TIMING if timing else 0) | (FMM_EVAL_KEEP_STAGES if keep_stages else 0)
             | (FMM_EVAL_SERIAL if serial else 0) | (FMM_EVAL_M2L_MFMA if m2l_mfma else 0)
             | (FMM_EVAL_MUTUAL_P2P if mutual_p2p else 0))
    o = _opts(p, precision, flags, fp64_top_levels)
    if body_range is None:
        _check(lib().fmm_evaluate(tree._h, lists._h, ctypes.byref(o), _t_ptr(q), _t_ptr(phi),
                                  _t_ptr(g), _stream()))
    else:
        b0, b1 = (int(v) for v in body_range)
        _check(lib().fmm_evaluate_range(tree._h, lists._h, ctypes.byref(o), b0, b1, _t_ptr(q),
                                        _t_ptr(phi), _t_ptr(g), _stream()))
    return phi, g


def evaluate_noalloc(tree, lists, q, phi, grad, p, precision="mixed", fp64_top_levels=-1):
    """fmm_evaluate_noalloc: the evaluation into the given output tensors (phi
    [n], grad [n,3] or None) with no device allocation by the library; the
    tree and lists must already be on the device for this precision (one
    evaluate() call puts them there).  Returns (phi, grad)."""
    dt = _dtype(precision)
    _check_tensor(q, tree.n, dt, "q")
    _check_tensor(phi, tree.n, dt, "phi")
    if grad is not None:
        _check_tensor(grad, tree.n, dt, "grad", 3)
    o = _opts(p, precision, 0, fp64_top_levels)
    _check(lib().fmm_evaluate_noalloc(tree._h, lists._h, ctypes.byref(o), _t_ptr(q),
                                      _t_ptr(phi), _t_ptr(grad), _stream()))
    return phi, grad


def noalloc_scratch_bytes():
    """Size of the fixed device array fmm_evaluate_noalloc works in."""
    return int(lib().fmm_noalloc_scratch_bytes())


def m2l_weight(p):
    """Estimated cost of one M2L entry in units of one P2P pair at order p: the
    contraction's multiply-adds, C(p+5, 6), plus about 8 operations per
    derivative term of the recurrence, over 14 instructions per pair."""
    from math import comb
    return (comb(p + 5, 6) + 8 * (p * (p + 1) * (p + 2) // 6)) / 14.0


def partition(tree, lists, n_parts, weight=None, p=4):
    """Split the targets into n_parts contiguous Morton ranges of about equal
    work (P2P pairs + weight * M2L entries; weight defaults to m2l_weight(p)).
    Returns int64 bounds [n_parts + 1]; range k is [bounds[k], bounds[k+1])."""
    w = m2l_weight(p) if weight is None else float(weight)
    bounds = np.zeros(int(n_parts) + 1, np.int64)
    _check(lib().fmm_partition_targets(tree._h, lists._h, int(n_parts), w, _np_ptr(bounds)))
    return bounds


def evaluate_backward(tree, lists, q, grad_q, w, p, precision="mixed", need_dq=True,
                      need_dx=True, fp64_top_levels=-1, v=None, mutual_p2p=False):
    """Backward of L = sum_i w_i phi_i + sum_i v_i . grad_i (v optional):
    returns (dL/dq [n], dL/dx [n,3]).  mutual_p2p=True: the pass with charges
    alone (v None) uses the mutual P2P."""
    import torch
    dt = _dtype(precision)
    _check_tensor(w, tree.n, dt, "w")
    if v is not None:
        _check_tensor(v, tree.n, dt, "v", 3)
    dq = torch.empty(tree.n, dtype=dt, device=w.device) if need_dq else None
    dx = torch.empty(tree.n, 3, dtype=dt, device=w.device) if need_dx else None
    o = _opts(p, precision, FMM_EVAL_MUTUAL_P2P if mutual_p2p else 0, fp64_top_levels)
    _check(lib().fmm_evaluate_backward(tree._h, lists._h, ctypes.byref(o), _t_ptr(q),
                                       _t_ptr(grad_q), _t_ptr(w), _t_ptr(v), _t_ptr(dq),
                                       _t_ptr(dx), _stream()))
    return dq, dx


def direct(xyz, q, targets):
    """FP64 direct sum on the GPU at the given target indices (int64 CUDA tensor)."""
    import torch
    n = xyz.shape[0]
    _check_tensor(xyz, n, torch.float64, "xyz", 3)
    _check_tensor(q, n, torch.float64, "q")
    m = targets.shape[0]
    phi = torch.empty(m, dtype=torch.float64, device=xyz.device)
    g = torch.empty(m, 3, dtype=torch.float64, device=xyz.device)
    _check(lib().fmm_direct(_t_ptr(xyz), _t_ptr(q), n, _t_ptr(targets), m, _t_ptr(phi),
                            _t_ptr(g), _stream()))
    return phi, g


def last_timings(lists):
    """Per-phase device times (ms) of the last evaluation run with timing=True."""
    ms = (ctypes.c_double * len(PHASES))()
    _check(lib().fmm_last_timings(lists._h, ms))
    return dict(zip(PHASES, list(ms)))


TIMING_HISTORY = 64


def mean_timings(lists, n):
    """Mean per-phase device times (ms) of the last n evaluations, all run with
    timing=True one after another (n <= TIMING_HISTORY); read after the run,
    so that the run itself has no waits between evaluations."""
    ms = (ctypes.c_double * len(PHASES))()
    _check(lib().fmm_mean_timings(lists._h, int(n), ms))
    return dict(zip(PHASES, list(ms)))


def copy_expansions(lists, kind, p):
    """Expansions of the last evaluation (order p) as (n_cells, T) float64, in the
    library's term order (term_exponents(p)): kind 0 multipoles, 1 locals after
    M2L (needs keep_stages=True), 2 locals after L2L."""
    T = num_terms(p)
    out = np.zeros((lists.tree.n_cells, T), np.float64)
    _check(lib().fmm_copy_expansions(lists._h, int(kind), _np_ptr(out)))
    return out


def _make_autograd():
    import torch

    class FMMPotential(torch.autograd.Function):
        """phi = FMM(x, q) with the tree and lists held fixed.  Backward of
        L = sum_i w_i phi_i: dL/dq = phi[w] (one more evaluation with charges w),
        dL/dx = w * grad[q] + q * grad[w], both from the library."""

        @staticmethod
        def forward(ctx, x, q, tree, lists, p, precision, fp64_top_levels):
            phi, g = evaluate(tree, lists, q.detach().contiguous(), p, precision, grad=True,
                              fp64_top_levels=fp64_top_levels)
            ctx.save_for_backward(q, g)
            ctx.cfg = (tree, lists, p, precision, fp64_top_levels)
            ctx.mark_non_differentiable(g)
            return phi

        @staticmethod
        def backward(ctx, w):
            q, g = ctx.saved_tensors
            tree, lists, p, precision, top = ctx.cfg
            need_dx, need_dq = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            dq, dx = evaluate_backward(tree, lists, q.detach().contiguous(), g,
                                       w.contiguous(), p, precision, need_dq=need_dq,
                                       need_dx=need_dx, fp64_top_levels=top)
            return dx, dq, None, None, None, None, None

    class FMMField(torch.autograd.Function):
        """(phi, grad phi) = FMM(x, q), both differentiable, tree and lists fixed.
        Backward of L = sum w.phi + sum v.grad: dL/dq = Phi (charges w plus
        dipoles -v), dL/dx = w grad[q] + q grad Phi + H[q] v."""

        @staticmethod
        def forward(ctx, x, q, tree, lists, p, precision, fp64_top_levels):
            phi, g = evaluate(tree, lists, q.detach().contiguous(), p, precision, grad=True,
                              fp64_top_levels=fp64_top_levels)
            ctx.save_for_backward(q, g)
            ctx.cfg = (tree, lists, p, precision, fp64_top_levels)
            return phi, g

        @staticmethod
        def backward(ctx, w, v):
            q, g = ctx.saved_tensors
            tree, lists, p, precision, top = ctx.cfg
            need_dx, need_dq = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            if w is None:
                w = torch.zeros_like(q)
            dq, dx = evaluate_backward(tree, lists, q.detach().contiguous(), g, w.contiguous(),
                                       p, precision, need_dq=need_dq, need_dx=need_dx,
                                       fp64_top_levels=top,
                                       v=None if v is None else v.contiguous())
            return dx, dq, None, None, None, None, None

    return FMMPotential, FMMField


_autograd_fn = None


def potential(x, q, tree, lists, p, precision="mixed", fp64_top_levels=-1):
    """Differentiable FMM potential.  x: CUDA tensor [n,3] - the positions the
    tree was built from (the tree holds its own copy; x carries the gradient);
    q: CUDA tensor [n].  Returns phi [n]."""
    global _autograd_fn
    if _autograd_fn is None:
        _autograd_fn = _make_autograd()
    return _autograd_fn[0].apply(x, q, tree, lists, p, precision, fp64_top_levels)


def field(x, q, tree, lists, p, precision="mixed", fp64_top_levels=-1):
    """Differentiable potential and gradient: returns (phi [n], grad [n,3]); a
    loss may depend on both (the backward then also uses dipole sources and
    Hessian-vector products)."""
    global _autograd_fn
    if _autograd_fn is None:
        _autograd_fn = _make_autograd()
    return _autograd_fn[1].apply(x, q, tree, lists, p, precision, fp64_top_levels)
