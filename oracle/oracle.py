"""ctypes wrapper of the FP64 oracle (oracle/liboracle.so).

Test infrastructure only.  Inputs and outputs are numpy float64 / int arrays.
"""
import ctypes
import os
import time

import numpy as np

from . import build_oracle

_lib = None

P2P = 0
M2L = 1


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(build_oracle.LIB):
        build_oracle.build()
    lib = ctypes.CDLL(build_oracle.LIB)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int
    dbl = ctypes.c_double
    lib.oracle_build.argtypes = [vp, i64, i32, dbl, i32, ctypes.POINTER(vp)]
    lib.oracle_build.restype = i32
    lib.oracle_build_hybrid.argtypes = [vp, i64, i32, dbl, i32, i32, ctypes.POINTER(vp)]
    lib.oracle_build_hybrid.restype = i32
    lib.oracle_build_tree.argtypes = [vp, i64, i32, i32, ctypes.POINTER(vp)]
    lib.oracle_build_tree.restype = i32
    lib.oracle_traverse.argtypes = [vp, dbl, i32, i32, vp, i64]
    lib.oracle_traverse.restype = i32
    lib.oracle_set_threads.argtypes = [i32]
    lib.oracle_set_threads.restype = None
    lib.oracle_get_threads.argtypes = []
    lib.oracle_get_threads.restype = i32
    lib.oracle_last_phase_seconds.argtypes = [vp]
    lib.oracle_last_phase_seconds.restype = None
    lib.oracle_free.argtypes = [vp]
    lib.oracle_free.restype = None
    lib.oracle_num_cells.argtypes = [vp]
    lib.oracle_num_cells.restype = i64
    lib.oracle_tree.argtypes = [vp] + [vp] * 10
    lib.oracle_tree.restype = None
    lib.oracle_list_nnz.argtypes = [vp, i32]
    lib.oracle_list_nnz.restype = i64
    lib.oracle_list.argtypes = [vp, i32, vp, vp]
    lib.oracle_list.restype = None
    lib.oracle_num_terms.argtypes = [i32]
    lib.oracle_num_terms.restype = i32
    lib.oracle_term_exponents.argtypes = [i32, vp]
    lib.oracle_term_exponents.restype = None
    lib.oracle_evaluate.argtypes = [vp, i32] + [vp] * 10
    lib.oracle_evaluate.restype = i32
    lib.oracle_evaluate_leaves.argtypes = [vp, i32, vp, vp, i64, vp, vp, vp]
    lib.oracle_evaluate_leaves.restype = i64
    lib.oracle_set_positions.argtypes = [vp, vp]
    lib.oracle_set_positions.restype = None
    lib.oracle_evaluate_general.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.oracle_evaluate_general.restype = i32
    lib.oracle_direct_general.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp, vp, vp]
    lib.oracle_direct_general.restype = None
    lib.oracle_op_p2m_dipole.argtypes = [i32, vp, vp, vp, i64, vp]
    lib.oracle_op_p2m_dipole.restype = None
    lib.oracle_op_l2p_hessian.argtypes = [i32, vp, vp, vp, vp, i64, vp]
    lib.oracle_op_l2p_hessian.restype = None
    lib.oracle_direct.argtypes = [vp, vp, i64, vp, i64, vp, vp]
    lib.oracle_direct.restype = None
    lib.oracle_op_derivatives.argtypes = [i32, vp, vp]
    lib.oracle_op_p2m.argtypes = [i32, vp, vp, vp, i64, vp]
    lib.oracle_op_m2m.argtypes = [i32, vp, vp, vp, vp]
    lib.oracle_op_m2l.argtypes = [i32, vp, vp, vp, vp]
    lib.oracle_op_l2l.argtypes = [i32, vp, vp, vp, vp]
    lib.oracle_op_l2p.argtypes = [i32, vp, vp, vp, i64, vp, vp]
    lib.oracle_op_m2p.argtypes = [i32, vp, vp, vp, i64, vp, vp]
    for name in ("oracle_op_derivatives", "oracle_op_p2m", "oracle_op_m2m", "oracle_op_m2l",
                 "oracle_op_l2l", "oracle_op_l2p"):
        getattr(lib, name).restype = None
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_terms(p):
    return _load().oracle_num_terms(p)


def term_exponents(p):
    """(T, 3) int array: exponents (nx, ny, nz) of each expansion term."""
    out = np.zeros((num_terms(p), 3), dtype=np.int32)
    _load().oracle_term_exponents(p, _p(out))
    return out


class OracleFMM:
    """Tree + interaction lists built by the oracle; evaluate() runs the FP64 FMM.
    m2p_max > 0: the treecode/FMM hybrid lists (accepted pairs whose target is
    a leaf of at most m2p_max bodies go to the M2P list, kind 2)."""

    def __init__(self, xyz, ncrit, theta, leaf_first=False, m2p_max=0, select_leaves=None,
                 box_centres=False):
        """select_leaves: None for the whole traversal, or a function of the
        tree (the dict of tree()) returning leaf cells; the lists then hold only
        the rows of those leaves and of their ancestors (the restricted
        traversal), enough for evaluate_leaves on them.  box_centres: cell
        centres at the centres of the Morton cubes instead of the middles of
        the cells' bounding boxes."""
        lib = _load()
        self.xyz = _f64(xyz, (-1, 3))
        self.n = self.xyz.shape[0]
        h = ctypes.c_void_p()
        self.restricted_to = None
        t0 = time.perf_counter()
        if lib.oracle_build_tree(_p(self.xyz), self.n, int(ncrit), 1 if box_centres else 0,
                                 ctypes.byref(h)) != 0:
            raise ValueError("oracle_build_tree failed")
        t1 = time.perf_counter()
        self._h = h
        leaves, n_leaves = None, 0
        if select_leaves is not None:
            leaves = np.ascontiguousarray(select_leaves(self.tree()), dtype=np.int32)
            n_leaves = leaves.shape[0]
            self.restricted_to = leaves
        t1b = time.perf_counter()
        if lib.oracle_traverse(h, float(theta), 1 if leaf_first else 0, int(m2p_max),
                               _p(leaves), n_leaves) != 0:
            raise ValueError("oracle_traverse failed")
        # wall-clock seconds of the tree build and of the traversal
        self.build_seconds = (t1 - t0, time.perf_counter() - t1b)
        self._h = h
        self.ncrit = ncrit
        self.theta = theta

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.oracle_free(self._h)
            self._h = None

    @property
    def num_cells(self):
        return _lib.oracle_num_cells(self._h)

    def tree(self):
        nc = self.num_cells
        n = self.n
        t = dict(perm=np.zeros(n, np.int32), keys=np.zeros(n, np.uint64),
                 level=np.zeros(nc, np.int32), parent=np.zeros(nc, np.int32),
                 child_begin=np.zeros(nc, np.int32), n_child=np.zeros(nc, np.int32),
                 body_begin=np.zeros(nc, np.int64), n_body=np.zeros(nc, np.int64),
                 center=np.zeros((nc, 3), np.float64), radius=np.zeros(nc, np.float64))
        _lib.oracle_tree(self._h, *[_p(t[k]) for k in (
            "perm", "keys", "level", "parent", "child_begin", "n_child", "body_begin",
            "n_body", "center", "radius")])
        return t

    def lists(self, kind):
        nnz = _lib.oracle_list_nnz(self._h, kind)
        ptr = np.zeros(self.num_cells + 1, np.int64)
        col = np.zeros(nnz, np.int32)
        _lib.oracle_list(self._h, kind, _p(ptr), _p(col))
        return ptr, col

    def evaluate(self, q, p, staged=False):
        """Returns dict(phi[n], grad[n,3]) in user order; with staged=True also
        near/far fields (sorted order) and the M, L_m2l, L arrays (cell order)."""
        if self.restricted_to is not None:
            raise ValueError("restricted lists: use evaluate_leaves on the chosen leaves")
        q = _f64(q, (-1,))
        n, nc, T = self.n, self.num_cells, num_terms(p)
        out = dict(phi=np.zeros(n), grad=np.zeros((n, 3)))
        if staged:
            out.update(near_phi=np.zeros(n), near_grad=np.zeros((n, 3)), far_phi=np.zeros(n),
                       far_grad=np.zeros((n, 3)), M=np.zeros((nc, T)), L_m2l=np.zeros((nc, T)),
                       L=np.zeros((nc, T)))
        g = out.get
        rc = _lib.oracle_evaluate(self._h, int(p), _p(q), _p(out["phi"]), _p(out["grad"]),
                                  _p(g("near_phi")), _p(g("near_grad")), _p(g("far_phi")),
                                  _p(g("far_grad")), _p(g("M")), _p(g("L_m2l")), _p(g("L")))
        if rc != 0:
            raise ValueError("oracle_evaluate failed")
        return out


PHASES = ("upward", "m2l", "downward", "l2p", "p2p")


def set_threads(n):
    """OpenMP threads of the oracle's later calls (n <= 0: all processors)."""
    _load().oracle_set_threads(int(n))


def get_threads():
    return _load().oracle_get_threads()


def last_phase_seconds():
    """Wall-clock seconds of the phases of the last full evaluation in this
    process: dict over PHASES."""
    out = np.zeros(5)
    _load().oracle_last_phase_seconds(_p(out))
    return dict(zip(PHASES, out.tolist()))


def set_positions(o, xyz):
    """Move the bodies (user order) with the tree, centres, radii and lists frozen."""
    _load().oracle_set_positions(o._h, _p(_f64(xyz, (-1, 3))))


def evaluate_general(o, p, q, s=None, v=None):
    """Charges q and optional dipoles s [n,3] as sources; optional per-body
    vectors v [n,3] for the Hessian of the charge field applied to v.
    Returns (phi, grad, hv) in user order (hv None without v)."""
    lib = _load()
    n = o.n
    q = _f64(q, (-1,))
    s = None if s is None else _f64(s, (-1, 3))
    v = None if v is None else _f64(v, (-1, 3))
    phi, grad = np.zeros(n), np.zeros((n, 3))
    hv = None if v is None else np.zeros((n, 3))
    rc = lib.oracle_evaluate_general(o._h, int(p), _p(q), _p(s), _p(v), _p(phi), _p(grad), _p(hv))
    if rc != 0:
        raise ValueError("oracle_evaluate_general failed")
    return phi, grad, hv


def direct_general(xyz, q, s=None, targets=None, v=None):
    """Direct sum with charges q and optional dipoles s; optional vectors v
    (one per target) for the Hessian of the charge field.  Returns (phi, grad, hv)."""
    lib = _load()
    xyz = _f64(xyz, (-1, 3))
    n = xyz.shape[0]
    q = _f64(q, (-1,))
    s = None if s is None else _f64(s, (-1, 3))
    targets = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(
        targets, dtype=np.int64)
    m = targets.shape[0]
    v = None if v is None else _f64(v, (-1, 3))
    phi, grad = np.zeros(m), np.zeros((m, 3))
    hv = None if v is None else np.zeros((m, 3))
    lib.oracle_direct_general(_p(xyz), _p(q), _p(s), n, _p(targets), m, _p(v), _p(phi), _p(grad),
                              _p(hv))
    return phi, grad, hv


def p2m_dipole(p, X, xyz, s):
    xyz = _f64(xyz, (-1, 3))
    M = np.zeros(num_terms(p))
    _load().oracle_op_p2m_dipole(p, _p(_f64(X, (3,))), _p(xyz), _p(_f64(s, (-1, 3))),
                                 xyz.shape[0], _p(M))
    return M


def l2p_hessian(p, XA, L, y, v):
    y = _f64(y, (-1, 3))
    hv = np.zeros((y.shape[0], 3))
    _load().oracle_op_l2p_hessian(p, _p(_f64(XA, (3,))), _p(_f64(L)), _p(y), _p(_f64(v, (-1, 3))),
                                  y.shape[0], _p(hv))
    return hv


def evaluate_leaves(o, q, p, leaves):
    """The full evaluation restricted to the bodies of the given leaf cells (same
    arithmetic in the same order).  Returns (user_index, phi, grad)."""
    lib = _load()
    q = _f64(q, (-1,))
    leaves = np.ascontiguousarray(leaves, dtype=np.int32)
    if o.restricted_to is not None and not np.all(np.isin(leaves, o.restricted_to)):
        raise ValueError("leaves outside the restricted traversal")
    t = o.tree()
    nb = int(t["n_body"][leaves].sum())
    idx = np.zeros(nb, np.int64)
    phi = np.zeros(nb)
    grad = np.zeros((nb, 3))
    got = lib.oracle_evaluate_leaves(o._h, int(p), _p(q), _p(leaves), leaves.shape[0], _p(idx),
                                     _p(phi), _p(grad))
    if got != nb:
        raise ValueError("oracle_evaluate_leaves failed")
    return idx, phi, grad


def direct(xyz, q, targets=None):
    """FP64 direct sum (zero-distance pairs skipped) at the given target indices."""
    lib = _load()
    xyz = _f64(xyz, (-1, 3))
    q = _f64(q, (-1,))
    n = xyz.shape[0]
    targets = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(
        targets, dtype=np.int64)
    m = targets.shape[0]
    phi = np.zeros(m)
    grad = np.zeros((m, 3))
    lib.oracle_direct(_p(xyz), _p(q), n, _p(targets), m, _p(phi), _p(grad))
    return phi, grad


def derivatives(p, R):
    D = np.zeros(num_terms(p))
    _load().oracle_op_derivatives(p, _p(_f64(R, (3,))), _p(D))
    return D


def p2m(p, X, xyz, q):
    xyz = _f64(xyz, (-1, 3))
    M = np.zeros(num_terms(p))
    _load().oracle_op_p2m(p, _p(_f64(X, (3,))), _p(xyz), _p(_f64(q, (-1,))), xyz.shape[0],
                          _p(M))
    return M


def m2m(p, XP, Xc, Mc):
    MP = np.zeros(num_terms(p))
    _load().oracle_op_m2m(p, _p(_f64(XP, (3,))), _p(_f64(Xc, (3,))), _p(_f64(Mc)), _p(MP))
    return MP


def m2l(p, XA, XB, M):
    L = np.zeros(num_terms(p))
    _load().oracle_op_m2l(p, _p(_f64(XA, (3,))), _p(_f64(XB, (3,))), _p(_f64(M)), _p(L))
    return L


def l2l(p, XP, Xc, LP):
    Lc = np.zeros(num_terms(p))
    _load().oracle_op_l2l(p, _p(_f64(XP, (3,))), _p(_f64(Xc, (3,))), _p(_f64(LP)), _p(Lc))
    return Lc


def m2p(p, XB, M, y):
    """Multipole M (order p, about XB) evaluated at the points y: (phi, grad)."""
    y = _f64(y, (-1, 3))
    phi = np.zeros(y.shape[0])
    grad = np.zeros((y.shape[0], 3))
    _load().oracle_op_m2p(p, _p(_f64(XB, (3,))), _p(_f64(M)), _p(y), y.shape[0], _p(phi),
                          _p(grad))
    return phi, grad


def l2p(p, XA, L, y):
    y = _f64(y, (-1, 3))
    phi = np.zeros(y.shape[0])
    grad = np.zeros((y.shape[0], 3))
    _load().oracle_op_l2p(p, _p(_f64(XA, (3,))), _p(_f64(L)), _p(y), y.shape[0], _p(phi),
                          _p(grad))
    return phi, grad
