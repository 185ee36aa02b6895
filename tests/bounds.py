"""Error measures shared by the parity tests.

Every comparison of a GPU result with the oracle checks two things:
  * the relative L2 error over all compared bodies (R12: e = |d|_2 / |ref|_2);
  * a per-body bound, so that an error confined to a few bodies (one leaf of
    thirty among a million moves the global norm by about 5e-6) cannot hide
    under the norm: for every body i,
        |got_i - ref_i| <= PER_BODY * tol * max(|ref_i|, rms(ref)),
    with |.| the Euclidean norm of the body's value (a scalar potential or a
    gradient 3-vector).  The floor rms(ref) keeps bodies whose exact value is
    near zero from demanding a relative accuracy no summation order gives.
"""
import numpy as np

PER_BODY = 10.0


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def per_body_ratio(got, ref):
    """max_i |got_i - ref_i| / max(|ref_i|, rms(ref)) over bodies i."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.ndim == 1:
        d, r = np.abs(got - ref), np.abs(ref)
    else:
        d, r = np.linalg.norm(got - ref, axis=1), np.linalg.norm(ref, axis=1)
    if r.size == 0:
        return 0.0
    rms = np.sqrt(np.mean(r * r))
    floor = np.maximum(r, rms if rms > 0 else 1.0)
    return float(np.max(d / floor))


def assert_close(got, ref, tol, what=""):
    """Relative L2 error <= tol and the per-body bound PER_BODY * tol."""
    e = rel(got, ref)
    m = per_body_ratio(got, ref)
    assert e <= tol, "%s: relative L2 error %.3e > %.1e" % (what, e, tol)
    assert m <= PER_BODY * tol, "%s: per-body error %.3e > %.1e" % (what, m, PER_BODY * tol)
    return e, m
