"""Seeded synthetic inputs for the Laplace FMM (positions, charges, weights).

This module holds only random-number generation: no part of the method's
arithmetic.  Every value is drawn in FP64 from numpy's PCG64 and rounded to
FP32 once, then returned as FP64, so every consumer (host tree, GPU kernels in
either precision, the FP64 oracle) sees exactly the same points and charges.

Workloads (the paper evaluates bodies placed at random in a cube, section 3.5):
  * uniform : x ~ U[0,1)^3
  * plummer : Plummer sphere with scale radius 1, cut at r = 10 (radius from
              the inverse of the enclosed-mass fraction r^3 / (1 + r^2)^(3/2),
              direction uniform on the sphere)
Charges: U[-1, 1] ("signed"), or 1/N ("positive").
Seeds: positions 1, charges 2, weights 3, sampled targets 4, dipoles 5.
"""
import numpy as np

SEED_POS = 1
SEED_CHARGE = 2
SEED_WEIGHT = 3
SEED_SAMPLE = 4
SEED_DIPOLE = 5


def _f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_cube(n, seed=SEED_POS):
    return _f32(_rng(seed).random((n, 3)))


def plummer(n, seed=SEED_POS, r_max=10.0):
    rng = _rng(seed)
    m_max = r_max ** 3 / (1.0 + r_max ** 2) ** 1.5
    X = rng.uniform(0.0, m_max, size=n)
    X = np.maximum(X, np.finfo(np.float64).tiny)
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    cos_t = rng.uniform(-1.0, 1.0, size=n)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    xyz = np.stack([r * sin_t * np.cos(phi), r * sin_t * np.sin(phi), r * cos_t], axis=1)
    return _f32(xyz)


def charges(n, kind="signed", seed=SEED_CHARGE):
    if kind == "signed":
        return _f32(_rng(seed).uniform(-1.0, 1.0, size=n))
    if kind == "positive":
        return _f32(np.full(n, 1.0 / n))
    raise ValueError(kind)


def weights(n, seed=SEED_WEIGHT):
    return _f32(_rng(seed).standard_normal(n))


def dipoles(n, seed=SEED_DIPOLE):
    return _f32(_rng(seed).standard_normal((n, 3)))


def sample_targets(n, s=1000, seed=SEED_SAMPLE):
    if s >= n:
        return np.arange(n, dtype=np.int64)
    return np.sort(_rng(seed).choice(n, s, replace=False)).astype(np.int64)


def positions(n, dist="uniform", seed=SEED_POS):
    if dist == "uniform":
        return uniform_cube(n, seed)
    if dist == "plummer":
        return plummer(n, seed)
    raise ValueError(dist)


# The evaluation workloads: (name, distribution, N, charges, p, theta, ncrit).
CONFIGS = {
    "uniform-1e4-p4": dict(dist="uniform", n=10_000, charges="signed", p=4, theta=0.4,
                           ncrit=64),
    "uniform-1e6-p4": dict(dist="uniform", n=1_000_000, charges="signed", p=4, theta=0.4,
                           ncrit=64),
    "plummer-1e6-p6": dict(dist="plummer", n=1_000_000, charges="positive", p=6,
                           theta=0.35, ncrit=32),
    "uniform-1e7-p8": dict(dist="uniform", n=10_000_000, charges="signed", p=8, theta=0.3,
                           ncrit=64),
}
