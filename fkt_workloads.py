"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers: it holds none of the method's
arithmetic (no kernels, no tree, no expansion), so that the CPU oracle and
the HIP path can both consume the same inputs without sharing code.

Every generator uses ``numpy.random.default_rng(seed)`` and returns float64
arrays in row-major layout (points: n x d, right-hand sides: n x nrhs).

The workloads stand in for the paper's synthetic runs (points uniform in a
box, Section 5.1) and for its real-data experiments, whose datasets are not
used here.
"""
from __future__ import annotations

import numpy as np


def uniform_cube(n: int, d: int, seed: int) -> np.ndarray:
    """n points i.i.d. uniform in [0, 1]^d."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n, d))


def gaussian_mixture(n: int, d: int, ncomp: int, std: float, seed: int) -> np.ndarray:
    """n points from an equal-weight isotropic Gaussian mixture.

    Component means are uniform in [0, 1]^d; each point picks a component
    uniformly at random and adds N(0, std^2 I) noise.
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(0.0, 1.0, size=(ncomp, d))
    comp = rng.integers(0, ncomp, size=n)
    return means[comp] + std * rng.standard_normal(size=(n, d))


def normal_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides x ~ N(0, 1), shape (n, nrhs)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(n, nrhs))


def subsample(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices out of range(n), sorted (without replacement)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def clustered_duplicates(n: int, d: int, ndistinct: int, seed: int) -> np.ndarray:
    """n points drawn (with repetition) from ndistinct uniform sites.

    Exercises coincident points: many exact duplicates of each site.
    """
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, 1.0, size=(ndistinct, d))
    return sites[rng.integers(0, ndistinct, size=n)]


def gp_targets(X: np.ndarray, lengthscale: float, sigma2: float, nfeat: int, seed: int) -> np.ndarray:
    """y = f(X) + noise, f a random-Fourier-feature draw of a Matern-5/2 GP.

    Frequencies follow the Matern-5/2 spectral density, a multivariate
    Student-t with 5 degrees of freedom scaled by 1/lengthscale; phases are
    uniform; f = sqrt(2/D) sum_i w_i cos(omega_i . x + b_i), w_i ~ N(0, 1);
    the noise is N(0, sigma2).
    """
    rng = np.random.default_rng(seed)
    n, d = X.shape
    g = rng.standard_normal(size=(nfeat, d))
    u = rng.chisquare(5.0, size=(nfeat, 1))
    omega = g / lengthscale * np.sqrt(5.0 / u)
    b = rng.uniform(0.0, 2.0 * np.pi, size=nfeat)
    w = rng.standard_normal(size=nfeat)
    f = np.sqrt(2.0 / nfeat) * (np.cos(X @ omega.T + b) @ w)
    return f + np.sqrt(sigma2) * rng.standard_normal(size=n)


def instance_sizes(ninst: int, nmin: int, nmax: int, seed: int) -> np.ndarray:
    """ninst sizes, log-uniform in [nmin, nmax] (rounded to integers)."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=ninst))).astype(np.int64)


def batched_instances(sizes, d: int, seed: int):
    """Independent point sets uniform in [0, 1]^d, one per size (instance i
    drawn with seed + i); returns (concatenated points, int64 offsets)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    X = np.concatenate([uniform_cube(int(m), d, seed + i) for i, m in enumerate(sizes)], axis=0) if len(sizes) else \
        np.zeros((0, d))
    return X, off


# Named workloads: (points recipe, rhs recipe). Sizes follow the problem
# statements; seeds are fixed so every consumer sees identical inputs.
WORKLOADS = {
    # small correctness case: Gaussian kernel, length scale 0.1, leaf 128, p=4
    "cube3_n2k_gauss": dict(n=2000, d=3, pts_seed=1001, rhs_seed=2001, nrhs=1,
                            kernel="gaussian", lengthscale=0.1, leaf=128, order=4),
    # headline case: one million uniform points in the unit cube, leaf 256, p=6
    "cube3_n1m_matern32": dict(n=1_000_000, d=3, pts_seed=1002, rhs_seed=2002, nrhs=1,
                               kernel="matern32", lengthscale=0.05, leaf=256, order=6),
    "cube3_n1m_laplace": dict(n=1_000_000, d=3, pts_seed=1002, rhs_seed=2002, nrhs=1,
                              kernel="laplace", lengthscale=1.0, leaf=256, order=6),
    # Gaussian-process solve: 200k points from an 8-component mixture in d=4
    # (std 0.15), Matern-5/2 length scale 0.3, noise variance 1e-2
    # many independent instances: 256 sets in d = 3, sizes log-uniform in
    # [1e3, 1e5], rational quadratic (alpha 1, length scale 0.2), 4 RHS, FP32
    "batch256_rq": dict(ninst=256, nmin=1000, nmax=100_000, d=3, size_seed=1004, pts_seed=10_000, rhs_seed=2004,
                        nrhs=4, kernel="ratquad", lengthscale=0.2, alpha=1.0, order=6),
    # mixed precision, many RHS: 500k points, 10-component mixture in d = 5
    # (std 0.1), Gaussian length scale 0.2, 32 RHS, p = 8
    "gmm5_n500k_gauss32": dict(n=500_000, d=5, ncomp=10, std=0.1, pts_seed=1003, rhs_seed=2003, nrhs=32,
                               kernel="gaussian", lengthscale=0.2, order=8),
    "gmm4_n200k_gp": dict(n=200_000, d=4, ncomp=8, std=0.15, pts_seed=1005, rhs_seed=2005,
                          kernel="matern52", lengthscale=0.3, sigma2=1e-2, nfeat=2048, leaf=256),
}


def make_points(spec: dict) -> np.ndarray:
    return uniform_cube(spec["n"], spec["d"], spec["pts_seed"])


def make_rhs(spec: dict) -> np.ndarray:
    return normal_rhs(spec["n"], spec["nrhs"], spec["rhs_seed"])
