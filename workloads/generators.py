"""Seeded synthetic stand-ins for the paper's evaluation data.

The paper measures on the seed-spreader generator of Gan and Tao (SS-simden /
SS-varden), on UniformFill and on real data sets (experiments section, data-set
paragraph).  None of those files or that generator are available, so every workload
here is drawn from numpy's PCG64 with a fixed seed.  The shapes follow the five
evaluation workloads of this project:

* 2D Gaussian blobs, n = 20,000 (10 blobs, sigma 50, 10 % uniform noise);
* a 3D seed-spreader random walk, n = 1,000,000 over [0, 1e5]^3;
* 5D and 7D Gaussian mixtures, n = 2,000,000 (20 components, sigma 1, 5 % noise);
* a 3D seed-spreader cloud of 10,000,000 points over [0, 1e6]^3 with a 4 x 4
  (eps, minPts) grid;
* 256 independent Gaussian-mixture clouds of log-uniform size 1e3 .. 1e6 in
  d in {2, 3, 5}.

Nothing in this module computes a distance or a cluster: it only draws numbers.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1912062550


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _unit_vectors(rng: np.random.Generator, m: int, d: int) -> np.ndarray:
    v = rng.standard_normal((m, d))
    nrm = np.sqrt((v * v).sum(axis=1, keepdims=True))
    nrm[nrm == 0.0] = 1.0
    return v / nrm


def gaussian_mixture(
    n: int,
    d: int,
    k: int,
    sigma,
    domain: float,
    noise_frac: float,
    rng: np.random.Generator,
) -> np.ndarray:
    """n points in [0, domain]^d: isotropic Gaussians around k uniform centres plus noise.

    ``sigma`` is a scalar or one value per component.  Component membership is uniform
    among the k components.  The result is shuffled so input order carries no structure.
    """
    n_noise = int(round(n * noise_frac))
    n_clu = n - n_noise
    centres = rng.uniform(0.0, domain, size=(k, d))
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (k,))
    comp = rng.integers(0, k, size=n_clu)
    pts = centres[comp] + rng.standard_normal((n_clu, d)) * sig[comp, None]
    noise = rng.uniform(0.0, domain, size=(n_noise, d))
    X = np.concatenate([pts, noise], axis=0)
    X = X[rng.permutation(n)]
    return np.ascontiguousarray(X, dtype=np.float64)


def blobs_2d(n: int = 20_000, seed: int = SEED_BASE + 0) -> np.ndarray:
    """2D: 90 % from 10 Gaussian blobs (sigma 50, centres U[0,1e4]^2), 10 % uniform noise."""
    return gaussian_mixture(n, 2, 10, 50.0, 1e4, 0.10, _rng(seed))


def seed_spreader_3d(
    n: int = 1_000_000,
    domain: float = 1e5,
    step: float = 50.0,
    radius: float = 100.0,
    per_pos: int = 100,
    restart: float = 1e-3,
    noise_frac: float = 1e-4,
    seed: int = SEED_BASE + 1,
) -> np.ndarray:
    """3D seed-spreader random walk.

    The walker starts uniform in [0, domain]^3.  At each position it emits ``per_pos``
    points uniform in a ball of ``radius``; then, with probability ``restart`` it jumps
    to a fresh uniform location, otherwise it moves ``step`` in a uniformly random
    direction.  The walker is not clamped to the domain.  ``noise_frac`` of the points
    are uniform noise over the domain.
    """
    rng = _rng(seed)
    n_noise = int(round(n * noise_frac))
    n_walk = n - n_noise
    n_pos = max(1, -(-n_walk // per_pos))
    jumps = rng.random(n_pos) < restart
    jumps[0] = True
    jump_to = rng.uniform(0.0, domain, size=(n_pos, 3))
    moves = step * _unit_vectors(rng, n_pos, 3)
    moves[jumps] = 0.0
    seg = np.cumsum(jumps) - 1
    heads = np.flatnonzero(jumps)
    cum = np.cumsum(moves, axis=0)
    pos = jump_to[heads][seg] + cum - cum[heads][seg]
    r = radius * np.cbrt(rng.random(n_pos * per_pos))
    offs = _unit_vectors(rng, n_pos * per_pos, 3) * r[:, None]
    walk = (np.repeat(pos, per_pos, axis=0) + offs)[:n_walk]
    noise = rng.uniform(0.0, domain, size=(n_noise, 3))
    X = np.concatenate([walk, noise], axis=0)
    X = X[rng.permutation(n)]
    return np.ascontiguousarray(X, dtype=np.float64)


def gaussian_mixture_hd(d: int, n: int = 2_000_000, seed: int = SEED_BASE + 2) -> np.ndarray:
    """5D / 7D mixture: 20 components, sigma 1, centres U[0,100]^d, 5 % uniform noise."""
    return gaussian_mixture(n, d, 20, 1.0, 100.0, 0.05, _rng(seed, d))


@dataclass
class Instance:
    """One point cloud and the (eps, minPts) settings run on it."""

    X: np.ndarray
    eps: list = field(default_factory=list)
    min_pts: list = field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])


def multi_cloud_batch(
    n_clouds: int = 256,
    n_lo: float = 1e3,
    n_hi: float = 1e6,
    seed: int = SEED_BASE + 4,
    size_scale: float = 1.0,
) -> list[Instance]:
    """256 independent clouds, sizes log-uniform in [1e3, 1e6], d in {2, 3, 5}.

    Each cloud is a mixture of k in {5..50} Gaussians with centres U[0,100]^d,
    per-component sigma log-uniform in [0.5, 2], plus 5 % uniform noise.  Its eps is
    half the median component sigma and minPts is 10.  ``size_scale`` shrinks every
    cloud (for tests) while keeping the draw of every other parameter.
    """
    rng = _rng(seed)
    out = []
    for i in range(n_clouds):
        n_i = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d_i = int(rng.choice([2, 3, 5]))
        k_i = int(rng.integers(5, 51))
        sig = np.exp(rng.uniform(math.log(0.5), math.log(2.0), size=k_i))
        eps_i = 0.5 * float(np.median(sig))
        n_use = max(1, int(round(n_i * size_scale)))
        X = gaussian_mixture(n_use, d_i, k_i, sig, 100.0, 0.05, _rng(seed, i))
        out.append(Instance(X=X, eps=[eps_i], min_pts=[10]))
    return out


def config_workload(index: int, scale: float = 1.0) -> list[Instance]:
    """The five evaluation workloads as lists of instances.

    ``scale`` < 1 shrinks the point counts (and, for the seed spreader, the domain so
    that density is kept) for tests that must finish quickly.
    """
    if index == 0:
        return [Instance(blobs_2d(max(1, int(round(20_000 * scale)))), [100.0], [10])]
    if index == 1:
        n = max(1, int(round(1_000_000 * scale)))
        dom = 1e5 * scale ** (1.0 / 3.0)
        return [Instance(seed_spreader_3d(n, domain=dom), [200.0], [10])]
    if index == 2:
        out = []
        for d in (5, 7):
            X = gaussian_mixture_hd(d, max(1, int(round(2_000_000 * scale))))
            out.append(Instance(X, [1.5, 2.0, 3.0], [10, 10, 10]))
        return out
    if index == 3:
        n = max(1, int(round(10_000_000 * scale)))
        dom = 1e6 * scale ** (1.0 / 3.0)
        X = seed_spreader_3d(n, domain=dom, seed=SEED_BASE + 3)
        eps, mp = [], []
        for e in (200.0, 400.0, 800.0, 1600.0):
            for m in (5, 10, 50, 100):
                eps.append(e)
                mp.append(m)
        return [Instance(X, eps, mp)]
    if index == 4:
        return multi_cloud_batch(size_scale=scale)
    raise ValueError(f"no workload {index}")
