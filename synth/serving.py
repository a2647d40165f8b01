"""Seeded job mix and arrival times of the serving stream.

Each job draws its probe size N from {128, 256, 512}, its wavelength count L
from 1..5 (the first L of harmonics 25, 23, 21, 19, 17 of an 800 nm
fundamental; harmonic 25 is the shortest wavelength and the pad reference),
its probe-mode count M from 1..8 (powers proportional to 2^-m) and its scan
length K from 100..1600, all uniform.  The scan is a Fermat spiral whose
step is about 0.075 N; the object is the smallest multiple of 64 pixels per
side that holds it.  Arrivals are a Poisson process.

Like the rest of this package, this only draws inputs: the job data are made
by ``synth.make_truth`` / ``synth.make_start`` from the per-job workload.
"""
from __future__ import annotations

import math

import numpy as np

from .configs import SERVING_HARMONICS, SERVING_SIZES, Workload, _geometric_weights


def serving_workload(job: int, N: int, L: int, M: int, K: int, seed: int,
                     exact_ratio: bool = False) -> Workload:
    """The workload of one serving job (object side from the spiral extent;
    ``exact_ratio``: propagate at the exact wavelength ratios)."""
    c = 0.075 * N
    side = 2.0 * c * math.sqrt(max(K - 1, 1)) + N + 2.0
    H = W = int(math.ceil(side / 64.0) * 64)
    harm = SERVING_HARMONICS[:L]
    return Workload(
        name=f"job{job}", K=K, L=L, M=M, N=N, H=H, W=W,
        harmonics=harm, ref_harmonic=harm[0], mode_weights=_geometric_weights(M),
        photons=1e5, scan="spiral", seed=seed, exact_ratio=exact_ratio,
        note="serving job",
    )


def serving_jobs(n_jobs: int = 64, seed: int = 4, sizes=SERVING_SIZES, L_max: int = 5,
                 M_max: int = 8, K_range=(100, 1600), exact_fraction: float = 0.0) -> list:
    """The job mix: a list of Workloads, job j seeded with seed * 1000 + j.
    A fraction ``exact_fraction`` of the jobs (drawn from a stream of its own,
    so the sizes do not change with it) uses the exact-ratio propagator."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rng_x = np.random.Generator(np.random.PCG64(seed + 555))
    jobs = []
    for j in range(n_jobs):
        N = int(rng.choice(np.asarray(sizes)))
        L = int(rng.integers(1, L_max + 1))
        M = int(rng.integers(1, M_max + 1))
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        exact = bool(rng_x.uniform() < exact_fraction)
        jobs.append(serving_workload(j, N, L, M, K, seed * 1000 + j, exact))
    return jobs


def poisson_arrivals(n: int, mean_gap: float, seed: int = 4) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given mean gap; the
    first job arrives at 0."""
    rng = np.random.Generator(np.random.PCG64(seed + 77))
    gaps = rng.exponential(mean_gap, size=n)
    gaps[0] = 0.0
    return np.cumsum(gaps)
