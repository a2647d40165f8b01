"""Scan geometry and per-wavelength detector pads.

Detector sampling: the far-field pixel pitch expressed in object-plane units
scales with the wavelength (Eq. 1's propagator depends on lambda_l).  With a
fixed detector of N x N pixels and a probe window of N x N object pixels, the
wavelength lambda_l is sampled by zero-padding the exit wave to an
N_l x N_l grid before a unitary DFT, N_l ~ N * lambda_l / lambda_min.  The
exact ratio is rarely an integer with small prime factors, so N_l is the
2,3,5,7-smooth integer nearest to it (ties to the larger), and exactly N at the
reference wavelength.  ``ratios_for`` gives the exact ratios themselves, for
the exact-ratio (chirp z-transform) propagator.
"""
from __future__ import annotations

import math

import numpy as np


def is_smooth7(n: int) -> bool:
    if n < 1:
        return False
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


def smooth_pad(N: int, ratio: float) -> int:
    """Nearest 7-smooth integer to N*ratio (ties -> larger), never below N."""
    if ratio <= 1.0:
        return N
    target = N * ratio
    best = None
    for cand in range(N, int(2 * target) + 8):
        if is_smooth7(cand):
            d = abs(cand - target)
            if best is None or d < best[0] or (d == best[0] and cand > best[1]):
                best = (d, cand)
    return best[1]


def pads_for(N: int, harmonics, ref_harmonic: int) -> tuple:
    """N_l per wavelength; lambda_l / lambda_ref = ref_harmonic / q_l."""
    return tuple(smooth_pad(N, ref_harmonic / q) if q != ref_harmonic else N
                 for q in harmonics)


def ratios_for(N: int, harmonics, ref_harmonic: int) -> tuple:
    """Exact sampling ratio per wavelength, N * lambda_l / lambda_ref =
    N * ref_harmonic / q_l, as Python floats (exactly N at the reference)."""
    return tuple(float(N) * ref_harmonic / q for q in harmonics)


def raster_uniform(side: int, step: float, origin: float, jitter: float,
                   rng: np.random.Generator) -> np.ndarray:
    """side x side raster (row-major), uniform jitter in [-jitter, jitter]."""
    i, j = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    base = np.stack([origin + step * i.ravel(), origin + step * j.ravel()], 1)
    return base + rng.uniform(-jitter, jitter, size=base.shape)


def raster_gauss(side: int, step: float, origin: float, sigma: float,
                 margin: float, H: int, W: int, N: int,
                 rng: np.random.Generator) -> np.ndarray:
    """Regular raster perturbed by N(0, sigma^2), clipped to a margin."""
    i, j = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    base = np.stack([origin + step * i.ravel(), origin + step * j.ravel()], 1)
    pos = base + rng.normal(0.0, sigma, size=base.shape)
    pos[:, 0] = np.clip(pos[:, 0], margin, H - N - margin)
    pos[:, 1] = np.clip(pos[:, 1], margin, W - N - margin)
    return pos


def fermat_spiral(K: int, H: int, W: int, N: int, c: float | None = None) -> np.ndarray:
    """Fermat spiral s_n = c0 + c sqrt(n) (sin n*g, cos n*g), g = golden angle.

    With the default c the outermost window touches a 1 px border, so every
    window lies inside the object.
    """
    g = math.pi * (3.0 - math.sqrt(5.0))
    cy, cx = (H - N) / 2.0, (W - N) / 2.0
    if c is None:
        c = (min(cy, cx) - 1.0) / math.sqrt(max(K - 1, 1))
    n = np.arange(K, dtype=np.float64)
    r = c * np.sqrt(n)
    return np.stack([cy + r * np.sin(n * g), cx + r * np.cos(n * g)], 1)


def positions_for(w, rng: np.random.Generator) -> np.ndarray:
    if w.scan == "raster_uniform":
        pos = raster_uniform(w.raster_side, w.scan_step, w.scan_origin,
                             w.scan_jitter, rng)
    elif w.scan == "raster_gauss":
        pos = raster_gauss(w.raster_side, w.scan_step, w.scan_origin,
                           w.scan_jitter, 8.0, w.H, w.W, w.N, rng)
    elif w.scan == "spiral":
        pos = fermat_spiral(w.K, w.H, w.W, w.N)
    else:
        raise ValueError(f"unknown scan {w.scan!r}")
    return pos[: w.K].astype(np.float32)
