"""Synthetic objects, probes, start states and photon-count sampling.

Object (dispersive sample, one complex image per wavelength): amplitude
U(0.5, 1) and phase U(-pi, pi), each smoothed by a periodic Gaussian of
sigma 2 px and rescaled back to its range; the phase is scaled by
lambda_min / lambda_l per wavelength.

Probe: a hard-edged disc of radius 0.3125 N with a quadratic phase
alpha r^2, alpha = 0.02 * 64 / N rad/px^2 (scaled by lambda_min / lambda_l).
Mutually incoherent modes are the Gram-Schmidt orthonormalisation of the
disc field times low-order polynomials, scaled by sqrt(mode weight).  The
photon budget is the incident power: sum over wavelengths and modes of
||P_{l,m}||^2 equals the photons per pattern, split equally over wavelengths.

Measured patterns need the forward model, which lives outside this package;
``sample_counts`` only draws Poisson counts from an intensity it is given.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter

from .geometry import pads_for, positions_for, ratios_for


def _rescale(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    mn, mx = x.min(), x.max()
    return lo + (x - mn) * ((hi - lo) / (mx - mn))


def make_object(H: int, W: int, harmonics, ref_harmonic: int,
                rng: np.random.Generator, Ns: int = 1) -> np.ndarray:
    """complex128 [L][Ns][H][W]."""
    L = len(harmonics)
    out = np.empty((L, Ns, H, W), dtype=np.complex128)
    for n in range(Ns):
        amp = rng.uniform(0.5, 1.0, size=(H, W))
        ph = rng.uniform(-np.pi, np.pi, size=(H, W))
        amp = _rescale(gaussian_filter(amp, 2.0, mode="wrap"), 0.5, 1.0)
        ph = _rescale(gaussian_filter(ph, 2.0, mode="wrap"), -np.pi, np.pi)
        for l, q in enumerate(harmonics):
            # lambda_min / lambda_l = q_l / q_ref  (lambda = 800 nm / q)
            out[l, n] = amp * np.exp(1j * ph * (q / ref_harmonic))
    return out


def _mode_polys(x: np.ndarray, y: np.ndarray, M: int):
    polys = [np.ones_like(x), x, y, x * x + y * y, x * y, x * x - y * y,
             x * (x * x + y * y), y * (x * x + y * y)]
    if M > len(polys):
        raise ValueError("at most 8 probe modes are generated")
    return polys[:M]


def make_probes(N: int, harmonics, ref_harmonic: int, mode_weights,
                photons: float) -> np.ndarray:
    """complex128 [L][M][N][N], orthogonal modes per wavelength."""
    L, M = len(harmonics), len(mode_weights)
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64)
    yy -= N / 2.0
    xx -= N / 2.0
    r2 = xx * xx + yy * yy
    radius = 0.3125 * N
    disc = (r2 <= radius * radius).astype(np.float64)
    alpha = 0.02 * 64.0 / N
    polys = _mode_polys(xx / radius, yy / radius, M)
    out = np.empty((L, M, N, N), dtype=np.complex128)
    w = np.asarray(mode_weights, dtype=np.float64)
    w = w / w.sum()
    for l, q in enumerate(harmonics):
        base = disc * np.exp(1j * alpha * (q / ref_harmonic) * r2)
        basis = []
        for h in polys:
            v = base * h
            for b in basis:
                v = v - np.vdot(b, v) * b
            v = v / np.linalg.norm(v)
            basis.append(v)
        for m in range(M):
            out[l, m] = basis[m] * np.sqrt(w[m] * photons / L)
    return out


def make_truth(w, Ns: int | None = None) -> dict:
    """Ground-truth state and fixed inputs of a workload (all seeded).

    Returns a dict with complex128 ``object`` [L][Ns][H][W], complex128
    ``probe`` [L][M][N][N], float32 ``pos`` [K][2] (y, x top-left of the
    window in object pixels), ``pads`` (N_l per wavelength; the exact ratios
    when the workload asks for them), ``ratios`` (the exact sampling ratio
    per wavelength, floats), ``sigma`` /
    ``background`` / ``mask`` (None: all ones / zero / all valid).
    """
    rng = np.random.Generator(np.random.PCG64(w.seed))
    ns = w.Ns if Ns is None else Ns
    obj = make_object(w.H, w.W, w.harmonics, w.ref_harmonic, rng, ns)
    prb = make_probes(w.N, w.harmonics, w.ref_harmonic, w.mode_weights, w.photons)
    pos = positions_for(w, rng)
    truth = dict(object=obj, probe=prb, pos=pos,
                 pads=pads_for(w.N, w.harmonics, w.ref_harmonic),
                 ratios=ratios_for(w.N, w.harmonics, w.ref_harmonic),
                 sigma=None, background=None, mask=None, resample=None)
    if w.exact_ratio:
        truth["pads"] = truth["ratios"]
    if w.tilt:
        from .tilt import tilt_table
        idx, wt, mask = tilt_table(w.N)
        truth["resample"] = (idx, wt)
        truth["mask"] = mask
    return truth


def make_start(truth: dict, w, level: float = 1.0) -> dict:
    """A perturbed state at which loss and gradient are evaluated.

    Object: multiplied by a smooth random complex factor; probe: plus 10 %
    smooth complex noise inside its support; positions: plus N(0, 0.5^2) px,
    kept at least 1 px inside the object.  ``level`` scales all perturbations.
    """
    rng = np.random.Generator(np.random.PCG64(w.seed + 1000))
    obj = truth["object"]
    L, Ns, H, W = obj.shape
    fa = gaussian_filter(rng.normal(size=(H, W)), 4.0, mode="wrap")
    fp = gaussian_filter(rng.normal(size=(H, W)), 4.0, mode="wrap")
    fa *= 0.15 * level / max(np.abs(fa).max(), 1e-30)
    fp *= 0.5 * level / max(np.abs(fp).max(), 1e-30)
    obj_s = obj * ((1.0 + fa) * np.exp(1j * fp))[None, None]
    prb = truth["probe"]
    noise = (rng.normal(size=prb.shape) + 1j * rng.normal(size=prb.shape))
    support = (np.abs(prb) > 0).astype(np.float64)
    scale = np.sqrt(np.mean(np.abs(prb) ** 2, axis=(-2, -1), keepdims=True) /
                    np.maximum(np.mean(support, axis=(-2, -1), keepdims=True), 1e-30))
    prb_s = prb + 0.1 * level * noise * support * scale
    pos = truth["pos"].astype(np.float64)
    pos_s = pos + rng.normal(0.0, 0.5 * level, size=pos.shape)
    N = prb.shape[-1]
    pos_s[:, 0] = np.clip(pos_s[:, 0], 1.0, H - N - 1.0)
    pos_s[:, 1] = np.clip(pos_s[:, 1], 1.0, W - N - 1.0)
    start = dict(truth)
    start.update(object=obj_s, probe=prb_s, pos=pos_s.astype(np.float32))
    return start


def sample_counts(intensity: np.ndarray, seed: int) -> np.ndarray:
    """Poisson photon counts drawn from a non-negative intensity, as float32."""
    rng = np.random.Generator(np.random.PCG64(seed + 2000))
    lam = np.maximum(np.asarray(intensity, dtype=np.float64), 0.0)
    return rng.poisson(lam).astype(np.float32)


def synthetic_counts(K: int, N: int, photons: float, seed: int, n_base: int = 16) -> np.ndarray:
    """Poisson photon counts with a workload's photon budget but no model
    behind them, float32 [K][N][N].

    ``n_base`` patterns (a bright centre on a smooth positive field, scaled
    to ``photons`` in total) are drawn once; position k gets pattern
    k mod n_base, shifted along x by k // n_base pixels.  Meant for tests at
    full size, where computing every position's pattern from a model would
    take too long; any fixed data serve for comparing two implementations of
    the same loss.
    """
    rng = np.random.Generator(np.random.PCG64(seed + 3000))
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64)
    r2 = (yy - N / 2.0) ** 2 + (xx - N / 2.0) ** 2
    centre = 50.0 * np.exp(-r2 / (0.05 * N) ** 2)
    base = []
    for _ in range(n_base):
        f = gaussian_filter(rng.normal(size=(N, N)), 3.0, mode="wrap")
        lam = np.exp(f / max(f.std(), 1e-30)) + centre
        lam *= photons / lam.sum()
        base.append(rng.poisson(lam).astype(np.float32))
    out = np.empty((K, N, N), dtype=np.float32)
    for k in range(K):
        out[k] = np.roll(base[k % n_base], (k // n_base) % N, axis=1)
    return out
