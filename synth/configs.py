"""Workload definitions (sizes, harmonics, mode powers, scan pattern, seed).

The paper reconstructs an experimental dataset (255 frames of a 2048x2048 EUV
camera, two harmonics, six illumination modes and one sample mode per
wavelength; Section "Experimental setup and ptychography reconstruction").
That dataset is not available, so five seeded synthetic workloads stand in
for it.  Wavelengths are harmonics q of an 800 nm fundamental,
lambda_q = 800/q nm; the shortest wavelength of a workload is the reference
at which the detector pad equals the probe size.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field


@dataclass(frozen=True)
class Workload:
    name: str
    K: int                      # scan positions
    L: int                      # wavelengths
    M: int                      # illumination (probe) modes per wavelength
    N: int                      # probe window / detector size (N x N)
    H: int                      # object height (px)
    W: int                      # object width (px)
    harmonics: tuple            # harmonic order q per wavelength, l = 0..L-1
    ref_harmonic: int           # q of the reference (shortest) wavelength
    mode_weights: tuple         # relative power of each probe mode (sums to 1)
    photons: float              # incident photons per diffraction pattern
    scan: str                   # "raster_uniform" | "spiral" | "raster_gauss"
    seed: int
    Ns: int = 1                 # sample modes
    tilt: bool = False          # tilted-plane resampling table (reflection)
    scan_step: float = 0.0      # raster step (px)
    scan_jitter: float = 0.0    # uniform half-width or Gaussian sigma (px)
    scan_origin: float = 0.0    # raster origin (px)
    raster_side: int = 0        # raster is raster_side x raster_side
    exact_ratio: bool = False   # propagate at the exact wavelength ratios (not smooth pads)
    note: str = ""

    @property
    def pattern_modes(self) -> int:
        """One (position, wavelength, probe mode, sample mode) propagation."""
        return self.K * self.L * self.M * self.Ns


def _geometric_weights(m: int) -> tuple:
    w = [2.0 ** (-i) for i in range(m)]
    s = sum(w)
    return tuple(x / s for x in w)


# C1: plain method, one wavelength, one mode, 10x10 raster with uniform jitter.
C1 = Workload(
    name="C1", K=100, L=1, M=1, N=64, H=256, W=256,
    harmonics=(23,), ref_harmonic=23, mode_weights=(1.0,), photons=1e4,
    scan="raster_uniform", seed=1, scan_step=16.0, scan_jitter=2.0,
    scan_origin=24.0, raster_side=10,
    note="single wavelength, single mode, 64^2 probe, 256^2 object",
)

# C2: four harmonics 17/19/21/23 x three modes 0.7/0.2/0.1, Fermat spiral.
C2 = Workload(
    name="C2", K=400, L=4, M=3, N=256, H=1024, W=1024,
    harmonics=(17, 19, 21, 23), ref_harmonic=23, mode_weights=(0.7, 0.2, 0.1),
    photons=1e5, scan="spiral", seed=2,
    note="4 harmonics x 3 modes, 256^2 probe, 1024^2 object, 400 spiral positions",
)

# C3: large multiplexed reconstruction (exit waves recomputed per chunk).
C3 = Workload(
    name="C3", K=2500, L=5, M=8, N=512, H=3072, W=3072,
    harmonics=(17, 19, 21, 23, 25), ref_harmonic=25,
    mode_weights=_geometric_weights(8), photons=1e5, scan="spiral", seed=3,
    note="5 harmonics x 8 modes, 512^2 probe, 3072^2 object, 2500 positions",
)

# C5: reflection geometry with a tilted-plane bilinear resampling table.
C5 = Workload(
    name="C5", K=900, L=3, M=4, N=384, H=1152, W=1152,
    harmonics=(17, 19, 21), ref_harmonic=21, mode_weights=_geometric_weights(4),
    photons=1e5, scan="raster_gauss", seed=5, tilt=True, scan_step=24.0,
    scan_jitter=1.5, scan_origin=36.0, raster_side=30,
    note="3 harmonics x 4 modes, 384^2 probe, 70 deg incidence tilt table",
)

WORKLOADS = {w.name: w for w in (C1, C2, C3, C5)}


def get_workload(name: str) -> Workload:
    return WORKLOADS[name]


def reduced(w: Workload, **changes) -> Workload:
    """A copy with some sizes changed (e.g. fewer positions for parity)."""
    name = changes.pop("name", w.name + "r")
    return dataclasses.replace(w, name=name, **changes)


# C4 (serving stream) job recipe: per-job draws are made in synth.serving.
SERVING_HARMONICS = (25, 23, 21, 19, 17)
SERVING_SIZES = (128, 256, 512)
