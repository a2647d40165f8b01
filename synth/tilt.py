"""Tilted-plane resampling table for the reflection workload.

In reflection geometry the diffraction pattern recorded on a camera that
faces the specular beam is a distorted view of the sample-plane spatial
frequencies.  The paper corrects it by interpolating each pattern onto a
uniform sample-frequency grid and produces a binary mask of valid pixels
(Section "Experimental setup and ptychography reconstruction": camera
2048x2048 px of 15 um, 88 mm from the sample, incidence 70 degrees from the
normal, i.e. 20 degrees grazing).

Here the mapping is applied inside the model instead: the predicted intensity
on the uniform grid is bilinearly resampled onto the camera grid,
I'(a) = sum_t w[a, t] I(idx[a, t]).  For camera pixel a with pixel offsets
(Y, X) from the centre and the distance z in pixels,
R = sqrt(X^2 + Y^2 + z^2),
u_x = z X / R,
u_t = (z / sin a) (cos a - (z cos a - Y sin a) / R),
which is the identity near the centre plus the non-paraxial curvature of the
tilted plane; the sin(a) compression along the tilt is absorbed into an
anisotropic sample pixel.  Camera pixels whose four taps are not all inside
the N x N grid are masked (weights 0, mask 0).
"""
from __future__ import annotations

import math

import numpy as np


def tilt_coordinates(N: int, z_mm: float = 88.0, pixel_um: float = 15.0,
                     grazing_deg: float = 20.0):
    """Sample-grid coordinates (u_t, u_x) of every camera pixel, float64."""
    z = z_mm * 1e3 / pixel_um
    a = math.radians(grazing_deg)
    Y, X = np.mgrid[0:N, 0:N].astype(np.float64)
    Y -= N / 2.0
    X -= N / 2.0
    R = np.sqrt(X * X + Y * Y + z * z)
    ux = z * X / R
    ut = (z / math.sin(a)) * (math.cos(a) - (z * math.cos(a) - Y * math.sin(a)) / R)
    return ut, ux


def tilt_table(N: int, **kw):
    """Bilinear table: idx int32 [N*N][4], w float32 [N*N][4], mask uint8 [N][N].

    Tap order (t): (y0,x0), (y0,x0+1), (y0+1,x0), (y0+1,x0+1); idx is the flat
    index y*N + x into the uniform N x N grid (DC at (N/2, N/2)).
    """
    ut, ux = tilt_coordinates(N, **kw)
    fy = ut + N / 2.0
    fx = ux + N / 2.0
    y0 = np.floor(fy).astype(np.int64)
    x0 = np.floor(fx).astype(np.int64)
    ty = fy - y0
    tx = fx - x0
    valid = (y0 >= 0) & (x0 >= 0) & (y0 + 1 <= N - 1) & (x0 + 1 <= N - 1)
    idx = np.stack([y0 * N + x0, y0 * N + x0 + 1, (y0 + 1) * N + x0,
                    (y0 + 1) * N + x0 + 1], -1)
    w = np.stack([(1 - ty) * (1 - tx), (1 - ty) * tx, ty * (1 - tx), ty * tx], -1)
    idx = np.where(valid[..., None], idx, 0).reshape(N * N, 4).astype(np.int32)
    w = np.where(valid[..., None], w, 0.0).reshape(N * N, 4).astype(np.float32)
    return idx, w, valid.astype(np.uint8)
