"""Input generators: pads, scan geometry, probes, tilt table (CPU only)."""
import math
import os

import numpy as np
import pytest

import synth
from synth import configs, fields, geometry, tilt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_pads_match_golden_table():
    for N, ref, qs, pads, targets in _read_golden("pads.txt"):
        N, ref = int(N), int(ref)
        qs = tuple(int(q) for q in qs.split(","))
        pads = tuple(int(p) for p in pads.split(","))
        targets = [float(t) for t in targets.split(",")]
        assert geometry.pads_for(N, qs, ref) == pads
        for q, t in zip(qs, targets):
            assert N * ref / q == pytest.approx(t, abs=0.01)
        for p in pads:
            assert geometry.is_smooth7(p) and p >= N


def test_pads_are_nearest_smooth():
    for N in (64, 128, 256, 384, 512):
        for ratio in np.linspace(1.0, 1.5, 23):
            p = geometry.smooth_pad(N, ratio)
            t = N * ratio
            for c in range(N, int(2 * t) + 2):
                if geometry.is_smooth7(c):
                    assert abs(p - t) <= abs(c - t) + 1e-9


@pytest.mark.parametrize("name", ["C1", "C2", "C3", "C5"])
def test_windows_inside_object(name):
    w = configs.get_workload(name)
    rng = np.random.Generator(np.random.PCG64(w.seed))
    pos = geometry.positions_for(w, rng)
    assert pos.shape == (w.K, 2) and pos.dtype == np.float32
    p = np.floor(pos + np.float32(0.5))
    assert p.min() >= 0
    assert p[:, 0].max() + w.N <= w.H and p[:, 1].max() + w.N <= w.W


def test_spiral_radius_bound():
    w = configs.get_workload("C2")
    pos = geometry.fermat_spiral(w.K, w.H, w.W, w.N)
    c = (w.H - w.N) / 2
    r = np.hypot(pos[:, 0] - c, pos[:, 1] - c)
    assert r.max() <= c - 1 + 1e-9


def test_probe_modes_orthogonal_and_normalised():
    w = configs.get_workload("C2")
    P = fields.make_probes(w.N, w.harmonics, w.ref_harmonic, w.mode_weights, w.photons)
    for l in range(w.L):
        G = np.array([[np.vdot(P[l, a], P[l, b]) for b in range(w.M)] for a in range(w.M)])
        off = G - np.diag(np.diag(G))
        assert np.max(np.abs(off)) < 1e-9 * w.photons
        assert np.allclose(np.diag(G).real, np.array(w.mode_weights) * w.photons / w.L)
    assert np.sum(np.abs(P) ** 2) == pytest.approx(w.photons)


def test_c1_probe_matches_recipe():
    # 64 x 64 probe: circular aperture of radius 20 px, quadratic phase 0.02 rad/px^2
    w = configs.get_workload("C1")
    P = fields.make_probes(w.N, w.harmonics, w.ref_harmonic, w.mode_weights, w.photons)[0, 0]
    yy, xx = np.mgrid[0:64, 0:64] - 32.0
    r2 = yy ** 2 + xx ** 2
    assert np.all(np.abs(P[r2 > 400]) == 0) and np.all(np.abs(P[r2 <= 400]) > 0)
    ph = np.angle(P[32, 32 + 10] / P[32, 32])
    assert ph == pytest.approx(0.02 * 100, abs=1e-9)


def test_object_ranges():
    rng = np.random.Generator(np.random.PCG64(0))
    O = fields.make_object(64, 64, (17, 23), 23, rng)
    a = np.abs(O[1, 0])
    assert a.min() == pytest.approx(0.5) and a.max() == pytest.approx(1.0)
    ph = np.angle(O[1, 0])
    assert ph.min() >= -np.pi - 1e-12 and ph.max() <= np.pi + 1e-12
    # dispersive: the longer wavelength carries a proportionally smaller phase
    assert np.allclose(np.angle(O[0, 0]), np.angle(O[1, 0]) * 17 / 23, atol=1e-12)
    assert np.allclose(np.abs(O[0, 0]), a)


def test_tilt_geometry_matches_printed_aperture():
    g = {r[0]: float(r[1]) for r in _read_golden("camera_geometry.txt")}
    n = int(g["camera_pixels"])
    ut, ux = tilt.tilt_coordinates(n, z_mm=g["distance_mm"], pixel_um=g["pixel_um"],
                                   grazing_deg=90 - g["incidence_deg_from_normal"])
    z = g["distance_mm"] * 1e3 / g["pixel_um"]
    # direction cosine at the camera edge along the untilted axis = NA
    na = ux[n // 2, 0] / z
    assert abs(na) == pytest.approx(g["na_untilted"], abs=0.003)
    # Abbe resolution lambda / (2 NA) is the printed ~50 nm
    assert g["wavelength_nm"] / (2 * abs(na)) == pytest.approx(g["resolution_untilted_nm"], rel=0.1)


def test_tilt_table_is_identity_near_centre_and_rows_sum_to_one():
    N = 384
    idx, w, mask = tilt.tilt_table(N)
    ws = w.sum(1)
    assert np.allclose(ws[mask.ravel() > 0], 1.0, atol=1e-6)
    assert np.all(ws[mask.ravel() == 0] == 0)
    c = (N // 2) * N + N // 2
    assert idx[c, 0] == c and w[c, 0] == pytest.approx(1.0, abs=1e-6)
    assert 0.9 < mask.mean() < 1.0


def test_sample_counts_deterministic():
    I = np.full((4, 4), 7.5)
    a = fields.sample_counts(I, 3)
    b = fields.sample_counts(I, 3)
    assert a.dtype == np.float32 and np.array_equal(a, b)
    assert np.all(a == np.round(a))


def test_exact_ratios_are_wavelength_ratios():
    # alpha_l = N lambda_l / lambda_ref with lambda proportional to 1/q
    for name in ("C2", "C3", "C5"):
        w = synth.get_workload(name)
        r = synth.ratios_for(w.N, w.harmonics, w.ref_harmonic)
        pads = synth.pads_for(w.N, w.harmonics, w.ref_harmonic)
        for q, a, p in zip(w.harmonics, r, pads):
            assert isinstance(a, float)
            assert abs(a * q - w.N * w.ref_harmonic) <= 1e-9 * a * q
            if q == w.ref_harmonic:
                assert a == float(w.N)
            # the smooth pad is within the documented 1.65 % of the ratio
            assert abs(p - a) <= 0.0165 * a
