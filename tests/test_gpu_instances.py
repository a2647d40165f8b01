"""GPU parity of every compiled DFT instance that the serving stream uses and
the other tests do not reach: window N = 128 with the zero-padded sizes 128,
140, 150, 168 and 189 (harmonics 25/23/21/19/17 of the serving mix) and its
exact-ratio instance (Bluestein length 256), and N = 256 with the sizes 336
and 375.  Each is the propagator D_{lambda,z} of Eq. 1 at one wavelength's
detector sampling.  Few positions at the real window, all wavelengths of
the serving recipe in one job, several position chunks with a ragged tail.

Bounds (against the FP64 oracle): intensities relative L2 and
max-abs/max-ref 1e-5; loss 1e-5; every gradient relative L2 and
max-abs/max-ref 1e-4; position and power gradients per position 1e-3 with a
floor of 0.1 rms.
"""
import numpy as np
import pytest

import synth
from synth.serving import serving_workload
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _serving_case(N, L, M, K, seed, exact=False, **kw):
    w = serving_workload(900 + N, N, L, M, K, seed)
    pads = synth.ratios_for(w.N, w.harmonics, w.ref_harmonic) if exact else None
    return U.make_case(w, pads=pads, **kw)


def _run(case, kinds=(0, 1), chunk=0, want=("object", "probe", "pos", "sigma", "background")):
    w = case["w"]
    print(f"{w.name}: N={w.N} K={w.K} L={w.L} M={w.M} object {w.H}x{w.W} pads {case['pads']} "
          f"chunk {chunk}", flush=True)
    prob = U.to_problem(case, DEV)
    fwd = U.gpu_forward(prob, chunk=chunk)
    ref = U.oracle_forward(case["obj"].astype(np.complex128), case["prb"].astype(np.complex128),
                           case["pos"], case["pads"], sigma=case["sigma"], bg=case["bg"],
                           table=case["table"])
    U.check_array(w.name + " forward", fwd, ref, 1e-5)
    for kind in kinds:
        got = U.gpu_grads(prob, kind=kind, chunk=chunk, want=want)
        U.compare(got, U.oracle_grads(case, kind=kind))


def test_n128_every_pad_of_the_serving_mix():
    case = _serving_case(128, 5, 2, 6, 41, with_sigma=True, with_bg=True, with_mask=True)
    assert case["pads"] == (128, 140, 150, 168, 189)
    _run(case, chunk=4)


def test_n128_exact_ratio_bluestein_256():
    case = _serving_case(128, 3, 2, 5, 42, exact=True, with_sigma=True, with_bg=True)
    assert all(isinstance(a, float) for a in case["pads"]) and case["pads"][0] == 128.0
    _run(case, kinds=(0, 1), chunk=3,
         want=("object", "probe", "pos", "sigma", "background", "ratio"))


def test_n256_pads_336_and_375():
    case = _serving_case(256, 5, 2, 5, 43, with_sigma=True, with_mask=True)
    assert case["pads"] == (256, 280, 300, 336, 375)
    _run(case, kinds=(0,), chunk=4)


def test_n512_serving_pads_mixed_with_a_single_mode():
    # the 512 serving job with one mode per wavelength (the column adjoint's
    # 512-window instances run with a one-mode accumulator)
    case = _serving_case(512, 5, 1, 3, 44)
    assert case["pads"] == (512, 560, 600, 675, 750)
    _run(case, kinds=(1,), chunk=2)
