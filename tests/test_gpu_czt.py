"""GPU parity of the exact-ratio propagator (chirp z-transform, evaluated by
Bluestein's method with FFTs of length 2N) against the FP64 oracle, which
evaluates the scaled DFT as written.

Tolerances as for the zero-padded DFT (relative L2 per array): intensities
1e-5, loss 1e-5, gradients 1e-4.  Ratios are the exact wavelength ratios of
the workloads (N lambda_l / lambda_min), which are not integers.
"""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _ratios(w):
    return synth.ratios_for(w.N, w.harmonics, w.ref_harmonic)


def _check(case, kinds=(0,), scale=1.0, workers=1, fwd=True):
    print(f"{case['w'].name}: N={case['w'].N} K={case['w'].K} L={case['w'].L} M={case['w'].M} "
          f"ratios={case['pads']}", flush=True)
    prob = U.to_problem(case, DEV)
    if fwd:
        got = U.gpu_forward(prob)
        ref = U.oracle_forward(case["obj"].astype(np.complex128), case["prb"].astype(np.complex128),
                               case["pos"], case["pads"], sigma=case["sigma"], bg=case["bg"],
                               table=case["table"], workers=workers)
        U.check_array("forward " + case["w"].name, got, ref, 1e-5)
    for kind in kinds:
        got = U.gpu_grads(prob, kind=kind, scale=scale)
        ref = U.oracle_grads(case, kind=kind, scale=scale, workers=workers)
        print("  kind", kind, U.compare(got, ref), flush=True)


def test_exact_ratios_three_wavelengths_sigma_background_mask():
    w = synth.reduced(synth.get_workload("C1"), L=3, M=2, harmonics=(19, 21, 23),
                      mode_weights=(0.75, 0.25), K=12, name="C1-ratio")
    case = U.make_case(w, with_sigma=True, with_bg=True, with_mask=True, pads=_ratios(w))
    assert all(isinstance(a, float) for a in case["pads"])
    _check(case, kinds=(0, 1, 2), scale=0.25)


def test_exact_ratios_c2_shapes():
    w = synth.get_workload("C2")
    case = U.make_case(w, K=5, pads=_ratios(w), workers=U.default_workers())
    _check(case, workers=U.default_workers())


def test_exact_ratios_tilted_plane_resampling():
    # N = 384 (Bluestein length 768) with the resampling table: the forward
    # detector pass keeps Psi for the separate adjoint pass
    w = synth.get_workload("C5")
    case = U.make_case(w, K=3, pads=_ratios(w), workers=U.default_workers())
    assert case["table"] is not None
    _check(case, workers=U.default_workers())


def test_exact_ratios_n512():
    # N = 512 (Bluestein length 1024), two modes to keep the oracle short
    w = synth.reduced(synth.get_workload("C3"), K=2, M=2, mode_weights=(0.7, 0.3), name="C3-ratio")
    case = U.make_case(w, pads=_ratios(w), workers=U.default_workers())
    _check(case, fwd=False, workers=U.default_workers())


def test_integer_ratio_agrees_with_the_zero_padded_dft():
    # alpha = 80.0 through Bluestein vs pad 80 through the padded DFT
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=6, name="C1-int")
    case = U.make_case(w, pads=(80, 64))
    a = U.gpu_grads(U.to_problem(case, DEV))
    b = U.gpu_grads(U.to_problem(dict(case, pads=(80.0, 64.0)), DEV))
    for k in ("g_object", "g_probe", "g_pos"):
        e = U.rel_l2(b[k], a[k])
        print(k, e)
        assert e <= 1e-5, k
    assert abs(a["loss"] - b["loss"]) <= 1e-6 * abs(a["loss"])


def test_exact_ratio_chunking_and_mixed_calls_are_bitwise_invariant():
    from paper_2311_14780_amd import binding as B
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=9, name="C1-mix")
    case_r = U.make_case(w, pads=_ratios(w))
    case_p = U.make_case(w, pads=(80, 64), seed_offset=1)
    pr, pp = U.to_problem(case_r, DEV), U.to_problem(case_p, DEV)
    whole = U.gpu_grads(pr)
    part = U.gpu_grads(pr, chunk=4)
    for k in ("loss", "g_object", "g_probe", "g_pos", "g_sigma", "g_background"):
        assert np.array_equal(np.asarray(whole[k]), np.asarray(part[k])), k
    # both jobs in one call: each equals its single-job result bitwise
    alone_p = U.gpu_grads(pp)
    gs = []
    for p in (pr, pp):
        gs.append(dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(p.object),
                       g_probe=torch.zeros_like(p.probe), g_pos=torch.zeros(p.K, 2, device=DEV),
                       g_sigma=torch.zeros(p.K, device=DEV),
                       g_background=torch.zeros(p.N, p.N, device=DEV)))
    ws = B.workspace([pr, pp], 1)
    B.ptycho_loss_grad([pr, pp], gs, workspace=ws)
    torch.cuda.synchronize()
    for g, ref in ((gs[0], whole), (gs[1], alone_p)):
        for k in ("g_object", "g_probe", "g_pos", "g_background"):
            assert np.array_equal(g[k].cpu().numpy(), ref[k]), k
        assert float(g["loss"].cpu()[0]) == ref["loss"]


ALL = ("object", "probe", "pos", "sigma", "background", "ratio")


def _check_ratio_grad(case, kinds=(0,), workers=1):
    prob = U.to_problem(case, DEV)
    for kind in kinds:
        got = U.gpu_grads(prob, kind=kind, want=ALL)
        ref = U.oracle_grads(case, kind=kind, workers=workers)
        print(f"  {case['w'].name} kind {kind} g_ratio gpu {got['g_ratio']} oracle {ref['g_ratio']}")
        print("  ", U.compare(got, ref), flush=True)
        # asking for dL/d alpha recomputes Psi in the adjoint: the other
        # gradients stay those of the plain call
        plain = U.gpu_grads(prob, kind=kind)
        for k in ("g_object", "g_probe", "g_pos", "g_sigma", "g_background"):
            e = U.rel_l2(got[k], plain[k])
            assert e <= 1e-6, (k, e)
        assert abs(got["loss"] - plain["loss"]) <= 1e-7 * abs(plain["loss"])


def test_ratio_gradient_three_wavelengths():
    # exact ratios 77.47 and 70.10 plus the reference wavelength at exactly N
    w = synth.reduced(synth.get_workload("C1"), L=3, M=2, harmonics=(19, 21, 23),
                      mode_weights=(0.75, 0.25), K=12, name="C1-dz")
    case = U.make_case(w, with_sigma=True, with_bg=True, with_mask=True, pads=_ratios(w))
    _check_ratio_grad(case, kinds=(0, 1))


def test_ratio_gradient_mixed_pad_and_ratio_wavelengths():
    # one zero-padded wavelength (no alpha, g_ratio 0) and one exact-ratio one
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=8, name="C1-dzmix")
    case = U.make_case(w, pads=(80, 64.0), with_sigma=True)
    got = U.gpu_grads(U.to_problem(case, DEV), want=ALL)
    assert got["g_ratio"][0] == 0.0
    _check_ratio_grad(case)


def test_ratio_gradient_c2_shapes():
    w = synth.get_workload("C2")
    case = U.make_case(w, K=4, pads=_ratios(w), workers=U.default_workers())
    _check_ratio_grad(case, workers=U.default_workers())


def test_ratio_gradient_tilted_plane_resampling():
    w = synth.get_workload("C5")
    case = U.make_case(w, K=3, pads=_ratios(w), workers=U.default_workers())
    _check_ratio_grad(case, workers=U.default_workers())


def test_ratio_gradient_n512():
    w = synth.reduced(synth.get_workload("C3"), K=2, M=2, mode_weights=(0.7, 0.3), name="C3-dz")
    case = U.make_case(w, pads=_ratios(w), workers=U.default_workers())
    _check_ratio_grad(case, workers=U.default_workers())


def test_ratio_gradient_is_chunk_invariant():
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=9, name="C1-dzc")
    prob = U.to_problem(U.make_case(w, pads=_ratios(w)), DEV)
    a = U.gpu_grads(prob, want=ALL)
    b = U.gpu_grads(prob, want=ALL, chunk=4)
    for k in ("g_ratio", "g_object", "g_probe", "g_pos", "g_background"):
        assert np.array_equal(a[k], b[k]), k
