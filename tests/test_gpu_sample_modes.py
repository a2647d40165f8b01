"""GPU parity with several sample modes O_{l,n} (Eq. 1's sum over n): every
(wavelength, sample mode) pair is propagated with every probe mode and
summed incoherently; the probe gradient sums over n.  Against the FP64
oracle at the usual tolerances (intensities 1e-5, loss 1e-5, gradients 1e-4).
"""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
ALL = ("object", "probe", "pos", "sigma", "background", "ratio")


def _case(L=2, M=2, Ns=2, K=10, pads=(80, 64), harm=(19, 23), **kw):
    w = synth.reduced(synth.get_workload("C1"), L=L, M=M, Ns=Ns, harmonics=harm,
                      mode_weights=tuple(0.5 ** np.arange(M) / np.sum(0.5 ** np.arange(M))),
                      K=K, name=f"C1-ns{Ns}")
    return U.make_case(w, pads=pads, **kw)


def test_two_sample_modes_forward_and_gradients():
    case = _case(with_sigma=True, with_bg=True, with_mask=True)
    assert case["obj"].shape[:2] == (2, 2)
    prob = U.to_problem(case, DEV)
    assert prob.Ns == 2
    fwd = U.gpu_forward(prob)
    ref = U.oracle_forward(case["obj"].astype(np.complex128), case["prb"].astype(np.complex128),
                           case["pos"], case["pads"], sigma=case["sigma"], bg=case["bg"])
    U.check_array("Ns=2 forward", fwd, ref, 1e-5)
    for kind in (0, 1, 2):
        got = U.gpu_grads(prob, kind=kind, scale=0.5)
        assert got["g_object"].shape == case["obj"].shape
        print("Ns=2 kind", kind, U.compare(got, U.oracle_grads(case, kind=kind, scale=0.5)))


def test_sample_modes_with_exact_ratios_and_distance_gradient():
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, Ns=3, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=6, name="C1-ns3r")
    case = U.make_case(w, pads=synth.ratios_for(w.N, w.harmonics, w.ref_harmonic))
    prob = U.to_problem(case, DEV)
    got = U.gpu_grads(prob, want=ALL)
    ref = U.oracle_grads(case)
    print("Ns=3 exact ratio", U.compare(got, ref))


def test_c2_shapes_two_sample_modes():
    # 4 wavelengths x 2 sample modes = 8 slots at N = 256
    w = synth.reduced(synth.get_workload("C2"), Ns=2, K=3, name="C2-ns2")
    case = U.make_case(w, workers=U.default_workers())
    prob = U.to_problem(case, DEV)
    got = U.gpu_grads(prob)
    ref = U.oracle_grads(case, workers=U.default_workers())
    print("C2 Ns=2", U.compare(got, ref))


def test_one_sample_mode_as_4d_object_is_the_3d_call():
    case = _case(Ns=1, K=7)
    p3 = U.to_problem(case, DEV)
    p4 = U.to_problem(dict(case, obj=case["obj"][:, None]), DEV)
    assert p4.Ns == 1
    a, b = U.gpu_grads(p3), U.gpu_grads(p4)
    assert a["loss"] == b["loss"]
    for k in ("g_probe", "g_pos", "g_sigma", "g_background"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["g_object"], b["g_object"][:, 0])


def test_sample_modes_chunk_invariance():
    prob = U.to_problem(_case(K=9), DEV)
    a = U.gpu_grads(prob)
    b = U.gpu_grads(prob, chunk=4)
    for k in ("loss", "g_object", "g_probe", "g_pos", "g_sigma", "g_background"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_sixteen_slots():
    # 8 wavelengths x 2 sample modes: the largest slot count of a job
    harm = (17, 18, 19, 20, 21, 22, 23, 24)
    w = synth.reduced(synth.get_workload("C1"), L=8, M=1, Ns=2, harmonics=harm,
                      ref_harmonic=24, mode_weights=(1.0,), K=4, name="C1-16slots")
    pads = (96, 90, 84, 80, 72, 72, 64, 64)  # compiled sizes for N = 64
    case = U.make_case(w, pads=pads, with_bg=True)
    prob = U.to_problem(case, DEV)
    got = U.gpu_grads(prob, chunk=2)
    print("16 slots", pads, U.compare(got, U.oracle_grads(case)))
