"""GPU parity of the mixed-noise loss and the amplitude L1 / TV regularisers
against the FP64 oracle (loss 1e-5, gradients 1e-4, relative L2)."""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
REG = dict(l1=0.02, tv=0.5, tv_eps=0.05)


def _c1(Ns=1, K=10):
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, Ns=Ns, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=K, name=f"C1-reg{Ns}")
    return U.make_case(w, pads=(80, 64), with_sigma=True, with_bg=True, with_mask=True)


def test_mixed_noise_loss():
    case = _c1()
    prob = U.to_problem(case, DEV)
    for v in (0.5, 20.0):
        got = U.gpu_grads(prob, kind=4, noise_var=v)
        print("mixed v", v, U.compare(got, U.oracle_grads(case, kind=4, noise_var=v)))


def test_mixed_noise_loss_with_resampling():
    w = synth.get_workload("C5")
    case = U.make_case(w, K=3, workers=U.default_workers())
    got = U.gpu_grads(U.to_problem(case, DEV), kind=4, noise_var=4.0)
    print("mixed C5", U.compare(got, U.oracle_grads(case, kind=4, noise_var=4.0,
                                                     workers=U.default_workers())))


@pytest.mark.parametrize("Ns", [1, 2])
def test_amplitude_regularisers(Ns):
    case = _c1(Ns=Ns)
    prob = U.to_problem(case, DEV)
    got = U.gpu_grads(prob, **REG)
    ref = U.oracle_grads(case, **REG)
    print("regularised Ns", Ns, U.compare(got, ref))
    # only the loss and the object gradient change
    plain = U.gpu_grads(prob)
    for k in ("g_probe", "g_pos", "g_sigma", "g_background"):
        assert np.array_equal(got[k], plain[k]), k
    assert not np.array_equal(got["g_object"], plain["g_object"])


def test_regulariser_alone_is_its_closed_form_on_a_flat_object():
    # constant amplitude: TV is tv * eps per pixel, L1 is l1 * a per pixel
    case = _c1(K=4)
    obj = 0.8 * np.exp(1j * np.angle(case["obj"])).astype(np.complex64)
    case = dict(case, obj=obj)
    prob = U.to_problem(case, DEV)
    a = U.gpu_grads(prob, **REG)
    b = U.gpu_grads(prob)
    L, H, W = obj.shape
    want = REG["l1"] * 0.8 * L * H * W + REG["tv"] * REG["tv_eps"] * L * H * W
    assert abs((a["loss"] - b["loss"]) - want) <= 2e-4 * want
