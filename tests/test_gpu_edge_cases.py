"""Edge cases of the exact-ratio propagator, sample modes, the extra
gradients and the loss options on the GPU: empty scans, windows that leave
the object, ragged position counts, the tilt table with several sample modes,
and the fused Adam step over every variable."""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
ALL = ("object", "probe", "pos", "sigma", "background", "ratio")


def _c1(K=7, Ns=1, exact=True, scan=None, **kw):
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, Ns=Ns, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=K, name=f"C1-edge{K}",
                      **({"scan": scan} if scan else {}))
    pads = synth.ratios_for(w.N, w.harmonics, w.ref_harmonic) if exact else (80, 64)
    return U.make_case(w, pads=pads, **kw)


def test_exact_ratio_empty_scan():
    case = _c1(K=3, with_bg=True)
    prob = U.to_problem(case, DEV)
    prob.pos = prob.pos[:0].contiguous()
    prob.measured = prob.measured[:0].contiguous()
    got = U.gpu_grads(prob, want=ALL, l1=0.0, tv=0.0)
    assert got["loss"] == 0.0
    for k in ("g_object", "g_probe", "g_background", "g_ratio"):
        assert not np.any(got[k]), k


def test_exact_ratio_window_outside_reports_erange():
    from paper_2311_14780_amd import binding as B
    case = _c1(K=6, with_bg=True)
    prob = U.to_problem(case, DEV)
    pos = prob.pos.clone()
    pos[2, 0] = 240.0  # window [240, 304) leaves the 256-px object
    prob.pos = pos
    got = U.gpu_grads(prob, want=ALL, l1=0.1, tv=0.1)
    assert np.isnan(got["loss"])
    assert B.ptycho_status(got["_ws"], 0) == B.PTYCHO_ERANGE
    for k in ("g_object", "g_probe", "g_background", "g_ratio", "g_pos"):
        assert not np.any(got[k]), k


@pytest.mark.parametrize("K,chunk", [(5, 2), (9, 3), (13, 0), (517, 130)])
def test_ragged_position_counts_and_chunks(K, chunk):
    # Ragged position counts and chunks.  Scans this small take one position
    # per column-adjoint block; 517 positions (a spiral over the object) take
    # groups of 4 (130 groups x 4 column sets >= 512 blocks): chunks rounded
    # up to the group (132), a ragged last chunk (121) and last group (1).
    kw = dict(scan="spiral") if K > 100 else {}
    case = _c1(K=K, with_sigma=True, with_bg=True, **kw)
    prob = U.to_problem(case, DEV)
    got = U.gpu_grads(prob, want=ALL, chunk=chunk)
    print(K, chunk, U.compare(got, U.oracle_grads(case)))
    ref = U.gpu_grads(prob, want=ALL)
    for k in ("g_object", "g_probe", "g_pos", "g_background", "g_ratio"):
        assert np.array_equal(got[k], ref[k]), k


def test_two_sample_modes_with_the_tilt_table():
    w = synth.reduced(synth.get_workload("C5"), Ns=2, K=2, name="C5-ns2")
    case = U.make_case(w, with_bg=True, workers=U.default_workers())
    assert case["table"] is not None and case["obj"].ndim == 4
    got = U.gpu_grads(U.to_problem(case, DEV), kind=4, noise_var=3.0)
    ref = U.oracle_grads(case, kind=4, noise_var=3.0, workers=U.default_workers())
    print("C5 Ns=2 mixed", U.compare(got, ref))


def test_fused_step_over_every_variable_uses_the_gradient_of_the_state_before():
    from paper_2311_14780_amd import binding as B
    case = _c1(K=8, with_sigma=True, with_bg=True)
    reg = dict(noise_var=2.0, l1=0.01, tv=0.1, tv_eps=0.05)
    prob = U.to_problem(case, DEV)
    ref = U.gpu_grads(prob, kind=4, want=ALL, **reg)  # loss + gradients alone
    g = dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(prob.object),
             g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(prob.K, 2, device=DEV),
             g_sigma=torch.zeros(prob.K, device=DEV),
             g_background=torch.zeros(prob.N, prob.N, device=DEV),
             g_ratio=torch.zeros(prob.L, device=DEV))
    z = lambda x: torch.zeros(x.numel() * (2 if x.is_complex() else 1), device=DEV)
    adam = dict(m_object=z(prob.object), v_object=z(prob.object), m_probe=z(prob.probe),
                v_probe=z(prob.probe), m_pos=z(prob.pos), v_pos=z(prob.pos),
                m_sigma=z(prob.sigma), v_sigma=z(prob.sigma), m_background=z(prob.background),
                v_background=z(prob.background), lr_object=1e-3, lr_probe=1e-3, lr_pos=1e-2,
                lr_sigma=1e-3, lr_background=1e-2, t=1)
    o0, s0, b0 = prob.object.clone(), prob.sigma.clone(), prob.background.clone()
    B.ptycho_step([prob], [g], [adam], kind=4, workspace=B.workspace([prob], 2), **reg)
    torch.cuda.synchronize()
    assert float(g["loss"].item()) == ref["loss"]
    for k in ("g_object", "g_probe", "g_pos", "g_sigma", "g_background", "g_ratio"):
        assert np.array_equal(g[k].cpu().numpy(), ref[k]), k
    # every variable with a learning rate moved by -lr g / (|g| + eps), which
    # is -lr sign(g) to 1e-4 where |g| > 1e-4
    for x0, x1, gg, lr in ((o0, prob.object, g["g_object"], 1e-3), (s0, prob.sigma, g["g_sigma"], 1e-3),
                           (b0, prob.background, g["g_background"], 1e-2)):
        r = lambda t: torch.view_as_real(t).reshape(-1) if t.is_complex() else t.reshape(-1)
        d = (r(x1) - r(x0)).double().cpu().numpy()
        want = -lr * np.sign(r(gg).double().cpu().numpy())
        mask = np.abs(r(gg).cpu().numpy()) > 1e-4
        assert mask.sum() > 0
        assert np.allclose(d[mask], want[mask], rtol=1e-3, atol=2e-7)
