"""The allocation-free loss + gradient entry point (ptycho_loss_grad_noalloc,
for callers that cannot allocate device memory) against ptycho_loss_grad,
through the C ABI: two calls in a row on the library's static scratch, the
second with a smaller job, each equal bitwise to the regular call with a
caller workspace (same kernels; sums over positions run in a fixed order, so
the chunking that the fixed scratch imposes does not change any bit).  The
second call also checks that nothing left in the scratch by the first one
leaks into it.  A job too large for the scratch is rejected before anything
is enqueued."""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
KEYS = ("loss", "g_object", "g_probe", "g_pos", "g_sigma", "g_background")


def _grads(prob):
    return dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(prob.object),
                g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(prob.K, 2, device=DEV),
                g_sigma=torch.zeros(prob.K, device=DEV),
                g_background=torch.zeros(prob.N, prob.N, device=DEV))


def _case(K, L, M, pads, seed, harmonics):
    w = synth.reduced(synth.get_workload("C1"), L=L, M=M, harmonics=harmonics,
                      mode_weights=tuple([1.0 / M] * M), K=K, name=f"C1-na{K}")
    return U.make_case(w, pads=pads, with_sigma=True, with_bg=True, with_mask=True,
                       seed_offset=seed)


def test_noalloc_matches_the_workspace_call_twice_in_a_row():
    from paper_2311_14780_amd import binding as B
    # first call: 10 positions of the four-wavelength 256 x 256 workload
    # (~10.5 MB of chunk workspace per position: the 64 MiB scratch runs it
    # in chunks of 4, the regular call in one chunk); second call: a smaller
    # job with another window and pad
    cases = [U.make_case(synth.get_workload("C2"), K=10, with_sigma=True, with_bg=True,
                         workers=U.default_workers()),
             _case(9, 1, 2, (72,), 2, (23,))]
    for i, case in enumerate(cases):
        prob = U.to_problem(case, DEV)
        print(f"call {i}: K={prob.K} L={prob.L} M={prob.M} pads={prob.pads}", flush=True)
        g_ref = _grads(prob)
        B.ptycho_loss_grad([prob], [g_ref], kind=1, scale=0.5, workspace=B.workspace([prob]))
        g = _grads(prob)
        for v in g.values():  # garbage in the outputs: the call must overwrite them
            v.fill_(7.0)
        B.ptycho_loss_grad_noalloc([prob], [g], kind=1, scale=0.5)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(g[k], g_ref[k]), (i, k)
        got = {k: (float(v.item()) if k == "loss" else v.cpu().numpy()) for k, v in g.items()}
        U.compare(got, U.oracle_grads(case, kind=1, scale=0.5, workers=U.default_workers()))


def test_noalloc_rejects_a_job_larger_than_the_scratch():
    from paper_2311_14780_amd import binding as B
    w = synth.get_workload("C3")
    # one position of the large workload needs ~110 MB of chunk workspace
    need = B.workspace_bytes_for_shapes([(1, w.L, w.M, w.N, w.H, w.W,
                                          synth.pads_for(w.N, w.harmonics, w.ref_harmonic))],
                                        which=1, chunk=1)
    assert need > B.NOALLOC_SCRATCH_BYTES
    t = lambda *s, **kw: torch.zeros(*s, device=DEV, **kw)
    prob = B.Problem(object=t(w.L, 512 + 8, 512 + 8, dtype=torch.complex64),
                     probe=t(w.L, w.M, w.N, w.N, dtype=torch.complex64),
                     pos=t(1, 2), pads=synth.pads_for(w.N, w.harmonics, w.ref_harmonic),
                     measured=t(1, w.N, w.N))
    g = dict(loss=t(1))
    with pytest.raises(B.PtychoError) as e:
        B.ptycho_loss_grad_noalloc([prob], [g])
    assert e.value.code == B.PTYCHO_ENOSPC
    assert float(g["loss"].item()) == 0.0  # nothing was enqueued
