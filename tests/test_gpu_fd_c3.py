"""The autograd wrapper (``PtychoLoss``, a torch.autograd.Function over the
hand-written adjoint) against central finite differences of its own forward
loss, at the shapes of the large multiplexed workload: 512 x 512 probe,
5 wavelengths x 8 modes, 3072 x 3072 object, here with 16 positions.
64 random directions, each moving 256 object pixels, 256 probe pixels and
every position.  This checks the backward path of Fig. 1B at those shapes
independently of the oracle (which is compared elsewhere at these shapes).

Float32 differences: dense random directions have a directional derivative
tiny next to the loss's curvature and rounding, so the directions are
sparse (pixels where the gradient lives, complex normal weights scaled to
the local magnitude) and Richardson extrapolation of two central
differences removes the h^2 term.  The bound adds the float32 noise of the
loss, |L| 1e-6 / h, to a relative 1e-2 of the analytic value.
"""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def test_autograd_loss_central_differences_at_large_multiplexed_shapes():
    from paper_2311_14780_amd import autograd as A
    w = synth.get_workload("C3")
    case = U.make_case(w, K=16, workers=U.default_workers())
    prob = U.to_problem(case, DEV)
    obj = prob.object.clone().requires_grad_(True)
    prb = prob.probe.clone().requires_grad_(True)
    pos = prob.pos.clone().requires_grad_(True)
    scale = 1.0 / prob.K
    loss = A.ptycho_loss(obj, prb, pos, prob.pads, prob.measured, scale=scale)
    loss.backward()
    go = obj.grad.cpu().numpy()
    gp = prb.grad.cpu().numpy()
    gs = pos.grad.cpu().numpy()
    L0 = float(loss.item())
    ob_np = obj.detach().cpu().numpy()
    pr_np = prb.detach().cpu().numpy()
    delta = case["pos"] - np.floor(case["pos"] + np.float32(0.5))
    rng = np.random.default_rng(33)
    o_live = np.flatnonzero(np.abs(go.ravel()) > 1e-3 * np.abs(go).max())
    p_live = np.flatnonzero(np.abs(pr_np.ravel()) > 0.05 * np.abs(pr_np).max())
    nnz = 256
    fails, worst = [], 0.0
    for trial in range(64):
        io = rng.choice(o_live, nnz, replace=False)
        ip = rng.choice(p_live, nnz, replace=False)
        vo = np.zeros(ob_np.size, np.complex128)
        vp = np.zeros(pr_np.size, np.complex128)
        vo[io] = (rng.normal(size=nnz) + 1j * rng.normal(size=nnz)) * np.abs(ob_np.ravel()[io])
        vp[ip] = (rng.normal(size=nnz) + 1j * rng.normal(size=nnz)) * np.abs(pr_np.ravel()[ip])
        # every position, ~0.1 px, except coordinates near a half pixel, where
        # the window corner floor(s + 1/2) would change inside the differences
        vs = rng.normal(size=gs.shape) * 0.1 * (np.abs(delta) < 0.4)
        an = float(np.sum(go.ravel().real * vo.real + go.ravel().imag * vo.imag)
                   + np.sum(gp.ravel().real * vp.real + gp.ravel().imag * vp.imag)
                   + np.sum(gs * vs))
        vo_t = torch.from_numpy(vo.reshape(ob_np.shape).astype(np.complex64)).to(DEV)
        vp_t = torch.from_numpy(vp.reshape(pr_np.shape).astype(np.complex64)).to(DEV)
        vs_t = torch.from_numpy(vs.astype(np.float32)).to(DEV)
        h = 1e-2

        def central(hh):
            with torch.no_grad():
                lp = A.ptycho_loss(obj + hh * vo_t, prb + hh * vp_t, pos + hh * vs_t, prob.pads,
                                   prob.measured, scale=scale).double().item()
                lm = A.ptycho_loss(obj - hh * vo_t, prb - hh * vp_t, pos - hh * vs_t, prob.pads,
                                   prob.measured, scale=scale).double().item()
            return (lp - lm) / (2.0 * hh)

        fd = (4.0 * central(h / 2) - central(h)) / 3.0
        tol = 1e-2 * abs(an) + 1e-6 * abs(L0) / h
        worst = max(worst, abs(fd - an) / tol)
        if abs(fd - an) > tol:
            fails.append((trial, fd, an))
        if trial < 4:
            print(f"direction {trial}: analytic {an:.6e} differences {fd:.6e} "
                  f"(noise part of the bound {1e-6 * abs(L0) / h:.2e})", flush=True)
    print(f"64 directions: worst |fd - analytic| / bound = {worst:.3f}", flush=True)
    assert not fails, fails
