"""The autograd wrapper (``PtychoLoss``, a torch.autograd.Function over the
hand-written adjoint) against central finite differences of its own forward
loss, at the shapes of the large multiplexed workload: 512 x 512 probe,
5 wavelengths x 8 modes, 3072 x 3072 object, here with 16 positions.
64 random directions, each moving 4096 object pixels, 4096 probe pixels and
every position (by steps that float32 positions represent exactly).  This checks the backward path of Fig. 1B at those shapes
independently of the oracle (which is compared elsewhere at these shapes).

The loss is a float32 scalar, so a difference of two losses carries about
one unit in the last place of the loss (ulp(L)); divided by 2h it must stay
well below the directional derivative.  So the data are noiseless (the
library's own forward model of the truth; the loss at the perturbed start
is the model mismatch alone, not Poisson noise), the directions are sparse,
drawn where |gradient| x |value| is large (probability proportional to it)
with complex normal weights scaled to the local magnitude, and Richardson
extrapolation of two central differences removes the h^2 term.  The bound
is 1e-2 of the analytic value plus 4 ulp(L) / h.
"""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _draw(rng, weight, n):
    p = weight / weight.sum()
    return rng.choice(weight.size, n, replace=False, p=p)


def test_autograd_loss_central_differences_at_large_multiplexed_shapes():
    from paper_2311_14780_amd import autograd as A
    from paper_2311_14780_amd import binding as B
    w = synth.get_workload("C3")
    case = U.make_case(w, K=16, workers=U.default_workers())
    prob = U.to_problem(case, DEV)
    # noiseless data: the library's forward model of the truth
    truth = case["truth"]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    tp = B.Problem(object=t(truth["object"][:, 0].astype(np.complex64)),
                   probe=t(truth["probe"].astype(np.complex64)), pos=t(truth["pos"]),
                   pads=case["pads"])
    meas = torch.empty(prob.K, prob.N, prob.N, device=DEV)
    B.ptycho_forward([tp], [meas], B.workspace([tp], 0))
    del tp
    obj = prob.object.clone().requires_grad_(True)
    prb = prob.probe.clone().requires_grad_(True)
    pos = prob.pos.clone().requires_grad_(True)
    scale = 1.0 / prob.K
    loss = A.ptycho_loss(obj, prb, pos, prob.pads, meas, scale=scale)
    loss.backward()
    go = obj.grad.cpu().numpy().ravel()
    gp = prb.grad.cpu().numpy().ravel()
    gs = pos.grad.cpu().numpy()
    L0 = float(loss.item())
    ulp = float(np.spacing(np.float32(abs(L0))))
    ob_np = obj.detach().cpu().numpy()
    pr_np = prb.detach().cpu().numpy()
    wo = np.abs(go) * np.abs(ob_np.ravel())
    wp = np.abs(gp) * np.abs(pr_np.ravel())
    delta = case["pos"] - np.floor(case["pos"] + np.float32(0.5))
    rng = np.random.default_rng(33)
    assert np.all(np.abs(case["pos"]) < 4096)
    nnz, h = 4096, 2.0 ** -6
    fails, worst, rels = [], 0.0, []
    for trial in range(64):
        io = _draw(rng, wo, nnz)
        ip = _draw(rng, wp, nnz)
        vo = np.zeros(ob_np.size, np.complex128)
        vp = np.zeros(pr_np.size, np.complex128)
        vo[io] = (rng.normal(size=nnz) + 1j * rng.normal(size=nnz)) * np.abs(ob_np.ravel()[io])
        vp[ip] = (rng.normal(size=nnz) + 1j * rng.normal(size=nnz)) * np.abs(pr_np.ravel()[ip])
        # every position: multiples of 1/16 px, so that s +- h vs and
        # s +- h vs / 2 (h = 2^-6) are exact in float32 (positions below
        # 4096 px are multiples of 2^-12 px) -- a rounded position step would
        # be a few per cent off at these magnitudes; coordinates near a half
        # pixel, where the window corner floor(s + 1/2) changes, stay put
        vs = rng.integers(-3, 4, size=gs.shape) * 2.0 ** -4 * (np.abs(delta) < 0.45)
        an = float(np.sum(go.real * vo.real + go.imag * vo.imag)
                   + np.sum(gp.real * vp.real + gp.imag * vp.imag) + np.sum(gs * vs))
        vo_t = torch.from_numpy(vo.reshape(ob_np.shape).astype(np.complex64)).to(DEV)
        vp_t = torch.from_numpy(vp.reshape(pr_np.shape).astype(np.complex64)).to(DEV)
        vs_t = torch.from_numpy(vs.astype(np.float32)).to(DEV)

        def central(hh):
            with torch.no_grad():
                lp = A.ptycho_loss(obj + hh * vo_t, prb + hh * vp_t, pos + hh * vs_t, prob.pads,
                                   meas, scale=scale).double().item()
                lm = A.ptycho_loss(obj - hh * vo_t, prb - hh * vp_t, pos - hh * vs_t, prob.pads,
                                   meas, scale=scale).double().item()
            return (lp - lm) / (2.0 * hh)

        fd = (4.0 * central(h / 2) - central(h)) / 3.0
        tol = 1e-2 * abs(an) + 4.0 * ulp / h
        worst = max(worst, abs(fd - an) / tol)
        rels.append(abs(fd - an) / abs(an))
        if abs(fd - an) > tol:
            fails.append((trial, fd, an))
        if trial < 4:
            print(f"direction {trial}: analytic {an:.6e} differences {fd:.6e} "
                  f"(float32 part of the bound {4.0 * ulp / h:.2e})", flush=True)
    print(f"64 directions: loss {L0:.6e}; |fd - analytic| / |analytic| median "
          f"{np.median(rels):.2e}, max {np.max(rels):.2e}; worst / bound {worst:.3f}", flush=True)
    assert not fails, fails
