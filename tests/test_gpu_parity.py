"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2 per array): intensities 1e-5, loss 1e-5, every
gradient 1e-4.  Inputs are the seeded synthetic workloads; measured counts
are Poisson draws from the oracle's own forward model of the truth.
"""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def c1():
    return U.make_case(synth.get_workload("C1"))


def test_c1_forward_matches_oracle(c1):
    prob = U.to_problem(c1, DEV)
    got = U.gpu_forward(prob)
    ref = U.oracle_forward(c1["obj"].astype(np.complex128), c1["prb"].astype(np.complex128),
                           c1["pos"], c1["pads"])
    U.check_array("C1 forward", got, ref, 1e-5)


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_c1_loss_grad_matches_oracle(c1, kind):
    prob = U.to_problem(c1, DEV)
    got = U.gpu_grads(prob, kind=kind)
    ref = U.oracle_grads(c1, kind=kind)
    print("C1 kind", kind, U.compare(got, ref))


def test_sigma_background_mask_multiwavelength():
    # three wavelengths with ragged pads, two modes, sigma, background, mask
    w = synth.reduced(synth.get_workload("C1"), L=3, M=2, harmonics=(19, 21, 23),
                      mode_weights=(0.75, 0.25), K=12, name="C1-multi")
    case = U.make_case(w, with_sigma=True, with_bg=True, with_mask=True, pads=(80, 72, 64))
    prob = U.to_problem(case, DEV)
    for kind in (0, 1):
        got = U.gpu_grads(prob, kind=kind, scale=0.25)
        ref = U.oracle_grads(case, kind=kind, scale=0.25)
        print("multi kind", kind, U.compare(got, ref))
    fwd = U.gpu_forward(prob)
    ref = U.oracle_forward(case["obj"].astype(np.complex128), case["prb"].astype(np.complex128),
                           case["pos"], case["pads"], sigma=case["sigma"], bg=case["bg"])
    U.check_array("multi forward", fwd, ref, 1e-5)


def test_c2_reduced_positions_full_shapes():
    case = U.make_case(synth.get_workload("C2"), K=6)
    prob = U.to_problem(case, DEV)
    fwd = U.gpu_forward(prob)
    ref = U.oracle_forward(case["obj"].astype(np.complex128), case["prb"].astype(np.complex128),
                           case["pos"], case["pads"])
    U.check_array("C2(K=6) forward", fwd, ref, 1e-5)
    got = U.gpu_grads(prob)
    rg = U.oracle_grads(case)
    print("C2(K=6) grads", U.compare(got, rg))


def test_chunking_is_bitwise_invariant(c1):
    prob = U.to_problem(c1, DEV)
    a = U.gpu_grads(prob, chunk=0)
    b = U.gpu_grads(prob, chunk=7)
    for k in ("loss", "g_object", "g_probe", "g_pos", "g_sigma", "g_background"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_multi_job_call_matches_single_jobs(c1):
    from paper_2311_14780_amd import binding as B
    case2 = U.make_case(synth.reduced(synth.get_workload("C1"), K=9, seed=11, name="C1b"))
    p1, p2 = U.to_problem(c1, DEV), U.to_problem(case2, DEV)
    s1, s2 = U.gpu_grads(p1), U.gpu_grads(p2)
    gs = []
    for p in (p1, p2):
        gs.append(dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(p.object),
                       g_probe=torch.zeros_like(p.probe), g_pos=torch.zeros(p.K, 2, device=DEV),
                       g_sigma=torch.zeros(p.K, device=DEV),
                       g_background=torch.zeros(p.N, p.N, device=DEV)))
    ws = B.workspace([p1, p2])
    B.ptycho_loss_grad([p1, p2], gs, workspace=ws)
    torch.cuda.synchronize()
    for single, g in ((s1, gs[0]), (s2, gs[1])):
        assert single["loss"] == float(g["loss"].item())
        for k in ("g_object", "g_probe", "g_pos", "g_sigma", "g_background"):
            assert np.array_equal(single[k], g[k].cpu().numpy()), k


def test_empty_scan():
    case = U.make_case(synth.reduced(synth.get_workload("C1"), K=3, name="C1e"))
    prob = U.to_problem(case, DEV)
    prob.pos = prob.pos[:0].contiguous()
    prob.measured = prob.measured[:0].contiguous()
    got = U.gpu_grads(prob)
    assert got["loss"] == 0.0
    assert not np.any(got["g_object"]) and not np.any(got["g_probe"])


def test_window_outside_object_reports_erange(c1):
    from paper_2311_14780_amd import binding as B
    prob = U.to_problem(c1, DEV)
    pos = prob.pos.clone()
    pos[3, 1] = 250.0  # window [250, 314) leaves the 256-px object
    prob.pos = pos
    got = U.gpu_grads(prob)
    assert np.isnan(got["loss"])
    assert B.ptycho_status(got["_ws"], 0) == B.PTYCHO_ERANGE
    assert not np.any(got["g_object"])
    # the same workspace reports OK again after a valid call
    prob.pos = U.to_problem(c1, DEV).pos
    got = U.gpu_grads(prob)
    assert B.ptycho_status(got["_ws"], 0) == B.PTYCHO_OK


def test_heterogeneous_jobs_in_one_fused_call():
    """Jobs of different sizes, wavelength and mode counts, pads, chunking
    and requested outputs share the launches of one call; each job's results
    are bitwise identical to running it alone."""
    from paper_2311_14780_amd import binding as B
    base = synth.get_workload("C1")
    specs = [
        dict(w=synth.reduced(base, K=7, name="h1"), pads=None, want=("object", "probe", "pos", "sigma")),
        dict(w=synth.reduced(base, K=11, L=2, M=3, harmonics=(21, 23), mode_weights=(0.6, 0.3, 0.1),
                             seed=21, name="h2"), pads=(72, 64), want=("object", "pos")),
        dict(w=synth.reduced(base, K=5, L=3, M=2, harmonics=(19, 21, 23), mode_weights=(0.7, 0.3),
                             seed=22, name="h3"), pads=(90, 80, 64), want=("probe",)),
        dict(w=synth.reduced(synth.get_workload("C2"), K=3, L=2, M=2, harmonics=(21, 23),
                             mode_weights=(0.6, 0.4), seed=23, name="h4"), pads=(280, 256),
             want=("object", "probe", "pos", "sigma")),
    ]
    probs, singles, gs = [], [], []
    for sp in specs:
        case = U.make_case(sp["w"], pads=sp["pads"], with_sigma=True)
        p = U.to_problem(case, DEV)
        probs.append(p)
        singles.append(U.gpu_grads(p, want=sp["want"]))
        g = dict(loss=torch.zeros(1, device=DEV))
        if "object" in sp["want"]:
            g["g_object"] = torch.zeros_like(p.object)
        if "probe" in sp["want"]:
            g["g_probe"] = torch.zeros_like(p.probe)
        if "pos" in sp["want"]:
            g["g_pos"] = torch.zeros(p.K, 2, device=DEV)
        if "sigma" in sp["want"]:
            g["g_sigma"] = torch.zeros(p.K, device=DEV)
        gs.append(g)
    ws = B.workspace(probs, 1, chunk=4)  # forces several chunk iterations
    B.ptycho_loss_grad(probs, gs, workspace=ws)
    torch.cuda.synchronize()
    for single, g in zip(singles, gs):
        assert single["loss"] == float(g["loss"].item())
        for k, v in g.items():
            if k != "loss":
                assert np.array_equal(single[k], v.cpu().numpy()), k
    # and the forward of the same mix
    outs = [torch.empty(p.K, p.N, p.N, device=DEV) for p in probs]
    B.ptycho_forward(probs, outs, B.workspace(probs, 0))
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        assert np.array_equal(U.gpu_forward(p), o.cpu().numpy())
