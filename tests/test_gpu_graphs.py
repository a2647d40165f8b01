"""HIP-graph capture of a loss + gradient call: the library enqueues only
kernels on the caller's stream (no allocation, no memset, no host
synchronisation), so a call can be captured once and replayed.  Each replay,
with the program's own eager work and synchronisations in between, must give
the eager result bitwise (the job table and the segment lists are kernel
arguments captured with the graph, so the same call is replayed)."""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.mark.parametrize("exact", [False, True])
def test_loss_grad_graph_replays_equal_the_eager_call(exact):
    from paper_2311_14780_amd import binding as B
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=12, name="C1-graph")
    pads = synth.ratios_for(w.N, w.harmonics, w.ref_harmonic) if exact else (80, 64)
    case = U.make_case(w, pads=pads, with_sigma=True, with_bg=True)
    prob = U.to_problem(case, DEV)
    want = ("object", "probe", "pos", "sigma", "background") + (("ratio",) if exact else ())
    eager = U.gpu_grads(prob, want=want, l1=0.01, tv=0.05)
    g = dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(prob.object),
             g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(prob.K, 2, device=DEV),
             g_sigma=torch.zeros(prob.K, device=DEV),
             g_background=torch.zeros(prob.N, prob.N, device=DEV))
    if exact:
        g["g_ratio"] = torch.zeros(prob.L, device=DEV)
    ws = B.workspace([prob], 1, 5)  # several chunks inside the graph
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside the capture (twiddle tables)
        B.ptycho_loss_grad([prob], [g], workspace=ws, stream=s, l1=0.01, tv=0.05)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        B.ptycho_loss_grad([prob], [g], workspace=ws, stream=s, l1=0.01, tv=0.05)
    for rep in range(4):
        for v in g.values():  # eager work between replays
            v.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert float(g["loss"].item()) == eager["loss"], rep
        for k, v in g.items():
            if k != "loss":
                assert np.array_equal(v.cpu().numpy(), eager[k]), (rep, k)
