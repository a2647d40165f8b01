"""GPU parity for jobs whose wavelengths use column-adjoint instances with
different column groups.  For N = 256 the DFT sizes 256, 280, 315 and 343 run
with 8 columns per block and the other sizes (and the exact-ratio length 2N)
with 16, so the number of per-block partial sums of the position and sigma
gradients differs between the slots of one job.  Checked against the FP64
oracle (tolerances as for the other parity tests) and for bitwise chunk
invariance."""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _workload(K):
    return synth.reduced(synth.get_workload("C2"), L=2, M=2, harmonics=(19, 23),
                         mode_weights=(0.75, 0.25), K=K, name="C2-groups")


def test_mixed_column_groups_zero_padded():
    # pad 300 (16-column blocks) next to pad 343 (8-column blocks)
    case = U.make_case(_workload(4), with_sigma=True, with_bg=True, pads=(300, 343))
    print("pads", case["pads"], flush=True)
    prob = U.to_problem(case, DEV)
    for kind in (0, 1):
        got = U.gpu_grads(prob, kind=kind, scale=0.5)
        ref = U.oracle_grads(case, kind=kind, scale=0.5)
        print("kind", kind, U.compare(got, ref), flush=True)


def test_mixed_column_groups_pad_and_exact_ratio():
    # pad 343 (8-column blocks) next to an exact ratio (length 512, 16 columns),
    # with the distance gradient, whose column terms use the same partials
    case = U.make_case(_workload(4), with_sigma=True, pads=(343, 300.7))
    print("pads", case["pads"], flush=True)
    prob = U.to_problem(case, DEV)
    got = U.gpu_grads(prob, want=("object", "probe", "pos", "sigma", "background", "ratio"))
    ref = U.oracle_grads(case)
    print(U.compare(got, ref), "g_ratio", got["g_ratio"], ref["g_ratio"], flush=True)
    assert got["g_ratio"][0] == 0.0


def test_mixed_column_groups_chunk_invariant():
    case = U.make_case(_workload(9), with_sigma=True, pads=(300, 343))
    prob = U.to_problem(case, DEV)
    whole = U.gpu_grads(prob)
    part = U.gpu_grads(prob, chunk=4)
    for k in ("loss", "g_object", "g_probe", "g_pos", "g_sigma", "g_background"):
        assert np.array_equal(np.asarray(whole[k]), np.asarray(part[k])), k
