"""GPU parity of the grouped-position column adjoint: jobs whose [M][N][G]
probe-gradient accumulator does not fit in LDS sum the terms of three
consecutive positions per block in registers (probe-gradient groups of
three).

N = 256 with 5 modes: at DFT size 300 (16-column blocks) the accumulator
needs 5 x 256 x 16 x 8 B = 160 KiB, more than a block's LDS, while three
positions' Ohat (96 KiB) next to the transform buffer and twiddles (44 KiB)
fit, so the job takes groups of three; its other DFT size, 343 (8-column
blocks), then runs the grouped-position instance as well.  Position counts
that are not multiples of three leave a short group (one position at K = 7,
two at K = 5) at the end of the scan.  Checked against the FP64 oracle, for
bitwise chunk invariance, and for bitwise equality alone and next to a job
with groups of four in one call."""
import numpy as np
import pytest

import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
KEYS = ("loss", "g_object", "g_probe", "g_pos", "g_sigma", "g_background")


def _workload(K, M=5):
    weights = tuple(0.5 ** m for m in range(M))
    return synth.reduced(synth.get_workload("C2"), L=2, M=M, harmonics=(19, 23),
                         mode_weights=weights, K=K, name="C2-pairs")


def test_pairs_against_oracle_odd_positions():
    case = U.make_case(_workload(7), with_sigma=True, with_bg=True, pads=(300, 343))
    print("pads", case["pads"], "K", case["pos"].shape[0], flush=True)
    prob = U.to_problem(case, DEV)
    for kind in (0, 1):
        got = U.gpu_grads(prob, kind=kind, scale=0.5)
        ref = U.oracle_grads(case, kind=kind, scale=0.5)
        print("kind", kind, U.compare(got, ref), flush=True)


def test_pairs_chunk_invariant():
    case = U.make_case(_workload(9), with_sigma=True, pads=(300, 343))
    prob = U.to_problem(case, DEV)
    whole = U.gpu_grads(prob)
    for chunk in (3, 4):  # 4 is rounded up to a whole number of groups (6)
        part = U.gpu_grads(prob, chunk=chunk)
        for k in KEYS:
            assert np.array_equal(np.asarray(whole[k]), np.asarray(part[k])), (chunk, k)


def _grads_of(prob):
    g = dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(prob.object),
             g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(prob.K, 2, device=DEV),
             g_sigma=torch.zeros(prob.K, device=DEV),
             g_background=torch.zeros(prob.N, prob.N, device=DEV))
    return g


def test_pairs_alone_and_next_to_a_grouped_job():
    from paper_2311_14780_amd import binding as B
    pair_case = U.make_case(_workload(5), with_sigma=True, pads=(300, 343))
    quad_case = U.make_case(_workload(6, M=2), with_sigma=True, pads=(300, 343), seed_offset=3)
    pa, pb = U.to_problem(pair_case, DEV), U.to_problem(quad_case, DEV)
    alone = [U.gpu_grads(pa), U.gpu_grads(pb)]
    ga, gb = _grads_of(pa), _grads_of(pb)
    ws = B.workspace([pa, pb], 1)
    B.ptycho_loss_grad([pa, pb], [ga, gb], workspace=ws)
    torch.cuda.synchronize()
    for ref, g in zip(alone, (ga, gb)):
        for k in KEYS:
            v = g[k].cpu().numpy()
            if k == "loss":
                v = float(v[0])
            assert np.array_equal(np.asarray(ref[k]), np.asarray(v)), k


def _n384(K, M=2):
    weights = tuple(0.5 ** m for m in range(M))
    return synth.reduced(synth.get_workload("C5"), L=2, M=M, harmonics=(19, 23),
                         mode_weights=weights, K=K, name="C5-groups")


def test_n384_register_groups_and_lds_groups_beside_an_exact_ratio():
    # zero-padded wavelengths at N = 384 take register groups of three (a
    # short group of one at K = 7); with one exact-ratio wavelength, which has
    # no grouped-position instance, the job takes LDS groups of four
    for pads in ((420, 480), (420, 384 * 23 / 19)):
        case = U.make_case(_n384(7), with_sigma=True, pads=pads)
        print("N=384 pads", case["pads"], flush=True)
        prob = U.to_problem(case, DEV)
        got = U.gpu_grads(prob, kind=0)
        ref = U.oracle_grads(case, kind=0)
        print("  ", U.compare(got, ref), flush=True)
        part = U.gpu_grads(prob, chunk=3)
        for k in KEYS:
            assert np.array_equal(np.asarray(got[k]), np.asarray(part[k])), (pads, k)
