"""The C ABI library loads, exports every declared symbol and validates its
arguments on the host (CPU only: no kernel is launched here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import synth
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptycho.h")

B = pytest.importorskip("paper_2311_14780_amd.binding")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(ptycho_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = _declared()
    assert len(names) >= 9
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (ptycho_\w+)", out))
    for n in names:
        assert n in exported, n
        getattr(lib, n)


def test_error_strings():
    for code in (0, -1, -2, -3, -4, -5):
        assert B.error_string(code)
    assert "unknown" in B.error_string(-99)


def test_supported_sizes():
    for N, pads in ((64, (64, 72, 80, 84, 90, 96)), (256, (256, 280, 315, 343)),
                    (384, (384, 420, 480)), (512, (512, 560, 600, 675, 750)),
                    (128, (128, 140, 150, 168, 189))):
        for p in pads:
            assert B.ptycho_supported(N, p)
    assert not B.ptycho_supported(256, 257)
    assert not B.ptycho_supported(100, 100)


def _job(K=4, L=2, M=3, N=64, H=128, W=128, pads=(64, 80)):
    j = B.JobT()
    j.K, j.L, j.M, j.N, j.H, j.W = K, L, M, N, H, W
    for l, p in enumerate(pads):
        j.pad[l] = p
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    j.object = j.probe = j.pos = j.measured = fake
    return j


def _ws_bytes(j, which=1, chunk=0):
    out = ctypes.c_size_t(0)
    code = B.lib().ptycho_workspace_bytes(ctypes.byref(j), 1, which, chunk, ctypes.byref(out))
    return code, out.value


def test_workspace_bytes_scale_with_chunk():
    j = _job(K=20)
    c_all, b_all = _ws_bytes(j)
    c_one, b_one = _ws_bytes(j, chunk=1)
    assert c_all == 0 and c_one == 0
    assert b_all > b_one > 0
    # per position: X, GX (L N^2 c64 each), Y (L M N^2 c64), ramps, partials
    per = 8 * 64 * 64 * (2 * 2 + 2 * 3)
    assert b_all - b_one >= 3 * per
    # a scan this small takes one position per column-adjoint block (groups of
    # four would leave the launch with 20 blocks): chunks are not rounded
    assert _ws_bytes(j, chunk=1)[1] < _ws_bytes(j, chunk=2)[1]
    # with enough positions (1100 / 4 x 4 column sets >= 512 blocks) loss +
    # gradient calls take positions in groups of 4 for the probe gradient:
    # a smaller chunk is rounded up to the group
    big = _job(K=1100)
    assert _ws_bytes(big, chunk=1) == _ws_bytes(big, chunk=4)
    assert _ws_bytes(big, chunk=5) == _ws_bytes(big, chunk=8)
    assert _ws_bytes(big, chunk=4)[1] < _ws_bytes(big, chunk=5)[1]
    # the forward pass does not group positions
    assert _ws_bytes(big, which=0, chunk=1)[1] < _ws_bytes(big, which=0, chunk=2)[1]


def test_probe_group_choice_at_n384():
    # zero-padded wavelengths at N = 384: register groups of three
    pad = _job(K=900, L=2, M=4, N=384, H=1024, W=1024, pads=(420, 480))
    assert _ws_bytes(pad, chunk=1) == _ws_bytes(pad, chunk=3)
    assert _ws_bytes(pad, chunk=3)[1] < _ws_bytes(pad, chunk=4)[1]
    # one exact-ratio wavelength (no grouped-position instance): LDS groups of
    # four, which both wavelengths fit
    mixed = _job(K=900, L=2, M=2, N=384, H=1024, W=1024, pads=(420, 0))
    mixed.ratio[1] = 401.5
    assert _ws_bytes(mixed, chunk=1) == _ws_bytes(mixed, chunk=4)
    assert _ws_bytes(mixed, chunk=4)[1] < _ws_bytes(mixed, chunk=5)[1]


@pytest.mark.parametrize("change,code", [
    (dict(L=0), B.PTYCHO_EINVAL), (dict(L=9), B.PTYCHO_EINVAL), (dict(M=0), B.PTYCHO_EINVAL),
    (dict(K=-1), B.PTYCHO_EINVAL), (dict(N=100), B.PTYCHO_EUNSUPPORTED),
    (dict(H=32), B.PTYCHO_ERANGE), (dict(pads=(64, 63)), B.PTYCHO_ERANGE),
    (dict(pads=(64, 81)), B.PTYCHO_EUNSUPPORTED)])
def test_invalid_jobs_rejected_on_host(change, code):
    kw = dict(K=4, L=2, M=3, N=64, H=128, W=128, pads=(64, 80))
    kw.update(change)
    j = _job(**kw)
    assert _ws_bytes(j)[0] == code
    loss = B.LossT(0, 1e-6, 1.0)
    grads = B.GradsT()
    rc = B.lib().ptycho_loss_grad(ctypes.byref(j), 1, ctypes.byref(loss), ctypes.byref(grads),
                                  ctypes.c_void_p(0x2000), 1 << 20, None)
    assert rc == code


def test_null_pointers_rejected():
    loss = B.LossT(0, 1e-6, 1.0)
    grads = B.GradsT()
    for field in ("object", "probe", "pos", "measured"):
        j = _job()
        setattr(j, field, None)
        rc = B.lib().ptycho_loss_grad(ctypes.byref(j), 1, ctypes.byref(loss), ctypes.byref(grads),
                                      ctypes.c_void_p(0x2000), 1 << 20, None)
        assert rc == B.PTYCHO_EINVAL, field
    rc = B.lib().ptycho_loss_grad(None, 1, ctypes.byref(loss), ctypes.byref(grads),
                                  ctypes.c_void_p(0x2000), 1 << 20, None)
    assert rc == B.PTYCHO_EINVAL


def test_partial_resample_table_rejected():
    j = _job()
    j.rs_idx = ctypes.c_void_p(0x3000)
    assert _ws_bytes(j)[0] == B.PTYCHO_EINVAL


def test_transpose_table_matches_oracle_adjoint():
    from oracle import model as om
    from synth.tilt import tilt_table
    N = 64
    idx, w, mask = tilt_table(N)
    ptr, col, val = B.ptycho_transpose_table(idx, w, N * N)
    assert ptr[0] == 0 and ptr[-1] == int(np.count_nonzero(w))
    g = np.random.default_rng(0).normal(size=(N, N))
    out = np.zeros(N * N)
    for j in range(N * N):
        s, e = ptr[j], ptr[j + 1]
        out[j] = np.sum(val[s:e].astype(np.float64) * g.ravel()[col[s:e]])
    ref = om.resample_adjoint(g, idx, w)
    assert np.allclose(out.reshape(N, N), ref, rtol=1e-12, atol=1e-12)
    # columns ascend inside each row (fixed summation order)
    for j in range(0, N * N, 97):
        s, e = ptr[j], ptr[j + 1]
        assert np.all(np.diff(col[s:e]) >= 0)


def test_transpose_table_rejects_bad_index():
    idx = np.array([[0, 1, 2, 99]], np.int32)
    w = np.full((1, 4), 0.25, np.float32)
    with pytest.raises(B.PtychoError):
        B.ptycho_transpose_table(idx, w, 4)


def test_workspace_query_reads_sizes_only():
    """A scheduler sizes a call before allocating: the query ignores the
    array pointers and gives the same answer as with them."""
    j = _job()
    ref = _ws_bytes(j, which=2, chunk=3)
    for field in ("object", "probe", "pos", "measured"):
        setattr(j, field, None)
    assert _ws_bytes(j, which=2, chunk=3) == ref
    got = B.workspace_bytes_for_shapes([(4, 2, 3, 64, 128, 128, (64, 80))], which=2, chunk=3)
    assert ref == (0, got)


def test_serving_mix_pads_are_compiled_in():
    import synth.serving as SS
    for w in SS.serving_jobs(64, 4):
        for p in synth.pads_for(w.N, w.harmonics, w.ref_harmonic):
            assert B.ptycho_supported(w.N, p), (w.N, p)


def _job_ratio(ratios, **kw):
    j = _job(**kw)
    for l, a in enumerate(ratios):
        if a:
            j.pad[l], j.ratio[l] = 0, a
    return j


def test_job_struct_layout():
    # six int32 sizes, pad[8], then ratio[8] (8-byte aligned), then pointers
    assert B.JobT.ratio.offset == 56
    assert B.JobT.object.offset == 56 + 64


@pytest.mark.parametrize("ratio,code", [
    (-1.0, B.PTYCHO_EINVAL), (float("nan"), B.PTYCHO_EINVAL), (float("inf"), B.PTYCHO_EINVAL),
    (63.5, B.PTYCHO_ERANGE)])
def test_invalid_ratio_rejected_on_host(ratio, code):
    j = _job_ratio((0.0, ratio))
    assert _ws_bytes(j)[0] == code
    loss = B.LossT(0, 1e-6, 1.0)
    grads = B.GradsT()
    rc = B.lib().ptycho_loss_grad(ctypes.byref(j), 1, ctypes.byref(loss), ctypes.byref(grads),
                                  ctypes.c_void_p(0x2000), 1 << 20, None)
    assert rc == code


def test_ratio_ignores_pad_and_workspace_holds_the_chirp_tables():
    # the pad of an exact-ratio wavelength is not validated (0 here)
    j = _job_ratio((0.0, 77.3), K=8)
    c, b = _ws_bytes(j, chunk=4)
    assert c == 0
    ref = _ws_bytes(_job(K=8), chunk=4)[1]
    # one table of 4N complex64 per wavelength of the job
    assert b - ref >= 2 * 4 * 64 * 8
    got = B.workspace_bytes_for_shapes([(8, 2, 3, 64, 128, 128, (64, 77.3))], which=1, chunk=4)
    assert got == b
    # an integer-valued ratio is still the exact-ratio propagator
    assert _ws_bytes(_job_ratio((64.0, 0.0), K=8), chunk=4)[1] > ref


def test_grads_and_adam_struct_layout():
    assert B.GradsT.g_background.offset == 5 * 8
    # six pointers, six floats, t, then the sigma / background extension
    assert B.AdamT.t.offset == 72
    assert B.AdamT.m_sigma.offset == 80
    assert B.AdamT.lr_background.offset == 80 + 32 + 4


def test_adam_of_sigma_needs_its_state():
    j = _job()
    loss = B.LossT(0, 1e-6, 1.0)
    grads = B.GradsT()
    adam = B.AdamT()
    adam.t, adam.beta1, adam.beta2, adam.lr_sigma = 1, 0.9, 0.999, 1e-3
    rc = B.lib().ptycho_step(ctypes.byref(j), 1, ctypes.byref(loss), ctypes.byref(grads),
                             ctypes.byref(adam), ctypes.c_void_p(0x2000), 1 << 20, None)
    assert rc == B.PTYCHO_EINVAL


@pytest.mark.parametrize("L,Ns,code", [(2, -1, B.PTYCHO_EINVAL), (2, 17, B.PTYCHO_EINVAL),
                                       (8, 3, B.PTYCHO_EINVAL), (8, 2, 0), (2, 0, 0)])
def test_sample_mode_limits(L, Ns, code):
    j = _job(L=L, pads=(64,) * L)
    j.Ns = Ns
    assert _ws_bytes(j)[0] == code


def test_sample_modes_scale_the_per_position_workspace():
    j1, j2 = _job(K=8), _job(K=8)
    j2.Ns = 3
    b1 = _ws_bytes(j1, chunk=4)[1]
    b2 = _ws_bytes(j2, chunk=4)[1]
    # X, GX and Y grow with the slot count (L Ns)
    assert b2 - b1 >= 4 * 8 * 64 * 64 * 2 * (2 + 3)


@pytest.mark.parametrize("fields", [
    dict(kind=5), dict(kind=4, noise_var=0.0), dict(kind=4, noise_var=float("nan")),
    dict(l1=-1.0), dict(tv=1.0, tv_eps=0.0), dict(tv=float("inf"))])
def test_invalid_loss_parameters_rejected_on_host(fields):
    j = _job()
    kw = dict(kind=0, eps=1e-6, scale=1.0, noise_var=1.0, l1=0.0, tv=0.0, tv_eps=1e-3)
    kw.update(fields)
    loss = B.LossT(kw["kind"], kw["eps"], kw["scale"], kw["noise_var"], kw["l1"], kw["tv"],
                   kw["tv_eps"])
    grads = B.GradsT()
    rc = B.lib().ptycho_loss_grad(ctypes.byref(j), 1, ctypes.byref(loss), ctypes.byref(grads),
                                  ctypes.c_void_p(0x2000), 1 << 20, None)
    assert rc == B.PTYCHO_EINVAL


def test_profile_class_selection_on_the_host():
    # the class mask is host state: set and cleared without launching anything
    B.ptycho_profile_classes(["det", "col_adj"])
    B.ptycho_profile_classes(None)
    with pytest.raises(KeyError):
        B.ptycho_profile_classes(["no_such_class"])
    assert B.lib().ptycho_profile_classes(0) == 0
    B.ptycho_profile(False)  # also resets the mask to every class


# ----------------------------------------------------- binding argument checks
# The C ABI takes bare device pointers, so the binding is the only layer that
# can see a tensor's dtype, shape and device.  These run without a GPU: dtype
# and shape are checked before the device.

def _cpu_problem(L=2, M=3, N=64, K=5, H=128, W=96, **over):
    import torch
    kw = dict(object=torch.zeros(L, H, W, dtype=torch.complex64),
              probe=torch.zeros(L, M, N, N, dtype=torch.complex64),
              pos=torch.zeros(K, 2), pads=(N,) * L,
              measured=torch.zeros(K, N, N))
    kw.update(over)
    return B.Problem(**kw)


@pytest.mark.parametrize("field,bad,what", [
    ("object", "2d", "object"),
    ("object", "real", "object"),
    ("measured", "wrong_k", "measured"),
    ("measured", "wrong_n", "measured"),
    ("pos", "flat", "pos"),
    ("sigma", "wrong_k", "sigma"),
    ("background", "float64", "background"),
    ("mask", "bool", "mask"),
])
def test_binding_rejects_bad_tensors(field, bad, what):
    import torch
    L, M, N, K, H, W = 2, 3, 64, 5, 128, 96
    t = {
        ("object", "2d"): torch.zeros(H, W, dtype=torch.complex64),
        ("object", "real"): torch.zeros(L, H, W),
        ("measured", "wrong_k"): torch.zeros(K + 1, N, N),
        ("measured", "wrong_n"): torch.zeros(K, N, N + 1),
        ("pos", "flat"): torch.zeros(2 * K),
        ("sigma", "wrong_k"): torch.zeros(K - 1),
        ("background", "float64"): torch.zeros(N, N, dtype=torch.float64),
        ("mask", "bool"): torch.zeros(N, N, dtype=torch.bool),
    }[(field, bad)]
    p = _cpu_problem(L, M, N, K, H, W, **{field: t})
    with pytest.raises(ValueError, match=what):
        p.to_job()


def test_binding_rejects_host_tensors_and_bad_gradients():
    import torch
    p = _cpu_problem()
    # correct shapes and dtypes, but host memory: never handed to the library
    with pytest.raises(ValueError, match="GPU"):
        p.to_job()
    with pytest.raises(ValueError, match="GPU"):
        B.ptycho_loss_grad([p], [dict(loss=torch.zeros(1))], workspace=torch.zeros(8, dtype=torch.uint8))
    # gradient outputs are checked against the job's shapes
    for key, t in (("g_object", torch.zeros(2, 128, 96)),                      # real
                   ("g_probe", torch.zeros(2, 3, 64, 63, dtype=torch.complex64)),
                   ("g_pos", torch.zeros(5)),
                   ("g_ratio", torch.zeros(3)),
                   ("loss", torch.zeros(2)),
                   ("g_bogus", torch.zeros(1))):
        with pytest.raises(ValueError, match=key):
            B._check_grads([p], [{key: t}])
    with pytest.raises(ValueError):
        B._check_grads([p, p], [{}])
