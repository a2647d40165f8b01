"""ctypes binding of libptycho.so (argument marshalling only).

The functions here carry the names of the C entry points declared in
include/ptycho.h and take torch tensors that already live on the GPU; every
step of the model, loss and gradient runs in the library's HIP kernels.
PyTorch only supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptycho.so")

MAX_WAVELENGTHS = 8
MAX_MODES = 16

PTYCHO_OK = 0
PTYCHO_EINVAL = -1
PTYCHO_ERANGE = -2
PTYCHO_EUNSUPPORTED = -3
PTYCHO_ENOSPC = -4
PTYCHO_EHIP = -5

LOSS_AMPLITUDE = 0
LOSS_POISSON = 1
LOSS_GAUSSIAN = 2
LOSS_VJP = 3
LOSS_MIXED = 4

_c_i32 = ctypes.c_int32
_c_p = ctypes.c_void_p


class JobT(ctypes.Structure):
    _fields_ = [("K", _c_i32), ("L", _c_i32), ("M", _c_i32), ("N", _c_i32), ("H", _c_i32),
                ("W", _c_i32), ("pad", _c_i32 * MAX_WAVELENGTHS),
                ("ratio", ctypes.c_double * MAX_WAVELENGTHS),
                ("object", _c_p), ("probe", _c_p), ("pos", _c_p), ("sigma", _c_p),
                ("background", _c_p), ("mask", _c_p), ("rs_idx", _c_p), ("rs_w", _c_p),
                ("rsT_ptr", _c_p), ("rsT_col", _c_p), ("rsT_val", _c_p), ("measured", _c_p),
                ("Ns", _c_i32)]


class LossT(ctypes.Structure):
    _fields_ = [("kind", _c_i32), ("eps", ctypes.c_float), ("scale", ctypes.c_float),
                ("noise_var", ctypes.c_float), ("l1", ctypes.c_float), ("tv", ctypes.c_float),
                ("tv_eps", ctypes.c_float)]


def _loss(kind, eps, scale, noise_var=1.0, l1=0.0, tv=0.0, tv_eps=1e-3) -> LossT:
    return LossT(int(kind), float(eps), float(scale), float(noise_var), float(l1), float(tv),
                 float(tv_eps))


class GradsT(ctypes.Structure):
    _fields_ = [("loss", _c_p), ("g_object", _c_p), ("g_probe", _c_p), ("g_pos", _c_p),
                ("g_sigma", _c_p), ("g_background", _c_p), ("g_ratio", _c_p)]


class AdamT(ctypes.Structure):
    _fields_ = [("m_object", _c_p), ("v_object", _c_p), ("m_probe", _c_p), ("v_probe", _c_p),
                ("m_pos", _c_p), ("v_pos", _c_p), ("lr_object", ctypes.c_float),
                ("lr_probe", ctypes.c_float), ("lr_pos", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("t", _c_i32), ("m_sigma", _c_p), ("v_sigma", _c_p), ("m_background", _c_p),
                ("v_background", _c_p), ("lr_sigma", ctypes.c_float),
                ("lr_background", ctypes.c_float)]


class PtychoError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {error_string(code)} ({code})")


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2311_14780_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.ptycho_supported.argtypes = [_c_i32, _c_i32]
        L.ptycho_supported.restype = _c_i32
        L.ptycho_workspace_bytes.argtypes = [ctypes.POINTER(JobT), _c_i32, _c_i32, _c_i32,
                                             ctypes.POINTER(ctypes.c_size_t)]
        L.ptycho_workspace_bytes.restype = _c_i32
        L.ptycho_forward.argtypes = [ctypes.POINTER(JobT), _c_i32, ctypes.POINTER(_c_p), _c_p,
                                     ctypes.c_size_t, _c_p]
        L.ptycho_forward.restype = _c_i32
        L.ptycho_loss_grad.argtypes = [ctypes.POINTER(JobT), _c_i32, ctypes.POINTER(LossT),
                                       ctypes.POINTER(GradsT), _c_p, ctypes.c_size_t, _c_p]
        L.ptycho_loss_grad.restype = _c_i32
        L.ptycho_loss_grad_noalloc.argtypes = [ctypes.POINTER(JobT), _c_i32,
                                               ctypes.POINTER(LossT), ctypes.POINTER(GradsT),
                                               _c_p]
        L.ptycho_loss_grad_noalloc.restype = _c_i32
        L.ptycho_step.argtypes = [ctypes.POINTER(JobT), _c_i32, ctypes.POINTER(LossT),
                                  ctypes.POINTER(GradsT), ctypes.POINTER(AdamT), _c_p,
                                  ctypes.c_size_t, _c_p]
        L.ptycho_step.restype = _c_i32
        L.ptycho_status.argtypes = [_c_p, _c_i32, _c_p]
        L.ptycho_status.restype = _c_i32
        L.ptycho_transpose_table.argtypes = [_c_p, _c_p, _c_i32, _c_i32, _c_p, _c_p, _c_p]
        L.ptycho_transpose_table.restype = _c_i32
        L.ptycho_error_string.argtypes = [_c_i32]
        L.ptycho_error_string.restype = ctypes.c_char_p
        L.ptycho_release.argtypes = []
        L.ptycho_release.restype = None
        L.ptycho_profile.argtypes = [_c_i32]
        L.ptycho_profile.restype = _c_i32
        L.ptycho_profile_read.argtypes = [_c_i32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64)]
        L.ptycho_profile_read.restype = _c_i32
        L.ptycho_profile_classes.argtypes = [ctypes.c_uint32]
        L.ptycho_profile_classes.restype = _c_i32
        L.ptycho_kernel_class_name.argtypes = [_c_i32]
        L.ptycho_kernel_class_name.restype = ctypes.c_char_p
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().ptycho_error_string(int(code)).decode()


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check(t, name: str, dtype, shape=None, device=None, numel=None, where=True) -> None:
    """Raises ValueError unless ``t`` (if not None) is a contiguous GPU tensor
    of this dtype and shape (or element count) on ``device``.  The C ABI
    receives bare device pointers and cannot know buffer sizes, so a wrong
    shape would become an out-of-bounds device access; this is where it is
    caught.  dtype and shape are checked before the device, so the checks
    also run on tensors that were never moved to a GPU."""
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if numel is not None and t.numel() != int(numel):
        raise ValueError(f"{name}: {t.numel()} elements, expected {int(numel)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensors passed to the library must be contiguous")
    if not where:
        return
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU (device) tensor, got {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name}: on {t.device}, the job's object is on {device}")


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class Problem:
    """Device tensors of one reconstruction job (the variables of Eq. 1).

    object complex64 [L][H][W] or [L][Ns][H][W] (Ns sample modes);
    probe complex64 [L][M][N][N]; pos float32
    [K][2]; pads: per wavelength, an int (zero-padded DFT size) or a float
    (exact sampling ratio alpha of the exact-ratio propagator); measured
    float32 [K][N][N];
    sigma float32 [K]; background float32 [N][N]; mask uint8 [N][N];
    resample: (idx int32 [N*N][4], w float32 [N*N][4], ptr, col, val) on
    the device, see ``resample_tables``.
    """
    object: torch.Tensor
    probe: torch.Tensor
    pos: torch.Tensor
    pads: Sequence[int]
    measured: Optional[torch.Tensor] = None
    sigma: Optional[torch.Tensor] = None
    background: Optional[torch.Tensor] = None
    mask: Optional[torch.Tensor] = None
    resample: Optional[tuple] = None

    @property
    def K(self):
        return int(self.pos.shape[0])

    @property
    def L(self):
        return int(self.probe.shape[0])

    @property
    def M(self):
        return int(self.probe.shape[1])

    @property
    def N(self):
        return int(self.probe.shape[-1])

    @property
    def Ns(self):
        return int(self.object.shape[1]) if self.object.dim() == 4 else 1

    def validate(self) -> None:
        """Dtype, shape and device of every tensor against the sizes the
        probe and the positions define (raises ValueError)."""
        if not isinstance(self.probe, torch.Tensor) or self.probe.dim() != 4 or \
                self.probe.shape[-1] != self.probe.shape[-2]:
            raise ValueError("probe: expected complex64 [L][M][N][N]")
        if not isinstance(self.pos, torch.Tensor) or self.pos.dim() != 2:
            raise ValueError("pos: expected float32 [K][2]")
        if not isinstance(self.object, torch.Tensor) or self.object.dim() not in (3, 4):
            raise ValueError("object: expected complex64 [L][H][W] or [L][Ns][H][W]")
        K, L, M, N = self.K, self.L, self.M, self.N
        dev = self.object.device
        H, W = int(self.object.shape[-2]), int(self.object.shape[-1])
        checks = [(self.object, "object", torch.complex64,
                   (L, H, W) if self.object.dim() == 3 else (L, self.Ns, H, W)),
                  (self.probe, "probe", torch.complex64, (L, M, N, N)),
                  (self.pos, "pos", torch.float32, (K, 2)),
                  (self.measured, "measured", torch.float32, (K, N, N)),
                  (self.sigma, "sigma", torch.float32, (K,)),
                  (self.background, "background", torch.float32, (N, N)),
                  (self.mask, "mask", torch.uint8, (N, N))]
        if self.resample is not None:
            if len(self.resample) != 5:
                raise ValueError("resample: expected (idx, w, ptr, col, val)")
            idx, w, ptr, col, val = self.resample
            n = N * N
            checks += [(idx, "resample idx", torch.int32, (n, 4)),
                       (w, "resample w", torch.float32, (n, 4)),
                       (ptr, "resample ptr", torch.int32, (n + 1,)),
                       (col, "resample col", torch.int32, (4 * n,)),
                       (val, "resample val", torch.float32, (4 * n,))]
        if len(self.pads) != L:
            raise ValueError("one pad per wavelength is required")
        for t, name, dt, shape in checks:  # dtype and shape of everything first
            _check(t, name, dt, shape, where=False)
        for t, name, dt, shape in checks:
            _check(t, name, dt, shape, device=dev)

    def to_job(self) -> JobT:
        self.validate()
        j = JobT()
        j.K, j.L, j.M, j.N = self.K, self.L, self.M, self.N
        j.H, j.W = int(self.object.shape[-2]), int(self.object.shape[-1])
        j.Ns = self.Ns
        if len(self.pads) != self.L:
            raise ValueError("one pad per wavelength is required")
        _set_pads(j, self.pads)
        j.object = _ptr(self.object)
        j.probe = _ptr(self.probe)
        j.pos = _ptr(self.pos)
        j.sigma = _ptr(self.sigma)
        j.background = _ptr(self.background)
        j.mask = _ptr(self.mask)
        if self.resample is not None:
            idx, w, ptr, col, val = self.resample
            j.rs_idx, j.rs_w = _ptr(idx), _ptr(w)
            j.rsT_ptr, j.rsT_col, j.rsT_val = _ptr(ptr), _ptr(col), _ptr(val)
        j.measured = _ptr(self.measured)
        return j


def _set_pads(j: JobT, pads) -> None:
    """Integers are zero-padded DFT sizes, floats exact sampling ratios."""
    for l, p in enumerate(pads):
        if isinstance(p, (float, np.floating)):
            j.pad[l], j.ratio[l] = 0, float(p)
        else:
            j.pad[l], j.ratio[l] = int(p), 0.0


def _jobs(problems: Sequence[Problem]):
    arr = (JobT * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = p.to_job()
    return arr


def ptycho_supported(N: int, pad: int) -> bool:
    return bool(lib().ptycho_supported(int(N), int(pad)))


def ptycho_workspace_bytes(problems: Sequence[Problem], which: int = 1, chunk: int = 0) -> int:
    out = ctypes.c_size_t(0)
    code = lib().ptycho_workspace_bytes(_jobs(problems), len(problems), int(which), int(chunk),
                                        ctypes.byref(out))
    if code:
        raise PtychoError(code, "ptycho_workspace_bytes")
    return int(out.value)


def workspace_bytes_for_shapes(shapes: Sequence[tuple], which: int = 1, chunk: int = 0) -> int:
    """Workspace bytes for jobs given only by their sizes
    (K, L, M, N, H, W, pads), without resampling tables."""
    arr = (JobT * len(shapes))()
    for i, (K, L, M, N, H, W, pads) in enumerate(shapes):
        arr[i].K, arr[i].L, arr[i].M, arr[i].N, arr[i].H, arr[i].W = K, L, M, N, H, W
        _set_pads(arr[i], pads)
    out = ctypes.c_size_t(0)
    code = lib().ptycho_workspace_bytes(arr, len(shapes), int(which), int(chunk), ctypes.byref(out))
    if code:
        raise PtychoError(code, "ptycho_workspace_bytes")
    return int(out.value)


def _check_workspace(workspace, problems) -> None:
    if workspace is None:
        raise ValueError("a workspace tensor is required")
    _check(workspace, "workspace", workspace.dtype if isinstance(workspace, torch.Tensor) else None,
           device=problems[0].object.device)


def ptycho_forward(problems: Sequence[Problem], intensities: Sequence[torch.Tensor],
                   workspace: torch.Tensor, stream=None) -> None:
    if len(intensities) != len(problems):
        raise ValueError("one intensity tensor per job is required")
    for p, t in zip(problems, intensities):
        _check(t, "intensity", torch.float32, (p.K, p.N, p.N), p.object.device)
    _check_workspace(workspace, problems)
    outs = (_c_p * len(problems))(*[t.data_ptr() for t in intensities])
    code = lib().ptycho_forward(_jobs(problems), len(problems), outs, _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream))
    if code:
        raise PtychoError(code, "ptycho_forward")


_GRAD_KEYS = ("loss", "g_object", "g_probe", "g_pos", "g_sigma", "g_background", "g_ratio")


def _check_grads(problems: Sequence[Problem], grads: Sequence[dict]) -> None:
    if len(grads) != len(problems):
        raise ValueError("one gradient dict per job is required")
    for p, g in zip(problems, grads):
        unknown = set(g) - set(_GRAD_KEYS)
        if unknown:
            raise ValueError(f"unknown gradient outputs {sorted(unknown)}")
        dev = p.object.device
        _check(g.get("loss"), "loss", torch.float32, (1,), dev)
        _check(g.get("g_object"), "g_object", torch.complex64, tuple(p.object.shape), dev)
        _check(g.get("g_probe"), "g_probe", torch.complex64, tuple(p.probe.shape), dev)
        _check(g.get("g_pos"), "g_pos", torch.float32, (p.K, 2), dev)
        _check(g.get("g_sigma"), "g_sigma", torch.float32, (p.K,), dev)
        _check(g.get("g_background"), "g_background", torch.float32, (p.N, p.N), dev)
        _check(g.get("g_ratio"), "g_ratio", torch.float32, (p.L,), dev)


def _grads_array(grads: Sequence[dict]):
    arr = (GradsT * len(grads))()
    for i, g in enumerate(grads):
        arr[i].loss = _ptr(g.get("loss"))
        arr[i].g_object = _ptr(g.get("g_object"))
        arr[i].g_probe = _ptr(g.get("g_probe"))
        arr[i].g_pos = _ptr(g.get("g_pos"))
        arr[i].g_sigma = _ptr(g.get("g_sigma"))
        arr[i].g_background = _ptr(g.get("g_background"))
        arr[i].g_ratio = _ptr(g.get("g_ratio"))
    return arr


def ptycho_loss_grad(problems: Sequence[Problem], grads: Sequence[dict], kind: int = 0,
                     eps: float = 1e-6, scale: float = 1.0, workspace: torch.Tensor = None,
                     stream=None, **reg) -> None:
    """``reg``: noise_var (mixed-noise loss), l1, tv, tv_eps (regularisers)."""
    loss = _loss(kind, eps, scale, **reg)
    jobs = _jobs(problems)
    _check_grads(problems, grads)
    _check_workspace(workspace, problems)
    code = lib().ptycho_loss_grad(jobs, len(problems), ctypes.byref(loss),
                                  _grads_array(grads), _ptr(workspace),
                                  workspace.numel() * workspace.element_size(), _stream(stream))
    if code:
        raise PtychoError(code, "ptycho_loss_grad")


NOALLOC_SCRATCH_BYTES = 64 << 20  # PTYCHO_NOALLOC_SCRATCH_BYTES


def ptycho_loss_grad_noalloc(problems: Sequence[Problem], grads: Sequence[dict], kind: int = 0,
                             eps: float = 1e-6, scale: float = 1.0, stream=None, **reg) -> None:
    """ptycho_loss_grad on the library's static scratch (no workspace, no
    device allocation); calls on one GPU must not overlap."""
    loss = _loss(kind, eps, scale, **reg)
    jobs = _jobs(problems)
    _check_grads(problems, grads)
    code = lib().ptycho_loss_grad_noalloc(jobs, len(problems), ctypes.byref(loss),
                                          _grads_array(grads), _stream(stream))
    if code:
        raise PtychoError(code, "ptycho_loss_grad_noalloc")


def ptycho_step(problems: Sequence[Problem], grads: Sequence[dict], adam: Sequence[dict],
                kind: int = 0, eps: float = 1e-6, scale: float = 1.0,
                workspace: torch.Tensor = None, stream=None, **reg) -> None:
    loss = _loss(kind, eps, scale, **reg)
    jobs = _jobs(problems)
    _check_grads(problems, grads)
    _check_workspace(workspace, problems)
    if len(adam) != len(problems):
        raise ValueError("one Adam dict per job is required")
    for p, a in zip(problems, adam):
        dev = p.object.device
        for var, t in (("object", p.object), ("probe", p.probe), ("pos", p.pos),
                       ("sigma", p.sigma), ("background", p.background)):
            n = 0 if t is None else t.numel() * (2 if t.is_complex() else 1)
            for mv in ("m_", "v_"):
                _check(a.get(mv + var), mv + var, torch.float32, device=dev, numel=n)
    arr = (AdamT * len(adam))()
    for i, a in enumerate(adam):
        arr[i].m_object, arr[i].v_object = _ptr(a.get("m_object")), _ptr(a.get("v_object"))
        arr[i].m_probe, arr[i].v_probe = _ptr(a.get("m_probe")), _ptr(a.get("v_probe"))
        arr[i].m_pos, arr[i].v_pos = _ptr(a.get("m_pos")), _ptr(a.get("v_pos"))
        arr[i].m_sigma, arr[i].v_sigma = _ptr(a.get("m_sigma")), _ptr(a.get("v_sigma"))
        arr[i].m_background = _ptr(a.get("m_background"))
        arr[i].v_background = _ptr(a.get("v_background"))
        arr[i].lr_object = float(a.get("lr_object", 0.0))
        arr[i].lr_probe = float(a.get("lr_probe", 0.0))
        arr[i].lr_pos = float(a.get("lr_pos", 0.0))
        arr[i].lr_sigma = float(a.get("lr_sigma", 0.0))
        arr[i].lr_background = float(a.get("lr_background", 0.0))
        arr[i].beta1 = float(a.get("beta1", 0.9))
        arr[i].beta2 = float(a.get("beta2", 0.999))
        arr[i].eps = float(a.get("eps", 1e-8))
        arr[i].t = int(a["t"])
    code = lib().ptycho_step(jobs, len(problems), ctypes.byref(loss),
                             _grads_array(grads), arr, _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream(stream))
    if code:
        raise PtychoError(code, "ptycho_step")


def ptycho_status(workspace: torch.Tensor, job: int = 0, stream=None) -> int:
    return int(lib().ptycho_status(_ptr(workspace), int(job), _stream(stream)))


def ptycho_transpose_table(idx, w, n_in: int):
    """CSR transpose of a host resampling table (numpy int32/float32 [n_out][4])."""
    import numpy as np
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    n_out = idx.shape[0]
    ptr = np.zeros(n_in + 1, np.int32)
    col = np.zeros(4 * n_out, np.int32)
    val = np.zeros(4 * n_out, np.float32)
    code = lib().ptycho_transpose_table(idx.ctypes.data, w.ctypes.data, n_out, n_in,
                                        ptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    if code:
        raise PtychoError(code, "ptycho_transpose_table")
    return ptr, col, val


def ptycho_release() -> None:
    lib().ptycho_release()


def ptycho_profile(enable: bool) -> None:
    code = lib().ptycho_profile(1 if enable else 0)
    if code:
        raise PtychoError(code, "ptycho_profile")


def ptycho_profile_classes(names) -> None:
    """Brackets only the named kernel classes (None: all) while profiling."""
    mask = 0xFFFFFFFF
    if names is not None:
        index = {}
        i = 0
        while True:
            n = lib().ptycho_kernel_class_name(i)
            if n is None:
                break
            index[n.decode()] = i
            i += 1
        mask = 0
        for n in names:
            mask |= 1 << index[n]
    code = lib().ptycho_profile_classes(mask)
    if code:
        raise PtychoError(code, "ptycho_profile_classes")


def ptycho_profile_read() -> dict:
    """{kernel class name: (total ms, launches)} since ptycho_profile(True)."""
    out = {}
    i = 0
    while True:
        name = lib().ptycho_kernel_class_name(i)
        if name is None:
            break
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        code = lib().ptycho_profile_read(i, ctypes.byref(ms), ctypes.byref(n))
        if code:
            raise PtychoError(code, "ptycho_profile_read")
        out[name.decode()] = (ms.value, n.value)
        i += 1
    return out


def resample_tables(idx, w, device) -> tuple:
    """Device copies of a resampling table and of its CSR transpose."""
    import numpy as np
    n = idx.shape[0]
    ptr, col, val = ptycho_transpose_table(idx, w, n)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return (to(np.asarray(idx, np.int32)), to(np.asarray(w, np.float32)), to(ptr), to(col), to(val))


def workspace(problems: Sequence[Problem], which: int = 1, chunk: int = 0,
              device=None) -> torch.Tensor:
    nbytes = ptycho_workspace_bytes(problems, which, chunk)
    dev = device if device is not None else problems[0].object.device
    return torch.empty(nbytes, dtype=torch.uint8, device=dev)
