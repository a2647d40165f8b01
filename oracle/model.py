"""Plain FP64 forward model, loss and gradient (test infrastructure only).

Notation follows Eq. 1: scan index k, wavelength l (L of them), illumination
mode m (M), sample mode n (Ns), probe P_{l,m}(r), object O_{l,n}(r), scan
position s_k, power coefficient sigma_k, background N(rho), measurement
operator M[.].  Eq. 2 splits the model into f1 (probe power scaling by
sigma_k), f2 (object shift by s_k), f3 (probe-object product), f4 (propagator
D_{lambda,z}) and f5 (measurement effects and background); the functions
below follow that order.

Readings of points the paper leaves open (each one is also listed in the
design notes):
* s_k is the top-left corner of the probe window in object pixels and the
  shifted object is O(r + s_k); p_k = floor(s_k + 1/2) (taken in float32, as
  the positions are float32), delta_k = s_k - p_k in [-1/2, 1/2).
* f2 (Fourier shift theorem): the gathered N x N patch A = O[p + r] is
  shifted by the circular Fourier shift
  ifft2(fft2(A) * exp(+2 pi i (f_y delta_y + f_x delta_x))), with
  f = numpy.fft.fftfreq(N) (the Nyquist bin is -1/2).
* f4 at wavelength lambda_l: the exit wave sits at [0, N)^2 of an
  N_l x N_l zero array, a unitary 2D DFT is taken and the N x N bins with
  frequencies u in [-N/2, N/2) are kept, DC at index (N/2, N/2).  N_l is an
  input (the per-wavelength detector sampling).
* f4 with an exact sampling ratio (the chirp z-transform propagator of the
  section "Benchmarking with state-of-art open-source ptychography
  algorithm"): when N_l is given as a float alpha (alpha = N lambda_l /
  lambda_min, generally not an integer), the propagator is the scaled DFT
  Psi[u, v] = alpha^-1 sum_{r, s} psi[r, s] exp(-2 pi i (u r + v s) / alpha)
  over the same output bins u, v in [-N/2, N/2).  For an integer alpha this
  is exactly the zero-padded DFT above; the chirp z-transform is one way to
  evaluate it, the oracle evaluates the sum as written.
* sigma_k multiplies the field, as written in Eq. 1.
* f5: I' = R(I + B) with R an optional bilinear resampling table (tilted
  plane) and B the additive background; the binary mask weights the loss.
* Losses (sum over positions and pixels, times ``scale``), eps inside:
  amplitude (MSE on the modulus): (sqrt(I'+eps) - sqrt(Î+eps))^2;
  Poisson: (I'+eps) - (Î+eps) ln(I'+eps);
  Gaussian: (I' - Î)^2;
  VJP: u * I' with u = ``measured`` an upstream gradient (mask ignored);
  mixed Poisson-Gaussian noise (the paper's MLE with mixed noise
  statistics), Gaussian approximation with variance I' + v (v the read-noise
  variance): (I' - Î)^2 / (I' + v) + ln(I' + v).
* Regularisers on the object amplitude a = |O| (the paper applies L1 and TV
  to the amplitude): R = l1 sum a + tv sum sqrt(dy^2 + dx^2 + delta^2), with
  forward differences dy = a[y+1, x] - a[y, x], dx = a[y, x+1] - a[y, x]
  (zero past the last row / column), summed over every wavelength and sample
  mode; R is added to the loss unscaled.
* Gradients use the convention G = dL/dRe + i dL/dIm.
"""
from __future__ import annotations

import numpy as np

LOSS_AMPLITUDE = 0
LOSS_POISSON = 1
LOSS_GAUSSIAN = 2
LOSS_VJP = 3
LOSS_MIXED = 4


# ----------------------------------------------------------------- f2: shift
def split_positions(pos):
    """Integer window corner p (int64) and sub-pixel remainder delta (float64).

    The rounding is taken in float32 because the positions are float32 and
    the GPU path takes the same decision in float32.
    """
    s32 = np.asarray(pos, dtype=np.float32)
    p = np.floor(s32 + np.float32(0.5)).astype(np.int64)
    delta = s32.astype(np.float64) - p.astype(np.float64)
    return p, delta


def _ramp(N: int, delta) -> np.ndarray:
    f = np.fft.fftfreq(N)
    ry = np.exp(2j * np.pi * f * delta[0])
    rx = np.exp(2j * np.pi * f * delta[1])
    return ry[:, None] * rx[None, :]


def shift_patch(A: np.ndarray, delta) -> np.ndarray:
    """Fourier-shift theorem: result(r) = A(r + delta) (circular)."""
    return np.fft.ifft2(np.fft.fft2(A) * _ramp(A.shape[-1], delta))


def shift_patch_adjoint(G: np.ndarray, delta) -> np.ndarray:
    """Adjoint (= inverse, the shift is unitary) of ``shift_patch``."""
    return np.fft.ifft2(np.fft.fft2(G) * np.conj(_ramp(G.shape[-1], delta)))


# ------------------------------------------------------------ f4: propagator
def _crop_index(N: int, nl: int) -> np.ndarray:
    return (np.arange(N) - N // 2) % nl


def is_ratio(nl) -> bool:
    """A float N_l is an exact sampling ratio (scaled DFT); an integer is a
    zero-padded DFT size."""
    return isinstance(nl, (float, np.floating))


def scaled_dft_matrix(N: int, alpha: float) -> np.ndarray:
    """F[j, r] = exp(-2 pi i u_j r / alpha) / sqrt(alpha), u_j = j - N/2:
    one axis of the exact-ratio propagator (rows are output bins)."""
    u = np.arange(N, dtype=np.float64) - N // 2
    r = np.arange(N, dtype=np.float64)
    return np.exp(-2j * np.pi * np.outer(u, r) / alpha) / np.sqrt(alpha)


def propagate(psi: np.ndarray, nl) -> np.ndarray:
    """Zero-pad the N x N exit wave to nl x nl, unitary DFT, keep N x N bins;
    for a float ``nl`` (exact ratio alpha) the scaled DFT F psi F^T."""
    N = psi.shape[-1]
    if is_ratio(nl):
        if not nl >= N:
            raise ValueError("sampling ratio smaller than the window")
        F = scaled_dft_matrix(N, float(nl))
        return F @ psi @ F.T
    if nl < N:
        raise ValueError("pad smaller than the window")
    z = np.zeros((nl, nl), dtype=np.complex128)
    z[:N, :N] = psi
    F = np.fft.fft2(z, norm="ortho")
    idx = _crop_index(N, nl)
    return F[np.ix_(idx, idx)]


def scaled_dft_matrix_dalpha(N: int, alpha: float) -> np.ndarray:
    """d/d alpha of ``scaled_dft_matrix``: F[j, r] (-1/(2 alpha) + 2 pi i u_j r / alpha^2)."""
    u = np.arange(N, dtype=np.float64) - N // 2
    r = np.arange(N, dtype=np.float64)
    E = -0.5 / alpha + 2j * np.pi * np.outer(u, r) / alpha ** 2
    return scaled_dft_matrix(N, alpha) * E


def propagate_dalpha(psi: np.ndarray, alpha: float) -> np.ndarray:
    """d Psi / d alpha of the exact-ratio propagator (product rule on F psi F^T)."""
    N = psi.shape[-1]
    F = scaled_dft_matrix(N, float(alpha))
    dF = scaled_dft_matrix_dalpha(N, float(alpha))
    return dF @ psi @ F.T + F @ psi @ dF.T


def propagate_adjoint(G: np.ndarray, nl) -> np.ndarray:
    """Adjoint of ``propagate``: embed the bins, unitary inverse DFT, crop;
    for a float ``nl``, F^H G conj(F)."""
    N = G.shape[-1]
    if is_ratio(nl):
        F = scaled_dft_matrix(N, float(nl))
        return F.conj().T @ G @ F.conj()
    z = np.zeros((nl, nl), dtype=np.complex128)
    idx = _crop_index(N, nl)
    z[np.ix_(idx, idx)] = G
    return np.fft.ifft2(z, norm="ortho")[:N, :N]


# ------------------------------------------------------- f5: measurement side
def resample(I: np.ndarray, idx: np.ndarray, w: np.ndarray) -> np.ndarray:
    """I'(a) = sum_t w[a,t] I(idx[a,t]) on a flattened N x N grid."""
    N = I.shape[-1]
    flat = I.reshape(N * N)
    out = (np.asarray(w, np.float64) * flat[np.asarray(idx)]).sum(axis=1)
    return out.reshape(N, N)


def resample_adjoint(g: np.ndarray, idx: np.ndarray, w: np.ndarray) -> np.ndarray:
    N = g.shape[-1]
    out = np.zeros(N * N, dtype=np.float64)
    np.add.at(out, np.asarray(idx).ravel(),
              (np.asarray(w, np.float64) * g.reshape(N * N, 1)).ravel())
    return out.reshape(N, N)


def pointwise_loss(I: np.ndarray, meas: np.ndarray, kind: int, eps: float, noise_var: float = 1.0):
    """Per-pixel loss and its derivative with respect to the prediction I."""
    I = np.asarray(I, np.float64)
    meas = np.asarray(meas, np.float64)
    if kind == LOSS_MIXED:
        q = I + noise_var
        d = I - meas
        return d * d / q + np.log(q), 2.0 * d / q - (d / q) ** 2 + 1.0 / q
    if kind == LOSS_AMPLITUDE:
        a = np.sqrt(I + eps)
        b = np.sqrt(meas + eps)
        return (a - b) ** 2, 1.0 - b / a
    if kind == LOSS_POISSON:
        return (I + eps) - (meas + eps) * np.log(I + eps), 1.0 - (meas + eps) / (I + eps)
    if kind == LOSS_GAUSSIAN:
        return (I - meas) ** 2, 2.0 * (I - meas)
    if kind == LOSS_VJP:
        return meas * I, meas.copy()
    raise ValueError(f"unknown loss kind {kind}")


# ------------------------------------------------------------ regularisers
def regulariser(obj, l1: float, tv: float, tv_eps: float):
    """Value and gradient (G = dR/dRe + i dR/dIm) of the amplitude L1 and
    smoothed isotropic TV terms, for an object [..., H, W]."""
    O = np.asarray(obj, np.complex128)
    a = np.abs(O)
    dy = np.zeros_like(a)
    dx = np.zeros_like(a)
    dy[..., :-1, :] = a[..., 1:, :] - a[..., :-1, :]
    dx[..., :, :-1] = a[..., :, 1:] - a[..., :, :-1]
    t = np.sqrt(dy * dy + dx * dx + tv_eps * tv_eps)
    value = l1 * float(np.sum(a)) + tv * float(np.sum(t))
    # dR/da: own term -(dy + dx)/t, plus the terms of the pixels above and left
    ga = np.full_like(a, l1) - tv * (dy + dx) / t
    ga[..., 1:, :] += tv * (dy / t)[..., :-1, :]
    ga[..., :, 1:] += tv * (dx / t)[..., :, :-1]
    phase = np.where(a > 0, O / np.where(a > 0, a, 1.0), 0.0)
    return value, ga * phase


# ------------------------------------------------------------- shape helpers
def _as_object(obj):
    obj = np.asarray(obj, dtype=np.complex128)
    if obj.ndim == 3:
        return obj[:, None], True
    return obj, False


def _window(obj_ln, p, N):
    py, px = int(p[0]), int(p[1])
    H, W = obj_ln.shape
    if py < 0 or px < 0 or py + N > H or px + N > W:
        raise ValueError("probe window outside the object")
    return obj_ln[py:py + N, px:px + N]


# ---------------------------------------------------------------- Eq. 1 / 2
def _exit_waves(obj, probe, pk, dk, sig, pads):
    """Per wavelength l and sample mode n: patch A, its FFT, shifted patch,
    and the detector fields Psi[l][n][m] of f4(f3(f1(sigma_k), f2(s_k)))."""
    L, Ns = obj.shape[:2]
    M, N = probe.shape[1], probe.shape[-1]
    A, Ahat, Osh, Psi = {}, {}, {}, {}
    for l in range(L):
        for n in range(Ns):
            a = _window(obj[l, n], pk, N)
            A[l, n] = a
            Ahat[l, n] = np.fft.fft2(a)
            Osh[l, n] = np.fft.ifft2(Ahat[l, n] * _ramp(N, dk))
            for m in range(M):
                psi = sig * probe[l, m] * Osh[l, n]
                Psi[l, n, m] = propagate(psi, pads[l])
    return A, Ahat, Osh, Psi


def forward(obj, probe, pos, pads, sigma=None, background=None, resample_table=None):
    """Predicted patterns I'_k, float64 [K][N][N] (Eq. 1)."""
    obj, _ = _as_object(obj)
    probe = np.asarray(probe, dtype=np.complex128)
    L, Ns = obj.shape[:2]
    M, N = probe.shape[1], probe.shape[-1]
    p, d = split_positions(pos)
    K = p.shape[0]
    out = np.empty((K, N, N), dtype=np.float64)
    for k in range(K):
        sig = 1.0 if sigma is None else float(sigma[k])
        _, _, _, Psi = _exit_waves(obj, probe, p[k], d[k], sig, pads)
        I = np.zeros((N, N))
        for key in Psi:
            I += np.abs(Psi[key]) ** 2
        if background is not None:
            I = I + np.asarray(background, np.float64)
        if resample_table is not None:
            I = resample(I, *resample_table)
        out[k] = I
    return out


def loss_grad(obj, probe, pos, pads, measured, kind=LOSS_AMPLITUDE, eps=1e-6,
              scale=1.0, sigma=None, background=None, mask=None,
              resample_table=None, positions=None, noise_var=1.0, l1=0.0, tv=0.0,
              tv_eps=1e-3):
    """Loss and gradients w.r.t. object, probe, positions and sigma.

    ``positions`` restricts the sums over k to a subset (the loss is a sum of
    per-position terms, so the full gradient is the sum over a partition);
    the regulariser (l1, tv) belongs to no position and is added only when
    ``positions`` is None.
    Returns a dict: loss (float), g_object (shape of ``obj``), g_probe
    [L][M][N][N], g_pos [K][2], g_sigma [K] (zero outside the subset),
    g_background [N][N] (the background enters f5 before the resampling, so
    its gradient is the sum over positions of the pulled-back dL/dI'),
    g_ratio [L] (dL/d alpha_l for exact-ratio wavelengths, 0 for zero-padded
    ones; alpha_l is proportional to the propagation distance z, so
    dL/dz = sum_l alpha_l / z * dL/d alpha_l).
    """
    obj, squeeze = _as_object(obj)
    probe = np.asarray(probe, dtype=np.complex128)
    L, Ns = obj.shape[:2]
    M, N = probe.shape[1], probe.shape[-1]
    p, d = split_positions(pos)
    K = p.shape[0]
    f = np.fft.fftfreq(N)
    w = np.ones((N, N)) if (mask is None or kind == LOSS_VJP) else np.asarray(mask, np.float64)
    g_obj = np.zeros_like(obj)
    g_prb = np.zeros_like(probe)
    g_pos = np.zeros((K, 2))
    g_sig = np.zeros(K)
    g_bg = np.zeros((N, N))
    g_ratio = np.zeros(L)
    total = 0.0
    ks = range(K) if positions is None else positions
    for k in ks:
        sig = 1.0 if sigma is None else float(sigma[k])
        A, Ahat, Osh, Psi = _exit_waves(obj, probe, p[k], d[k], sig, pads)
        I = np.zeros((N, N))
        for key in Psi:
            I += np.abs(Psi[key]) ** 2
        if background is not None:
            I = I + np.asarray(background, np.float64)
        Ip = resample(I, *resample_table) if resample_table is not None else I
        ell, dell = pointwise_loss(Ip, measured[k], kind, eps, noise_var)
        total += float(np.sum(w * ell))
        # dL/dI, pulled back through the resampling
        g = w * dell
        if resample_table is not None:
            g = resample_adjoint(g, *resample_table)
        g_bg += g
        ramp = _ramp(N, d[k])
        for l in range(L):
            for n in range(Ns):
                G_osh = np.zeros((N, N), dtype=np.complex128)
                for m in range(M):
                    # |Psi|^2 -> Psi: G_Psi = 2 g Psi; f4 adjoint
                    chi = propagate_adjoint(2.0 * g * Psi[l, n, m], pads[l])
                    if is_ratio(pads[l]):
                        # dL/d alpha_l = Re <G_Psi, dPsi/d alpha>
                        dpsi = propagate_dalpha(sig * probe[l, m] * Osh[l, n], pads[l])
                        g_ratio[l] += float(np.real(np.vdot(2.0 * g * Psi[l, n, m], dpsi)))
                    g_prb[l, m] += np.conj(sig * Osh[l, n]) * chi
                    G_osh += np.conj(sig * probe[l, m]) * chi
                    g_sig[k] += float(np.real(np.sum(np.conj(chi) * probe[l, m] * Osh[l, n])))
                # f2 adjoint and the position derivative at fixed p
                Ghat = np.fft.fft2(G_osh)
                G_A = np.fft.ifft2(Ghat * np.conj(ramp))
                py, px = int(p[k, 0]), int(p[k, 1])
                g_obj[l, n, py:py + N, px:px + N] += G_A
                core = np.conj(Ghat) * ramp * Ahat[l, n] * (2j * np.pi)
                g_pos[k, 0] += float(np.real(np.sum(core * f[:, None]))) / (N * N)
                g_pos[k, 1] += float(np.real(np.sum(core * f[None, :]))) / (N * N)
    g_obj *= scale
    g_prb *= scale
    g_pos *= scale
    g_sig *= scale
    g_bg *= scale
    g_ratio *= scale
    total *= scale
    if (l1 or tv) and positions is None:
        rv, rg = regulariser(obj, l1, tv, tv_eps)
        total += rv
        g_obj += rg
    return dict(loss=total, g_object=g_obj[:, 0] if squeeze else g_obj,
                g_probe=g_prb, g_pos=g_pos, g_sigma=g_sig, g_background=g_bg,
                g_ratio=g_ratio)


# -------------------------------------------------------------------- Adam
def adam_step(x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (the optimiser the paper uses, Section "Universal
    Ptychography Algorithm based on Automatic Differentiation"), elementwise
    on real coordinates: a complex array is treated as its real and
    imaginary parts.  Kingma and Ba's rule with step number t (1-based):

        m <- beta1 m + (1 - beta1) g
        v <- beta2 v + (1 - beta2) g^2
        x <- x - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)

    ``m`` and ``v`` are real arrays with one entry per real coordinate of x
    (interleaved real, imaginary for a complex x).  Returns the new
    (x, m, v) in float64 (complex128 for a complex x); the inputs are not
    modified.
    """
    x = np.asarray(x)
    cplx = np.iscomplexobj(x)
    xr = (np.stack([x.real, x.imag], -1) if cplx else x).astype(np.float64).ravel()
    g = np.asarray(g)
    gr = (np.stack([g.real, g.imag], -1) if np.iscomplexobj(g) else g).astype(np.float64).ravel()
    mr = np.asarray(m, np.float64).ravel()
    vr = np.asarray(v, np.float64).ravel()
    if not (xr.shape == gr.shape == mr.shape == vr.shape):
        raise ValueError("x, g, m and v must have the same number of real coordinates")
    if t < 1:
        raise ValueError("the step number t is 1-based")
    m_new = beta1 * mr + (1.0 - beta1) * gr
    v_new = beta2 * vr + (1.0 - beta2) * gr * gr
    m_hat = m_new / (1.0 - beta1 ** t)
    v_hat = v_new / (1.0 - beta2 ** t)
    x_new = xr - lr * m_hat / (np.sqrt(v_hat) + eps)
    if cplx:
        xc = x_new.reshape(x.shape + (2,))
        x_new = xc[..., 0] + 1j * xc[..., 1]
    else:
        x_new = x_new.reshape(x.shape)
    return x_new, m_new, v_new
