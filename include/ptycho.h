/*
 * ptycho.h - C ABI of the MI355X (gfx950) ptychography loss + gradient library.
 *
 * The library evaluates the wavelength-multiplexed, multi-mode ptychography
 * model of Eq. 1 (Section "Universal Ptychography Algorithm based on
 * Automatic Differentiation"):
 *
 *   I_k(rho) = M[ sum_l sum_m | D_{lambda_l}[ sigma_k P_{l,m}(r) O_l(r + s_k) ](rho) |^2 + N(rho) ]
 *
 * in the composite order of Eq. 2 (f1 power scaling, f2 object shift by the
 * Fourier shift theorem, f3 probe-object product, f4 propagation, f5
 * measurement), scores it against measured patterns with one of the losses
 * named in the same section (MSE on the modulus, Poisson or Gaussian
 * maximum likelihood), and returns the exact gradient with respect to the
 * object, the probe modes, the scan positions and the power coefficients,
 * as automatic differentiation would (Fig. 1B's backward path), computed by
 * a hand-written adjoint.  Adam (same section) is available as a fused step.
 *
 * Conventions (all entry points)
 *  - Every array pointer in ptycho_job_t / ptycho_grads_t / ptycho_adam_t is
 *    a DEVICE pointer on the current HIP device, owned by the caller.  The
 *    library never frees or retains caller memory.
 *  - Complex arrays are complex64: interleaved (re, im) float32 pairs.  All
 *    2D arrays are C-order with x (the second index) fastest.
 *  - The window of position k covers object pixels [p_k, p_k + N) per axis,
 *    p_k = floor(s_k + 1/2) taken in float32, s_k = pos[k] = (y, x); the
 *    shifted object inside the window is O(r + s_k) (circular Fourier shift
 *    of the gathered patch by s_k - p_k).
 *  - Propagation at wavelength l: the N x N exit wave is zero-padded to
 *    pad[l] x pad[l], a unitary DFT is taken and the N x N bins with signed
 *    frequencies in [-N/2, N/2) are kept (DC at index (N/2, N/2)).
 *    With ratio[l] = alpha > 0 instead, the propagator is the exact-ratio
 *    scaled DFT that the paper evaluates with a chirp z-transform (Section
 *    "Benchmarking with state-of-art open-source ptychography algorithm"):
 *    per axis Psi[j] = alpha^-1/2 sum_r psi[r] exp(-2 pi i (j - N/2) r / alpha),
 *    j, r in [0, N).  alpha = N lambda_l / lambda_min samples every
 *    wavelength on the detector grid without rounding the ratio; an integer
 *    alpha gives exactly the zero-padded DFT of size alpha.  It is computed
 *    by Bluestein's method with FFTs of length 2N (about twice the work of a
 *    zero-padded DFT of similar size).
 *  - Gradients follow G = dL/dRe + i dL/dIm (the convention of autodiff
 *    frameworks' .grad for complex tensors).
 *  - All work is enqueued on `stream` (a hipStream_t, NULL = default) and is
 *    asynchronous; the loss is a device scalar.
 *  - Return value: 0 on success or a negative PTYCHO_E* code.  Argument
 *    errors (NULL pointers, sizes, unsupported pad sizes, workspace too
 *    small) are detected on the host before anything is enqueued, so on
 *    such an error no output has been touched.  Window bounds depend on the
 *    device-resident positions and are checked on the device: when a window
 *    leaves the object, no out-of-bounds access happens, the loss is set to
 *    NaN, the gradients are left zeroed, ptycho_step leaves that job's
 *    variables and Adam moments bitwise unchanged, and ptycho_status()
 *    reports PTYCHO_ERANGE for that job.  The other jobs of the call are
 *    not affected.
 *  - Results are deterministic: no floating-point atomics are used; sums run
 *    in a fixed order that does not depend on the workspace size or on the
 *    other jobs of a call.
 */
#ifndef PTYCHO_H
#define PTYCHO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PTYCHO_MAX_WAVELENGTHS 8
#define PTYCHO_MAX_MODES 16
#define PTYCHO_MAX_SAMPLE_MODES 16  /* and L * Ns <= 16 */

enum {
  PTYCHO_OK = 0,
  PTYCHO_EINVAL = -1,       /* NULL pointer, negative or inconsistent size */
  PTYCHO_ERANGE = -2,       /* window outside the object, pad < N or ratio < N */
  PTYCHO_EUNSUPPORTED = -3, /* N or pad size not compiled into the library */
  PTYCHO_ENOSPC = -4,       /* workspace smaller than the minimum */
  PTYCHO_EHIP = -5          /* HIP runtime or launch error */
};

/* Loss kinds (Section "Universal Ptychography Algorithm ..."): */
enum {
  PTYCHO_LOSS_AMPLITUDE = 0, /* sum w (sqrt(I'+eps) - sqrt(Î+eps))^2, MSE on the modulus */
  PTYCHO_LOSS_POISSON = 1,   /* sum w ((I'+eps) - (Î+eps) ln(I'+eps)), Poisson NLL */
  PTYCHO_LOSS_GAUSSIAN = 2,  /* sum w (I' - Î)^2, Gaussian NLL with unit variance */
  PTYCHO_LOSS_VJP = 3,       /* sum u I' with u = `measured`: vector-Jacobian product of
                                the forward model (mask ignored) */
  PTYCHO_LOSS_MIXED = 4      /* sum w ((I' - Î)^2 / (I' + v) + ln(I' + v)): MLE with mixed
                                Poisson-Gaussian noise statistics (same section), Gaussian
                                approximation with variance I' + v, v = noise_var (the read-
                                noise variance in photons^2, > 0) */
};

/* One reconstruction job: the variables and fixed inputs of Eq. 1. */
typedef struct ptycho_job {
  int32_t K;   /* scan positions (>= 0) */
  int32_t L;   /* wavelengths, 1..PTYCHO_MAX_WAVELENGTHS */
  int32_t M;   /* probe (illumination) modes per wavelength, 1..PTYCHO_MAX_MODES */
  int32_t N;   /* window = detector size, N x N (see ptycho_supported) */
  int32_t H;   /* object height, >= N */
  int32_t W;   /* object width, >= N */
  int32_t pad[PTYCHO_MAX_WAVELENGTHS]; /* DFT size per wavelength, pad[l] >= N (ignored
                                          where ratio[l] != 0) */
  double ratio[PTYCHO_MAX_WAVELENGTHS]; /* exact sampling ratio alpha_l >= N of the
                                           exact-ratio propagator, or 0 (zero-padded DFT
                                           of size pad[l]); negative, NaN or infinite:
                                           PTYCHO_EINVAL; 0 < alpha < N: PTYCHO_ERANGE */
  float* object;            /* complex64 [L][Ns][H][W] O_{l,n}; written only by ptycho_step */
  float* probe;             /* complex64 [L][M][N][N] P_{l,m}; written only by ptycho_step */
  float* pos;               /* float32 [K][2]        s_k = (y, x); written only by ptycho_step */
  float* sigma;             /* float32 [K] power coefficients sigma_k, or NULL (= 1);
                               written only by ptycho_step (lr_sigma != 0) */
  float* background;        /* float32 [N][N] additive background N(rho), or NULL (= 0);
                               written only by ptycho_step (lr_background != 0) */
  const uint8_t* mask;      /* uint8 [N][N] loss weight 0/1, or NULL (= all 1) */
  /* Optional bilinear resampling of the predicted pattern (tilted plane):
     I'(a) = sum_{t<4} rs_w[a][t] * I(rs_idx[a][t]), flat indices into N x N.
     rsT_* is the same map transposed in CSR form (rows = model pixels):
     rsT_ptr [N*N+1], rsT_col [4*N*N] (camera pixel), rsT_val [4*N*N]; build
     it with ptycho_transpose_table().  All five NULL = identity.  Indices
     outside [0, N*N) are clamped (never dereferenced out of bounds). */
  const int32_t* rs_idx;
  const float* rs_w;
  const int32_t* rsT_ptr;
  const int32_t* rsT_col;
  const float* rsT_val;
  const float* measured;    /* float32 [K][N][N] measured Î_k, or upstream dL/dI' (VJP) */
  int32_t Ns;               /* sample modes O_{l,n} of Eq. 1 (0 or 1: one).  With Ns > 1
                               the object is complex64 [L][Ns][H][W], every (l, n) pair is
                               propagated with every probe mode P_{l,m} and summed
                               incoherently; L * Ns <= 16 */
} ptycho_job_t;

typedef struct ptycho_loss {
  int32_t kind;     /* PTYCHO_LOSS_* */
  float eps;        /* added inside sqrt / log (photons); e.g. 1e-6 */
  float scale;      /* the data term and its gradients are multiplied by scale (e.g. 1/K) */
  float noise_var;  /* PTYCHO_LOSS_MIXED: read-noise variance v > 0 */
  /* Regularisation of the object amplitude a = |O| (the paper's L1 and TV
     regularisations, applied to the amplitude), added to the loss unscaled:
     l1 sum a + tv sum sqrt(dy^2 + dx^2 + tv_eps^2), dy, dx forward differences
     of a within each (wavelength, sample mode) plane, zero past the last
     row / column.  Zero weights switch a term off (and cost nothing). */
  float l1, tv, tv_eps;
} ptycho_loss_t;

/* Outputs, one per job.  Every pointer may be NULL to skip that output
   (a NULL gradient also skips the work that only it needs). */
typedef struct ptycho_grads {
  float* loss;          /* float32 [1] */
  float* g_object;      /* complex64 [L][Ns][H][W] */
  float* g_probe;       /* complex64 [L][M][N][N] */
  float* g_pos;         /* float32 [K][2] */
  float* g_sigma;       /* float32 [K] */
  float* g_background;  /* float32 [N][N]: dL/dN(rho); the background enters before the
                           resampling, so this is the sum over positions of the
                           pulled-back dL/dI' (Eq. 1's common background, Fig. 1B) */
  float* g_ratio;       /* float32 [L]: dL/dalpha_l for the exact-ratio wavelengths (0 for
                           zero-padded ones).  alpha_l = lambda_l z / (p dx) is proportional
                           to the propagation distance z of D_{lambda,z}, so
                           dL/dz = sum_l (alpha_l / z) dL/dalpha_l (the distance correction of
                           Section "Benchmarking with state-of-art open-source ptychography
                           algorithm").  Costs one extra row and one extra column transform
                           per (position, wavelength, mode) and recomputes Psi in the
                           adjoint. */
} ptycho_grads_t;

/* Adam state and hyper-parameters, one per job (real and imaginary parts
   are independent coordinates).  m_* / v_* have the shapes of the variables
   (complex arrays as interleaved floats).  A zero learning rate leaves that
   variable unchanged; a non-zero one needs its m/v pair and its gradient
   output (and, for sigma and background, the job's array).  t is the
   1-based step number used for bias correction.  The paper optimises all of
   these variables with Adam (Section "Universal Ptychography Algorithm
   based on Automatic Differentiation"). */
typedef struct ptycho_adam {
  float *m_object, *v_object, *m_probe, *v_probe, *m_pos, *v_pos;
  float lr_object, lr_probe, lr_pos;
  float beta1, beta2, eps;
  int32_t t;
  float *m_sigma, *v_sigma, *m_background, *v_background;
  float lr_sigma, lr_background;
} ptycho_adam_t;

/* Returns 1 if window N with DFT size pad is compiled in, else 0. */
int32_t ptycho_supported(int32_t N, int32_t pad);

/* Workspace bytes needed to run `which` (0 forward, 1 loss+gradient, 2 step)
   for these jobs with at most `chunk` positions per pass (chunk <= 0: all K).
   Any workspace of at least the chunk = 1 size works; a larger workspace
   lets the library process more positions per launch.  Loss + gradient
   calls that want the probe gradient sum it over groups of consecutive
   positions of a job (3 at windows of 384 and 512 pixels and wherever the
   sums of 4 do not fit in on-chip memory, 4 when they fit and the scan is
   long enough to keep the launch filled, else 1; a function of the job
   alone), so for them `chunk` is rounded up to a
   multiple of the job's group size.  Only the size fields
   (K, L, M, N, H, W, pad, ratio) and whether rs_idx is non-NULL are read: the array
   pointers may be NULL, so a scheduler can size a call before allocating. */
int32_t ptycho_workspace_bytes(const ptycho_job_t* jobs, int32_t n_jobs, int32_t which,
                               int32_t chunk, size_t* bytes);

/* Forward model (Eq. 1 without the loss): intensity[j] is a device float32
   [K][N][N] array per job receiving I'_k (background added, resampling
   applied, mask not applied). */
int32_t ptycho_forward(const ptycho_job_t* jobs, int32_t n_jobs, float* const* intensity,
                       void* workspace, size_t workspace_bytes, void* stream);

/* Loss and gradients for each job (grads[j] belongs to jobs[j]): the model
   of Eq. 1 evaluated in the order of Eq. 2, one of the losses of Section
   "Universal Ptychography Algorithm based on Automatic Differentiation"
   summed over positions and pixels, and the exact gradient of that loss with
   respect to every variable whose output pointer is non-NULL -- the reverse
   pass of Fig. 1B (intensity residual back through the measurement, the
   conjugate propagator, the probe-object product and the Fourier shift),
   written out by hand instead of taken by automatic differentiation.
   Outputs are overwritten (not accumulated).  The workspace is scratch for
   the call; ptycho_status() reads the per-job window check from it. */
int32_t ptycho_loss_grad(const ptycho_job_t* jobs, int32_t n_jobs, const ptycho_loss_t* loss,
                         const ptycho_grads_t* grads, void* workspace, size_t workspace_bytes,
                         void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   loss and gradients as ptycho_loss_grad, with the library's own scratch
   instead of a caller workspace.  The scratch is a static device array of
   PTYCHO_NOALLOC_SCRATCH_BYTES per GPU, created when the library is loaded
   and held until the process ends; this call allocates nothing (no
   hipMalloc/hipFree, no events: profiling does not bracket it).  Jobs whose
   smallest workspace (one position per chunk, see ptycho_workspace_bytes)
   exceeds the scratch are rejected with PTYCHO_ENOSPC before anything is
   enqueued; larger scans run in more, smaller position chunks, with results
   bitwise equal to ptycho_loss_grad.  The first call on a device copies the
   twiddle tables into their static array (a synchronous copy, no
   allocation).  Every call on one GPU shares that GPU's scratch and leaves
   its contents behind (each call initialises everything it reads): calls
   that overlap on one GPU race, so serialise them (one stream, or events).
   A window outside the object sets that job's loss to NaN and leaves its
   gradients zeroed, as in ptycho_loss_grad; ptycho_status() cannot read this
   call's status (the caller has no pointer to the scratch). */
#define PTYCHO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int32_t ptycho_loss_grad_noalloc(const ptycho_job_t* jobs, int32_t n_jobs,
                                 const ptycho_loss_t* loss, const ptycho_grads_t* grads,
                                 void* stream);

/* Loss, gradients and one Adam update of object, probe, positions, power
   coefficients and background of each job, in place.  grads[j].g_* must be non-NULL for every variable whose
   learning rate is non-zero (they receive the gradient at the state before
   the update). */
int32_t ptycho_step(const ptycho_job_t* jobs, int32_t n_jobs, const ptycho_loss_t* loss,
                    const ptycho_grads_t* grads, const ptycho_adam_t* adam, void* workspace,
                    size_t workspace_bytes, void* stream);

/* Device-side status of job `job` (index into that call's job array) of
   the last call that used this workspace; synchronises `stream` first.
   Returns PTYCHO_OK or PTYCHO_ERANGE (a window left the object), or
   PTYCHO_EINVAL / PTYCHO_EHIP if the query itself failed. */
int32_t ptycho_status(const void* workspace, int32_t job, void* stream);

/* Host helper: CSR transpose of a resampling table.  idx/w are HOST arrays
   [n_out][4]; rows of the result are the n_in model pixels.  ptr must hold
   n_in + 1 entries, col and val 4 * n_out entries (unused tail set to 0). */
int32_t ptycho_transpose_table(const int32_t* idx, const float* w, int32_t n_out, int32_t n_in,
                               int32_t* ptr, int32_t* col, float* val);

/* Per-kernel-class timing, for measurement (not needed for computation).
   ptycho_profile(1) clears the totals and starts bracketing every launch of
   every call with two HIP events on its stream; ptycho_profile(0) stops.
   ptycho_profile_read() waits for the recorded launches and returns the
   summed GPU milliseconds and the launch count of one kernel class
   (0 <= kernel_class < number of classes; ptycho_kernel_class_name() gives
   its name and returns NULL past the last class).  Not thread-safe against
   concurrent calls on other host threads while enabled. */
int32_t ptycho_profile(int32_t enable);
int32_t ptycho_profile_read(int32_t kernel_class, double* total_ms, int64_t* launches);
const char* ptycho_kernel_class_name(int32_t kernel_class);
/* Restricts the bracketing to the kernel classes whose bit (1 << kernel_class)
   is set in class_mask, for launches enqueued after the call (all classes by
   default and after ptycho_profile(0)); fewer events per call perturb the
   timed launches less.  Always returns PTYCHO_OK. */
int32_t ptycho_profile_classes(uint32_t class_mask);

/* Static description of an error code. */
const char* ptycho_error_string(int32_t code);

/* Forgets the library's device tables (twiddles, kept in static device
   arrays), so that the next call on each device fills them again, and frees
   the profiling events. */
void ptycho_release(void);

#ifdef __cplusplus
}
#endif

#endif /* PTYCHO_H */
