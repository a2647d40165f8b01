// kernels.hpp - host-side launch interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace ptycho {

constexpr int kMaxL = 8;

// Job view passed to kernels by value.
struct JobDev {
  const float2* object;   // [L][H][W]
  const float2* probe;    // [L][M][N][N]
  const float* pos;       // [K][2]
  const float* sigma;     // [K] or null
  const float* background;  // [N][N] or null
  const uint8_t* mask;    // [N][N] or null
  const int32_t* rs_idx;  // [N*N][4] or null
  const float* rs_w;
  const int32_t* rsT_ptr;  // [N*N+1]
  const int32_t* rsT_col;
  const float* rsT_val;
  const float* measured;  // [K][N][N]
  int K, L, M, N, H, W;
  int pad[kMaxL];
  float pad_scale[kMaxL];  // 1 / sqrt(pad[l])
  const float2* tw_N;            // twiddles of length N
  const float2* tw_pad[kMaxL];   // twiddles of length pad[l]
};

// Loss parameters as used by the kernels.
struct LossDev {
  int kind;
  float eps;
  float gscale;  // 2 * scale: folds the factor of G_Psi = 2 g Psi
};

// Per-chunk workspace views (positions k0 .. k0 + C - 1).
struct Work {
  int* status;        // one int for this job
  float2* ramp;       // [C][2][N]    exp(+2 pi i f delta), y then x
  float2* X;          // [C][L][N][N] row-shifted patch, later G_A
  float2* Y;          // [C][L][M][N][N] column DFT -> Psi -> Z -> probe-gradient terms
  float2* GX;         // [C][L][N][N] gradient after the adjoint column shift
  float* loss_part;   // [C][N / RBdet]
  float* dy_part;     // [C][L][N / G]
  float* sg_part;     // [C][L][N / G]
  float* dx_part;     // [C][L][N / RBadj]
  float* ibuf;        // [C][N][N] (resampling only) I + B, then R^T g
  float* gbuf;        // [C][N][N] (resampling only) weighted dloss/dI'
  double* loss_k;     // [K] per-position loss (whole job)
  int k0, C;
};

// Radix plan of an FFT length (returns the number of passes, 0 if unknown).
int plan_radices(int n, int* out);

// Per-pass twiddle table of length n on this device (layout in fft.hpp).
const float2* twiddles(int n);
int init_twiddles();  // returns 0 or a PTYCHO_E* code
void release_twiddles();

bool supported(int N, int nl);
int rows_per_det_block(int N);
int rows_per_adj_block(int N);
int col_group_of(int N);

// Launchers (all asynchronous on `s`; return hipError_t).
hipError_t launch_fill_zero(float* p, size_t n, hipStream_t s);
hipError_t launch_fill_value(float* p, size_t n, float v, hipStream_t s);
hipError_t launch_set_status(int* status, hipStream_t s);
hipError_t launch_validate(const JobDev& jb, int* status, hipStream_t s);
hipError_t launch_prep(const JobDev& jb, const Work& w, hipStream_t s);
hipError_t launch_row_fwd(const JobDev& jb, const Work& w, int l, hipStream_t s);
hipError_t launch_col_fwd(const JobDev& jb, const Work& w, int l, hipStream_t s);
// mode: 0 fused loss+adjoint, 1 forward -> write I + B to `out` (spill: keep Psi),
//       2 adjoint from ibuf (R^T g), 3 loss only (no adjoint)
hipError_t launch_det(const JobDev& jb, const Work& w, const LossDev& loss, int mode, bool spill,
                      float* out, hipStream_t s);
hipError_t launch_resample_loss(const JobDev& jb, const Work& w, const LossDev& loss,
                                float* out, hipStream_t s);
hipError_t launch_resample_T(const JobDev& jb, const Work& w, hipStream_t s);
hipError_t launch_col_adj(const JobDev& jb, const Work& w, int l, bool want_probe,
                          hipStream_t s);
hipError_t launch_probe_reduce(const JobDev& jb, const Work& w, float2* g_probe, hipStream_t s);
hipError_t launch_row_adj(const JobDev& jb, const Work& w, int l, hipStream_t s);
hipError_t launch_obj_gather(const JobDev& jb, const Work& w, int l, float2* g_object,
                             hipStream_t s);
// n_loss: loss partials per position (N / rows_per_det_block, or the
// resampling kernel's block count)
hipError_t launch_finalize_chunk(const JobDev& jb, const Work& w, int n_loss, float* g_pos,
                                 float* g_sigma, hipStream_t s);
hipError_t launch_loss_total(const JobDev& jb, const Work& w, float scale, float* loss,
                             hipStream_t s);
hipError_t launch_adam(float* x, const float* g, float* m, float* v, size_t n, float lr,
                       float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s);

}  // namespace ptycho
