// kernels.hip - gfx950 kernels of the ptychography loss + gradient path.
//
// Per position chunk the path runs (Eq. 2 order, then its adjoint):
//   prep      : p_k = floor(s_k + 1/2), delta_k, phase ramps exp(+2 pi i f delta)
//   row_fwd   : gather object rows, x-shift (FFT, ramp, IFFT)            -> X
//   col_fwd   : y-shift of X columns, times sigma P_{l,m} for every mode,
//               first (column) pass of the padded, cropped DFT            -> Y
//   det       : second (row) pass of the DFT, incoherent sum over l and m,
//               background, loss and its derivative, 2 g Psi, adjoint row
//               DFT                                                        -> Z (in Y)
//   col_adj   : adjoint column DFT -> chi; G_Osh = sum_m conj(sigma P) chi;
//               probe-gradient terms conj(sigma Osh) chi (in Y); sigma and
//               y-position derivatives; adjoint y-shift                  -> GX
//   probe_red : ordered sum over positions of the probe-gradient terms
//   row_adj   : adjoint x-shift -> G_A (in X); x-position derivative
//   obj_gather: object gradient tiles gather G_A of every overlapping window
//               in ascending k (no atomics)
//   finalize  : ordered per-position sums of the partials
// The C ABI (api.cpp) sequences these launches on one stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "fft.hpp"
#include "kernels.hpp"

namespace ptycho {

constexpr int NT = 256;   // threads per workgroup (row kernels)
constexpr int CNT = 512;  // threads per workgroup (column kernels)
constexpr int kERange = -2;

template <int... Ps>
struct IntList {};
template <int... Ps>
constexpr int max_row_lp(IntList<Ps...>) {
  int m = 0;
  for (int p : {Ps...}) m = row_lp(p) > m ? row_lp(p) : m;
  return m;
}

// DFT sizes compiled in, per window size N.
template <int N>
struct PadList;
template <> struct PadList<64> { using type = IntList<64, 72, 80, 84, 90, 96>; static constexpr int max = 96; };
template <> struct PadList<128> { using type = IntList<128, 140, 150, 168, 189>; static constexpr int max = 189; };
template <> struct PadList<256> { using type = IntList<256, 280, 300, 315, 336, 343, 375>; static constexpr int max = 375; };
template <> struct PadList<384> { using type = IntList<384, 420, 480>; static constexpr int max = 480; };
template <> struct PadList<512> { using type = IntList<512, 560, 600, 675, 750>; static constexpr int max = 750; };

template <int N> constexpr int rb_row() { return N == 64 ? 32 : (N <= 256 ? 16 : 8); }
template <int N> constexpr int rb_det() { return N <= 128 ? 16 : (N == 512 ? 4 : 8); }
template <int N> constexpr int rb_adj() { return N <= 128 ? 16 : (N == 512 ? 4 : 8); }
template <int N> constexpr int col_group() { return N <= 256 ? 16 : 8; }

template <class F, int P, int... Ps>
__device__ __forceinline__ void pad_switch(int nl, const F& f, IntList<P, Ps...>) {
  if (nl == P) {
    f(std::integral_constant<int, P>{});
  } else {
    if constexpr (sizeof...(Ps) > 0) pad_switch(nl, f, IntList<Ps...>{});
  }
}

// Select element l of a small kernel-argument array with constant indices
// only: a run-time index into a by-value argument would force the whole
// argument block into registers or scratch.
template <class T>
__device__ __forceinline__ T pick(const T (&a)[kMaxL], int l) {
  T r = a[0];
#pragma unroll
  for (int i = 1; i < kMaxL; ++i) r = (l == i) ? a[i] : r;
  return r;
}

__device__ __forceinline__ void split_pos(const float* __restrict__ pos, int k, int& py, int& px,
                                          float& dy, float& dx) {
  const float sy = pos[2 * k], sx = pos[2 * k + 1];
  const float fy = floorf(sy + 0.5f), fx = floorf(sx + 0.5f);
  py = static_cast<int>(fy);
  px = static_cast<int>(fx);
  dy = sy - fy;
  dx = sx - fx;
}

// signed DFT frequency of bin i for length n (numpy fftfreq convention)
__device__ __forceinline__ float freq(int i, int n) {
  return static_cast<float>(i < n / 2 ? i : i - n) / static_cast<float>(n);
}

// Deterministic workgroup sum over BS threads; the result is valid in thread 0.
template <int BS = NT>
__device__ __forceinline__ float block_sum(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

// ------------------------------------------------------------------ utility
__global__ void k_fill(float* __restrict__ p, size_t n, float v) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t j = i; j < n; j += stride) p[j] = v;
}

__global__ void k_set_status(int* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *status = 0;
}

__global__ void k_validate(JobDev jb, int* status) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= jb.K) return;
  const float sy = jb.pos[2 * k], sx = jb.pos[2 * k + 1];
  bool bad = !(isfinite(sy) && isfinite(sx));
  if (!bad) {
    const float fy = floorf(sy + 0.5f), fx = floorf(sx + 0.5f);
    bad = fy < 0.f || fx < 0.f || fy + jb.N > jb.H || fx + jb.N > jb.W;
  }
  if (bad) *status = kERange;  // every writer stores the same value
}

// ramps[c][0][f] = exp(2 pi i nu_f delta_y), ramps[c][1][f] likewise for x
__global__ void k_prep(JobDev jb, Work w) {
  if (*w.status) return;
  const int c = blockIdx.x, k = w.k0 + c;
  int py, px;
  float dy, dx;
  split_pos(jb.pos, k, py, px, dy, dx);
  const int N = jb.N;
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
    const int f = i % N;
    const double d = (i < N) ? static_cast<double>(dy) : static_cast<double>(dx);
    const double nu = static_cast<double>(f < N / 2 ? f : f - N) / N;
    double sn, cs;
    sincospi(2.0 * nu * d, &sn, &cs);
    w.ramp[static_cast<size_t>(c) * 2 * N + i] = make_float2(static_cast<float>(cs),
                                                             static_cast<float>(sn));
  }
}

// ------------------------------------------------------------- row forward
// X[c][l][y][:] = IFFT_x( ramp_x * FFT_x( O_l[p_y + y][p_x : p_x + N] ) ) / N
template <int N>
__global__ __launch_bounds__(NT) void k_row_fwd(JobDev jb, Work w, int l) {
  if (*w.status) return;
  constexpr int RB = rb_row<N>();
  constexpr int LP = row_lp(N);
  using Ix = Lds<N, LP, false>;
  __shared__ float2 buf[RB * LP];
  const int c = blockIdx.y, k = w.k0 + c;
  const int y0 = blockIdx.x * RB;
  int py, px;
  float dy, dx;
  split_pos(jb.pos, k, py, px, dy, dx);
  const float2* __restrict__ O =
      jb.object + static_cast<size_t>(l) * jb.H * jb.W + static_cast<size_t>(py + y0) * jb.W + px;
  const float2* __restrict__ rx = w.ramp + (static_cast<size_t>(c) * 2 + 1) * N;
  const float2* __restrict__ tw = jb.tw_N;
  const int Wd = jb.W;
  auto ld_obj = [&](int line, int i) { return O[static_cast<size_t>(line) * Wd + i]; };
  auto st_ramp = [&](int line, int i, float2 v) { buf[Ix::at(line, i)] = cmul(v, rx[i]); };
  fft_lines<N, false, RB, NT, LP, false>(buf, tw, ld_obj, st_ramp);
  float2* __restrict__ X = w.X + ((static_cast<size_t>(c) * jb.L + l) * N + y0) * N;
  constexpr float inv = 1.0f / N;
  auto ld_buf = [&](int line, int i) { return buf[Ix::at(line, i)]; };
  auto st_x = [&](int line, int i, float2 v) { X[line * N + i] = cscale(v, inv); };
  fft_lines<N, true, RB, NT, LP, false>(buf, tw, ld_buf, st_x);
}

// ---------------------------------------------------------- column forward
// Osh = y-shift of X columns; Y_m = (1/sqrt(NL)) crop( DFT_NL_y( sigma P_m Osh ) )
template <int N, int NL>
__global__ __launch_bounds__(CNT) void k_col_fwd(JobDev jb, Work w, int l) {
  if (*w.status) return;
  constexpr int G = col_group<N>();
  constexpr int LP = G + 1;
  constexpr int NE = N * G / CNT;
  static_assert(N * G % CNT == 0, "natural layout");
  __shared__ float2 buf[NL * LP];
  const int c = blockIdx.y, k = w.k0 + c, x0 = blockIdx.x * G;
  const int tid = threadIdx.x;
  const float2* __restrict__ X = w.X + (static_cast<size_t>(c) * jb.L + l) * N * N + x0;
  const float2* __restrict__ ry = w.ramp + static_cast<size_t>(c) * 2 * N;
  const float2* __restrict__ twN = jb.tw_N;
  const float2* __restrict__ twL = pick(jb.tw_pad, l);

  auto ld_x = [&](int line, int i) { return X[i * N + line]; };
  auto st_ramp = [&](int line, int i, float2 v) { buf[i * LP + line] = cmul(v, ry[i]); };
  fft_lines<N, false, G, CNT, LP, true>(buf, twN, ld_x, st_ramp);
  auto ld_buf = [&](int line, int i) { return buf[i * LP + line]; };
  auto st_buf = [&](int line, int i, float2 v) { buf[i * LP + line] = v; };
  fft_lines<N, true, G, CNT, LP, true>(buf, twN, ld_buf, st_buf);

  const float sg = (jb.sigma ? jb.sigma[k] : 1.0f) / N;
  float2 o[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * CNT, line = e % G, i = e / G;
    o[q] = cscale(buf[i * LP + line], sg);
  }
  __syncthreads();
  const float ps = pick(jb.pad_scale, l);
  for (int m = 0; m < jb.M; ++m) {
    const float2* __restrict__ P = jb.probe + (static_cast<size_t>(l) * jb.M + m) * N * N + x0;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * CNT, line = e % G, i = e / G;
      buf[i * LP + line] = cmul(P[i * N + line], o[q]);
    }
    __syncthreads();
    float2* __restrict__ Y =
        w.Y + ((static_cast<size_t>(c) * jb.L + l) * jb.M + m) * N * N + x0;
    auto ld_psi = [&](int line, int t) {
      return t < N ? buf[t * LP + line] : make_float2(0.f, 0.f);
    };
    auto st_y = [&](int line, int t, float2 v) {
      int u = t + N / 2;
      if (u >= NL) u -= NL;
      if (u < N) Y[u * N + line] = cscale(v, ps);
    };
    fft_lines<NL, false, G, CNT, LP, true>(buf, twL, ld_psi, st_y);
  }
}

// ------------------------------------------------------------ detector rows
// Row pass of the padded DFT for one (l, m) and RB detector rows:
// Psi[u][:] = (1/sqrt(NL)) crop( DFT_NL_x( Y[u][:] ) ), acc += |Psi|^2.
// Kept out of line so that each DFT size gets its own register allocation
// inside the kernel's run-time switch over the wavelengths' pad sizes.
template <int N, int NL, int RB>
__device__ __noinline__ void det_rows_fwd(lf2* buf, lf32* acc, gf2* __restrict__ Yr,
                                          const gf2* __restrict__ twL, float ps, bool keep) {
  constexpr int LP = row_lp(NL);
  auto ld = [&](int line, int t) { return t < N ? ldv(Yr, line * N + t) : make_float2(0.f, 0.f); };
  auto st = [&](int line, int t, float2 v) {
    int u = t + N / 2;
    if (u >= NL) u -= NL;
    if (u < N) {
      v = cscale(v, ps);
      if (keep) stv(Yr, line * N + u, v);
      acc[line * N + u] += cabs2(v);
    }
  };
  fft_lines<NL, false, RB, NT, LP, false>(buf, twL, ld, st);
}

// Adjoint row pass: Z[u][:] = (1/sqrt(NL)) DFT^H_NL_x( embed( g2 Psi[u][:] ) )[0:N],
// g2 = acc (2 scale w dloss/dI), written over Psi.
template <int N, int NL, int RB>
__device__ __noinline__ void det_rows_adj(lf2* buf, const lf32* acc, gf2* __restrict__ Yr,
                                          const gf2* __restrict__ twL, float ps) {
  constexpr int LP = row_lp(NL);
  auto ld = [&](int line, int t) {
    int u = t + N / 2;
    if (u >= NL) u -= NL;
    return u < N ? cscale(ldv(Yr, line * N + u), acc[line * N + u]) : make_float2(0.f, 0.f);
  };
  auto st = [&](int line, int t, float2 v) {
    if (t < N) stv(Yr, line * N + t, cscale(v, ps));
  };
  fft_lines<NL, true, RB, NT, LP, false>(buf, twL, ld, st);
}

// MODE 0: fused forward + loss + adjoint; 1: forward, write I + B to out;
// 2: adjoint from g rows in w.ibuf; 3: forward + loss only.
// `spill` (MODE 1) writes Psi back over Y for a later MODE 2.
template <int N, int MODE>
__global__ __launch_bounds__(NT) void k_det(JobDev jb, Work w, LossDev loss, bool spill,
                                            float* __restrict__ out) {
  if (*w.status) return;
  constexpr int RB = rb_det<N>();
  constexpr int LPMAX = max_row_lp(typename PadList<N>::type{});
  __shared__ float2 buf[RB * LPMAX];
  __shared__ float acc[RB * N];
  __shared__ float red[NT / 64];
  const int c = blockIdx.y, k = w.k0 + c, u0 = blockIdx.x * RB;
  const int tid = threadIdx.x;
  const size_t plane = static_cast<size_t>(N) * N;

  if (MODE != 2) {
    for (int e = tid; e < RB * N; e += NT) acc[e] = 0.f;
    __syncthreads();
    const bool keep = (MODE == 0) || (MODE == 1 && spill);
    for (int l = 0; l < jb.L; ++l) {
      const float ps = pick(jb.pad_scale, l);
      const float2* twL = pick(jb.tw_pad, l);
      const int nl = pick(jb.pad, l);
      for (int m = 0; m < jb.M; ++m) {
        float2* Yr = w.Y + ((static_cast<size_t>(c) * jb.L + l) * jb.M + m) * plane +
                     static_cast<size_t>(u0) * N;
        pad_switch(nl, [&](auto nlc) {
          constexpr int NL = decltype(nlc)::value;
          det_rows_fwd<N, NL, RB>((lf2*)buf, (lf32*)acc, (gf2*)Yr, (const gf2*)twL, ps, keep);
        }, typename PadList<N>::type{});
      }
    }
    // acc = sum_{l,m} |Psi|^2 for RB rows
    float lsum = 0.f;
    for (int e = tid; e < RB * N; e += NT) {
      const int line = e / N, x = e % N;
      const int pix = (u0 + line) * N + x;
      float I = acc[e];
      if (jb.background) I += jb.background[pix];
      if (MODE == 1) {
        out[static_cast<size_t>(c) * plane + pix] = I;
        continue;
      }
      const float meas = jb.measured[static_cast<size_t>(k) * plane + pix];
      const float wt = (loss.kind != 3 && jb.mask) ? static_cast<float>(jb.mask[pix]) : 1.f;
      float ell, dell;
      if (loss.kind == 0) {
        const float a = sqrtf(I + loss.eps), b = sqrtf(meas + loss.eps);
        ell = (a - b) * (a - b);
        dell = 1.f - b / a;
      } else if (loss.kind == 1) {
        const float a = I + loss.eps, b = meas + loss.eps;
        ell = a - b * logf(a);
        dell = 1.f - b / a;
      } else if (loss.kind == 2) {
        ell = (I - meas) * (I - meas);
        dell = 2.f * (I - meas);
      } else {
        ell = meas * I;
        dell = meas;
      }
      lsum += wt * ell;
      acc[e] = loss.gscale * wt * dell;  // 2 * scale * w * dloss/dI
    }
    if (MODE == 1) return;
    const float s = block_sum(lsum, red);
    if (tid == 0) w.loss_part[static_cast<size_t>(c) * gridDim.x + blockIdx.x] = s;
    if (MODE == 3) return;
  } else {
    for (int e = tid; e < RB * N; e += NT) {
      const int line = e / N, x = e % N;
      acc[e] = w.ibuf[static_cast<size_t>(c) * plane + (u0 + line) * N + x];
    }
    __syncthreads();
  }
  for (int l = 0; l < jb.L; ++l) {
    const float ps = pick(jb.pad_scale, l);
    const float2* twL = pick(jb.tw_pad, l);
    const int nl = pick(jb.pad, l);
    for (int m = 0; m < jb.M; ++m) {
      float2* Yr = w.Y + ((static_cast<size_t>(c) * jb.L + l) * jb.M + m) * plane +
                   static_cast<size_t>(u0) * N;
      pad_switch(nl, [&](auto nlc) {
        constexpr int NL = decltype(nlc)::value;
        det_rows_adj<N, NL, RB>((lf2*)buf, (const lf32*)acc, (gf2*)Yr, (const gf2*)twL, ps);
      }, typename PadList<N>::type{});
    }
  }
}

// ----------------------------------------------- tilted-plane resampling
// out != null: forward, write I' = R(I + B).  Else: loss on I' and
// gbuf = 2 scale w dloss/dI'.
__global__ __launch_bounds__(NT) void k_resample_loss(JobDev jb, Work w, LossDev loss,
                                                      float* __restrict__ out) {
  if (*w.status) return;
  __shared__ float red[NT / 64];
  const int c = blockIdx.y, k = w.k0 + c;
  const int N = jb.N;
  const size_t plane = static_cast<size_t>(N) * N;
  const int a = blockIdx.x * NT + threadIdx.x;
  float lsum = 0.f;
  if (a < N * N) {
    const float* __restrict__ I = w.ibuf + static_cast<size_t>(c) * plane;
    float Ip = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = min(max(jb.rs_idx[4 * a + t], 0), N * N - 1);  // caller tables are clamped
      Ip = fmaf(jb.rs_w[4 * a + t], I[j], Ip);
    }
    if (out) {
      out[static_cast<size_t>(c) * plane + a] = Ip;
    } else {
      const float meas = jb.measured[static_cast<size_t>(k) * plane + a];
      const float wt = (loss.kind != 3 && jb.mask) ? static_cast<float>(jb.mask[a]) : 1.f;
      float ell, dell;
      if (loss.kind == 0) {
        const float x = sqrtf(Ip + loss.eps), y = sqrtf(meas + loss.eps);
        ell = (x - y) * (x - y);
        dell = 1.f - y / x;
      } else if (loss.kind == 1) {
        const float x = Ip + loss.eps, y = meas + loss.eps;
        ell = x - y * logf(x);
        dell = 1.f - y / x;
      } else if (loss.kind == 2) {
        ell = (Ip - meas) * (Ip - meas);
        dell = 2.f * (Ip - meas);
      } else {
        ell = meas * Ip;
        dell = meas;
      }
      lsum = wt * ell;
      w.gbuf[static_cast<size_t>(c) * plane + a] = loss.gscale * wt * dell;
    }
  }
  if (out) return;
  const float s = block_sum(lsum, red);
  if (threadIdx.x == 0) w.loss_part[static_cast<size_t>(c) * gridDim.x + blockIdx.x] = s;
}

// ibuf[c][j] = sum over the transposed table row j of val * gbuf[c][col]
__global__ __launch_bounds__(NT) void k_resample_T(JobDev jb, Work w) {
  if (*w.status) return;
  const int c = blockIdx.y;
  const int N = jb.N;
  const size_t plane = static_cast<size_t>(N) * N;
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= N * N) return;
  const float* __restrict__ g = w.gbuf + static_cast<size_t>(c) * plane;
  float s = 0.f;
  const int nnz_max = 4 * N * N;
  const int p0 = min(max(jb.rsT_ptr[j], 0), nnz_max), p1 = min(max(jb.rsT_ptr[j + 1], p0), nnz_max);
  for (int p = p0; p < p1; ++p) s = fmaf(jb.rsT_val[p], g[min(max(jb.rsT_col[p], 0), N * N - 1)], s);
  w.ibuf[static_cast<size_t>(c) * plane + j] = s;
}

// ---------------------------------------------------------- column adjoint
template <int N, int NL>
__global__ __launch_bounds__(CNT) void k_col_adj(JobDev jb, Work w, int l, bool want_probe) {
  if (*w.status) return;
  constexpr int G = col_group<N>();
  constexpr int LP = G + 1;
  constexpr int NE = N * G / CNT;
  __shared__ float2 buf[NL * LP];
  __shared__ float red[CNT / 64];
  const int c = blockIdx.y, k = w.k0 + c, x0 = blockIdx.x * G;
  const int tid = threadIdx.x;
  const float2* __restrict__ X = w.X + (static_cast<size_t>(c) * jb.L + l) * N * N + x0;
  const float2* __restrict__ ry = w.ramp + static_cast<size_t>(c) * 2 * N;
  const float2* __restrict__ twN = jb.tw_N;
  const float2* __restrict__ twL = pick(jb.tw_pad, l);
  const float sig = jb.sigma ? jb.sigma[k] : 1.0f;

  // recompute Ohat = ramp_y FFT_y(X) and Osh = IFFT_y(Ohat) / N
  auto ld_x = [&](int line, int i) { return X[i * N + line]; };
  auto st_ramp = [&](int line, int i, float2 v) { buf[i * LP + line] = cmul(v, ry[i]); };
  fft_lines<N, false, G, CNT, LP, true>(buf, twN, ld_x, st_ramp);
  float2 ohat[NE], o[NE], go[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * CNT, line = e % G, i = e / G;
    ohat[q] = buf[i * LP + line];
  }
  auto ld_buf = [&](int line, int i) { return buf[i * LP + line]; };
  auto st_buf = [&](int line, int i, float2 v) { buf[i * LP + line] = v; };
  fft_lines<N, true, G, CNT, LP, true>(buf, twN, ld_buf, st_buf);
  constexpr float invN = 1.0f / N;
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * CNT, line = e % G, i = e / G;
    o[q] = cscale(buf[i * LP + line], invN);
    go[q] = make_float2(0.f, 0.f);
  }
  __syncthreads();

  const float ps = pick(jb.pad_scale, l);
  float sgsum = 0.f;
  for (int m = 0; m < jb.M; ++m) {
    float2* __restrict__ Z = w.Y + ((static_cast<size_t>(c) * jb.L + l) * jb.M + m) * N * N + x0;
    const float2* __restrict__ P = jb.probe + (static_cast<size_t>(l) * jb.M + m) * N * N + x0;
    auto ld_z = [&](int line, int t) {
      int u = t + N / 2;
      if (u >= NL) u -= NL;
      return u < N ? Z[u * N + line] : make_float2(0.f, 0.f);
    };
    auto st_chi = [&](int line, int t, float2 v) {
      if (t < N) buf[t * LP + line] = cscale(v, ps);
    };
    fft_lines<NL, true, G, CNT, LP, true>(buf, twL, ld_z, st_chi);
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * CNT, line = e % G, i = e / G;
      const float2 chi = buf[i * LP + line];
      const float2 p = P[i * N + line];
      const float2 pc = cmulconj(p, chi);  // conj(P) chi
      go[q].x = fmaf(sig, pc.x, go[q].x);
      go[q].y = fmaf(sig, pc.y, go[q].y);
      // Re( conj(chi) P Osh ) = Re( conj(conj(P) chi) Osh )
      sgsum += pc.x * o[q].x + pc.y * o[q].y;
      if (want_probe) Z[i * N + line] = cscale(cmulconj(o[q], chi), sig);
    }
    __syncthreads();
  }
  {
    const float s = block_sum<CNT>(sgsum, red);
    if (tid == 0)
      w.sg_part[(static_cast<size_t>(c) * jb.L + l) * gridDim.x + blockIdx.x] = s;
  }
  // Ghat = FFT_y(G_Osh): y-position derivative and adjoint y-shift
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * CNT, line = e % G, i = e / G;
    buf[i * LP + line] = go[q];
  }
  __syncthreads();
  fft_lines<N, false, G, CNT, LP, true>(buf, twN, ld_buf, st_buf);
  float dsum = 0.f;
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * CNT, line = e % G, i = e / G;
    const float2 gh = buf[i * LP + line];
    const float nu = 2.0f * static_cast<float>(kPi) * freq(i, N);
    // Re( conj(gh) * (i nu ohat) )
    dsum += nu * (gh.y * ohat[q].x - gh.x * ohat[q].y);
    buf[i * LP + line] = cmul(gh, cconj(ry[i]));
  }
  __syncthreads();
  float2* __restrict__ GX = w.GX + (static_cast<size_t>(c) * jb.L + l) * N * N + x0;
  auto st_gx = [&](int line, int i, float2 v) { GX[i * N + line] = cscale(v, invN); };
  fft_lines<N, true, G, CNT, LP, true>(buf, twN, ld_buf, st_gx);
  const float s = block_sum<CNT>(dsum, red);
  if (tid == 0)
    w.dy_part[(static_cast<size_t>(c) * jb.L + l) * gridDim.x + blockIdx.x] = s * invN;
}

// ------------------------------------------- probe gradient: ordered k sum
// g_probe[l][m][pix] += sum_{c ascending} Y[c][l][m][pix]
__global__ __launch_bounds__(NT) void k_probe_reduce(JobDev jb, Work w, float2* __restrict__ gp) {
  if (*w.status) return;
  const size_t plane = static_cast<size_t>(jb.N) * jb.N;
  const size_t pix = static_cast<size_t>(blockIdx.x) * NT + threadIdx.x;
  if (pix >= plane) return;
  const int lm = blockIdx.y;  // l * M + m
  const size_t stride = static_cast<size_t>(jb.L) * jb.M * plane;
  const float2* __restrict__ src = w.Y + static_cast<size_t>(lm) * plane + pix;
  float2 acc = gp[static_cast<size_t>(lm) * plane + pix];
  for (int c = 0; c < w.C; ++c) acc = cadd(acc, src[c * stride]);
  gp[static_cast<size_t>(lm) * plane + pix] = acc;
}

// -------------------------------------------------------------- row adjoint
// lines [0, RB): G_X rows; [RB, 2 RB): X rows.  x-position derivative from
// Re sum conj(FFT(G_X)) (2 pi i nu) FFT(X) / N; G_A = IFFT(conj(ramp) FFT(G_X)) / N
template <int N>
__global__ __launch_bounds__(NT) void k_row_adj(JobDev jb, Work w, int l) {
  if (*w.status) return;
  constexpr int RB = rb_adj<N>();
  constexpr int LP = row_lp(N);
  using Ix2 = Lds<N, LP, false>;
  using Ix1 = Lds<N, LP, false>;
  __shared__ float2 buf[2 * RB * LP];
  __shared__ float red[NT / 64];
  const int c = blockIdx.y, y0 = blockIdx.x * RB;
  const int tid = threadIdx.x;
  const size_t off = (static_cast<size_t>(c) * jb.L + l) * N * N + static_cast<size_t>(y0) * N;
  const float2* __restrict__ GXr = w.GX + off;
  float2* __restrict__ Xr = w.X + off;
  const float2* __restrict__ rx = w.ramp + (static_cast<size_t>(c) * 2 + 1) * N;
  const float2* __restrict__ twN = jb.tw_N;
  auto ld = [&](int line, int i) {
    return line < RB ? GXr[line * N + i] : Xr[(line - RB) * N + i];
  };
  auto st = [&](int line, int i, float2 v) { buf[Ix2::at(line, i)] = v; };
  fft_lines<N, false, 2 * RB, NT, LP, false>(buf, twN, ld, st);
  float dsum = 0.f;
  for (int e = tid; e < RB * N; e += NT) {
    const int line = e / N, i = e % N;
    const float2 gh = buf[Ix2::at(line, i)];
    const float2 xh = buf[Ix2::at(line + RB, i)];
    const float nu = 2.0f * static_cast<float>(kPi) * freq(i, N);
    dsum += nu * (gh.y * xh.x - gh.x * xh.y);
    buf[Ix2::at(line, i)] = cmul(gh, cconj(rx[i]));
  }
  __syncthreads();
  constexpr float invN = 1.0f / N;
  auto ld1 = [&](int line, int i) { return buf[Ix1::at(line, i)]; };
  auto st1 = [&](int line, int i, float2 v) { Xr[line * N + i] = cscale(v, invN); };
  fft_lines<N, true, RB, NT, LP, false>(buf, twN, ld1, st1);
  const float s = block_sum(dsum, red);
  if (tid == 0) w.dx_part[(static_cast<size_t>(c) * jb.L + l) * gridDim.x + blockIdx.x] = s * invN;
}

// ---------------------------------------------------- object gradient gather
// Tile of 16 x 64 object pixels; every window of the chunk that overlaps the
// tile adds its G_A values in ascending k.  No atomics: each pixel has one
// owner thread, so the sum order is fixed.
constexpr int kTileW = 64, kTileH = 16;
__global__ __launch_bounds__(NT) void k_obj_gather(JobDev jb, Work w, int l,
                                                   float2* __restrict__ gobj) {
  if (*w.status) return;
  const int N = jb.N;
  const int tx0 = blockIdx.x * kTileW, ty0 = blockIdx.y * kTileH;
  const int tx = threadIdx.x % kTileW, tyb = threadIdx.x / kTileW;  // tyb in [0, 4)
  const int x = tx0 + tx;
  constexpr int PER = kTileH / (NT / kTileW);
  float2 acc[PER];
  float2* __restrict__ G = gobj + static_cast<size_t>(l) * jb.H * jb.W;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int y = ty0 + tyb + q * (NT / kTileW);
    acc[q] = (x < jb.W && y < jb.H) ? G[static_cast<size_t>(y) * jb.W + x] : make_float2(0.f, 0.f);
  }
  const size_t plane = static_cast<size_t>(N) * N;
  for (int c = 0; c < w.C; ++c) {
    int py, px;
    float dy, dx;
    split_pos(jb.pos, w.k0 + c, py, px, dy, dx);
    if (py >= ty0 + kTileH || py + N <= ty0 || px >= tx0 + kTileW || px + N <= tx0) continue;
    const float2* __restrict__ GA = w.X + (static_cast<size_t>(c) * jb.L + l) * plane;
    const int xr = x - px;
    if (xr < 0 || xr >= N) continue;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int yr = ty0 + tyb + q * (NT / kTileW) - py;
      if (yr >= 0 && yr < N) acc[q] = cadd(acc[q], GA[yr * N + xr]);
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int y = ty0 + tyb + q * (NT / kTileW);
    if (x < jb.W && y < jb.H) G[static_cast<size_t>(y) * jb.W + x] = acc[q];
  }
}

// ---------------------------------------------------------------- finalize
__global__ void k_finalize_chunk(JobDev jb, Work w, int n_loss, int n_dy, int n_dx,
                                 float* __restrict__ g_pos, float* __restrict__ g_sigma) {
  if (*w.status) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= w.C) return;
  const int k = w.k0 + c;
  double ls = 0.0;
  for (int i = 0; i < n_loss; ++i) ls += w.loss_part[static_cast<size_t>(c) * n_loss + i];
  w.loss_k[k] = ls;
  float gy = 0.f, gx = 0.f, gs = 0.f;
  for (int l = 0; l < jb.L; ++l) {
    for (int i = 0; i < n_dy; ++i) {
      gy += w.dy_part[(static_cast<size_t>(c) * jb.L + l) * n_dy + i];
      gs += w.sg_part[(static_cast<size_t>(c) * jb.L + l) * n_dy + i];
    }
    for (int i = 0; i < n_dx; ++i) gx += w.dx_part[(static_cast<size_t>(c) * jb.L + l) * n_dx + i];
  }
  if (g_pos) {
    g_pos[2 * k] = gy;
    g_pos[2 * k + 1] = gx;
  }
  if (g_sigma) g_sigma[k] = gs;
}

__global__ void k_loss_total(JobDev jb, Work w, float scale, float* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (*w.status) {
    *loss = __int_as_float(0x7fc00000);
    return;
  }
  double s = 0.0;
  for (int k = 0; k < jb.K; ++k) s += w.loss_k[k];
  *loss = static_cast<float>(s * scale);
}

__global__ void k_adam(float* __restrict__ x, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2) {
  const size_t i0 = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t i = i0; i < n; i += stride) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    x[i] -= lr * (mi * bc1) / (sqrtf(vi * bc2) + eps);
  }
}

// =================================================================== host
namespace {

template <class F>
hipError_t with_N(int N, const F& f) {
  switch (N) {
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 384: return f(std::integral_constant<int, 384>{});
    case 512: return f(std::integral_constant<int, 512>{});
    default: return hipErrorInvalidValue;
  }
}

template <class F, int P, int... Ps>
hipError_t host_pad(int nl, const F& f, IntList<P, Ps...>) {
  if (nl == P) return f(std::integral_constant<int, P>{});
  if constexpr (sizeof...(Ps) > 0) return host_pad(nl, f, IntList<Ps...>{});
  return hipErrorInvalidValue;
}

template <int P, int... Ps>
bool in_list(int nl, IntList<P, Ps...>) {
  if (nl == P) return true;
  if constexpr (sizeof...(Ps) > 0) return in_list(nl, IntList<Ps...>{});
  return false;
}

inline unsigned blocks_for(size_t n, unsigned per) {
  size_t b = (n + per - 1) / per;
  if (b > 65535u * 8u) b = 65535u * 8u;
  return static_cast<unsigned>(b < 1 ? 1 : b);
}

}  // namespace

namespace {
template <int P, int... Ps>
int plan_of(int n, int* out, IntList<P, Ps...>) {
  if (n == P) {
    plan_fill(typename Plan<P>::type{}, out);
    return PlanInfo<P>::passes;
  }
  if constexpr (sizeof...(Ps) > 0) return plan_of(n, out, IntList<Ps...>{});
  return 0;
}
}  // namespace

int plan_radices(int n, int* out) {
  using All = IntList<64, 72, 80, 84, 90, 96, 128, 140, 150, 168, 189, 256, 280, 300, 315, 336,
                      343, 375, 384, 420, 480, 512, 560, 600, 675, 750>;
  return plan_of(n, out, All{});
}

bool supported(int N, int nl) {
  switch (N) {
    case 64: return in_list(nl, PadList<64>::type{});
    case 128: return in_list(nl, PadList<128>::type{});
    case 256: return in_list(nl, PadList<256>::type{});
    case 384: return in_list(nl, PadList<384>::type{});
    case 512: return in_list(nl, PadList<512>::type{});
    default: return false;
  }
}

int rows_per_det_block(int N) {
  switch (N) {
    case 64: return rb_det<64>();
    case 128: return rb_det<128>();
    case 256: return rb_det<256>();
    case 384: return rb_det<384>();
    case 512: return rb_det<512>();
    default: return 1;
  }
}
int rows_per_adj_block(int N) {
  switch (N) {
    case 64: return rb_adj<64>();
    case 128: return rb_adj<128>();
    case 256: return rb_adj<256>();
    case 384: return rb_adj<384>();
    case 512: return rb_adj<512>();
    default: return 1;
  }
}
int col_group_of(int N) { return N <= 256 ? 16 : 8; }

hipError_t launch_fill_zero(float* p, size_t n, hipStream_t s) { return launch_fill_value(p, n, 0.f, s); }

hipError_t launch_fill_value(float* p, size_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, NT)), dim3(NT), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_set_status(int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_set_status, dim3(1), dim3(64), 0, s, status);
  return hipGetLastError();
}

hipError_t launch_validate(const JobDev& jb, int* status, hipStream_t s) {
  if (jb.K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3((jb.K + NT - 1) / NT), dim3(NT), 0, s, jb, status);
  return hipGetLastError();
}

hipError_t launch_prep(const JobDev& jb, const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(w.C), dim3(NT), 0, s, jb, w);
  return hipGetLastError();
}

hipError_t launch_row_fwd(const JobDev& jb, const Work& w, int l, hipStream_t s) {
  return with_N(jb.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    hipLaunchKernelGGL(k_row_fwd<N>, dim3(N / rb_row<N>(), w.C), dim3(NT), 0, s, jb, w, l);
    return hipGetLastError();
  });
}

hipError_t launch_col_fwd(const JobDev& jb, const Work& w, int l, hipStream_t s) {
  return with_N(jb.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    return host_pad(jb.pad[l], [&](auto pc) {
      constexpr int NL = decltype(pc)::value;
      hipLaunchKernelGGL((k_col_fwd<N, NL>), dim3(N / col_group<N>(), w.C), dim3(CNT), 0, s, jb, w, l);
      return hipGetLastError();
    }, typename PadList<N>::type{});
  });
}

hipError_t launch_det(const JobDev& jb, const Work& w, const LossDev& loss, int mode, bool spill,
                      float* out, hipStream_t s) {
  return with_N(jb.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    dim3 grid(N / rb_det<N>(), w.C);
    switch (mode) {
      case 0: hipLaunchKernelGGL((k_det<N, 0>), grid, dim3(NT), 0, s, jb, w, loss, spill, out); break;
      case 1: hipLaunchKernelGGL((k_det<N, 1>), grid, dim3(NT), 0, s, jb, w, loss, spill, out); break;
      case 2: hipLaunchKernelGGL((k_det<N, 2>), grid, dim3(NT), 0, s, jb, w, loss, spill, out); break;
      default: hipLaunchKernelGGL((k_det<N, 3>), grid, dim3(NT), 0, s, jb, w, loss, spill, out); break;
    }
    return hipGetLastError();
  });
}

hipError_t launch_resample_loss(const JobDev& jb, const Work& w, const LossDev& loss, float* out,
                                hipStream_t s) {
  dim3 grid((jb.N * jb.N + NT - 1) / NT, w.C);
  hipLaunchKernelGGL(k_resample_loss, grid, dim3(NT), 0, s, jb, w, loss, out);
  return hipGetLastError();
}

hipError_t launch_resample_T(const JobDev& jb, const Work& w, hipStream_t s) {
  dim3 grid((jb.N * jb.N + NT - 1) / NT, w.C);
  hipLaunchKernelGGL(k_resample_T, grid, dim3(NT), 0, s, jb, w);
  return hipGetLastError();
}

hipError_t launch_col_adj(const JobDev& jb, const Work& w, int l, bool want_probe, hipStream_t s) {
  return with_N(jb.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    return host_pad(jb.pad[l], [&](auto pc) {
      constexpr int NL = decltype(pc)::value;
      hipLaunchKernelGGL((k_col_adj<N, NL>), dim3(N / col_group<N>(), w.C), dim3(CNT), 0, s, jb, w, l,
                         want_probe);
      return hipGetLastError();
    }, typename PadList<N>::type{});
  });
}

hipError_t launch_probe_reduce(const JobDev& jb, const Work& w, float2* g_probe, hipStream_t s) {
  const size_t plane = static_cast<size_t>(jb.N) * jb.N;
  dim3 grid((plane + NT - 1) / NT, jb.L * jb.M);
  hipLaunchKernelGGL(k_probe_reduce, grid, dim3(NT), 0, s, jb, w, g_probe);
  return hipGetLastError();
}

hipError_t launch_row_adj(const JobDev& jb, const Work& w, int l, hipStream_t s) {
  return with_N(jb.N, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    hipLaunchKernelGGL(k_row_adj<N>, dim3(N / rb_adj<N>(), w.C), dim3(NT), 0, s, jb, w, l);
    return hipGetLastError();
  });
}

hipError_t launch_obj_gather(const JobDev& jb, const Work& w, int l, float2* g_object,
                             hipStream_t s) {
  dim3 grid((jb.W + kTileW - 1) / kTileW, (jb.H + kTileH - 1) / kTileH);
  hipLaunchKernelGGL(k_obj_gather, grid, dim3(NT), 0, s, jb, w, l, g_object);
  return hipGetLastError();
}

hipError_t launch_finalize_chunk(const JobDev& jb, const Work& w, int n_loss, float* g_pos,
                                 float* g_sigma, hipStream_t s) {
  const int n_dy = jb.N / col_group_of(jb.N);
  const int n_dx = jb.N / rows_per_adj_block(jb.N);
  hipLaunchKernelGGL(k_finalize_chunk, dim3((w.C + 63) / 64), dim3(64), 0, s, jb, w, n_loss, n_dy,
                     n_dx, g_pos, g_sigma);
  return hipGetLastError();
}

hipError_t launch_loss_total(const JobDev& jb, const Work& w, float scale, float* loss,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, s, jb, w, scale, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* x, const float* g, float* m, float* v, size_t n, float lr,
                       float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, NT)), dim3(NT), 0, s, x, g, m, v, n, lr, beta1,
                     beta2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace ptycho
