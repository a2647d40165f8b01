// kernels.hip - gfx950 kernels of the ptychography loss + gradient path.
//
// Per position chunk the path runs (Eq. 2 order, then its adjoint):
//   prep      : p_k = floor(s_k + 1/2), delta_k, phase ramps exp(+2 pi i f delta)
//   row_fwd   : gather object rows, x-shift (FFT, ramp, IFFT)            -> X
//   col_fwd   : y-shift of X columns, times sigma P_{l,m} for every mode,
//               first (column) pass of the padded, cropped DFT            -> Y
//   det       : second (row) pass of the DFT, incoherent sum over l and m,
//               background, loss and its derivative, then per plane the far
//               field again from Y (not stored), 2 g Psi, adjoint row DFT  -> Z (in Y)
//   col_adj   : adjoint column DFT -> chi; G_Osh = sum_m conj(sigma P) chi;
//               probe-gradient terms conj(sigma Osh) chi (in Y); sigma and
//               y-position derivatives; adjoint y-shift                  -> GX
//   probe_red : ordered sum over positions of the probe-gradient terms
//   row_adj   : adjoint x-shift -> G_A (in X); x-position derivative
//   obj_gather: object gradient tiles gather G_A of every overlapping window
//               in ascending k (no atomics)
//   finalize  : ordered per-position sums of the partials
// Optional stages: chirp tables of the exact-ratio propagator (Bluestein,
// FFT length 2N, at the start of a call), the background-gradient sum, the
// alpha-derivative terms (detector and column adjoint), the amplitude
// regulariser (once per call, after the data gradient).  Wavelengths and
// sample modes are "slots" s = l Ns + n; the probe of slot s is P_{s / Ns}.
// The C ABI (api.cpp) sequences these launches on one stream.
//
// Every launch covers the work of one or more jobs: the job descriptors live
// in device memory (JobDev) and each launch receives a list of segments
// (job, wavelength, first unit); block b handles unit b / GX, and the
// segment that contains it names its job and wavelength.  A single job is
// the one-segment case, so the multi-job (serving) path and the single-job
// path run the same kernels.
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

// Exact-ratio propagator (chirp z-transform, Bluestein's method): per axis
// Psi[j] = alpha^-1/2 sum_r psi[r] exp(-2 pi i u_j r / alpha), u_j = j - N/2,
// written as cout[j] sum_r (cin[r] psi[r]) h[j - r] with the chirps
// cin[r] = exp(-i pi r^2 / alpha), cout[j] = alpha^-1/2 exp(-i pi u_j^2 / alpha)
// and h[t] = exp(+i pi (t - N/2)^2 / alpha).  The lags j - r span 2N - 1
// values, so a circular convolution of length 2N evaluates it exactly:
// FFT, times the kernel's DFT (precomputed per call), inverse FFT.  The
// length 2N is never a zero-padded DFT size of the same N, so it marks the
// exact-ratio instances of the DFT-size-templated kernels.
template <int N> constexpr int czt_nb() { return 2 * N; }
template <class List, int X> struct Append;
template <int... Ps, int X> struct Append<IntList<Ps...>, X> { using type = IntList<Ps..., X>; };
// DFT lengths of the column kernels: the pads, then the Bluestein length.
template <int N> using ColList = typename Append<typename PadList<N>::type, czt_nb<N>()>::type;
// Row lengths of a detector-kernel instance.
template <int N, bool WIDE>
using DetList = std::conditional_t<WIDE, ColList<N>, typename PadList<N>::type>;
static_assert(czt_nb<64>() > PadList<64>::max && czt_nb<128>() > PadList<128>::max &&
              czt_nb<256>() > PadList<256>::max && czt_nb<384>() > PadList<384>::max &&
              czt_nb<512>() > PadList<512>::max, "the Bluestein length must not be a pad size");

template <int N> constexpr int rb_row() { return N == 64 ? 32 : (N <= 256 ? 16 : 8); }
template <int N> constexpr int rb_det() { return N <= 128 ? 16 : (N == 512 ? 4 : 8); }
template <int N> constexpr int rb_adj() { return N <= 128 ? 16 : (N == 512 ? 4 : 8); }
template <int N> constexpr int col_group() { return N <= 256 ? 16 : 8; }
// Column group of the column adjoint for DFT size nl.  With N = 256 and the
// sizes listed, 8 columns per block keep the live registers within 128 VGPRs,
// so two 512-thread blocks share a CU (4 waves per SIMD instead of 2; column
// adjoint of 400 positions x 4 wavelengths x 3 modes at N = 256: 2.86 -> 2.65
// ms per step).  The other instances spill at that bound (exact-ratio length
// 2N: 3.97 -> 6.9 ms) and keep 16 columns.
__host__ __device__ constexpr bool adj_narrow(int N, int nl) {
  return N == 256 && (nl == 256 || nl == 280 || nl == 315 || nl == 343);
}
__host__ __device__ constexpr int col_group_adj(int N, int nl) {
  return adj_narrow(N, nl) ? 8 : (N <= 256 ? 16 : 8);
}
// Row pitch (in elements) of the block-wide column adjoint's LDS transform
// buffer, whose rows hold the G columns of one element index.  Unpadded
// rows for the zero-padded sizes at N >= 384 (3 harmonics x 4 modes at
// N = 384: 14.4 -> 14.1 ms per step; the paired kernel, while its transforms
// were block-wide too, went 172.3 -> 162.8 ms at 5 x 8, N = 512); one
// element of padding at N <= 256, where the unpadded rows were slower
// (4 x 3 at N = 256: +0.03 ms), and for the Bluestein lengths 2N, whose
// instances then spill.  Pitches G + 2 and G + 3 were no faster.
__host__ __device__ constexpr int col_adj_lp(int N, int nl, int G) {
  return (N >= 384 && nl != 2 * N) ? G : G + 1;
}
// Row pitch of the grouped-position column adjoint's transposed tile: the
// detector rows' pitch (with their skew at lengths that are multiples of 16),
// padded to 32 / G modulo 32 so that the coalesced tile stores and reads
// (G rows x 32 / G elements per half-wave) meet distinct banks.
__host__ __device__ constexpr int pair_row_pitch(int nl, int G) {
  return row_lp(nl) + ((32 / G - row_lp(nl) % 32) + 32) % 32;
}
// Threads per block of the column adjoint instance.
__host__ __device__ constexpr int col_adj_threads(int N, int nl) { return CNT; }
// Row stride of the column adjoint's per-block partial sums ([C][L][stride]):
// the most blocks per column set of any instance of N.
__host__ __device__ constexpr int adj_stride(int N) { return N <= 128 ? N / 16 : N / 8; }

template <class F, int P, int... Ps>
__device__ __forceinline__ void pad_switch(int nl, const F& f, IntList<P, Ps...>) {
  if (nl == P) {
    f(std::integral_constant<int, P>{});
  } else {
    if constexpr (sizeof...(Ps) > 0) pad_switch(nl, f, IntList<Ps...>{});
  }
}

__device__ __forceinline__ void split_pos(const gf32* __restrict__ pos, int k, int& py, int& px,
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


__device__ __forceinline__ int rb_adj_dev(int N) { return N <= 128 ? 16 : (N == 512 ? 4 : 8); }
__device__ __forceinline__ int rb_det_dev(int N) { return N <= 128 ? 16 : (N == 512 ? 4 : 8); }

// Mixed Poisson-Gaussian noise, Gaussian approximation with variance I + v:
// ell = (I - m)^2 / (I + v) + ln(I + v) and its derivative in I.
__device__ __forceinline__ void mixed_loss(float I, float m, float v, float& ell, float& dell) {
  const float q = I + v, d = I - m, r = d / q;
  ell = d * r + logf(q);
  dell = 2.f * r - r * r + 1.f / q;
}

// ------------------------------------------------------- work decomposition
// Largest s with segs[s].unit0 <= unit (segs sorted, segs[0].unit0 == 0).
// The arguments are wave-uniform, so the search runs on the scalar unit.
__device__ __forceinline__ int find_seg(const Seg* __restrict__ segs, int nseg, int unit) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].unit0 <= unit) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct UnitRef {
  const JobDev* jb;
  int l;      // wavelength (or sub-selector) of the segment
  int u;      // unit index inside the segment
  int sub;    // block index inside the unit
};

template <int GX>
__device__ __forceinline__ UnitRef decode(const Launch& la, int b = -1) {
  if (b < 0) b = blockIdx.x;
  const int unit = b / GX;
  const int s = find_seg(la.segs, la.nseg, unit);
  const Seg sg = la.segs[s];
  return UnitRef{la.jobs + sg.job, sg.l, unit - sg.unit0, b - unit * GX};
}

// Copies a table carried in the launch's own argument block to device
// memory: the payload is the first kernel argument, so it starts at the
// kernel-argument segment pointer.
// decode() for the column and detector kernels.  Workgroups are dealt to the
// 8 XCDs in turn (block b to XCD b mod 8), and each XCD has its own L2.
// Renumbering the blocks so that each XCD receives one contiguous run of block
// indices keeps the neighbouring column groups of a plane, whose 64-byte
// column segments share 128-byte lines, in the same L2, and the row blocks of
// one position together.  Per step, N = 256 (400 positions, 4 wavelengths x 3
// modes): column adjoint 2.65 -> 2.37 ms; N = 512 (2500 positions, 5 x 8):
// column adjoint 216 -> 178 ms, column forward 105 -> 95 ms, detector
// 188 -> 181 ms.
template <int GX>
__device__ __forceinline__ UnitRef decode_xcd(const Launch& la) {
  const int n = gridDim.x, b = blockIdx.x;
  const int x = b & 7, i = b >> 3, q = n >> 3, rem = n & 7;
  // XCD x holds q + (x < rem) blocks; they take the run starting at x q + min(x, rem)
  return decode<GX>(la, x * q + min(x, rem) + i);
}

// decode() for the column kernels of windows N >= 384: block b runs on XCD
// x = b mod 8, and XCD x takes the column groups [x GX/8, (x+1) GX/8) of
// every unit, units in ascending order.  Each XCD's L2 then keeps the probe columns of its own
// column groups (every mode) while it works through the positions, instead
// of fetching the whole probe of the wavelength again for every position;
// neighbouring groups, whose 64-byte column segments share 128-byte lines,
// stay on one XCD.  Without it every launch of the column forward and the
// column adjoint (512 x 512 probe, 8 modes, 2500 positions) read the probe
// once per position: about 42 GB of L2 misses on top of ~47 GB of planes
// (column forward 98.6 -> 81.2 ms per step).  For N = 256 (3 modes, probe
// 1.5 MB) the per-XCD runs of whole positions stay faster (column adjoint of
// 400 positions x 4 wavelengths: 2.44 against 2.59 ms).
template <int GX>
__device__ __forceinline__ UnitRef decode_cols(const Launch& la) {
  if constexpr (GX % 8 == 0 && GX * 8 >= 384) {
    constexpr int PER = GX / 8;
    const int b = blockIdx.x, x = b & 7, i = b >> 3;
    const int unit = i / PER, sub = x * PER + (i - (i / PER) * PER);
    return decode<GX>(la, unit * GX + sub);
  } else {
    return decode_xcd<GX>(la);
  }
}

__global__ void k_write_table(TablePayload payload, int* __restrict__ dst, int n) {
  (void)payload;
  const __attribute__((address_space(4))) int* src =
      (const __attribute__((address_space(4))) int*)__builtin_amdgcn_kernarg_segment_ptr();
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// ------------------------------------------------------------------ utility
// Zero the requested gradient outputs.  Segment l selects the array
// (0 object, 1 probe, 2 positions, 3 sigma); units are 1024-float blocks.
__global__ __launch_bounds__(NT) void k_zero_grads(Launch la) {
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  gf32* __restrict__ p = gmem(jb.grad_flat[r.l]);
  const long long n = jb.flat_n[r.l];
  const long long base = static_cast<long long>(r.u) * 1024;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long long i = base + threadIdx.x + q * NT;
    if (i < n) p[i] = 0.f;
  }
}

__global__ void k_set_status(Launch la) {
  const UnitRef r = decode<1>(la);
  if (threadIdx.x == 0) *gmem(r.jb->status) = 0;
}

// units: blocks of 256 positions
__global__ __launch_bounds__(NT) void k_validate(Launch la) {
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  const int k = r.u * NT + threadIdx.x;
  if (k >= jb.K) return;
  const gf32* pos = gmem(jb.pos);
  const float sy = pos[2 * k], sx = pos[2 * k + 1];
  bool bad = !(isfinite(sy) && isfinite(sx));
  if (!bad) {
    const float fy = floorf(sy + 0.5f), fx = floorf(sx + 0.5f);
    bad = fy < 0.f || fx < 0.f || fy + jb.N > jb.H || fx + jb.N > jb.W;
  }
  if (bad) *gmem(jb.status) = kERange;  // every writer stores the same value
}

// ramps[c][0][f] = exp(2 pi i nu_f delta_y), ramps[c][1][f] likewise for x
__global__ __launch_bounds__(NT) void k_prep(Launch la) {
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  const int c = r.u, k = la.iter * jb.C + c;
  int py, px;
  float dy, dx;
  split_pos(gmem(jb.pos), k, py, px, dy, dx);
  const int N = jb.N;
  for (int i = threadIdx.x; i < 2 * N; i += NT) {
    const int f = i % N;
    const double d = (i < N) ? static_cast<double>(dy) : static_cast<double>(dx);
    const double nu = static_cast<double>(f < N / 2 ? f : f - N) / N;
    double sn, cs;
    sincospi(2.0 * nu * d, &sn, &cs);
    stv(gmem(jb.ramp), static_cast<size_t>(c) * 2 * N + i,
        make_float2(static_cast<float>(cs), static_cast<float>(sn)));
  }
}

// ------------------------------------------ exact-ratio propagator tables
// Per (job, wavelength l with alpha_l > 0) the table of czt_nb: cin[N],
// cout[N] and hk[2N] = DFT_2N(h) / 2N, h[t] = exp(+i pi (t' - N/2)^2 / alpha)
// at lag t' = t (t < N) or t - 2N (t > N), h[N] = 0 (that lag never occurs).
// Evaluated in float64 with the chirp arguments reduced exactly
// (r^2 mod 2 alpha) and rounded to float32 once; the DFT is a plain ordered
// sum, so the table is the same in every call.
// units: (job, l) x czt_table_blocks(N): chirp blocks, then kernel blocks
constexpr int kCztMaxNB = 1024;
__global__ __launch_bounds__(NT) void k_czt_tables(Launch la) {
  __shared__ double2 hk[kCztMaxNB];
  __shared__ double2 tw[kCztMaxNB];
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  const int l = r.l, N = jb.N, NB = 2 * N;
  const double a = jb.czt_alpha[l];
  gf2* __restrict__ tb = gmem(jb.czt[l]);
  const int CB = (2 * N + NT - 1) / NT;  // chirp blocks
  if (r.u < CB) {
    const int e = r.u * NT + threadIdx.x;
    double sn, cs;
    if (e < N) {
      sincospi(-fmod(static_cast<double>(e) * e, 2.0 * a) / a, &sn, &cs);
      stv(tb, e, make_float2(static_cast<float>(cs), static_cast<float>(sn)));
    } else if (e < 2 * N) {
      const double u = static_cast<double>(e - N - N / 2);
      sincospi(-fmod(u * u, 2.0 * a) / a, &sn, &cs);
      const double sc = 1.0 / sqrt(a);
      stv(tb, e, make_float2(static_cast<float>(cs * sc), static_cast<float>(sn * sc)));
    }
    return;  // block-uniform
  }
  for (int t = threadIdx.x; t < NB; t += NT) {
    double sn = 0.0, cs = 0.0;
    if (t != N) {
      const double d = static_cast<double>((t < N ? t : t - NB) - N / 2);
      sincospi(fmod(d * d, 2.0 * a) / a, &sn, &cs);
    }
    hk[t] = make_double2(cs, sn);
    sincospi(-2.0 * static_cast<double>(t) / NB, &sn, &cs);
    tw[t] = make_double2(cs, sn);
  }
  __syncthreads();
  const int f = (r.u - CB) * NT + threadIdx.x;
  if (f >= NB) return;
  double re = 0.0, im = 0.0;
  int q = 0;  // f t mod NB
  for (int t = 0; t < NB; ++t) {
    const double2 h = hk[t], w = tw[q];
    re += h.x * w.x - h.y * w.y;
    im += h.x * w.y + h.y * w.x;
    q += f;
    if (q >= NB) q -= NB;
  }
  stv(tb, 2 * N + f, make_float2(static_cast<float>(re / NB), static_cast<float>(im / NB)));
}

// ------------------------------------------------------------- row forward
// X[c][l][y][:] = IFFT_x( ramp_x * FFT_x( O_l[p_y + y][p_x : p_x + N] ) ) / N
// units: (l, c) positions of every wavelength
template <int N>
__global__ __launch_bounds__(NT) void k_row_fwd(Launch la) {
  constexpr int RB = rb_row<N>();
  // each wave transforms RW of the block's RB rows in an LDS region of its
  // own, so the passes need no workgroup barriers
  constexpr int RW = RB / (NT / 64);
  static_assert(RB % (NT / 64) == 0, "whole rows per wave");
  const UnitRef r = decode<N / RB>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  constexpr int LP = row_lp(N);
  using Ix = Lds<N, LP, false>;
  __shared__ float2 buf[RB * LP];
  const int wv = static_cast<int>(threadIdx.x >> 6);
  lf2* const bufw = (lf2*)buf + wv * RW * LP;
  const int l = r.l, c = r.u, k = la.iter * jb.C + c;
  const int y0 = r.sub * RB + wv * RW;
  int py, px;
  float dy, dx;
  split_pos(gmem(jb.pos), k, py, px, dy, dx);
  const gf2* __restrict__ O = gmem(jb.object) + static_cast<size_t>(l) * jb.H * jb.W +
                              static_cast<size_t>(py + y0) * jb.W + px;
  const gf2* __restrict__ rx = gmem(jb.ramp) + (static_cast<size_t>(c) * 2 + 1) * N;
  const float2* __restrict__ tw = jb.tw_N;
  const int Wd = jb.W;
  auto ld_obj = [&](int line, int i) { return ldv(O, line * Wd + i); };
  auto st_ramp = [&](int line, int i, float2 v) { stv(bufw, Ix::at(line, i), cmul(v, ldv(rx, i))); };
  fft_lines<N, false, RW, 64, LP, false>(bufw, tw, ld_obj, st_ramp);
  gf2* __restrict__ X = gmem(jb.X) + ((static_cast<size_t>(c) * jb.L + l) * N + y0) * N;
  constexpr float inv = 1.0f / N;
  auto ld_buf = [&](int line, int i) { return ldv(bufw, Ix::at(line, i)); };
  // streaming stores of whole rows (row forward, 400 positions x 4 wavelengths
  // at N = 256: 0.266 -> 0.225 ms; 900 x 3 at N = 384: 1.02 -> 0.87 ms)
  auto st_x = [&](int line, int i, float2 v) { stv_nt(X, line * N + i, cscale(v, inv)); };
  fft_lines<N, true, RW, 64, LP, false>(bufw, tw, ld_buf, st_x);
}

// ---------------------------------------------------------- column forward
// Osh = y-shift of X columns; Y_m = (1/sqrt(NL)) crop( DFT_NL_y( sigma P_m Osh ) )
// units: (l, c) for the wavelengths whose DFT size is NL
// Waves per SIMD the column forward is compiled for.  Two instances that
// need a few more than 128 VGPRs unbounded are held to 128, so that two
// 512-thread blocks share a CU: DFT size 750 at N = 512 (27.8 -> 18.6 ms per
// launch, no spills) and the Bluestein length 768 at N = 384 (140 VGPRs ->
// 128 with 17 spilled; exact-ratio, 3 harmonics x 4 modes: column forward
// 19.2 -> 15.1 ms per step).  The Bluestein length 512 at N = 256 was slower
// so bounded (29 spilled; 3.0 -> 3.16 ms) and keeps 156 VGPRs.
__host__ __device__ constexpr int col_fwd_waves(int N, int nl) {
  return ((N == 512 && nl == 750) || (N == 384 && nl == 768)) ? 4 : 2;
}

template <int N, int NL>
__global__ __launch_bounds__(CNT, col_fwd_waves(N, NL)) void k_col_fwd(Launch la) {
  constexpr int G = col_group<N>();
  const UnitRef r = decode_cols<N / G>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  constexpr int LP = G + 1;
  constexpr int NE = N * G / CNT;
  static_assert(N * G % CNT == 0, "natural layout");
  __shared__ float2 buf[NL * LP];
  const int l = r.l, c = r.u, k = la.iter * jb.C + c, x0 = r.sub * G;
  const int tid = threadIdx.x;
  const gf2* __restrict__ X = gmem(jb.X) + (static_cast<size_t>(c) * jb.L + l) * N * N + x0;
  const gf2* __restrict__ ry = gmem(jb.ramp) + static_cast<size_t>(c) * 2 * N;
  const float2* __restrict__ twN = jb.tw_N;
  const float2* __restrict__ twL = jb.tw_pad[l];

  auto ld_x = [&](int line, int i) { return ldv(X, i * N + line); };
  auto st_ramp = [&](int line, int i, float2 v) { buf[i * LP + line] = cmul(v, ldv(ry, i)); };
  fft_lines<N, false, G, CNT, LP, true>(buf, twN, ld_x, st_ramp);
  auto ld_buf = [&](int line, int i) { return buf[i * LP + line]; };
  auto st_buf = [&](int line, int i, float2 v) { buf[i * LP + line] = v; };
  fft_lines<N, true, G, CNT, LP, true>(buf, twN, ld_buf, st_buf);

  const float sg = (jb.sigma ? gmem(jb.sigma)[k] : 1.0f) / N;
  float2 o[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * CNT, line = e % G, i = e / G;
    o[q] = cscale(buf[i * LP + line], sg);
  }
  __syncthreads();
  const float ps = jb.pad_scale[l];
  for (int m = 0; m < jb.M; ++m) {
    const gf2* __restrict__ P =
        gmem(jb.probe) + (static_cast<size_t>(l / jb.Ns) * jb.M + m) * N * N + x0;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * CNT, line = e % G, i = e / G;
      buf[i * LP + line] = cmul(ldv(P, i * N + line), o[q]);
    }
    __syncthreads();
    gf2* __restrict__ Y =
        gmem(jb.Y) + ((static_cast<size_t>(c) * jb.L + l) * jb.M + m) * N * N + x0;
    if constexpr (NL == czt_nb<N>()) {
      // exact ratio: cin psi -> FFT -> times the kernel DFT -> IFFT -> cout
      const gf2* __restrict__ tb = opaque_table(jb.czt[l]);  // loads stay in the mode loop
      auto ld_c = [&](int line, int t) {
        return t < N ? cmul(buf[t * LP + line], ldv(tb, t)) : make_float2(0.f, 0.f);
      };
      auto st_h = [&](int line, int t, float2 v) { buf[t * LP + line] = cmul(v, ldv(tb, 2 * N + t)); };
      fft_lines<NL, false, G, CNT, LP, true>(buf, twL, ld_c, st_h);
      auto ld_b = [&](int line, int t) { return buf[t * LP + line]; };
      auto st_y = [&](int line, int t, float2 v) {
        if (t < N) {
          if constexpr (G == 16) stv_nt(Y, t * N + line, cmul(v, ldv(tb, N + t)));
          else stv(Y, t * N + line, cmul(v, ldv(tb, N + t)));
        }
      };
      fft_lines<NL, true, G, CNT, LP, true>(buf, twL, ld_b, st_y);
    } else {
      auto ld_psi = [&](int line, int t) {
        return t < N ? buf[t * LP + line] : make_float2(0.f, 0.f);
      };
      auto st_y = [&](int line, int t, float2 v) {
        int u = t + N / 2;
        if (u >= NL) u -= NL;
        if (u < N) {
          // 16-column groups write whole 128-byte lines: streaming stores
          // (400 positions x 4 wavelengths x 3 modes at N = 256: 1.20 ->
          // 1.14 ms per step); 8-column groups keep ordinary stores, whose
          // line halves L2 merges
          if constexpr (G == 16) stv_nt(Y, u * N + line, cscale(v, ps));
          else stv(Y, u * N + line, cscale(v, ps));
        }
      };
      fft_lines<NL, false, G, CNT, LP, true>(buf, twL, ld_psi, st_y);
    }
  }
}

// ------------------------------------------------------------ detector rows
// The detector-row passes below run per wave: the RB rows (and `buf`, `acc`,
// `Yr`, `psi`) are the calling wave's own, and the transforms synchronise the
// wave only (see fft_sync), so a wave waiting for its rows' loads does not
// hold the other waves of the block.
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
  fft_lines<NL, false, RB, 64, LP, false>(buf, twL, ld, st);
}

// Zero-padded adjoint row pass: recomputes Psi = crop(DFT(Y)) from the kept
// column output instead of reading a stored Psi, scales by g2 in LDS and
// applies the adjoint transform Z[u][:] = (1/sqrt(NL)) DFT^H(embed(g2 Psi))[0:N],
// written over Y.  One more row transform, and one plane written and read
// less per (l, m): neutral where the kernel is issue-bound, faster where it
// is HBM-bound (N = 512, M = 8: 205 -> 188 ms per step).
template <int N, int NL, int RB>
__device__ __noinline__ void det_rows_recomp(lf2* buf, const lf32* acc, gf2* __restrict__ Yr,
                                             const gf2* __restrict__ twL, float ps) {
  constexpr int LP = row_lp(NL);
  using Ix = Lds<NL, LP, false>;
  auto ld = [&](int line, int t) { return t < N ? ldv(Yr, line * N + t) : make_float2(0.f, 0.f); };
  auto st = [&](int line, int t, float2 v) {
    int u = t + N / 2;
    if (u >= NL) u -= NL;
    if (u < N) stv(buf, Ix::at(line, u), cscale(v, ps * acc[line * N + u]));
  };
  fft_lines<NL, false, RB, 64, LP, false>(buf, twL, ld, st);
  auto ld2 = [&](int line, int t) {
    int u = t + N / 2;
    if (u >= NL) u -= NL;
    return u < N ? ldv(buf, Ix::at(line, u)) : make_float2(0.f, 0.f);
  };
  auto st2 = [&](int line, int t, float2 v) {
    if (t < N) stv(Yr, line * N + t, cscale(v, ps));
  };
  fft_lines<NL, true, RB, 64, LP, false>(buf, twL, ld2, st2);
}

// Exact-ratio row pass: Psi[u][:] = cout (IFFT( FFT(cin Y[u][:]) hk ))[0:N],
// acc += |Psi|^2 (tb: the wavelength's chirp table, see czt_nb).
template <int N, int NB, int RB>
__device__ __noinline__ void det_rows_fwd_czt(lf2* buf, lf32* acc, gf2* __restrict__ Yr,
                                              const gf2* __restrict__ twB,
                                              const gf2* __restrict__ tb, bool keep) {
  constexpr int LP = row_lp(NB);
  using Ix = Lds<NB, LP, false>;
  auto ld = [&](int line, int t) {
    return t < N ? cmul(ldv(Yr, line * N + t), ldv(tb, t)) : make_float2(0.f, 0.f);
  };
  auto st = [&](int line, int t, float2 v) { stv(buf, Ix::at(line, t), cmul(v, ldv(tb, 2 * N + t))); };
  fft_lines<NB, false, RB, 64, LP, false>(buf, twB, ld, st);
  auto ld2 = [&](int line, int t) { return ldv(buf, Ix::at(line, t)); };
  auto st2 = [&](int line, int t, float2 v) {
    if (t < N) {
      v = cmul(v, ldv(tb, N + t));
      if (keep) stv(Yr, line * N + t, v);
      acc[line * N + t] += cabs2(v);
    }
  };
  fft_lines<NB, true, RB, 64, LP, false>(buf, twB, ld2, st2);
}

// Its adjoint: Z[u][:] = conj(cin) (IFFT( FFT(conj(cout) g2 Psi[u][:]) conj(hk) ))[0:N],
// written over Psi.
template <int N, int NB, int RB>
__device__ __noinline__ void det_rows_adj_czt(lf2* buf, const lf32* acc, gf2* __restrict__ Yr,
                                              const gf2* __restrict__ twB,
                                              const gf2* __restrict__ tb) {
  constexpr int LP = row_lp(NB);
  using Ix = Lds<NB, LP, false>;
  auto ld = [&](int line, int t) {
    return t < N ? cmulconj(ldv(tb, N + t), cscale(ldv(Yr, line * N + t), acc[line * N + t]))
                 : make_float2(0.f, 0.f);
  };
  auto st = [&](int line, int t, float2 v) { stv(buf, Ix::at(line, t), cmulconj(ldv(tb, 2 * N + t), v)); };
  fft_lines<NB, false, RB, 64, LP, false>(buf, twB, ld, st);
  auto ld2 = [&](int line, int t) { return ldv(buf, Ix::at(line, t)); };
  auto st2 = [&](int line, int t, float2 v) {
    if (t < N) stv(Yr, line * N + t, cmulconj(ldv(tb, t), v));
  };
  fft_lines<NB, true, RB, 64, LP, false>(buf, twB, ld2, st2);
}

// Exact-ratio adjoint row pass that also returns this thread's share of the
// detector-side terms of dL/d alpha (Y kept, Psi recomputed):
//   Psi = F_x Y, Psi_s = F_x (s Y) (s the column index), G = g2 Psi,
//   -(1/alpha) Re<G, Psi> + (2 pi / alpha^2) sum u_i Re(i conj(G) Psi_s)
// (the x-axis factor and the normalisation of dPsi/d alpha), then
// Z = F_x^H G written over Y.  psi: LDS [RB][N] holding Psi.
template <int N, int NB, int RB>
__device__ __noinline__ float det_rows_adj_czt_ratio(lf2* buf, lf2* psi, const lf32* acc,
                                                     gf2* __restrict__ Yr,
                                                     const gf2* __restrict__ twB,
                                                     const gf2* __restrict__ tb, float inv_a,
                                                     float c2) {
  constexpr int LP = row_lp(NB);
  using Ix = Lds<NB, LP, false>;
  auto st_h = [&](int line, int t, float2 v) { stv(buf, Ix::at(line, t), cmul(v, ldv(tb, 2 * N + t))); };
  auto ld_b = [&](int line, int t) { return ldv(buf, Ix::at(line, t)); };
  // Psi
  auto ld_y = [&](int line, int t) {
    return t < N ? cmul(ldv(Yr, line * N + t), ldv(tb, t)) : make_float2(0.f, 0.f);
  };
  fft_lines<NB, false, RB, 64, LP, false>(buf, twB, ld_y, st_h);
  auto st_psi = [&](int line, int t, float2 v) {
    if (t < N) stv(psi, line * N + t, cmul(v, ldv(tb, N + t)));
  };
  fft_lines<NB, true, RB, 64, LP, false>(buf, twB, ld_b, st_psi);
  // Psi_s and the terms
  auto ld_sy = [&](int line, int t) {
    return t < N ? cscale(cmul(ldv(Yr, line * N + t), ldv(tb, t)), static_cast<float>(t))
                 : make_float2(0.f, 0.f);
  };
  fft_lines<NB, false, RB, 64, LP, false>(buf, twB, ld_sy, st_h);
  float ta = 0.f, tc = 0.f;
  auto st_terms = [&](int line, int t, float2 v) {
    if (t < N) {
      const float2 ps = cmul(v, ldv(tb, N + t));
      const float g2 = acc[line * N + t];
      const float2 pv = ldv(psi, line * N + t);
      const float2 G = cscale(pv, g2);
      ta += g2 * cabs2(pv);
      tc += static_cast<float>(t - N / 2) * (G.y * ps.x - G.x * ps.y);
    }
  };
  fft_lines<NB, true, RB, 64, LP, false>(buf, twB, ld_b, st_terms);
  // Z = F_x^H G over Y
  auto ld_g = [&](int line, int t) {
    return t < N ? cmulconj(ldv(tb, N + t), cscale(ldv(psi, line * N + t), acc[line * N + t]))
                 : make_float2(0.f, 0.f);
  };
  auto st_hc = [&](int line, int t, float2 v) { stv(buf, Ix::at(line, t), cmulconj(ldv(tb, 2 * N + t), v)); };
  fft_lines<NB, false, RB, 64, LP, false>(buf, twB, ld_g, st_hc);
  auto st_z = [&](int line, int t, float2 v) {
    if (t < N) stv(Yr, line * N + t, cmulconj(ldv(tb, t), v));
  };
  fft_lines<NB, true, RB, 64, LP, false>(buf, twB, ld_b, st_z);
  return c2 * tc - inv_a * ta;
}

// MODE 0: fused forward + loss + adjoint; 1: forward, write I + B to out;
// 2: adjoint from g rows in the resampling buffer; 3: forward + loss only.
// `spill` (MODE 1) writes Psi back over Y for a later MODE 2.
// VAR 1: the instance for launches with exact-ratio wavelengths (rows of
// 2N); VAR 2: as 1, for jobs that want dL/d alpha (the exact-ratio
// wavelengths keep Y instead of Psi, and the adjoint recomputes Psi).
// units: positions c
template <int N, int MODE, int VAR>
__global__ __launch_bounds__(NT) void k_det(Launch la, LossDev loss, bool spill) {
  constexpr int RB = rb_det<N>();
  using Rows = DetList<N, (VAR >= 1)>;
  const UnitRef r = decode_xcd<N / RB>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  constexpr int LPMAX = max_row_lp(Rows{});
  __shared__ float2 buf[RB * LPMAX];
  __shared__ float acc[RB * N];
  __shared__ float red[NT / 64];
  __shared__ float2 psi[VAR == 2 ? RB * N : 1];
  // exact-ratio wavelength whose alpha-derivative this call computes
  auto ratio_l = [&](int l) { return VAR == 2 && jb.g_ratio != nullptr && jb.czt[l] != nullptr; };
  const int c = r.u, k = la.iter * jb.C + c;
  // Each wave owns RW of the block's RB rows: their transforms, intensities,
  // loss derivatives and adjoint rows; the waves meet only in the block sums.
  constexpr int RW = RB / (NT / 64);
  static_assert(RB % (NT / 64) == 0, "whole rows per wave");
  const int wv = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
  const int u0 = r.sub * RB + wv * RW;  // first row of this wave
  lf2* const bufw = (lf2*)buf + wv * RW * LPMAX;
  lf32* const accw = (lf32*)acc + wv * RW * N;
  lf2* const psiw = (lf2*)psi + (VAR == 2 ? wv * RW * N : 0);
  const size_t plane = static_cast<size_t>(N) * N;
  auto wave_fence = [] {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };

  if (MODE != 2) {
    for (int e = lane; e < RW * N; e += 64) accw[e] = 0.f;
    wave_fence();
    for (int l = 0; l < jb.L; ++l) {
      const float ps = jb.pad_scale[l];
      const float2* twL = jb.tw_pad[l];
      const int nl = jb.pad[l];
      // Psi is kept for the adjoint only on exact-ratio rows (whose recompute
      // costs two transforms) of jobs that do not want dL/d alpha; zero-padded
      // rows keep Y and the adjoint recomputes Psi from it
      const bool keep = ((MODE == 0) || (MODE == 1 && spill)) && jb.czt[l] &&
                        !(jb.g_ratio && jb.czt[l]);
      for (int m = 0; m < jb.M; ++m) {
        gf2* Yr = gmem(jb.Y) + ((static_cast<size_t>(c) * jb.L + l) * jb.M + m) * plane +
                  static_cast<size_t>(u0) * N;
        pad_switch(nl, [&](auto nlc) {
          constexpr int NL = decltype(nlc)::value;
          if constexpr (NL == czt_nb<N>())
            det_rows_fwd_czt<N, NL, RW>(bufw, accw, Yr, gmem(twL), gmem(jb.czt[l]), keep);
          else
            det_rows_fwd<N, NL, RW>(bufw, accw, Yr, gmem(twL), ps, keep);
        }, Rows{});
      }
    }
    // acc = sum_{l,m} |Psi|^2 for this wave's rows
    float lsum = 0.f;
    for (int e = lane; e < RW * N; e += 64) {
      const int line = e / N, x = e % N;
      const int pix = (u0 + line) * N + x;
      float I = accw[e];
      if (jb.background) I += gmem(jb.background)[pix];
      if (MODE == 1) {
        // I + B to the resampling buffer, or the final forward output
        if (jb.ibuf) gmem(jb.ibuf)[static_cast<size_t>(c) * plane + pix] = I;
        else gmem(jb.out)[static_cast<size_t>(k) * plane + pix] = I;
        continue;
      }
      const float meas = gmem(jb.measured)[static_cast<size_t>(k) * plane + pix];
      const float wt = (loss.kind != 3 && jb.mask) ? static_cast<float>(gmem(jb.mask)[pix]) : 1.f;
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
      } else if (loss.kind == 4) {
        mixed_loss(I, meas, loss.noise_var, ell, dell);
      } else {
        ell = meas * I;
        dell = meas;
      }
      lsum += wt * ell;
      accw[e] = loss.gscale * wt * dell;  // 2 * scale * w * dloss/dI
      // background gradient terms, summed over positions by k_bg_reduce
      if (MODE == 0 && jb.g_background)
        gmem(reinterpret_cast<float*>(jb.GX))[static_cast<size_t>(c) * plane + pix] = accw[e];
    }
    if (MODE == 1) return;
    wave_fence();
    const float s = block_sum(lsum, red);
    if (threadIdx.x == 0) gmem(jb.loss_part)[static_cast<size_t>(c) * (N / RB) + r.sub] = s;
    if (MODE == 3) return;
  } else {
    for (int e = lane; e < RW * N; e += 64) {
      const int line = e / N, x = e % N;
      accw[e] = gmem(jb.ibuf)[static_cast<size_t>(c) * plane + (u0 + line) * N + x];
    }
    wave_fence();
  }
  for (int l = 0; l < jb.L; ++l) {
    const float ps = jb.pad_scale[l];
    const float2* twL = jb.tw_pad[l];
    const int nl = jb.pad[l];
    const bool rl = ratio_l(l);
    float da = 0.f;  // this thread's share of the rows' dL/d alpha_l terms
    for (int m = 0; m < jb.M; ++m) {
      gf2* Yr = gmem(jb.Y) + ((static_cast<size_t>(c) * jb.L + l) * jb.M + m) * plane +
                static_cast<size_t>(u0) * N;
      pad_switch(nl, [&](auto nlc) {
        constexpr int NL = decltype(nlc)::value;
        if constexpr (NL == czt_nb<N>()) {
          if (VAR == 2 && rl) {
            const double a = jb.czt_alpha[l];
            da += det_rows_adj_czt_ratio<N, NL, RW>(
                bufw, psiw, accw, Yr, gmem(twL), gmem(jb.czt[l]),
                static_cast<float>(1.0 / a), static_cast<float>(2.0 * kPi / (a * a)));
          } else {
            det_rows_adj_czt<N, NL, RW>(bufw, accw, Yr, gmem(twL), gmem(jb.czt[l]));
          }
        } else {
          det_rows_recomp<N, NL, RW>(bufw, accw, Yr, gmem(twL), ps);
        }
      }, Rows{});
    }
    if (VAR == 2 && rl) {
      const float sum = block_sum(da, red);
      if (threadIdx.x == 0)
        gmem(jb.ra_part)[(static_cast<size_t>(c) * jb.L + l) * (N / RB) + r.sub] = sum;
    }
  }
}

// ----------------------------------------------- tilted-plane resampling
// out != null: forward, write I' = R(I + B).  Else: loss on I' and
// gbuf = 2 scale w dloss/dI'.
// units: positions c, NT camera pixels per block (gx blocks per position)
__global__ __launch_bounds__(NT) void k_resample_loss(Launch la, LossDev loss, bool forward, int gx) {
  const int unit = blockIdx.x / gx;
  const int sidx = find_seg(la.segs, la.nseg, unit);
  const JobDev& jb = la.jobs[la.segs[sidx].job];
  if (*gmem(jb.status)) return;
  __shared__ float red[NT / 64];
  const int c = unit - la.segs[sidx].unit0, k = la.iter * jb.C + c;
  const int N = jb.N;
  const size_t plane = static_cast<size_t>(N) * N;
  const int sub = blockIdx.x - unit * gx;
  const int a = sub * NT + threadIdx.x;
  float lsum = 0.f;
  if (a < N * N) {
    const gf32* __restrict__ I = gmem(jb.ibuf) + static_cast<size_t>(c) * plane;
    const PTYCHO_GLOBAL int32_t* __restrict__ ridx = gmem(jb.rs_idx);
    const gf32* __restrict__ rw = gmem(jb.rs_w);
    float Ip = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = min(max(ridx[4 * a + t], 0), N * N - 1);  // caller tables are clamped
      Ip = fmaf(rw[4 * a + t], I[j], Ip);
    }
    if (forward) {
      gmem(jb.out)[static_cast<size_t>(k) * plane + a] = Ip;
    } else {
      const float meas = gmem(jb.measured)[static_cast<size_t>(k) * plane + a];
      const float wt = (loss.kind != 3 && jb.mask) ? static_cast<float>(gmem(jb.mask)[a]) : 1.f;
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
      } else if (loss.kind == 4) {
        mixed_loss(Ip, meas, loss.noise_var, ell, dell);
      } else {
        ell = meas * Ip;
        dell = meas;
      }
      lsum = wt * ell;
      gmem(jb.gbuf)[static_cast<size_t>(c) * plane + a] = loss.gscale * wt * dell;
    }
  }
  if (forward) return;
  const float t = block_sum(lsum, red);
  if (threadIdx.x == 0) gmem(jb.loss_part)[static_cast<size_t>(c) * gx + sub] = t;
}

// ibuf[c][j] = sum over the transposed table row j of val * gbuf[c][col]
__global__ __launch_bounds__(NT) void k_resample_T(Launch la, int gx) {
  const int unit = blockIdx.x / gx;
  const int sidx = find_seg(la.segs, la.nseg, unit);
  const JobDev& jb = la.jobs[la.segs[sidx].job];
  if (*gmem(jb.status)) return;
  const int c = unit - la.segs[sidx].unit0;
  const int N = jb.N;
  const size_t plane = static_cast<size_t>(N) * N;
  const int j = (blockIdx.x - unit * gx) * NT + threadIdx.x;
  if (j >= N * N) return;
  const gf32* __restrict__ g = gmem(jb.gbuf) + static_cast<size_t>(c) * plane;
  const PTYCHO_GLOBAL int32_t* __restrict__ tptr = gmem(jb.rsT_ptr);
  const PTYCHO_GLOBAL int32_t* __restrict__ tcol = gmem(jb.rsT_col);
  const gf32* __restrict__ tval = gmem(jb.rsT_val);
  float acc_s = 0.f;
  const int nnz_max = 4 * N * N;
  const int p0 = min(max(tptr[j], 0), nnz_max), p1 = min(max(tptr[j + 1], p0), nnz_max);
  for (int p = p0; p < p1; ++p) acc_s = fmaf(tval[p], g[min(max(tcol[p], 0), N * N - 1)], acc_s);
  gmem(jb.ibuf)[static_cast<size_t>(c) * plane + j] = acc_s;
}

// ---------------------------------------------------------- column adjoint
// units: (l, group of jb.probe_group positions) for the wavelengths whose DFT
// size is NL.  A block takes its group's positions in ascending order; with
// groups of more than one position the probe-gradient terms of the group
// are summed in LDS (pacc, [M][N][G], dynamic shared memory) and written once,
// into the slot of the group's first position.  GROUPED = false is the
// instance for launches whose jobs all have groups of one: one position per
// block, and the columns of mode m + 1 are loaded while mode m is processed
// (too many registers on top of the group loop).
// RATIO: the exact-ratio instance that also computes the y-axis terms of
// dL/d alpha (launches whose jobs want them).
template <int N, int NL, bool GROUPED, bool RATIO>
__global__ __launch_bounds__(col_adj_threads(N, NL), adj_narrow(N, NL) ? 4 : 2) void k_col_adj(Launch la) {
  constexpr int G = col_group_adj(N, NL);
  constexpr int AT = col_adj_threads(N, NL);
  const UnitRef r = decode_cols<N / G>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  const bool want_probe = jb.g_probe != nullptr;
  // the Bluestein length 768 at N = 384 without the distance gradient: unpadded
  // rows too (its one instance that does not spill then; 3 harmonics x 4
  // modes, exact ratio: column adjoint 22.6 -> 21.3 ms per step).  The host's
  // LDS budget uses col_adj_lp, the larger pitch.
  constexpr int LP = (NL == czt_nb<N>() && N == 384 && !RATIO) ? G : col_adj_lp(N, NL, G);
  constexpr int NE = N * G / AT;
  __shared__ float2 buf[NL * LP];
  __shared__ float red[AT / 64];
  extern __shared__ float2 pacc[];
  const int l = r.l, x0 = r.sub * G;
  const int tid = threadIdx.x;
  const int PG = GROUPED ? jb.probe_group : 1;
  const bool group_acc = GROUPED && want_probe && PG > 1;
  const int cbeg = r.u * PG;
  const int cend = min(cbeg + PG, min(jb.C, jb.K - la.iter * jb.C));
  if (group_acc)
    for (int e = tid; e < jb.M * N * G; e += AT) pacc[e] = make_float2(0.f, 0.f);
  // (the transforms below synchronise the block before pacc is first used)
  for (int c = cbeg; c < cend; ++c) {
  const int k = la.iter * jb.C + c;
  const gf2* __restrict__ X = gmem(jb.X) + (static_cast<size_t>(c) * jb.L + l) * N * N + x0;
  const gf2* __restrict__ ry = gmem(jb.ramp) + static_cast<size_t>(c) * 2 * N;
  const float2* __restrict__ twN = jb.tw_N;
  const float2* __restrict__ twL = jb.tw_pad[l];
  const float sig = jb.sigma ? gmem(jb.sigma)[k] : 1.0f;

  // recompute Ohat = ramp_y FFT_y(X) and Osh = IFFT_y(Ohat) / N
  auto ld_x = [&](int line, int i) { return ldv(X, i * N + line); };
  auto st_ramp = [&](int line, int i, float2 v) { buf[i * LP + line] = cmul(v, ldv(ry, i)); };
  fft_lines<N, false, G, AT, LP, true>(buf, twN, ld_x, st_ramp);
  float2 ohat[NE], o[NE], go[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * AT, line = e % G, i = e / G;
    ohat[q] = buf[i * LP + line];
  }
  auto ld_buf = [&](int line, int i) { return buf[i * LP + line]; };
  auto st_buf = [&](int line, int i, float2 v) { buf[i * LP + line] = v; };
  fft_lines<N, true, G, AT, LP, true>(buf, twN, ld_buf, st_buf);
  constexpr float invN = 1.0f / N;
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * AT, line = e % G, i = e / G;
    o[q] = cscale(buf[i * LP + line], invN);
    go[q] = make_float2(0.f, 0.f);
  }
  __syncthreads();

  const float ps = jb.pad_scale[l];
  float sgsum = 0.f;
  float rsum = 0.f;  // y-axis terms of dL/d alpha (exact ratio, g_ratio wanted)
  gf2* __restrict__ Z0 = gmem(jb.Y) + (static_cast<size_t>(c) * jb.L + l) * jb.M * N * N + x0;
  constexpr bool CZT = NL == czt_nb<N>();
  const gf2* __restrict__ tb = CZT ? gmem(jb.czt[l]) : nullptr;
  static_assert(!RATIO || CZT, "alpha derivative of the exact-ratio propagator only");
  const bool want_ratio = RATIO && jb.g_ratio != nullptr;
  // first-transform input of mode m at FFT index t: the cropped bins embedded
  // at their frequencies, or (exact ratio) conj(cout) Z in detector order
  auto zin_at = [&](const gf2* __restrict__ Zm, const gf2* __restrict__ tbm, int line, int t) {
    if constexpr (CZT) {
      return t < N ? cmulconj(ldv(tbm, N + t), ldv(Zm, t * N + line)) : make_float2(0.f, 0.f);
    } else {
      int u = t + N / 2;
      if (u >= NL) u -= NL;
      return u < N ? ldv(Zm, u * N + line) : make_float2(0.f, 0.f);
    }
  };
  // The next mode's first-pass inputs are loaded during the current mode in
  // the single-position zero-padded instances; the grouped and the
  // exact-ratio (length 2N) instances have no registers left for them.
  constexpr bool PREFETCH = !GROUPED && !CZT;
  using ZIn = PreIn<NL, G, AT, true>;
  auto zload = [&](int m, ZIn& zin) {
    const gf2* __restrict__ Zm = Z0 + static_cast<size_t>(m) * N * N;
    fft_first_load(zin, [&](int line, int t) { return zin_at(Zm, tb, line, t); });
  };
  ZIn zcur;
  if constexpr (PREFETCH) zload(0, zcur);
#pragma unroll 1
  for (int m = 0; m < jb.M; ++m) {
    gf2* __restrict__ Z = Z0 + static_cast<size_t>(m) * N * N;
    const gf2* __restrict__ P =
        gmem(jb.probe) + (static_cast<size_t>(l / jb.Ns) * jb.M + m) * N * N + x0;
    // the chirp table is read through a pointer the compiler cannot see
    // through, so that its loads stay in the mode loop instead of every
    // thread's table values being held in registers across it (the grouped
    // exact-ratio instances spilled 20 to 87 registers before)
    const gf2* __restrict__ tbm = CZT ? opaque_table(tb) : nullptr;
    auto st_chi = [&](int line, int t, float2 v) {
      if (t < N) buf[t * LP + line] = cscale(v, ps);
    };
    // exact ratio: FFT, times conj(kernel DFT), IFFT, conj(cin)
    auto st_hc = [&](int line, int t, float2 v) { buf[t * LP + line] = cmulconj(ldv(tbm, 2 * N + t), v); };
    auto ld_b = [&](int line, int t) { return buf[t * LP + line]; };
    auto st_chic = [&](int line, int t, float2 v) {
      if (t < N) buf[t * LP + line] = cmulconj(ldv(tbm, t), v);
    };
    if constexpr (RATIO) {
      if (want_ratio) {
        // y-axis term of dL/d alpha: chi_u = F_y^H (u Z), summed against r psi
        auto ld_u = [&](int line, int t) {
          return cscale(zin_at(Z, tbm, line, t), static_cast<float>(t - N / 2));
        };
        fft_lines<NL, false, G, AT, LP, true>(buf, twL, ld_u, st_hc);
        fft_lines<NL, true, G, AT, LP, true>(buf, twL, ld_b, st_chic);
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          const int e = tid + q * AT, line = e % G, i = e / G;
          const float2 cu = buf[i * LP + line];
          const float2 ps = cscale(cmul(ldv(P, i * N + line), o[q]), sig);
          rsum += static_cast<float>(i) * (cu.y * ps.x - cu.x * ps.y);
        }
        __syncthreads();
      }
    }
    if constexpr (!PREFETCH) {
      auto ld_z = [&](int line, int t) { return zin_at(Z, tbm, line, t); };
      if constexpr (CZT) {
        fft_lines<NL, false, G, AT, LP, true>(buf, twL, ld_z, st_hc);
        fft_lines<NL, true, G, AT, LP, true>(buf, twL, ld_b, st_chic);
      } else {
        fft_lines<NL, true, G, AT, LP, true>(buf, twL, ld_z, st_chi);
      }
    } else {
      ZIn znext;
      if (m + 1 < jb.M) zload(m + 1, znext);
      else znext = zcur;  // (no next mode: a defined value, not used)
      fft_lines<NL, true, G, AT, LP, true>(buf, twL, zcur, st_chi);
      zcur = znext;
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * AT, line = e % G, i = e / G;
      const float2 chi = buf[i * LP + line];
      const float2 p = ldv(P, i * N + line);
      const float2 pc = cmulconj(p, chi);  // conj(P) chi
      go[q].x = fmaf(sig, pc.x, go[q].x);
      go[q].y = fmaf(sig, pc.y, go[q].y);
      // Re( conj(chi) P Osh ) = Re( conj(conj(P) chi) Osh )
      sgsum += pc.x * o[q].x + pc.y * o[q].y;
      if (want_probe) {
        const float2 term = cscale(cmulconj(o[q], chi), sig);
        if (group_acc) {
          float2& a = pacc[(m * N + i) * G + line];  // one owner thread per element
          a = cadd(a, term);
        } else {
          stv(Z, i * N + line, term);
        }
      }
    }
    __syncthreads();
  }
  {
    const float s = block_sum<AT>(sgsum, red);
    if (tid == 0)
      gmem(jb.sg_part)[(static_cast<size_t>(c) * jb.L + l) * adj_stride(N) + r.sub] = s;
  }
  if (want_ratio) {
    const double a = jb.czt_alpha[l];
    const float s = block_sum<AT>(rsum, red);
    if (tid == 0)
      gmem(jb.rb_part)[(static_cast<size_t>(c) * jb.L + l) * adj_stride(N) + r.sub] =
          static_cast<float>(2.0 * kPi / (a * a)) * s;
  }
  // Ghat = FFT_y(G_Osh): y-position derivative and adjoint y-shift
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * AT, line = e % G, i = e / G;
    buf[i * LP + line] = go[q];
  }
  __syncthreads();
  fft_lines<N, false, G, AT, LP, true>(buf, twN, ld_buf, st_buf);
  float dsum = 0.f;
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + q * AT, line = e % G, i = e / G;
    const float2 gh = buf[i * LP + line];
    const float nu = 2.0f * static_cast<float>(kPi) * freq(i, N);
    // Re( conj(gh) * (i nu ohat) )
    dsum += nu * (gh.y * ohat[q].x - gh.x * ohat[q].y);
    buf[i * LP + line] = cmul(gh, cconj(ldv(ry, i)));
  }
  __syncthreads();
  gf2* __restrict__ GX = gmem(jb.GX) + (static_cast<size_t>(c) * jb.L + l) * N * N + x0;
  auto st_gx = [&](int line, int i, float2 v) { stv(GX, i * N + line, cscale(v, invN)); };
  fft_lines<N, true, G, AT, LP, true>(buf, twN, ld_buf, st_gx);
  const float s = block_sum<AT>(dsum, red);
  if (tid == 0)
    gmem(jb.dy_part)[(static_cast<size_t>(c) * jb.L + l) * adj_stride(N) + r.sub] = s * invN;
  }  // positions of the group
  if (group_acc && cbeg < cend) {
    gf2* __restrict__ Zg = gmem(jb.Y) + (static_cast<size_t>(cbeg) * jb.L + l) * jb.M * N * N + x0;
    for (int m = 0; m < jb.M; ++m) {
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = tid + q * AT, line = e % G, i = e / G;
        stv(Zg + static_cast<size_t>(m) * N * N, i * N + line, pacc[(m * N + i) * G + line]);
      }
    }
  }
}

// Column adjoint over groups of PG = kRegGroup (3) consecutive positions: the
// probe-gradient groups of jobs whose [M][N][G] LDS accumulator does not fit
// (many modes at N = 512).  The modes are the outer loop: for mode m the
// block transforms the group's columns and adds their probe-gradient terms
// in registers, in ascending position order, and writes the sum once, into
// the first position's slot.  So the probe columns of a mode are read once
// per group, and the terms that the column adjoint writes and the probe
// reduction reads are divided by PG.  Per position the arithmetic is that of
// k_col_adj (the same transforms and products), and the group's sum
// ((t0 + t1) + t2) is the value that an LDS group of the same positions
// forms.  Ohat of the group's positions waits in LDS (dynamic, [PG][N][G])
// until the y-shift adjoint at the end; the shifted patches and the
// gradients go_p stay in registers.  Three positions rather than two (5
// harmonics x 8 modes, N = 512: column adjoint 159.4 -> 151.5 ms, probe
// reduction 17.1 -> 11.4 ms per step); every compiled size fits them.
// units: (l, group of PG positions) for the wavelengths whose DFT size is NL.
template <int N, int NL>
__global__ __launch_bounds__(col_adj_threads(N, NL), 2) void k_col_adj_pair(Launch la) {
  static_assert(NL != czt_nb<N>(), "zero-padded sizes only");
  constexpr int G = col_group_adj(N, NL);
  constexpr int AT = col_adj_threads(N, NL);
  // The Z tile of a transform is stored transposed, one column per LDS row
  // in the detector rows' layout, and each wave transforms its own rows
  // (wave fences only).  Columns left in place instead need an odd pitch
  // (unpadded: 254 ms per step of 5 harmonics x 8 modes at N = 512, against
  // 158 ms), and at lengths that are multiples of 16 their radix-16 and -8
  // strides meet the same banks at any odd pitch, so those sizes transformed
  // block-wide: 137.7 ms for that mix, 135.7 ms with the transposed tile.
  constexpr int LPC = pair_row_pitch(NL, G);
  using TI = Lds<NL, LPC, false>;
  // the N-point transforms (object columns, gradient tail) on a transposed
  // tile as well, with coalesced loads and stores around them (5 x 8 at
  // N = 512: column adjoint 135.6 -> 131.9 ms per step; 3 x 4 at N = 384:
  // 12.33 -> 12.42 ms)
  constexpr int LPN = pair_row_pitch(N, G);
  using TN = Lds<N, LPN, false>;
  constexpr int NE = N * G / AT;
  const UnitRef r = decode_cols<N / G>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  __shared__ float2 buf[G * LPC > G * LPN ? G * LPC : G * LPN];
  __shared__ float red[AT / 64];
  extern __shared__ float2 ohs[];  // [PG][N * G], element e of this thread at e = tid + q AT
  // The twiddle tables are copied to LDS and the transforms read them there:
  // the next transform's column inputs are loaded during the current one,
  // and a twiddle load from global memory issued after them would make the
  // transform wait for them too (the vector-memory counter completes in
  // order); LDS loads wait on their own counter.  (5 harmonics x 8 modes,
  // N = 512: 174.0 -> 171.4 ms per step.)
  constexpr int TWL = tw_len<NL>(), TWN = tw_len<N>();
  __shared__ float2 tws[TWL + TWN];
  const int l = r.l, x0 = r.sub * G;
  const int tid = threadIdx.x;
  constexpr int PG = kRegGroup;
  const int c0 = r.u * PG;
  const int np = min(PG, min(jb.C, jb.K - la.iter * jb.C) - c0);  // 1 .. PG
  const bool want_probe = jb.g_probe != nullptr;
  {
    const gf2* __restrict__ gL = gmem(jb.tw_pad[l]);
    const gf2* __restrict__ gN = gmem(jb.tw_N);
    for (int e = tid; e < TWL; e += AT) tws[e] = ldv(gL, e);
    for (int e = tid; e < TWN; e += AT) tws[TWL + e] = ldv(gN, e);
  }
  __syncthreads();
  const lf2* const twL = (const lf2*)tws;
  const lf2* const twN = (const lf2*)tws + TWL;
  const float ps = jb.pad_scale[l];
  const size_t plane = static_cast<size_t>(N) * N;
  constexpr float invN = 1.0f / N;
  constexpr int LWN = G / (AT / 64);  // rows per wave
  lf2* const rown = (lf2*)buf + (tid >> 6) * LWN * LPN;
  auto ldn = [&](int j, int i) { return ldv(rown, TN::at(j, i)); };
  auto stn = [&](int j, int i, float2 v) { stv(rown, TN::at(j, i), v); };
  float2 o[PG][NE], go[PG][NE];
  float sig[PG], sgsum[PG] = {};

  // recompute Ohat = ramp_y FFT_y(X) (to LDS) and Osh = IFFT_y(Ohat) / N;
  // the X tile is loaded coalesced into the transposed rows
#pragma unroll
  for (int p = 0; p < PG; ++p) {
    if (p < np) {
      const int c = c0 + p, k = la.iter * jb.C + c;
      const gf2* __restrict__ X = gmem(jb.X) + (static_cast<size_t>(c) * jb.L + l) * plane + x0;
      const gf2* __restrict__ ry = gmem(jb.ramp) + static_cast<size_t>(c) * 2 * N;
      sig[p] = jb.sigma ? gmem(jb.sigma)[k] : 1.0f;
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = tid + q * AT, line = e % G, i = e / G;
        buf[TN::at(line, i)] = ldv(X, i * N + line);
      }
      __syncthreads();
      auto st_ramp = [&](int j, int i, float2 v) { stv(rown, TN::at(j, i), cmul(v, ldv(ry, i))); };
      fft_lines<N, false, LWN, 64, LPN, false>(rown, twN, ldn, st_ramp);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = tid + q * AT, line = e % G, i = e / G;
        ohs[p * N * G + e] = buf[TN::at(line, i)];
      }
      __syncthreads();
      fft_lines<N, true, LWN, 64, LPN, false>(rown, twN, ldn, stn);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = tid + q * AT, line = e % G, i = e / G;
        o[p][q] = cscale(buf[TN::at(line, i)], invN);
        go[p][q] = make_float2(0.f, 0.f);
      }
      __syncthreads();
    }
  }

  // chi_{p,m} = crop(DFT^H(embed(Z_{p,m}))); go_p += sig_p conj(P_m) chi;
  // probe term sum_p sig_p conj(Osh_p) chi.  The block stores the Z tile of
  // a transform (rows u < N of its G columns, coalesced) in the buffer,
  // then each wave transforms its columns there on its own (wave fences, no
  // workgroup barrier per pass), and the block meets again for the
  // pointwise products.  The next tile's loads are in flight meanwhile.
  constexpr int LW = G / (AT / 64);  // columns per wave
  static_assert(G % (AT / 64) == 0, "whole columns per wave");
  auto z_at = [&](int p, int m) {
    return gmem(jb.Y) + ((static_cast<size_t>(c0 + p) * jb.L + l) * jb.M + m) * plane + x0;
  };
  float2 zt[NE];  // element e = tid + q AT of the tile: column e % G, row e / G
  auto zload = [&](int p, int m) {
    const gf2* __restrict__ Zm = z_at(p, m);
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * AT, line = e % G, i = e / G;
      zt[q] = ldv(Zm, i * N + line);
    }
  };
  // this wave's rows (columns j of the tile): element t at roww[TI::at(j, t)]
  lf2* const roww = (lf2*)buf + (tid >> 6) * LW * LPC;
  auto ld_w = [&](int j, int t) {
    int u = t + N / 2;
    if (u >= NL) u -= NL;
    return u < N ? ldv(roww, TI::at(j, u)) : make_float2(0.f, 0.f);
  };
  auto st_w = [&](int j, int t, float2 v) {
    if (t < N) stv(roww, TI::at(j, t), cscale(v, ps));
  };
  zload(0, 0);
  for (int m = 0; m < jb.M; ++m) {
    const gf2* __restrict__ P =
        gmem(jb.probe) + (static_cast<size_t>(l / jb.Ns) * jb.M + m) * plane + x0;
    // the mode's probe columns, read once for the group's positions
    float2 term[NE], pm[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * AT, line = e % G, i = e / G;
      pm[q] = ldv(P, i * N + line);
    }
#pragma unroll
    for (int p = 0; p < PG; ++p) {
      if (p < np) {
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          const int e = tid + q * AT, line = e % G, i = e / G;
          buf[TI::at(line, i)] = zt[q];
        }
        {
          // the next transform's tile: the next position of this mode,
          // else position 0 of the next mode
          const int pn = p + 1 < np ? p + 1 : 0, mn = pn ? m : m + 1;
          if (mn < jb.M) zload(pn, mn);
        }
        __syncthreads();
        fft_lines<NL, true, LW, 64, LPC, false>(roww, twL, ld_w, st_w);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          const int e = tid + q * AT, line = e % G, i = e / G;
          const float2 chi = buf[TI::at(line, i)];
          const float2 pc = cmulconj(pm[q], chi);  // conj(P) chi
          go[p][q].x = fmaf(sig[p], pc.x, go[p][q].x);
          go[p][q].y = fmaf(sig[p], pc.y, go[p][q].y);
          sgsum[p] += pc.x * o[p][q].x + pc.y * o[p][q].y;
          if (want_probe) {
            const float2 t = cscale(cmulconj(o[p][q], chi), sig[p]);
            term[q] = p == 0 ? t : cadd(term[q], t);
          }
        }
        __syncthreads();
      }
    }
    if (want_probe) {
      gf2* __restrict__ Z0 =
          gmem(jb.Y) + ((static_cast<size_t>(c0) * jb.L + l) * jb.M + m) * plane + x0;
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = tid + q * AT, line = e % G, i = e / G;
        stv(Z0, i * N + line, term[q]);
      }
    }
  }

  // per position: sigma partial, Ghat = FFT_y(go) (y-position derivative),
  // adjoint y-shift to GX
#pragma unroll
  for (int p = 0; p < PG; ++p) {
    if (p < np) {
      const int c = c0 + p;
      const size_t slot = (static_cast<size_t>(c) * jb.L + l) * adj_stride(N) + r.sub;
      {
        const float s = block_sum<AT>(sgsum[p], red);
        if (tid == 0) gmem(jb.sg_part)[slot] = s;
      }
      const gf2* __restrict__ ry = gmem(jb.ramp) + static_cast<size_t>(c) * 2 * N;
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = tid + q * AT, line = e % G, i = e / G;
        buf[TN::at(line, i)] = go[p][q];
      }
      __syncthreads();
      fft_lines<N, false, LWN, 64, LPN, false>(rown, twN, ldn, stn);
      __syncthreads();
      float dsum = 0.f;
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = tid + q * AT, line = e % G, i = e / G;
        const float2 gh = buf[TN::at(line, i)];
        const float2 oh = ohs[p * N * G + e];
        const float nu = 2.0f * static_cast<float>(kPi) * freq(i, N);
        dsum += nu * (gh.y * oh.x - gh.x * oh.y);
        buf[TN::at(line, i)] = cmul(gh, cconj(ldv(ry, i)));
      }
      __syncthreads();
      fft_lines<N, true, LWN, 64, LPN, false>(rown, twN, ldn, stn);
      __syncthreads();
      gf2* __restrict__ GX = gmem(jb.GX) + (static_cast<size_t>(c) * jb.L + l) * plane + x0;
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = tid + q * AT, line = e % G, i = e / G;
        stv(GX, i * N + line, cscale(buf[TN::at(line, i)], invN));
      }
      const float s = block_sum<AT>(dsum, red);
      if (tid == 0) gmem(jb.dy_part)[slot] = s * invN;
    }
  }
}

// ------------------------------------------- probe gradient: ordered k sum
// g_probe[l][m][pix] += sum over position groups (ascending) and sample
// modes n (ascending) of Y[first c of group][l Ns + n][m][pix]
// units: (wavelength l, m * nblk + pixel block), nblk = ceil(N^2 / NT)
__global__ __launch_bounds__(NT) void k_probe_reduce(Launch la) {
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  const size_t plane = static_cast<size_t>(jb.N) * jb.N;
  const int nblk = static_cast<int>((plane + NT - 1) / NT);
  const int m = r.u / nblk, blk = r.u - m * nblk;
  const size_t pix = static_cast<size_t>(blk) * NT + threadIdx.x;
  if (pix >= plane) return;
  const int lm = r.l * jb.M + m;
  const size_t stride = static_cast<size_t>(jb.L) * jb.M * plane;  // one position
  const size_t nstride = static_cast<size_t>(jb.M) * plane;         // one sample mode
  const gf2* __restrict__ src =
      gmem(jb.Y) + (static_cast<size_t>(r.l) * jb.Ns * jb.M + m) * plane + pix;
  gf2* __restrict__ gp = gmem(jb.g_probe);
  float2 acc = ldv(gp, static_cast<size_t>(lm) * plane + pix);
  const int C = min(jb.C, jb.K - la.iter * jb.C);
  const int PG = jb.probe_group;  // one summed term per group of positions
  int c = 0;
  if (jb.Ns == 1) {
    // eight groups' terms loaded before their additions, which keep the
    // ascending order (probe reduction, N = 512, 8 modes: 35.2 -> 33.6 ms per step)
    for (; c + 8 * PG <= C; c += 8 * PG) {
      float2 v[8];
#pragma unroll
      for (int h = 0; h < 8; ++h) v[h] = ldv(src, static_cast<size_t>(c + h * PG) * stride);
#pragma unroll
      for (int h = 0; h < 8; ++h) acc = cadd(acc, v[h]);
    }
  }
  for (; c < C; c += PG)
    for (int n = 0; n < jb.Ns; ++n) acc = cadd(acc, ldv(src, c * stride + n * nstride));
  stv(gp, static_cast<size_t>(lm) * plane + pix, acc);
}

// --------------------------------------- background gradient: ordered k sum
// g_background[pix] += sum over the chunk's positions, ascending, of
// (1/2) (2 scale w dL/dI')-pulled-back: from the resampling buffer (after
// R^T) or from the detector kernel's terms parked in GX.
// units: pixel blocks of NT per job
__global__ __launch_bounds__(NT) void k_bg_reduce(Launch la) {
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  const size_t plane = static_cast<size_t>(jb.N) * jb.N;
  const size_t pix = static_cast<size_t>(r.u) * NT + threadIdx.x;
  if (pix >= plane) return;
  const gf32* __restrict__ src = gmem(jb.ibuf ? jb.ibuf : reinterpret_cast<const float*>(jb.GX)) + pix;
  gf32* __restrict__ gb = gmem(jb.g_background);
  float acc = gb[pix];
  const int C = min(jb.C, jb.K - la.iter * jb.C);
  for (int c = 0; c < C; ++c) acc += 0.5f * src[static_cast<size_t>(c) * plane];
  gb[pix] = acc;
}

// -------------------------------------------------------------- row adjoint
// per wave, lines [0, RW): G_X rows; [RW, 2 RW): X rows.  x-position derivative from
// Re sum conj(FFT(G_X)) (2 pi i nu) FFT(X) / N; G_A = IFFT(conj(ramp) FFT(G_X)) / N
// units: (l, c)
template <int N>
__global__ __launch_bounds__(NT) void k_row_adj(Launch la) {
  constexpr int RB = rb_adj<N>();
  // each wave owns RW of the block's RB rows (their G_X and X lines) in an
  // LDS region of its own; the waves meet only in the block sum
  constexpr int RW = RB / (NT / 64);
  static_assert(RB % (NT / 64) == 0, "whole rows per wave");
  const UnitRef r = decode<N / RB>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  constexpr int LP = row_lp(N);
  using Ix = Lds<N, LP, false>;
  __shared__ float2 buf[2 * RB * LP];
  __shared__ float red[NT / 64];
  const int wv = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
  lf2* const bufw = (lf2*)buf + wv * 2 * RW * LP;
  const int l = r.l, c = r.u, y0 = r.sub * RB + wv * RW;
  const int tid = threadIdx.x;
  const size_t off = (static_cast<size_t>(c) * jb.L + l) * N * N + static_cast<size_t>(y0) * N;
  const gf2* __restrict__ GXr = gmem(jb.GX) + off;
  gf2* __restrict__ Xr = gmem(jb.X) + off;
  const gf2* __restrict__ rx = gmem(jb.ramp) + (static_cast<size_t>(c) * 2 + 1) * N;
  const float2* __restrict__ twN = jb.tw_N;
  auto ld = [&](int line, int i) {
    return line < RW ? ldv(GXr, line * N + i) : ldv(Xr, (line - RW) * N + i);
  };
  auto st = [&](int line, int i, float2 v) { stv(bufw, Ix::at(line, i), v); };
  fft_lines<N, false, 2 * RW, 64, LP, false>(bufw, twN, ld, st);
  float dsum = 0.f;
  for (int e = lane; e < RW * N; e += 64) {
    const int line = e / N, i = e % N;
    const float2 gh = ldv(bufw, Ix::at(line, i));
    const float2 xh = ldv(bufw, Ix::at(line + RW, i));
    const float nu = 2.0f * static_cast<float>(kPi) * freq(i, N);
    dsum += nu * (gh.y * xh.x - gh.x * xh.y);
    stv(bufw, Ix::at(line, i), cmul(gh, cconj(ldv(rx, i))));
  }
  fft_sync<64>();  // the inverse reads other lanes' elements
  constexpr float invN = 1.0f / N;
  auto ld1 = [&](int line, int i) { return ldv(bufw, Ix::at(line, i)); };
  auto st1 = [&](int line, int i, float2 v) { stv(Xr, line * N + i, cscale(v, invN)); };
  fft_lines<N, true, RW, 64, LP, false>(bufw, twN, ld1, st1);
  const float s = block_sum(dsum, red);
  if (tid == 0) gmem(jb.dx_part)[(static_cast<size_t>(c) * jb.L + l) * (N / RB) + r.sub] = s * invN;
}

// ---------------------------------------------------- object gradient gather
// Tile of 16 x 64 object pixels; every window of the chunk that overlaps the
// tile adds its G_A values in ascending k.  No atomics: each pixel has one
// owner thread, so the sum order is fixed.  The block first tests the
// chunk's windows in parallel and compacts the overlapping ones, in
// ascending order, into an LDS list (wave ballots), then accumulates over
// that list only.  units: (l, tile)
constexpr int kTileW = kObjTileW, kTileHMax = 16;
constexpr int kListMax = 1024;  // windows tested per round
__global__ __launch_bounds__(NT) void k_obj_gather(Launch la) {
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  __shared__ int list_c[kListMax], list_py[kListMax], list_px[kListMax];
  __shared__ int wave_cnt[NT / 64];
  const int N = jb.N, l = r.l;
  const int tiles_x = (jb.W + kTileW - 1) / kTileW;
  const int TH = jb.obj_tile_h;  // 4, 8 or 16 rows
  const int ty = r.u / tiles_x, txi = r.u - ty * tiles_x;
  const int tx0 = txi * kTileW, ty0 = ty * TH;
  const int tx = threadIdx.x % kTileW, tyb = threadIdx.x / kTileW;  // tyb in [0, 4)
  const int x = tx0 + tx;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int PER = kTileHMax / (NT / kTileW);  // rows per thread, at most
  const int per = TH / (NT / kTileW);
  float2 acc[PER];
  gf2* __restrict__ G = gmem(jb.g_object) + static_cast<size_t>(l) * jb.H * jb.W;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int y = ty0 + tyb + q * (NT / kTileW);
    acc[q] = (q < per && x < jb.W && y < jb.H) ? ldv(G, static_cast<size_t>(y) * jb.W + x)
                                              : make_float2(0.f, 0.f);
  }
  const size_t plane = static_cast<size_t>(N) * N;
  const int C = min(jb.C, jb.K - la.iter * jb.C);
  const int kbase = la.iter * jb.C;
  const gf32* __restrict__ pos = gmem(jb.pos);
  for (int c0 = 0; c0 < C; c0 += kListMax) {
    const int cn = min(kListMax, C - c0);
    int count = 0;  // block-uniform
    for (int s0 = 0; s0 < cn; s0 += NT) {
      const int c = c0 + s0 + threadIdx.x;
      bool hit = false;
      int py = 0, px = 0;
      if (s0 + threadIdx.x < cn) {
        float dy, dx;
        split_pos(pos, kbase + c, py, px, dy, dx);
        hit = !(py >= ty0 + TH || py + N <= ty0 || px >= tx0 + kTileW || px + N <= tx0);
      }
      const unsigned long long m = __ballot(hit);
      if (lane == 0) wave_cnt[wid] = __popcll(m);
      __syncthreads();
      int before = 0, total = 0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) {
        const int n = wave_cnt[w];
        before += w < wid ? n : 0;
        total += n;
      }
      if (hit) {
        const int idx = count + before + __popcll(m & ((1ull << lane) - 1ull));
        list_c[idx] = c;
        list_py[idx] = py;
        list_px[idx] = px;
      }
      count += total;
      __syncthreads();  // wave_cnt is rewritten next round; the list is complete
    }
    // four windows per iteration: all their loads are issued before the
    // additions, which keep the ascending window order (object gather:
    // 0.36 -> 0.25 ms per step for 400 positions x 4 wavelengths at N = 256)
    for (int i = 0; i < count; i += 4) {
      float2 v[4][PER];
      bool ok[4][PER];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const bool live = i + h < count;
        const int c = live ? list_c[i + h] : 0;
        const int py = live ? list_py[i + h] : 0, px = live ? list_px[i + h] : 0;
        const gf2* __restrict__ GA = gmem(jb.X) + (static_cast<size_t>(c) * jb.L + l) * plane;
        const int xr = x - px;
        const bool inx = live && xr >= 0 && xr < N;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int yr = ty0 + tyb + q * (NT / kTileW) - py;
          ok[h][q] = q < per && inx && yr >= 0 && yr < N;
          v[h][q] = ok[h][q] ? ldv(GA, yr * N + xr) : make_float2(0.f, 0.f);
        }
      }
#pragma unroll
      for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int q = 0; q < PER; ++q)
          if (ok[h][q]) acc[q] = cadd(acc[q], v[h][q]);
    }
    __syncthreads();  // the list is rebuilt for the next round
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int y = ty0 + tyb + q * (NT / kTileW);
    if (q < per && x < jb.W && y < jb.H) stv(G, static_cast<size_t>(y) * jb.W + x, acc[q]);
  }
}

// ---------------------------------------------------------------- finalize
// s + p[0] + p[stride] + ... + p[(n - 1) stride], added left to right in the
// accumulator's type, with eight loads in flight before their additions
// (the single-thread sums were bound by one load latency per term).
template <class A, class T>
__device__ __forceinline__ A ordered_sum(A s, const PTYCHO_GLOBAL T* p, long long n,
                                         long long stride = 1) {
  long long i = 0;
  for (; i + 8 <= n; i += 8) {
    T v[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) v[h] = p[(i + h) * stride];
#pragma unroll
    for (int h = 0; h < 8; ++h) s += v[h];
  }
  for (; i < n; ++i) s += p[i * stride];
  return s;
}

// Ordered per-position sums of the partials.  units: blocks of 64 positions
__global__ void k_finalize_chunk(Launch la) {
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  const int c = r.u * 64 + threadIdx.x;
  const int C = min(jb.C, jb.K - la.iter * jb.C);
  if (c >= C) return;
  const int k = la.iter * jb.C + c;
  // column-adjoint partials: n_dy(l) per slot, row stride sdy
  const int sdy = adj_stride(jb.N), n_dx = jb.N / rb_adj_dev(jb.N);
  auto n_dy = [&](int l) { return jb.N / col_group_adj(jb.N, jb.pad[l]); };
  const double ls =
      ordered_sum(0.0, gmem(jb.loss_part) + static_cast<size_t>(c) * jb.n_loss, jb.n_loss);
  gmem(jb.loss_k)[k] = ls;
  if (!jb.want_adjoint) return;
  float gy = 0.f, gx = 0.f, gs = 0.f;
  for (int l = 0; l < jb.L; ++l) {
    const size_t row = static_cast<size_t>(c) * jb.L + l;
    gy = ordered_sum(gy, gmem(jb.dy_part) + row * sdy, n_dy(l));
    gs = ordered_sum(gs, gmem(jb.sg_part) + row * sdy, n_dy(l));
    gx = ordered_sum(gx, gmem(jb.dx_part) + row * n_dx, n_dx);
  }
  if (jb.g_pos) {
    gmem(jb.g_pos)[2 * k] = gy;
    gmem(jb.g_pos)[2 * k + 1] = gx;
  }
  if (jb.g_sigma) gmem(jb.g_sigma)[k] = gs;
  if (jb.g_ratio) {
    const int n_ra = jb.N / rb_det_dev(jb.N);
    for (int w = 0; w < jb.Lw; ++w) {
      double da = 0.0;
      for (int l = w * jb.Ns; l < (w + 1) * jb.Ns; ++l) {  // slots of wavelength w
        if (!jb.czt[l]) continue;
        const size_t row = static_cast<size_t>(c) * jb.L + l;
        da = ordered_sum(da, gmem(jb.ra_part) + row * n_ra, n_ra);
        da = ordered_sum(da, gmem(jb.rb_part) + row * sdy, n_dy(l));
      }
      gmem(jb.ratio_k)[static_cast<size_t>(k) * jb.Lw + w] = da;
    }
  }
}

// ------------------------------------------------------------ regulariser
// Amplitude a = |O| of every slot: l1 sum a + tv sum sqrt(dy^2 + dx^2 + d^2)
// with forward differences (zero past the last row / column).  Each thread
// owns one pixel: its value term, and its gradient
// (l1 - tv (dy + dx) / t + tv dy_up / t_up + tv dx_left / t_left) O / a
// (the last two from the terms of the pixels above and to the left) added to
// g_object once per call, after every chunk's data gradient.
// units: (job, slot) x ceil(H W / kRegBlock) pixel blocks
__device__ __forceinline__ float amp_at(const gf2* __restrict__ O, int H, int W, int y, int x) {
  const float2 v = ldv(O, static_cast<size_t>(y) * W + x);
  return sqrtf(v.x * v.x + v.y * v.y);
}

__global__ __launch_bounds__(kRegBlock) void k_regulariser(Launch la, LossDev loss) {
  __shared__ float red[kRegBlock / 64];
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  const int H = jb.H, W = jb.W;
  const size_t hw = static_cast<size_t>(H) * W;
  const gf2* __restrict__ O = gmem(jb.object) + static_cast<size_t>(r.l) * hw;
  const size_t p = static_cast<size_t>(r.u) * kRegBlock + threadIdx.x;
  const float d2 = loss.tv_eps * loss.tv_eps;
  float val = 0.f;
  if (p < hw) {
    const int y = static_cast<int>(p / W), x = static_cast<int>(p - static_cast<size_t>(y) * W);
    const float2 o = ldv(O, p);
    const float a = sqrtf(o.x * o.x + o.y * o.y);
    const float dy = y + 1 < H ? amp_at(O, H, W, y + 1, x) - a : 0.f;
    const float dx = x + 1 < W ? amp_at(O, H, W, y, x + 1) - a : 0.f;
    const float t = sqrtf(dy * dy + dx * dx + d2);
    val = loss.l1 * a + loss.tv * t;
    float ga = loss.l1 - loss.tv * (dy + dx) / t;
    if (y > 0) {  // term of the pixel above: its dy is a - a_up
      const float au = amp_at(O, H, W, y - 1, x);
      const float dxu = x + 1 < W ? amp_at(O, H, W, y - 1, x + 1) - au : 0.f;
      const float dyu = a - au;
      ga += loss.tv * dyu / sqrtf(dyu * dyu + dxu * dxu + d2);
    }
    if (x > 0) {  // term of the pixel to the left: its dx is a - a_left
      const float al = amp_at(O, H, W, y, x - 1);
      const float dyl = y + 1 < H ? amp_at(O, H, W, y + 1, x - 1) - al : 0.f;
      const float dxl = a - al;
      ga += loss.tv * dxl / sqrtf(dyl * dyl + dxl * dxl + d2);
    }
    if (jb.g_object && a > 0.f) {
      gf2* __restrict__ G = gmem(jb.g_object) + static_cast<size_t>(r.l) * hw;
      const float s = ga / a;
      stv(G, p, cadd(ldv(G, p), make_float2(s * o.x, s * o.y)));
    }
  }
  const float bs = block_sum<kRegBlock>(val, red);
  if (threadIdx.x == 0)
    gmem(jb.reg_part)[static_cast<size_t>(r.l) * ((hw + kRegBlock - 1) / kRegBlock) + r.u] = bs;
}

// one unit per job
__global__ void k_loss_total(Launch la, LossDev loss, float scale) {
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  if (threadIdx.x != 0) return;
  if (*gmem(jb.status)) {
    if (jb.loss) *gmem(jb.loss) = __int_as_float(0x7fc00000);
    return;
  }
  if (jb.loss) {
    double s = ordered_sum(0.0, gmem(jb.loss_k), jb.K);
    s *= scale;
    if (loss.l1 != 0.f || loss.tv != 0.f) {  // the regulariser, added unscaled
      const size_t n = static_cast<size_t>(jb.L) *
                       ((static_cast<size_t>(jb.H) * jb.W + kRegBlock - 1) / kRegBlock);
      s += ordered_sum(0.0, gmem(jb.reg_part), static_cast<long long>(n));
    }
    *gmem(jb.loss) = static_cast<float>(s);
  }
  if (jb.g_ratio) {
    // dL/d alpha_l: ordered sum over positions (the terms carry the scale)
    for (int w = 0; w < jb.Lw; ++w) {
      const double s = ordered_sum(0.0, gmem(jb.ratio_k) + w, jb.K, jb.Lw);
      gmem(jb.g_ratio)[w] = static_cast<float>(s);
    }
  }
}

// Adam on real coordinates.  Segment l selects the variable (0 object,
// 1 probe, 2 positions, 3 sigma, 4 background); units are 1024-float blocks.
// A job whose window check failed keeps its variables and moments: its
// gradients are not valid, so no update is taken from them.
__global__ __launch_bounds__(NT) void k_adam(Launch la) {
  const UnitRef r = decode<1>(la);
  const JobDev& jb = *r.jb;
  if (*gmem(jb.status)) return;
  const int v = r.l;
  gf32* __restrict__ x = gmem(jb.var_flat[v]);
  const gf32* __restrict__ g = gmem(jb.grad_flat[v]);
  gf32* __restrict__ m = gmem(jb.adam_m[v]);
  gf32* __restrict__ s2 = gmem(jb.adam_v[v]);
  const float lr = jb.adam_lr[v];
  const long long n = jb.flat_n[v];
  const float b1 = jb.adam_beta1, b2 = jb.adam_beta2, eps = jb.adam_eps;
  const float bc1 = jb.adam_bc1, bc2 = jb.adam_bc2;
  const long long base = static_cast<long long>(r.u) * 1024;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long long i = base + threadIdx.x + q * NT;
    if (i < n) {
      const float gi = g[i];
      const float mi = b1 * m[i] + (1.f - b1) * gi;
      const float vi = b2 * s2[i] + (1.f - b2) * gi * gi;
      m[i] = mi;
      s2[i] = vi;
      x[i] -= lr * (mi * bc1) / (sqrtf(vi * bc2) + eps);
    }
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

template <int P, int... Ps>
int plan_of(int n, int* out, IntList<P, Ps...>) {
  if (n == P) {
    plan_fill(typename Plan<P>::type{}, out);
    return PlanInfo<P>::passes;
  }
  if constexpr (sizeof...(Ps) > 0) return plan_of(n, out, IntList<Ps...>{});
  return 0;
}

inline dim3 grid1(long long blocks) { return dim3(static_cast<unsigned>(blocks)); }

}  // namespace

int plan_radices(int n, int* out) {
  using All = IntList<64, 72, 80, 84, 90, 96, 128, 140, 150, 168, 189, 256, 280, 300, 315, 336,
                      343, 375, 384, 420, 480, 512, 560, 600, 675, 750, 768, 1024>;
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

int czt_len(int N) { return 2 * N; }
int czt_table_blocks(int N) { return (2 * N + NT - 1) / NT + (2 * N + NT - 1) / NT; }

int rows_per_det_block(int N) { return N <= 128 ? 16 : (N == 512 ? 4 : 8); }
int rows_per_adj_block(int N) { return N <= 128 ? 16 : (N == 512 ? 4 : 8); }
int rows_per_row_block(int N) { return N == 64 ? 32 : (N <= 256 ? 16 : 8); }
int adj_part_stride(int N) { return adj_stride(N); }

// LDS a column-adjoint block may use (gfx950: 160 KB per workgroup), less a
// margin for the reduction scratch.
constexpr size_t kColAdjLds = 156 * 1024;
constexpr size_t kLdsMax = 160 * 1024;  // LDS of one workgroup

// Zero-padded DFT sizes of N >= 256 have a grouped-position column-adjoint instance.
bool pair_capable(int N, int nl) { return N >= 256 && nl != czt_len(N); }

bool lds_group_fits(int N, int M, int nl) {
  const size_t G = static_cast<size_t>(col_group_adj(N, nl));
  const size_t acc = static_cast<size_t>(M) * N * G * sizeof(float2);
  const size_t buf = static_cast<size_t>(nl) * col_adj_lp(N, nl, static_cast<int>(G)) * sizeof(float2);
  return acc + buf <= kColAdjLds;
}

int probe_group_of(int N, int M, int nl) {
  // at N >= 384 register groups of three beat LDS groups of four where both
  // fit (3 harmonics x 4 modes at N = 384: column adjoint 13.9 -> 12.2 ms,
  // probe reduction 0.55 -> 0.73 ms per step); at N = 256 they do not
  // (4 x 3 modes: 2.45 -> 3.03 ms)
  if (N >= 384 && pair_fits(N, nl, kRegGroup)) return kRegGroup;
  if (lds_group_fits(N, M, nl)) return kProbeGroup;
  if (pair_fits(N, nl, kRegGroup)) return kRegGroup;
  return 1;
}

int col_sets_adj(int N, int nl) { return N / col_group_adj(N, nl); }

int obj_tile_rows(int H, int W, int slots) {
  const long long tiles16 =
      static_cast<long long>((W + kObjTileW - 1) / kObjTileW) * ((H + 15) / 16) * slots;
  if (tiles16 >= 1024) return 16;
  return tiles16 * 2 >= 1024 ? 8 : 4;
}

size_t col_adj_pair_lds(int N, int nl, int pg) {
  return static_cast<size_t>(pg) * N * col_group_adj(N, nl) * sizeof(float2);
}

// Whether the grouped column adjoint over pg positions fits in a block's
// LDS: Ohat of the group (dynamic) next to the transform buffer, the twiddle
// tables (at most nl + N entries) and the block sums.
bool pair_fits(int N, int nl, int pg) {
  if (!pair_capable(N, nl)) return false;
  const size_t G = static_cast<size_t>(col_group_adj(N, nl));
  const size_t tile = static_cast<size_t>(G) * pair_row_pitch(nl, static_cast<int>(G));
  const size_t nbuf = static_cast<size_t>(G) * pair_row_pitch(N, static_cast<int>(G));
  const size_t stat = ((tile > nbuf ? tile : nbuf) + nl + N) * sizeof(float2) + 64;
  return col_adj_pair_lds(N, nl, pg) + stat <= kLdsMax;
}

size_t col_adj_lds_of(int N, int nl, int M, int group) {
  if (group <= 1) return 0;
  return static_cast<size_t>(M) * N * col_group_adj(N, nl) * sizeof(float2);
}

hipError_t launch_write_table(int* dst, const int* data, int n, hipStream_t s) {
  for (int off = 0; off < n; off += kTableInts) {
    TablePayload p;
    const int cnt = n - off < kTableInts ? n - off : kTableInts;
    for (int i = 0; i < cnt; ++i) p.w[i] = data[off + i];
    hipLaunchKernelGGL(k_write_table, dim3(1), dim3(NT), 0, s, p, dst + off, cnt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_simple(int kind, const Launch& la, long long units, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  switch (kind) {
    case KZeroGrads: hipLaunchKernelGGL(k_zero_grads, grid1(units), dim3(NT), 0, s, la); break;
    case KSetStatus: hipLaunchKernelGGL(k_set_status, grid1(units), dim3(64), 0, s, la); break;
    case KValidate: hipLaunchKernelGGL(k_validate, grid1(units), dim3(NT), 0, s, la); break;
    case KPrep: hipLaunchKernelGGL(k_prep, grid1(units), dim3(NT), 0, s, la); break;
    case KProbeReduce: hipLaunchKernelGGL(k_probe_reduce, grid1(units), dim3(NT), 0, s, la); break;
    case KObjGather: hipLaunchKernelGGL(k_obj_gather, grid1(units), dim3(NT), 0, s, la); break;
    case KFinalize: hipLaunchKernelGGL(k_finalize_chunk, grid1(units), dim3(64), 0, s, la); break;
    case KAdam: hipLaunchKernelGGL(k_adam, grid1(units), dim3(NT), 0, s, la); break;
    case KCztTables: hipLaunchKernelGGL(k_czt_tables, grid1(units), dim3(NT), 0, s, la); break;
    case KBgReduce: hipLaunchKernelGGL(k_bg_reduce, grid1(units), dim3(NT), 0, s, la); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_loss_total(const Launch& la, long long units, const LossDev& loss, float scale,
                             hipStream_t s) {
  if (units <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_loss_total, grid1(units), dim3(64), 0, s, la, loss, scale);
  return hipGetLastError();
}

hipError_t launch_regulariser(const Launch& la, long long units, const LossDev& loss, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_regulariser, grid1(units), dim3(kRegBlock), 0, s, la, loss);
  return hipGetLastError();
}

hipError_t launch_row_fwd(int N, const Launch& la, long long units, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  return with_N(N, [&](auto nc) {
    constexpr int NN = decltype(nc)::value;
    hipLaunchKernelGGL(k_row_fwd<NN>, grid1(units * (NN / rb_row<NN>())), dim3(NT), 0, s, la);
    return hipGetLastError();
  });
}

hipError_t launch_col_fwd(int N, int nl, const Launch& la, long long units, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  return with_N(N, [&](auto nc) {
    constexpr int NN = decltype(nc)::value;
    return host_pad(nl, [&](auto pc) {
      constexpr int NL = decltype(pc)::value;
      hipLaunchKernelGGL((k_col_fwd<NN, NL>), grid1(units * (NN / col_group<NN>())), dim3(CNT), 0, s, la);
      return hipGetLastError();
    }, ColList<NN>{});
  });
}

template <int NN, int VAR>
void launch_det_inst(dim3 g, const Launch& la, const LossDev& loss, int mode, bool spill,
                     hipStream_t s) {
  switch (mode) {
    case 0: hipLaunchKernelGGL((k_det<NN, 0, VAR>), g, dim3(NT), 0, s, la, loss, spill); break;
    case 1: hipLaunchKernelGGL((k_det<NN, 1, (VAR > 1 ? 1 : VAR)>), g, dim3(NT), 0, s, la, loss, spill); break;
    case 2: hipLaunchKernelGGL((k_det<NN, 2, VAR>), g, dim3(NT), 0, s, la, loss, spill); break;
    default: hipLaunchKernelGGL((k_det<NN, 3, (VAR > 1 ? 1 : VAR)>), g, dim3(NT), 0, s, la, loss, spill); break;
  }
}

hipError_t launch_det(int N, const Launch& la, long long units, const LossDev& loss, int mode,
                      bool spill, int var, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  return with_N(N, [&](auto nc) {
    constexpr int NN = decltype(nc)::value;
    const dim3 g = grid1(units * (NN / rb_det<NN>()));
    if (var == 2) launch_det_inst<NN, 2>(g, la, loss, mode, spill, s);
    else if (var == 1) launch_det_inst<NN, 1>(g, la, loss, mode, spill, s);
    else launch_det_inst<NN, 0>(g, la, loss, mode, spill, s);
    return hipGetLastError();
  });
}

hipError_t launch_resample_loss(int N, const Launch& la, long long units, const LossDev& loss,
                                bool forward, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  const int gx = (N * N + NT - 1) / NT;
  hipLaunchKernelGGL(k_resample_loss, grid1(units * gx), dim3(NT), 0, s, la, loss, forward, gx);
  return hipGetLastError();
}

hipError_t launch_resample_T(int N, const Launch& la, long long units, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  const int gx = (N * N + NT - 1) / NT;
  hipLaunchKernelGGL(k_resample_T, grid1(units * gx), dim3(NT), 0, s, la, gx);
  return hipGetLastError();
}

template <int NN, int NL, bool RATIO>
hipError_t launch_col_adj_inst(dim3 g, const Launch& la, size_t dyn_lds, bool grouped,
                               hipStream_t s) {
  if (!grouped) {
    hipLaunchKernelGGL((k_col_adj<NN, NL, false, RATIO>), g, dim3(col_adj_threads(NN, NL)), 0, s, la);
    return hipGetLastError();
  }
  if (dyn_lds) {
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_col_adj<NN, NL, true, RATIO>),
        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(dyn_lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_col_adj<NN, NL, true, RATIO>), g, dim3(col_adj_threads(NN, NL)), dyn_lds, s, la);
  return hipGetLastError();
}

template <int NN, int NL>
hipError_t launch_col_adj_pair_inst(dim3 g, const Launch& la, hipStream_t s) {
  const size_t dyn = col_adj_pair_lds(NN, NL, kRegGroup);
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_col_adj_pair<NN, NL>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(dyn));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_col_adj_pair<NN, NL>), g, dim3(col_adj_threads(NN, NL)), dyn, s, la);
  return hipGetLastError();
}

hipError_t launch_col_adj_pair(int N, int nl, const Launch& la, long long units, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  if (!pair_capable(N, nl)) return hipErrorInvalidValue;
  return with_N(N, [&](auto nc) {
    constexpr int NN = decltype(nc)::value;
    return host_pad(nl, [&](auto pc) {
      constexpr int NL = decltype(pc)::value;
      if constexpr (NN >= 256 && NL != czt_nb<NN>())
        return launch_col_adj_pair_inst<NN, NL>(grid1(units * (NN / col_group_adj(NN, NL))), la, s);
      return hipErrorInvalidValue;
    }, ColList<NN>{});
  });
}

hipError_t launch_col_adj(int N, int nl, const Launch& la, long long units, size_t dyn_lds,
                          bool grouped, bool ratio, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  return with_N(N, [&](auto nc) {
    constexpr int NN = decltype(nc)::value;
    return host_pad(nl, [&](auto pc) {
      constexpr int NL = decltype(pc)::value;
      const dim3 g = grid1(units * (NN / col_group_adj(NN, NL)));
      if constexpr (NL == czt_nb<NN>()) {
        if (ratio) return launch_col_adj_inst<NN, NL, true>(g, la, dyn_lds, grouped, s);
      }
      return launch_col_adj_inst<NN, NL, false>(g, la, dyn_lds, grouped, s);
    }, ColList<NN>{});
  });
}

hipError_t launch_row_adj(int N, const Launch& la, long long units, hipStream_t s) {
  if (units <= 0) return hipSuccess;
  return with_N(N, [&](auto nc) {
    constexpr int NN = decltype(nc)::value;
    hipLaunchKernelGGL(k_row_adj<NN>, grid1(units * (NN / rb_adj<NN>())), dim3(NT), 0, s, la);
    return hipGetLastError();
  });
}

}  // namespace ptycho
