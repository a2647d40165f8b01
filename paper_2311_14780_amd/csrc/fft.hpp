// fft.hpp - LDS-resident mixed-radix Stockham FFTs for gfx950 (wave64).
//
// A workgroup transforms LINES lines of length n at once.  The length and its
// radix plan are compile-time constants, so every butterfly, twiddle index and
// LDS address is resolved by the compiler.  Each pass reads all of its inputs
// into registers, synchronises, and writes its outputs back in place (one LDS
// buffer, no ping-pong), so the whole FFT needs n * LINES complex words of LDS.
// The first pass may take its inputs from a caller functor (global memory with
// zero padding, fused pointwise products) and the last pass hands its outputs
// to a caller functor (cropping, scaling, fused products, global stores).
//
// Stockham autosort (natural-order output) for pass radix R with Ns = product
// of earlier radices: butterfly j reads x[j + r n/R], multiplies by
// w_{Ns R}^{r (j mod Ns)}, takes a length-R DFT and writes
// y[(j / Ns) Ns R + (j mod Ns) + r Ns].  Twiddles come from a table
// T_n[t] = exp(-2 pi i t / n) computed in float64 on the host.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace ptycho {

// Address-space qualified pointers.  Pointers that reach a kernel through
// memory (the job table) or through an out-of-line function's arguments are
// generic, and generic accesses compile to flat instructions, which also
// hold the LDS wait counter: every LDS wait of an FFT pass would then wait
// for outstanding HBM traffic too.  Kernels therefore convert such pointers
// with gmem() and access complex data through ldv/stv.
// Complex values behind such pointers use the native two-float vector type.
#define PTYCHO_GLOBAL __attribute__((address_space(1)))
#define PTYCHO_LDS __attribute__((address_space(3)))
using vf2 = float __attribute__((ext_vector_type(2)));
using gf2 = PTYCHO_GLOBAL vf2;
using lf2 = PTYCHO_LDS vf2;
using lf32 = PTYCHO_LDS float;
using gf32 = PTYCHO_GLOBAL float;

__device__ __forceinline__ gf2* gmem(float2* p) { return (gf2*)p; }
__device__ __forceinline__ const gf2* gmem(const float2* p) { return (const gf2*)p; }
template <class T>
__device__ __forceinline__ PTYCHO_GLOBAL T* gmem(T* p) { return (PTYCHO_GLOBAL T*)p; }
template <class T>
__device__ __forceinline__ const PTYCHO_GLOBAL T* gmem(const T* p) { return (const PTYCHO_GLOBAL T*)p; }

// A wave-uniform table pointer that the compiler cannot see through.  Loads
// through it are not hoisted out of an enclosing loop, which would keep every
// thread's loaded table values in registers across the whole loop.  The
// table lives in global memory: the rebuilt pointer says so.
template <class P>
__device__ __forceinline__ const gf2* opaque_table(P p) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(p);
  unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a));
  unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi));
  return reinterpret_cast<const gf2*>((static_cast<unsigned long long>(hi) << 32) | lo);
}

// A wave-uniform global pointer held in scalar registers (loads through it
// take a scalar base and a vector offset).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a >> 32));
  return reinterpret_cast<T*>((static_cast<unsigned long long>(hi) << 32) | lo);
}

// Element access that works for generic float2 pointers and for the
// address-space qualified vector pointers above.
__device__ __forceinline__ float2 ldv(const float2* p, int i) { return p[i]; }
__device__ __forceinline__ float2 ldv(const lf2* p, int i) {
  const vf2 t = p[i];
  return make_float2(t.x, t.y);
}
template <class I>
__device__ __forceinline__ float2 ldv(const gf2* p, I i) {
  const vf2 t = p[i];
  return make_float2(t.x, t.y);
}
__device__ __forceinline__ void stv(float2* p, int i, float2 v) { p[i] = v; }
__device__ __forceinline__ void stv(lf2* p, int i, float2 v) { p[i] = vf2{v.x, v.y}; }
template <class I>
__device__ __forceinline__ void stv(gf2* p, I i, float2 v) { p[i] = vf2{v.x, v.y}; }
// Streaming store (nontemporal): for planes written once and read by a later
// kernel, in runs of whole 128-byte lines.  Partial lines written this way are
// not merged in L2 (64-byte column segments got slower).
template <class I>
__device__ __forceinline__ void stv_nt(gf2* p, I i, float2 v) {
  __builtin_nontemporal_store(vf2{v.x, v.y}, p + i);
}

// ----------------------------------------------------------- complex helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulconj(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 cmul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------ compile-time cos / sin table
// Taylor series in float64 after reduction to [-pi, pi]; used only in constant
// expressions (radix constants), never at run time.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_reduce(double x) {
  while (x > kPi) x -= 2.0 * kPi;
  while (x < -kPi) x += 2.0 * kPi;
  return x;
}
constexpr double ct_sin(double x) {
  x = ct_reduce(x);
  double term = x, sum = x;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos(double x) {
  x = ct_reduce(x);
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// c[j] = cos(2 pi j / R), s[j] = sin(2 pi j / R)
template <int R>
struct Roots {
  float c[R];
  float s[R];
  constexpr Roots() : c(), s() {
    for (int j = 0; j < R; ++j) {
      c[j] = static_cast<float>(ct_cos(2.0 * kPi * j / R));
      s[j] = static_cast<float>(ct_sin(2.0 * kPi * j / R));
    }
  }
};

// --------------------------------------------------------- small DFT kernels
// In-place length-R DFT, forward (exp(-2 pi i k r / R)) or inverse (exp(+...)).
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = cmul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

// Odd prime R (3, 5, 7): symmetric/antisymmetric pairs.
template <int R, bool INV>
struct DftOdd {
  __device__ __forceinline__ static void run(float2* v) {
    constexpr int h = (R - 1) / 2;
    constexpr Roots<R> w{};
    float2 sp[h], sm[h];
#pragma unroll
    for (int r = 1; r <= h; ++r) {
      sp[r - 1] = cadd(v[r], v[R - r]);
      sm[r - 1] = csub(v[r], v[R - r]);
    }
    float2 out[R];
    float2 y0 = v[0];
#pragma unroll
    for (int r = 0; r < h; ++r) y0 = cadd(y0, sp[r]);
    out[0] = y0;
#pragma unroll
    for (int k = 1; k <= h; ++k) {
      float2 a = v[0];
      float2 b = make_float2(0.f, 0.f);
#pragma unroll
      for (int r = 1; r <= h; ++r) {
        const int j = (k * r) % R;
        a.x = fmaf(sp[r - 1].x, w.c[j], a.x);
        a.y = fmaf(sp[r - 1].y, w.c[j], a.y);
        b.x = fmaf(sm[r - 1].x, w.s[j], b.x);
        b.y = fmaf(sm[r - 1].y, w.s[j], b.y);
      }
      // forward: y_k = a - i b, y_{R-k} = a + i b
      const float2 mib = cmul_mi<INV>(b);
      out[k] = cadd(a, mib);
      out[R - k] = csub(a, mib);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = out[r];
  }
};

template <bool INV> struct Dft<3, INV> : DftOdd<3, INV> {};
template <bool INV> struct Dft<5, INV> : DftOdd<5, INV> {};
template <bool INV> struct Dft<7, INV> : DftOdd<7, INV> {};

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    constexpr float h = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    // o[k] *= w8^k ; w8 = exp(-+ 2 pi i / 8)
    const float sg = INV ? 1.f : -1.f;
    float2 o1 = make_float2(h * (o[1].x - sg * o[1].y), h * (o[1].y + sg * o[1].x));
    float2 o2 = cmul_mi<INV>(o[2]);
    float2 o3 = make_float2(h * (-o[3].x - sg * o[3].y), h * (-o[3].y + sg * o[3].x));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// Composite R = R1 * R2 by one decimation-in-time step:
// y[k1 + R1 k2] = sum_{n2} w_R^{n2 k1} w_R2^{n2 k2} DFT_R1(v[R2 n1 + n2])[k1].
template <int R1, int R2, bool INV>
struct DftComposite {
  __device__ __forceinline__ static void run(float2* v) {
    constexpr int R = R1 * R2;
    constexpr Roots<R> w{};
    float2 e[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) e[n2][n1] = v[R2 * n1 + n2];
      Dft<R1, INV>::run(e[n2]);
#pragma unroll
      for (int k1 = 1; k1 < R1; ++k1) {
        const int j = (n2 * k1) % R;
        if (j != 0) {
          const float2 tw = make_float2(w.c[j], INV ? w.s[j] : -w.s[j]);
          e[n2][k1] = cmul(e[n2][k1], tw);
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = e[n2][k1];
      Dft<R2, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
  }
};

// Coprime R = R1 * R2 by the prime-factor (Good-Thomas) index maps, which
// need no internal twiddle products: with input n = (R2 n1 + R1 n2) mod R and
// output k = (e1 k1 + e2 k2) mod R, where e1 = R2 (R2^-1 mod R1) and
// e2 = R1 (R1^-1 mod R2), n k = R2 n1 k1 + R1 n2 k2 (mod R), so the length-R
// DFT is a length-R1 DFT over n1 for every n2 followed by a length-R2 DFT
// over n2 for every k1.  Both maps are compile-time register renamings.
constexpr int ct_inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;  // m == 1
}
template <int R1, int R2, bool INV>
struct DftPfa {
  __device__ __forceinline__ static void run(float2* v) {
    constexpr int R = R1 * R2;
    constexpr int E1 = R2 * ct_inv_mod(R2 % R1, R1);
    constexpr int E2 = R1 * ct_inv_mod(R1 % R2, R2);
    float2 a[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) a[n2][n1] = v[(R2 * n1 + R1 * n2) % R];
      Dft<R1, INV>::run(a[n2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = a[n2][k1];
      Dft<R2, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[(E1 * k1 + E2 * k2) % R] = t[k2];
    }
  }
};

template <bool INV> struct Dft<6, INV> : DftPfa<2, 3, INV> {};
template <bool INV> struct Dft<9, INV> : DftComposite<3, 3, INV> {};
template <bool INV> struct Dft<10, INV> : DftPfa<2, 5, INV> {};
template <bool INV> struct Dft<12, INV> : DftPfa<4, 3, INV> {};
template <bool INV> struct Dft<14, INV> : DftPfa<2, 7, INV> {};
template <bool INV> struct Dft<15, INV> : DftPfa<3, 5, INV> {};
template <bool INV> struct Dft<16, INV> : DftComposite<4, 4, INV> {};
template <bool INV> struct Dft<18, INV> : DftPfa<2, 9, INV> {};
template <bool INV> struct Dft<20, INV> : DftPfa<4, 5, INV> {};
template <bool INV> struct Dft<21, INV> : DftPfa<3, 7, INV> {};
template <bool INV> struct Dft<24, INV> : DftPfa<8, 3, INV> {};
template <bool INV> struct Dft<25, INV> : DftComposite<5, 5, INV> {};
template <bool INV> struct Dft<27, INV> : DftComposite<3, 9, INV> {};
template <bool INV> struct Dft<28, INV> : DftPfa<4, 7, INV> {};
template <bool INV> struct Dft<30, INV> : DftPfa<5, 6, INV> {};
template <bool INV> struct Dft<32, INV> : DftComposite<4, 8, INV> {};
template <bool INV> struct Dft<35, INV> : DftPfa<5, 7, INV> {};

// ------------------------------------------------------------- radix plans
template <int... Rs>
struct Radices {};

template <int n>
struct Plan;  // Plan<n>::type = Radices<...>, product n

#define PTYCHO_PLAN(n, ...) \
  template <>               \
  struct Plan<n> {          \
    using type = Radices<__VA_ARGS__>; \
  };

// Lengths that are multiples of 16 use the skewed row layout (see Lds) and
// power-of-two radices first; most others start with an odd radix, so that the
// strided writes of the first pass do not pile onto a few LDS banks.  420, 600,
// 675 and 750 instead take the order with the fewest butterfly instructions per
// line when one wave transforms a line on its own (the detector kernel, which
// is bound by vector-ALU issue there): 750 as 10 x 15 x 5 needs 635 wave
// instructions per line against 717 for 5 x 15 x 10 (5 harmonics x 8 modes,
// N = 512: detector kernel 172.7 -> 166.3 ms, column forward 80.9 -> 79.3 ms).
PTYCHO_PLAN(64, 8, 8)
PTYCHO_PLAN(72, 9, 8)
PTYCHO_PLAN(80, 16, 5)
PTYCHO_PLAN(84, 7, 12)
PTYCHO_PLAN(90, 9, 10)
PTYCHO_PLAN(96, 8, 12)
PTYCHO_PLAN(128, 16, 8)
PTYCHO_PLAN(140, 7, 5, 4)
PTYCHO_PLAN(150, 15, 10)
PTYCHO_PLAN(168, 7, 3, 8)
PTYCHO_PLAN(189, 7, 3, 9)
// 256: three passes (32, 32 and 64 butterflies per line) rather than 16 x 16,
// whose 16 butterflies per line left half the threads of a 16-line, 512-thread
// column block idle (loss + gradient step of 400 positions x 4 wavelengths x
// 3 modes at N = 256: 8.13 -> 8.03 ms)
PTYCHO_PLAN(256, 8, 8, 4)
PTYCHO_PLAN(280, 7, 5, 8)
PTYCHO_PLAN(300, 5, 5, 12)
PTYCHO_PLAN(315, 7, 5, 9)
PTYCHO_PLAN(336, 16, 3, 7)
PTYCHO_PLAN(343, 7, 7, 7)
PTYCHO_PLAN(375, 15, 5, 5)
PTYCHO_PLAN(384, 16, 8, 3)
PTYCHO_PLAN(420, 12, 5, 7)
PTYCHO_PLAN(480, 16, 6, 5)
PTYCHO_PLAN(512, 8, 8, 8)
PTYCHO_PLAN(560, 16, 5, 7)
PTYCHO_PLAN(600, 12, 10, 5)
PTYCHO_PLAN(675, 15, 15, 3)
PTYCHO_PLAN(750, 10, 15, 5)
// Bluestein lengths 2N of the exact-ratio propagator (N = 384, 512)
PTYCHO_PLAN(768, 16, 16, 3)
PTYCHO_PLAN(1024, 16, 16, 4)
#undef PTYCHO_PLAN

// Radices of a plan as a host/device array (for building twiddle tables).
template <int... Rs>
constexpr int plan_count(Radices<Rs...>) { return sizeof...(Rs); }
template <int n>
struct PlanInfo {
  static constexpr int passes = plan_count(typename Plan<n>::type{});
};
template <int... Rs>
inline void plan_fill(Radices<Rs...>, int* out) {
  const int r[] = {Rs...};
  for (int i = 0; i < static_cast<int>(sizeof...(Rs)); ++i) out[i] = r[i];
}

// ------------------------------------------------------ the Stockham engine
// Layout of element i of line `line` in the LDS buffer.
//  LINE_FAST = true : buf[i * LP + line]  (column groups: lanes walk lines;
//                     LP = lines + 1)
//  LINE_FAST = false: buf[line * LP + i (+ i / 16 if n % 16 == 0)]  (rows:
//                     lanes walk elements; for lengths that are multiples of
//                     16 one skew word per 16 elements keeps the power-of-two
//                     strided writes spread over the LDS banks).
template <int n>
constexpr bool row_skew() { return n % 16 == 0; }
constexpr int row_lp(int n) { return n % 16 == 0 ? n + (n >> 4) + 1 : n + 1; }

template <int n, int LP, bool LINE_FAST>
struct Lds {
  __device__ __forceinline__ static int at(int line, int i) {
    if (LINE_FAST) return i * LP + line;
    return row_skew<n>() ? line * LP + i + (i >> 4) : line * LP + i;
  }
  // Address of element base + r * STRIDE, r a compile-time loop index.  When
  // the skew of the element is known up to a constant per r it is folded into
  // an immediate offset from the address of `base`:
  //  MODE 1: the R elements lie in one aligned 16-element block (same skew);
  //  MODE 2: base < STRIDE and STRIDE divides 16 (skew = (r STRIDE) / 16);
  //  MODE 0: anything else, computed per element.
  template <int STRIDE, int MODE>
  __device__ __forceinline__ static int at_r(int line, int base, int r) {
    if (LINE_FAST) return at(line, base) + r * STRIDE * LP;
    if (!row_skew<n>()) return at(line, base) + r * STRIDE;
    if (STRIDE % 16 == 0) return at(line, base) + r * (STRIDE + STRIDE / 16);
    if (MODE == 1) return at(line, base) + r * STRIDE;
    if (MODE == 2) return at(line, base) + r * STRIDE + ((r * STRIDE) >> 4);
    return at(line, base + r * STRIDE);
  }
};

// Twiddle table of length n (host-built, float64 -> float32): for every pass
// p > 0 with radix R and Ns = product of earlier radices, Ns * (R - 1)
// entries w_{Ns R}^{r k} (forward sign) stored as [k][r - 1], k < Ns,
// 1 <= r < R; passes are concatenated in plan order.

template <int R, int... Rest>
struct FirstRadix {
  static constexpr int value = R;
};
template <class P>
struct FirstRadixOf;
template <int... Rs>
struct FirstRadixOf<Radices<Rs...>> {
  static constexpr int value = FirstRadix<Rs...>::value;
};

// Synchronisation of a transform.  With NT = 64 the lines belong to one
// wave (its own LDS region): a wave's LDS operations complete in program
// order, so the passes need only a compiler fence between the reads and the
// writes of the in-place buffer, and waves never wait for each other (a
// wave stalled on a global load does not hold the others of its block).
// With NT > 64 the whole workgroup shares the lines and each pass ends with
// a workgroup barrier.
template <int NT>
__device__ __forceinline__ int fft_tid() {
  return NT == 64 ? static_cast<int>(threadIdx.x & 63u) : static_cast<int>(threadIdx.x);
}
template <int NT>
__device__ __forceinline__ void fft_sync() {
  if constexpr (NT == 64) {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Inputs of the first pass of an FFT, loaded ahead of time with
// fft_first_load and handed to fft_lines in place of a load functor, so that
// the loads of the next transform are in flight during the current one.
template <int n, int LINES, int NT, bool LINE_FAST>
struct PreIn {
  static constexpr int R = FirstRadixOf<typename Plan<n>::type>::value;
  static constexpr int NB = n / R;
  static constexpr int BF = LINES * NB;
  static constexpr int ITER = (BF + NT - 1) / NT;
  float2 v[ITER][R];
};
template <class T>
struct IsPreIn : std::false_type {};
template <int n, int LINES, int NT, bool LF>
struct IsPreIn<PreIn<n, LINES, NT, LF>> : std::true_type {};

// Issues the first-pass loads of an FFT: in.v[it][r] = load(line, j + r NB).
template <int n, int LINES, int NT, bool LINE_FAST, class Load>
__device__ __forceinline__ void fft_first_load(PreIn<n, LINES, NT, LINE_FAST>& in,
                                               const Load& load) {
  using P = PreIn<n, LINES, NT, LINE_FAST>;
  const int tid = fft_tid<NT>();
#pragma unroll
  for (int it = 0; it < P::ITER; ++it) {
    const int b = tid + it * NT;
    if ((P::BF % NT == 0) || b < P::BF) {
      const int line = LINE_FAST ? (b % LINES) : (b / P::NB);
      const int j = LINE_FAST ? (b / LINES) : (b % P::NB);
#pragma unroll
      for (int r = 0; r < P::R; ++r) in.v[it][r] = load(line, j + r * P::NB);
    }
  }
}

// Entries of the twiddle table of length n: sum over the passes after the
// first of Ns (R - 1), i.e. n - R1.
template <int n>
constexpr int tw_len() { return n - FirstRadixOf<typename Plan<n>::type>::value; }

// Twiddles loaded per butterfly: w and w^2 (one 16-byte load); the higher
// powers are products w^r = w^(r/2) w^(r - r/2) (at most a few roundings).
// Loading all R - 1 values per thread made the twiddle reads the largest
// stream through the L1 cache (every thread reads its own copy).  Short
// transforms (n < 192: windows of 64 and 128, whose launches are small and
// latency-bound) load every power instead, which keeps each twiddle at one
// rounding: the Poisson-loss gradient weighs dim pixels by 1 - I^/I', so it
// amplifies the transform error there (64 x 64 window, 1e4 photons: object
// gradient 8e-5 -> 3e-5 relative L2 against the float64 oracle).
constexpr int tw_loaded(int n) { return n < 192 ? 16 : 2; }

// Twiddles of one pass for this thread's butterflies, [iteration][r - 1].
template <int n, int R, int LINES, int NT>
struct PassTw {
  static constexpr int NB = n / R;
  static constexpr int BF = LINES * NB;
  static constexpr int ITER = (BF + NT - 1) / NT;
  static constexpr int Q = R - 1 < tw_loaded(n) ? R - 1 : tw_loaded(n);
  float2 w[ITER][Q > 0 ? Q : 1];
};

// Issues the loads of the twiddles of pass (R, Ns, TOFF) for this thread.
template <int n, int R, int Ns, int TOFF, int LINES, int NT, bool LINE_FAST, class Tw>
__device__ __forceinline__ void load_pass_tw(Tw tw, PassTw<n, R, LINES, NT>& out) {
  if constexpr (Ns > 1) {
    using P = PassTw<n, R, LINES, NT>;
    const int tid = fft_tid<NT>();
#pragma unroll
    for (int it = 0; it < P::ITER; ++it) {
      const int b = tid + it * NT;
      if ((P::BF % NT == 0) || b < P::BF) {
        const int j = LINE_FAST ? (b / LINES) : (b % P::NB);
        // one address, constant offsets: the values are contiguous
        const auto t = tw + TOFF + (j % Ns) * (R - 1);
#pragma unroll
        for (int r = 1; r <= P::Q; ++r) out.w[it][r - 1] = ldv(t, r - 1);
      }
    }
  }
}

// One Stockham pass.  FIRST: inputs from `load(line, i)`; otherwise from LDS.
// LAST: outputs to `store(line, i, v)`; otherwise to LDS.  `wcur` holds this
// pass's twiddles, loaded during the previous pass; `prefetch()` issues the
// next pass's twiddle loads once this pass's reads are done, so that they
// are in flight across the barrier and the write phase.
template <int n, int R, int Ns, bool FIRST, bool LAST, bool INV, int LINES, int NT, int LP,
          bool LINE_FAST, class Buf, class Load, class Store, class Prefetch>
__device__ __forceinline__ void stockham_pass(Buf buf, const PassTw<n, R, LINES, NT>& wcur,
                                              const Load& load, const Store& store,
                                              const Prefetch& prefetch) {
  constexpr int NB = n / R;             // butterflies per line
  constexpr int BF = LINES * NB;        // butterflies per pass
  constexpr int ITER = (BF + NT - 1) / NT;
  using Ix = Lds<n, LP, LINE_FAST>;
  // reads: i = j + r NB with j < NB
  constexpr int RD_MODE = (16 % NB == 0) ? 2 : 0;
  // writes: o = base + r Ns, base = (j / Ns) Ns R + j % Ns; all o of a
  // butterfly lie in one aligned block of Ns R elements
  constexpr int WR_MODE = (16 % (Ns * R) == 0) ? 1 : 0;
  const int tid = fft_tid<NT>();
  float2 v[ITER][R];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int b = tid + it * NT;
    if ((BF % NT == 0) || b < BF) {
      const int line = LINE_FAST ? (b % LINES) : (b / NB);
      const int j = LINE_FAST ? (b / LINES) : (b % NB);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (!FIRST)
          v[it][r] = ldv(buf, Ix::template at_r<NB, RD_MODE>(line, j, r));
        else if constexpr (IsPreIn<Load>::value)
          v[it][r] = load.v[it][r];
        else
          v[it][r] = load(line, j + r * NB);
      }
      if (Ns > 1) {
        constexpr int Q = PassTw<n, R, LINES, NT>::Q;
        float2 wr[R];
#pragma unroll
        for (int r = 1; r < R; ++r) wr[r] = r <= Q ? wcur.w[it][r - 1] : cmul(wr[r / 2], wr[r - r / 2]);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 ww = wr[r];
          if (INV) ww.y = -ww.y;
          v[it][r] = cmul(v[it][r], ww);
        }
      }
      Dft<R, INV>::run(v[it]);
    }
  }
  prefetch();
  fft_sync<NT>();  // every read of this pass precedes any write (in-place LDS)
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int b = tid + it * NT;
    if ((BF % NT == 0) || b < BF) {
      const int line = LINE_FAST ? (b % LINES) : (b / NB);
      const int j = LINE_FAST ? (b / LINES) : (b % NB);
      const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (LAST)
          store(line, base + r * Ns, v[it][r]);
        else
          stv(buf, Ix::template at_r<Ns, WR_MODE>(line, base, r), v[it][r]);
      }
    }
  }
  fft_sync<NT>();
}


template <int n, int Ns, int TOFF, bool FIRST, bool INV, int LINES, int NT, int LP, bool LINE_FAST,
          class Buf, class Tw, class Load, class Store, int R, int... Rest>
__device__ __forceinline__ void stockham_run(Buf buf, Tw tw, const PassTw<n, R, LINES, NT>& wcur,
                                             const Load& load, const Store& store,
                                             Radices<R, Rest...>) {
  constexpr bool LAST = sizeof...(Rest) == 0;
  if constexpr (LAST) {
    stockham_pass<n, R, Ns, FIRST, true, INV, LINES, NT, LP, LINE_FAST>(buf, wcur, load, store,
                                                                          [] {});
  } else {
    constexpr int NEXT_TOFF = TOFF + (Ns > 1 ? Ns * (R - 1) : 0);
    constexpr int R2 = FirstRadix<Rest...>::value;
    PassTw<n, R2, LINES, NT> wnext;
    stockham_pass<n, R, Ns, FIRST, false, INV, LINES, NT, LP, LINE_FAST>(
        buf, wcur, load, store, [&] {
          load_pass_tw<n, R2, Ns * R, NEXT_TOFF, LINES, NT, LINE_FAST>(tw, wnext);
        });
    stockham_run<n, Ns * R, NEXT_TOFF, false, INV, LINES, NT, LP, LINE_FAST>(
        buf, tw, wnext, load, store, Radices<Rest...>{});
  }
}

// Full FFT of LINES lines of length n: inputs via load(line, i) (i in [0, n)),
// outputs via store(line, i, value).  `buf` must hold LINES lines laid out as
// Lds<n, LP, LINE_FAST>.  The call begins with the first pass's reads (the
// caller must have synchronised any earlier use of `buf`) and ends with a
// workgroup barrier (NT = 64: a wave fence; the lines and `buf` are then the
// calling wave's own).  Unnormalised in both directions.
template <int n, bool INV, int LINES, int NT, int LP, bool LINE_FAST, class Buf, class Tw,
          class Load, class Store>
__device__ __forceinline__ void fft_lines(Buf buf, Tw tw, const Load& load, const Store& store) {
  using Plan0 = typename Plan<n>::type;
  PassTw<n, FirstRadixOf<Plan0>::value, LINES, NT> w0;  // the first pass has no twiddles
  if constexpr (std::is_same_v<Tw, const lf2*>) {
    // a table in LDS: its loads wait on the LDS counter, not behind the
    // global loads in flight
    stockham_run<n, 1, 0, true, INV, LINES, NT, LP, LINE_FAST>(buf, tw, w0, load, store, Plan0{});
  } else {
    // The twiddle base is made opaque so that the (loop-invariant) twiddle
    // loads of an FFT stay inside any loop around the call.
    const gf2* tg = opaque_table(tw);
    stockham_run<n, 1, 0, true, INV, LINES, NT, LP, LINE_FAST>(buf, tg, w0, load, store, Plan0{});
  }
}

}  // namespace ptycho
