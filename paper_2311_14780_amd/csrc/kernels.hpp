// kernels.hpp - host-side launch interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace ptycho {

constexpr int kMaxL = 16;  // slots: wavelength x sample mode
constexpr int kVars = 5;  // object, probe, positions, sigma, background

// One job of a call, as seen by the kernels (kept in device memory; every
// launch reads it through the job index of its work segments).
struct JobDev {
  // variables and fixed inputs (caller memory)
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
  // L counts slots s = l Ns + n (wavelength l, sample mode n): the object,
  // every per-wavelength workspace array and the per-slot tables below are
  // indexed by slot; the probe of slot s is P_{s / Ns} (Eq. 1's sample modes
  // share the illumination).
  int K, L, M, N, H, W;
  int Lw, Ns;              // wavelengths, sample modes (L = Lw Ns)
  int pad[kMaxL];          // DFT length per wavelength (2N for the exact-ratio propagator)
  float pad_scale[kMaxL];  // 1 / sqrt(pad[l]) (zero-padded DFT only)
  const float2* tw_N;            // twiddles of length N
  const float2* tw_pad[kMaxL];   // twiddles of length pad[l]
  // Exact-ratio (chirp z-transform) propagator of wavelength l, or null:
  // [N] exp(-i pi r^2 / alpha) | [N] alpha^-1/2 exp(-i pi u_j^2 / alpha) |
  // [2N] DFT of the chirp kernel / 2N (workspace, filled by k_czt_tables)
  float2* czt[kMaxL];
  double czt_alpha[kMaxL];  // alpha_l (0: zero-padded DFT)
  // outputs (caller memory, each may be null)
  float* loss;
  float2* g_object;
  float2* g_probe;
  float* g_pos;
  float* g_sigma;
  float* g_background;  // [N][N]
  float* g_ratio;       // [L] dL/d alpha_l (exact-ratio wavelengths), or null
  float* out;           // forward intensities [K][N][N]
  // workspace of this job for one chunk of C positions
  int* status;
  double* loss_k;       // [K]
  double* ratio_k;      // [K][Lw] per-position dL/d alpha_l (g_ratio only)
  float2* ramp;         // [C][2][N]    exp(+2 pi i f delta), y then x
  float2* X;            // [C][L][N][N] row-shifted patch, later G_A
  float2* Y;            // [C][L][M][N][N] column DFT -> Psi -> Z -> probe-gradient terms
  float2* GX;           // [C][L][N][N] gradient after the adjoint column shift; between
                        // the detector kernel and the column adjoint its first C N^2
                        // floats hold 2 scale w dL/dI per position (background gradient)
  float* loss_part;     // [C][n_loss]
  float* dy_part;       // [C][L][N / G]
  float* sg_part;       // [C][L][N / G]
  float* dx_part;       // [C][L][N / RBadj]
  float* reg_part;      // [L][ceil(H W / 256)] regulariser value per pixel block
  float* ra_part;       // [C][L][N / RBdet] alpha-derivative terms of the detector rows
  float* rb_part;       // [C][L][N / G]     alpha-derivative terms of the columns
  float* ibuf;          // [C][N][N] (resampling only) I + B, then R^T g
  float* gbuf;          // [C][N][N] (resampling only) weighted dloss/dI'
  int C;                // positions per chunk (iteration i covers [i C, i C + C))
  int n_loss;           // loss partials per position
  int want_adjoint;
  int probe_group;      // positions whose probe-gradient terms one column-adjoint
                        // block sums in LDS (1: one term per position)
  int obj_tile_h;       // rows of the object-gradient gather's tiles (4, 8 or 16)
  // Flat float views selected by a segment's l in the gradient-zeroing and
  // Adam launches (0 object, 1 probe, 2 positions, 3 sigma, 4 background).
  // The host fills them so that those kernels pick their arrays by index:
  // a multi-way branch on l that assigns pointers was compiled into code
  // that left the pointer registers of the later cases unset.
  float* var_flat[kVars];
  float* grad_flat[kVars + 1];  // may be null; [kVars] = g_ratio (zeroing only)
  long long flat_n[kVars + 1];  // floats in each
  // Adam (ptycho_step)
  float* adam_m[kVars];
  float* adam_v[kVars];
  float adam_lr[kVars];
  float adam_beta1, adam_beta2, adam_eps, adam_bc1, adam_bc2;
};
static_assert(sizeof(JobDev) % sizeof(int) == 0, "the table writer copies whole ints");

// A run of work units of one job (and one wavelength, or sub-selector l).
struct Seg {
  int job;
  int l;
  int unit0;  // first unit (units of all segments of a launch are numbered 0..)
  int unused;
};

// Arguments common to every launch.
struct Launch {
  const JobDev* jobs;
  const Seg* segs;
  int nseg;
  int iter;  // chunk index
};

// Loss parameters as used by the kernels.
struct LossDev {
  int kind;
  float eps;
  float gscale;     // 2 * scale: folds the factor of G_Psi = 2 g Psi
  float noise_var;  // read-noise variance of the mixed-noise loss
  float l1, tv, tv_eps;  // amplitude regularisers
};

// Kernel-argument payload of the table writer.
constexpr int kTableInts = 512;
struct TablePayload {
  int w[kTableInts];
};

// Kinds of the simple launches (launch_simple).
enum SimpleKind {
  KZeroGrads, KSetStatus, KValidate, KPrep, KProbeReduce, KObjGather, KFinalize, KAdam, KCztTables,
  KBgReduce
};
// Blocks of k_czt_tables per (job, wavelength) with the exact-ratio propagator.
int czt_table_blocks(int N);

// Radix plan of an FFT length (returns the number of passes, 0 if unknown).
int plan_radices(int n, int* out);

// Per-pass twiddle table of length n on this device (layout in fft.hpp).
const float2* twiddles(int n);
int init_twiddles();  // returns 0 or a PTYCHO_E* code
void release_twiddles();

bool supported(int N, int nl);
// Bluestein FFT length of the exact-ratio propagator for window N (2N).
int czt_len(int N);
int rows_per_det_block(int N);
int rows_per_adj_block(int N);
int rows_per_row_block(int N);
// Row stride of the column adjoint's per-block partial sums (dy, sigma and
// alpha parts are [C][L][stride]).
int adj_part_stride(int N);
// Positions per probe-gradient group that the column-adjoint instance of DFT
// size nl allows for a job with M modes: kRegGroup (the grouped-position
// instance, which sums in registers and whose LDS holds the group's Ohat) at
// N >= 384 where that instance fits, else 4 when an M x N x G accumulator
// fits in LDS, else kRegGroup where that instance fits, else 1.  A job's group is the least over its slots' sizes, and 1
// when some slot does not fit the grouped-position instance at that size (an
// exact-ratio wavelength: that instance is zero-padded only).
constexpr int kRegGroup = 3;
constexpr int kProbeGroup = 4;  // positions of an LDS group
// The [M][N][G] LDS accumulator of a group of kProbeGroup fits next to the
// transform buffer of the column-adjoint instance of DFT size nl.
bool lds_group_fits(int N, int M, int nl);
int probe_group_of(int N, int M, int nl);
// Groups of four only pay when the launch keeps enough blocks to fill the
// GPU (two per CU): a job with fewer than this many (positions / 4 x column
// sets) takes groups of one.
constexpr long long kMinGroupedBlocks = 512;
// Column sets (blocks per position) of the column-adjoint instance of DFT size nl.
int col_sets_adj(int N, int nl);
// Rows of the object-gather tiles of a job: 16, or 8 or 4 when 16-row tiles
// would give fewer than 1024 blocks (small objects: more, shorter blocks).
int obj_tile_rows(int H, int W, int slots);
constexpr int kObjTileW = 64;
// The grouped-position column-adjoint instance exists for (N, nl).
bool pair_capable(int N, int nl);
// Dynamic LDS bytes of the grouped-position column adjoint over pg positions.
size_t col_adj_pair_lds(int N, int nl, int pg);
// That instance exists for (N, nl) and its pg-position LDS fits a workgroup.
bool pair_fits(int N, int nl, int pg);
// Dynamic LDS bytes of the column-adjoint instance of DFT size nl for a job
// with M modes (0 if the job's group is 1).
size_t col_adj_lds_of(int N, int nl, int M, int group);

// Launchers (asynchronous on `s`).  `units` is the total number of work
// units of the launch's segments.
hipError_t launch_write_table(int* dst, const int* data, int n, hipStream_t s);
hipError_t launch_simple(int kind, const Launch& la, long long units, hipStream_t s);
hipError_t launch_loss_total(const Launch& la, long long units, const LossDev& loss, float scale,
                             hipStream_t s);
// Amplitude L1 / TV regulariser: value per pixel block, gradient into g_object.
hipError_t launch_regulariser(const Launch& la, long long units, const LossDev& loss, hipStream_t s);
constexpr int kRegBlock = 256;  // pixels per regulariser block
hipError_t launch_row_fwd(int N, const Launch& la, long long units, hipStream_t s);
hipError_t launch_col_fwd(int N, int nl, const Launch& la, long long units, hipStream_t s);
// mode: 0 fused loss + adjoint, 1 forward (I + B to ibuf or out; `spill`
// keeps Psi of exact-ratio rows for mode 2; zero-padded rows keep Y and the
// adjoint recomputes Psi), 2 adjoint from ibuf (R^T g), 3 loss only.
// var: 0 zero-padded DFTs only; 1 some wavelength uses the exact-ratio
// propagator (LDS rows of length 2N); 2 as 1, and the jobs want dL/d alpha
// (modes 0 and 2: the adjoint recomputes Psi and the alpha-derivative terms)
hipError_t launch_det(int N, const Launch& la, long long units, const LossDev& loss, int mode,
                      bool spill, int var, hipStream_t s);
hipError_t launch_resample_loss(int N, const Launch& la, long long units, const LossDev& loss,
                                bool forward, hipStream_t s);
hipError_t launch_resample_T(int N, const Launch& la, long long units, hipStream_t s);
// grouped: some job of the launch sums its probe-gradient terms over groups
// of positions (else the single-position instance runs); ratio: the jobs want
// dL/d alpha (exact-ratio launches only)
hipError_t launch_col_adj(int N, int nl, const Launch& la, long long units, size_t dyn_lds,
                          bool grouped, bool ratio, hipStream_t s);
// Grouped-position column adjoint (jobs whose probe-gradient group is
// kRegGroup; zero-padded DFT sizes of N >= 256 only, see pair_capable).
hipError_t launch_col_adj_pair(int N, int nl, const Launch& la, long long units, hipStream_t s);
hipError_t launch_row_adj(int N, const Launch& la, long long units, hipStream_t s);

}  // namespace ptycho
