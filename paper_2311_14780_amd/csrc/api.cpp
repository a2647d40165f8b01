// api.cpp - C ABI of the ptychography library (see include/ptycho.h).
//
// Host side only: argument validation, workspace layout, twiddle tables and
// the launch sequence.  Every step of the model, loss and gradient runs in
// the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <vector>

#include "../../include/ptycho.h"
#include "kernels.hpp"

using namespace ptycho;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------ twiddle tables
// The per-pass twiddles of every compiled length live in one static device
// array (each GPU holds its own copy from module load to process end); the
// first call on a device copies the float64-built values into it.  No entry
// point allocates device memory for them.
constexpr size_t kTwCapacity = 16384;  // float2 entries (all lengths need 9728)
__device__ __align__(256) float2 tw_store[kTwCapacity];

struct DeviceTables {
  float2* base = nullptr;  // device address of tw_store on that device
  std::map<int, size_t> offset;  // length -> element offset
};
std::mutex g_mutex;
std::map<int, DeviceTables> g_tables;  // device id -> tables

// Scratch of the allocation-free entry point (ptycho_loss_grad_noalloc): a
// file-scope device array of fixed size.  In host code `scratch` only names
// the symbol; its address on a device comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is passed
// to kernels and copies.
constexpr size_t kScratchBytes = PTYCHO_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::map<int, void*> g_scratch;  // device id -> device address of scratch

const int kLengths[] = {64,  72,  80,  84,  90,  96,  128, 140, 150, 168, 189, 256, 280, 300,
                        315, 336, 343, 375, 384, 420, 480, 512, 560, 600, 675, 750, 768, 1024};

}  // namespace

namespace ptycho {

int init_twiddles() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PTYCHO_EHIP;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_tables.count(dev)) return PTYCHO_OK;
  std::vector<float2> host;
  DeviceTables t;
  for (int n : kLengths) {
    t.offset[n] = host.size();
    int rad[16];
    const int np = plan_radices(n, rad);
    if (np < 1) return PTYCHO_EHIP;
    // per pass p > 0: [k][r - 1] = exp(-2 pi i r k / (Ns R)), k < Ns, 1 <= r < R,
    // evaluated in float64 and rounded to float32
    int Ns = rad[0];
    for (int p = 1; p < np; ++p) {
      const int R = rad[p];
      for (int k = 0; k < Ns; ++k) {
        for (int r = 1; r < R; ++r) {
          const double a = 2.0 * M_PI * static_cast<double>(r * k) / static_cast<double>(Ns * R);
          host.push_back(make_float2(static_cast<float>(std::cos(a)), static_cast<float>(-std::sin(a))));
        }
      }
      Ns *= R;
    }
    while (host.size() % 32) host.push_back(make_float2(0.f, 0.f));
  }
  if (host.size() > kTwCapacity) return PTYCHO_EHIP;
  void* base = nullptr;
  if (hipGetSymbolAddress(&base, HIP_SYMBOL(tw_store)) != hipSuccess || !base) return PTYCHO_EHIP;
  t.base = static_cast<float2*>(base);
  if (hipMemcpy(t.base, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice) !=
      hipSuccess)
    return PTYCHO_EHIP;
  g_tables[dev] = t;
  return PTYCHO_OK;
}

// Device address of the static scratch on the current device (looked up
// once per device), or null on a runtime error.
void* scratch_address() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_mutex);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) return it->second;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
  g_scratch[dev] = ptr;
  return ptr;
}

const float2* twiddles(int n) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_mutex);
  auto it = g_tables.find(dev);
  if (it == g_tables.end()) return nullptr;
  auto o = it->second.offset.find(n);
  if (o == it->second.offset.end()) return nullptr;
  return it->second.base + o->second;
}

void release_twiddles() {
  // the tables are static device arrays: forgetting them makes the next call
  // fill them again
  std::lock_guard<std::mutex> lock(g_mutex);
  g_tables.clear();
}

}  // namespace ptycho

namespace {

// --------------------------------------------------- per-kernel-class timing
// Diagnostics only: when enabled, each launch is bracketed by two HIP events
// recorded on the launch stream; ptycho_profile_read() turns them into
// total milliseconds per kernel class.
enum KernelClass {
  KC_PREP = 0, KC_ROW_FWD, KC_COL_FWD, KC_DET, KC_RESAMPLE, KC_COL_ADJ, KC_PROBE_REDUCE,
  KC_ROW_ADJ, KC_OBJ_GATHER, KC_FINALIZE, KC_FILL, KC_ADAM, KC_TABLES, KC_COUNT
};
const char* const kClassNames[KC_COUNT] = {
    "prep", "row_fwd", "col_fwd", "det", "resample", "col_adj", "probe_reduce",
    "row_adj", "obj_gather", "finalize", "fill", "adam", "tables"};

struct ProfRec {
  int cls;
  hipEvent_t a, b;
};
std::mutex g_prof_mutex;
bool g_prof_on = false;
uint32_t g_prof_mask = ~0u;  // kernel classes bracketed while profiling is on
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;
double g_prof_ms[KC_COUNT];
long long g_prof_n[KC_COUNT];

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Folds finished records into the totals (caller holds the mutex).
int prof_collect() {
  for (auto& r : g_prof_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return PTYCHO_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return PTYCHO_EHIP;
    g_prof_ms[r.cls] += ms;
    g_prof_n[r.cls] += 1;
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  return PTYCHO_OK;
}

struct ProfScope {
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(int c, hipStream_t st, bool allowed) : cls(c), s(st) {
    if (!allowed) return;  // the allocation-free entry point creates no events
    std::lock_guard<std::mutex> lock(g_prof_mutex);
    if (!g_prof_on || !((g_prof_mask >> cls) & 1u)) return;
    a = prof_event();
    if (a && hipEventRecord(a, s) != hipSuccess) a = nullptr;
  }
  ~ProfScope() {
    if (!a) return;
    std::lock_guard<std::mutex> lock(g_prof_mutex);
    hipEvent_t b = prof_event();
    if (b && hipEventRecord(b, s) == hipSuccess) g_prof_recs.push_back({cls, a, b});
    if (g_prof_recs.size() > 8192) (void)prof_collect();
  }
};

}  // namespace

namespace {

bool has_resample(const ptycho_job_t& j) { return j.rs_idx != nullptr; }

// check_ptrs = false: only sizes are validated (workspace queries).
int validate_job(const ptycho_job_t& j, bool need_measured, bool check_ptrs = true) {
  if (j.Ns < 0 || j.Ns > PTYCHO_MAX_SAMPLE_MODES) return PTYCHO_EINVAL;
  if (j.K < 0 || j.L < 1 || j.L > PTYCHO_MAX_WAVELENGTHS || j.M < 1 || j.M > PTYCHO_MAX_MODES ||
      j.N < 1 || j.H < 1 || j.W < 1)
    return PTYCHO_EINVAL;
  if (j.L * std::max(j.Ns, 1) > kMaxL) return PTYCHO_EINVAL;  // slots
  if (j.H < j.N || j.W < j.N) return PTYCHO_ERANGE;
  if (static_cast<long long>(j.H) * j.W >= (1LL << 31)) return PTYCHO_EINVAL;
  bool n_ok = false;
  for (int n : {64, 128, 256, 384, 512}) n_ok |= (j.N == n);
  if (!n_ok) return PTYCHO_EUNSUPPORTED;
  for (int l = 0; l < j.L; ++l) {
    const double a = j.ratio[l];
    if (a != 0.0) {  // exact-ratio propagator
      if (!std::isfinite(a) || a < 0.0) return PTYCHO_EINVAL;
      if (a < j.N) return PTYCHO_ERANGE;
      continue;
    }
    if (j.pad[l] < j.N) return PTYCHO_ERANGE;
    if (!supported(j.N, j.pad[l])) return PTYCHO_EUNSUPPORTED;
  }
  if (check_ptrs) {
    if (!j.object || !j.probe) return PTYCHO_EINVAL;
    if (j.K > 0 && !j.pos) return PTYCHO_EINVAL;
    if (need_measured && j.K > 0 && !j.measured) return PTYCHO_EINVAL;
  }
  const int nrs = (j.rs_idx != nullptr) + (j.rs_w != nullptr) + (j.rsT_ptr != nullptr) +
                  (j.rsT_col != nullptr) + (j.rsT_val != nullptr);
  if (nrs != 0 && nrs != 5) return PTYCHO_EINVAL;
  return PTYCHO_OK;
}

// Sample modes (0 means one) and slots s = l Ns + n (wavelength, sample mode).
int ns_of(const ptycho_job_t& j) { return j.Ns > 1 ? j.Ns : 1; }
int slots_of(const ptycho_job_t& j) { return j.L * ns_of(j); }

bool is_czt(const ptycho_job_t& j, int l) { return j.ratio[l] != 0.0; }

bool any_czt(const ptycho_job_t& j) {
  for (int l = 0; l < j.L; ++l)
    if (is_czt(j, l)) return true;
  return false;
}

// DFT length the kernels run for wavelength l: the pad, or the Bluestein
// length of the exact-ratio propagator.
int eff_pad(const ptycho_job_t& j, int l) { return is_czt(j, l) ? czt_len(j.N) : j.pad[l]; }
int eff_pad_slot(const ptycho_job_t& j, int s) { return eff_pad(j, s / ns_of(j)); }

// Chirp tables of a job's exact-ratio wavelengths (one region per wavelength).
size_t czt_table_bytes(const ptycho_job_t& j) {
  return any_czt(j) ? static_cast<size_t>(j.L) * align_up(4 * static_cast<size_t>(j.N) * sizeof(float2))
                    : 0;
}

// Per-position dL/d alpha_l ([K][L] float64) of a job with exact-ratio wavelengths.
size_t ratio_k_bytes(const ptycho_job_t& j) {
  return any_czt(j) ? align_up(std::max<size_t>(j.K, 1) * j.L * sizeof(double)) : 0;
}

// Regulariser values per pixel block of every slot of the object.
size_t reg_blocks(const ptycho_job_t& j) {
  return (static_cast<size_t>(j.H) * j.W + kRegBlock - 1) / kRegBlock;
}
size_t reg_bytes(const ptycho_job_t& j) {
  return align_up(static_cast<size_t>(slots_of(j)) * reg_blocks(j) * sizeof(float));
}

int n_loss_of(const ptycho_job_t& j) {
  const int plane = j.N * j.N;
  return has_resample(j) ? (plane + 255) / 256 : j.N / rows_per_det_block(j.N);
}

// Bytes of workspace that scale with the number of positions in a chunk.
size_t per_position_bytes(const ptycho_job_t& j, int which) {
  const size_t N = j.N, L = slots_of(j), M = j.M;
  const size_t plane = N * N;
  size_t b = 0;
  b += align_up(2 * N * sizeof(float2));          // ramp
  b += align_up(L * plane * sizeof(float2));      // X
  b += align_up(L * M * plane * sizeof(float2));  // Y
  if (which != 0) {
    b += align_up(L * plane * sizeof(float2));  // GX
    b += align_up(static_cast<size_t>(n_loss_of(j)) * sizeof(float));
    b += 2 * align_up(L * adj_part_stride(j.N) * sizeof(float));  // dy, sigma
    b += align_up(L * (N / rows_per_adj_block(j.N)) * sizeof(float));  // dx
    if (any_czt(j)) {  // alpha-derivative terms
      b += align_up(L * (N / rows_per_det_block(j.N)) * sizeof(float));
      b += align_up(L * adj_part_stride(j.N) * sizeof(float));
    }
  }
  if (has_resample(j)) b += 2 * align_up(plane * sizeof(float));  // ibuf, gbuf
  return b;
}

// Bound on the segments one job adds to one phase.  Phase::add appends at
// most one segment per (job, selector) and launch, so the bound follows from
// the selectors each phase enumerates:
//  - a chunk iteration: 5 per slot (row forward, column forward, column
//    adjoint (the plain or the grouped-position launch, never both), row
//    adjoint, object gather), one per wavelength (probe
//    reduction) and one each for ramps, detector, background sum, finalise;
//  - the prologue: one per gradient output (kVars + distance ratio), status,
//    window check, and one chirp table per wavelength;
//  - the epilogue: one regulariser segment per slot, the loss total and one
//    Adam segment per variable.
// The pool is sized from this bound, so no phase can overflow it and no call
// fails after its first launch has been enqueued.
constexpr int kSegsPerJob = 5 * kMaxL + PTYCHO_MAX_WAVELENGTHS + 4;
static_assert(kSegsPerJob >= (kVars + 1) + 2 + PTYCHO_MAX_WAVELENGTHS, "prologue segments");
static_assert(kSegsPerJob >= kMaxL + 1 + kVars, "epilogue segments");
static_assert(PTYCHO_MAX_WAVELENGTHS <= kMaxL, "one slot per wavelength at least");

size_t fixed_bytes(const ptycho_job_t* jobs, int n_jobs) {
  size_t b = align_up(sizeof(int) * n_jobs);                        // status
  b += align_up(sizeof(JobDev) * n_jobs);                           // job table
  b += align_up(sizeof(Seg) * static_cast<size_t>(kSegsPerJob) * n_jobs);  // segment pool
  for (int i = 0; i < n_jobs; ++i) b += align_up(std::max<size_t>(jobs[i].K, 1) * sizeof(double));
  for (int i = 0; i < n_jobs; ++i)
    b += czt_table_bytes(jobs[i]) + ratio_k_bytes(jobs[i]) + reg_bytes(jobs[i]);
  return b;
}

// Key of a launch group: jobs of one group share every kernel instance.
// `wide` (some wavelength uses the exact-ratio propagator) selects the
// detector-kernel instance, so it is part of the key: a job's instances never
// depend on the other jobs of a call.
// `ratio_grad` (dL/d alpha wanted for exact-ratio wavelengths) selects the
// detector instance that recomputes Psi in the adjoint.
struct GroupKey {
  int N;
  bool resample;
  bool adjoint;
  bool wide;
  bool ratio_grad;
  bool operator<(const GroupKey& o) const {
    return std::tie(N, resample, adjoint, wide, ratio_grad) <
           std::tie(o.N, o.resample, o.adjoint, o.wide, o.ratio_grad);
  }
};

// Host view of one call.
struct Call {
  int which;  // 0 forward, 1 loss + gradient, 2 step
  int n;
  const ptycho_job_t* jobs;
  const ptycho_grads_t* grads;  // [n] or null (forward)
  const ptycho_adam_t* adam;    // [n] or null
  float* const* out;            // [n] or null
  LossDev loss{};
  float scale = 1.f;
  // workspace
  int* status = nullptr;
  JobDev* jobs_dev = nullptr;
  Seg* seg_pool = nullptr;
  std::vector<double*> loss_k;
  std::vector<char*> czt_tab;    // per job, or null
  std::vector<double*> ratio_k;  // per job, or null
  std::vector<float*> reg_part;  // per job
  char* chunk_base = nullptr;
  size_t chunk_bytes = 0;
  std::vector<JobDev> host_jobs;
  std::vector<int> chunk;   // C per job
  std::vector<int> pgroup;  // probe-gradient group size per job
  bool profile = true;      // launches may be bracketed by profiling events
};

// Positions whose probe-gradient terms are summed in one column-adjoint
// block (a function of the job alone, so results do not depend on the
// other jobs of a call).
int job_probe_group(const ptycho_job_t& j, bool want_probe) {
  if (!want_probe) return 1;
  int g = probe_group_of(j.N, j.M, eff_pad(j, 0));
  int sets = col_sets_adj(j.N, eff_pad(j, 0));
  for (int l = 1; l < j.L; ++l) {
    g = std::min(g, probe_group_of(j.N, j.M, eff_pad(j, l)));
    sets = std::min(sets, col_sets_adj(j.N, eff_pad(j, l)));
  }
  // register groups run the grouped-position instance on every wavelength:
  // each must have it and fit it, else the job takes LDS groups where every
  // wavelength fits them (a job with an exact-ratio wavelength)
  if (g == kRegGroup) {
    bool reg = true, lds = true;
    for (int l = 0; l < j.L; ++l) {
      reg = reg && pair_fits(j.N, eff_pad(j, l), kRegGroup);
      lds = lds && lds_group_fits(j.N, j.M, eff_pad(j, l));
    }
    if (!reg) g = lds ? kProbeGroup : 1;
  }
  // small scans: one position per block keeps the column adjoint's launch
  // filled (100 positions at N = 64: 100 -> 400 blocks)
  if (g >= kProbeGroup && static_cast<long long>((j.K + g - 1) / g) * sets < kMinGroupedBlocks) g = 1;
  return g;
}

// Chunk sizes are multiples of the group size (except a chunk holding the
// whole scan), so that groups never straddle chunks.
int round_chunk(int C, int K, int group) {
  if (group <= 1 || C >= K) return std::min(C, std::max(K, 1));
  return std::min(K, (C + group - 1) / group * group);
}

bool wants_adjoint(const Call& c, int i) {
  if (c.which == 0) return false;
  const ptycho_grads_t& g = c.grads[i];
  return g.g_object || g.g_probe || g.g_pos || g.g_sigma || g.g_background || g.g_ratio;
}

// dL/d alpha wanted, and the job has exact-ratio wavelengths
bool wants_ratio(const Call& c, int i) {
  return c.which != 0 && c.grads[i].g_ratio != nullptr && any_czt(c.jobs[i]);
}

// Floats of variable v (0 object, 1 probe, 2 positions, 3 sigma, 4 background).
size_t var_floats(const ptycho_job_t& j, int v) {
  switch (v) {
    case 0: return 2ull * slots_of(j) * j.H * j.W;
    case 1: return 2ull * j.L * j.M * j.N * j.N;
    case 2: return 2ull * j.K;
    case 3: return static_cast<size_t>(j.K);
    default: return static_cast<size_t>(j.N) * j.N;
  }
}

float* grad_of(const ptycho_grads_t& g, int v) {
  float* const p[kVars] = {g.g_object, g.g_probe, g.g_pos, g.g_sigma, g.g_background};
  return p[v];
}

float adam_lr(const ptycho_adam_t& a, int v) {
  const float lr[kVars] = {a.lr_object, a.lr_probe, a.lr_pos, a.lr_sigma, a.lr_background};
  return lr[v];
}

int layout(Call& c, void* ws, size_t ws_bytes) {
  char* p = static_cast<char*>(ws);
  char* end = p + ws_bytes;
  c.status = reinterpret_cast<int*>(p);
  p += align_up(sizeof(int) * c.n);
  c.jobs_dev = reinterpret_cast<JobDev*>(p);
  p += align_up(sizeof(JobDev) * c.n);
  c.seg_pool = reinterpret_cast<Seg*>(p);
  p += align_up(sizeof(Seg) * static_cast<size_t>(kSegsPerJob) * c.n);
  c.loss_k.resize(c.n);
  for (int i = 0; i < c.n; ++i) {
    c.loss_k[i] = reinterpret_cast<double*>(p);
    p += align_up(std::max<size_t>(c.jobs[i].K, 1) * sizeof(double));
  }
  c.czt_tab.assign(c.n, nullptr);
  c.ratio_k.assign(c.n, nullptr);
  c.reg_part.assign(c.n, nullptr);
  for (int i = 0; i < c.n; ++i) {
    const size_t tb = czt_table_bytes(c.jobs[i]);
    if (tb) c.czt_tab[i] = p;
    p += tb;
    const size_t rb = ratio_k_bytes(c.jobs[i]);
    if (rb) c.ratio_k[i] = reinterpret_cast<double*>(p);
    p += rb;
    c.reg_part[i] = reinterpret_cast<float*>(p);
    p += reg_bytes(c.jobs[i]);
  }
  if (p > end) return PTYCHO_ENOSPC;
  c.chunk_base = p;
  c.chunk_bytes = static_cast<size_t>(end - p);
  return PTYCHO_OK;
}

// Chunk sizes of the jobs of one group: the fewest iterations T such that
// the group's per-chunk workspaces fit; C_j = ceil(K_j / T).
int plan_chunks(Call& c, const std::vector<int>& members, int* iters) {
  int kmax = 0;
  for (int i : members) kmax = std::max(kmax, c.jobs[i].K);
  if (kmax == 0) {
    for (int i : members) c.chunk[i] = 1;
    *iters = 0;
    return PTYCHO_OK;
  }
  const int w = c.which == 0 ? 0 : 1;
  auto chunk_of = [&](int i, int T) {
    const int K = c.jobs[i].K;
    return round_chunk((K + T - 1) / T, K, c.pgroup[i]);
  };
  auto need = [&](int T) {
    size_t b = 0;
    for (int i : members) {
      if (c.jobs[i].K == 0) continue;
      b += per_position_bytes(c.jobs[i], w) * static_cast<size_t>(chunk_of(i, T));
    }
    return b;
  };
  if (need(kmax) > c.chunk_bytes) return PTYCHO_ENOSPC;
  int lo = 1, hi = kmax;  // smallest T with need(T) <= chunk_bytes
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (need(mid) <= c.chunk_bytes) hi = mid; else lo = mid + 1;
  }
  int T = lo;
  for (int i : members) c.chunk[i] = c.jobs[i].K == 0 ? 1 : chunk_of(i, T);
  // iterations actually needed with these chunk sizes
  int it = 0;
  for (int i : members) {
    const int K = c.jobs[i].K;
    if (K) it = std::max(it, (K + c.chunk[i] - 1) / c.chunk[i]);
  }
  *iters = it;
  return PTYCHO_OK;
}

// Fill the device view of job i, its workspace starting at *cursor.
void fill_job(Call& c, int i, char** cursor) {
  const ptycho_job_t& j = c.jobs[i];
  JobDev& d = c.host_jobs[i];
  d = JobDev{};
  d.object = reinterpret_cast<const float2*>(j.object);
  d.probe = reinterpret_cast<const float2*>(j.probe);
  d.pos = j.pos;
  d.sigma = j.sigma;
  d.background = j.background;
  d.mask = j.mask;
  d.rs_idx = j.rs_idx;
  d.rs_w = j.rs_w;
  d.rsT_ptr = j.rsT_ptr;
  d.rsT_col = j.rsT_col;
  d.rsT_val = j.rsT_val;
  d.measured = j.measured;
  d.K = j.K;
  d.L = slots_of(j);
  d.Lw = j.L;
  d.Ns = ns_of(j);
  d.M = j.M;
  d.N = j.N;
  d.H = j.H;
  d.W = j.W;
  d.tw_N = twiddles(j.N);
  for (int sl = 0; sl < kMaxL; ++sl) {  // per slot, from its wavelength w
    const bool used = sl < slots_of(j);
    const int w = sl / ns_of(j);
    const int nl = used ? eff_pad(j, w) : j.N;
    d.pad[sl] = nl;
    d.pad_scale[sl] = static_cast<float>(1.0 / std::sqrt(static_cast<double>(nl)));
    d.tw_pad[sl] = twiddles(nl);
    if (used && is_czt(j, w)) {
      d.czt[sl] = reinterpret_cast<float2*>(c.czt_tab[i] + w * align_up(4 * static_cast<size_t>(j.N) *
                                                                         sizeof(float2)));
      d.czt_alpha[sl] = j.ratio[w];
    }
  }
  if (c.grads) {
    const ptycho_grads_t& g = c.grads[i];
    d.loss = g.loss;
    d.g_object = reinterpret_cast<float2*>(g.g_object);
    d.g_probe = reinterpret_cast<float2*>(g.g_probe);
    d.g_pos = g.g_pos;
    d.g_sigma = g.g_sigma;
    d.g_background = g.g_background;
    d.g_ratio = g.g_ratio;
  }
  d.var_flat[0] = j.object;
  d.var_flat[1] = j.probe;
  d.var_flat[2] = j.pos;
  d.var_flat[3] = j.sigma;
  d.var_flat[4] = j.background;
  d.grad_flat[0] = reinterpret_cast<float*>(d.g_object);
  d.grad_flat[1] = reinterpret_cast<float*>(d.g_probe);
  d.grad_flat[2] = d.g_pos;
  d.grad_flat[3] = d.g_sigma;
  d.grad_flat[4] = d.g_background;
  for (int v = 0; v < kVars; ++v) d.flat_n[v] = static_cast<long long>(var_floats(j, v));
  d.grad_flat[kVars] = d.g_ratio;
  d.flat_n[kVars] = j.L;
  d.ratio_k = c.ratio_k[i];
  d.reg_part = c.reg_part[i];
  d.out = c.out ? c.out[i] : nullptr;
  d.status = c.status + i;
  d.loss_k = c.loss_k[i];
  const int C = c.chunk[i];
  const size_t N = j.N, L = slots_of(j), M = j.M, plane = N * N;
  auto take = [&](size_t bytes) {
    char* r = *cursor;
    *cursor += align_up(bytes);
    return r;
  };
  d.ramp = reinterpret_cast<float2*>(take(C * 2 * N * sizeof(float2)));
  d.X = reinterpret_cast<float2*>(take(C * L * plane * sizeof(float2)));
  d.Y = reinterpret_cast<float2*>(take(C * L * M * plane * sizeof(float2)));
  if (c.which != 0) {
    d.GX = reinterpret_cast<float2*>(take(C * L * plane * sizeof(float2)));
    d.loss_part = reinterpret_cast<float*>(take(C * static_cast<size_t>(n_loss_of(j)) * sizeof(float)));
    d.dy_part = reinterpret_cast<float*>(take(C * L * adj_part_stride(j.N) * sizeof(float)));
    d.sg_part = reinterpret_cast<float*>(take(C * L * adj_part_stride(j.N) * sizeof(float)));
    d.dx_part = reinterpret_cast<float*>(take(C * L * (N / rows_per_adj_block(j.N)) * sizeof(float)));
    if (any_czt(j)) {
      d.ra_part = reinterpret_cast<float*>(take(C * L * (N / rows_per_det_block(j.N)) * sizeof(float)));
      d.rb_part = reinterpret_cast<float*>(take(C * L * adj_part_stride(j.N) * sizeof(float)));
    }
  }
  if (has_resample(j)) {
    d.ibuf = reinterpret_cast<float*>(take(C * plane * sizeof(float)));
    d.gbuf = reinterpret_cast<float*>(take(C * plane * sizeof(float)));
  }
  d.C = C;
  d.n_loss = n_loss_of(j);
  d.want_adjoint = wants_adjoint(c, i) ? 1 : 0;
  d.probe_group = c.pgroup[i];
  d.obj_tile_h = obj_tile_rows(j.H, j.W, slots_of(j));
  if (c.adam) {
    const ptycho_adam_t& a = c.adam[i];
    float* const m[kVars] = {a.m_object, a.m_probe, a.m_pos, a.m_sigma, a.m_background};
    float* const v[kVars] = {a.v_object, a.v_probe, a.v_pos, a.v_sigma, a.v_background};
    for (int q = 0; q < kVars; ++q) {
      d.adam_m[q] = m[q];
      d.adam_v[q] = v[q];
      d.adam_lr[q] = adam_lr(a, q);
    }
    d.adam_beta1 = a.beta1;
    d.adam_beta2 = a.beta2;
    d.adam_eps = a.eps;
    d.adam_bc1 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(a.beta1), a.t)));
    d.adam_bc2 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(a.beta2), a.t)));
  }
}

// Segments of the launches of one phase, written to the pool in one go.
struct Phase {
  std::vector<Seg> segs;
  struct Item {
    int first, count;
    long long units;
  };
  Item begin() const { return Item{static_cast<int>(segs.size()), 0, 0}; }
  void add(Item& it, int job, int l, long long units) {
    if (units <= 0) return;
    segs.push_back(Seg{job, l, static_cast<int>(it.units), 0});
    it.count += 1;
    it.units += units;
  }
};

#define CHECK_HIP(x)                           \
  do {                                         \
    if ((x) != hipSuccess) return PTYCHO_EHIP; \
  } while (0)

// A launch, timed per kernel class when profiling is on.
#define LAUNCH(cls, x)                         \
  do {                                         \
    ProfScope prof_scope_(cls, s, c.profile);  \
    if ((x) != hipSuccess) return PTYCHO_EHIP; \
  } while (0)
// A launch over `units` work units: skipped, with its profiling events, when
// there are none (the launchers enqueue nothing then), so that the profile
// counts kernels that ran.
#define LAUNCH_U(cls, units, x)     \
  do {                              \
    if ((units) > 0) LAUNCH(cls, x); \
  } while (0)

int upload_phase(const Call& c, const Phase& ph, hipStream_t s) {
  if (ph.segs.empty()) return PTYCHO_OK;
  // ph.segs.size() <= kSegsPerJob * c.n by construction (see kSegsPerJob)
  LAUNCH(KC_TABLES, launch_write_table(reinterpret_cast<int*>(c.seg_pool),
                                       reinterpret_cast<const int*>(ph.segs.data()),
                                       static_cast<int>(ph.segs.size() * sizeof(Seg) / sizeof(int)), s));
  return PTYCHO_OK;
}

Launch launch_of(const Call& c, const Phase::Item& it, int iter) {
  return Launch{c.jobs_dev, c.seg_pool + it.first, it.count, iter};
}

int run_prologue(Call& c, hipStream_t s) {
  Phase ph;
  auto zero = ph.begin();
  if (c.grads) {
    for (int i = 0; i < c.n; ++i) {
      for (int v = 0; v < kVars; ++v)
        if (grad_of(c.grads[i], v))
          ph.add(zero, i, v, static_cast<long long>((var_floats(c.jobs[i], v) + 1023) / 1024));
      if (c.grads[i].g_ratio) ph.add(zero, i, kVars, 1);
    }
  }
  auto stat = ph.begin();
  for (int i = 0; i < c.n; ++i) ph.add(stat, i, 0, 1);
  auto val = ph.begin();
  for (int i = 0; i < c.n; ++i) ph.add(val, i, 0, (c.jobs[i].K + 255) / 256);
  auto czt = ph.begin();
  for (int i = 0; i < c.n; ++i)
    for (int l = 0; l < c.jobs[i].L; ++l)  // one table per wavelength, at its first slot
      if (is_czt(c.jobs[i], l)) ph.add(czt, i, l * ns_of(c.jobs[i]), czt_table_blocks(c.jobs[i].N));
  int e = upload_phase(c, ph, s);
  if (e) return e;
  LAUNCH_U(KC_FILL, zero.units, launch_simple(KZeroGrads, launch_of(c, zero, 0), zero.units, s));
  LAUNCH_U(KC_PREP, stat.units, launch_simple(KSetStatus, launch_of(c, stat, 0), stat.units, s));
  LAUNCH_U(KC_PREP, val.units, launch_simple(KValidate, launch_of(c, val, 0), val.units, s));
  LAUNCH_U(KC_PREP, czt.units, launch_simple(KCztTables, launch_of(c, czt, 0), czt.units, s));
  return PTYCHO_OK;
}

// One chunk iteration of a group of jobs that share N, resampling and adjoint.
int run_iteration(Call& c, const GroupKey& key, const std::vector<int>& members, int iter,
                  hipStream_t s) {
  // positions of each member in this iteration
  std::vector<int> cnt(members.size());
  for (size_t q = 0; q < members.size(); ++q) {
    const ptycho_job_t& j = c.jobs[members[q]];
    const int k0 = iter * c.chunk[members[q]];
    cnt[q] = std::max(0, std::min(c.chunk[members[q]], j.K - k0));
  }
  const int N = key.N;
  const size_t plane = static_cast<size_t>(N) * N;
  Phase ph;
  auto prep = ph.begin();
  for (size_t q = 0; q < members.size(); ++q) ph.add(prep, members[q], 0, cnt[q]);
  auto rowf = ph.begin();
  for (size_t q = 0; q < members.size(); ++q)
    for (int l = 0; l < slots_of(c.jobs[members[q]]); ++l) ph.add(rowf, members[q], l, cnt[q]);
  // distinct DFT sizes of the group, in first-seen order
  std::vector<int> nls;
  const int var = key.ratio_grad ? 2 : (key.wide ? 1 : 0);
  for (int i : members) {
    for (int l = 0; l < c.jobs[i].L; ++l)
      if (std::find(nls.begin(), nls.end(), eff_pad(c.jobs[i], l)) == nls.end())
        nls.push_back(eff_pad(c.jobs[i], l));
  }
  // work units below run over slots (wavelength x sample mode)
  std::vector<Phase::Item> colf(nls.size()), cola(nls.size()), colp(nls.size());
  for (size_t p = 0; p < nls.size(); ++p) {
    colf[p] = ph.begin();
    for (size_t q = 0; q < members.size(); ++q)
      for (int l = 0; l < slots_of(c.jobs[members[q]]); ++l)
        if (eff_pad_slot(c.jobs[members[q]], l) == nls[p]) ph.add(colf[p], members[q], l, cnt[q]);
  }
  auto det = ph.begin();
  for (size_t q = 0; q < members.size(); ++q) ph.add(det, members[q], 0, cnt[q]);
  Phase::Item prob = ph.begin(), rowa = ph.begin(), obj = ph.begin();
  if (key.adjoint) {
    // jobs with register groups run the grouped-position instance (its own
    // launch)
    for (size_t p = 0; p < nls.size(); ++p) {
      for (int pass = 0; pass < 2; ++pass) {
        Phase::Item& it = pass == 0 ? cola[p] : colp[p];
        it = ph.begin();
        for (size_t q = 0; q < members.size(); ++q) {
          const int pg = c.pgroup[members[q]];
          if ((pg == kRegGroup) != (pass == 1)) continue;
          for (int l = 0; l < slots_of(c.jobs[members[q]]); ++l)
            if (eff_pad_slot(c.jobs[members[q]], l) == nls[p])
              ph.add(it, members[q], l, (cnt[q] + pg - 1) / pg);
        }
      }
    }
    prob = ph.begin();
    const long long nblk = static_cast<long long>((plane + 255) / 256);
    for (size_t q = 0; q < members.size(); ++q) {
      if (!cnt[q] || !c.grads[members[q]].g_probe) continue;
      for (int l = 0; l < c.jobs[members[q]].L; ++l) ph.add(prob, members[q], l, c.jobs[members[q]].M * nblk);
    }
    rowa = ph.begin();
    for (size_t q = 0; q < members.size(); ++q) {
      const ptycho_grads_t& g = c.grads[members[q]];
      if (!(g.g_object || g.g_pos)) continue;
      for (int l = 0; l < slots_of(c.jobs[members[q]]); ++l) ph.add(rowa, members[q], l, cnt[q]);
    }
    obj = ph.begin();
    for (size_t q = 0; q < members.size(); ++q) {
      const ptycho_job_t& j = c.jobs[members[q]];
      if (!cnt[q] || !c.grads[members[q]].g_object) continue;
      const int th = obj_tile_rows(j.H, j.W, slots_of(j));
      const long long tiles = static_cast<long long>((j.W + kObjTileW - 1) / kObjTileW) *
                              ((j.H + th - 1) / th);
      for (int l = 0; l < slots_of(j); ++l) ph.add(obj, members[q], l, tiles);
    }
  }
  auto bgr = ph.begin();
  if (key.adjoint) {
    const long long nblk = static_cast<long long>((plane + 255) / 256);
    for (size_t q = 0; q < members.size(); ++q)
      if (cnt[q] && c.grads[members[q]].g_background) ph.add(bgr, members[q], 0, nblk);
  }
  auto fin = ph.begin();
  if (c.which != 0)
    for (size_t q = 0; q < members.size(); ++q) ph.add(fin, members[q], 0, (cnt[q] + 63) / 64);
  int e = upload_phase(c, ph, s);
  if (e) return e;

  LAUNCH_U(KC_PREP, prep.units, launch_simple(KPrep, launch_of(c, prep, iter), prep.units, s));
  LAUNCH_U(KC_ROW_FWD, rowf.units, launch_row_fwd(N, launch_of(c, rowf, iter), rowf.units, s));
  for (size_t p = 0; p < nls.size(); ++p)
    LAUNCH_U(KC_COL_FWD, colf[p].units,
             launch_col_fwd(N, nls[p], launch_of(c, colf[p], iter), colf[p].units, s));
  const Launch ldet = launch_of(c, det, iter);
  if (c.which == 0) {
    LAUNCH_U(KC_DET, det.units, launch_det(N, ldet, det.units, c.loss, 1, false, var, s));
    if (key.resample)
      LAUNCH_U(KC_RESAMPLE, det.units, launch_resample_loss(N, ldet, det.units, c.loss, true, s));
    return PTYCHO_OK;
  }
  if (!key.resample) {
    LAUNCH_U(KC_DET, det.units,
             launch_det(N, ldet, det.units, c.loss, key.adjoint ? 0 : 3, false, var, s));
  } else {
    LAUNCH_U(KC_DET, det.units, launch_det(N, ldet, det.units, c.loss, 1, key.adjoint, var, s));
    LAUNCH_U(KC_RESAMPLE, det.units, launch_resample_loss(N, ldet, det.units, c.loss, false, s));
    if (key.adjoint) {
      LAUNCH_U(KC_RESAMPLE, det.units, launch_resample_T(N, ldet, det.units, s));
      LAUNCH_U(KC_DET, det.units, launch_det(N, ldet, det.units, c.loss, 2, false, var, s));
    }
  }
  if (key.adjoint) {
    // background gradient: before the column adjoint reuses GX
    LAUNCH_U(KC_FINALIZE, bgr.units, launch_simple(KBgReduce, launch_of(c, bgr, iter), bgr.units, s));
    for (size_t p = 0; p < nls.size(); ++p) {
      size_t lds = 0;  // the launch's largest probe-gradient accumulator
      bool grouped = false;
      for (size_t q = 0; q < members.size(); ++q) {
        const ptycho_job_t& j = c.jobs[members[q]];
        bool uses = false;
        for (int l = 0; l < j.L; ++l) uses |= eff_pad(j, l) == nls[p];
        if (!uses || !cnt[q]) continue;
        if (c.pgroup[members[q]] == kRegGroup) continue;  // grouped-position launch below
        grouped |= c.pgroup[members[q]] > 1;
        lds = std::max(lds, col_adj_lds_of(N, nls[p], j.M, c.pgroup[members[q]]));
      }
      LAUNCH_U(KC_COL_ADJ, cola[p].units,
               launch_col_adj(N, nls[p], launch_of(c, cola[p], iter), cola[p].units, lds,
                              grouped, key.ratio_grad, s));
      LAUNCH_U(KC_COL_ADJ, colp[p].units,
               launch_col_adj_pair(N, nls[p], launch_of(c, colp[p], iter), colp[p].units, s));
    }
    LAUNCH_U(KC_PROBE_REDUCE, prob.units,
             launch_simple(KProbeReduce, launch_of(c, prob, iter), prob.units, s));
    LAUNCH_U(KC_ROW_ADJ, rowa.units, launch_row_adj(N, launch_of(c, rowa, iter), rowa.units, s));
    LAUNCH_U(KC_OBJ_GATHER, obj.units, launch_simple(KObjGather, launch_of(c, obj, iter), obj.units, s));
  }
  LAUNCH_U(KC_FINALIZE, fin.units, launch_simple(KFinalize, launch_of(c, fin, iter), fin.units, s));
  return PTYCHO_OK;
}

int run_epilogue(Call& c, hipStream_t s) {
  if (c.which == 0) return PTYCHO_OK;
  Phase ph;
  auto reg = ph.begin();
  if (c.loss.l1 != 0.f || c.loss.tv != 0.f)
    for (int i = 0; i < c.n; ++i)
      if (c.grads[i].loss || c.grads[i].g_object)
        for (int sl = 0; sl < slots_of(c.jobs[i]); ++sl)
          ph.add(reg, i, sl, static_cast<long long>(reg_blocks(c.jobs[i])));
  auto tot = ph.begin();
  for (int i = 0; i < c.n; ++i)
    if (c.grads[i].loss || c.grads[i].g_ratio) ph.add(tot, i, 0, 1);
  auto ad = ph.begin();
  if (c.adam) {
    for (int i = 0; i < c.n; ++i)
      for (int v = 0; v < kVars; ++v)
        if (adam_lr(c.adam[i], v) != 0.f)
          ph.add(ad, i, v, static_cast<long long>((var_floats(c.jobs[i], v) + 1023) / 1024));
  }
  int e = upload_phase(c, ph, s);
  if (e) return e;
  LAUNCH_U(KC_FINALIZE, reg.units, launch_regulariser(launch_of(c, reg, 0), reg.units, c.loss, s));
  LAUNCH_U(KC_FINALIZE, tot.units, launch_loss_total(launch_of(c, tot, 0), tot.units, c.loss, c.scale, s));
  LAUNCH_U(KC_ADAM, ad.units, launch_simple(KAdam, launch_of(c, ad, 0), ad.units, s));
  return PTYCHO_OK;
}

int run_call(Call& c, void* ws, size_t ws_bytes, hipStream_t s) {
  int e = layout(c, ws, ws_bytes);
  if (e) return e;
  // groups of jobs sharing every kernel instance
  std::map<GroupKey, std::vector<int>> groups;
  for (int i = 0; i < c.n; ++i)
    groups[GroupKey{c.jobs[i].N, has_resample(c.jobs[i]), wants_adjoint(c, i), any_czt(c.jobs[i]),
                    wants_ratio(c, i)}]
        .push_back(i);
  c.chunk.assign(c.n, 1);
  c.pgroup.assign(c.n, 1);
  for (int i = 0; i < c.n; ++i)
    c.pgroup[i] = job_probe_group(c.jobs[i], wants_adjoint(c, i) && c.grads[i].g_probe != nullptr);
  std::map<GroupKey, int> iters;
  for (auto& kv : groups) {
    int it = 0;
    e = plan_chunks(c, kv.second, &it);
    if (e) return e;
    iters[kv.first] = it;
  }
  // job table: every group reuses the same chunk region (groups run in turn)
  c.host_jobs.assign(c.n, JobDev{});
  for (auto& kv : groups) {
    char* cursor = c.chunk_base;
    for (int i : kv.second) fill_job(c, i, &cursor);
  }
  LAUNCH(KC_TABLES, launch_write_table(reinterpret_cast<int*>(c.jobs_dev),
                                       reinterpret_cast<const int*>(c.host_jobs.data()),
                                       static_cast<int>(c.n * sizeof(JobDev) / sizeof(int)), s));
  e = run_prologue(c, s);
  if (e) return e;
  for (auto& kv : groups)
    for (int it = 0; it < iters[kv.first]; ++it) {
      e = run_iteration(c, kv.first, kv.second, it, s);
      if (e) return e;
    }
  return run_epilogue(c, s);
}

bool finite_nonneg(float x) { return std::isfinite(x) && x >= 0.f; }

int check_loss(const ptycho_loss_t& l) {
  if (l.kind < 0 || l.kind > PTYCHO_LOSS_MIXED || !(l.eps >= 0.f) || !std::isfinite(l.scale))
    return PTYCHO_EINVAL;
  if (l.kind == PTYCHO_LOSS_MIXED && !(std::isfinite(l.noise_var) && l.noise_var > 0.f))
    return PTYCHO_EINVAL;
  if (!finite_nonneg(l.l1) || !finite_nonneg(l.tv)) return PTYCHO_EINVAL;
  if (l.tv > 0.f && !(std::isfinite(l.tv_eps) && l.tv_eps > 0.f)) return PTYCHO_EINVAL;
  return PTYCHO_OK;
}

// Argument checks shared by the entry points (host only, nothing touches
// the device); each entry point calls init_twiddles() after all its checks.
int common_checks(const ptycho_job_t* jobs, int n_jobs, bool need_measured) {
  if (!jobs || n_jobs < 1) return PTYCHO_EINVAL;
  for (int i = 0; i < n_jobs; ++i) {
    const int e = validate_job(jobs[i], need_measured);
    if (e) return e;
  }
  return PTYCHO_OK;
}

}  // namespace

extern "C" {

int32_t ptycho_supported(int32_t N, int32_t pad) { return supported(N, pad) ? 1 : 0; }

int32_t ptycho_workspace_bytes(const ptycho_job_t* jobs, int32_t n_jobs, int32_t which,
                               int32_t chunk, size_t* bytes) {
  if (!bytes || !jobs || n_jobs < 1 || which < 0 || which > 2) return PTYCHO_EINVAL;
  for (int i = 0; i < n_jobs; ++i) {
    const int e = validate_job(jobs[i], false, false);
    if (e) return e;
  }
  // chunk region: the largest group needs its jobs' chunks side by side
  std::map<std::tuple<int, bool, bool>, size_t> group_bytes;
  for (int i = 0; i < n_jobs; ++i) {
    const int K = jobs[i].K;
    int c = chunk <= 0 ? std::max(K, 1) : std::max(1, std::min<int>(chunk, std::max(K, 1)));
    // a loss + gradient call may group positions for the probe gradient
    if (which != 0) c = std::max(1, round_chunk(c, K, job_probe_group(jobs[i], true)));
    group_bytes[std::make_tuple(jobs[i].N, has_resample(jobs[i]), any_czt(jobs[i]))] +=
        per_position_bytes(jobs[i], which == 0 ? 0 : 1) * static_cast<size_t>(c);
  }
  size_t worst = 0;
  for (auto& kv : group_bytes) worst = std::max(worst, kv.second);
  *bytes = fixed_bytes(jobs, n_jobs) + worst;
  return PTYCHO_OK;
}

int32_t ptycho_forward(const ptycho_job_t* jobs, int32_t n_jobs, float* const* intensity,
                       void* workspace, size_t workspace_bytes, void* stream) {
  int e = common_checks(jobs, n_jobs, false);
  if (e) return e;
  if (!intensity || !workspace) return PTYCHO_EINVAL;
  for (int i = 0; i < n_jobs; ++i)
    if (jobs[i].K > 0 && !intensity[i]) return PTYCHO_EINVAL;
  e = init_twiddles();
  if (e) return e;
  Call c;
  c.which = 0;
  c.n = n_jobs;
  c.jobs = jobs;
  c.grads = nullptr;
  c.adam = nullptr;
  c.out = intensity;
  c.loss = LossDev{0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  return run_call(c, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int32_t ptycho_loss_grad(const ptycho_job_t* jobs, int32_t n_jobs, const ptycho_loss_t* loss,
                         const ptycho_grads_t* grads, void* workspace, size_t workspace_bytes,
                         void* stream) {
  int e = common_checks(jobs, n_jobs, true);
  if (e) return e;
  if (!loss || !grads || !workspace) return PTYCHO_EINVAL;
  e = check_loss(*loss);
  if (e) return e;
  e = init_twiddles();
  if (e) return e;
  Call c;
  c.which = 1;
  c.n = n_jobs;
  c.jobs = jobs;
  c.grads = grads;
  c.adam = nullptr;
  c.out = nullptr;
  c.loss = LossDev{loss->kind, loss->eps, 2.0f * loss->scale, loss->noise_var,
                   loss->l1, loss->tv, loss->tv_eps};
  c.scale = loss->scale;
  return run_call(c, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int32_t ptycho_loss_grad_noalloc(const ptycho_job_t* jobs, int32_t n_jobs,
                                 const ptycho_loss_t* loss, const ptycho_grads_t* grads,
                                 void* stream) {
  int e = common_checks(jobs, n_jobs, true);
  if (e) return e;
  if (!loss || !grads) return PTYCHO_EINVAL;
  e = check_loss(*loss);
  if (e) return e;
  // the smallest workspace these jobs can run in (one position per chunk)
  size_t need = 0;
  e = ptycho_workspace_bytes(jobs, n_jobs, 1, 1, &need);
  if (e) return e;
  if (need > kScratchBytes) return PTYCHO_ENOSPC;
  e = init_twiddles();
  if (e) return e;
  void* ws = scratch_address();
  if (!ws) return PTYCHO_EHIP;
  Call c;
  c.which = 1;
  c.n = n_jobs;
  c.jobs = jobs;
  c.grads = grads;
  c.adam = nullptr;
  c.out = nullptr;
  c.loss = LossDev{loss->kind, loss->eps, 2.0f * loss->scale, loss->noise_var,
                   loss->l1, loss->tv, loss->tv_eps};
  c.scale = loss->scale;
  c.profile = false;
  return run_call(c, ws, kScratchBytes, static_cast<hipStream_t>(stream));
}

int32_t ptycho_step(const ptycho_job_t* jobs, int32_t n_jobs, const ptycho_loss_t* loss,
                    const ptycho_grads_t* grads, const ptycho_adam_t* adam, void* workspace,
                    size_t workspace_bytes, void* stream) {
  int e = common_checks(jobs, n_jobs, true);
  if (e) return e;
  if (!loss || !grads || !adam || !workspace) return PTYCHO_EINVAL;
  e = check_loss(*loss);
  if (e) return e;
  for (int i = 0; i < n_jobs; ++i) {
    const ptycho_adam_t& a = adam[i];
    if (a.t < 1 || !(a.beta1 >= 0.f && a.beta1 < 1.f) || !(a.beta2 >= 0.f && a.beta2 < 1.f))
      return PTYCHO_EINVAL;
    if (a.lr_object != 0.f && (!a.m_object || !a.v_object || !grads[i].g_object)) return PTYCHO_EINVAL;
    if (a.lr_probe != 0.f && (!a.m_probe || !a.v_probe || !grads[i].g_probe)) return PTYCHO_EINVAL;
    if (a.lr_pos != 0.f && (!a.m_pos || !a.v_pos || !grads[i].g_pos)) return PTYCHO_EINVAL;
    if (a.lr_sigma != 0.f && (!a.m_sigma || !a.v_sigma || !grads[i].g_sigma || !jobs[i].sigma))
      return PTYCHO_EINVAL;
    if (a.lr_background != 0.f &&
        (!a.m_background || !a.v_background || !grads[i].g_background || !jobs[i].background))
      return PTYCHO_EINVAL;
  }
  e = init_twiddles();
  if (e) return e;
  Call c;
  c.which = 2;
  c.n = n_jobs;
  c.jobs = jobs;
  c.grads = grads;
  c.adam = adam;
  c.out = nullptr;
  c.loss = LossDev{loss->kind, loss->eps, 2.0f * loss->scale, loss->noise_var,
                   loss->l1, loss->tv, loss->tv_eps};
  c.scale = loss->scale;
  return run_call(c, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int32_t ptycho_status(const void* workspace, int32_t job, void* stream) {
  if (!workspace || job < 0) return PTYCHO_EINVAL;
  int v = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return PTYCHO_EHIP;
  if (hipMemcpy(&v, static_cast<const int*>(workspace) + job, sizeof(int), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return PTYCHO_EHIP;
  return v;
}

int32_t ptycho_transpose_table(const int32_t* idx, const float* w, int32_t n_out, int32_t n_in,
                               int32_t* ptr, int32_t* col, float* val) {
  if (!idx || !w || !ptr || !col || !val || n_out < 0 || n_in < 0) return PTYCHO_EINVAL;
  std::vector<int32_t> count(static_cast<size_t>(n_in) + 1, 0);
  for (int64_t a = 0; a < static_cast<int64_t>(n_out) * 4; ++a) {
    if (w[a] == 0.f) continue;
    if (idx[a] < 0 || idx[a] >= n_in) return PTYCHO_ERANGE;
    ++count[idx[a] + 1];
  }
  for (int32_t i = 0; i < n_in; ++i) count[i + 1] += count[i];
  std::memcpy(ptr, count.data(), sizeof(int32_t) * (static_cast<size_t>(n_in) + 1));
  std::vector<int32_t> fill(count.begin(), count.end() - 1);
  // camera pixels in ascending order within each row: fixed summation order
  for (int64_t a = 0; a < n_out; ++a) {
    for (int t = 0; t < 4; ++t) {
      const int64_t q = a * 4 + t;
      if (w[q] == 0.f) continue;
      const int32_t r = idx[q];
      col[fill[r]] = static_cast<int32_t>(a);
      val[fill[r]] = w[q];
      ++fill[r];
    }
  }
  for (int64_t q = count[n_in]; q < static_cast<int64_t>(n_out) * 4; ++q) {
    col[q] = 0;
    val[q] = 0.f;
  }
  return PTYCHO_OK;
}

const char* ptycho_error_string(int32_t code) {
  switch (code) {
    case PTYCHO_OK: return "ok";
    case PTYCHO_EINVAL: return "invalid argument (null pointer or inconsistent size)";
    case PTYCHO_ERANGE: return "out of range (probe window outside the object, or pad < N)";
    case PTYCHO_EUNSUPPORTED: return "unsupported window or DFT size";
    case PTYCHO_ENOSPC: return "workspace too small";
    case PTYCHO_EHIP: return "HIP runtime or launch error";
    default: return "unknown error";
  }
}

void ptycho_release(void) {
  release_twiddles();
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  (void)prof_collect();
  for (hipEvent_t e : g_prof_pool) (void)hipEventDestroy(e);
  g_prof_pool.clear();
}

int32_t ptycho_profile(int32_t enable) {
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  if (prof_collect() != PTYCHO_OK) return PTYCHO_EHIP;
  if (enable) {
    for (int i = 0; i < KC_COUNT; ++i) {
      g_prof_ms[i] = 0.0;
      g_prof_n[i] = 0;
    }
  }
  g_prof_on = enable != 0;
  if (!g_prof_on) g_prof_mask = ~0u;
  return PTYCHO_OK;
}

int32_t ptycho_profile_classes(uint32_t class_mask) {
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  g_prof_mask = class_mask;
  return PTYCHO_OK;
}

int32_t ptycho_profile_read(int32_t kernel_class, double* total_ms, int64_t* launches) {
  if (kernel_class < 0 || kernel_class >= KC_COUNT || !total_ms || !launches) return PTYCHO_EINVAL;
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  if (prof_collect() != PTYCHO_OK) return PTYCHO_EHIP;
  *total_ms = g_prof_ms[kernel_class];
  *launches = g_prof_n[kernel_class];
  return PTYCHO_OK;
}

const char* ptycho_kernel_class_name(int32_t kernel_class) {
  if (kernel_class < 0 || kernel_class >= KC_COUNT) return nullptr;
  return kClassNames[kernel_class];
}

}  // extern "C"
