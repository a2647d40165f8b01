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
#include <mutex>
#include <vector>

#include "../../include/ptycho.h"
#include "kernels.hpp"

using namespace ptycho;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------ twiddle tables
struct DeviceTables {
  float2* base = nullptr;
  std::map<int, size_t> offset;  // length -> element offset
};
std::mutex g_mutex;
std::map<int, DeviceTables> g_tables;  // device id -> tables

const int kLengths[] = {64,  72,  80,  84,  90,  96,  128, 140, 150, 168, 189, 256, 280,
                        300, 315, 336, 343, 375, 384, 420, 480, 512, 560, 600, 675, 750};

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
  if (hipMalloc(&t.base, host.size() * sizeof(float2)) != hipSuccess) return PTYCHO_EHIP;
  if (hipMemcpy(t.base, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice) !=
      hipSuccess) {
    (void)hipFree(t.base);
    return PTYCHO_EHIP;
  }
  g_tables[dev] = t;
  return PTYCHO_OK;
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
  std::lock_guard<std::mutex> lock(g_mutex);
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  for (auto& kv : g_tables) {
    if (hipSetDevice(kv.first) == hipSuccess) (void)hipFree(kv.second.base);
  }
  g_tables.clear();
  if (have) (void)hipSetDevice(cur);
}

}  // namespace ptycho

namespace {

// --------------------------------------------------- per-kernel-class timing
// Diagnostics only: when enabled, each launch is bracketed by two HIP events
// recorded on the launch stream; ptycho_profile_read() turns them into
// total milliseconds per kernel class.
enum KernelClass {
  KC_PREP = 0, KC_ROW_FWD, KC_COL_FWD, KC_DET, KC_RESAMPLE, KC_COL_ADJ, KC_PROBE_REDUCE,
  KC_ROW_ADJ, KC_OBJ_GATHER, KC_FINALIZE, KC_FILL, KC_ADAM, KC_COUNT
};
const char* const kClassNames[KC_COUNT] = {
    "prep", "row_fwd", "col_fwd", "det", "resample", "col_adj", "probe_reduce",
    "row_adj", "obj_gather", "finalize", "fill", "adam"};

struct ProfRec {
  int cls;
  hipEvent_t a, b;
};
std::mutex g_prof_mutex;
bool g_prof_on = false;
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
  ProfScope(int c, hipStream_t st) : cls(c), s(st) {
    std::lock_guard<std::mutex> lock(g_prof_mutex);
    if (!g_prof_on) return;
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

int validate_job(const ptycho_job_t& j, bool need_measured) {
  if (j.K < 0 || j.L < 1 || j.L > PTYCHO_MAX_WAVELENGTHS || j.M < 1 || j.M > PTYCHO_MAX_MODES ||
      j.N < 1 || j.H < 1 || j.W < 1)
    return PTYCHO_EINVAL;
  if (j.H < j.N || j.W < j.N) return PTYCHO_ERANGE;
  if (static_cast<long long>(j.H) * j.W >= (1LL << 31)) return PTYCHO_EINVAL;
  bool n_ok = false;
  for (int n : {64, 128, 256, 384, 512}) n_ok |= (j.N == n);
  if (!n_ok) return PTYCHO_EUNSUPPORTED;
  for (int l = 0; l < j.L; ++l) {
    if (j.pad[l] < j.N) return PTYCHO_ERANGE;
    if (!supported(j.N, j.pad[l])) return PTYCHO_EUNSUPPORTED;
  }
  if (!j.object || !j.probe) return PTYCHO_EINVAL;
  if (j.K > 0 && !j.pos) return PTYCHO_EINVAL;
  if (need_measured && j.K > 0 && !j.measured) return PTYCHO_EINVAL;
  const int nrs = (j.rs_idx != nullptr) + (j.rs_w != nullptr) + (j.rsT_ptr != nullptr) +
                  (j.rsT_col != nullptr) + (j.rsT_val != nullptr);
  if (nrs != 0 && nrs != 5) return PTYCHO_EINVAL;
  return PTYCHO_OK;
}

// Bytes of workspace that scale with the number of positions in a chunk.
size_t per_position_bytes(const ptycho_job_t& j, int which) {
  const size_t N = j.N, L = j.L, M = j.M;
  const size_t plane = N * N;
  size_t b = 0;
  b += align_up(2 * N * sizeof(float2));      // ramp
  b += align_up(L * plane * sizeof(float2));  // X
  b += align_up(L * M * plane * sizeof(float2));  // Y
  if (which != 0) {
    b += align_up(L * plane * sizeof(float2));  // GX
    const size_t nloss = std::max<size_t>(N / rows_per_det_block(j.N), (plane + 255) / 256);
    b += align_up(nloss * sizeof(float));
    b += 2 * align_up(L * (N / col_group_of(j.N)) * sizeof(float));  // dy, sigma
    b += align_up(L * (N / rows_per_adj_block(j.N)) * sizeof(float));  // dx
  }
  if (has_resample(j)) b += 2 * align_up(plane * sizeof(float));  // ibuf, gbuf
  return b;
}

size_t fixed_bytes(const ptycho_job_t* jobs, int n_jobs) {
  size_t kmax = 0;
  for (int i = 0; i < n_jobs; ++i) kmax = std::max<size_t>(kmax, jobs[i].K);
  return align_up(sizeof(int) * n_jobs) + align_up(std::max<size_t>(kmax, 1) * sizeof(double));
}

struct Layout {
  int* status;
  double* loss_k;
  char* chunk_base;
  size_t chunk_bytes;
};

Layout make_layout(void* ws, size_t ws_bytes, const ptycho_job_t* jobs, int n_jobs) {
  Layout lay;
  char* p = static_cast<char*>(ws);
  lay.status = reinterpret_cast<int*>(p);
  p += align_up(sizeof(int) * n_jobs);
  size_t kmax = 0;
  for (int i = 0; i < n_jobs; ++i) kmax = std::max<size_t>(kmax, jobs[i].K);
  lay.loss_k = reinterpret_cast<double*>(p);
  p += align_up(std::max<size_t>(kmax, 1) * sizeof(double));
  lay.chunk_base = p;
  const size_t used = static_cast<size_t>(p - static_cast<char*>(ws));
  lay.chunk_bytes = ws_bytes > used ? ws_bytes - used : 0;
  return lay;
}

Work chunk_views(const ptycho_job_t& j, int which, char* base, int C) {
  const size_t N = j.N, L = j.L, M = j.M, plane = N * N;
  Work w{};
  char* p = base;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += align_up(bytes);
    return r;
  };
  w.ramp = reinterpret_cast<float2*>(take(C * 2 * N * sizeof(float2)));
  w.X = reinterpret_cast<float2*>(take(C * L * plane * sizeof(float2)));
  w.Y = reinterpret_cast<float2*>(take(C * L * M * plane * sizeof(float2)));
  if (which != 0) {
    w.GX = reinterpret_cast<float2*>(take(C * L * plane * sizeof(float2)));
    const size_t nloss = std::max<size_t>(N / rows_per_det_block(j.N), (plane + 255) / 256);
    w.loss_part = reinterpret_cast<float*>(take(C * nloss * sizeof(float)));
    w.dy_part = reinterpret_cast<float*>(take(C * L * (N / col_group_of(j.N)) * sizeof(float)));
    w.sg_part = reinterpret_cast<float*>(take(C * L * (N / col_group_of(j.N)) * sizeof(float)));
    w.dx_part = reinterpret_cast<float*>(take(C * L * (N / rows_per_adj_block(j.N)) * sizeof(float)));
  }
  if (has_resample(j)) {
    w.ibuf = reinterpret_cast<float*>(take(C * plane * sizeof(float)));
    w.gbuf = reinterpret_cast<float*>(take(C * plane * sizeof(float)));
  }
  w.C = C;
  return w;
}

JobDev to_dev(const ptycho_job_t& j) {
  JobDev d{};
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
  d.L = j.L;
  d.M = j.M;
  d.N = j.N;
  d.H = j.H;
  d.W = j.W;
  d.tw_N = twiddles(j.N);
  for (int l = 0; l < kMaxL; ++l) {
    const int nl = l < j.L ? j.pad[l] : j.N;
    d.pad[l] = nl;
    d.pad_scale[l] = static_cast<float>(1.0 / std::sqrt(static_cast<double>(nl)));
    d.tw_pad[l] = twiddles(nl);
  }
  return d;
}

#define CHECK_HIP(x)                       \
  do {                                     \
    if ((x) != hipSuccess) return PTYCHO_EHIP; \
  } while (0)

// A launch, timed per kernel class when profiling is on.
#define LAUNCH(cls, x)                         \
  do {                                         \
    ProfScope prof_scope_(cls, s);             \
    if ((x) != hipSuccess) return PTYCHO_EHIP; \
  } while (0)

int common_checks(const ptycho_job_t* jobs, int n_jobs, bool need_measured) {
  if (!jobs || n_jobs < 1) return PTYCHO_EINVAL;
  for (int i = 0; i < n_jobs; ++i) {
    const int e = validate_job(jobs[i], need_measured);
    if (e) return e;
  }
  return init_twiddles();
}

int chunk_for(const ptycho_job_t& j, int which, size_t avail) {
  if (j.K == 0) return 0;
  const size_t per = per_position_bytes(j, which);
  const size_t c = avail / per;
  return static_cast<int>(std::min<size_t>(c, j.K));
}

// Runs the loss + gradient sequence for one job.
int run_loss_grad(const ptycho_job_t& job, const ptycho_loss_t& lp, const ptycho_grads_t& g,
                  int* status, double* loss_k, char* chunk_base, int C, hipStream_t s) {
  JobDev jb = to_dev(job);
  const size_t plane = static_cast<size_t>(job.N) * job.N;
  if (g.g_object) LAUNCH(KC_FILL, launch_fill_zero(g.g_object, 2ull * job.L * job.H * job.W, s));
  if (g.g_probe) LAUNCH(KC_FILL, launch_fill_zero(g.g_probe, 2ull * job.L * job.M * plane, s));
  if (g.g_pos) LAUNCH(KC_FILL, launch_fill_zero(g.g_pos, 2ull * job.K, s));
  if (g.g_sigma) LAUNCH(KC_FILL, launch_fill_zero(g.g_sigma, job.K, s));
  LAUNCH(KC_PREP, launch_set_status(status, s));
  LAUNCH(KC_PREP, launch_validate(jb, status, s));
  const bool want_grad = g.g_object || g.g_probe || g.g_pos || g.g_sigma;
  LossDev ld{lp.kind, lp.eps, 2.0f * lp.scale};
  for (int k0 = 0; k0 < job.K; k0 += C) {
    const int c = std::min(C, job.K - k0);
    Work w = chunk_views(job, 1, chunk_base, c);
    w.status = status;
    w.loss_k = loss_k;
    w.k0 = k0;
    LAUNCH(KC_PREP, launch_prep(jb, w, s));
    for (int l = 0; l < job.L; ++l) LAUNCH(KC_ROW_FWD, launch_row_fwd(jb, w, l, s));
    for (int l = 0; l < job.L; ++l) LAUNCH(KC_COL_FWD, launch_col_fwd(jb, w, l, s));
    int n_loss;
    if (!has_resample(job)) {
      LAUNCH(KC_DET, launch_det(jb, w, ld, want_grad ? 0 : 3, false, nullptr, s));
      n_loss = job.N / rows_per_det_block(job.N);
    } else {
      LAUNCH(KC_DET, launch_det(jb, w, ld, 1, want_grad, w.ibuf, s));
      LAUNCH(KC_RESAMPLE, launch_resample_loss(jb, w, ld, nullptr, s));
      n_loss = static_cast<int>((plane + 255) / 256);
      if (want_grad) {
        LAUNCH(KC_RESAMPLE, launch_resample_T(jb, w, s));
        LAUNCH(KC_DET, launch_det(jb, w, ld, 2, false, nullptr, s));
      }
    }
    if (want_grad) {
      for (int l = 0; l < job.L; ++l) LAUNCH(KC_COL_ADJ, launch_col_adj(jb, w, l, g.g_probe != nullptr, s));
      if (g.g_probe)
        LAUNCH(KC_PROBE_REDUCE, launch_probe_reduce(jb, w, reinterpret_cast<float2*>(g.g_probe), s));
      if (g.g_object || g.g_pos) {
        for (int l = 0; l < job.L; ++l) LAUNCH(KC_ROW_ADJ, launch_row_adj(jb, w, l, s));
      }
      if (g.g_object) {
        for (int l = 0; l < job.L; ++l)
          LAUNCH(KC_OBJ_GATHER, launch_obj_gather(jb, w, l, reinterpret_cast<float2*>(g.g_object), s));
      }
    } else {
      // partial buffers of the adjoint are not produced: keep them zero
      const size_t nd = static_cast<size_t>(c) * job.L * (job.N / col_group_of(job.N));
      LAUNCH(KC_FILL, launch_fill_zero(w.dy_part, nd, s));
      LAUNCH(KC_FILL, launch_fill_zero(w.sg_part, nd, s));
      LAUNCH(KC_FILL, launch_fill_zero(w.dx_part,
                                 static_cast<size_t>(c) * job.L * (job.N / rows_per_adj_block(job.N)), s));
    }
    LAUNCH(KC_FINALIZE, launch_finalize_chunk(jb, w, n_loss, g.g_pos, g.g_sigma, s));
  }
  if (g.loss) {
    Work w{};
    w.status = status;
    w.loss_k = loss_k;
    LAUNCH(KC_FINALIZE, launch_loss_total(jb, w, lp.scale, g.loss, s));
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
    const int e = validate_job(jobs[i], false);
    if (e) return e;
  }
  size_t worst = 0;
  for (int i = 0; i < n_jobs; ++i) {
    const int K = jobs[i].K;
    const int c = chunk <= 0 ? std::max(K, 1) : std::max(1, std::min<int>(chunk, std::max(K, 1)));
    worst = std::max(worst, per_position_bytes(jobs[i], which) * static_cast<size_t>(c));
  }
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
  Layout lay = make_layout(workspace, workspace_bytes, jobs, n_jobs);
  std::vector<int> chunks(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    chunks[i] = chunk_for(jobs[i], 0, lay.chunk_bytes);
    if (jobs[i].K > 0 && chunks[i] < 1) return PTYCHO_ENOSPC;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int i = 0; i < n_jobs; ++i) {
    const ptycho_job_t& job = jobs[i];
    JobDev jb = to_dev(job);
    int* status = lay.status + i;
    LAUNCH(KC_PREP, launch_set_status(status, s));
    LAUNCH(KC_PREP, launch_validate(jb, status, s));
    const size_t plane = static_cast<size_t>(job.N) * job.N;
    for (int k0 = 0; k0 < job.K; k0 += chunks[i]) {
      const int c = std::min(chunks[i], job.K - k0);
      Work w = chunk_views(job, 0, lay.chunk_base, c);
      w.status = status;
      w.loss_k = lay.loss_k;
      w.k0 = k0;
      LAUNCH(KC_PREP, launch_prep(jb, w, s));
      for (int l = 0; l < job.L; ++l) LAUNCH(KC_ROW_FWD, launch_row_fwd(jb, w, l, s));
      for (int l = 0; l < job.L; ++l) LAUNCH(KC_COL_FWD, launch_col_fwd(jb, w, l, s));
      LossDev ld{0, 0.f, 0.f};
      float* out = intensity[i] + static_cast<size_t>(k0) * plane;
      if (!has_resample(job)) {
        LAUNCH(KC_DET, launch_det(jb, w, ld, 1, false, out, s));
      } else {
        LAUNCH(KC_DET, launch_det(jb, w, ld, 1, false, w.ibuf, s));
        LAUNCH(KC_RESAMPLE, launch_resample_loss(jb, w, ld, out, s));
      }
    }
  }
  return PTYCHO_OK;
}

int32_t ptycho_loss_grad(const ptycho_job_t* jobs, int32_t n_jobs, const ptycho_loss_t* loss,
                         const ptycho_grads_t* grads, void* workspace, size_t workspace_bytes,
                         void* stream) {
  int e = common_checks(jobs, n_jobs, true);
  if (e) return e;
  if (!loss || !grads || !workspace) return PTYCHO_EINVAL;
  if (loss->kind < 0 || loss->kind > 3 || !(loss->eps >= 0.f) || !std::isfinite(loss->scale))
    return PTYCHO_EINVAL;
  Layout lay = make_layout(workspace, workspace_bytes, jobs, n_jobs);
  std::vector<int> chunks(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    chunks[i] = chunk_for(jobs[i], 1, lay.chunk_bytes);
    if (jobs[i].K > 0 && chunks[i] < 1) return PTYCHO_ENOSPC;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int i = 0; i < n_jobs; ++i) {
    e = run_loss_grad(jobs[i], *loss, grads[i], lay.status + i, lay.loss_k, lay.chunk_base,
                      std::max(chunks[i], 1), s);
    if (e) return e;
  }
  return PTYCHO_OK;
}

int32_t ptycho_step(const ptycho_job_t* jobs, int32_t n_jobs, const ptycho_loss_t* loss,
                    const ptycho_grads_t* grads, const ptycho_adam_t* adam, void* workspace,
                    size_t workspace_bytes, void* stream) {
  if (!adam || !grads) return PTYCHO_EINVAL;
  for (int i = 0; n_jobs > 0 && jobs && i < n_jobs; ++i) {
    const ptycho_adam_t& a = adam[i];
    if (a.t < 1 || !(a.beta1 >= 0.f && a.beta1 < 1.f) || !(a.beta2 >= 0.f && a.beta2 < 1.f))
      return PTYCHO_EINVAL;
    if (a.lr_object != 0.f && (!a.m_object || !a.v_object || !grads[i].g_object)) return PTYCHO_EINVAL;
    if (a.lr_probe != 0.f && (!a.m_probe || !a.v_probe || !grads[i].g_probe)) return PTYCHO_EINVAL;
    if (a.lr_pos != 0.f && (!a.m_pos || !a.v_pos || !grads[i].g_pos)) return PTYCHO_EINVAL;
  }
  int e = ptycho_loss_grad(jobs, n_jobs, loss, grads, workspace, workspace_bytes, stream);
  if (e) return e;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int i = 0; i < n_jobs; ++i) {
    const ptycho_job_t& j = jobs[i];
    const ptycho_adam_t& a = adam[i];
    const float bc1 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(a.beta1), a.t)));
    const float bc2 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(a.beta2), a.t)));
    const size_t plane = static_cast<size_t>(j.N) * j.N;
    if (a.lr_object != 0.f)
      LAUNCH(KC_ADAM, launch_adam(j.object, grads[i].g_object, a.m_object, a.v_object,
                            2ull * j.L * j.H * j.W, a.lr_object, a.beta1, a.beta2, a.eps, bc1, bc2, s));
    if (a.lr_probe != 0.f)
      LAUNCH(KC_ADAM, launch_adam(j.probe, grads[i].g_probe, a.m_probe, a.v_probe, 2ull * j.L * j.M * plane,
                            a.lr_probe, a.beta1, a.beta2, a.eps, bc1, bc2, s));
    if (a.lr_pos != 0.f && j.K > 0)
      LAUNCH(KC_ADAM, launch_adam(j.pos, grads[i].g_pos, a.m_pos, a.v_pos, 2ull * j.K, a.lr_pos, a.beta1,
                            a.beta2, a.eps, bc1, bc2, s));
  }
  return PTYCHO_OK;
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
