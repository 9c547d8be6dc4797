// Stencil dispatch, autotuner and launch timer for the Wilson hopping
// stencil (arXiv:1106.4964 Sec. II, eq. 1-2).  The kernels themselves are in
// stencil_kernels.h, instantiated per storage precision.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <tuple>

#include "stencil_kernels.h"

namespace ovl {
namespace {

void launch_shape(const StencilArgs& A, int prec, int recon, int nrhs, Shape sh, hipStream_t s) {
  switch (prec) {
    case OVL_F64: launch_stencil_f64(A, recon, nrhs, sh, s); break;
    case OVL_F32: launch_stencil_f32(A, recon, nrhs, sh, s); break;
    case OVL_F16: launch_stencil_f16(A, recon, nrhs, sh, s); break;
    case OVL_BF16: launch_stencil_bf16(A, recon, nrhs, sh, s); break;
    default: throw Error(OVL_E_PRECISION, "unknown precision");
  }
}

// ------------------------------------------------------------------ tuner
// The shape (vectors per thread, block size) of each stencil configuration
// is chosen once per process by timing every candidate with HIP events on a
// scratch output; OVL_TUNE=0 keeps the static default.  Results are cached
// in memory, keyed by precision, link format, extra vectors, batch size,
// output parities and lattice volume.
struct TuneKey {
  int prec, recon, nv, nrhs, npar, nh;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, recon, nv, nrhs, npar, nh) < std::tie(o.prec, o.recon, o.nv, o.nrhs, o.npar, o.nh);
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, Shape> g_tuned;

std::atomic<int> g_tune_mode{-1};  // -1: not read yet, 0: static default, 1: autotune

bool tuning_enabled() {
  int m = g_tune_mode.load();
  if (m < 0) {
    const char* e = std::getenv("OVL_TUNE");
    m = (e && e[0] == '0') ? 0 : 1;
    g_tune_mode.store(m);
  }
  return m == 1;
}

std::vector<Shape> candidates(int prec, int nrhs, int Lz) {
  std::vector<Shape> c;
  const int kmax = prec == OVL_F64 ? 2 : 4;
  // block orders: by h, t-major, and z-slabs of 4 and 8 planes
  for (int tm : {0, 1, 4, 8}) {
    if (tm > Lz) continue;
    for (int kr = 1; kr <= kmax; ++kr)
      if (nrhs % kr == 0) {
        for (int bs : {128, 256}) c.push_back({kr, bs, 0, 0, tm});
        if (nrhs > kr)  // several groups: try them side by side in one workgroup
          for (int bs : {32, 64})
            if (bs * (nrhs / kr) <= 512) c.push_back({kr, bs, 0, 1, tm});
      }
    for (int dep : {2, 3, 4})
      if (prec != OVL_F64 || dep == 2)
        for (int bs : {128, 256}) c.push_back({1, bs, dep, 0, tm});
  }
  return c;
}

Shape default_shape(int prec, int nrhs) {
  const int kmax = prec == OVL_F64 ? 2 : 4;
  for (int kr = kmax; kr >= 1; --kr)
    if (nrhs % kr == 0) return {kr, 256, 0, 0, 0};
  return {1, 256, 0, 0, 0};
}

Shape pick_shape(const StencilArgs& A, int prec, int recon, int nrhs, hipStream_t s) {
  const TuneKey key{prec, recon, A.nv, nrhs, A.npar, A.g.Nh};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  const Shape def = default_shape(prec, nrhs);
  if (!tuning_enabled()) return def;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return def;
  // time every candidate on a scratch output (the real output may alias an input)
  StencilArgs T = A;
  WsBuf scratch(A.vstride * nrhs, s);
  T.out = scratch.p;
  hipEvent_t e0, e1;
  OVL_HIP(hipEventCreate(&e0));
  OVL_HIP(hipEventCreate(&e1));
  // two rounds over the candidates, each timed over 3 launches after a
  // warm-up launch; a candidate's time is its better round.  The first
  // candidate (in list order) within 2% of the fastest wins, so that shapes
  // that time alike give the same choice from run to run.
  const std::vector<Shape> cand = candidates(prec, nrhs, A.g.Lz);
  std::vector<float> best_ms(cand.size(), 1e30f);
  for (int round = 0; round < 2; ++round)
    for (size_t i = 0; i < cand.size(); ++i) {
      launch_shape(T, prec, recon, nrhs, cand[i], s);  // warm-up
      OVL_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) launch_shape(T, prec, recon, nrhs, cand[i], s);
      OVL_HIP(hipEventRecord(e1, s));
      OVL_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      OVL_HIP(hipEventElapsedTime(&ms, e0, e1));
      best_ms[i] = std::min(best_ms[i], ms);
    }
  float fastest = 1e30f;
  for (float t : best_ms) fastest = std::min(fastest, t);
  Shape best = def;
  for (size_t i = 0; i < cand.size(); ++i)
    if (best_ms[i] <= 1.02f * fastest) {
      best = cand[i];
      break;
    }
  OVL_HIP(hipEventDestroy(e0));
  OVL_HIP(hipEventDestroy(e1));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

}  // namespace

// Per-configuration launch timer: HIP events recorded on the launch stream
// around each stencil launch while enabled (not during stream capture).
namespace {
struct TimerKey {
  int prec, recon, nv, nrhs;
  bool operator<(const TimerKey& o) const {
    return std::tie(prec, recon, nv, nrhs) < std::tie(o.prec, o.recon, o.nv, o.nrhs);
  }
};
struct TimerRec {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  int64_t launches = 0;
  double ms = 0.0;
};
std::atomic<bool> g_timing{false};
std::mutex g_timer_mu;
std::map<TimerKey, TimerRec> g_timer;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t timer_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  OVL_HIP(hipEventCreate(&e));
  return e;
}

void timer_settle(TimerRec& r) {
  for (auto& pr : r.pending) {
    OVL_HIP(hipEventSynchronize(pr.second));
    float ms = 0.f;
    OVL_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    r.ms += ms;
    r.launches += 1;
    g_event_pool.push_back(pr.first);
    g_event_pool.push_back(pr.second);
  }
  r.pending.clear();
}
}  // namespace

void launch_stencil(const StencilArgs& A, int prec, int recon, int nrhs, hipStream_t s) {
  OVL_REQUIRE(recon == 18 || recon == 12, OVL_E_PRECISION, "link representation missing");
  count_stencil(nrhs);
  const Shape sh = pick_shape(A, prec, recon, nrhs, s);
  bool timed = false;
  if (g_timing.load(std::memory_order_relaxed)) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    timed = hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone;
  }
  if (!timed) {
    launch_shape(A, prec, recon, nrhs, sh, s);
    return;
  }
  std::lock_guard<std::mutex> lk(g_timer_mu);
  hipEvent_t e0 = timer_event(), e1 = timer_event();
  OVL_HIP(hipEventRecord(e0, s));
  launch_shape(A, prec, recon, nrhs, sh, s);
  OVL_HIP(hipEventRecord(e1, s));
  g_timer[TimerKey{prec, recon, A.nv, nrhs}].pending.emplace_back(e0, e1);
}

void stencil_timer(int mode) {
  std::lock_guard<std::mutex> lk(g_timer_mu);
  if (mode == 1 || mode == 2) {
    for (auto& kv : g_timer) timer_settle(kv.second);
    g_timer.clear();
  }
  if (mode == 0 || mode == 1) g_timing.store(mode == 1);
}

void stencil_timer_read(int prec, int recon, int nv, int nrhs, int64_t* launches, double* ms) {
  std::lock_guard<std::mutex> lk(g_timer_mu);
  auto it = g_timer.find(TimerKey{prec, recon, nv, nrhs});
  if (it == g_timer.end()) {
    *launches = 0;
    *ms = 0.0;
    return;
  }
  timer_settle(it->second);
  *launches = it->second.launches;
  *ms = it->second.ms;
}

void set_tune_mode(int mode) {
  g_tune_mode.store(mode ? 1 : 0);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
}

int stencil_shape(int prec, int recon, int nv, int nrhs, int npar, int nh, int* shape5) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(TuneKey{prec, recon, nv, nrhs, npar, nh});
  if (it == g_tuned.end()) return 0;
  const Shape& sh = it->second;
  shape5[0] = sh.kr;
  shape5[1] = sh.bs;
  shape5[2] = sh.pipe;
  shape5[3] = sh.rin;
  shape5[4] = sh.tm;
  return 1;
}

void force_shape(int prec, int recon, int nv, int nrhs, int npar, int nh, const int* shape5) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[TuneKey{prec, recon, nv, nrhs, npar, nh}] = Shape{shape5[0], shape5[1], shape5[2], shape5[3], shape5[4]};
}

}  // namespace ovl
