// sbs_runtime.cpp -- host runtime behind the C ABI of include/sbs.h.
//
// Device memory: every buffer is carved from the caller's arena by a
// first-fit allocator (persistent controller state at init, step workspaces
// per launched batch, released when the batch completes).  Pinned host
// staging comes from one hipHostMalloc block carved the same way.
//
// A batch is the unit of launch: its descriptors and block maps go to the
// device in one copy, then per iteration one launch per stage covers every
// controller of the batch, then one copy brings all actions back and an
// event marks completion.  Direct mode launches each submission at once;
// serving mode queues submissions for a scheduler thread that forms batches
// from whatever is pending whenever a stream slot frees up and the arena can
// hold the workspace (continuous batching with memory admission).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <sys/prctl.h>

#include "../../include/sbs.h"
#include "sbs_device.h"

namespace sbs {
hipError_t launch_iteration(const LaunchTab &tab, int precision, hipStream_t s, int timing,
                            hipEvent_t *ev, const TickDesc *inl,
                            const std::function<hipError_t()> *after_rollout = nullptr);
hipError_t launch_noise_only(const LaunchTab &tab, hipStream_t s, const TickDesc *inl);
hipError_t launch_empty_timed(hipStream_t s, hipEvent_t e0, hipEvent_t e1);
}

using namespace sbs;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

constexpr uint64_t kAlign = 256;
// auto policy: four lanes per sample up to this many samples in one launch
constexpr long long kQuadMaxSamples = 32768;
// Mean rows per elite / best-sample update workgroup in a batch: at most
// kUpdMaxChunk, and no more than keeps kUpdTargetGroups workgroups (eight
// per compute unit).  A workgroup reduces its rows one after the other, so
// rows run in parallel until the device is several times full.
constexpr long long kUpdMaxChunk = 8;
constexpr long long kUpdTargetGroups = 2048;

// Step workspace of sbs_submit_tick_noalloc: one file-scope device array per
// GPU, held until the process ends.  Host code never names it directly (its
// name is a host-side stand-in there): each device's address is taken once,
// with that device current, when a runtime is created on it.
constexpr uint64_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch array (taken on first use per device).
// Caller has the device current.
int scratch_address(int device, char **out) {
  if (device < 0 || device >= kMaxDevices) return fail(SBS_EDEVICE, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SBS_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<char *>(p);
  }
  *out = g_scratch_ptr[device];
  return SBS_OK;
}
// noise rows per thread of a single controller's ahead-of-time noise
constexpr int kPrefetchRows = 10;  // measured at C1: 1, 4, 10, 25 rows -> 60.2, 58.9, 58.1, 71.9 us per tick

// With several batches in flight per stream the next batch is formed as late
// as keeps the stream busy: when the batches ahead of it are estimated to
// end within kJitMarginNs (the host's batch assembly and launch fit in it),
// so that it takes every request submitted meanwhile.  The estimate uses
// the device rate of retired batches of at least kJitMinSteps rollout-steps.
constexpr int64_t kJitMarginNs = 150000;
constexpr double kJitMinSteps = 1e6;
constexpr int64_t kDispatchNs = 20000;  // launch to device start of an idle stream
// A batch header goes up on the copy stream when the work ahead of the
// batch on its stream is estimated to run for longer than this (measured at C4:
// 30 us against always or never).
constexpr int64_t kHdrAheadNs = 30000;
// MPPI costs the update holds in registers (16 per thread of 1024): a
// rollout may leave the noise rows to the update (which lists the samples it
// weighs from those registers) only up to this many samples.
constexpr int kMppiRegN = 16 * 1024;

// Rollout form: lanes per sample (0 = automatic), workgroup size, step-loop
// unroll.  Only the forms the kernel dispatcher instantiates are valid.
struct Tune {
  int lanes = 0;
  int block = 256;  // four waves per workgroup: measured faster than 64 or 128 at C1
  int unroll = 1;
  bool pairs = true;  // stance-pair one-lane rollouts where the gait allows
  // one-lane FP32 per-step rollouts make their own noise: 0 no (a noise
  // launch), 1 every row, 2 only the stance legs' Gaussians for controllers
  // in the stance-pair form (every row for the others)
  int gen = 2;
};

bool valid_form(int lanes, int block, int unroll) {
  if (lanes == 4) return unroll == 1 && (block == 64 || block == 128 || block == 256);
  if (lanes == 1)
    return (unroll == 1 && (block == 64 || block == 128 || block == 256)) ||
           (unroll == 2 && (block == 64 || block == 128));
  return false;
}
uint64_t align_up(uint64_t v, uint64_t a = kAlign) { return (v + a - 1) / a * a; }

// Rows of the mean: the spline knot count P, else the horizon H.
int rows_of(const sbs_controller_cfg &c) { return c.knots > 0 ? c.knots : c.H; }

// GRF spline of Sec. IV-B as weights on the knots.  Knot p sits at
// t_p = p T / (P - 1), T = (H - 1) dt.  On [t_p, t_{p+1}] (h = t_{p+1} - t_p,
// s = (t - t_p) / h) the spline is the cubic Hermite form
//   (2s^3 - 3s^2 + 1) y_p + (s^3 - 2s^2 + s) h m_p + (-2s^3 + 3s^2) y_{p+1}
//   + (s^3 - s^2) h m_{p+1}
// with slopes m_p = (y_b - y_a) / (t_b - t_a), a = max(p-1, 0),
// b = min(p+1, P-1).  Every step therefore weighs at most the four knots
// p-1 .. p+2; the window starts at max(0, min(p-1, P-4)).
struct SplineRow {
  int32_t base;
  double w[4];
};

// seg >= 0 gives the segment of t directly (steps on the grid, below);
// seg < 0 finds it by comparing t with the knot times.
SplineRow spline_row(int P, int H, double dt, double t, int seg = -1) {
  const double T = (double)(H - 1) * dt;
  auto tk = [&](int p) { return (double)p * T / (double)(P - 1); };
  t = std::min(std::max(t, 0.0), T);
  int p = 0;
  if (seg >= 0) p = std::min(seg, P - 2);
  else while (p < P - 2 && t >= tk(p + 1)) ++p;
  const double h = tk(p + 1) - tk(p), s = (t - tk(p)) / h;
  const double h00 = 2 * s * s * s - 3 * s * s + 1, h10 = s * s * s - 2 * s * s + s;
  const double h01 = -2 * s * s * s + 3 * s * s, h11 = s * s * s - s * s;
  std::vector<double> coef(P, 0.0);
  auto slope = [&](int q, double scale) {  // adds scale * h * m_q
    const int a = std::max(q - 1, 0), b = std::min(q + 1, P - 1);
    const double g = scale * h / (tk(b) - tk(a));
    coef[b] += g;
    coef[a] -= g;
  };
  coef[p] += h00;
  coef[p + 1] += h01;
  slope(p, h10);
  slope(p + 1, h11);
  SplineRow r{};
  r.base = std::max(0, std::min(p - 1, P - 4));
  for (int i = 0; i < 4; ++i) r.w[i] = (r.base + i < P) ? coef[r.base + i] : 0.0;
  return r;
}

// First-fit allocator over [0, size) with coalescing frees.
class Carver {
 public:
  void reset(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
    used_ = 0;
  }
  bool alloc(uint64_t bytes, uint64_t *off) {
    bytes = align_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        uint64_t rest = it->second - bytes, roff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = align_up(bytes ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }
  uint64_t size() const { return size_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t size_ = 0, used_ = 0;
};

struct Controller {
  int32_t id = -1;
  sbs_controller_cfg cfg{};
  uint64_t st_off = 0, st_bytes = 0;
  void *mu_buf[2] = {nullptr, nullptr};  // double-buffered mean [rows][12]
  uint64_t mu_bytes = 0;
  // spline tables (knots > 0): device copies inside the persistent state,
  // host copies for the warm-start shift of sbs_get_state
  const double *sp_w = nullptr, *sh_w = nullptr;
  const int32_t *sp_b = nullptr, *sh_b = nullptr;
  std::vector<double> h_sh_w;
  std::vector<int32_t> h_sh_b;
  int par = 0;              // buffer holding the current mean
  bool needs_shift = false; // it is the previous tick's mean (unshifted)
  double *ctl = nullptr;
  uint32_t next_tick = 0;
  bool debug = false;
  uint64_t dbg_off = 0, dbg_bytes = 0;
  double *dbg_J = nullptr;
  uint32_t *dbg_q = nullptr;
  double *dbg_mean = nullptr;
  int inflight = 0;
  int plan = -1;
  // noise prefetch: two buffers of iterations x H x N x 12 floats; the next
  // tick's noise is written into the idle one on the second stream
  bool prefetch = false;
  uint64_t pf_off = 0, pf_bytes = 0;
  float *pf_z[2] = {nullptr, nullptr};
  int64_t pf_tick[2] = {-1, -1};
  hipEvent_t pf_ready[2] = {nullptr, nullptr};
  hipEvent_t pf_free[2] = {nullptr, nullptr};
};

struct Request {
  uint64_t ticket;
  int32_t id;
  sbs_tick_input in;
  int64_t t_submit;
};

struct TicketRec {
  int32_t controller = -1;
  uint32_t tick = 0;
  int status = 1;  // 1 pending, 0 done, <0 error
  int64_t t_submit = 0, t_launch = 0, t_done = 0;
  double res[kResultDoubles];
  // the launched tick's action record in pinned memory: complete once its
  // sequence word reads tick + 1 (before the batch itself has retired)
  const double *rec = nullptr;
};

// Completes a pending ticket from its action record if the kernel has
// finished writing it.
bool complete_from_record(TicketRec &t) {
  if (t.status != 1 || !t.rec) return false;
  const uint64_t *seq = reinterpret_cast<const uint64_t *>(t.rec + RES_SEQ);
  if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) != (uint64_t)t.tick + 1u) return false;
  std::memcpy(t.res, t.rec, sizeof t.res);
  t.status = 0;
  t.t_done = now_ns();
  return true;
}

// A completed ticket's action record as the C ABI returns it.
void fill_action(const TicketRec &t, sbs_action *out) {
  std::memset(out, 0, sizeof *out);
  for (int i = 0; i < 12; ++i) out->grf[i] = t.res[RES_GRF + i];
  for (int l = 0; l < 4; ++l) out->contact[l] = (int32_t)t.res[RES_CONTACT + l];
  out->freq_hz = t.res[RES_FREQ];
  out->q = (uint32_t)t.res[RES_Q];
  out->best_cost = t.res[RES_BEST];
  out->flags = (int32_t)t.res[RES_FLAGS];
  out->tick = t.tick;
  out->controller = t.controller;
  out->t_submit_ns = t.t_submit;
  out->t_launch_ns = t.t_launch;
  out->t_done_ns = t.t_done;
  out->n_active = (uint32_t)t.res[RES_NACT];
}

// Byte layout of one batch (device workspace and host staging share the
// header part so that one copy uploads it).
struct Layout {
  uint64_t desc = 0, tabs = 0, hdr_bytes = 0, results = 0, items = 0, total = 0;
  std::vector<uint64_t> item_off;  // per item workspace offset
  uint64_t host_total = 0;         // header + results
};

struct ItemWs {
  uint64_t z, q, J, w, act, sigma, it, bytes;
};

ItemWs item_ws(const sbs_controller_cfg &c) {
  ItemWs o{};
  const uint64_t N = (uint64_t)c.N, M = (uint64_t)rows_of(c);
  const uint64_t ts = c.precision == SBS_FP64 ? 8 : 4;
  uint64_t p = 0;
  o.z = p; p = align_up(p + M * N * 12 * 4);
  o.q = p; p = align_up(p + N * 4);
  o.J = p; p = align_up(p + N * ts);
  o.w = p; p = align_up(p + N * ts);
  o.act = p; p = align_up(p + N * 4);
  o.sigma = p; p = align_up(p + M * 12 * 8);
  o.it = p; p = align_up(p + kItScalars * 8);
  o.bytes = p;
  return o;
}

struct Batch {
  int id = 0;
  int stream_slot = 0;
  hipEvent_t done = nullptr;
  hipEvent_t hdr = nullptr;  // header upload on the copy stream
  std::vector<uint64_t> tickets;
  std::vector<int32_t> ctrls;
  uint64_t ws_off = 0, ws_bytes = 0, host_off = 0, host_bytes = 0;
  double *host_results = nullptr;
  int plan = -1;
  std::vector<hipEvent_t> timing;  // 5 per launched (iteration, precision)
  // modes 1 and 3: per timed rollout launch, its form (RollForm) and
  // rollout-steps
  std::vector<std::pair<int, double>> timing_work;
  bool owns_memory = true;  // device workspace carved from the arena
  bool owns_host = true;    // pinned staging carved from the runtime's block
  // serving schedule: rollout-steps of all iterations, and the estimated
  // device start (host clock), re-anchored when the batch ahead retires
  double steps = 0;
  int64_t t_start_est = 0;
};

// Rollout forms told apart by the per-form timing accumulators.
enum RollForm {
  FORM_FP32_ONE_LANE = 0, FORM_FP32_QUAD = 1, FORM_FP64 = 2, FORM_FP32_ONE_LANE_NOISE = 3,
  FORM_FP32_ONE_LANE_STANCE_NOISE = 4, kForms = 5
};
int roll_form(const LaunchTab &t, int precision) {
  if (precision == SBS_FP64) return FORM_FP64;
  if (t.lanes == 4) return FORM_FP32_QUAD;
  if (t.gen_noise == 2) return FORM_FP32_ONE_LANE_STANCE_NOISE;
  return t.gen_noise ? FORM_FP32_ONE_LANE_NOISE : FORM_FP32_ONE_LANE;
}

struct Plan {
  int id = -1;
  std::vector<int32_t> ctrls;
  Layout lay;
  uint64_t ws_off = 0, host_off = 0;
  char *host = nullptr;
  char *dev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = false;
  bool busy = false;
  hipEvent_t done = nullptr;
  Tune tune;
};

}  // namespace

struct sbs_runtime {
  std::mutex mu;
  std::condition_variable cv;
  int device = 0;
  char *arena = nullptr;
  Carver dev_alloc;
  char *pinned = nullptr;
  char *pinned_dev = nullptr;  // device-visible address of the pinned block
  Carver host_alloc;
  hipStream_t streams[2] = {nullptr, nullptr};
  int nstreams = 1;
  int slot_depth = 1;  // serving: batches in flight per stream
  // batch headers go up on their own stream, so that the copy runs while the
  // batches ahead of it compute
  hipStream_t copy_stream = nullptr;
  double jit_rate = 0;  // rollout-steps per ns of retired batches (EMA), 0: none yet
  int mode = SBS_MODE_DIRECT;
  int32_t next_id = 0;
  std::unordered_map<int32_t, Controller> ctrls;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, TicketRec> tickets;
  std::deque<Request> pending;
  std::deque<std::unique_ptr<Batch>> inflight;  // launch order
  int next_batch = 0;
  std::unordered_map<int, std::unique_ptr<Plan>> plans;
  int next_plan = 0;
  std::vector<hipEvent_t> event_pool;
  std::vector<hipEvent_t> timing_pool;  // hipEventDisableSystemFence: timing only
  // serving
  std::thread sched;
  std::atomic<bool> stop{false};
  uint64_t n_ticks = 0, n_batches = 0, n_admit_waits = 0;
  // timing
  int timing = 0;  // 0 off, 1 rollout kernel (sampled launches), 2 all stages
  uint64_t timing_seq = 0;  // launches seen in mode 1
  Tune tune;  // default rollout form of direct and serving launches
  char *scratch = nullptr;  // this device's scratch array (sbs_submit_tick_noalloc)
  double stage_ns[4] = {0, 0, 0, 0};
  uint64_t stage_n[4] = {0, 0, 0, 0};
  // rollout timing per form (modes 1 and 3): device time, launches and
  // rollout-steps of the timed launches
  double form_ns[5] = {0, 0, 0, 0, 0}, form_steps[5] = {0, 0, 0, 0, 0};
  uint64_t form_n[5] = {0, 0, 0, 0, 0};
};

namespace {

hipEvent_t take_event(sbs_runtime *rt) {
  if (!rt->event_pool.empty()) {
    hipEvent_t e = rt->event_pool.back();
    rt->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void give_event(sbs_runtime *rt, hipEvent_t e) {
  if (e) rt->event_pool.push_back(e);
}

// Events that only time work: without the system-scope fence, recording one
// does not write back and invalidate the caches, so the measured interval
// holds the bracketed work and no cache maintenance of its own.
hipEvent_t take_timing_event(sbs_runtime *rt) {
  if (!rt->timing_pool.empty()) {
    hipEvent_t e = rt->timing_pool.back();
    rt->timing_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

void give_timing_event(sbs_runtime *rt, hipEvent_t e) {
  if (e) rt->timing_pool.push_back(e);
}

bool finite_vec(const double *v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

uint32_t host_q_of_freq(double f, double dt) {
  double v = std::rint((f * dt) * 4294967296.0);
  if (!(v > 0.0)) return 0u;
  if (v > 4294967295.0) return 4294967295u;
  return (uint32_t)v;
}

int validate_cfg(const sbs_controller_cfg &c) {
  if (c.N < 1 || c.N > (1 << 22)) return fail(SBS_EINVAL, "N=%d out of [1, 2^22]", c.N);
  if (c.H < 1 || c.H > kMaxH) return fail(SBS_EINVAL, "H=%d out of [1, %d]", c.H, kMaxH);
  if (c.knots != 0 && (c.knots < 2 || c.knots > c.H))
    return fail(SBS_EINVAL, "knots=%d: 0, or 2 <= knots <= H=%d", c.knots, c.H);
  if (c.iterations < 1 || c.iterations > 64)
    return fail(SBS_EINVAL, "iterations=%d out of [1, 64]", c.iterations);
  if (c.method < 0 || c.method > 2) return fail(SBS_EINVAL, "unknown method %d", c.method);
  if (c.freq_mode < 0 || c.freq_mode > 3) return fail(SBS_EINVAL, "unknown freq_mode %d", c.freq_mode);
  if (c.freq_mode == SBS_FREQ_SET) {
    if (c.n_fset < 1 || c.n_fset > 4) return fail(SBS_EINVAL, "n_fset=%d out of [1, 4]", c.n_fset);
    for (int i = 0; i < c.n_fset; ++i)
      if (!(c.f_set[i] > 0)) return fail(SBS_EINVAL, "frequency set members must be > 0");
  }
  if (c.precision != SBS_FP32 && c.precision != SBS_FP64)
    return fail(SBS_EINVAL, "unknown precision %d", c.precision);
  if (!(c.dt > 0) || !(c.mass > 0) || !(c.gravity > 0) || !(c.inertia[0] > 0) ||
      !(c.inertia[1] > 0) || !(c.inertia[2] > 0))
    return fail(SBS_EINVAL, "dt, mass, gravity and inertia must be positive");
  if (c.method == SBS_MPPI && !(c.lambda > 0)) return fail(SBS_EINVAL, "lambda must be positive");
  if (!(c.duty >= 0.0 && c.duty <= 1.0)) return fail(SBS_EINVAL, "duty must be in [0, 1]");
  if (!(c.sigma_grf >= 0.0)) return fail(SBS_EINVAL, "sigma_grf must be >= 0");
  if ((c.freq_mode == SBS_FREQ_UNIFORM || c.freq_mode == SBS_FREQ_GAUSSIAN) &&
      !(c.f_min > 0 && c.f_max >= c.f_min))
    return fail(SBS_EINVAL, "frequency range must satisfy 0 < f_min <= f_max");
  if (c.freq_mode == SBS_FREQ_FIXED && !(c.f_fixed > 0)) return fail(SBS_EINVAL, "f_fixed must be > 0");
  return SBS_OK;
}

// Diagonal trot at duty 1/2 (leg 3 in phase with leg 0, legs 1 and 2 half a
// cycle later, stance iff phase < 2^31): exactly one diagonal pair is in
// stance at every step, which the stance-pair rollouts exploit.
bool pair_gait(const sbs_controller_cfg &c) {
  const uint32_t o0 = c.phase_offset[0], half = 0x80000000u;
  return std::rint(c.duty * 4294967296.0) == 2147483648.0 &&
         c.phase_offset[3] == o0 && c.phase_offset[1] == o0 + half &&
         c.phase_offset[2] == o0 + half;
}

// Whether a controller's one-lane FP32 rollout may make only its stance
// legs' noise (the update then makes the rows of the samples it weighs or
// chooses).  It depends on the configuration alone, so a controller takes
// the same form in every tick, alone, in a batch, in a plan and after a
// resume; a controller whose noise is produced ahead of its ticks keeps
// reading stored rows in every tick.
bool stance_noise(const Controller &C, const Tune &tn) {
  const sbs_controller_cfg &c = C.cfg;
  return tn.gen == 2 && tn.pairs && !C.prefetch && c.precision == SBS_FP32 && c.knots == 0 &&
         c.N <= kMppiRegN && pair_gait(c);
}

void fill_desc(const sbs_runtime *rt, const Controller &C, const ItemWs &w, char *dev_item,
               double *dev_result, const sbs_tick_input &in, uint32_t tick, int slot,
               TickDesc *d) {
  const sbs_controller_cfg &c = C.cfg;
  std::memset(d, 0, sizeof *d);
  d->N = c.N;
  d->H = c.H;
  d->R = c.iterations;
  d->method = c.method;
  d->freq_mode = c.freq_mode;
  d->friction_on = c.friction_on ? 1 : 0;
  d->precision = c.precision;
  double kef = std::floor(c.elite_frac * (double)c.N);
  int32_t ke = (int32_t)std::min<double>(std::max<double>(kef, 1.0), (double)c.N);
  d->Ke = c.method == SBS_NAIVE ? 1 : ke;
  d->mu_par0 = C.par;
  d->shift0 = C.needs_shift ? 1 : 0;
  d->tick = tick;
  d->phase_robot = in.phase_robot;
  d->q_fixed = host_q_of_freq(c.f_fixed, c.dt);
  d->q_lo = host_q_of_freq(c.f_min, c.dt);
  d->q_hi = host_q_of_freq(c.f_max, c.dt);
  d->n_fset = c.freq_mode == SBS_FREQ_SET ? c.n_fset : 0;
  for (int i = 0; i < 4; ++i) d->q_set[i] = i < d->n_fset ? host_q_of_freq(c.f_set[i], c.dt) : 0u;
  for (int l = 0; l < 4; ++l) d->phase_offset[l] = c.phase_offset[l];
  const double dq = std::rint(c.duty * 4294967296.0);
  d->duty_full = dq >= 4294967296.0 ? 1 : 0;
  d->duty_q = d->duty_full ? 0xFFFFFFFFu : (uint32_t)dq;
  // diagonal trot at duty 1/2: leg 3 in phase with leg 0 and legs 1, 2 half
  // a cycle later, so exactly one diagonal pair is in stance at every step
  d->slot = slot;
  d->M = rows_of(c);
  d->spline = c.knots > 0 ? 1 : 0;
  d->sp_w = C.sp_w;
  d->sp_b = C.sp_b;
  d->sh_w = C.sh_w;
  d->sh_b = C.sh_b;
  d->seed = c.seed;
  d->dt = c.dt;
  d->inv_lambda = c.method == SBS_MPPI ? 1.0 / c.lambda : 0.0;
  d->mu_fric = c.mu_fric;
  d->rho = c.rho;
  d->f_nominal = c.f_nominal;
  d->mass = c.mass;
  d->inv_mass = 1.0 / c.mass;
  d->gravity = c.gravity;
  d->inv_g = 1.0 / c.gravity;
  for (int i = 0; i < 3; ++i) {
    d->inertia[i] = c.inertia[i];
    d->inv_inertia[i] = 1.0 / c.inertia[i];
  }
  for (int i = 0; i < 12; ++i) {
    d->hip[i] = c.hip[i];
    d->Q[i] = c.Q[i];
    d->Rw[i] = c.R[i];
    d->x0[i] = in.x0[i];
    d->foot[i] = in.foot_pos[i];
  }
  d->sigma0 = c.sigma_grf;
  d->sigma_f0 = c.sigma_f;
  d->sigma_min_grf = c.sigma_min_grf;
  d->sigma_min_f = c.sigma_min_f;
  d->f_min = c.f_min;
  d->f_max = c.f_max;
  d->f_fixed = c.f_fixed;
  d->half_duty = 0.5 * c.duty;
  d->inv_q_scale = 1.0 / (c.dt * 4294967296.0);
  for (int i = 0; i < 3; ++i) {
    d->p_ref0[i] = in.p_ref0[i];
    d->v_ref[i] = in.v_ref[i];
  }
  d->yaw_ref = in.yaw_ref;
  d->mu_buf[0] = C.mu_buf[0];
  d->mu_buf[1] = C.mu_buf[1];
  d->ctl = C.ctl;
  d->z = reinterpret_cast<float *>(dev_item + w.z);
  d->q = reinterpret_cast<uint32_t *>(dev_item + w.q);
  d->J = dev_item + w.J;
  d->w = dev_item + w.w;
  d->act = reinterpret_cast<uint32_t *>(dev_item + w.act);
  d->sigma = reinterpret_cast<double *>(dev_item + w.sigma);
  d->it = reinterpret_cast<double *>(dev_item + w.it);
  d->result = dev_result;
  if (C.debug) {
    d->dbg_J = C.dbg_J;
    d->dbg_q = C.dbg_q;
    d->dbg_mean = C.dbg_mean;
  }
  (void)rt;
}

// Launch groups per iteration: precision x parametrisation x stance-pair form.
constexpr int kGroups = 16;

// Byte offset of the first item workspace in a batch of n controllers with
// at most rmax iterations: descriptors, then per (iteration, launch group)
// item[n] + 3 x start[n+1], then the action records.
uint64_t layout_items_offset(uint64_t n, int rmax) {
  const uint64_t tabs = align_up(n * sizeof(TickDesc));
  const uint64_t tab_bytes = align_up((n + 3 * (n + 1)) * 4);
  const uint64_t hdr = align_up(tabs + (uint64_t)rmax * kGroups * tab_bytes);
  return align_up(hdr + n * kResultDoubles * 8);
}

// Layout of a batch over the given controllers.
Layout make_layout(const std::vector<const Controller *> &cs) {
  Layout L;
  const uint64_t n = cs.size();
  int rmax = 1;
  for (auto *c : cs) rmax = std::max(rmax, c->cfg.iterations);
  L.desc = 0;
  L.tabs = align_up(n * sizeof(TickDesc));
  // per (iteration, precision, parametrisation): item[n] + 3 x start[n+1]
  const uint64_t tab_bytes = align_up((n + 3 * (n + 1)) * 4);
  L.hdr_bytes = align_up(L.tabs + (uint64_t)rmax * kGroups * tab_bytes);
  L.results = L.hdr_bytes;
  L.items = align_up(L.results + n * kResultDoubles * 8);
  uint64_t p = L.items;
  for (auto *c : cs) {
    L.item_off.push_back(p);
    p = align_up(p + item_ws(c->cfg).bytes);
  }
  L.total = p;
  L.host_total = L.items;  // header + results
  return L;
}

// Builds descriptors and block maps into host staging `host` for a batch
// whose device base is `dev`; returns the per-(iteration, precision) tables.
std::vector<std::pair<LaunchTab, int>> build_batch(sbs_runtime *rt,
                                                   const std::vector<const Controller *> &cs,
                                                   const std::vector<const sbs_tick_input *> &ins,
                                                   const std::vector<uint32_t> &ticks,
                                                   const Layout &L, char *host, char *dev,
                                                   char *host_dev, const Tune &tn,
                                                   std::vector<double> *steps_out = nullptr) {
  const int n = (int)cs.size();
  int rmax = 1;
  for (auto *c : cs) rmax = std::max(rmax, c->cfg.iterations);
  TickDesc *hd = reinterpret_cast<TickDesc *>(host + L.desc);
  for (int i = 0; i < n; ++i) {
    uint64_t *seq = reinterpret_cast<uint64_t *>(host + L.results) + (size_t)i * kResultDoubles + RES_SEQ;
    __atomic_store_n(seq, (uint64_t)0, __ATOMIC_RELEASE);
    // the action record goes straight to pinned host memory (no copy back)
    fill_desc(rt, *cs[i], item_ws(cs[i]->cfg), dev + L.item_off[i],
              reinterpret_cast<double *>(host_dev + L.results) + (size_t)i * kResultDoubles,
              *ins[i], ticks[i], i, &hd[i]);
  }
  std::vector<std::pair<LaunchTab, int>> out;
  const uint64_t tab_bytes = align_up(((uint64_t)n + 3 * ((uint64_t)n + 1)) * 4);
  for (int r = 0; r < rmax; ++r) {
    for (int grp = 0; grp < kGroups; ++grp) {
      // one launch per (precision, parametrisation, stance-pair form, noise
      // of the stance legs only) group
      const int prec = (grp >> 3) & 1, spl = (grp >> 2) & 1, pair = (grp >> 1) & 1, sto = grp & 1;
      const uint64_t off = L.tabs + ((uint64_t)r * kGroups + grp) * tab_bytes;
      int32_t *item = reinterpret_cast<int32_t *>(host + off);
      int32_t *ns = item + n, *rs = ns + (n + 1), *us = rs + (n + 1);
      // longest horizon first: the rollout stage's tail is the longest lanes
      std::vector<int> idx;
      for (int i = 0; i < n; ++i)
        if (cs[i]->cfg.iterations > r && cs[i]->cfg.precision == prec &&
            (cs[i]->cfg.knots > 0 ? 1 : 0) == spl && ((tn.pairs && pair_gait(cs[i]->cfg)) ? 1 : 0) == pair &&
            (stance_noise(*cs[i], tn) ? 1 : 0) == sto)
          idx.push_back(i);
      std::stable_sort(idx.begin(), idx.end(),
                       [&](int a, int b) { return cs[a]->cfg.H > cs[b]->cfg.H; });
      int m = (int)idx.size();
      int max_h = 1;
      // four lanes per sample when the launch has few samples (latency
      // bound); one lane per sample otherwise
      long long nsum = 0;
      for (int t = 0; t < m; ++t) nsum += cs[idx[t]]->cfg.N;
      int lanes = 1, block = 64, unroll = 1;
      if (prec == SBS_FP32) {
        lanes = tn.lanes == 0 ? (nsum <= kQuadMaxSamples ? 4 : 1) : tn.lanes;
        if (valid_form(lanes, tn.block, tn.unroll)) {
          block = tn.block;
          unroll = spl ? 1 : tn.unroll;  // spline rollouts: unroll 1 only
        }
      }
      const int per_block = block / lanes;
      // elite / best-sample update workgroups cover `chunk` mean rows each
      // (MPPI items get none: their update is k_update_mppi, one workgroup
      // per controller): one row for a lone controller (its rows run side by
      // side, the latency path), more in a large batch while at least
      // kUpdTargetGroups workgroups remain (results do not depend on the
      // chunk length)
      long long rows_sel = 0;
      for (int t = 0; t < m; ++t)
        if (cs[idx[t]]->cfg.method != SBS_MPPI) rows_sel += rows_of(cs[idx[t]]->cfg);
      const int chunk = m <= 1 ? 1
                               : (int)std::max<long long>(1, std::min<long long>(kUpdMaxChunk,
                                                                                 rows_sel / kUpdTargetGroups));
      int max_rows = 1;
      ns[0] = rs[0] = us[0] = 0;
      for (int t = 0; t < m; ++t) {
        max_h = std::max(max_h, cs[idx[t]]->cfg.H);
        max_rows = std::max(max_rows, rows_of(cs[idx[t]]->cfg));
        const sbs_controller_cfg &c = cs[idx[t]]->cfg;
        item[t] = idx[t];
        ns[t + 1] = ns[t] + rows_of(c) * ((c.N + kNoiseBlock - 1) / kNoiseBlock);
        rs[t + 1] = rs[t] + (c.N + per_block - 1) / per_block;
        us[t + 1] = us[t] + (c.method != SBS_MPPI ? (rows_of(c) + chunk - 1) / chunk : 0);
      }
      if (m == 0) continue;
      LaunchTab tab{};
      tab.n = m;
      tab.r = r;
      tab.total_noise = ns[m];
      tab.total_roll = rs[m];
      tab.total_upd = us[m];
      tab.max_h = max_h;
      tab.max_rows = max_rows;
      tab.spline = spl;
      tab.lanes = lanes;
      tab.pairs = pair;
      tab.upd_chunk = chunk;
      tab.gen_noise = (tn.gen && prec == SBS_FP32 && lanes == 1 && !spl && unroll == 1) ? 1 : 0;
      if (tab.gen_noise && sto && pair && block == 256) tab.gen_noise = 2;
      tab.roll_block = block;
      tab.unroll = unroll;
      tab.r_count = 1;
      for (int t = 0; t < m; ++t) tab.n_select += cs[idx[t]]->cfg.method != SBS_MPPI ? 1 : 0;
      tab.desc = reinterpret_cast<const TickDesc *>(dev + L.desc);
      tab.item = reinterpret_cast<const int32_t *>(dev + off);
      tab.noise_start = tab.item + n;
      tab.roll_start = tab.noise_start + (n + 1);
      tab.upd_start = tab.roll_start + (n + 1);
      out.push_back({tab, prec});
      if (steps_out) {  // rollout-steps of this launch (N H per controller)
        double st = 0.0;
        for (int t = 0; t < m; ++t) st += (double)cs[idx[t]]->cfg.N * (double)cs[idx[t]]->cfg.H;
        steps_out->push_back(st);
      }
    }
  }
  return out;
}

// Timing mode of the next launch: mode 1 attaches the rollout's dispatch
// events to one launch in kTimingStride (attaching them costs the tick about
// as much as the kernel's own launch), mode 3 to every launch; mode 2 puts
// event commands around every stage of every launch.
constexpr uint64_t kTimingStride = 16;
int timing_mode_now(sbs_runtime *rt) {
  if (rt->timing == 3) return 1;  // dispatch events on every launch
  if (rt->timing != 1) return rt->timing;
  return (rt->timing_seq++ % kTimingStride) == 0 ? 1 : 0;
}

void record_timing(sbs_runtime *rt, Batch &b) {
  // mode 2: groups of 5 events around the 4 stages; mode 1: pairs around the
  // rollout stage
  const size_t g = rt->timing == 2 ? 5 : 2;  // modes 1 and 3: rollout pairs
  for (size_t o = 0; o + g <= b.timing.size(); o += g) {
    for (size_t s = 0; s + 1 < g; ++s) {
      float ms = 0.f;
      const int stage = g == 5 ? (int)s : 1;
      if (hipEventElapsedTime(&ms, b.timing[o + s], b.timing[o + s + 1]) == hipSuccess) {
        rt->stage_ns[stage] += (double)ms * 1e6;
        rt->stage_n[stage] += 1;
        const size_t p = o / g;
        if (g == 2 && p < b.timing_work.size()) {
          const int f = b.timing_work[p].first;
          rt->form_ns[f] += (double)ms * 1e6;
          rt->form_steps[f] += b.timing_work[p].second;
          rt->form_n[f] += 1;
        }
      }
    }
  }
  for (auto e : b.timing) give_timing_event(rt, e);
  b.timing.clear();
  b.timing_work.clear();
}

// Complete a finished batch: copy the actions into the tickets, free memory.
void finish_batch(sbs_runtime *rt, Batch &b) {
  const int64_t t = now_ns();
  for (size_t i = 0; i < b.tickets.size(); ++i) {
    auto it = rt->tickets.find(b.tickets[i]);
    if (it != rt->tickets.end() && it->second.status == 1) {
      std::memcpy(it->second.res, b.host_results + i * kResultDoubles, sizeof(it->second.res));
      it->second.status = 0;
      it->second.t_done = t;
      rt->n_ticks += 1;
    }
    if (it != rt->tickets.end()) it->second.rec = nullptr;  // the record is released below
    auto c = rt->ctrls.find(b.ctrls[i]);
    if (c != rt->ctrls.end()) c->second.inflight -= 1;
  }
  if (rt->timing) record_timing(rt, b);
  else {
    for (auto e : b.timing) give_timing_event(rt, e);
    b.timing.clear();
  }
  if (b.owns_memory) rt->dev_alloc.release(b.ws_off, b.ws_bytes);
  if (b.owns_host) rt->host_alloc.release(b.host_off, b.host_bytes);
  if (b.plan >= 0) {
    auto p = rt->plans.find(b.plan);
    if (p != rt->plans.end()) p->second->busy = false;
  }
  give_event(rt, b.done);
  give_event(rt, b.hdr);
  b.done = nullptr;
  b.hdr = nullptr;
}

// Retire completed batches in launch order per stream.  Returns the number
// retired.  Caller holds rt->mu.
int reap(sbs_runtime *rt) {
  int n = 0;
  for (auto it = rt->inflight.begin(); it != rt->inflight.end();) {
    hipError_t q = hipEventQuery((*it)->done);
    if (q == hipSuccess) {
      const int64_t t = now_ns();
      Batch &b = **it;
      // the device rate of large batches, and the start of the batch queued
      // behind this one on its stream
      const double dur = (double)(t - b.t_start_est);
      if (b.steps >= kJitMinSteps && dur > 0) {
        const double r = b.steps / dur;
        rt->jit_rate = rt->jit_rate > 0 ? 0.8 * rt->jit_rate + 0.2 * r : r;
      }
      for (auto nx = std::next(it); nx != rt->inflight.end(); ++nx)
        if ((*nx)->stream_slot == b.stream_slot) {
          (*nx)->t_start_est = t;
          break;
        }
      finish_batch(rt, b);
      it = rt->inflight.erase(it);
      ++n;
    } else {
      if (q != hipErrorNotReady) {
        (void)hipGetLastError();
      }
      ++it;
    }
  }
  return n;
}

// Launch one batch of (controller, input) pairs on stream slot `slot`.
// Caller holds rt->mu; returns SBS_ENOMEM when memory is short.
// With `scratch_dev` the step workspace is that device buffer (of
// kScratchBytes) instead of arena memory.
int launch(sbs_runtime *rt, const std::vector<int32_t> &ids,
           const std::vector<const sbs_tick_input *> &ins, const std::vector<uint64_t> &tks,
           int slot, char *scratch_dev = nullptr) {
  std::vector<const Controller *> cs;
  for (int32_t id : ids) cs.push_back(&rt->ctrls.at(id));
  Layout L = make_layout(cs);
  uint64_t ws_off = 0, host_off = 0;
  if (scratch_dev) {
    if (L.total > kScratchBytes)
      return fail(SBS_EINVAL, "step workspace of %llu bytes exceeds the %llu-byte scratch",
                  (unsigned long long)L.total, (unsigned long long)kScratchBytes);
  } else if (!rt->dev_alloc.alloc(L.total, &ws_off)) {
    return fail(SBS_ENOMEM, "arena cannot hold %llu bytes of step workspace",
                (unsigned long long)L.total);
  }
  if (!rt->host_alloc.alloc(L.host_total, &host_off)) {
    if (!scratch_dev) rt->dev_alloc.release(ws_off, L.total);
    return fail(SBS_ENOMEM, "pinned staging exhausted");
  }
  char *dev = scratch_dev ? scratch_dev : rt->arena + ws_off;
  char *host = rt->pinned + host_off;
  std::vector<uint32_t> ticks;
  for (int32_t id : ids) ticks.push_back(rt->ctrls.at(id).next_tick);
  std::vector<double> tab_steps;
  auto tabs = build_batch(rt, cs, ins, ticks, L, host, dev, rt->pinned_dev + host_off, rt->tune,
                          &tab_steps);
  hipStream_t s = rt->streams[slot];
  auto b = std::make_unique<Batch>();
  b->id = rt->next_batch++;
  b->stream_slot = slot;
  b->ws_off = ws_off;
  b->ws_bytes = L.total;
  b->owns_memory = scratch_dev == nullptr;
  b->host_off = host_off;
  b->host_bytes = L.host_total;
  b->host_results = reinterpret_cast<double *>(host + L.results);
  b->tickets = tks;
  b->ctrls = ids;
  b->done = take_event(rt);
  for (const Controller *c : cs) b->steps += (double)c->cfg.N * c->cfg.H * c->cfg.iterations;
  {
    // device start: behind the last batch in flight on this stream, if any
    int64_t start = now_ns() + kDispatchNs;
    for (auto &ob : rt->inflight)
      if (ob->stream_slot == slot && rt->jit_rate > 0)
        start = std::max(start, ob->t_start_est + (int64_t)(ob->steps / rt->jit_rate));
    b->t_start_est = start;
  }
  // a single controller's descriptor travels in the kernel arguments; a
  // batch's descriptors and block maps go up in one copy, on the copy stream
  // when there is one (it need not wait for the work ahead on the stream)
  TickDesc *inl = ids.size() == 1 ? reinterpret_cast<TickDesc *>(host + L.desc) : nullptr;
  hipError_t e = hipSuccess;
  // the copy stream pays off only while the work ahead on this stream runs
  // for a while yet; behind an idle or nearly done stream the copy goes on
  // the stream itself, which saves the wait across queues
  bool ahead = false;
  for (auto &ob : rt->inflight)
    if (!ahead && ob->stream_slot == slot && hipEventQuery(ob->done) != hipSuccess)
      ahead = rt->jit_rate <= 0 ||
              ob->t_start_est + (int64_t)(ob->steps / rt->jit_rate) > now_ns() + kHdrAheadNs;
  (void)hipGetLastError();  // the queries' not-ready status
  if (!inl && rt->copy_stream && ahead) {
    b->hdr = take_event(rt);
    e = hipMemcpyAsync(dev, host, L.hdr_bytes, hipMemcpyHostToDevice, rt->copy_stream);
    if (e == hipSuccess) e = hipEventRecord(b->hdr, rt->copy_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->hdr, 0);
  } else if (!inl) {
    e = hipMemcpyAsync(dev, host, L.hdr_bytes, hipMemcpyHostToDevice, s);
  }
  // noise prefetch (single controller, direct mode): read this tick's noise
  // from the buffer the previous submission filled ahead of time
  Controller *pc = nullptr;
  int pbuf = 0;
  if (inl && rt->mode == SBS_MODE_DIRECT && slot == 0 && rt->streams[1] && !scratch_dev) {
    Controller &C0 = rt->ctrls.at(ids[0]);
    if (C0.prefetch) {
      pc = &C0;
      pbuf = (int)(ticks[0] & 1u);
      inl->z = C0.pf_z[pbuf];
      inl->z_iter_stride = (uint64_t)rows_of(C0.cfg) * C0.cfg.N * 12;
      if (C0.pf_tick[pbuf] == (int64_t)ticks[0]) {
        e = hipStreamWaitEvent(s, C0.pf_ready[pbuf], 0);
        for (auto &tp : tabs) {
          tp.first.skip_noise = 1;
          tp.first.gen_noise = 0;  // the noise is there already
        }
      }
    }
  }
  const int64_t t_launch = now_ns();
  const int tmode = timing_mode_now(rt);
  // the next tick's noise goes into the other buffer on the second stream,
  // after the tick that last read it.  With several iterations per tick the
  // host enqueues it right after the first rollout, so that it runs beside
  // that rollout rather than beside the later iterations' select and update
  // stages; with one iteration it is enqueued after the tick, so that the
  // rollout runs alone and the noise overlaps the short update and the
  // host's turnaround (both orders measured on the MI355X: each is the
  // faster one for its case).
  std::function<hipError_t()> prefetch_next;
  if (pc) {
    prefetch_next = [&, pc, pbuf]() -> hipError_t {
      hipStream_t s2 = rt->streams[1];
      const int nb = pbuf ^ 1;
      TickDesc nd = *inl;
      nd.tick = ticks[0] + 1u;
      nd.z = pc->pf_z[nb];
      LaunchTab nt = tabs[0].first;
      nt.r = 0;
      nt.r_count = pc->cfg.iterations;
      nt.skip_noise = 0;
      nt.write_q = 0;
      // fewer, longer noise waves: each thread makes kPrefetchRows rows
      const int rows = rows_of(pc->cfg), nkb = (pc->cfg.N + kNoiseBlock - 1) / kNoiseBlock;
      nt.noise_rpt = kPrefetchRows;
      nt.total_noise = ((rows + kPrefetchRows - 1) / kPrefetchRows) * nkb;
      hipError_t pe = hipStreamWaitEvent(s2, pc->pf_free[nb], 0);
      if (pe == hipSuccess) pe = launch_noise_only(nt, s2, &nd);
      if (pe == hipSuccess) pe = hipEventRecord(pc->pf_ready[nb], s2);
      if (pe == hipSuccess) pc->pf_tick[nb] = (int64_t)ticks[0] + 1;
      return pe;
    };
  }
  bool first = true;
  for (size_t ti = 0; ti < tabs.size(); ++ti) {
    auto &tp = tabs[ti];
    if (e != hipSuccess) break;
    hipEvent_t *ev = nullptr;
    if (tmode) {
      size_t base = b->timing.size();
      const int ne = tmode == 2 ? 5 : 2;
      for (int i = 0; i < ne; ++i) b->timing.push_back(take_timing_event(rt));
      ev = &b->timing[base];
      if (tmode == 1) b->timing_work.push_back({roll_form(tp.first, tp.second), tab_steps[ti]});
    }
    const bool early = first && pc && pc->cfg.iterations > 1;
    e = launch_iteration(tp.first, tp.second, s, tmode, ev, inl, early ? &prefetch_next : nullptr);
    first = false;
  }
  if (e == hipSuccess) e = hipEventRecord(b->done, s);
  // the buffer this tick read is free once the whole tick is done
  if (pc && e == hipSuccess) e = hipEventRecord(pc->pf_free[pbuf], s);
  if (pc && pc->cfg.iterations == 1 && e == hipSuccess) e = prefetch_next();
  if (e != hipSuccess) {
    // the streams may still run what was enqueued: wait before freeing
    (void)hipStreamSynchronize(s);
    if (rt->copy_stream) (void)hipStreamSynchronize(rt->copy_stream);
    if (!scratch_dev) rt->dev_alloc.release(ws_off, L.total);
    rt->host_alloc.release(host_off, L.host_total);
    give_event(rt, b->done);
    give_event(rt, b->hdr);
    for (auto ev : b->timing) give_timing_event(rt, ev);
    return fail(SBS_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  }
  for (size_t i = 0; i < ids.size(); ++i) {
    Controller &c = rt->ctrls.at(ids[i]);
    c.next_tick += 1;
    c.inflight += 1;
    c.par = (c.par + c.cfg.iterations) & 1;
    c.needs_shift = true;
    TicketRec &t = rt->tickets[tks[i]];
    t.t_launch = t_launch;
    t.tick = ticks[i];
    t.rec = b->host_results + i * kResultDoubles;
  }
  rt->n_batches += 1;
  rt->inflight.push_back(std::move(b));
  return SBS_OK;
}

int slot_busy(sbs_runtime *rt, int slot) {
  int n = 0;
  for (auto &b : rt->inflight)
    if (b->stream_slot == slot) ++n;
  return n;
}

// Arena bytes that step workspaces can ever use: everything but the
// persistent allocations (controller states, debug and prefetch buffers,
// plan workspaces), i.e. the free bytes plus those of the batches in flight.
uint64_t workspace_room(const sbs_runtime *rt) {
  uint64_t transient = 0;
  for (auto &b : rt->inflight)
    if (b->owns_memory) transient += align_up(b->ws_bytes);
  return rt->dev_alloc.size() - (rt->dev_alloc.used() - transient);
}

// Ends a pending request's ticket with an error status.
void fail_request(sbs_runtime *rt, size_t i, int status) {
  rt->tickets[rt->pending[i].ticket].status = status;
  rt->pending.erase(rt->pending.begin() + i);
  rt->cv.notify_all();
}

// Scheduler poll interval when nothing can be launched: the delay between a
// batch's completion and the launch of the next one on its stream.
constexpr int kSchedPollUs = 5;

// Serving scheduler: continuous batching with memory admission.  Progress:
// with no batch in flight the arena holds only persistent state, so a head
// request that cannot be placed then can never be; its ticket fails with
// SBS_ENOMEM instead of blocking every later request.
void scheduler_loop(sbs_runtime *rt) {
  (void)hipSetDevice(rt->device);
  // Linux lengthens a thread's sleeps by its timer slack (50 us by default),
  // ten times the poll interval: 1 us keeps the polls close to kSchedPollUs
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  std::unique_lock<std::mutex> lk(rt->mu);
  while (!rt->stop.load()) {
    int retired = reap(rt);
    if (retired) rt->cv.notify_all();
    // a stream with room for another batch (the least busy one)?
    int slot = -1;
    for (int s = 0, least = rt->slot_depth; s < rt->nstreams; ++s) {
      const int busy = slot_busy(rt, s);
      if (busy < least) {
        least = busy;
        slot = s;
      }
    }
    if (slot >= 0 && rt->slot_depth > 1 && rt->jit_rate > 0) {
      // several batches per stream: hold the next one back while the work
      // ahead of it on the stream keeps the device busy for longer than the
      // margin
      int64_t end = 0;
      for (auto &ob : rt->inflight)
        if (ob->stream_slot == slot)
          end = std::max(end, ob->t_start_est + (int64_t)(ob->steps / rt->jit_rate));
      if (end > 0 && now_ns() < end - kJitMarginNs) slot = -1;
    }
    if (slot >= 0 && !rt->pending.empty()) {
      // admit in arrival order: one tick per controller per batch, skip
      // controllers with a tick in flight (their next tick needs the warm
      // start), stop when the arena cannot hold the workspace
      std::vector<int32_t> ids;
      std::vector<const sbs_tick_input *> ins;
      std::vector<uint64_t> tks;
      std::vector<size_t> taken;
      std::unordered_map<int32_t, bool> seen;
      uint64_t avail = rt->dev_alloc.size() - rt->dev_alloc.used();
      bool waited = false;
      // the batch's workspace grows by one item at a time: header and
      // records from the count, plus the sum of the item workspaces
      uint64_t items_bytes = 0;
      int rmax = 1;
      for (size_t i = 0; i < rt->pending.size() && ids.size() < 1024; ++i) {
        Request &rq = rt->pending[i];
        if (seen.count(rq.id)) continue;
        seen[rq.id] = true;
        auto cit = rt->ctrls.find(rq.id);
        if (cit == rt->ctrls.end()) continue;
        if (cit->second.inflight > 0) continue;
        const uint64_t ib = align_up(item_ws(cit->second.cfg).bytes);
        const int rm = std::max(rmax, cit->second.cfg.iterations);
        const uint64_t total = layout_items_offset(ids.size() + 1, rm) + items_bytes + ib;
        if (total + kAlign > avail) {
          waited = true;
          break;
        }
        items_bytes += ib;
        rmax = rm;
        ids.push_back(rq.id);
        ins.push_back(&rq.in);
        tks.push_back(rq.ticket);
        taken.push_back(i);
      }
      if (waited) rt->n_admit_waits += 1;
      if (ids.empty() && waited && rt->inflight.empty()) {
        // the first admissible request does not fit beside the persistent
        // state alone: it never will
        for (size_t i = 0; i < rt->pending.size(); ++i) {
          auto cit = rt->ctrls.find(rt->pending[i].id);
          if (cit == rt->ctrls.end() || cit->second.inflight > 0) continue;
          (void)fail(SBS_ENOMEM, "controller %d: step workspace does not fit in the arena",
                     rt->pending[i].id);
          fail_request(rt, i, SBS_ENOMEM);
          break;
        }
        continue;
      }
      if (!ids.empty()) {
        int rc = launch(rt, ids, ins, tks, slot);
        if (rc == SBS_ENOMEM && rt->inflight.empty() && ids.size() > 1) {
          // fragmented arena with nothing to retire: the head request alone
          ids.resize(1);
          ins.resize(1);
          tks.resize(1);
          taken.resize(1);
          rc = launch(rt, ids, ins, tks, slot);
        }
        if (rc == SBS_OK) {
          for (size_t t = taken.size(); t-- > 0;) rt->pending.erase(rt->pending.begin() + taken[t]);
          continue;
        }
        if (rc != SBS_ENOMEM || rt->inflight.empty()) {
          for (uint64_t tk : tks) rt->tickets[tk].status = rc;
          for (size_t t = taken.size(); t-- > 0;) rt->pending.erase(rt->pending.begin() + taken[t]);
          rt->cv.notify_all();
          continue;
        }
        // fragmented arena: wait for a batch to retire
        rt->n_admit_waits += 1;
      }
    }
    // nothing to launch: poll briefly (completion detection latency)
    lk.unlock();
    std::this_thread::sleep_for(std::chrono::microseconds(kSchedPollUs));
    lk.lock();
  }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *sbs_last_error(void) { return g_err.c_str(); }
int32_t sbs_abi_version(void) { return SBS_ABI_VERSION; }

int sbs_runtime_create(void *arena, uint64_t arena_bytes, void *stream, void *stream2,
                       int32_t mode, sbs_runtime **out) {
  if (!out) return fail(SBS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!arena || arena_bytes < (1u << 20)) return fail(SBS_EINVAL, "arena missing or below 1 MiB");
  if (((uintptr_t)arena) % kAlign) return fail(SBS_EINVAL, "arena must be 256-byte aligned");
  if (mode != SBS_MODE_DIRECT && mode != SBS_MODE_SERVING) return fail(SBS_EINVAL, "bad mode");
  auto rt = std::make_unique<sbs_runtime>();
  if (hipGetDevice(&rt->device) != hipSuccess) return fail(SBS_EDEVICE, "no HIP device");
  rt->arena = static_cast<char *>(arena);
  rt->dev_alloc.reset(arena_bytes);
  {
    const int rc = scratch_address(rt->device, &rt->scratch);
    if (rc != SBS_OK) return rc;
  }
  const uint64_t pinned_bytes = 64ull << 20;
  // coherent (fine-grained) so that kernels can write action records into it
  if (hipHostMalloc((void **)&rt->pinned, pinned_bytes,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return fail(SBS_EDEVICE, "hipHostMalloc of %llu bytes failed", (unsigned long long)pinned_bytes);
  if (hipHostGetDevicePointer((void **)&rt->pinned_dev, rt->pinned, 0) != hipSuccess) {
    (void)hipHostFree(rt->pinned);
    return fail(SBS_EDEVICE, "hipHostGetDevicePointer failed");
  }
  rt->host_alloc.reset(pinned_bytes);
  rt->streams[0] = static_cast<hipStream_t>(stream);
  rt->streams[1] = static_cast<hipStream_t>(stream2);
  rt->nstreams = stream2 ? 2 : 1;
  rt->mode = mode;
  if (hipStreamCreateWithFlags(&rt->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipHostFree(rt->pinned);
    return fail(SBS_EDEVICE, "copy stream creation failed");
  }
  if (mode == SBS_MODE_SERVING) {
    sbs_runtime *raw = rt.get();
    rt->sched = std::thread([raw] { scheduler_loop(raw); });
  }
  *out = rt.release();
  return SBS_OK;
}

int sbs_runtime_destroy(sbs_runtime *rt) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  if (rt->sched.joinable()) {
    rt->stop.store(true);
    rt->sched.join();
  }
  for (int s = 0; s < rt->nstreams; ++s) (void)hipStreamSynchronize(rt->streams[s]);
  if (rt->copy_stream) (void)hipStreamSynchronize(rt->copy_stream);
  {
    std::lock_guard<std::mutex> lk(rt->mu);
    reap(rt);
    for (auto &p : rt->plans) {
      if (p.second->exec) (void)hipGraphExecDestroy(p.second->exec);
      if (p.second->graph) (void)hipGraphDestroy(p.second->graph);
      if (p.second->done) (void)hipEventDestroy(p.second->done);
    }
    for (auto e : rt->event_pool) (void)hipEventDestroy(e);
    for (auto e : rt->timing_pool) (void)hipEventDestroy(e);
  }
  if (rt->copy_stream) (void)hipStreamDestroy(rt->copy_stream);
  (void)hipHostFree(rt->pinned);
  delete rt;
  return SBS_OK;
}

int sbs_init_controller(sbs_runtime *rt, const sbs_controller_cfg *cfg, int32_t *id) {
  if (!rt || !cfg || !id) return fail(SBS_EINVAL, "NULL argument");
  int rc = validate_cfg(*cfg);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(rt->mu);
  Controller C;
  C.cfg = *cfg;
  const uint64_t ts = cfg->precision == SBS_FP64 ? 8 : 4;
  const int M = rows_of(*cfg);
  C.mu_bytes = align_up((uint64_t)M * 12 * ts);
  // spline tables after the frequency mean: sp_w [H][4], sh_w [M][4] (FP64),
  // sp_b [H], sh_b [M] (int32)
  const uint64_t sp_off = 2 * C.mu_bytes + kAlign;
  const uint64_t sh_off = align_up(sp_off + (uint64_t)cfg->H * 4 * 8);
  const uint64_t spb_off = align_up(sh_off + (uint64_t)M * 4 * 8);
  const uint64_t shb_off = align_up(spb_off + (uint64_t)cfg->H * 4);
  C.st_bytes = cfg->knots > 0 ? align_up(shb_off + (uint64_t)M * 4) : sp_off;
  if (!rt->dev_alloc.alloc(C.st_bytes, &C.st_off)) {
    reap(rt);
    if (!rt->dev_alloc.alloc(C.st_bytes, &C.st_off))
      return fail(SBS_ENOMEM, "arena cannot hold the controller state");
  }
  char *base = rt->arena + C.st_off;
  C.mu_buf[0] = base;
  C.mu_buf[1] = base + C.mu_bytes;
  C.ctl = reinterpret_cast<double *>(base + 2 * C.mu_bytes);
  // hover mean: (0, 0, m g / 2) on every leg and row
  std::vector<char> hostbuf(C.st_bytes, 0);
  const double hover = 0.5 * cfg->mass * cfg->gravity;
  if (cfg->knots > 0) {
    const int P = cfg->knots;
    double *spw = reinterpret_cast<double *>(hostbuf.data() + sp_off);
    double *shw = reinterpret_cast<double *>(hostbuf.data() + sh_off);
    int32_t *spb = reinterpret_cast<int32_t *>(hostbuf.data() + spb_off);
    int32_t *shb = reinterpret_cast<int32_t *>(hostbuf.data() + shb_off);
    // step j (t_j = j dt) lies on segment floor(j (P - 1) / (H - 1)): exact
    // in integers, whereas comparing j dt with the rounded knot times can
    // put a step that sits on a knot into the segment before it.  With
    // P <= H the segment, and so the window base, moves on by at most one
    // knot per step.
    for (int j = 0; j < cfg->H; ++j) {
      const int seg = cfg->H > 1 ? (int)(((int64_t)j * (P - 1)) / (cfg->H - 1)) : 0;
      const SplineRow r = spline_row(P, cfg->H, cfg->dt, (double)j * cfg->dt, seg);
      spb[j] = r.base;
      for (int i = 0; i < 4; ++i) spw[4 * j + i] = r.w[i];
    }
    // shifted mean: knot p < P - 1 takes the spline one step later; the
    // last knot is hover (its row of the table is unused)
    C.h_sh_w.assign((size_t)4 * P, 0.0);
    C.h_sh_b.assign((size_t)P, 0);
    for (int p = 0; p + 1 < P; ++p) {
      const double tp = (double)p * ((double)(cfg->H - 1) * cfg->dt) / (double)(P - 1);
      const SplineRow r = spline_row(P, cfg->H, cfg->dt, tp + cfg->dt);
      C.h_sh_b[p] = r.base;
      for (int i = 0; i < 4; ++i) C.h_sh_w[4 * p + i] = r.w[i];
    }
    std::memcpy(shw, C.h_sh_w.data(), sizeof(double) * 4 * P);
    std::memcpy(shb, C.h_sh_b.data(), sizeof(int32_t) * P);
    C.sp_w = reinterpret_cast<const double *>(base + sp_off);
    C.sh_w = reinterpret_cast<const double *>(base + sh_off);
    C.sp_b = reinterpret_cast<const int32_t *>(base + spb_off);
    C.sh_b = reinterpret_cast<const int32_t *>(base + shb_off);
  }
  for (int j = 0; j < M; ++j)
    for (int c = 0; c < 12; ++c) {
      const double v = (c % 3 == 2) ? hover : 0.0;
      if (ts == 8) reinterpret_cast<double *>(hostbuf.data())[j * 12 + c] = v;
      else reinterpret_cast<float *>(hostbuf.data())[j * 12 + c] = (float)v;
    }
  *reinterpret_cast<double *>(hostbuf.data() + 2 * C.mu_bytes) = cfg->mu_f0;
  hipStream_t s = rt->streams[0];
  if (hipMemcpyAsync(base, hostbuf.data(), C.st_bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    rt->dev_alloc.release(C.st_off, C.st_bytes);
    return fail(SBS_EDEVICE, "controller state upload failed");
  }
  C.id = rt->next_id++;
  *id = C.id;
  rt->ctrls[C.id] = C;
  return SBS_OK;
}

int sbs_destroy_controller(sbs_runtime *rt, int32_t id) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::unique_lock<std::mutex> lk(rt->mu);
  auto it = rt->ctrls.find(id);
  if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "unknown controller %d", id);
  if (it->second.plan >= 0) return fail(SBS_EINVAL, "controller %d belongs to plan %d", id, it->second.plan);
  // cancel queued requests
  for (auto r = rt->pending.begin(); r != rt->pending.end();) {
    if (r->id == id) {
      rt->tickets[r->ticket].status = SBS_ECANCELED;
      r = rt->pending.erase(r);
    } else {
      ++r;
    }
  }
  while (it->second.inflight > 0) {
    reap(rt);
    if (it->second.inflight > 0) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      lk.lock();
      it = rt->ctrls.find(id);
    }
  }
  rt->dev_alloc.release(it->second.st_off, it->second.st_bytes);
  if (it->second.dbg_bytes) rt->dev_alloc.release(it->second.dbg_off, it->second.dbg_bytes);
  if (it->second.prefetch) {
    (void)hipStreamSynchronize(rt->streams[1]);
    for (int i = 0; i < 2; ++i) {
      (void)hipEventDestroy(it->second.pf_ready[i]);
      (void)hipEventDestroy(it->second.pf_free[i]);
    }
    rt->dev_alloc.release(it->second.pf_off, it->second.pf_bytes);
  }
  rt->ctrls.erase(it);
  rt->cv.notify_all();
  return SBS_OK;
}

static int check_input(const sbs_tick_input *in) {
  if (!in) return fail(SBS_EINVAL, "input is NULL");
  if (!finite_vec(in->x0, 12) || !finite_vec(in->foot_pos, 12) || !finite_vec(in->p_ref0, 3) ||
      !finite_vec(in->v_ref, 3) || !std::isfinite(in->yaw_ref))
    return fail(SBS_EINVAL, "non-finite tick input");
  return SBS_OK;
}

int sbs_submit_batch(sbs_runtime *rt, int32_t n, const int32_t *ids, const sbs_tick_input *in,
                     uint64_t *tickets) {
  if (!rt || n < 1 || !ids || !in || !tickets) return fail(SBS_EINVAL, "bad batch arguments");
  for (int i = 0; i < n; ++i) {
    int rc = check_input(&in[i]);
    if (rc) return rc;
  }
  std::lock_guard<std::mutex> lk(rt->mu);
  std::vector<int32_t> vid(ids, ids + n);
  {
    std::vector<int32_t> sorted = vid;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(SBS_EINVAL, "a batch may hold each controller once");
  }
  for (int32_t id : vid)
    if (!rt->ctrls.count(id)) return fail(SBS_EINVAL, "unknown controller %d", id);
  const int64_t t = now_ns();
  std::vector<uint64_t> tks;
  for (int i = 0; i < n; ++i) {
    uint64_t tk = rt->next_ticket++;
    TicketRec rec;
    rec.controller = vid[i];
    rec.t_submit = t;
    rt->tickets[tk] = rec;
    tks.push_back(tk);
    tickets[i] = tk;
  }
  if (rt->mode == SBS_MODE_SERVING) {
    // a controller whose step workspace cannot fit beside the persistent
    // state would wait forever: refused here
    const uint64_t room = workspace_room(rt);
    for (int i = 0; i < n; ++i) {
      const Layout L = make_layout({&rt->ctrls.at(vid[i])});
      if (L.total + kAlign > room) {
        for (uint64_t tk : tks) rt->tickets.erase(tk);
        return fail(SBS_ENOMEM, "controller %d: step workspace of %llu bytes exceeds the %llu "
                    "bytes the arena can ever lend to steps", vid[i],
                    (unsigned long long)L.total, (unsigned long long)room);
      }
    }
    for (int i = 0; i < n; ++i) rt->pending.push_back({tks[i], vid[i], in[i], t});
    return SBS_OK;
  }
  std::vector<const sbs_tick_input *> ins;
  for (int i = 0; i < n; ++i) ins.push_back(&in[i]);
  int rc = launch(rt, vid, ins, tks, 0);
  if (rc == SBS_ENOMEM) {
    reap(rt);
    rc = launch(rt, vid, ins, tks, 0);
  }
  if (rc != SBS_OK) {
    for (uint64_t tk : tks) rt->tickets.erase(tk);
    return rc;
  }
  return SBS_OK;
}

int sbs_submit_tick(sbs_runtime *rt, int32_t id, const sbs_tick_input *in, uint64_t *ticket) {
  return sbs_submit_batch(rt, 1, &id, in, ticket);
}

int sbs_submit_tick_noalloc(sbs_runtime *rt, int32_t id, const sbs_tick_input *in,
                            uint64_t *ticket) {
  if (!rt || !ticket) return fail(SBS_EINVAL, "runtime or ticket is NULL");
  int rc = check_input(in);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(rt->mu);
  if (rt->mode != SBS_MODE_DIRECT) return fail(SBS_EINVAL, "sbs_submit_tick_noalloc needs direct mode");
  auto it = rt->ctrls.find(id);
  if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "unknown controller %d", id);
  if (!rt->scratch) return fail(SBS_EDEVICE, "no scratch address for device %d", rt->device);
  const Layout L = make_layout({&it->second});
  if (L.total > kScratchBytes)
    return fail(SBS_EINVAL, "controller %d: step workspace of %llu bytes exceeds the %llu-byte "
                "scratch", id, (unsigned long long)L.total, (unsigned long long)kScratchBytes);
  const uint64_t tk = rt->next_ticket++;
  TicketRec rec;
  rec.controller = id;
  rec.t_submit = now_ns();
  rt->tickets[tk] = rec;
  // every launch of this runtime goes to its first stream, in order, so a
  // tick reads the scratch only after the previous user of it has finished
  rc = launch(rt, {id}, {in}, {tk}, 0, rt->scratch);
  if (rc != SBS_OK) {
    rt->tickets.erase(tk);
    return rc;
  }
  *ticket = tk;
  return SBS_OK;
}

int sbs_fetch_ready(sbs_runtime *rt, int32_t max, uint64_t *tickets, sbs_action *out,
                    int32_t *count, int64_t timeout_us) {
  if (!rt || !tickets || !out || !count || max < 0)
    return fail(SBS_EINVAL, "bad sbs_fetch_ready arguments");
  *count = 0;
  const int64_t t0 = now_ns();
  std::unique_lock<std::mutex> lk(rt->mu);
  for (;;) {
    if (rt->mode == SBS_MODE_DIRECT) reap(rt);
    int32_t n = 0;
    for (auto it = rt->tickets.begin(); it != rt->tickets.end() && n < max;) {
      TicketRec &t = it->second;
      if (t.status == 1 && complete_from_record(t)) rt->n_ticks += 1;
      if (t.status == 0) {
        tickets[n] = it->first;
        fill_action(t, &out[n]);
        ++n;
        it = rt->tickets.erase(it);
      } else {
        ++it;  // pending, or failed: left for sbs_fetch_action to report
      }
    }
    *count = n;
    if (n > 0 || max == 0) return SBS_OK;
    // nothing ready: give the lock (and the CPU) to the scheduler before
    // returning or polling again, so that a client polling in a tight loop
    // cannot keep it from launching the work it waits for
    lk.unlock();
    std::this_thread::yield();
    if (timeout_us == 0 || (timeout_us > 0 && now_ns() - t0 > timeout_us * 1000)) return SBS_OK;
    lk.lock();
  }
}

int sbs_fetch_action(sbs_runtime *rt, uint64_t ticket, sbs_action *out, int64_t timeout_us) {
  if (!rt || !out) return fail(SBS_EINVAL, "NULL argument");
  const int64_t t0 = now_ns();
  std::unique_lock<std::mutex> lk(rt->mu);
  for (;;) {
    auto it = rt->tickets.find(ticket);
    if (it == rt->tickets.end()) return fail(SBS_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    TicketRec &t = it->second;
    if (t.status == 1) {
      if (complete_from_record(t)) rt->n_ticks += 1;  // counted once: the batch then skips it
      else if (rt->mode == SBS_MODE_DIRECT) reap(rt);
    }
    if (t.status <= 0) {
      int st = t.status;
      if (st == 0) fill_action(t, out);
      rt->tickets.erase(it);
      if (st < 0) return fail(st, "tick failed or was cancelled");
      return SBS_OK;
    }
    lk.unlock();
    std::this_thread::yield();  // see sbs_fetch_ready: a polling client yields
    if (timeout_us == 0) return fail(SBS_EAGAIN, "not ready");
    if (timeout_us > 0 && now_ns() - t0 > timeout_us * 1000) return fail(SBS_ETIMEDOUT, "timed out");
    lk.lock();
  }
}

int sbs_fetch_actions(sbs_runtime *rt, int32_t n, const uint64_t *tickets, sbs_action *out,
                      int64_t timeout_us) {
  if (!rt || n < 0 || (n > 0 && (!tickets || !out))) return fail(SBS_EINVAL, "NULL argument or n < 0");
  for (int32_t i = 0; i < n; ++i) {
    const int rc = sbs_fetch_action(rt, tickets[i], out + i, timeout_us);
    if (rc != SBS_OK) return rc;
  }
  return SBS_OK;
}

int sbs_get_state(sbs_runtime *rt, int32_t id, double *mu, double *mu_f, uint32_t *tick) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::unique_lock<std::mutex> lk(rt->mu);
  auto it = rt->ctrls.find(id);
  if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "unknown controller %d", id);
  while (it->second.inflight > 0) {
    reap(rt);
    if (it->second.inflight > 0) {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
      it = rt->ctrls.find(id);
      if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "controller destroyed");
    }
  }
  Controller &C = it->second;
  const int H = rows_of(C.cfg), n = H * 12;
  const bool f64 = C.cfg.precision == SBS_FP64;
  std::vector<char> buf((size_t)n * (f64 ? 8 : 4));
  double mf = 0;
  hipStream_t s = rt->streams[0];
  if (hipMemcpyAsync(buf.data(), C.mu_buf[C.par], buf.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&mf, C.ctl, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(SBS_EDEVICE, "state download failed");
  if (mu) {
    // the warm-started mean: shifted by one step when the stored one is
    // the previous tick's
    const double hover = 0.5 * C.cfg.mass * C.cfg.gravity;
    auto stored = [&](int i) {
      return f64 ? reinterpret_cast<double *>(buf.data())[i]
                 : (double)reinterpret_cast<float *>(buf.data())[i];
    };
    for (int i = 0; i < n; ++i) {
      const int j = i / 12, c = i % 12;
      double v;
      if (C.needs_shift && j == H - 1) {
        v = (c % 3 == 2) ? hover : 0.0;
      } else if (C.needs_shift && C.cfg.knots > 0) {
#pragma clang fp contract(off)
        // the spline one step later: the kernels' sum, in the same order
        const int b = C.h_sh_b[j];
        v = C.h_sh_w[4 * j] * stored(b * 12 + c);
        for (int t = 1; t < 4; ++t)
          if (b + t < H) v = v + C.h_sh_w[4 * j + t] * stored((b + t) * 12 + c);
      } else {
        v = stored(C.needs_shift ? i + 12 : i);
      }
      mu[i] = v;
    }
  }
  if (mu_f) *mu_f = mf;
  if (tick) *tick = C.next_tick;
  return SBS_OK;
}

int sbs_set_state(sbs_runtime *rt, int32_t id, const double *mu, double mu_f, uint32_t tick) {
  if (!rt || !mu) return fail(SBS_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(rt->mu);
  auto it = rt->ctrls.find(id);
  if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "unknown controller %d", id);
  while (it->second.inflight > 0) {
    reap(rt);
    if (it->second.inflight > 0) {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
      it = rt->ctrls.find(id);
      if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "controller destroyed");
    }
  }
  Controller &C = it->second;
  const int n = rows_of(C.cfg) * 12;
  if (!finite_vec(mu, n) || !std::isfinite(mu_f)) return fail(SBS_EINVAL, "non-finite state");
  const bool f64 = C.cfg.precision == SBS_FP64;
  std::vector<char> buf((size_t)n * (f64 ? 8 : 4));
  for (int i = 0; i < n; ++i) {
    if (f64) reinterpret_cast<double *>(buf.data())[i] = mu[i];
    else reinterpret_cast<float *>(buf.data())[i] = (float)mu[i];
  }
  hipStream_t s = rt->streams[0];
  if (hipMemcpyAsync(C.mu_buf[C.par], buf.data(), buf.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(C.ctl, &mu_f, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(SBS_EDEVICE, "state upload failed");
  C.needs_shift = false;
  C.next_tick = tick;
  C.pf_tick[0] = C.pf_tick[1] = -1;
  return SBS_OK;
}

int sbs_export_state(sbs_runtime *rt, int32_t id, double *mu, double *mu_f, uint32_t *tick) {
  return sbs_get_state(rt, id, mu, mu_f, tick);
}

int sbs_import_state(sbs_runtime *rt, int32_t id, const double *mu, double mu_f, uint32_t tick) {
  return sbs_set_state(rt, id, mu, mu_f, tick);
}

int sbs_set_debug(sbs_runtime *rt, int32_t id, int32_t enable) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::lock_guard<std::mutex> lk(rt->mu);
  auto it = rt->ctrls.find(id);
  if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "unknown controller %d", id);
  Controller &C = it->second;
  if (enable && !C.debug) {
    const uint64_t RN = (uint64_t)C.cfg.iterations * C.cfg.N;
    const uint64_t bJ = align_up(RN * 8), bq = align_up(RN * 4),
                   bm = align_up((uint64_t)rows_of(C.cfg) * 12 * 8);
    C.dbg_bytes = bJ + bq + bm;
    if (!rt->dev_alloc.alloc(C.dbg_bytes, &C.dbg_off)) {
      C.dbg_bytes = 0;
      return fail(SBS_ENOMEM, "arena cannot hold the debug buffers");
    }
    char *b = rt->arena + C.dbg_off;
    C.dbg_J = reinterpret_cast<double *>(b);
    C.dbg_q = reinterpret_cast<uint32_t *>(b + bJ);
    C.dbg_mean = reinterpret_cast<double *>(b + bJ + bq);
    C.debug = true;
  } else if (!enable && C.debug) {
    if (C.inflight > 0) return fail(SBS_EAGAIN, "controller has ticks in flight");
    rt->dev_alloc.release(C.dbg_off, C.dbg_bytes);
    C.dbg_bytes = 0;
    C.debug = false;
    C.dbg_J = nullptr;
    C.dbg_q = nullptr;
    C.dbg_mean = nullptr;
  }
  return SBS_OK;
}

int sbs_debug_fetch(sbs_runtime *rt, int32_t id, double *costs, uint32_t *q, double *mean) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::unique_lock<std::mutex> lk(rt->mu);
  auto it = rt->ctrls.find(id);
  if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "unknown controller %d", id);
  if (!it->second.debug) return fail(SBS_EINVAL, "debug is off for controller %d", id);
  while (it->second.inflight > 0) {
    reap(rt);
    if (it->second.inflight > 0) {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
      it = rt->ctrls.find(id);
      if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "controller destroyed");
    }
  }
  Controller &C = it->second;
  const uint64_t RN = (uint64_t)C.cfg.iterations * C.cfg.N;
  hipStream_t s = rt->streams[0];
  hipError_t e = hipSuccess;
  if (costs) e = hipMemcpyAsync(costs, C.dbg_J, RN * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && q) e = hipMemcpyAsync(q, C.dbg_q, RN * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && mean)
    e = hipMemcpyAsync(mean, C.dbg_mean, (size_t)rows_of(C.cfg) * 12 * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(SBS_EDEVICE, "debug download failed: %s", hipGetErrorString(e));
  return SBS_OK;
}

int sbs_debug_costs(sbs_runtime *rt, int32_t id, double *costs, uint32_t *q, double *mean) {
  return sbs_debug_fetch(rt, id, costs, q, mean);
}

int sbs_debug_noise(sbs_runtime *rt, int32_t id, uint32_t tick, uint32_t r, float *z, uint32_t *q) {
  if (!rt || !z || !q) return fail(SBS_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(rt->mu);
  auto it = rt->ctrls.find(id);
  if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "unknown controller %d", id);
  while (it->second.inflight > 0) {
    reap(rt);
    if (it->second.inflight > 0) {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
      it = rt->ctrls.find(id);
      if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "controller destroyed");
    }
  }
  Controller &C = it->second;
  std::vector<const Controller *> cs{&C};
  Layout L = make_layout(cs);
  uint64_t off = 0, hoff = 0;
  if (!rt->dev_alloc.alloc(L.total, &off)) return fail(SBS_ENOMEM, "arena cannot hold the workspace");
  if (!rt->host_alloc.alloc(L.host_total, &hoff)) {
    rt->dev_alloc.release(off, L.total);
    return fail(SBS_ENOMEM, "pinned staging exhausted");
  }
  char *dev = rt->arena + off, *host = rt->pinned + hoff;
  sbs_tick_input in{};
  std::vector<const sbs_tick_input *> ins{&in};
  std::vector<uint32_t> ticks{tick};
  auto tabs = build_batch(rt, cs, ins, ticks, L, host, dev, rt->pinned_dev + hoff, rt->tune);
  TickDesc *hd = reinterpret_cast<TickDesc *>(host);
  LaunchTab tab = tabs[0].first;
  tab.r = (int32_t)r;
  tab.write_q = 1;
  const ItemWs w = item_ws(C.cfg);
  hipStream_t s = rt->streams[0];
  const double sf = C.cfg.sigma_f;
  hipError_t e = hipMemcpyAsync(dev, host, L.hdr_bytes, hipMemcpyHostToDevice, s);
  // for r > 0 the noise stage reads the running frequency mean and std
  if (e == hipSuccess)
    e = hipMemcpyAsync(hd[0].it + IT_MUF, C.ctl, 8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hd[0].it + IT_SIGF, &sf, 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_noise_only(tab, s, nullptr);
  std::vector<float> zj((size_t)rows_of(C.cfg) * C.cfg.N * 12);
  if (e == hipSuccess)
    e = hipMemcpyAsync(zj.data(), dev + L.item_off[0] + w.z, zj.size() * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(q, dev + L.item_off[0] + w.q, (size_t)C.cfg.N * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  rt->dev_alloc.release(off, L.total);
  rt->host_alloc.release(hoff, L.host_total);
  if (e != hipSuccess) return fail(SBS_EDEVICE, "noise tap failed: %s", hipGetErrorString(e));
  const int N = C.cfg.N, H = rows_of(C.cfg);
  for (int j = 0; j < H; ++j)
    for (int k = 0; k < N; ++k)
      std::memcpy(&z[((size_t)k * H + j) * 12], &zj[((size_t)j * N + k) * 12], 48);
  return SBS_OK;
}

int sbs_set_prefetch(sbs_runtime *rt, int32_t id, int32_t enable) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::unique_lock<std::mutex> lk(rt->mu);
  auto it = rt->ctrls.find(id);
  if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "unknown controller %d", id);
  Controller &C = it->second;
  if (enable && (rt->mode != SBS_MODE_DIRECT || !rt->streams[1]))
    return fail(SBS_EINVAL, "prefetch needs a direct-mode runtime with a second stream");
  while (C.inflight > 0) {
    reap(rt);
    if (C.inflight > 0) {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    }
  }
  if (enable && !C.prefetch) {
    const uint64_t one = align_up((uint64_t)C.cfg.iterations * rows_of(C.cfg) * C.cfg.N * 12 * 4);
    C.pf_bytes = 2 * one;
    if (!rt->dev_alloc.alloc(C.pf_bytes, &C.pf_off)) {
      C.pf_bytes = 0;
      return fail(SBS_ENOMEM, "arena cannot hold the prefetch buffers");
    }
    for (int i = 0; i < 2; ++i) {
      C.pf_z[i] = reinterpret_cast<float *>(rt->arena + C.pf_off + i * one);
      C.pf_tick[i] = -1;
      if (hipEventCreateWithFlags(&C.pf_ready[i], hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&C.pf_free[i], hipEventDisableTiming) != hipSuccess)
        return fail(SBS_EDEVICE, "event creation failed");
    }
    C.prefetch = true;
  } else if (!enable && C.prefetch) {
    (void)hipStreamSynchronize(rt->streams[1]);
    for (int i = 0; i < 2; ++i) {
      (void)hipEventDestroy(C.pf_ready[i]);
      (void)hipEventDestroy(C.pf_free[i]);
      C.pf_ready[i] = C.pf_free[i] = nullptr;
      C.pf_z[i] = nullptr;
      C.pf_tick[i] = -1;
    }
    rt->dev_alloc.release(C.pf_off, C.pf_bytes);
    C.pf_bytes = 0;
    C.prefetch = false;
  }
  return SBS_OK;
}

int sbs_stats(sbs_runtime *rt, uint64_t *ticks, uint64_t *batches, uint64_t *admit_waits) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::lock_guard<std::mutex> lk(rt->mu);
  if (ticks) *ticks = rt->n_ticks;
  if (batches) *batches = rt->n_batches;
  if (admit_waits) *admit_waits = rt->n_admit_waits;
  return SBS_OK;
}

int sbs_set_timing(sbs_runtime *rt, int32_t mode) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  if (mode < 0 || mode > 3) return fail(SBS_EINVAL, "timing mode must be 0, 1, 2 or 3");
  std::lock_guard<std::mutex> lk(rt->mu);
  reap(rt);
  rt->timing = mode;
  rt->timing_seq = 0;
  return SBS_OK;
}

int sbs_set_rollout_pairs(sbs_runtime *rt, int32_t enable) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::lock_guard<std::mutex> lk(rt->mu);
  rt->tune.pairs = enable != 0;
  return SBS_OK;
}

int sbs_set_serving_depth(sbs_runtime *rt, int32_t depth) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  if (depth < 1 || depth > 4) return fail(SBS_EINVAL, "serving depth must be 1 to 4");
  std::lock_guard<std::mutex> lk(rt->mu);
  rt->slot_depth = depth;
  return SBS_OK;
}

int sbs_set_rollout_noise(sbs_runtime *rt, int32_t in_rollout) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::lock_guard<std::mutex> lk(rt->mu);
  if (in_rollout < 0 || in_rollout > 2) return fail(SBS_EINVAL, "rollout noise mode must be 0 to 2");
  rt->tune.gen = in_rollout;
  return SBS_OK;
}

int sbs_set_rollout_lanes(sbs_runtime *rt, int32_t lanes) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  if (lanes != 0 && lanes != 1 && lanes != 4) return fail(SBS_EINVAL, "lanes must be 0, 1 or 4");
  std::lock_guard<std::mutex> lk(rt->mu);
  rt->tune.lanes = lanes;
  return SBS_OK;
}

int sbs_timing(sbs_runtime *rt, double *avg_ns, uint64_t *launches) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::lock_guard<std::mutex> lk(rt->mu);
  reap(rt);
  for (int s = 0; s < 4; ++s) {
    if (avg_ns) avg_ns[s] = rt->stage_n[s] ? rt->stage_ns[s] / (double)rt->stage_n[s] : 0.0;
    if (launches) launches[s] = rt->stage_n[s];
    rt->stage_ns[s] = 0;
    rt->stage_n[s] = 0;
  }
  return SBS_OK;
}

int sbs_timing_rollout(sbs_runtime *rt, int32_t form, double *avg_ns, uint64_t *launches,
                       double *steps) {
  if (!rt || form < 0 || form >= kForms) return fail(SBS_EINVAL, "bad runtime or rollout form");
  std::lock_guard<std::mutex> lk(rt->mu);
  reap(rt);
  const uint64_t n = rt->form_n[form];
  if (avg_ns) *avg_ns = n ? rt->form_ns[form] / (double)n : 0.0;
  if (launches) *launches = n;
  if (steps) *steps = rt->form_steps[form];
  rt->form_ns[form] = 0;
  rt->form_steps[form] = 0;
  rt->form_n[form] = 0;
  return SBS_OK;
}

int sbs_timing_overhead(sbs_runtime *rt, int32_t reps, double *avg_ns) {
  if (!rt || !avg_ns) return fail(SBS_EINVAL, "runtime or output is NULL");
  if (reps < 1 || reps > 4096) return fail(SBS_EINVAL, "reps=%d out of [1, 4096]", reps);
  std::lock_guard<std::mutex> lk(rt->mu);
  reap(rt);
  hipEvent_t e0 = take_timing_event(rt), e1 = take_timing_event(rt);
  if (!e0 || !e1) {
    give_timing_event(rt, e0);
    give_timing_event(rt, e1);
    return fail(SBS_EDEVICE, "event creation failed");
  }
  double total = 0.0;
  hipError_t e = hipSuccess;
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    e = launch_empty_timed(rt->streams[0], e0, e1);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    total += (double)ms * 1e6;
  }
  give_timing_event(rt, e0);
  give_timing_event(rt, e1);
  if (e != hipSuccess) return fail(SBS_EDEVICE, "timing overhead: %s", hipGetErrorString(e));
  *avg_ns = total / reps;
  return SBS_OK;
}

// ---------------------------------------------------------------------------
// Plans: fixed membership, workspace reserved once, optionally a HIP graph.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

std::vector<const Controller *> plan_ctrls(sbs_runtime *rt, const Plan &P) {
  std::vector<const Controller *> cs;
  for (int32_t id : P.ctrls) cs.push_back(&rt->ctrls.at(id));
  return cs;
}

// Records the plan's whole tick as a HIP graph: the header copy from pinned
// staging (read at replay time, so new inputs need no re-recording), then
// every stage of every iteration.  Replaces a previous graph.
hipError_t capture_plan(sbs_runtime *rt, Plan &P) {
  if (P.exec) (void)hipGraphExecDestroy(P.exec);
  if (P.graph) (void)hipGraphDestroy(P.graph);
  P.exec = nullptr;
  P.graph = nullptr;
  const int n = (int)P.ctrls.size();
  auto cs = plan_ctrls(rt, P);
  std::vector<sbs_tick_input> dummy(n);
  for (auto &d : dummy) std::memset(&d, 0, sizeof d);
  std::vector<const sbs_tick_input *> ins;
  for (auto &d : dummy) ins.push_back(&d);
  std::vector<uint32_t> ticks(n, 0);
  auto tabs = build_batch(rt, cs, ins, ticks, P.lay, P.host, P.dev, rt->pinned_dev + P.host_off,
                          P.tune);
  hipStream_t s = rt->streams[0];
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(P.dev, P.host, P.lay.hdr_bytes, hipMemcpyHostToDevice, s);
  for (auto &tp : tabs)
    if (e == hipSuccess) e = launch_iteration(tp.first, tp.second, s, 0, nullptr, nullptr);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e == hipSuccess) e = e2;
  P.graph = g;
  if (e == hipSuccess) e = hipGraphInstantiate(&P.exec, g, nullptr, nullptr, 0);
  return e;
}

}  // namespace

extern "C" {

int sbs_plan_create(sbs_runtime *rt, int32_t n, const int32_t *ids, int32_t use_graph, int32_t *plan) {
  if (!rt || n < 1 || !ids || !plan) return fail(SBS_EINVAL, "bad plan arguments");
  std::lock_guard<std::mutex> lk(rt->mu);
  if (rt->mode != SBS_MODE_DIRECT) return fail(SBS_EINVAL, "plans need a direct-mode runtime");
  std::vector<int32_t> vid(ids, ids + n);
  std::vector<int32_t> sorted = vid;
  std::sort(sorted.begin(), sorted.end());
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
    return fail(SBS_EINVAL, "a plan may hold each controller once");
  std::vector<const Controller *> cs;
  for (int32_t id : vid) {
    auto it = rt->ctrls.find(id);
    if (it == rt->ctrls.end()) return fail(SBS_EINVAL, "unknown controller %d", id);
    if (it->second.plan >= 0) return fail(SBS_EINVAL, "controller %d already in a plan", id);
    cs.push_back(&it->second);
  }
  auto P = std::make_unique<Plan>();
  P->lay = make_layout(cs);
  if (!rt->dev_alloc.alloc(P->lay.total, &P->ws_off)) return fail(SBS_ENOMEM, "arena cannot hold the plan");
  if (!rt->host_alloc.alloc(P->lay.host_total, &P->host_off)) {
    rt->dev_alloc.release(P->ws_off, P->lay.total);
    return fail(SBS_ENOMEM, "pinned staging exhausted");
  }
  P->dev = rt->arena + P->ws_off;
  P->host = rt->pinned + P->host_off;
  P->ctrls = vid;
  P->use_graph = use_graph != 0;
  P->tune = rt->tune;
  P->id = rt->next_plan++;
  if (hipEventCreateWithFlags(&P->done, hipEventDisableTiming) != hipSuccess) {
    rt->dev_alloc.release(P->ws_off, P->lay.total);
    rt->host_alloc.release(P->host_off, P->lay.host_total);
    return fail(SBS_EDEVICE, "event creation failed");
  }
  if (P->use_graph) {
    hipError_t e = capture_plan(rt, *P);
    if (e != hipSuccess) {
      if (P->exec) (void)hipGraphExecDestroy(P->exec);
      if (P->graph) (void)hipGraphDestroy(P->graph);
      (void)hipEventDestroy(P->done);
      rt->dev_alloc.release(P->ws_off, P->lay.total);
      rt->host_alloc.release(P->host_off, P->lay.host_total);
      return fail(SBS_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
  }
  for (int32_t id : vid) rt->ctrls.at(id).plan = P->id;
  *plan = P->id;
  rt->plans[P->id] = std::move(P);
  return SBS_OK;
}

int sbs_plan_set_tune(sbs_runtime *rt, int32_t plan, const sbs_tune *t) {
  if (!rt || !t) return fail(SBS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(rt->mu);
  auto pit = rt->plans.find(plan);
  if (pit == rt->plans.end()) return fail(SBS_EINVAL, "unknown plan %d", plan);
  Plan &P = *pit->second;
  if (t->lanes != 0 && !valid_form(t->lanes, t->block, t->unroll))
    return fail(SBS_EINVAL, "unsupported rollout form (lanes %d, block %d, unroll %d)", t->lanes,
                t->block, t->unroll);
  while (P.busy) {
    reap(rt);
    if (P.busy) std::this_thread::yield();
  }
  P.tune.lanes = t->lanes;
  P.tune.block = t->block;
  P.tune.unroll = t->unroll;
  if (P.use_graph) {
    hipError_t e = capture_plan(rt, P);
    if (e != hipSuccess) return fail(SBS_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  }
  return SBS_OK;
}

int sbs_plan_autotune(sbs_runtime *rt, int32_t plan, const sbs_tick_input *in, int32_t reps,
                      sbs_tune *best) {
  if (!rt || !in || !best || reps < 1) return fail(SBS_EINVAL, "bad autotune arguments");
  std::lock_guard<std::mutex> lk(rt->mu);
  auto pit = rt->plans.find(plan);
  if (pit == rt->plans.end()) return fail(SBS_EINVAL, "unknown plan %d", plan);
  Plan &P = *pit->second;
  const int n = (int)P.ctrls.size();
  for (int i = 0; i < n; ++i) {
    int rc = check_input(&in[i]);
    if (rc) return rc;
  }
  hipStream_t s = rt->streams[0];
  while (P.busy || !rt->inflight.empty()) {
    reap(rt);
    if (P.busy || !rt->inflight.empty()) std::this_thread::yield();
  }
  auto cs = plan_ctrls(rt, P);
  // snapshot every controller's state: mean, frequency mean, tick
  uint64_t snap_bytes = 0;
  std::vector<uint64_t> mu_bytes(n);
  for (int i = 0; i < n; ++i) {
    mu_bytes[i] = cs[i]->mu_bytes;
    snap_bytes += mu_bytes[i] + kAlign;
  }
  uint64_t snap_off = 0;
  if (!rt->dev_alloc.alloc(snap_bytes, &snap_off)) return fail(SBS_ENOMEM, "arena cannot hold the snapshot");
  char *snap = rt->arena + snap_off;
  std::vector<uint32_t> ticks0(n);
  auto copy_state = [&](bool save) -> hipError_t {
    char *p = snap;
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
      const Controller &C = *cs[i];
      void *cur = C.mu_buf[C.par];  // the plan's trials never change the host parity
      e = save ? hipMemcpyAsync(p, cur, mu_bytes[i], hipMemcpyDeviceToDevice, s)
               : hipMemcpyAsync(cur, p, mu_bytes[i], hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess)
        e = save ? hipMemcpyAsync(p + mu_bytes[i], C.ctl, 8, hipMemcpyDeviceToDevice, s)
                 : hipMemcpyAsync(C.ctl, p + mu_bytes[i], 8, hipMemcpyDeviceToDevice, s);
      p += mu_bytes[i] + kAlign;
    }
    return e;
  };
  for (int i = 0; i < n; ++i) ticks0[i] = cs[i]->next_tick;
  hipError_t e = copy_state(true);
  hipEvent_t t0 = take_timing_event(rt), t1 = take_timing_event(rt);
  static const int forms[][3] = {{4, 64, 1}, {4, 128, 1}, {4, 256, 1}, {1, 64, 1},
                                 {1, 128, 1}, {1, 256, 1}, {1, 64, 2}, {1, 128, 2}};
  bool any_fp32 = false;
  for (auto *c : cs) any_fp32 |= c->cfg.precision == SBS_FP32;
  const int nforms = any_fp32 ? (int)(sizeof forms / sizeof forms[0]) : 1;
  double best_us = 1e300;
  Tune best_t = P.tune;
  std::vector<const sbs_tick_input *> ins;
  for (int i = 0; i < n; ++i) ins.push_back(&in[i]);
  for (int f = 0; f < nforms && e == hipSuccess; ++f) {
    Tune tn = P.tune;  // the plan's stance-pair and noise settings stay
    tn.lanes = forms[f][0];
    tn.block = forms[f][1];
    tn.unroll = forms[f][2];
    double total_ms = 0.0;
    for (int rep = 0; rep <= reps && e == hipSuccess; ++rep) {  // rep 0 warms up
      std::vector<uint32_t> ticks;
      for (int i = 0; i < n; ++i) ticks.push_back(ticks0[i] + (uint32_t)rep);
      auto tabs = build_batch(rt, cs, ins, ticks, P.lay, P.host, P.dev,
                              rt->pinned_dev + P.host_off, tn);
      e = hipMemcpyAsync(P.dev, P.host, P.lay.hdr_bytes, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipEventRecord(t0, s);
      for (auto &tp : tabs)
        if (e == hipSuccess) e = launch_iteration(tp.first, tp.second, s, 0, nullptr, nullptr);
      if (e == hipSuccess) e = hipEventRecord(t1, s);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (rep > 0) total_ms += ms;
      if (e == hipSuccess) e = copy_state(false);  // every trial starts from the snapshot
    }
    const double us = total_ms * 1e3 / reps;
    if (e == hipSuccess && us < best_us) {
      best_us = us;
      best_t = tn;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  give_timing_event(rt, t0);
  give_timing_event(rt, t1);
  rt->dev_alloc.release(snap_off, snap_bytes);
  if (e != hipSuccess) return fail(SBS_EDEVICE, "autotune failed: %s", hipGetErrorString(e));
  P.tune = best_t;
  if (P.use_graph) {
    e = capture_plan(rt, P);
    if (e != hipSuccess) return fail(SBS_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  }
  best->lanes = best_t.lanes;
  best->block = best_t.block;
  best->unroll = best_t.unroll;
  best->reserved = 0;
  best->tick_us = best_us;
  return SBS_OK;
}

int sbs_plan_submit(sbs_runtime *rt, int32_t plan, const sbs_tick_input *in, uint64_t *tickets) {
  if (!rt || !in || !tickets) return fail(SBS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(rt->mu);
  auto pit = rt->plans.find(plan);
  if (pit == rt->plans.end()) return fail(SBS_EINVAL, "unknown plan %d", plan);
  Plan &P = *pit->second;
  const int n = (int)P.ctrls.size();
  for (int i = 0; i < n; ++i) {
    int rc = check_input(&in[i]);
    if (rc) return rc;
  }
  if (P.busy) {
    reap(rt);
    if (P.busy) return fail(SBS_EAGAIN, "previous replay of plan %d still running", plan);
  }
  std::vector<const Controller *> cs;
  std::vector<const sbs_tick_input *> ins;
  std::vector<uint32_t> ticks;
  for (int i = 0; i < n; ++i) {
    Controller &c = rt->ctrls.at(P.ctrls[i]);
    if (c.inflight > 0) {
      reap(rt);
      if (c.inflight > 0) return fail(SBS_EAGAIN, "controller %d has a tick in flight", c.id);
    }
    cs.push_back(&c);
    ins.push_back(&in[i]);
    ticks.push_back(c.next_tick);
  }
  std::vector<double> tab_steps;
  auto tabs = build_batch(rt, cs, ins, ticks, P.lay, P.host, P.dev, rt->pinned_dev + P.host_off,
                          P.tune, &tab_steps);
  hipStream_t s = rt->streams[0];
  auto b = std::make_unique<Batch>();
  b->id = rt->next_batch++;
  b->stream_slot = 0;
  b->owns_memory = false;
  b->owns_host = false;
  b->plan = P.id;
  b->host_results = reinterpret_cast<double *>(P.host + P.lay.results);
  b->ctrls = P.ctrls;
  b->done = take_event(rt);
  const int64_t t = now_ns();
  hipError_t e = hipSuccess;
  if (P.use_graph) {
    e = hipGraphLaunch(P.exec, s);
  } else {
    e = hipMemcpyAsync(P.dev, P.host, P.lay.hdr_bytes, hipMemcpyHostToDevice, s);
    const int tmode = timing_mode_now(rt);
    for (size_t ti = 0; ti < tabs.size(); ++ti) {
      auto &tp = tabs[ti];
      if (e != hipSuccess) break;
      hipEvent_t *ev = nullptr;
      if (tmode) {
        size_t base = b->timing.size();
        const int ne = tmode == 2 ? 5 : 2;
        for (int i = 0; i < ne; ++i) b->timing.push_back(take_timing_event(rt));
        ev = &b->timing[base];
        if (tmode == 1) b->timing_work.push_back({roll_form(tp.first, tp.second), tab_steps[ti]});
      }
      e = launch_iteration(tp.first, tp.second, s, tmode, ev, nullptr);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(b->done, s);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);
    give_event(rt, b->done);
    for (auto ev : b->timing) give_timing_event(rt, ev);
    return fail(SBS_EDEVICE, "plan launch failed: %s", hipGetErrorString(e));
  }
  for (int i = 0; i < n; ++i) {
    uint64_t tk = rt->next_ticket++;
    TicketRec rec;
    rec.controller = P.ctrls[i];
    rec.t_submit = t;
    rec.t_launch = t;
    rec.tick = ticks[i];
    rec.rec = b->host_results + i * kResultDoubles;
    rt->tickets[tk] = rec;
    b->tickets.push_back(tk);
    tickets[i] = tk;
    Controller &c = rt->ctrls.at(P.ctrls[i]);
    c.next_tick += 1;
    c.inflight += 1;
    c.par = (c.par + c.cfg.iterations) & 1;
    c.needs_shift = true;
  }
  P.busy = true;
  rt->n_batches += 1;
  rt->inflight.push_back(std::move(b));
  return SBS_OK;
}

int sbs_plan_destroy(sbs_runtime *rt, int32_t plan) {
  if (!rt) return fail(SBS_EINVAL, "runtime is NULL");
  std::unique_lock<std::mutex> lk(rt->mu);
  auto pit = rt->plans.find(plan);
  if (pit == rt->plans.end()) return fail(SBS_EINVAL, "unknown plan %d", plan);
  while (pit->second->busy) {
    reap(rt);
    if (pit->second->busy) {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
      pit = rt->plans.find(plan);
    }
  }
  Plan &P = *pit->second;
  if (P.exec) (void)hipGraphExecDestroy(P.exec);
  if (P.graph) (void)hipGraphDestroy(P.graph);
  if (P.done) (void)hipEventDestroy(P.done);
  rt->dev_alloc.release(P.ws_off, P.lay.total);
  rt->host_alloc.release(P.host_off, P.lay.host_total);
  for (int32_t id : P.ctrls) {
    auto c = rt->ctrls.find(id);
    if (c != rt->ctrls.end()) c->second.plan = -1;
  }
  rt->plans.erase(pit);
  return SBS_OK;
}

}  // extern "C"
