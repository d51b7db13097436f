// Optional per-kernel timing with HIP events recorded on the launch stream.
// When enabled, every launch of a timed kernel family is bracketed by two
// events; reco_timing_read() waits for the recorded events and accumulates
// their elapsed times per family.  Disabled by default (no events recorded).
#include <atomic>

#include "internal.h"
#include "timing.h"

namespace reco {

namespace {
struct Pending {
  int kind;
  hipEvent_t a, b;
};
struct Timer {
  std::atomic<bool> on{false};
  std::mutex mu;
  std::vector<Pending> pend;
  std::vector<hipEvent_t> pool;
  double total_ms[kTimedKinds] = {};
  long long count[kTimedKinds] = {};
};
Timer& timer() {
  static Timer* t = new Timer();
  return *t;
}
hipEvent_t take_event(Timer& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_CHECK(hipEventCreate(&e));
  return e;
}
}  // namespace

bool timing_on() { return timer().on.load(std::memory_order_relaxed); }

TimedLaunch::TimedLaunch(int kind, hipStream_t st) : kind_(kind), st_(st) {
  if (!timing_on()) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  if (cs != hipStreamCaptureStatusNone) return;
  Timer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  a_ = take_event(t);
  b_ = take_event(t);
  HIP_CHECK(hipEventRecord(a_, st_));
  active_ = true;
}

TimedLaunch::~TimedLaunch() {
  if (!active_) return;
  Timer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  if (hipEventRecord(b_, st_) != hipSuccess) {
    (void)hipGetLastError();
    t.pool.push_back(a_);
    t.pool.push_back(b_);
    return;
  }
  t.pend.push_back({kind_, a_, b_});
}

void timing_enable(bool on) { timer().on.store(on); }

void timing_collect() {
  Timer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  for (const Pending& p : t.pend) {
    HIP_CHECK(hipEventSynchronize(p.b));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, p.a, p.b));
    t.total_ms[p.kind] += ms;
    t.count[p.kind] += 1;
    t.pool.push_back(p.a);
    t.pool.push_back(p.b);
  }
  t.pend.clear();
}

void timing_read(int kind, long long* launches, double* total_ms) {
  timing_collect();
  Timer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  *launches = t.count[kind];
  *total_ms = t.total_ms[kind];
}

void timing_reset() {
  timing_collect();
  Timer& t = timer();
  std::lock_guard<std::mutex> lk(t.mu);
  for (int i = 0; i < kTimedKinds; ++i) {
    t.total_ms[i] = 0.0;
    t.count[i] = 0;
  }
}

}  // namespace reco

extern "C" {
reco_status reco_timing_enable(int32_t on) {
  reco::clear_error();
  reco::timing_enable(on != 0);
  return RECO_OK;
}

reco_status reco_timing_read(int32_t kind, int64_t* launches, double* total_ms) {
  reco::clear_error();
  if (kind < 0 || kind >= reco::kTimedKinds || !launches || !total_ms) {
    reco::set_error("invalid timing query");
    return RECO_EINVAL;
  }
  try {
    long long l = 0;
    reco::timing_read(kind, &l, total_ms);
    *launches = l;
  } catch (const reco::Error& e) {
    reco::set_error(e.msg);
    return e.code;
  }
  return RECO_OK;
}

reco_status reco_timing_reset(void) {
  reco::clear_error();
  try {
    reco::timing_reset();
  } catch (const reco::Error& e) {
    reco::set_error(e.msg);
    return e.code;
  }
  return RECO_OK;
}
}
