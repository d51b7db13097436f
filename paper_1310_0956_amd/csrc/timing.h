// Per-kernel-family HIP event timing (see timing.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace reco {

// Kernel families; the numbering is part of reco_timing_read's contract.
enum TimedKind {
  TK_FORWARD = 0,      // forward projector
  TK_BACKWARD = 1,     // backprojector
  TK_WMG = 2,          // WMG apply (packet transform, diagonal scaling, inverse)
  TK_UPDATE = 3,       // fused CGLS vector update
  TK_PACKET_DIAG = 4,  // packet-diagonal setup
  TK_PREP = 5,         // image padding / transposition
  TK_GRAPH = 6,        // one replay of a batched-iteration graph
  kTimedKinds = 7
};

bool timing_on();

// Records an event on `st` when constructed and another when destroyed.
// Launches made while `st` is being captured into a graph are not timed.
class TimedLaunch {
 public:
  TimedLaunch(int kind, hipStream_t st);
  ~TimedLaunch();
  TimedLaunch(const TimedLaunch&) = delete;
  TimedLaunch& operator=(const TimedLaunch&) = delete;

 private:
  int kind_;
  hipStream_t st_;
  hipEvent_t a_{}, b_{};
  bool active_ = false;
};

void timing_collect();

}  // namespace reco
