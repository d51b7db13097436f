// Pool of reusable solver workspaces (host side, no device code).
//
// A workspace returns to the pool only if its last solve ended cleanly.  A
// solve whose reduction gave up waiting for partial sums, whose host guard
// tripped, or that threw while its kernels may still be queued can leave
// stale partials in the finisher slots or a nonzero ticket counter, which
// the next solve on that workspace would take for its own: such a workspace
// is dropped (the caller's `drop` waits for the device and frees it).
#pragma once

#include <mutex>
#include <vector>

namespace reco {

template <typename T>
class ReusePool {
 public:
  ReusePool() = default;
  ReusePool(const ReusePool&) = delete;
  ReusePool& operator=(const ReusePool&) = delete;

  // A pooled object, or nullptr when the pool is empty.
  T* take() {
    std::lock_guard<std::mutex> lk(mu_);
    if (free_.empty()) return nullptr;
    T* p = free_.back();
    free_.pop_back();
    return p;
  }

  // Pool p if `reusable`, else destroy it with drop(p).  True when pooled.
  template <typename Drop>
  bool give_back(T* p, bool reusable, Drop drop) {
    if (!p) return false;
    if (!reusable) {
      drop(p);
      return false;
    }
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(p);
    return true;
  }

  // Destroy every pooled object; returns how many there were.
  template <typename Drop>
  size_t drain(Drop drop) {
    std::vector<T*> all;
    {
      std::lock_guard<std::mutex> lk(mu_);
      all.swap(free_);
    }
    for (T* p : all) drop(p);
    return all.size();
  }

  size_t size() const {
    std::lock_guard<std::mutex> lk(mu_);
    return free_.size();
  }

 private:
  mutable std::mutex mu_;
  std::vector<T*> free_;
};

// Whether a workspace may be reused after a solve: its device state ended
// normally (done 4 means a reduction's partial sums never all arrived), no
// host guard tripped, and the solve did not end in an exception.
inline bool workspace_reusable(int done, bool guard_failed, bool unwinding) {
  return done != 4 && !guard_failed && !unwinding;
}

}  // namespace reco
