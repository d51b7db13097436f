// Many independent CGLS reconstructions advanced together.
//
// Every problem keeps its own device state, workspace and reduction scratch,
// exactly as in a solo solve; what is shared is the launch.  Each Krylov
// phase (forward projection, vector update, backprojection, WMG apply) of all
// running problems is one launch over a flat list of blocks: a per-launch
// table maps the flat block index to (problem, block of that problem's grid)
// and holds each problem's kernel arguments.  The per-problem arithmetic and
// reduction order are those of the solo kernels, so every problem's iterates
// are bitwise those of reco_solve_cgls on the same input.
//
// A "tick" advances all running problems by a fixed number of iterations.
// While the set of running problems does not change, the launches of a tick
// are captured once into a HIP graph and replayed.  After every tick the
// host gathers the problems' done flags (one small kernel and one copy);
// finished problems leave the work lists, new ones join (continuous
// batching: the server below admits requests between ticks).
#include <algorithm>
#include <condition_variable>
#include <deque>
#include <exception>
#include <map>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "device_common.h"
#include "solve.h"
#include "timing.h"

namespace reco {

// ---------------------------------------------------------------------------
// Device launch tables
// ---------------------------------------------------------------------------
constexpr size_t kTableFloor = 64;   // problems a launch table holds before it first grows

void DevTable::upload(const void* host_args, size_t arg_size, const std::vector<int>& blocks,
                      const std::vector<int>& widths, hipStream_t st) {
  const int cnt = (int)blocks.size();
  std::vector<int> idx(2 * (size_t)cnt + 1);
  long long tot = 0;
  for (int i = 0; i < cnt; ++i) {
    if (blocks[i] <= 0 || widths[i] <= 0 || blocks[i] % widths[i] != 0)
      fail(RECO_EINVAL, "internal: malformed launch table");
    idx[i] = (int)tot;
    tot += blocks[i];
    idx[cnt + 1 + i] = widths[i];
  }
  if (tot > 0x7fffffffLL) fail(RECO_EINVAL, "batched launch has too many blocks");
  idx[cnt] = (int)tot;
  const size_t abytes = arg_size * (size_t)cnt;
  const size_t ibytes = sizeof(int) * idx.size();
  // Capacity for at least kTableFloor problems, doubled when exceeded: hipFree
  // waits for the whole device (every stream), so a table that grew one
  // problem at a time stalled a server's small tier behind the other tier's
  // long kernels each time its batch reached a new size (small requests
  // finished 0.5 s late under load).
  if (abytes > args_cap) {
    const size_t cap = std::max({abytes, 2 * args_cap, arg_size * kTableFloor});
    if (args) (void)hipFree(args);
    args = nullptr;
    args_cap = 0;
    HIP_CHECK(hipMalloc(&args, cap));
    args_cap = cap;
  }
  if (ibytes > idx_cap) {
    const size_t cap = std::max({ibytes, 2 * idx_cap, sizeof(int) * (2 * kTableFloor + 2)});
    if (start) (void)hipFree(start);
    start = nullptr;
    idx_cap = 0;
    HIP_CHECK(hipMalloc((void**)&start, cap));
    idx_cap = cap;
  }
  gx = start + cnt + 1;
  count = cnt;
  total_blocks = (int)tot;
  if (cnt == 0) return;
  HIP_CHECK(hipMemcpyAsync(args, host_args, abytes, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(start, idx.data(), ibytes, hipMemcpyHostToDevice, st));
  // the host arrays are temporaries: wait until the copies have read them
  HIP_CHECK(hipStreamSynchronize(st));
}

DevTable::~DevTable() {
  if (args) (void)hipFree(args);
  if (start) (void)hipFree(start);
}

namespace {

struct Flag {
  int done, iter;
};

__global__ void k_gather_flags(const SolverState* const* __restrict__ sts, int count,
                               Flag* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    const SolverState* s = sts[i];
    out[i] = Flag{s->done, s->iter};
  }
}

// One running problem.
struct Slot {
  Geometry* g = nullptr;
  Workspace* w = nullptr;
  const void* b = nullptr;
  void* x = nullptr;
  reco_solve_opts o{};
  int limit = 0;        // iteration cap on the device (max_iter or fixed_iters)
  int ticks = 0;        // ticks run while in the work lists
  SolverState fin{};    // device state copied back when finished
  double t_admit = 0.0, t_done = 0.0;
  bool failed = false;  // host-side guard tripped
  void* owner = nullptr;
};

class Engine {
 public:
  // own_stream: st is used by this engine only (its graphs are captured on
  // it); otherwise a capture stream of its own is created.  Every stream a
  // process uses beyond the device's hardware queues shares a queue with
  // another and then waits behind that stream's work.
  Engine(hipStream_t st, int iters_per_tick, bool use_graph, bool own_stream = false)
      : st_(st), iters_(iters_per_tick), use_graph_(use_graph) {
    if (own_stream) cap_ = st_;
    else HIP_CHECK(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
  }
  ~Engine() {
    drop_graph();
    if (d_sts_) (void)hipFree(d_sts_);
    if (d_flags_) (void)hipFree(d_flags_);
    if (h_flags_) (void)hipHostFree(h_flags_);
    if (cap_ && cap_ != st_) (void)hipStreamDestroy(cap_);
  }
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  bool empty() const { return active_.empty(); }
  size_t running() const { return active_.size(); }

  // Initialise new problems (state, x = 0, r = b, s = W^T b, z = M^-1 s) and
  // add them to the work lists from the next tick on.
  void add(const std::vector<Slot*>& slots) {
    if (slots.empty()) return;
    std::vector<const Geometry*> gs, gw;
    std::vector<InitArgs> ia;
    std::vector<BwdArgs> ba;
    std::vector<WmgArgs> wa;
    for (Slot* s : slots) {
      Workspace& w = *s->w;
      const bool fixed = s->o.fixed_iters > 0;
      s->limit = fixed ? s->o.fixed_iters : s->o.max_iter;
      ensure_history(w, s->limit);
      gs.push_back(s->g);
      InitArgs i{};
      i.x = s->x;
      i.p = w.p;
      i.q = w.q;
      i.r = w.r;
      i.b = s->b;
      i.st = w.st;
      i.tol = s->o.tol;
      i.lambda = s->o.lambda;
      i.hist = w.hist;
      i.max_iter = s->limit;
      i.fixed = fixed ? 1 : 0;
      i.hist_cap = s->limit;
      ia.push_back(i);
      ba.push_back(bwd_of(*s));
      if (!backward_fuses_wmg(*s->g)) {
        gw.push_back(s->g);
        wa.push_back(wmg_of(*s));
      }
    }
    prepare_init_batch(t_init_, gs, ia, st_);
    launch_init_batch(t_init_, st_);
    prepare_backward_batch(t_ib_, gs, ba, st_);
    launch_backward_batch(t_ib_, BWD_CGLS_INIT, st_);
    prepare_wmg_batch(t_iw_, gw, wa, st_);
    launch_wmg_batch(t_iw_, WMG_CGLS_INIT, st_);
    for (Slot* s : slots) active_.push_back(s);
    dirty_ = true;
  }

  // Advance every running problem by one tick; return the ones that finished
  // (removed from the work lists, final state in Slot::fin, workspace still
  // owned by the caller; nothing in flight references it any more).
  std::vector<Slot*> tick() {
    std::vector<Slot*> out;
    if (active_.empty()) return out;
    if (dirty_) rebuild();
    if (use_graph_ && !exec_ && clean_ticks_ >= 1) capture();
    if (exec_) {
      TimedLaunch tl(TK_GRAPH, st_);
      HIP_CHECK(hipGraphLaunch(exec_, st_));
    } else {
      for (int i = 0; i < iters_; ++i) iteration(st_);
    }
    ++clean_ticks_;
    const int cnt = (int)active_.size();
    hipLaunchKernelGGL(k_gather_flags, dim3((cnt + 255) / 256), dim3(256), 0, st_,
                       (const SolverState* const*)d_sts_, cnt, d_flags_);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(h_flags_, d_flags_, sizeof(Flag) * cnt, hipMemcpyDeviceToHost, st_));
    HIP_CHECK(hipStreamSynchronize(st_));
    const double t = now_ms();
    std::vector<Slot*> keep;
    for (int i = 0; i < cnt; ++i) {
      Slot* s = active_[i];
      ++s->ticks;
      // The device caps every problem at `limit` iterations; a problem still
      // running well past that means its state is corrupt.
      if (!h_flags_[i].done && (long long)s->ticks * iters_ > (long long)s->limit + 2 * iters_ + 2)
        s->failed = true;
      if (h_flags_[i].done || s->failed) {
        s->t_done = t;
        out.push_back(s);
      } else {
        keep.push_back(s);
      }
    }
    if (!out.empty()) {
      for (Slot* s : out)
        HIP_CHECK(hipMemcpyAsync(&s->fin, s->w->st, sizeof(SolverState), hipMemcpyDeviceToHost,
                                 st_));
      HIP_CHECK(hipStreamSynchronize(st_));
      active_.swap(keep);
      dirty_ = true;
    }
    return out;
  }

 private:
  static BwdArgs bwd_of(const Slot& s) {
    BwdArgs a{};
    a.sino = s.w->r;
    a.q = s.w->q;
    a.out = s.w->s;
    a.x = s.x;
    a.p = s.w->p;
    a.zP = s.w->zP;
    a.zTP = s.w->zTP;
    a.identity = s.o.precond == RECO_PRECOND_NONE;
    a.st = s.w->st;
    a.red = red_of(*s.w, 1);
    a.fwd_part = fwd_partials(*s.w);
    a.fwd_blocks = forward_blocks(*s.g);
    a.slots = fin_slots(*s.w);
    return a;
  }
  static WmgArgs wmg_of(const Slot& s) {
    WmgArgs a{};
    a.s = s.w->s;
    a.zP = s.w->zP;
    a.zTP = s.w->zTP;
    a.pold = s.w->p;
    a.lambda = s.o.lambda;
    a.identity = s.o.precond == RECO_PRECOND_NONE;
    a.st = s.w->st;
    a.red = red_of(*s.w, 1);
    return a;
  }

  // One CGLS iteration of every running problem (the solo iteration's
  // launches, each over the shared work list; the WMG list holds only the
  // problems whose preconditioner is not applied inside the backprojection).
  void iteration(hipStream_t s) {
    launch_forward_batch(t_fwd_, FWD_CGLS, s);
    launch_backward_batch(t_bwd_, BWD_CGLS, s);
    launch_wmg_batch(t_wmg_, WMG_CGLS, s);
  }

  void rebuild() {
    drop_graph();
    // Largest problems first: a batched launch's blocks are dispatched in
    // grid order, so the longest work starts first and the small problems'
    // blocks fill in behind it.  (Results do not depend on the order.)
    std::stable_sort(active_.begin(), active_.end(), [](const Slot* a, const Slot* b) {
      const double ca = (double)a->g->n * a->g->n * a->g->m;
      const double cb = (double)b->g->n * b->g->n * b->g->m;
      return ca > cb;
    });
    std::vector<const Geometry*> gs, gw;
    std::vector<FwdArgs> fa;
    std::vector<BwdArgs> ba;
    std::vector<WmgArgs> wa;
    std::vector<SolverState*> sts;
    for (Slot* s : active_) {
      Workspace& w = *s->w;
      gs.push_back(s->g);
      FwdArgs f{};
      f.imgP = w.zP;
      f.imgTP = w.zTP;
      f.out = w.q;
      f.r = w.r;
      f.st = w.st;
      f.part = fwd_partials(w);
      fa.push_back(f);
      ba.push_back(bwd_of(*s));
      if (!backward_fuses_wmg(*s->g)) {
        gw.push_back(s->g);
        wa.push_back(wmg_of(*s));
      }
      sts.push_back(w.st);
    }
    prepare_forward_batch(t_fwd_, gs, fa, st_);
    prepare_backward_batch(t_bwd_, gs, ba, st_);
    prepare_wmg_batch(t_wmg_, gw, wa, st_);
    const int cnt = (int)sts.size();
    if (cnt > flag_cap_) {
      // grown geometrically from kTableFloor problems (each hipFree waits for the device)
      const int cap = std::max({cnt, 2 * flag_cap_, (int)kTableFloor});
      if (d_sts_) (void)hipFree(d_sts_);
      if (d_flags_) (void)hipFree(d_flags_);
      if (h_flags_) (void)hipHostFree(h_flags_);
      d_sts_ = nullptr;
      d_flags_ = nullptr;
      h_flags_ = nullptr;
      flag_cap_ = 0;
      HIP_CHECK(hipMalloc((void**)&d_sts_, sizeof(SolverState*) * cap));
      HIP_CHECK(hipMalloc((void**)&d_flags_, sizeof(Flag) * cap));
      HIP_CHECK(hipHostMalloc((void**)&h_flags_, sizeof(Flag) * cap, hipHostMallocDefault));
      flag_cap_ = cap;
    }
    if (cnt > 0) {
      HIP_CHECK(hipMemcpyAsync(d_sts_, sts.data(), sizeof(SolverState*) * cnt,
                               hipMemcpyHostToDevice, st_));
      HIP_CHECK(hipStreamSynchronize(st_));
    }
    dirty_ = false;
    clean_ticks_ = 0;
  }

  void capture() {
    hipGraph_t graph = nullptr;
    HIP_CHECK(hipStreamBeginCapture(cap_, hipStreamCaptureModeRelaxed));
    try {
      for (int i = 0; i < iters_; ++i) iteration(cap_);
    } catch (...) {
      if (hipStreamEndCapture(cap_, &graph) == hipSuccess && graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      throw;
    }
    HIP_CHECK(hipStreamEndCapture(cap_, &graph));
    const hipError_t e = hipGraphInstantiate(&exec_, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      exec_ = nullptr;
      check_hip(e, "hipGraphInstantiate", __FILE__, __LINE__);
    }
  }

  void drop_graph() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    exec_ = nullptr;
  }

  hipStream_t st_;
  hipStream_t cap_ = nullptr;
  int iters_;
  bool use_graph_;
  std::vector<Slot*> active_;
  bool dirty_ = true;
  int clean_ticks_ = 0;
  hipGraphExec_t exec_ = nullptr;
  FwdTables t_fwd_;                          // iteration work lists
  DevTable t_bwd_, t_wmg_;
  DevTable t_init_, t_ib_, t_iw_;            // initialisation of new problems
  SolverState** d_sts_ = nullptr;
  Flag* d_flags_ = nullptr;
  Flag* h_flags_ = nullptr;
  int flag_cap_ = 0;
};

void fill_info(const Slot& s, reco_solve_info* info) {
  if (!info) return;
  info->iters = s.fin.iter;
  info->matvecs = 1 + s.fin.iter;
  info->relres = s.fin.relres;
  info->status = s.failed ? RECO_EDEVICE : status_of(s.fin.done);
  info->reserved = 0;
  info->elapsed_ms = s.t_done - s.t_admit;
}

// A finished problem's workspace is not pooled again when its solve ended
// abnormally (see ReusePool).
void mark_if_unusable(Slot& s) {
  if (!workspace_reusable(s.fin.done, s.failed, false)) s.w->tainted = true;
}

// Workspaces checked out for a batch, returned on every exit path.
struct Leases {
  std::vector<std::pair<Geometry*, Workspace*>> held;
  int unwinding0 = std::uncaught_exceptions();
  ~Leases() {
    const bool unwinding = std::uncaught_exceptions() > unwinding0;
    for (auto& p : held) {
      if (unwinding) p.second->tainted = true;
      return_workspace(*p.first, p.second);
    }
  }
};

}  // namespace

reco_status solve_batch(int32_t count, const reco_geometry* geoms, const void* const* b,
                        void* const* x, const reco_solve_opts* opts, reco_solve_info* info,
                        hipStream_t st) {
  if (count < 0) fail(RECO_EINVAL, "count must be >= 0");
  if (count == 0) return RECO_OK;
  if (!geoms || !b || !x || !opts) fail(RECO_EINVAL, "null array argument");
  for (int i = 0; i < count; ++i) {
    if (!geoms[i] || !b[i] || !x[i]) fail(RECO_EINVAL, "null geometry or buffer in batch");
    const Geometry* g = reinterpret_cast<const Geometry*>(geoms[i]);
    if (g->f64) fail(RECO_EINVAL, "batched solves take RECO_F32 geometries");
    validate_opts(opts[i], false);
  }
  const double t0 = now_ms();
  std::vector<Slot> slots(count);
  Leases leases;
  std::vector<Slot*> ptrs;
  for (int i = 0; i < count; ++i) {
    Slot& s = slots[i];
    s.g = reinterpret_cast<Geometry*>(geoms[i]);
    s.w = checkout_workspace(*s.g, st);
    leases.held.push_back({s.g, s.w});
    s.b = b[i];
    s.x = x[i];
    s.o = opts[i];
    s.t_admit = t0;
    ptrs.push_back(&s);
  }
  int per_tick = 0;
  for (int i = 0; i < count; ++i) per_tick = std::max(per_tick, opts[i].check_every);
  Engine eng(st, per_tick > 0 ? std::min(per_tick, 64) : 2, true);
  eng.add(ptrs);
  while (!eng.empty()) eng.tick();
  reco_status worst = RECO_OK;
  for (int i = 0; i < count; ++i) {
    mark_if_unusable(slots[i]);
    fill_info(slots[i], info ? &info[i] : nullptr);
    const reco_status rc = slots[i].failed ? RECO_EDEVICE : status_of(slots[i].fin.done);
    if (rc != RECO_OK && (worst == RECO_OK || rc < 0)) worst = rc;
  }
  if (worst == RECO_EDEVICE) set_error("a batched problem did not terminate on the device");
  return worst;
}

// ---------------------------------------------------------------------------
// Server: continuous batching with admission by device-memory budget
// ---------------------------------------------------------------------------
// Threads: the caller's (submit / poll), a scheduler per cost tier
// (admission, ticks of the tier's batched engine on its own stream) and a
// geometry builder for the large tier (tables and packet diagonal of
// descriptions seen for the first time, on a stream of its own, so that
// running requests keep advancing meanwhile).
namespace {

struct Request {
  uint64_t ticket = 0;
  reco_geometry_desc desc{};
  const void* b = nullptr;
  void* x = nullptr;
  reco_solve_opts o{};
  reco_status status = RECO_PENDING;
  reco_solve_info info{};
  double t[3] = {-1.0, -1.0, -1.0};
  std::string error;
  Slot slot;
  size_t need = 0;        // device bytes added to the server's account at admission
  bool fresh_ws = false;  // admission added a workspace (none was pooled)
};

using DescKey = std::tuple<int, int, int, int, int, int>;

struct GeoEntry {
  reco_geometry_desc desc{};
  Geometry* g = nullptr;
  bool building = false;
  reco_status err = RECO_OK;
  std::string err_msg;
  size_t bytes = 0;
  size_t ws_bytes = 0;   // bytes of one workspace
  int running = 0;       // admitted requests using it
  int workspaces = 0;    // workspaces it holds or will hold (admitted + pooled)
};

DescKey key_of(const reco_geometry_desc& d) {
  return DescKey{d.n, d.n_angles, d.n_bins, d.wmg_levels, d.dtype, d.projector};
}

}  // namespace

// Requests are split into two tiers by the cost of one iteration, each with
// its own scheduler thread, batched engine and stream: the GPU interleaves
// the streams, so a small problem is not held to one iteration per tick of a
// batch that also advances 2048^2 problems.  The large tier runs one problem
// at a time (in admission order), each at the speed of a solo solve, and
// builds new geometries (up to ~150 ms of GPU work) on a builder thread and
// stream of their own; the small tier batches all of its admitted problems
// and builds its geometries (about a millisecond each) itself between ticks.
// Three streams in all, so that each keeps a hardware queue to itself.
// Admission (arrival order, slot and memory accounting) is shared.  The
// builder works at most kBuildAhead requests ahead of its tier: while that
// many of the tier's admitted requests already have their geometry and wait
// to start, it waits too.  One build beside the running solve keeps the GPU
// busy through the solve's launch gaps (building only while the tier is
// idle measured a 10% longer p99 at 0.9 of saturation); building further
// ahead shares the GPU between the running solve and geometries whose
// requests cannot start before it ends, which delays every request of a
// backlog (p99 913 against 564 ms at 0.9 of saturation).
constexpr int kTiers = 2;
constexpr int kBuildAhead = 1;
constexpr int kTierRunning[kTiers] = {1 << 30, 1};   // problems a tier advances at once
constexpr bool kTierBuilder[kTiers] = {false, true};  // geometries built on a thread of their own

int tier_of(const reco_geometry_desc& d) {
  const double cost = (double)d.n * d.n * d.n_angles;   // ~ updates per iteration
  return cost >= 1024.0 * 1024.0 * 512.0 ? 1 : 0;
}

struct Server {
  size_t budget = 0;
  int max_slots = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
  uint64_t next_ticket = 1;
  // change counters the schedulers wait on: submissions, finished builds,
  // requests that left a tier (freeing slots and memory)
  uint64_t submits = 0, builds = 0, retires = 0;
  bool stop = false, stop_builder = false;
  std::string fatal;                  // a scheduler could not start: every request fails
  std::thread th[kTiers], builder[kTiers];   // builder[t] runs only if kTierBuilder[t]
  std::map<DescKey, GeoEntry> geos;
  std::deque<DescKey> to_build[kTiers];
  std::vector<Request*> waiting;      // admitted, geometry not built yet
  size_t used = 0;                    // geometries + workspaces held
  int running = 0;                    // admitted requests

  void run(int tier);
  void build_loop(int tier);
  int ready_ahead(int tier) const;
  void build_one(const DescKey& k, const reco_geometry_desc& d, hipStream_t st,
                 const std::string& err_stream);
  void admit();
  void finish(Request* r, reco_status st, const std::string& err);
  void release(Request* r);
  bool make_room(size_t need);
  void stop_threads();
};

static double seconds_now() { return now_ms() * 1e-3; }

void Server::finish(Request* r, reco_status st, const std::string& err) {
  r->status = st;
  r->info = reco_solve_info{};
  r->info.status = st;
  r->error = err;
  r->t[2] = seconds_now();
}

// Undo the admission accounting of a request that never ran.  Lock held.
void Server::release(Request* r) {
  const DescKey k = key_of(r->desc);
  GeoEntry& e = geos[k];
  used -= r->need;
  --running;
  --e.running;
  if (r->fresh_ws) --e.workspaces;
  if (!e.g && !e.building && e.running == 0) geos.erase(k);
}

// Free pooled workspaces and unused geometries until `need` more bytes fit.
// Lock held.
bool Server::make_room(size_t need) {
  if (used + need <= budget) return true;
  for (auto& kv : geos) {
    GeoEntry& e = kv.second;
    const int pooled = e.workspaces - e.running;
    if (pooled > 0 && e.g) {
      release_workspaces(*e.g);
      used -= (size_t)pooled * e.ws_bytes;
      e.workspaces = e.running;
    }
  }
  for (auto it = geos.begin(); it != geos.end() && used + need > budget;) {
    GeoEntry& e = it->second;
    if (e.running == 0 && !e.building) {
      used -= e.bytes;
      if (e.g) {
        release_workspaces(*e.g);
        delete e.g;
      }
      it = geos.erase(it);
    } else {
      ++it;
    }
  }
  return used + need <= budget;
}

// Admit queued requests in arrival order while slots and memory allow; a
// request whose geometry is new queues its build with its tier's builder.
// Lock held.
void Server::admit() {
  bool new_builds = false;
  while (!queue.empty() && running < max_slots) {
    Request* r = queue.front();
    const DescKey k = key_of(r->desc);
    auto need_of = [&]() {
      auto it = geos.find(k);
      if (it == geos.end()) return geometry_bytes(r->desc) + cgls_workspace_bytes(r->desc);
      const GeoEntry& e = it->second;
      return e.workspaces - e.running > 0 ? (size_t)0 : e.ws_bytes;
    };
    size_t need = need_of();
    if (need > budget) {
      queue.pop_front();
      finish(r, RECO_ENOMEM, "request needs " + std::to_string(need) +
                                 " device bytes, more than the server budget");
      continue;
    }
    if (used + need > budget) {
      make_room(need);
      need = need_of();   // eviction may have dropped its geometry
      if (used + need > budget) break;
    }
    queue.pop_front();
    GeoEntry& e = geos[k];
    if (e.ws_bytes == 0) {
      e.desc = r->desc;
      e.bytes = geometry_bytes(r->desc);
      e.ws_bytes = cgls_workspace_bytes(r->desc);
    }
    if (!e.g && !e.building) {
      e.building = true;
      e.err = RECO_OK;
      to_build[tier_of(r->desc)].push_back(k);
      new_builds = true;
    }
    r->fresh_ws = e.workspaces - e.running <= 0;
    if (r->fresh_ws) ++e.workspaces;
    ++e.running;
    r->need = need;
    used += need;
    ++running;
    waiting.push_back(r);
  }
  if (new_builds) cv.notify_all();
}

// Requests of `tier` admitted with their geometry built, waiting to start.
// Lock held.
int Server::ready_ahead(int tier) const {
  int n = 0;
  for (const Request* r : waiting) {
    if (tier_of(r->desc) != tier) continue;
    const auto it = geos.find(key_of(r->desc));
    if (it != geos.end() && it->second.g) ++n;
  }
  return n;
}

void Server::build_loop(int tier) {
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  std::string err_stream;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    err_stream = "could not create a geometry builder's stream";
  }
  for (;;) {
    reco_geometry_desc d{};
    DescKey k;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] {
        return stop_builder ||
               (!to_build[tier].empty() && ready_ahead(tier) < kBuildAhead);
      });
      if (to_build[tier].empty()) break;
      k = to_build[tier].front();
      to_build[tier].pop_front();
      d = geos[k].desc;
    }
    build_one(k, d, st, err_stream);
  }
  if (st) (void)hipStreamDestroy(st);
}

// Build one geometry and publish it (or its error).  Lock not held.
void Server::build_one(const DescKey& k, const reco_geometry_desc& d, hipStream_t st,
                       const std::string& err_stream) {
  Geometry* g = nullptr;
  reco_status err = RECO_OK;
  std::string msg;
  if (!err_stream.empty()) {
    err = RECO_EDEVICE;
    msg = err_stream;
  } else {
    try {
      g = create_geometry(d, st);
    } catch (const Error& e) {
      err = e.code;
      msg = e.msg;
    }
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    GeoEntry& e = geos[k];
    e.building = false;
    e.g = g;
    e.err = err;
    e.err_msg = msg;
    ++builds;
  }
  cv.notify_all();
}

void Server::run(int tier) {
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  std::unique_ptr<Engine> eng;
  try {
    HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    eng.reset(new Engine(st, 1, true, true));
  } catch (const Error& e) {
    {
      std::lock_guard<std::mutex> lk(mu);
      if (fatal.empty()) fatal = e.msg;
    }
    cv.notify_all();
  }
  std::vector<Request*> active;
  uint64_t seen_submits = ~0ull, seen_builds = ~0ull, seen_retires = ~0ull;
  for (;;) {
    std::vector<Request*> ready;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (!fatal.empty()) {
        // no request can be served: fail what is queued or waiting
        for (Request* r : queue) finish(r, RECO_EDEVICE, fatal);
        queue.clear();
        for (Request* r : waiting) {
          release(r);
          finish(r, RECO_EDEVICE, fatal);
        }
        waiting.clear();
        if (active.empty()) {
          if (stop) break;
          cv.wait(lk, [&] { return stop || !queue.empty(); });
          continue;
        }
      }
      const bool changed =
          seen_submits != submits || seen_builds != builds || seen_retires != retires;
      seen_submits = submits;
      seen_builds = builds;
      seen_retires = retires;
      if (active.empty() && !changed) {
        const bool mine_waiting = std::any_of(waiting.begin(), waiting.end(), [&](Request* r) {
          return tier_of(r->desc) == tier;
        });
        if (stop && queue.empty() && !mine_waiting) break;
        cv.wait(lk, [&] {
          return stop || submits != seen_submits || builds != seen_builds ||
                 retires != seen_retires || !fatal.empty();
        });
        continue;
      }
      if (fatal.empty()) admit();
      if (!kTierBuilder[tier]) {
        // this tier builds its new geometries itself, on its own stream
        std::vector<std::pair<DescKey, reco_geometry_desc>> todo;
        for (const DescKey& k : to_build[tier]) todo.emplace_back(k, geos[k].desc);
        to_build[tier].clear();
        if (!todo.empty()) {
          lk.unlock();
          for (const auto& kd : todo) build_one(kd.first, kd.second, st, "");
          lk.lock();
        }
      }
      // this tier's requests whose geometry is ready (or failed) leave the
      // waiting list, up to the tier's running limit, in admission order
      std::vector<Request*> still;
      size_t room = (size_t)kTierRunning[tier] > active.size()
                        ? (size_t)kTierRunning[tier] - active.size() : 0;
      for (Request* r : waiting) {
        if (tier_of(r->desc) != tier) {
          still.push_back(r);
          continue;
        }
        GeoEntry& e = geos[key_of(r->desc)];
        if (e.g) {
          if (room == 0) {
            still.push_back(r);
            continue;
          }
          --room;
          ready.push_back(r);
        } else if (!e.building) {
          const reco_status code = e.err != RECO_OK ? e.err : RECO_EDEVICE;
          const std::string msg = e.err_msg;
          release(r);
          finish(r, code, msg.empty() ? "geometry creation failed" : msg);
          ++retires;
        } else {
          still.push_back(r);
        }
      }
      waiting.swap(still);
    }
    if (!ready.empty()) cv.notify_all();   // the builder may go on
    // check out workspaces outside the lock
    std::vector<Slot*> slots;
    for (Request* r : ready) {
      Geometry* g;
      {
        std::lock_guard<std::mutex> lk(mu);
        g = geos[key_of(r->desc)].g;
      }
      try {
        r->slot.g = g;
        r->slot.w = checkout_workspace(*g, st);
        r->slot.b = r->b;
        r->slot.x = r->x;
        r->slot.o = r->o;
        r->slot.owner = r;
        r->slot.t_admit = now_ms();
        std::lock_guard<std::mutex> lk(mu);
        r->t[1] = r->slot.t_admit * 1e-3;
        slots.push_back(&r->slot);
        active.push_back(r);
      } catch (const Error& err) {
        {
          std::lock_guard<std::mutex> lk(mu);
          release(r);
          finish(r, err.code, err.msg);
          ++retires;
        }
        cv.notify_all();
      }
    }
    if (active.empty()) continue;
    try {
      eng->add(slots);
      std::vector<Slot*> done = eng->tick();
      if (!done.empty()) {
        {
          std::lock_guard<std::mutex> lk(mu);
          for (Slot* s : done) {
            Request* r = (Request*)s->owner;
            GeoEntry& e = geos[key_of(r->desc)];
            mark_if_unusable(*s);
            if (!return_workspace(*e.g, s->w)) {   // dropped: no longer held
              --e.workspaces;
              used -= e.ws_bytes;
            }
            --e.running;
            --running;
            fill_info(*s, &r->info);
            r->status = r->info.status;
            r->t[2] = s->t_done * 1e-3;
            if (s->failed) r->error = "solver state did not terminate on the device";
            active.erase(std::find(active.begin(), active.end(), r));
          }
          ++retires;
        }
        cv.notify_all();
      }
    } catch (const Error& err) {
      {
        std::lock_guard<std::mutex> lk(mu);
        if (fatal.empty()) fatal = err.msg;
        for (Request* r : active) finish(r, RECO_EDEVICE, err.msg);
        active.clear();
        ++retires;
      }
      cv.notify_all();
    }
  }
  eng.reset();
  if (st) (void)hipStreamDestroy(st);
}

// Stop and join the schedulers, then the builders, then free the geometries.
void Server::stop_threads() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv.notify_all();
  for (auto& t : th)
    if (t.joinable()) t.join();
  {
    std::lock_guard<std::mutex> lk(mu);
    stop_builder = true;
  }
  cv.notify_all();
  for (auto& t : builder)
    if (t.joinable()) t.join();
  for (auto& kv : geos) {
    if (!kv.second.g) continue;
    release_workspaces(*kv.second.g);
    delete kv.second.g;
  }
  geos.clear();
}

}  // namespace reco

extern "C" {

reco_status reco_server_create(size_t hbm_budget_bytes, int32_t max_slots, reco_server* out) {
  if (!out) {
    reco::set_error("out must not be NULL");
    return RECO_EINVAL;
  }
  *out = nullptr;
  if (hbm_budget_bytes == 0 || max_slots < 1) {
    reco::set_error("budget must be > 0 and max_slots >= 1");
    return RECO_EINVAL;
  }
  try {
    std::unique_ptr<reco::Server> s(new reco::Server());
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    reco::check_hip(hipGetDevice(&s->device), "hipGetDevice", __FILE__, __LINE__);
    reco::Server* p = s.get();
    try {
      for (int t = 0; t < reco::kTiers; ++t) {
        if (reco::kTierBuilder[t]) s->builder[t] = std::thread([p, t] { p->build_loop(t); });
        s->th[t] = std::thread([p, t] { p->run(t); });
      }
    } catch (...) {
      p->stop_threads();
      throw;
    }
    *out = reinterpret_cast<reco_server>(s.release());
    return RECO_OK;
  } catch (const reco::Error& e) {
    reco::set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    reco::set_error(e.what());
    return RECO_EDEVICE;
  }
}

reco_status reco_server_destroy(reco_server h) {
  if (!h) return RECO_OK;
  reco::Server* s = reinterpret_cast<reco::Server*>(h);
  s->stop_threads();
  delete s;
  return RECO_OK;
}

reco_status reco_submit(reco_server h, const reco_geometry_desc* desc, const void* b, void* x,
                        const reco_solve_opts* opts, uint64_t* ticket) {
  if (!h || !desc || !b || !x || !opts || !ticket) {
    reco::set_error("null argument");
    return RECO_EINVAL;
  }
  reco::Server* s = reinterpret_cast<reco::Server*>(h);
  try {
    if (desc->dtype != RECO_F32) reco::fail(RECO_EINVAL, "the server solves RECO_F32 problems");
    if (desc->projector != RECO_PROJ_EXACT && desc->projector != RECO_PROJ_JOSEPH)
      reco::fail(RECO_EINVAL, "projector must be RECO_PROJ_EXACT or RECO_PROJ_JOSEPH");
    if (desc->n < 2 || desc->n > 65536 || desc->n_angles < 1 || desc->n_bins < 1 ||
        desc->wmg_levels < 1 || desc->wmg_levels > 6 ||
        desc->n % (1 << (desc->wmg_levels - 1)) != 0)
      reco::fail(RECO_EINVAL, "invalid geometry description");
    reco::validate_opts(*opts, false);
    std::unique_ptr<reco::Request> r(new reco::Request());
    r->desc = *desc;
    r->b = b;
    r->x = x;
    r->o = *opts;
    r->o.history = nullptr;
    r->o.history_cap = 0;
    r->t[0] = reco::seconds_now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->stop) reco::fail(RECO_EINVAL, "server is shutting down");
      r->ticket = s->next_ticket++;
      ++s->submits;
      *ticket = r->ticket;
      s->queue.push_back(r.get());
      s->all[r->ticket] = std::move(r);
    }
    s->cv.notify_all();
    return RECO_OK;
  } catch (const reco::Error& e) {
    reco::set_error(e.msg);
    return e.code;
  }
}

reco_status reco_poll(reco_server h, uint64_t ticket, reco_solve_info* info,
                      double t_submit_admit_done[3]) {
  if (!h) {
    reco::set_error("null server");
    return RECO_EINVAL;
  }
  reco::Server* s = reinterpret_cast<reco::Server*>(h);
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) {
    reco::set_error("unknown ticket");
    return RECO_ENOTFOUND;
  }
  const reco::Request& r = *it->second;
  if (t_submit_admit_done)
    for (int i = 0; i < 3; ++i) t_submit_admit_done[i] = r.t[i];
  if (r.status == RECO_PENDING) return RECO_PENDING;
  if (info) *info = r.info;
  if (!r.error.empty()) reco::set_error(r.error);
  return r.status;
}

}  // extern "C"
