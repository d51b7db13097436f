// Solver drivers: CGLS (a Krylov method, Section 2.3.1, with an SPD
// preconditioner on the normal equations), restarted right-preconditioned GMRES (eq. sys_prec) and SIRT
// (eq. sirt_it).  The Krylov state stays on the device; scalars are float64.
// The host only enqueues iterations and polls a pinned copy of the device
// state every few iterations; once the device marks the solve finished every
// further kernel of the chunk returns immediately.
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>

#include "device_common.h"
#include "hybrid.h"
#include "solve.h"
#include "timing.h"

namespace reco {

// ---------------------------------------------------------------------------
// Workspaces
// ---------------------------------------------------------------------------
Workspace::~Workspace() {
  auto f = [](void* p) { if (p) (void)hipFree(p); };
  f(r); f(q); f(s); f(p); f(zP); f(zTP); f(xP); f(xTP); f(tmp); f(fvec);
  f(partial); f(counter); f(st); f(hist); f(V); f(gm);
  if (h_st) (void)hipHostFree(h_st);
  delete hyb;
}

static void alloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    fail(RECO_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
}

Workspace* checkout_workspace(Geometry& g, hipStream_t st) {
  if (Workspace* w = g.ws_pool.take()) return w;
  std::unique_ptr<Workspace> w(new Workspace());
  const size_t es = g.esize();
  alloc(&w->r, es * g.M());
  alloc(&w->q, es * g.M());
  alloc(&w->s, es * g.N());
  alloc(&w->p, es * g.N());
  alloc(&w->zP, es * g.padded_elems());
  alloc(&w->zTP, es * g.padded_elems());
  int cap = std::max(forward_blocks(g), std::max(backward_blocks(g), wmg_blocks(g)));
  w->red_cap = cap * 4;
  alloc((void**)&w->partial, sizeof(double) * (2 * w->red_cap + cap));
  alloc((void**)&w->counter, sizeof(unsigned) * 4);
  alloc((void**)&w->st, sizeof(SolverState));
  if (hipHostMalloc((void**)&w->h_st, sizeof(SolverState), hipHostMallocDefault) != hipSuccess)
    fail(RECO_ENOMEM, "pinned host allocation failed");
  std::memset(w->h_st, 0, sizeof(SolverState));
  HIP_CHECK(hipMemsetAsync(w->counter, 0, sizeof(unsigned) * 4, st));
  double empty;
  std::memcpy(&empty, &kSlotEmpty, sizeof(empty));
  launch_fill(fin_slots(*w), w->red_cap, true, empty, st);
  // zero padding columns of the padded image copies once; kernels only write interiors
  launch_fill(w->zP, g.padded_elems(), g.f64, 0.0, st);
  launch_fill(w->zTP, g.padded_elems(), g.f64, 0.0, st);
  return w.release();
}

void ensure_aux(Geometry& g, Workspace& w) {
  const size_t es = g.esize();
  if (!w.xP) alloc(&w.xP, es * g.padded_elems());
  if (!w.xTP) alloc(&w.xTP, es * g.padded_elems());
  if (!w.tmp) alloc(&w.tmp, es * std::max(g.N(), g.M()));
  if (!w.fvec) alloc(&w.fvec, es * g.N());
}

size_t cgls_workspace_bytes(const reco_geometry_desc& d) {
  const size_t es = d.dtype == RECO_F64 ? 8 : 4;
  const size_t n = (size_t)d.n, N = n * n, M = (size_t)d.n_angles * d.n_bins;
  const size_t padded = n * (n + 2 * kPad);
  const size_t tiles = (n + 15) / 16;
  const size_t fblocks = (size_t)((d.n_bins + 31) / 32) * (size_t)((d.n_angles + 7) / 8 + 2);
  const size_t blocks = std::max(fblocks, tiles * tiles) * 2;
  const size_t hist = 8 * 4096;
  // reduction partials, forward partials and finisher slots: 9 doubles per block
  return es * (2 * M + 2 * N + 2 * padded) + sizeof(double) * 9 * blocks + hist + 4096;
}

size_t geometry_bytes(const reco_geometry_desc& d) {
  const size_t es = d.dtype == RECO_F64 ? 8 : 4;
  const size_t N = (size_t)d.n * d.n;
  // forward block tables: at most (m + 7) / 8 + 3 angle groups (runs of up to
  // 8 angles, broken at the two walk-axis changes)
  const size_t groups = (size_t)(d.n_angles + 7) / 8 + 3;
  const size_t bands = (size_t)(d.n + 15) / 16;
  const size_t blocks = groups * (size_t)((d.n_bins + 31) / 32);
  return (sizeof(FwdAngle) + sizeof(BwdAngle) + 8 * sizeof(int)) * (size_t)(d.n_angles + 8) +
         blocks * ((bands + 1) * 8 + 4 + sizeof(FwdBlk)) + N * 8 +
         std::max(N * es, diag_sum_bytes(d.n, d.wmg_levels - 1)) + 4096;
}

bool return_workspace(Geometry& g, Workspace* w) {
  if (!w) return false;
  const int done = w->h_st ? w->h_st->done : 0;
  const bool reusable = workspace_reusable(done, w->tainted, false);
  return g.ws_pool.give_back(w, reusable, [](Workspace* p) {
    // late partial stores or queued kernels may still target its buffers
    (void)hipDeviceSynchronize();
    delete p;
  });
}

void release_workspaces(Geometry& g) {
  g.ws_pool.drain([](Workspace* p) { delete p; });
}

void ensure_history(Workspace& w, int cap) {
  if (cap <= w.hist_cap) return;
  if (w.hist) (void)hipFree(w.hist);
  w.hist = nullptr;
  w.hist_cap = 0;
  alloc((void**)&w.hist, sizeof(double) * cap);
  w.hist_cap = cap;
}

double* fwd_partials(Workspace& w) { return w.partial + w.red_cap; }
double* fin_slots(Workspace& w) { return w.partial + w.red_cap + w.red_cap / 4; }

RedScratch red_of(Workspace& w, int slot) {
  RedScratch r;
  r.partial = w.partial;
  r.counter = w.counter + slot;
  r.capacity = w.red_cap;
  return r;
}

struct Lease {
  Geometry& g;
  Workspace* w;
  int unwinding0;
  Lease(Geometry& gg, hipStream_t st)
      : g(gg), w(checkout_workspace(gg, st)), unwinding0(std::uncaught_exceptions()) {}
  ~Lease() {
    if (std::uncaught_exceptions() > unwinding0) w->tainted = true;
    return_workspace(g, w);
  }
};

void validate_opts(const reco_solve_opts& o, bool gmres) {
  if (!(o.tol > 0.0) && o.fixed_iters <= 0) fail(RECO_EINVAL, "tol must be > 0");
  if (o.max_iter < 1 && o.fixed_iters <= 0) fail(RECO_EINVAL, "max_iter must be >= 1");
  if (!(o.lambda >= 0.0)) fail(RECO_EINVAL, "lambda must be >= 0");
  if (o.precond == RECO_PRECOND_WMG_HYBRID && !gmres)
    fail(RECO_EINVAL, "the hybrid wavelet cycle is not symmetric: use it with GMRES or BiCGStab");
  if (o.precond != RECO_PRECOND_NONE && o.precond != RECO_PRECOND_WMG &&
      o.precond != RECO_PRECOND_WMG_HYBRID)
    fail(RECO_EINVAL, "unknown preconditioner");
  if (gmres && (o.restart < 1 || o.restart > 64)) fail(RECO_EINVAL, "restart must be in [1, 64]");
  if (o.history_cap < 0) fail(RECO_EINVAL, "history_cap must be >= 0");
  if (o.check_every < 0) fail(RECO_EINVAL, "check_every must be >= 0");
}

reco_status status_of(int done) {
  switch (done) {
    case 1: return RECO_OK;
    case 2: return RECO_ENOTCONV;
    case 3: return RECO_ENUMERIC;
    case 4: return RECO_EDEVICE;   // a reduction's partial sums never arrived
    default: return RECO_ENOTCONV;
  }
}

static void poll_state(Workspace& w, hipStream_t st) {
  HIP_CHECK(hipMemcpyAsync(w.h_st, w.st, sizeof(SolverState), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
}

static void finish_info(Workspace& w, const reco_solve_opts& o, reco_solve_info* info,
                        int matvecs, double ms, hipStream_t st) {
  const SolverState& s = *w.h_st;
  if (o.history && o.history_cap > 0 && s.iter > 0 && w.hist) {
    const int cnt = std::min(std::min(o.history_cap, s.iter), w.hist_cap);
    HIP_CHECK(hipMemcpyAsync(o.history, w.hist, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
  }
  if (info) {
    info->iters = s.iter;
    info->matvecs = matvecs;
    info->relres = s.relres;
    info->status = status_of(s.done);
    info->reserved = 0;
    info->elapsed_ms = ms;
  }
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Run `step` repeatedly until the device reports done, polling every few calls.
template <typename F>
static void drive(Workspace& w, const reco_solve_opts& o, int limit, hipStream_t st, F step) {
  int launched = 0;
  int chunk = o.check_every > 0 ? o.check_every : 2;
  for (;;) {
    const int todo = std::min(chunk, limit - launched);
    for (int i = 0; i < todo; ++i) step();
    launched += todo;
    poll_state(w, st);
    if (w.h_st->done || launched >= limit) break;
    if (o.check_every == 0) chunk = std::min(chunk * 2, 16);
  }
}

// ---------------------------------------------------------------------------
// CGLS
// ---------------------------------------------------------------------------
// One iteration (2 launches; 3 when 2^L > 16):
//   K1 forward:  r -= alpha_prev q (the previous step, deferred);
//                q = W z + beta q (= W p_new);  delta = ||q||^2 + lambda ||p_new||^2;
//                alpha = gamma / delta
//   K2 backward: p = z + beta p;  x += alpha p;  s = W^T (r - alpha q) - lambda x;
//                z = M^-1 s (in the same launch when 2^L <= 16, else K4);
//                gamma' = <s,z>, beta = gamma'/gamma, relres = ||s||/||s_0||, stop test
static FwdArgs cgls_fwd_args(Workspace& w) {
  FwdArgs fa{};
  fa.imgP = w.zP;
  fa.imgTP = w.zTP;
  fa.out = w.q;
  fa.r = w.r;
  fa.st = w.st;
  fa.part = fwd_partials(w);
  return fa;
}

static BwdArgs cgls_bwd_args(const Geometry& g, Workspace& w, void* x, const reco_solve_opts& o) {
  BwdArgs ba{};
  ba.sino = w.r;
  ba.q = w.q;
  ba.out = w.s;
  ba.x = x;
  ba.p = w.p;
  ba.zP = w.zP;
  ba.zTP = w.zTP;
  ba.identity = o.precond == RECO_PRECOND_NONE;
  ba.st = w.st;
  ba.red = red_of(w, 1);
  ba.fwd_part = fwd_partials(w);
  ba.fwd_blocks = forward_blocks(g);
  ba.slots = fin_slots(w);
  return ba;
}

static WmgArgs cgls_wmg_args(Workspace& w, const reco_solve_opts& o) {
  WmgArgs wa{};
  wa.s = w.s;
  wa.zP = w.zP;
  wa.zTP = w.zTP;
  wa.pold = w.p;
  wa.lambda = o.lambda;
  wa.identity = o.precond == RECO_PRECOND_NONE;
  wa.st = w.st;
  wa.red = red_of(w, 1);
  return wa;
}

void cgls_iteration(Geometry& g, Workspace& w, void* x, const reco_solve_opts& o, hipStream_t st) {
  launch_forward(g, FWD_CGLS, cgls_fwd_args(w), st);
  launch_backward(g, BWD_CGLS, cgls_bwd_args(g, w, x, o), st);
  if (!backward_fuses_wmg(g)) launch_wmg(g, WMG_CGLS, cgls_wmg_args(w, o), st);
}

// x = p = q = 0, r = b, then s_0 = W^T b - lambda x, z_0 = M^-1 s_0.
void cgls_setup(Geometry& g, Workspace& w, const void* b, void* x, const reco_solve_opts& o,
                hipStream_t st) {
  const bool fixed = o.fixed_iters > 0;
  const int limit = fixed ? o.fixed_iters : o.max_iter;
  ensure_history(w, limit);
  launch_cgls_prepare(w.st, o.tol, limit, fixed ? 1 : 0, o.lambda, w.hist, limit, x, w.p, w.q, w.r,
                      b, g.N(), g.M(), g.f64, st);
  launch_backward(g, BWD_CGLS_INIT, cgls_bwd_args(g, w, x, o), st);
  if (!backward_fuses_wmg(g)) launch_wmg(g, WMG_CGLS_INIT, cgls_wmg_args(w, o), st);
}

static reco_status run_cgls(Geometry& g, Workspace& w, const void* b, void* x,
                            const reco_solve_opts& o, reco_solve_info* info, hipStream_t st,
                            double t0) {
  cgls_setup(g, w, b, x, o, st);
  const int limit = o.fixed_iters > 0 ? o.fixed_iters : o.max_iter;
  drive(w, o, limit, st, [&] { cgls_iteration(g, w, x, o, st); });
  const SolverState& s = *w.h_st;
  finish_info(w, o, info, 1 + s.iter, now_ms() - t0, st);
  return status_of(s.done);
}

reco_status solve_cgls(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                       reco_solve_info* info, hipStream_t st) {
  validate_opts(o, false);
  const double t0 = now_ms();
  Lease lease(g, st);
  return run_cgls(g, *lease.w, b, x, o, info, st, t0);
}

// ---------------------------------------------------------------------------
// Allocation-free CGLS
// ---------------------------------------------------------------------------
// Every device buffer of the solve is carved from one fixed device array and
// the host copy of the solver state lives on the caller's stack, so the call
// makes no device or host allocation.  The array's name is a host-side
// stand-in, not a device address: its address on each device is looked up
// once, with that device current, and only that address reaches kernels and
// fills.  All calls on one device share the array, so calls that overlap on
// one device race; every buffer whose contents the kernels assume (ticket
// counters at zero, finisher slots empty-marked, zero padding columns) is
// re-established by fill kernels at the start of each call.
static_assert(RECO_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[RECO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
void* scratch_address() {
  int dev = -1;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(RECO_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(RECO_EDEVICE, "scratch array has no device address");
    g_scratch_addr[dev] = p;
  }
  return g_scratch_addr[dev];
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of the CGLS buffers inside the scratch array.
struct ScratchLayout {
  size_t r, q, s, p, zP, zTP, partial, counter, st, hist, total;
  int red_cap;
};

ScratchLayout scratch_layout(const Geometry& g, int hist_cap) {
  ScratchLayout l{};
  const size_t es = g.esize();
  const int cap = std::max(forward_blocks(g), std::max(backward_blocks(g), wmg_blocks(g)));
  l.red_cap = cap * 4;
  size_t off = 0;
  auto put = [&](size_t bytes) { const size_t at = off; off = align_up(off + bytes); return at; };
  l.r = put(es * g.M());
  l.q = put(es * g.M());
  l.s = put(es * g.N());
  l.p = put(es * g.N());
  l.zP = put(es * g.padded_elems());
  l.zTP = put(es * g.padded_elems());
  l.partial = put(sizeof(double) * (2 * (size_t)l.red_cap + cap));
  l.counter = put(sizeof(unsigned) * 4);
  l.st = put(sizeof(SolverState));
  l.hist = put(sizeof(double) * (size_t)hist_cap);
  l.total = off;
  return l;
}

// A Workspace whose buffers point into the scratch array: never freed.
struct BorrowedWorkspace {
  Workspace w;
  SolverState host_state{};
  ~BorrowedWorkspace() {
    w.r = w.q = w.s = w.p = w.zP = w.zTP = nullptr;
    w.partial = nullptr;
    w.counter = nullptr;
    w.st = nullptr;
    w.h_st = nullptr;
    w.hist = nullptr;
  }
};
}  // namespace

reco_status solve_cgls_noalloc(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                               reco_solve_info* info, hipStream_t st) {
  validate_opts(o, false);
  if (timing_on())
    fail(RECO_EINVAL, "per-kernel timing is enabled; its events are created on demand");
  const int limit = o.fixed_iters > 0 ? o.fixed_iters : o.max_iter;
  const ScratchLayout l = scratch_layout(g, limit);
  if (l.total > (size_t)RECO_NOALLOC_SCRATCH_BYTES)
    fail(RECO_EINVAL, "problem needs " + std::to_string(l.total) +
                          " bytes of solver scratch; the fixed scratch array holds " +
                          std::to_string((size_t)RECO_NOALLOC_SCRATCH_BYTES));
  const double t0 = now_ms();
  char* base = static_cast<char*>(scratch_address());
  BorrowedWorkspace bw;
  Workspace& w = bw.w;
  w.r = base + l.r;
  w.q = base + l.q;
  w.s = base + l.s;
  w.p = base + l.p;
  w.zP = base + l.zP;
  w.zTP = base + l.zTP;
  w.partial = reinterpret_cast<double*>(base + l.partial);
  w.red_cap = l.red_cap;
  w.counter = reinterpret_cast<unsigned*>(base + l.counter);
  w.st = reinterpret_cast<SolverState*>(base + l.st);
  w.h_st = &bw.host_state;
  w.hist = reinterpret_cast<double*>(base + l.hist);
  w.hist_cap = limit;
  // what the kernels assume of a fresh workspace: zero ticket counters (four
  // 32-bit words, filled as floats of value 0), empty-marked finisher slots,
  // zero padding columns of the padded image copies
  launch_fill(w.counter, 4, false, 0.0, st);
  double empty;
  std::memcpy(&empty, &kSlotEmpty, sizeof(empty));
  launch_fill(fin_slots(w), w.red_cap, true, empty, st);
  launch_fill(w.zP, g.padded_elems(), g.f64, 0.0, st);
  launch_fill(w.zTP, g.padded_elems(), g.f64, 0.0, st);
  return run_cgls(g, w, b, x, o, info, st, t0);
}

// ---------------------------------------------------------------------------
// SIRT
// ---------------------------------------------------------------------------
void ensure_sirt_weights(Geometry& g, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g.sirt_mu);
  if (g.d_sirtR) return;
  const size_t es = g.esize();
  void *R = nullptr, *C = nullptr, *ones = nullptr, *P = nullptr, *PT = nullptr;
  alloc(&R, es * g.M());
  alloc(&C, es * g.N());
  alloc(&ones, es * std::max(g.N(), g.M()));
  alloc(&P, es * g.padded_elems());
  alloc(&PT, es * g.padded_elems());
  launch_fill(ones, std::max(g.N(), g.M()), g.f64, 1.0, st);
  launch_pad_transpose(g, ones, P, PT, st);
  FwdArgs fa{};
  fa.imgP = P;
  fa.imgTP = PT;
  fa.out = R;
  launch_forward(g, FWD_PLAIN, fa, st);
  launch_invert(R, g.M(), g.f64, st);
  BwdArgs ba{};
  ba.sino = ones;
  ba.out = C;
  launch_backward(g, BWD_PLAIN, ba, st);
  launch_invert(C, g.N(), g.f64, st);
  HIP_CHECK(hipStreamSynchronize(st));
  (void)hipFree(ones);
  (void)hipFree(P);
  (void)hipFree(PT);
  g.d_sirtR = R;
  g.d_sirtC = C;
}

reco_status solve_sirt(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                       reco_solve_info* info, hipStream_t st) {
  validate_opts(o, false);
  const double t0 = now_ms();
  ensure_sirt_weights(g, st);
  Lease lease(g, st);
  Workspace& w = *lease.w;
  ensure_aux(g, w);
  const bool fixed = o.fixed_iters > 0;
  const int limit = fixed ? o.fixed_iters : o.max_iter;
  ensure_history(w, limit);
  launch_state_init(w.st, o.tol, limit, fixed ? 1 : 0, 0.0, w.hist, limit, st);
  launch_fill(x, g.N(), g.f64, 0.0, st);
  drive(w, o, limit, st, [&] {
    launch_pad_transpose(g, x, w.xP, w.xTP, st);
    FwdArgs fa{};
    fa.imgP = w.xP;
    fa.imgTP = w.xTP;
    fa.out = w.r;
    fa.b = b;
    fa.R = g.d_sirtR;
    fa.st = w.st;
    launch_forward(g, FWD_SIRT, fa, st);
    BwdArgs ba{};
    ba.sino = w.r;
    ba.out = x;
    ba.C = g.d_sirtC;
    ba.st = w.st;
    ba.red = red_of(w, 2);
    launch_backward(g, BWD_SIRT, ba, st);
  });
  const SolverState& s = *w.h_st;
  finish_info(w, o, info, s.iter, now_ms() - t0, st);
  return status_of(s.done);
}

}  // namespace reco
