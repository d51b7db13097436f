// BiCGStab (van der Vorst), right preconditioned, on the normal equations
//   (W^T W + lambda I) M^-1 u = f = W^T b,   x = M^-1 u
// (Section 2.3.1: the paper's primary Krylov solver, with A = W^T W and
// f = W^T b; right preconditioning as in eq. sys_prec).  x0 = 0, r0 = f and
// the shadow vector rhat = r0; per iteration
//   rho = <rhat, r>;  beta = (rho / rho_prev) (alpha / omega)
//   p = r + beta (p - omega v);  phat = M^-1 p;  v = K phat
//   alpha = rho / <rhat, v>;  s = r - alpha v
//   shat = M^-1 s;  t = K shat;  omega = <t, s> / <t, t>   (0 when t = 0)
//   x += alpha phat + omega shat;  r = s - omega t;  relres = ||r|| / ||r0||
// K v = W^T W v + lambda v: the WMG apply writes M^-1 of its input into a pair
// of padded image copies, the forward projector reads them, and the
// backprojector's AXPY mode adds lambda times the padded copy.  phat and shat
// keep their own pairs (zP/zTP and xP/xTP) until x is updated.
//
// Scalars live in the device solver state (FP64): gamma = rho_prev,
// delta = rho, alpha, pp = omega, beta, s0 = ||r0||.  Each dot product is a
// fixed-order FP64 reduction: block partials over chunks of 2048 elements,
// summed by a one-block kernel that also forms the next scalar.  A breakdown
// (rho = 0 or <rhat, v> = 0 before convergence, or omega = 0 with the
// residual still above the tolerance) ends the solve with code 5
// (RECO_ENOTCONV, x = the last iterate); a non-finite scalar with code 3.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "device_common.h"
#include "hybrid.h"
#include "solve.h"

namespace reco {

namespace {

constexpr int kChunk = 2048;   // elements per partial-sum block
constexpr int kBreakdown = 5;

unsigned grid_of(size_t N) {
  const size_t b = (N + 255) / 256;
  return (unsigned)(b > 8192 ? 8192 : (b == 0 ? 1 : b));
}

// Partial sums over chunk blockIdx.x of <a0, b0> and (if a1) <a1, b1>.
template <typename T>
__global__ __launch_bounds__(256) void k_bs_dots(const T* __restrict__ a0, const T* __restrict__ b0,
                                                 const T* __restrict__ a1, const T* __restrict__ b1,
                                                 size_t N, double* d0, double* d1,
                                                 const SolverState* st) {
  if (st->done) return;
  const size_t base = (size_t)blockIdx.x * kChunk;
  double v[2] = {0.0, 0.0};
  for (int e = threadIdx.x; e < kChunk; e += 256) {
    const size_t i = base + e;
    if (i < N) {
      v[0] += (double)a0[i] * (double)b0[i];
      if (a1) v[1] += (double)a1[i] * (double)b1[i];
    }
  }
  __shared__ double sh[8];
  block_sum256<2>(v, sh);
  if (threadIdx.x == 0) {
    d0[blockIdx.x] = v[0];
    if (a1) d1[blockIdx.x] = v[1];
  }
}

// sum of d[0..chunks) in a fixed order (valid in thread 0)
__device__ __forceinline__ double sum_chunks(const double* d, int chunks) {
  double acc = 0.0;
  for (int c = threadIdx.x; c < chunks; c += 256) acc += d[c];
  double v[1] = {acc};
  __shared__ double sh[4];
  block_sum256<1>(v, sh);
  return v[0];
}

// Start: s0 = ||r0||, rho = <rhat, r0> (= ||r0||^2), rho_prev = alpha = omega = 1.
__global__ __launch_bounds__(256) void k_bs_start(SolverState* st, const double* drr,
                                                  const double* drho, int chunks) {
  const double rr = sum_chunks(drr, chunks);
  const double rho = sum_chunks(drho, chunks);
  if (threadIdx.x != 0) return;
  st->s0 = sqrt(rr);
  st->delta = rho;
  st->gamma = 1.0;
  st->alpha = 1.0;
  st->pp = 1.0;
  st->beta = 0.0;
  st->relres = 1.0;
  st->iter = 0;
  if (!finite(st->s0) || !finite(rho)) st->done = 3;
  else if (st->s0 == 0.0) { st->done = 1; st->relres = 0.0; }
}

// p = r + beta (p - omega v), beta = (rho / rho_prev) (alpha / omega), formed
// identically by every thread from the state.
template <typename T>
__global__ __launch_bounds__(256) void k_bs_p(T* __restrict__ p, const T* __restrict__ r,
                                              const T* __restrict__ v, size_t N, SolverState* st) {
  if (st->done) return;
  const double omega = st->pp;
  const double beta = (st->delta / st->gamma) * (st->alpha / omega);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->beta = beta;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256)
    p[i] = (T)((double)r[i] + beta * ((double)p[i] - omega * (double)v[i]));
}

// alpha = rho / <rhat, v>
__global__ __launch_bounds__(256) void k_bs_alpha(SolverState* st, const double* drv, int chunks) {
  if (st->done) return;
  const double rv = sum_chunks(drv, chunks);
  if (threadIdx.x != 0) return;
  const double alpha = st->delta / rv;
  if (!finite(rv) || !finite(alpha)) st->done = 3;
  else if (rv == 0.0) st->done = kBreakdown;
  else st->alpha = alpha;
}

// s = r - alpha v
template <typename T>
__global__ __launch_bounds__(256) void k_bs_s(T* __restrict__ s, const T* __restrict__ r,
                                              const T* __restrict__ v, size_t N,
                                              const SolverState* st) {
  if (st->done) return;
  const double alpha = st->alpha;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256)
    s[i] = (T)((double)r[i] - alpha * (double)v[i]);
}

// omega = <t, s> / <t, t>, 0 when t = 0
__global__ __launch_bounds__(256) void k_bs_omega(SolverState* st, const double* dts,
                                                  const double* dtt, int chunks) {
  if (st->done) return;
  const double ts = sum_chunks(dts, chunks);
  const double tt = sum_chunks(dtt, chunks);
  if (threadIdx.x != 0) return;
  const double omega = tt != 0.0 ? ts / tt : 0.0;
  if (!finite(omega)) st->done = 3;
  else st->pp = omega;
}

// x += alpha phat + omega shat (phat, shat from their padded copies);
// r = s - omega t; partials of ||r||^2 and <rhat, r> over chunk blockIdx.x.
template <typename T>
__global__ __launch_bounds__(256) void k_bs_xr(T* __restrict__ x, T* __restrict__ r,
                                               const T* __restrict__ s, const T* __restrict__ t,
                                               const T* __restrict__ rhat,
                                               const T* __restrict__ phatP,
                                               const T* __restrict__ shatP, int n, int ld,
                                               size_t N, double* drr, double* drho,
                                               const SolverState* st) {
  if (st->done) return;
  const double alpha = st->alpha, omega = st->pp;
  const size_t base = (size_t)blockIdx.x * kChunk;
  double v[2] = {0.0, 0.0};
  for (int e = threadIdx.x; e < kChunk; e += 256) {
    const size_t i = base + e;
    if (i < N) {
      const size_t iy = i / (size_t)n, ix = i - iy * (size_t)n;
      const size_t ip = iy * (size_t)ld + ix + kPad;
      x[i] = (T)((double)x[i] + alpha * (double)phatP[ip] + omega * (double)shatP[ip]);
      const T rn = (T)((double)s[i] - omega * (double)t[i]);
      r[i] = rn;
      v[0] += (double)rn * (double)rn;
      v[1] += (double)rhat[i] * (double)rn;
    }
  }
  __shared__ double sh[8];
  block_sum256<2>(v, sh);
  if (threadIdx.x == 0) {
    drr[blockIdx.x] = v[0];
    drho[blockIdx.x] = v[1];
  }
}

// End of an iteration: relres, history, stopping test, rho_prev = rho,
// rho = <rhat, r>; breakdowns as in the header.
__global__ __launch_bounds__(256) void k_bs_finish(SolverState* st, const double* drr,
                                                   const double* drho, int chunks) {
  if (st->done) return;
  const double rr = sum_chunks(drr, chunks);
  const double rho = sum_chunks(drho, chunks);
  if (threadIdx.x != 0) return;
  const int iter = st->iter + 1;
  st->iter = iter;
  const double rel = sqrt(rr) / st->s0;
  st->relres = rel;
  if (st->hist && iter <= st->hist_cap) st->hist[iter - 1] = rel;
  st->gamma = st->delta;
  st->delta = rho;
  const bool conv = st->fixed ? false : rel <= st->tol;
  if (!finite(rel) || !finite(rho)) st->done = 3;
  else if (st->fixed) { if (iter >= st->max_iter) st->done = 1; }
  else if (conv) st->done = 1;
  else if (iter >= st->max_iter) st->done = 2;
  else if (rho == 0.0 || st->pp == 0.0) st->done = kBreakdown;
}

template <typename T>
reco_status bicgstab_impl(Geometry& g, const void* bvoid, void* xvoid, const reco_solve_opts& o,
                          reco_solve_info* info, hipStream_t st, Workspace& w) {
  const size_t N = g.N();
  const int chunks = (int)((N + kChunk - 1) / kChunk);
  // two more image vectors (s and t) in the basis buffer, five partial-sum rows
  if (w.v_cap < 2) {
    if (w.V) (void)hipFree(w.V);
    w.V = nullptr;
    w.v_cap = 0;
    if (hipMalloc(&w.V, sizeof(T) * N * 2) != hipSuccess) {
      (void)hipGetLastError();
      fail(RECO_ENOMEM, "BiCGStab vector allocation failed");
    }
    w.v_cap = 2;
  }
  const size_t gm_need = (size_t)5 * chunks + 8;
  if (!w.gm || w.gm_cap < gm_need) {
    if (w.gm) (void)hipFree(w.gm);
    w.gm = nullptr;
    w.gm_cap = 0;
    if (hipMalloc((void**)&w.gm, sizeof(double) * gm_need) != hipSuccess) {
      (void)hipGetLastError();
      fail(RECO_ENOMEM, "BiCGStab scratch allocation failed");
    }
    w.gm_cap = gm_need;
  }
  const bool fixed = o.fixed_iters > 0;
  const int limit = fixed ? o.fixed_iters : o.max_iter;
  ensure_history(w, limit);
  T* x = (T*)xvoid;
  T* r = (T*)w.s;
  T* rhat = (T*)w.fvec;
  T* p = (T*)w.p;
  T* v = (T*)w.tmp;
  T* s = (T*)w.V;
  T* t = s + N;
  double* D = w.gm;
  double *d0 = D, *d1 = D + chunks, *d2 = D + 2 * chunks, *d3 = D + 3 * chunks;
  const bool ident = o.precond == RECO_PRECOND_NONE;
  const bool hyb = o.precond == RECO_PRECOND_WMG_HYBRID;
  const HybridFactors* hf = hyb ? &ensure_hybrid(g, o.lambda, st) : nullptr;
  HybridScratch* hs = hyb ? &hybrid_scratch(g, w, st) : nullptr;
  SolverState* ds = w.st;
  const unsigned gN = grid_of(N);
  launch_state_init(ds, o.tol, limit, fixed ? 1 : 0, o.lambda, w.hist, limit, st);
  launch_fill(x, N, g.f64, 0.0, st);
  // shat's padded pair: the WMG apply writes interiors only; the forward
  // projector reads the zero margins
  launch_fill(w.xP, g.padded_elems(), g.f64, 0.0, st);
  launch_fill(w.xTP, g.padded_elems(), g.f64, 0.0, st);
  launch_fill(p, N, g.f64, 0.0, st);
  launch_fill(v, N, g.f64, 0.0, st);
  {
    BwdArgs ba{};
    ba.sino = bvoid;
    ba.out = r;
    launch_backward(g, BWD_PLAIN, ba, st);   // r0 = f = W^T b
  }
  launch_copy(r, rhat, N, g.f64, st);
  hipLaunchKernelGGL(k_bs_dots<T>, dim3(chunks), dim3(256), 0, st, r, r, rhat, r, N, d0, d1,
                     (const SolverState*)ds);
  hipLaunchKernelGGL(k_bs_start, dim3(1), dim3(256), 0, st, ds, d0, d1, chunks);
  HIP_CHECK(hipGetLastError());
  // M^-1 of `in` into the padded pair (P, TP), then out = K M^-1 in
  auto apply_K = [&](const T* in, void* P, void* TP, T* out) {
    if (hyb) {
      hybrid_apply(g, *hf, *hs, in, P, TP, nullptr, st);
    } else {
      WmgArgs wa{};
      wa.s = in;
      wa.zP = P;
      wa.zTP = TP;
      wa.lambda = o.lambda;
      wa.identity = ident;
      wa.st = ds;
      launch_wmg(g, WMG_GMRES, wa, st);
    }
    FwdArgs fa{};
    fa.imgP = P;
    fa.imgTP = TP;
    fa.out = w.q;
    fa.st = ds;
    launch_forward(g, FWD_PLAIN, fa, st);
    BwdArgs ba{};
    ba.sino = w.q;
    ba.out = out;
    ba.x = P;
    ba.x_ld = g.ld;
    ba.x_off = kPad;
    ba.sa = 1.0;
    ba.sx = o.lambda;
    ba.st = ds;
    launch_backward(g, BWD_AXPY, ba, st);
  };
  const int poll_every = o.check_every > 0 ? o.check_every : 4;
  int launched = 0;
  for (;;) {
    hipLaunchKernelGGL(k_bs_p<T>, dim3(gN), dim3(256), 0, st, p, (const T*)r, (const T*)v, N, ds);
    apply_K(p, w.zP, w.zTP, v);
    hipLaunchKernelGGL(k_bs_dots<T>, dim3(chunks), dim3(256), 0, st, rhat, v, (const T*)nullptr,
                       (const T*)nullptr, N, d0, d1, (const SolverState*)ds);
    hipLaunchKernelGGL(k_bs_alpha, dim3(1), dim3(256), 0, st, ds, d0, chunks);
    hipLaunchKernelGGL(k_bs_s<T>, dim3(gN), dim3(256), 0, st, s, (const T*)r, (const T*)v, N,
                       (const SolverState*)ds);
    apply_K(s, w.xP, w.xTP, t);
    hipLaunchKernelGGL(k_bs_dots<T>, dim3(chunks), dim3(256), 0, st, t, s, t, t, N, d0, d1,
                       (const SolverState*)ds);
    hipLaunchKernelGGL(k_bs_omega, dim3(1), dim3(256), 0, st, ds, d0, d1, chunks);
    hipLaunchKernelGGL(k_bs_xr<T>, dim3(chunks), dim3(256), 0, st, x, r, (const T*)s, (const T*)t,
                       (const T*)rhat, (const T*)w.zP, (const T*)w.xP, g.n, g.ld, N, d2, d3,
                       (const SolverState*)ds);
    hipLaunchKernelGGL(k_bs_finish, dim3(1), dim3(256), 0, st, ds, d2, d3, chunks);
    HIP_CHECK(hipGetLastError());
    ++launched;
    if (launched % poll_every == 0 || launched >= limit) {
      HIP_CHECK(hipMemcpyAsync(w.h_st, ds, sizeof(SolverState), hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      if (w.h_st->done || launched >= limit) break;
    }
  }
  const SolverState& sv = *w.h_st;
  if (o.history && o.history_cap > 0 && sv.iter > 0) {
    const int cnt = std::min(std::min(o.history_cap, sv.iter), w.hist_cap);
    HIP_CHECK(hipMemcpyAsync(o.history, w.hist, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
  }
  const reco_status rc = sv.done == 1 ? RECO_OK : (sv.done == 3 ? RECO_ENUMERIC : RECO_ENOTCONV);
  if (info) {
    info->iters = sv.iter;
    info->matvecs = 2 * sv.iter;
    info->relres = sv.relres;
    info->status = rc;
    info->reserved = 0;
  }
  return rc;
}

}  // namespace

reco_status solve_bicgstab(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                           reco_solve_info* info, hipStream_t st) {
  if (!(o.tol > 0.0) && o.fixed_iters <= 0) fail(RECO_EINVAL, "tol must be > 0");
  if (o.max_iter < 1 && o.fixed_iters <= 0) fail(RECO_EINVAL, "max_iter must be >= 1");
  if (!(o.lambda >= 0.0)) fail(RECO_EINVAL, "lambda must be >= 0");
  if (o.precond != RECO_PRECOND_NONE && o.precond != RECO_PRECOND_WMG &&
      o.precond != RECO_PRECOND_WMG_HYBRID)
    fail(RECO_EINVAL, "unknown preconditioner");
  if (o.history_cap < 0) fail(RECO_EINVAL, "history_cap must be >= 0");
  if (o.check_every < 0) fail(RECO_EINVAL, "check_every must be >= 0");
  const auto t0 = std::chrono::steady_clock::now();
  Workspace* w = checkout_workspace(g, st);
  reco_status rc;
  try {
    ensure_aux(g, *w);
    rc = g.f64 ? bicgstab_impl<double>(g, b, x, o, info, st, *w)
               : bicgstab_impl<float>(g, b, x, o, info, st, *w);
  } catch (...) {
    w->tainted = true;
    return_workspace(g, w);
    throw;
  }
  return_workspace(g, w);
  if (info)
    info->elapsed_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

}  // namespace reco
