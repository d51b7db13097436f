// Restarted GMRES on the right-preconditioned normal equations
//   (W^T W + lambda I) M^-1 u = f = W^T b,   x = M^-1 u   (eq. sys_prec)
// Arnoldi with classical Gram-Schmidt applied twice (CGS2: two projections
// against the whole basis, float64 dot products), Givens rotations on the
// Hessenberg matrix in float64 on the device, residual estimate |g_{j+1}|/||f||.
// Basis vectors are stored in the geometry dtype, one image each.
#include <chrono>
#include <cmath>

#include "device_common.h"
#include "hybrid.h"
#include "solve.h"

namespace reco {

namespace {

constexpr int kChunkElems = 2048;   // elements per dot-product block

// Layout of the float64 GMRES scratch (restart R):
//   H [(R+1) x R] row-major, cs [R], sn [R], g [R+1], y [R], h1 [R+1], h2 [R+1]
struct GmLayout {
  int R;
  __host__ __device__ double* H(double* b) const { return b; }
  __host__ __device__ double* cs(double* b) const { return b + (R + 1) * R; }
  __host__ __device__ double* sn(double* b) const { return cs(b) + R; }
  __host__ __device__ double* g(double* b) const { return sn(b) + R; }
  __host__ __device__ double* y(double* b) const { return g(b) + R + 1; }
  __host__ __device__ double* h1(double* b) const { return y(b) + R; }
  __host__ __device__ double* h2(double* b) const { return h1(b) + R + 1; }
  __host__ __device__ double* dots(double* b) const { return h2(b) + R + 1; }  // [nv x chunks]
  size_t count(int chunks) const { return (size_t)(R + 1) * R + 2 * R + (R + 1) + R + 2 * (R + 1) + (size_t)(R + 2) * chunks; }
};

// partial dots of w with v_0..v_{nv-1} (blockIdx.y = vector), or of v_0 with itself
template <typename T>
__global__ __launch_bounds__(256) void k_mdot(const T* __restrict__ V, const T* __restrict__ w,
                                              size_t N, double* dots, int chunks,
                                              const SolverState* st) {
  if (st && st->done) return;
  const int i = blockIdx.y;
  const T* v = V + (size_t)i * N;
  const size_t base = (size_t)blockIdx.x * kChunkElems;
  double acc = 0.0;
  for (int e = threadIdx.x; e < kChunkElems; e += 256) {
    const size_t idx = base + e;
    if (idx < N) acc += (double)v[idx] * (double)w[idx];
  }
  double vv[1] = {acc};
  __shared__ double sh[4];
  block_sum256<1>(vv, sh);
  if (threadIdx.x == 0) dots[(size_t)i * chunks + blockIdx.x] = vv[0];
}

// out[i] = sum over chunks of dots[i][.] (fixed order); one block per vector
__global__ __launch_bounds__(256) void k_dot_sum(const double* dots, int chunks, double* out,
                                                 const SolverState* st) {
  if (st && st->done) return;
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int c = threadIdx.x; c < chunks; c += 256) acc += dots[(size_t)i * chunks + c];
  double vv[1] = {acc};
  __shared__ double sh[4];
  block_sum256<1>(vv, sh);
  if (threadIdx.x == 0) out[i] = vv[0];
}

// w -= sum_{i<nv} h[i] v_i ; optionally accumulate ||w||^2 partials into dots
template <typename T>
__global__ __launch_bounds__(256) void k_maxpy(const T* __restrict__ V, T* __restrict__ w, size_t N,
                                               const double* __restrict__ h, int nv, double* dots,
                                               const SolverState* st) {
  if (st && st->done) return;
  const size_t base = (size_t)blockIdx.x * kChunkElems;
  double nrm = 0.0;
  for (int e = threadIdx.x; e < kChunkElems; e += 256) {
    const size_t idx = base + e;
    if (idx < N) {
      double acc = (double)w[idx];
      for (int i = 0; i < nv; ++i) acc -= h[i] * (double)V[(size_t)i * N + idx];
      const T wn = (T)acc;
      w[idx] = wn;
      nrm += (double)wn * (double)wn;
    }
  }
  if (dots) {
    double vv[1] = {nrm};
    __shared__ double sh[4];
    block_sum256<1>(vv, sh);
    if (threadIdx.x == 0) dots[blockIdx.x] = vv[0];
  }
}

// out = sum_{i<nv} y[i] v_i  (nv read from the state: the inner steps done)
template <typename T>
__global__ __launch_bounds__(256) void k_lincomb(const T* __restrict__ V, T* __restrict__ out,
                                                 size_t N, const double* __restrict__ y,
                                                 const SolverState* st) {
  const int nv = st->j;
  for (size_t idx = blockIdx.x * (size_t)256 + threadIdx.x; idx < N;
       idx += (size_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int i = 0; i < nv; ++i) acc += y[i] * (double)V[(size_t)i * N + idx];
    out[idx] = (T)acc;
  }
}

// x += z
template <typename T>
__global__ void k_add(T* __restrict__ x, const T* __restrict__ z, size_t N, const SolverState* st) {
  if (st->j == 0) return;
  for (size_t idx = blockIdx.x * (size_t)256 + threadIdx.x; idx < N; idx += (size_t)gridDim.x * 256)
    x[idx] = (T)((double)x[idx] + (double)z[idx]);
}

// v <- v * (1 / norm) where norm = sqrt(sum of dots[0..chunks)) (computed per block, fixed order)
template <typename T>
__global__ __launch_bounds__(256) void k_scale_by(T* __restrict__ v, size_t N, const double* scale,
                                                  const SolverState* st) {
  if (st && st->done) return;
  const double s = *scale;
  for (size_t idx = blockIdx.x * (size_t)256 + threadIdx.x; idx < N; idx += (size_t)gridDim.x * 256)
    v[idx] = (T)((double)v[idx] * s);
}

// Arnoldi column j: H[i][j] = h1[i] + h2[i] (i <= j), H[j+1][j] = ||w||, Givens.
__global__ void k_givens(double* gm, GmLayout lay, SolverState* st, const double* nrm_dots,
                         int chunks) {
  if (st->done) return;
  const int R = lay.R;
  double* H = lay.H(gm);
  double* cs = lay.cs(gm);
  double* sn = lay.sn(gm);
  double* g = lay.g(gm);
  const double* h1 = lay.h1(gm);
  const double* h2 = lay.h2(gm);
  const int j = st->j;
  double nn = 0.0;
  for (int c = 0; c < chunks; ++c) nn += nrm_dots[c];
  const double wn = sqrt(nn);
  double col[65];
  for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
  col[j + 1] = wn;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[j], col[j + 1]);
  double c = 1.0, s = 0.0;
  if (den != 0.0) { c = col[j] / den; s = col[j + 1] / den; }
  cs[j] = c;
  sn[j] = s;
  col[j] = den;
  col[j + 1] = 0.0;
  for (int i = 0; i <= j + 1 && i <= R; ++i) H[i * R + j] = col[i];
  g[j + 1] = -s * g[j];
  g[j] = c * g[j];
  st->wnorm = wn;
  st->alpha = wn != 0.0 ? 1.0 / wn : 0.0;   // scale for the next basis vector
  st->j = j + 1;
  st->iter += 1;
  const double rr = fabs(g[j + 1]) / st->fnorm;
  st->relres = rr;
  if (st->hist && st->iter <= st->hist_cap) st->hist[st->iter - 1] = rr;
  if (!finite(rr) || !finite(den)) st->done = 3;
  else if (st->fixed) { if (st->iter >= st->max_iter) st->done = 1; }
  else if (rr <= st->tol) st->done = 1;
  else if (st->iter >= st->max_iter) st->done = 2;
  else if (wn == 0.0) st->done = 1;   // lucky breakdown: exact solution in the space
}

// y = H[0:jd,0:jd]^-1 g[0:jd]
__global__ void k_backsub(double* gm, GmLayout lay, const SolverState* st) {
  const int R = lay.R;
  const int jd = st->j;
  const double* H = lay.H(gm);
  const double* g = lay.g(gm);
  double* y = lay.y(gm);
  for (int i = jd - 1; i >= 0; --i) {
    double acc = g[i];
    for (int k = i + 1; k < jd; ++k) acc -= H[i * R + k] * y[k];
    y[i] = H[i * R + i] != 0.0 ? acc / H[i * R + i] : 0.0;
  }
}

// Start of a cycle: beta = ||v0|| (from dots), g = (beta, 0, ...), scale factor 1/beta.
__global__ void k_cycle_start(double* gm, GmLayout lay, SolverState* st, const double* dots,
                              int chunks, int first) {
  double nn = 0.0;
  for (int c = 0; c < chunks; ++c) nn += dots[c];
  const double beta = sqrt(nn);
  double* g = lay.g(gm);
  for (int i = 0; i <= lay.R; ++i) g[i] = 0.0;
  g[0] = beta;
  st->j = 0;
  st->alpha = beta != 0.0 ? 1.0 / beta : 0.0;
  if (first) {
    st->fnorm = beta;
    st->relres = 1.0;
    if (!finite(beta)) st->done = 3;
    else if (beta == 0.0) { st->done = 1; st->relres = 0.0; }
  }
}

unsigned grid1(size_t N) {
  size_t b = (N + 255) / 256;
  return (unsigned)(b > 8192 ? 8192 : (b == 0 ? 1 : b));
}

template <typename T>
reco_status gmres_impl(Geometry& g, const void* bvoid, void* xvoid, const reco_solve_opts& o,
                       reco_solve_info* info, hipStream_t st, Workspace& w) {
  const size_t N = g.N();
  const int R = o.restart;
  const int chunks = (int)((N + kChunkElems - 1) / kChunkElems);
  GmLayout lay{R};
  // buffers
  if (w.v_cap < R + 1) {
    if (w.V) (void)hipFree(w.V);
    w.V = nullptr;
    w.v_cap = 0;
    if (hipMalloc(&w.V, sizeof(T) * N * (R + 1)) != hipSuccess) {
      (void)hipGetLastError();
      fail(RECO_ENOMEM, "GMRES basis allocation failed");
    }
    w.v_cap = R + 1;
  }
  const size_t gm_need = lay.count(chunks) + 8;
  if (!w.gm || w.gm_cap < gm_need) {
    if (w.gm) (void)hipFree(w.gm);
    w.gm = nullptr;
    w.gm_cap = 0;
    if (hipMalloc((void**)&w.gm, sizeof(double) * gm_need) != hipSuccess) {
      (void)hipGetLastError();
      fail(RECO_ENOMEM, "GMRES scratch allocation failed");
    }
    w.gm_cap = gm_need;
  }
  T* V = (T*)w.V;
  T* x = (T*)xvoid;
  T* f = (T*)w.fvec;
  T* u = (T*)w.tmp;
  double* gm = w.gm;
  double* dots = lay.dots(gm);
  const bool fixed = o.fixed_iters > 0;
  const int limit = fixed ? o.fixed_iters : o.max_iter;
  if (w.hist_cap < limit) {
    if (w.hist) (void)hipFree(w.hist);
    w.hist = nullptr;
    w.hist_cap = 0;
    if (hipMalloc((void**)&w.hist, sizeof(double) * limit) != hipSuccess) {
      (void)hipGetLastError();
      fail(RECO_ENOMEM, "history allocation failed");
    }
    w.hist_cap = limit;
  }
  launch_state_init(w.st, o.tol, limit, fixed ? 1 : 0, o.lambda, w.hist, limit, st);
  launch_fill(x, N, g.f64, 0.0, st);
  const bool ident = o.precond == RECO_PRECOND_NONE;
  const bool hyb = o.precond == RECO_PRECOND_WMG_HYBRID;
  const HybridFactors* hf = hyb ? &ensure_hybrid(g, o.lambda, st) : nullptr;
  HybridScratch* hs = hyb ? &hybrid_scratch(g, w, st) : nullptr;
  // f = W^T b ; v0 = f / ||f||
  {
    BwdArgs ba{};
    ba.sino = bvoid;
    ba.out = f;
    launch_backward(g, BWD_PLAIN, ba, st);
  }
  launch_copy(f, V, N, g.f64, st);
  hipLaunchKernelGGL(k_mdot<T>, dim3(chunks, 1), dim3(256), 0, st, V, V, N, dots, chunks,
                     (const SolverState*)nullptr);
  hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(1), 0, st, gm, lay, w.st, dots, chunks, 1);
  hipLaunchKernelGGL(k_scale_by<T>, dim3(grid1(N)), dim3(256), 0, st, V, N,
                     (const double*)&w.st->alpha, (const SolverState*)w.st);
  HIP_CHECK(hipGetLastError());
  int matvecs = 0;
  int total = 0;
  int cycles = 0;
  for (;;) {
    // ---- one Arnoldi cycle
    int poll_every = o.check_every > 0 ? o.check_every : 4;
    int steps = 0;
    for (int j = 0; j < R && total < limit; ++j) {
      T* vj = V + (size_t)j * N;
      T* wv = V + (size_t)(j + 1) * N;
      if (hyb) {
        hybrid_apply(g, *hf, *hs, vj, w.zP, w.zTP, nullptr, st);
      } else {
        WmgArgs wa{};
        wa.s = vj;
        wa.zP = w.zP;
        wa.zTP = w.zTP;
        wa.lambda = o.lambda;
        wa.identity = ident;
        wa.st = w.st;
        launch_wmg(g, WMG_GMRES, wa, st);
      }
      FwdArgs fa{};
      fa.imgP = w.zP;
      fa.imgTP = w.zTP;
      fa.out = w.q;
      fa.st = w.st;
      launch_forward(g, FWD_PLAIN, fa, st);
      BwdArgs ba{};
      ba.sino = w.q;
      ba.out = wv;
      ba.x = w.zP;
      ba.x_ld = g.ld;
      ba.x_off = kPad;
      ba.sa = 1.0;
      ba.sx = o.lambda;
      ba.st = w.st;
      launch_backward(g, BWD_AXPY, ba, st);
      const int nv = j + 1;
      // CGS2
      double* h1 = lay.h1(gm);
      double* h2 = lay.h2(gm);
      hipLaunchKernelGGL(k_mdot<T>, dim3(chunks, nv), dim3(256), 0, st, V, wv, N, dots, chunks,
                         (const SolverState*)w.st);
      hipLaunchKernelGGL(k_dot_sum, dim3(nv), dim3(256), 0, st, dots, chunks, h1,
                         (const SolverState*)w.st);
      hipLaunchKernelGGL(k_maxpy<T>, dim3(chunks), dim3(256), 0, st, V, wv, N, h1, nv,
                         (double*)nullptr, (const SolverState*)w.st);
      hipLaunchKernelGGL(k_mdot<T>, dim3(chunks, nv), dim3(256), 0, st, V, wv, N, dots, chunks,
                         (const SolverState*)w.st);
      hipLaunchKernelGGL(k_dot_sum, dim3(nv), dim3(256), 0, st, dots, chunks, h2,
                         (const SolverState*)w.st);
      hipLaunchKernelGGL(k_maxpy<T>, dim3(chunks), dim3(256), 0, st, V, wv, N, h2, nv,
                         dots + (size_t)(R + 1) * chunks, (const SolverState*)w.st);
      hipLaunchKernelGGL(k_givens, dim3(1), dim3(1), 0, st, gm, lay, w.st,
                         dots + (size_t)(R + 1) * chunks, chunks);
      hipLaunchKernelGGL(k_scale_by<T>, dim3(grid1(N)), dim3(256), 0, st, wv, N,
                         (const double*)&w.st->alpha, (const SolverState*)w.st);
      HIP_CHECK(hipGetLastError());
      ++steps;
      ++total;
      if (steps % poll_every == 0) {
        HIP_CHECK(hipMemcpyAsync(w.h_st, w.st, sizeof(SolverState), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        if (w.h_st->done) break;
      }
    }
    // ---- end of cycle: x += M^-1 (V y)
    hipLaunchKernelGGL(k_backsub, dim3(1), dim3(1), 0, st, gm, lay, (const SolverState*)w.st);
    hipLaunchKernelGGL(k_lincomb<T>, dim3(grid1(N)), dim3(256), 0, st, V, u, N,
                       (const double*)lay.y(gm), (const SolverState*)w.st);
    if (hyb) {
      hybrid_apply(g, *hf, *hs, u, nullptr, nullptr, w.s, st);
    } else {
      WmgArgs wa{};
      wa.s = u;
      wa.z = w.s;
      wa.lambda = o.lambda;
      wa.identity = ident;
      launch_wmg(g, WMG_PLAIN, wa, st);
    }
    hipLaunchKernelGGL(k_add<T>, dim3(grid1(N)), dim3(256), 0, st, x, (const T*)w.s, N,
                       (const SolverState*)w.st);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(w.h_st, w.st, sizeof(SolverState), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    matvecs = w.h_st->iter + cycles;
    if (w.h_st->done || w.h_st->iter >= limit) break;
    // ---- restart from the true residual r = f - (W^T W + lambda) x
    ++cycles;
    launch_pad_transpose(g, x, w.xP, w.xTP, st);
    FwdArgs fa{};
    fa.imgP = w.xP;
    fa.imgTP = w.xTP;
    fa.out = w.q;
    launch_forward(g, FWD_PLAIN, fa, st);
    BwdArgs ba{};
    ba.sino = w.q;
    ba.out = V;
    ba.x = x;
    ba.x_ld = g.n;
    ba.x_off = 0;
    ba.f = f;
    ba.sa = -1.0;
    ba.sx = -o.lambda;
    ba.sf = 1.0;
    launch_backward(g, BWD_AXPY, ba, st);
    hipLaunchKernelGGL(k_mdot<T>, dim3(chunks, 1), dim3(256), 0, st, V, V, N, dots, chunks,
                       (const SolverState*)nullptr);
    hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(1), 0, st, gm, lay, w.st, dots, chunks, 0);
    hipLaunchKernelGGL(k_scale_by<T>, dim3(grid1(N)), dim3(256), 0, st, V, N,
                       (const double*)&w.st->alpha, (const SolverState*)nullptr);
    HIP_CHECK(hipGetLastError());
  }
  const SolverState& s = *w.h_st;
  if (o.history && o.history_cap > 0 && s.iter > 0) {
    const int cnt = std::min(std::min(o.history_cap, s.iter), w.hist_cap);
    HIP_CHECK(hipMemcpyAsync(o.history, w.hist, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
  }
  if (info) {
    info->iters = s.iter;
    info->matvecs = matvecs;
    info->relres = s.relres;
    info->status = s.done == 1 ? RECO_OK : (s.done == 3 ? RECO_ENUMERIC : RECO_ENOTCONV);
    info->reserved = 0;
  }
  return s.done == 1 ? RECO_OK : (s.done == 3 ? RECO_ENUMERIC : RECO_ENOTCONV);
}

}  // namespace

reco_status solve_gmres(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                        reco_solve_info* info, hipStream_t st) {
  if (!(o.tol > 0.0) && o.fixed_iters <= 0) fail(RECO_EINVAL, "tol must be > 0");
  if (o.max_iter < 1 && o.fixed_iters <= 0) fail(RECO_EINVAL, "max_iter must be >= 1");
  if (o.restart < 1 || o.restart > 64) fail(RECO_EINVAL, "restart must be in [1, 64]");
  if (!(o.lambda >= 0.0)) fail(RECO_EINVAL, "lambda must be >= 0");
  if (o.precond != RECO_PRECOND_NONE && o.precond != RECO_PRECOND_WMG &&
      o.precond != RECO_PRECOND_WMG_HYBRID)
    fail(RECO_EINVAL, "unknown preconditioner");
  const auto t0 = std::chrono::steady_clock::now();
  Workspace* w = checkout_workspace(g, st);
  reco_status rc;
  try {
    ensure_aux(g, *w);
    rc = g.f64 ? gmres_impl<double>(g, b, x, o, info, st, *w)
               : gmres_impl<float>(g, b, x, o, info, st, *w);
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
