// Streaming vector kernels of the Krylov solvers (HBM bound): fills, copies,
// reciprocal with 1/0 := 0, state initialisation (also for a whole batch).
#include "device_common.h"
#include "timing.h"

namespace reco {

namespace {

template <typename T>
__global__ void k_fill(T* p, size_t count, T v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
__global__ void k_copy(const T* __restrict__ s, T* __restrict__ d, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

template <typename T>
__global__ void k_invert(T* p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    const T v = p[i];
    p[i] = v != T(0) ? T(1) / v : T(0);
  }
}

// Start of a CGLS solve for one problem of a batch: state, x = p = q = 0, r = b.
struct InitK {
  float *x, *p, *q, *r;
  const float* b;
  SolverState* st;
  double tol, lambda;
  double* hist;
  int max_iter, fixed, hist_cap;
  size_t N, M;
};

__global__ __launch_bounds__(256) void k_init_batch(const InitK* __restrict__ args,
                                                    const int* __restrict__ start,
                                                    const int* __restrict__ gx, int count) {
  const int rr = batch_find(start, count, blockIdx.x);
  const InitK& a = args[rr];
  const int lb = (int)blockIdx.x - start[rr];
  const int nblk = start[rr + 1] - start[rr];
  if (lb == 0 && threadIdx.x == 0) {
    SolverState s{};
    s.tol = a.tol;
    s.max_iter = a.max_iter;
    s.fixed = a.fixed;
    s.lambda = a.lambda;
    s.hist = a.hist;
    s.hist_cap = a.hist_cap;
    *a.st = s;
  }
  const size_t stride = (size_t)nblk * 256;
  for (size_t i = (size_t)lb * 256 + threadIdx.x; i < a.N; i += stride) {
    a.x[i] = 0.0f;
    a.p[i] = 0.0f;
  }
  for (size_t i = (size_t)lb * 256 + threadIdx.x; i < a.M; i += stride) {
    a.q[i] = 0.0f;
    a.r[i] = a.b[i];
  }
}

__global__ void k_state_init(SolverState* st, double tol, int max_iter, int fixed, double lambda,
                             double* hist, int hist_cap) {
  SolverState s{};
  s.tol = tol;
  s.max_iter = max_iter;
  s.fixed = fixed;
  s.lambda = lambda;
  s.hist = hist;
  s.hist_cap = hist_cap;
  *st = s;
}

// CGLS set-up in one launch: the solver state, x = p = 0, q = 0, r = b.
template <typename T>
__global__ __launch_bounds__(256) void k_cgls_prepare(SolverState* st, double tol, int max_iter,
                                                      int fixed, double lambda, double* hist,
                                                      int hist_cap, T* __restrict__ x,
                                                      T* __restrict__ p, T* __restrict__ q,
                                                      T* __restrict__ r, const T* __restrict__ b,
                                                      size_t N, size_t M) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SolverState s{};
    s.tol = tol;
    s.max_iter = max_iter;
    s.fixed = fixed;
    s.lambda = lambda;
    s.hist = hist;
    s.hist_cap = hist_cap;
    *st = s;
  }
  const size_t n = N > M ? N : M;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    if (i < N) {
      x[i] = T(0);
      p[i] = T(0);
    }
    if (i < M) {
      q[i] = T(0);
      r[i] = b[i];
    }
  }
}

unsigned grid_for(size_t count) {
  size_t b = (count + 255) / 256;
  return (unsigned)(b > 65536 ? 65536 : (b == 0 ? 1 : b));
}

}  // namespace

void launch_fill(void* p, size_t count, bool f64, double value, hipStream_t st) {
  if (count == 0) return;
  if (f64) hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(count)), dim3(256), 0, st, (double*)p, count, value);
  else hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(count)), dim3(256), 0, st, (float*)p, count, (float)value);
  HIP_CHECK(hipGetLastError());
}

void launch_copy(const void* src, void* dst, size_t count, bool f64, hipStream_t st) {
  if (count == 0) return;
  if (f64) hipLaunchKernelGGL(k_copy<double>, dim3(grid_for(count)), dim3(256), 0, st, (const double*)src, (double*)dst, count);
  else hipLaunchKernelGGL(k_copy<float>, dim3(grid_for(count)), dim3(256), 0, st, (const float*)src, (float*)dst, count);
  HIP_CHECK(hipGetLastError());
}

void launch_invert(void* v, size_t count, bool f64, hipStream_t st) {
  if (count == 0) return;
  if (f64) hipLaunchKernelGGL(k_invert<double>, dim3(grid_for(count)), dim3(256), 0, st, (double*)v, count);
  else hipLaunchKernelGGL(k_invert<float>, dim3(grid_for(count)), dim3(256), 0, st, (float*)v, count);
  HIP_CHECK(hipGetLastError());
}

void prepare_init_batch(DevTable& t, const std::vector<const Geometry*>& gs,
                        const std::vector<InitArgs>& as, hipStream_t st) {
  std::vector<InitK> host(gs.size());
  std::vector<int> blocks(gs.size()), widths(gs.size());
  for (size_t i = 0; i < gs.size(); ++i) {
    InitK k;
    k.x = (float*)as[i].x;
    k.p = (float*)as[i].p;
    k.q = (float*)as[i].q;
    k.r = (float*)as[i].r;
    k.b = (const float*)as[i].b;
    k.st = as[i].st;
    k.tol = as[i].tol;
    k.lambda = as[i].lambda;
    k.hist = as[i].hist;
    k.max_iter = as[i].max_iter;
    k.fixed = as[i].fixed;
    k.hist_cap = as[i].hist_cap;
    k.N = gs[i]->N();
    k.M = gs[i]->M();
    host[i] = k;
    const size_t big = std::max(k.N, k.M);
    blocks[i] = (int)std::min<size_t>((big + 1023) / 1024, 4096);
    widths[i] = blocks[i];
  }
  t.upload(host.data(), sizeof(InitK), blocks, widths, st);
}

void launch_init_batch(const DevTable& t, hipStream_t st) {
  if (t.count == 0) return;
  hipLaunchKernelGGL(k_init_batch, dim3(t.total_blocks), dim3(256), 0, st,
                     (const InitK*)t.args, t.start, t.gx, t.count);
  HIP_CHECK(hipGetLastError());
}

void launch_cgls_prepare(SolverState* st, double tol, int max_iter, int fixed, double lambda,
                         double* hist, int hist_cap, void* x, void* p, void* q, void* r,
                         const void* b, size_t N, size_t M, bool f64, hipStream_t s) {
  const unsigned grid = grid_for(N > M ? N : M);
  if (f64)
    hipLaunchKernelGGL(k_cgls_prepare<double>, dim3(grid), dim3(256), 0, s, st, tol, max_iter,
                       fixed, lambda, hist, hist_cap, (double*)x, (double*)p, (double*)q,
                       (double*)r, (const double*)b, N, M);
  else
    hipLaunchKernelGGL(k_cgls_prepare<float>, dim3(grid), dim3(256), 0, s, st, tol, max_iter,
                       fixed, lambda, hist, hist_cap, (float*)x, (float*)p, (float*)q, (float*)r,
                       (const float*)b, N, M);
  HIP_CHECK(hipGetLastError());
}

void launch_state_init(SolverState* st, double tol, int max_iter, int fixed, double lambda,
                       double* hist, int hist_cap, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, tol, max_iter, fixed, lambda, hist,
                     hist_cap);
  HIP_CHECK(hipGetLastError());
}

}  // namespace reco
