// Streaming vector kernels of the Krylov solvers (HBM bound): fills, copies,
// the fused CGLS update, reciprocal with 1/0 := 0, state initialisation.
// Update arithmetic is done in float64 and rounded to the storage type.
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

// p = z + beta p; x += alpha p   (pixels, blocks [0, nbN))
// r -= alpha q                   (rays,   blocks [nbN, ...))
template <typename T>
__global__ __launch_bounds__(256) void k_cgls_update(T* __restrict__ x, T* __restrict__ p,
                                                     const T* __restrict__ zP, T* __restrict__ r,
                                                     const T* __restrict__ q, const SolverState* st,
                                                     int n, int ld, size_t M, int nbN) {
  if (st->done) return;
  const double alpha = st->alpha, beta = st->beta;
  if ((int)blockIdx.x < nbN) {
    const size_t N = (size_t)n * n;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < N) {
      const size_t iy = i / n, ix = i % n;
      const double z = (double)zP[iy * ld + ix + kPad];
      const T pn = (T)(z + beta * (double)p[i]);
      p[i] = pn;
      x[i] = (T)((double)x[i] + alpha * (double)pn);
    }
  } else {
    const size_t i = (size_t)(blockIdx.x - nbN) * 256 + threadIdx.x;
    if (i < M) r[i] = (T)((double)r[i] - alpha * (double)q[i]);
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

void launch_cgls_update(const Geometry& g, void* x, void* p, const void* zP, void* r, const void* q,
                        SolverState* st, hipStream_t s) {
  const int nbN = (int)((g.N() + 255) / 256);
  const int nbM = (int)((g.M() + 255) / 256);
  TimedLaunch tl(TK_UPDATE, s);
  if (g.f64)
    hipLaunchKernelGGL(k_cgls_update<double>, dim3(nbN + nbM), dim3(256), 0, s, (double*)x,
                       (double*)p, (const double*)zP, (double*)r, (const double*)q, st, g.n, g.ld,
                       g.M(), nbN);
  else
    hipLaunchKernelGGL(k_cgls_update<float>, dim3(nbN + nbM), dim3(256), 0, s, (float*)x,
                       (float*)p, (const float*)zP, (float*)r, (const float*)q, st, g.n, g.ld,
                       g.M(), nbN);
  HIP_CHECK(hipGetLastError());
}

void launch_state_init(SolverState* st, double tol, int max_iter, int fixed, double lambda,
                       double* hist, int hist_cap, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, tol, max_iter, fixed, lambda, hist,
                     hist_cap);
  HIP_CHECK(hipGetLastError());
}

}  // namespace reco
