// Forward projector q = W x (Section 2.1, eq. sys), ray driven, matrix free.
//
// One thread per ray; a wave holds 64 consecutive detector bins of one angle,
// a block 4 consecutive angles.  Each ray is walked along its major axis: at
// every row (or column, for angles closer to the x axis, via a transposed image
// copy so that the wave's loads stay contiguous) the ray overlaps exactly two
// candidate pixels, floor(P) and floor(P)+1, where P is the crossing position
// in pixel units.  With f = P - floor(P) the exact intersection lengths are
//   w0 = h clamp((1/2 - f) B + C, 0, 1/u),  w1 = h/u - w0,
// u = |major direction cosine|, B = 1/v, C = 1/(2u), v = |minor cosine|
// (the trapezoid of the chord length versus offset; the two weights of a row
// always sum to the row's chord h/u).  Images are read with two zero columns
// of padding on each side so rays leaving the image need no masking.
//
// Positions are walked in 32.32 fixed point (float path) or float64 (double
// path), so the geometry error stays far below the float weight error.
#include "device_common.h"
#include "timing.h"

namespace reco {

namespace {

constexpr int kFwdWaves = 4;

template <typename T>
struct FwdK {
  const T* imgP;
  const T* imgTP;
  T* out;
  const T* b;
  const T* R;
  const FwdAngle* ang;
  SolverState* st;
  RedScratch red;
  unsigned long long* count;
  int n, ld, nb, m;
  double h;
};

template <typename T>
struct Walker;

template <>
struct Walker<float> {
  long long p, dp;
  __device__ void init(double P, const FwdAngle& a) {
    p = __double2ll_rn(P * 4294967296.0);
    dp = a.dP;
  }
  __device__ int idx() const { return (int)(p >> 32); }
  __device__ float frac() const {
    return (float)(unsigned)(p & 0xffffffffll) * 2.3283064365386963e-10f;
  }
  __device__ void step() { p += dp; }
};

template <>
struct Walker<double> {
  double P0, slope;
  int r;
  double cur;
  __device__ void init(double P, const FwdAngle& a) {
    P0 = P;
    slope = a.slope;
    r = 0;
    cur = P;
  }
  __device__ int idx() const { return (int)floor(cur); }
  __device__ double frac() const { return cur - floor(cur); }
  __device__ void step() {
    ++r;
    cur = fma((double)r, slope, P0);
  }
};

template <typename T>
__device__ __forceinline__ T wB(const FwdAngle& a);
template <>
__device__ __forceinline__ float wB<float>(const FwdAngle& a) { return a.Bf; }
template <>
__device__ __forceinline__ double wB<double>(const FwdAngle& a) { return a.B; }
template <typename T>
__device__ __forceinline__ T wC(const FwdAngle& a);
template <>
__device__ __forceinline__ float wC<float>(const FwdAngle& a) { return a.Cf; }
template <>
__device__ __forceinline__ double wC<double>(const FwdAngle& a) { return a.C; }
template <typename T>
__device__ __forceinline__ T wM(const FwdAngle& a);
template <>
__device__ __forceinline__ float wM<float>(const FwdAngle& a) { return a.Wmaxf; }
template <>
__device__ __forceinline__ double wM<double>(const FwdAngle& a) { return a.Wmax; }

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_forward(FwdK<T> a) {
  if (a.st && a.st->done) return;   // solver finished: later launches are no-ops
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.y * kFwdWaves + (threadIdx.x >> 6);
  const int j = blockIdx.x * 64 + lane;
  const int n = a.n;
  const bool valid = (k < a.m) && (j < a.nb);
  T result = T(0);
  unsigned long long cnt = 0;
  if (k < a.m) {
    const FwdAngle ang = a.ang[k];
    const T* __restrict__ img = ang.major ? a.imgTP : a.imgP;
    const double P0 = fma((double)j, ang.inv, ang.A0);
    int lo = n, hi = -1;
    if (valid) {
      if (ang.slope == 0.0) {
        if (P0 >= -1.5 && P0 <= n + 0.5) { lo = 0; hi = n - 1; }
      } else {
        const double t1 = (-1.5 - P0) / ang.slope, t2 = (n + 0.5 - P0) / ang.slope;
        const double tl = fmin(t1, t2), th = fmax(t1, t2);
        lo = (int)fmin(fmax(0.0, ceil(tl)), (double)n);
        hi = (int)fmax(fmin((double)(n - 1), floor(th)), -1.0);
      }
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    const T B = wB<T>(ang), C = wC<T>(ang), Wm = wM<T>(ang);
    T acc0 = T(0), acc1 = T(0);
    if (lo <= hi) {
      Walker<T> w;
      w.init(fma((double)lo, ang.slope, P0), ang);
      const T* __restrict__ row = img + (size_t)lo * a.ld + 2;
      for (int r = lo; r <= hi; ++r) {
        const int i0 = min(max(w.idx(), -2), n);
        const T f = w.frac();
        const T w0 = clamp01<T>(fma(T(0.5) - f, B, C), Wm);
        if constexpr (MODE == FWD_COUNT) {
          const T w1 = Wm - w0;
          const T eps = T(1e-9) * Wm;
          cnt += (w0 > eps && i0 >= 0 && i0 < n) ? 1 : 0;
          cnt += (w1 > eps && i0 + 1 >= 0 && i0 + 1 < n) ? 1 : 0;
        } else {
          const T x0 = row[i0], x1 = row[i0 + 1];
          acc0 = fma(w0, x0 - x1, acc0);
          acc1 += x1;
        }
        w.step();
        row += a.ld;
      }
    }
    result = (T)a.h * fma(Wm, acc1, acc0);
  }
  const size_t i = (size_t)k * a.nb + j;
  if constexpr (MODE == FWD_PLAIN) {
    if (valid) a.out[i] = result;
  } else if constexpr (MODE == FWD_SIRT) {
    if (valid) a.out[i] = (T)((double)a.R[i] * ((double)a.b[i] - (double)result));
  } else if constexpr (MODE == FWD_COUNT) {
    double v[1] = {(double)cnt};
    __shared__ double sh[4];
    block_sum256<1>(v, sh);
    if (threadIdx.x == 0) atomicAdd(a.count, (unsigned long long)v[0]);
  } else if constexpr (MODE == FWD_CGLS) {
    // q = W z + beta q_old  (q_old = W p_old, so q = W (z + beta p_old) = W p_new)
    double q = 0.0;
    if (valid) {
      q = (double)result + a.st->beta * (double)a.out[i];
      a.out[i] = (T)q;
      q = (double)(T)q;
    }
    double v[1] = {q * q};
    SolverState* st = a.st;
    const int nblk = gridDim.x * gridDim.y;
    reduce_and_finish<1>(v, a.red, nblk, blockIdx.y * gridDim.x + blockIdx.x,
                         [st](double (&tot)[1]) {
                           const double delta = tot[0] + st->lambda * st->pp;
                           st->delta = delta;
                           if (!finite(delta)) {
                             st->done = 3;
                             st->alpha = 0.0;
                           } else if (delta <= 0.0) {
                             st->done = 1;   // zero direction: nothing left to do
                             st->alpha = 0.0;
                           } else {
                             st->alpha = st->gamma / delta;
                           }
                         });
  }
}

// x[n][n] -> xP[n][ld] (2 zero columns on each side) and its transpose xTP.
template <typename T>
__global__ __launch_bounds__(256) void k_pad_transpose(const T* __restrict__ x, T* __restrict__ xP,
                                                       T* __restrict__ xTP, int n, int ld) {
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ty + 8 * i;
    const int iy = y0 + r, ix = x0 + tx;
    T v = T(0);
    if (iy < n && ix < n) {
      v = x[(size_t)iy * n + ix];
      xP[(size_t)iy * ld + ix + 2] = v;
    }
    tile[r][tx] = v;
  }
  // pad columns
  if (blockIdx.x == 0 && threadIdx.x < 32) {
    const int iy = y0 + threadIdx.x;
    if (iy < n) {
      xP[(size_t)iy * ld + 0] = T(0);
      xP[(size_t)iy * ld + 1] = T(0);
      xP[(size_t)iy * ld + n + 2] = T(0);
      xP[(size_t)iy * ld + n + 3] = T(0);
      xTP[(size_t)iy * ld + 0] = T(0);
      xTP[(size_t)iy * ld + 1] = T(0);
      xTP[(size_t)iy * ld + n + 2] = T(0);
      xTP[(size_t)iy * ld + n + 3] = T(0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ty + 8 * i;
    const int ox = x0 + r, oy = y0 + tx;  // output row = original column
    if (ox < n && oy < n) xTP[(size_t)ox * ld + oy + 2] = tile[tx][r];
  }
}

template <typename T>
FwdK<T> make_args(const Geometry& g, const FwdArgs& a) {
  FwdK<T> k;
  k.imgP = (const T*)a.imgP;
  k.imgTP = (const T*)a.imgTP;
  k.out = (T*)a.out;
  k.b = (const T*)a.b;
  k.R = (const T*)a.R;
  k.ang = g.d_fwd;
  k.st = a.st;
  k.red = a.red;
  k.count = a.count;
  k.n = g.n;
  k.ld = g.ld;
  k.nb = g.nb;
  k.m = g.m;
  k.h = g.h;
  return k;
}

template <typename T>
void fwd_dispatch(const Geometry& g, FwdMode mode, const FwdArgs& a, hipStream_t st) {
  dim3 grid((g.nb + 63) / 64, (g.m + kFwdWaves - 1) / kFwdWaves);
  FwdK<T> k = make_args<T>(g, a);
  TimedLaunch tl(TK_FORWARD, st);
  switch (mode) {
    case FWD_PLAIN: hipLaunchKernelGGL((k_forward<T, FWD_PLAIN>), grid, dim3(256), 0, st, k); break;
    case FWD_CGLS: hipLaunchKernelGGL((k_forward<T, FWD_CGLS>), grid, dim3(256), 0, st, k); break;
    case FWD_SIRT: hipLaunchKernelGGL((k_forward<T, FWD_SIRT>), grid, dim3(256), 0, st, k); break;
    case FWD_COUNT: hipLaunchKernelGGL((k_forward<T, FWD_COUNT>), grid, dim3(256), 0, st, k); break;
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace

int forward_blocks(const Geometry& g) {
  return ((g.nb + 63) / 64) * ((g.m + kFwdWaves - 1) / kFwdWaves);
}

void launch_forward(const Geometry& g, FwdMode mode, const FwdArgs& a, hipStream_t st) {
  if (g.f64) fwd_dispatch<double>(g, mode, a, st);
  else fwd_dispatch<float>(g, mode, a, st);
}

void launch_pad_transpose(const Geometry& g, const void* x, void* xP, void* xTP, hipStream_t st) {
  dim3 grid((g.n + 31) / 32, (g.n + 31) / 32);
  TimedLaunch tl(TK_PREP, st);
  if (g.f64)
    hipLaunchKernelGGL(k_pad_transpose<double>, grid, dim3(256), 0, st, (const double*)x,
                       (double*)xP, (double*)xTP, g.n, g.ld);
  else
    hipLaunchKernelGGL(k_pad_transpose<float>, grid, dim3(256), 0, st, (const float*)x,
                       (float*)xP, (float*)xTP, g.n, g.ld);
  HIP_CHECK(hipGetLastError());
}

}  // namespace reco
