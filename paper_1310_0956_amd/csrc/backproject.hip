// Backprojector s = W^T r (Section 2.1), pixel driven, no atomics.
//
// A block owns a 16 x 16 pixel tile and loops over the angles in chunks of 32.
// For each angle of a chunk the tile's detector footprint (at most 24 bins for
// a 16-pixel tile) is staged in LDS; every pixel then reads its two candidate
// bins floor(J) and floor(J)+1, J being the bin coordinate of the pixel
// centre, and weights them with the same exact intersection length w(t) the
// forward projector uses (trapezoid in the ray offset t), so the result is the
// transpose of the forward matrix up to rounding.  Pixel coordinates are taken
// relative to the tile centre, whose bin coordinate is computed in float64.
#include "device_common.h"
#include "timing.h"

namespace reco {

namespace {

constexpr int kTile = 16;
constexpr int kChunk = 32;   // angles per LDS stage
constexpr int kWin = 32;     // bins staged per angle
constexpr int kHalf = 12;    // window starts kHalf bins below the tile centre

template <typename T>
struct BwdK {
  const T* sino;
  T* out;
  const T* xin;      // extra term source (plain or padded layout)
  const T* fin;      // residual form: right-hand side
  const T* C;        // SIRT: inverse column sums
  const BwdAngle* ang;
  SolverState* st;
  RedScratch red;
  int n, nb, m;
  int x_ld, x_off;   // layout of xin
  double h;
  double sa, sx, sf; // out = sa*(W^T r) + sx*xin + sf*fin
};

template <typename T>
struct BC;
template <>
struct BC<float> {
  float c, s, B, C0, C1, Wm;
  __device__ BC(const BwdAngle& a) : c(a.cf), s(a.sf), B(a.Bf), C0(a.C0f), C1(a.C1f), Wm(a.Wmaxf) {}
};
template <>
struct BC<double> {
  double c, s, B, C0, C1, Wm;
  __device__ BC(const BwdAngle& a) : c(a.c), s(a.s), B(a.B), C0(a.C0), C1(a.C1), Wm(a.Wmax) {}
};

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_backward(BwdK<T> a) {
  if (a.st && a.st->done) return;   // solver finished: later launches are no-ops
  __shared__ T win[kChunk * kWin];
  __shared__ T sbase[kChunk];
  __shared__ int sjw[kChunk];
  const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
  const int ix = blockIdx.x * kTile + tx, iy = blockIdx.y * kTile + ty;
  const int n = a.n, nb = a.nb, m = a.m;
  const double hc = 0.5 * (n - 1), hb = 0.5 * (nb - 1);
  const double Xc = blockIdx.x * kTile + 0.5 * (kTile - 1) - hc;
  const double Yc = blockIdx.y * kTile + 0.5 * (kTile - 1) - hc;
  const T dX = T(tx) - T(0.5 * (kTile - 1)), dY = T(ty) - T(0.5 * (kTile - 1));
  T acc = T(0);
  for (int k0 = 0; k0 < m; k0 += kChunk) {
    const int kc = min(kChunk, m - k0);
    __syncthreads();
    if ((int)threadIdx.x < kc) {
      const BwdAngle A = a.ang[k0 + threadIdx.x];
      const double Jc = fma(Xc, A.c, fma(Yc, A.s, hb));
      const double fl = floor(Jc);
      sjw[threadIdx.x] = (int)fl - kHalf;
      sbase[threadIdx.x] = (T)((Jc - fl) + kHalf);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kc * kWin; e += 256) {
      const int kk = e / kWin, jj = e % kWin;
      const int j = sjw[kk] + jj;
      win[e] = (j >= 0 && j < nb) ? a.sino[(size_t)(k0 + kk) * nb + j] : T(0);
    }
    __syncthreads();
    for (int kk = 0; kk < kc; ++kk) {
      const BC<T> A(a.ang[k0 + kk]);
      const T J = fma(dX, A.c, fma(dY, A.s, sbase[kk]));
      const T fl = floor(J);
      const int j0 = (int)fl;
      const T f = J - fl;
      const T* wp = win + kk * kWin + j0;
      const T r0 = wp[0], r1 = wp[1];
      const T w0 = clamp01<T>(fma(f, -A.B, A.C0), A.Wm);
      const T w1 = clamp01<T>(fma(f, A.B, A.C1), A.Wm);
      acc = fma(w0, r0, acc);
      acc = fma(w1, r1, acc);
    }
  }
  const bool inside = ix < n && iy < n;
  const size_t p = (size_t)iy * n + ix;
  const double bp = a.h * (double)acc;
  if constexpr (MODE == BWD_PLAIN) {
    if (inside) a.out[p] = (T)bp;
  } else if constexpr (MODE == BWD_CGLS) {
    // s = W^T r - lambda x
    if (inside) a.out[p] = (T)(bp - a.st->lambda * (double)a.xin[p]);
  } else if constexpr (MODE == BWD_AXPY) {
    if (inside) {
      double v = a.sa * bp;
      if (a.sx != 0.0) v += a.sx * (double)a.xin[(size_t)iy * a.x_ld + ix + a.x_off];
      if (a.sf != 0.0) v += a.sf * (double)a.fin[p];
      a.out[p] = (T)v;
    }
  } else if constexpr (MODE == BWD_SIRT) {
    // x += C W^T r, with r = R (b - W x) from the forward pass
    double u = 0.0;
    if (inside) {
      u = (double)a.C[p] * bp;
      const T xn = (T)((double)a.out[p] + u);
      u = (double)xn - (double)a.out[p];
      a.out[p] = xn;
    }
    double v[1] = {u * u};
    SolverState* st = a.st;
    reduce_and_finish<1>(v, a.red, gridDim.x * gridDim.y, blockIdx.y * gridDim.x + blockIdx.x,
                         [st](double (&tot)[1]) {
                           const double nrm = sqrt(tot[0]);
                           if (!st->init) {
                             st->s0 = nrm;
                             st->init = 1;
                             if (nrm == 0.0) {   // b = 0: x = 0 is exact, no iteration
                               st->relres = 0.0;
                               st->done = 1;
                               return;
                             }
                           }
                           st->iter += 1;
                           const double rr = st->s0 > 0.0 ? nrm / st->s0 : 0.0;
                           st->relres = rr;
                           if (st->hist && st->iter <= st->hist_cap) st->hist[st->iter - 1] = rr;
                           if (!finite(nrm)) st->done = 3;
                           else if (st->s0 == 0.0) st->done = 1;
                           else if (st->fixed) { if (st->iter >= st->max_iter) st->done = 1; }
                           else if (rr <= st->tol) st->done = 1;
                           else if (st->iter >= st->max_iter) st->done = 2;
                         });
  }
}

template <typename T>
void bwd_dispatch(const Geometry& g, BwdMode mode, const BwdArgs& a, hipStream_t st) {
  BwdK<T> k;
  k.sino = (const T*)a.sino;
  k.out = (T*)a.out;
  k.xin = (const T*)a.x;
  k.fin = (const T*)a.f;
  k.C = (const T*)a.C;
  k.ang = g.d_bwd;
  k.st = a.st;
  k.red = a.red;
  k.n = g.n;
  k.nb = g.nb;
  k.m = g.m;
  k.x_ld = a.x_ld;
  k.x_off = a.x_off;
  k.h = g.h;
  k.sa = a.sa;
  k.sx = a.sx;
  k.sf = a.sf;
  dim3 grid((g.n + kTile - 1) / kTile, (g.n + kTile - 1) / kTile);
  TimedLaunch tl(TK_BACKWARD, st);
  switch (mode) {
    case BWD_PLAIN: hipLaunchKernelGGL((k_backward<T, BWD_PLAIN>), grid, dim3(256), 0, st, k); break;
    case BWD_CGLS: hipLaunchKernelGGL((k_backward<T, BWD_CGLS>), grid, dim3(256), 0, st, k); break;
    case BWD_SIRT: hipLaunchKernelGGL((k_backward<T, BWD_SIRT>), grid, dim3(256), 0, st, k); break;
    case BWD_AXPY: hipLaunchKernelGGL((k_backward<T, BWD_AXPY>), grid, dim3(256), 0, st, k); break;
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace

int backward_blocks(const Geometry& g) {
  const int t = (g.n + kTile - 1) / kTile;
  return t * t;
}

void launch_backward(const Geometry& g, BwdMode mode, const BwdArgs& a, hipStream_t st) {
  if (g.f64) bwd_dispatch<double>(g, mode, a, st);
  else bwd_dispatch<float>(g, mode, a, st);
}

}  // namespace reco
