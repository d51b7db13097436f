// Wavelet multigrid preconditioner, additive form with packet-diagonal
// coarsest solves:  z = H_L^T diag(1/(d + lambda)) H_L s.
//
// H_L is the full Haar packet transform of L = ell - 1 levels (eq. intops,
// eq. intops_wav, eq. 1of4 - 4of4, recursed into every subband as in Section
// 3.1.3).  Each of its basis functions is a +-2^-L Walsh pattern on one
// T x T pixel tile (T = 2^L), so the transform is a tile-local 2D
// Walsh-Hadamard transform.  Coefficients are kept "in place": the
// coefficient stored at pixel (iy, ix) belongs to tile (iy >> L, ix >> L) and
// its level-l code in x (y) is bit l-1 of ix (iy) within the tile (0 = scaling
// function, 1 = wavelet).
//
// d_q = ||W H_L^T e_q||^2 is the diagonal of the Galerkin operators of the
// coarsest subproblems in the packet basis (eq. galerkin).  It is computed once
// per geometry, tile by tile: for every angle and every detector bin crossing a
// tile, the tile's weights are Walsh-transformed by the lanes that hold the
// tile (one row per lane); their squares are summed per angle and added to
// float64 sums, in a fixed order (deterministic, no atomics).
#include <algorithm>

#include "device_common.h"
#include "timing.h"

namespace reco {

namespace {

// ------------------------------- apply ------------------------------------
template <typename T>
struct WmgK {
  const T* s;
  T* z;
  T* zP;
  T* zTP;
  const T* pold;
  const T* d;
  SolverState* st;
  RedScratch red;
  int n, ld;
  int L;           // packet levels (batched launches dispatch on it)
  int identity;    // 1: no preconditioner (batched launches dispatch on it)
  double lambda;
};

template <typename T, int L>
__device__ __forceinline__ void wht_region(T (&tile)[32][33]) {
  // butterflies along x (columns within rows) then along y
#pragma unroll
  for (int b = 0; b < L; ++b) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int pidx = threadIdx.x + 256 * q;   // 512 pairs: 32 rows x 16 pairs
      const int row = pidx >> 4, pi = pidx & 15;
      const int xa = ((pi >> b) << (b + 1)) | (pi & ((1 << b) - 1));
      const int xb = xa | (1 << b);
      const T u = tile[row][xa], v = tile[row][xb];
      tile[row][xa] = u + v;
      tile[row][xb] = u - v;
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < L; ++b) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int pidx = threadIdx.x + 256 * q;
      const int col = pidx & 31, pi = pidx >> 5;
      const int ya = ((pi >> b) << (b + 1)) | (pi & ((1 << b) - 1));
      const int yb = ya | (1 << b);
      const T u = tile[ya][col], v = tile[yb][col];
      tile[ya][col] = u + v;
      tile[yb][col] = u - v;
    }
    __syncthreads();
  }
}

template <typename T, int L, int MODE, bool IDENT>
__device__ __forceinline__ void wmg_body(const WmgK<T>& a, const BlockPos bp) {
  if (a.st && a.st->done) return;   // solver finished: later launches are no-ops
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x0 = bp.x * 32, y0 = bp.y * 32;
  const int n = a.n;
  T sv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ty + 8 * i, iy = y0 + r, ix = x0 + tx;
    sv[i] = (iy < n && ix < n) ? a.s[(size_t)iy * n + ix] : T(0);
    tile[r][tx] = sv[i];
  }
  __syncthreads();
  if constexpr (!IDENT) {
    wht_region<T, L>(tile);
    const double scale = 1.0 / (double)(1u << (2 * L));   // 4^-L, exact
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = ty + 8 * i, iy = y0 + r, ix = x0 + tx;
      double inv = 0.0;
      if (iy < n && ix < n) {
        const double dd = (double)a.d[(size_t)iy * n + ix] + a.lambda;
        inv = dd != 0.0 ? scale / dd : 0.0;
      }
      tile[r][tx] = (T)((double)tile[r][tx] * inv);
    }
    __syncthreads();
    wht_region<T, L>(tile);
  }
  T zv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ty + 8 * i, iy = y0 + r, ix = x0 + tx;
    zv[i] = tile[r][tx];
    if (iy < n && ix < n) {
      if (a.z) a.z[(size_t)iy * n + ix] = zv[i];
      if (a.zP) a.zP[(size_t)iy * a.ld + ix + kPad] = zv[i];
    }
  }
  if (a.zTP) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = ty + 8 * i;
      const int ox = x0 + r, oy = y0 + tx;
      if (ox < n && oy < n) a.zTP[(size_t)ox * a.ld + oy + kPad] = tile[tx][r];
    }
  }
  if constexpr (MODE == WMG_CGLS || MODE == WMG_CGLS_INIT) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};   // <s,z>, ||s||^2, ||z||^2, <z,p_old>
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = ty + 8 * i, iy = y0 + r, ix = x0 + tx;
      const double s = (double)sv[i], z = (double)zv[i];
      v[0] += s * z;
      v[1] += s * s;
      v[2] += z * z;
      if (MODE == WMG_CGLS && a.lambda != 0.0 && iy < n && ix < n)
        v[3] += z * (double)a.pold[(size_t)iy * n + ix];
    }
    SolverState* st = a.st;
    reduce_and_finish<4>(v, a.red, bp.count(), bp.id(), [st](double (&t)[4]) {
      cgls_precond_finish(st, t, MODE == WMG_CGLS_INIT,
                          MODE == WMG_CGLS ? cgls_degenerate(st->delta) : 0);
    });
  }
}

template <typename T, int L, int MODE, bool IDENT>
__global__ __launch_bounds__(256) void k_wmg(WmgK<T> a) {
  wmg_body<T, L, MODE, IDENT>(a, grid_pos());
}

// Batched apply: the level count and the preconditioner switch are per problem.
template <int MODE>
__global__ __launch_bounds__(256) void k_wmg_batch(const WmgK<float>* __restrict__ args,
                                                   const int* __restrict__ start,
                                                   const int* __restrict__ gx, int count) {
  const int r = batch_find(start, count, blockIdx.x);
  const WmgK<float>& a = args[r];
  const BlockPos bp = batch_pos(start, gx, r);
  if (a.identity) {
    wmg_body<float, 0, MODE, true>(a, bp);
    return;
  }
  switch (a.L) {
    case 0: wmg_body<float, 0, MODE, false>(a, bp); break;
    case 1: wmg_body<float, 1, MODE, false>(a, bp); break;
    case 2: wmg_body<float, 2, MODE, false>(a, bp); break;
    case 3: wmg_body<float, 3, MODE, false>(a, bp); break;
    case 4: wmg_body<float, 4, MODE, false>(a, bp); break;
    default: wmg_body<float, 5, MODE, false>(a, bp); break;
  }
}

template <typename T>
WmgK<T> wmg_args(const Geometry& g, const WmgArgs& a) {
  WmgK<T> k;
  k.s = (const T*)a.s;
  k.z = (T*)a.z;
  k.zP = (T*)a.zP;
  k.zTP = (T*)a.zTP;
  k.pold = (const T*)a.pold;
  k.d = (const T*)g.d_diag;
  k.st = a.st;
  k.red = a.red;
  k.n = g.n;
  k.ld = g.ld;
  k.L = g.L;
  k.identity = a.identity ? 1 : 0;
  k.lambda = a.lambda;
  return k;
}

template <typename T, int L>
void wmg_launch_L(const Geometry& g, WmgMode mode, const WmgArgs& a, hipStream_t st) {
  const WmgK<T> k = wmg_args<T>(g, a);
  dim3 grid((g.n + 31) / 32, (g.n + 31) / 32);
  TimedLaunch tl(TK_WMG, st);
#define RECO_WMG_CASE(M)                                                                   \
  case M:                                                                                  \
    if (a.identity) hipLaunchKernelGGL((k_wmg<T, L, M, true>), grid, dim3(256), 0, st, k); \
    else hipLaunchKernelGGL((k_wmg<T, L, M, false>), grid, dim3(256), 0, st, k);           \
    break;
  switch (mode) {
    RECO_WMG_CASE(WMG_PLAIN)
    RECO_WMG_CASE(WMG_CGLS)
    RECO_WMG_CASE(WMG_CGLS_INIT)
    RECO_WMG_CASE(WMG_GMRES)
  }
#undef RECO_WMG_CASE
  HIP_CHECK(hipGetLastError());
}

template <typename T>
void wmg_launch(const Geometry& g, WmgMode mode, const WmgArgs& a, hipStream_t st) {
  switch (a.identity ? 0 : g.L) {
    case 0: wmg_launch_L<T, 0>(g, mode, a, st); break;
    case 1: wmg_launch_L<T, 1>(g, mode, a, st); break;
    case 2: wmg_launch_L<T, 2>(g, mode, a, st); break;
    case 3: wmg_launch_L<T, 3>(g, mode, a, st); break;
    case 4: wmg_launch_L<T, 4>(g, mode, a, st); break;
    case 5: wmg_launch_L<T, 5>(g, mode, a, st); break;
    default: fail(RECO_EINVAL, "unsupported number of packet levels");
  }
}

// The unit clamp, which the compiler folds into the producing FMA's output
// clamp modifier.
__device__ __forceinline__ float unit_clamp(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 1.0f); }
__device__ __forceinline__ double unit_clamp(double v) { return fmin(fmax(v, 0.0), 1.0); }

// y stages of the transform.  Stage b exchanges with lane y ^ m_b, where the
// masks m_b = 1, 2, 7, 8, 16 (a basis of the tile's lane indices) each take
// one DPP move (2^2 = 4 would take two).  In the coordinates y' of y over
// that basis (y'_0 = y_0 ^ y_2, y'_1 = y_1 ^ y_2, y'_b = y_b otherwise) the
// stages are the butterflies of a Walsh-Hadamard transform along y'_b, the
// lane with y'_b = 0 keeping u + v: afterwards lane y holds, up to sign, the
// coefficient of y frequency ywalsh_row(y) (the squares are summed, so the
// sign does not matter).
template <int B>
constexpr int kYMask = B == 2 ? 7 : 1 << B;
__device__ __forceinline__ int ywalsh_role(int y, int b) {
  return b < 2 ? ((y >> b) ^ (y >> 2)) & 1 : (y >> b) & 1;
}
template <int L>
__device__ __forceinline__ int ywalsh_row(int y) {
  if constexpr (L < 3) return y;
  const int y0 = y & 1, y1 = (y >> 1) & 1, y2 = (y >> 2) & 1;
  return (y & ~7) | (y0 ^ y2) | ((y1 ^ y2) << 1) | ((y0 ^ y1 ^ y2) << 2);
}
template <typename T, int L, int B = 0>
__device__ __forceinline__ void y_stages(T (&w)[1 << L], const T (&sgn)[L > 0 ? L : 1]) {
  if constexpr (B < L) {
#pragma unroll
    for (int x = 0; x < (1 << L); ++x) w[x] = fma(sgn[B], w[x], xor_lane<kYMask<B>>(w[x]));
    y_stages<T, L, B + 1>(w, sgn);
  }
}

// --------------------------- packet diagonal --------------------------------
// Lane layout: a tile of T x T pixels (T = 2^L) is held by T consecutive
// lanes, lane y holding the tile's row y with its T pixels in registers, so a
// wave holds 64 / T tiles.  For every angle and every bin that reaches a
// tile, the tile's weights are Walsh-Hadamard transformed (x stages within
// the registers of a lane, y stages across the tile's lanes); the squares are
// summed per angle in the tile's precision and added to float64 sums, in a
// fixed order (deterministic, no atomics).
// The x butterflies keep the low element as u + v and the high one as u - v,
// so x frequency u lands in register u; each lane stores its sums in the row
// of the y frequency it holds (y_stages), so the sums take the in-place layout
// of the apply (x frequency u at tile column u, y frequency v at tile row v).
//
// Symmetries of the geometry cut the work by about eight (N tiles per side;
// tile (tx, ty); each map below changes only the signs of the Walsh
// coefficients, which are squared, or exchanges u and v).
//  - Bins are centred on the rotation centre, so the tile mirrored through the
//    image centre sees, at every angle, the mirrored weights of bin
//    nb - 1 - j: equal sums, so only the tiles t < ceil(N^2 / 2) (row-major
//    index) are computed.
//  - Angle m - k is angle k reflected left-right: on tile T it gives angle k's
//    sums of X T = (N - 1 - tx, ty).
//  - With m even, angle k + m/2 is angle k turned by a quarter (on T: angle
//    k's sums of R T = (ty, N - 1 - tx), u and v exchanged), and so angle
//    m/2 - k is angle k reflected about the diagonal (on T: angle k's sums of
//    the transposed tile (ty, tx), u and v exchanged).
// So with A = sum of d_k over k = 0 .. floor(m/4) (m even) or
// k = 0 .. (m - 1)/2 (m odd), angle 0 and, when 4 divides m, angle m/4
// weighted 1/2 (the maps send them to themselves or to each other),
//   d(T) = A(T) + A(X T)                                   (m odd)
//   d(T) = A(T) + A(X T) + A(T^T)^T + A(R T)^T              (m even).
// k_diag_assemble forms these sums.
// One launch covers angles [k0, k1) of that range: the running float64 sums,
// compact per computed tile ([tile][row][column]), are kept in memory between
// launches (first: start from zero).  The angle order, hence the result, does
// not depend on how the angles are split over launches.
template <typename T, int L>
__global__ __launch_bounds__(256) void k_packet_diag(const BwdAngle* __restrict__ ang, double* S,
                                                     int n, int nb, int k0, int k1, int first,
                                                     int nh, int khalf) {
  constexpr int Tt = 1 << L;
  constexpr int TPW = 64 / Tt;   // tiles per wave
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tiles_x = n / Tt;
  const int tile = (blockIdx.x * 4 + wv) * TPW + lane / Tt;
  const int y = lane & (Tt - 1);
  const bool active = tile < nh;
  const int tyT = active ? tile / tiles_x : 0, txT = active ? tile % tiles_x : 0;
  const double hc = 0.5 * (n - 1), hb = 0.5 * (nb - 1);
  const double Xt = txT * Tt + 0.5 * (Tt - 1) - hc;   // tile centre, pixel units
  const double Yt = tyT * Tt + 0.5 * (Tt - 1) - hc;
  const T dY = T(y - 0.5 * (Tt - 1));
  T sgn[L > 0 ? L : 1];   // y stage b: +1 keeps u + v (low lane), -1 gives u - v (high lane)
#pragma unroll
  for (int b = 0; b < L; ++b) sgn[b] = ywalsh_role(y, b) ? T(-1) : T(1);
  // this lane's row of the tile's sums: that of the y frequency it ends with
  double* const mine = S + ((size_t)tile * Tt + ywalsh_row<L>(y)) * Tt;
  double acc[Tt];
#pragma unroll
  for (int x = 0; x < Tt; ++x) acc[x] = (first || !active) ? 0.0 : mine[x];

  for (int k = k0; k < k1; ++k) {
    const BwdAngle A = ang[k];
    const double Jt = fma(Xt, A.c, fma(Yt, A.s, hb));
    const double jbase = floor(Jt);
    const T rel = (T)(Jt - jbase);
    T c, s;
    if constexpr (sizeof(T) == 4) { c = A.cf; s = A.sf; }
    else { c = A.c; s = A.s; }
    // the trapezoid w = clamp(cc - dist inv_uv, 0, Wmax) divided by its
    // plateau: the unit clamp is the weight FMA's output clamp, and Wmax^2
    // scales the angle's sums of squares
    const T Bn = (T)(A.inv_uv_d / A.Wmax), Cn = (T)(A.cc_d / A.Wmax);
    const T by = fma(dY, s, rel);
    T Jp[Tt];
#pragma unroll
    for (int x = 0; x < Tt; ++x) Jp[x] = fma(T(x - 0.5 * (Tt - 1)), c, by);
    // bins with nonzero weight satisfy |jj - rel| < Tt * (u+v)/2 (+1 for rel in [0,1))
    const double reach = Tt * A.half_u_plus_v;
    const int jlo = (int)floor(-reach), jhi = (int)ceil(1.0 + reach);
    const int jb = (int)jbase;
    T part[Tt];   // this angle's sums of squares (a few dozen terms)
#pragma unroll
    for (int x = 0; x < Tt; ++x) part[x] = T(0);
    for (int jj = jlo; jj <= jhi; ++jj) {
      const int j = jb + jj;
      const bool inb = active && j >= 0 && j < nb;
      // a bin off the detector (or an idle lane) gets weight 0 through its intercept
      const T Ce = inb ? Cn : T(-1e30);
      T w[Tt];
#pragma unroll
      for (int x = 0; x < Tt; ++x) w[x] = unit_clamp(fma(-fabs(T(jj) - Jp[x]), Bn, Ce));
#pragma unroll
      for (int b = 0; b < L; ++b) {   // along x, in registers
#pragma unroll
        for (int x = 0; x < Tt; ++x) {
          if (!(x & (1 << b))) {
            const T u = w[x], v = w[x | (1 << b)];
            w[x] = u + v;
            w[x | (1 << b)] = u - v;
          }
        }
      }
      y_stages<T, L>(w, sgn);   // along y, across the tile's lanes
#pragma unroll
      for (int x = 0; x < Tt; ++x) part[x] = fma(w[x], w[x], part[x]);
    }
    const double wk = ((k == 0 || k == khalf) ? 0.5 : 1.0) * A.Wmax * A.Wmax;
#pragma unroll
    for (int x = 0; x < Tt; ++x) acc[x] += wk * (double)part[x];
  }
  if (active) {
#pragma unroll
    for (int x = 0; x < Tt; ++x) mine[x] = acc[x];
  }
}

// d (float64, in-place layout) from the sums A of the computed tiles (a tile
// past them is its mirror's): A(T) + A(X T), plus A(T^T)^T + A(R T)^T when m
// is even, times h^2 4^-L.
template <int L>
__global__ __launch_bounds__(256) void k_diag_assemble(const double* __restrict__ S,
                                                       double* __restrict__ d64, int n, int even,
                                                       double scale) {
  constexpr int Tt = 1 << L;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)n * n) return;
  const int iy = (int)(i / n), ix = (int)(i % n);
  const int N = n >> L, nt = N * N, nh = (nt + 1) / 2;
  const int tx = ix >> L, ty = iy >> L, u = ix & (Tt - 1), v = iy & (Tt - 1);
  auto tile = [&](int t) { return S + (size_t)(t < nh ? t : nt - 1 - t) * Tt * Tt; };
  double sum = tile(ty * N + tx)[v * Tt + u];              // A(T)
  sum += tile(ty * N + (N - 1 - tx))[v * Tt + u];          // A(X T)
  if (even) {
    sum += tile(tx * N + ty)[u * Tt + v];                  // A(T^T)^T, T^T = (ty, tx)
    sum += tile((N - 1 - tx) * N + ty)[u * Tt + v];        // A(R T)^T, R T = (ty, N - 1 - tx)
  }
  d64[i] = sum * scale;
}

template <typename T>
__global__ __launch_bounds__(256) void k_diag_round(const double* __restrict__ d64,
                                                    T* __restrict__ dT, size_t count) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) dT[i] = (T)d64[i];
}

// The angles are split over launches of about a millisecond each: every block
// of a launch stays resident for the whole launch, so kernels of other
// streams (the solves of a server) get the CUs between launches.  The running
// sums live in the memory of the dtype copy of d (diag_sum_bytes), which is
// written last.
template <typename T, int L>
void diag_launch_L(Geometry& g, hipStream_t st) {
  const int ntiles = (g.n >> L) * (g.n >> L);
  const int nh = (ntiles + 1) / 2;
  const int even = g.m % 2 == 0 ? 1 : 0;
  // angles summed: 0 .. floor(m/4) (m even) or 0 .. (m - 1)/2 (m odd); angle 0
  // and, when 4 divides m, angle m/4 with weight 1/2
  const int mh = even ? g.m / 4 + 1 : (g.m - 1) / 2 + 1;
  const int khalf = g.m % 4 == 0 ? g.m / 4 : -1;
  double* S = (double*)g.d_diag;
  const int tiles_per_block = 4 * (64 >> L);
  const int blocks = (nh + tiles_per_block - 1) / tiles_per_block;
  // butterfly work of one angle: tiles x bins reaching a tile x 4^L * 2L;
  // about 1.5e13 of these per second (measured at 2048^2, 2^L = 16)
  const double Tt = (double)(1 << L);
  const double per_angle = (double)nh * (1.2 * Tt + 3.0) * Tt * Tt * (2.0 * L + 1.0);
  const int per_launch = (int)std::max(1.0, std::min((double)mh, 1.5e10 / per_angle));
  for (int k0 = 0; k0 < mh; k0 += per_launch) {
    const int k1 = std::min(mh, k0 + per_launch);
    TimedLaunch tl(TK_PACKET_DIAG, st);
    hipLaunchKernelGGL((k_packet_diag<T, L>), dim3(blocks), dim3(256), 0, st, g.d_bwd, S, g.n,
                       g.nb, k0, k1, k0 == 0 ? 1 : 0, nh, khalf);
    HIP_CHECK(hipGetLastError());
  }
  const size_t N = (size_t)g.n * g.n;
  const unsigned eblocks = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL((k_diag_assemble<L>), dim3(eblocks), dim3(256), 0, st, S, g.d_diag64, g.n,
                     even, g.h * g.h / (double)(1u << (2 * L)));
  HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL((k_diag_round<T>), dim3(eblocks), dim3(256), 0, st, g.d_diag64, (T*)g.d_diag,
                     N);
  HIP_CHECK(hipGetLastError());
}

template <typename T>
void diag_launch(Geometry& g, hipStream_t st) {
  switch (g.L) {
    case 0: diag_launch_L<T, 0>(g, st); break;
    case 1: diag_launch_L<T, 1>(g, st); break;
    case 2: diag_launch_L<T, 2>(g, st); break;
    case 3: diag_launch_L<T, 3>(g, st); break;
    case 4: diag_launch_L<T, 4>(g, st); break;
    case 5: diag_launch_L<T, 5>(g, st); break;
    default: fail(RECO_EINVAL, "unsupported number of packet levels");
  }
}

}  // namespace

int wmg_blocks(const Geometry& g) {
  const int t = (g.n + 31) / 32;
  return t * t;
}

void launch_wmg(const Geometry& g, WmgMode mode, const WmgArgs& a, hipStream_t st) {
  if (g.f64) wmg_launch<double>(g, mode, a, st);
  else wmg_launch<float>(g, mode, a, st);
}

void prepare_wmg_batch(DevTable& t, const std::vector<const Geometry*>& gs,
                       const std::vector<WmgArgs>& as, hipStream_t st) {
  std::vector<WmgK<float>> host(gs.size());
  std::vector<int> blocks(gs.size()), widths(gs.size());
  for (size_t i = 0; i < gs.size(); ++i) {
    if (gs[i]->f64) fail(RECO_EINVAL, "batched solves take float32 geometries");
    if (gs[i]->L > 5) fail(RECO_EINVAL, "unsupported number of packet levels");
    host[i] = wmg_args<float>(*gs[i], as[i]);
    widths[i] = (gs[i]->n + 31) / 32;
    blocks[i] = widths[i] * widths[i];
  }
  t.upload(host.data(), sizeof(WmgK<float>), blocks, widths, st);
}

void launch_wmg_batch(const DevTable& t, WmgMode mode, hipStream_t st) {
  if (t.count == 0) return;
  TimedLaunch tl(TK_WMG, st);
  const auto* args = (const WmgK<float>*)t.args;
  switch (mode) {
    case WMG_CGLS:
      hipLaunchKernelGGL(k_wmg_batch<WMG_CGLS>, dim3(t.total_blocks), dim3(256), 0, st, args,
                         t.start, t.gx, t.count);
      break;
    case WMG_CGLS_INIT:
      hipLaunchKernelGGL(k_wmg_batch<WMG_CGLS_INIT>, dim3(t.total_blocks), dim3(256), 0, st, args,
                         t.start, t.gx, t.count);
      break;
    default: fail(RECO_EINVAL, "unsupported batched WMG mode");
  }
  HIP_CHECK(hipGetLastError());
}

size_t diag_sum_bytes(int n, int L) {
  const size_t N = (size_t)(n >> L);
  return sizeof(double) * ((N * N + 1) / 2) * ((size_t)1 << (2 * L));
}

void compute_packet_diagonal(Geometry& g, hipStream_t st) {
  if (g.f64) diag_launch<double>(g, st);
  else diag_launch<float>(g, st);
}

}  // namespace reco
