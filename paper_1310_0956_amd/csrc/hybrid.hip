// The hybrid wavelet multigrid cycle with exact coarsest solves (Section
// 3.1.2, hybrid variant; recursion of Section 3.1.3; Cholesky coarsest solves
// of Section 4.1), used as a right preconditioner by BiCGStab and GMRES.
//
// Coefficient layout: the L-level full Haar packet transform of an image is
// the tile-local 2D Walsh-Hadamard transform of its 2^L x 2^L tiles, scaled by
// 2^-L; the coefficient of packet (py, px) of tile (ty, tx) sits at pixel
// (ty 2^L + py, tx 2^L + px).  Bit l of py (px) is the band (0 low, 1 high)
// along y (x) at level l + 1, so the subproblems of depth l of the recursion
// are the sets of positions whose local index has given low l bits: node P =
// (cy, cx) at depth l owns the positions with (py, px) mod 2^l = (cy, cx), its
// LL child the ones with bit l of both zero, LH bit l of px set, HL of py, HH
// of both.  The Galerkin operator of node P, R_P K R_P^T with
// K = W^T W + lambda I, is applied on the fine grid: the node's vector is
// synthesised into an image, projected, backprojected (plus lambda times the
// image) and analysed again.  The coarsest problems (one packet over all
// tiles, c = (n / 2^L)^2 unknowns) are solved with the inverse Cholesky
// factors built at set-up: A_p^-1 = X^T X, X = L^-1.
//
// The cycle on node P with residual r (coefficients on P's positions):
//   depth L:  e = A_P^-1 r
//   else:     e_LL = cycle(P LL, r);  r' = r - A_P e_LL  (on the LH, HL, HH
//             positions);  e_id = cycle(P id, r') for id = LH, HL, HH.
//
// Set-up (float64): A_p[i][j] = v_j^T K v_i, v_i the packet-p basis image of
// tile i (its Walsh pattern times 2^-L), formed for every packet and tile pair
// in the packet domain from the projection weights (k_galerkin_pairs); then a
// Cholesky factorisation of every block in natural order in which pivots at
// most 1e-12 of the largest coarsest diagonal entry are dropped (not
// eliminated; zero correction), then X = L^-1 and its transpose; both run
// right looking in panels of 16 steps.
#include <cmath>
#include <map>
#include <memory>

#include "device_common.h"
#include "hybrid.h"
#include "solve.h"

namespace reco {

namespace {

// ---------------------------------------------------------------------------
// Tile-local Walsh-Hadamard transform (orthonormal; its own inverse)
// ---------------------------------------------------------------------------
struct WhtArgs {
  const void* src;
  int src_ld, src_off;           // source [n][src_ld], image column 0 at src_off
  void* dst;
  int dst_ld, dst_off;
  void* dstT;                    // transposed copy (same ld / offset), may be null
  const void* base;              // subtract mode: dst = base - transform
  int n, tiles;
  int in_depth, in_cy, in_cx;    // input mask: keep positions with this prefix (depth 0: all)
  int sub;                       // subtract mode on the positions with prefix
  int out_depth, out_cy, out_cx; // (out_depth, out_c) except its LL child's
};

template <typename T, int TS>
__global__ __launch_bounds__(256) void k_tile_wht(WhtArgs a) {
  const int tile = blockIdx.x * 256 + threadIdx.x;
  if (tile >= a.tiles * a.tiles) return;
  const int ty = tile / a.tiles, tx = tile - ty * a.tiles;
  const T* __restrict__ src = (const T*)a.src;
  const int mi = (1 << a.in_depth) - 1;
  T v[TS][TS];
#pragma unroll
  for (int qy = 0; qy < TS; ++qy) {
#pragma unroll
    for (int qx = 0; qx < TS; ++qx) {
      const size_t iy = (size_t)ty * TS + qy, ix = (size_t)tx * TS + qx;
      T val = src[iy * a.src_ld + a.src_off + ix];
      if ((qy & mi) != a.in_cy || (qx & mi) != a.in_cx) val = T(0);
      v[qy][qx] = val;
    }
  }
#pragma unroll
  for (int b = 1; b < TS; b <<= 1) {
#pragma unroll
    for (int qy = 0; qy < TS; ++qy) {
#pragma unroll
      for (int qx = 0; qx < TS; ++qx) {
        if (qx & b) continue;
        const T u = v[qy][qx], w = v[qy][qx | b];
        v[qy][qx] = u + w;
        v[qy][qx | b] = u - w;
      }
    }
  }
#pragma unroll
  for (int b = 1; b < TS; b <<= 1) {
#pragma unroll
    for (int qy = 0; qy < TS; ++qy) {
      if (qy & b) continue;
#pragma unroll
      for (int qx = 0; qx < TS; ++qx) {
        const T u = v[qy][qx], w = v[qy | b][qx];
        v[qy][qx] = u + w;
        v[qy | b][qx] = u - w;
      }
    }
  }
  const T scale = T(1) / T(TS);   // 2^-L, exact
  T* __restrict__ dst = (T*)a.dst;
  T* __restrict__ dstT = (T*)a.dstT;
  const T* __restrict__ base = (const T*)a.base;
  const int mo = (1 << a.out_depth) - 1, hb = 1 << a.out_depth;
#pragma unroll
  for (int qy = 0; qy < TS; ++qy) {
#pragma unroll
    for (int qx = 0; qx < TS; ++qx) {
      const size_t iy = (size_t)ty * TS + qy, ix = (size_t)tx * TS + qx;
      const T val = v[qy][qx] * scale;
      if (!a.sub) {
        dst[iy * a.dst_ld + a.dst_off + ix] = val;
        if (dstT) dstT[ix * a.dst_ld + a.dst_off + iy] = val;
      } else if ((qy & mo) == a.out_cy && (qx & mo) == a.out_cx && ((qy & hb) | (qx & hb))) {
        dst[iy * a.n + ix] = base[iy * a.n + ix] - val;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Coarsest solves: y = X r_p (gathered from a coefficient image), then
// e_p = XT y (scattered into one), for up to three packets per launch.
// ---------------------------------------------------------------------------
constexpr int kLeafRows = 16;   // rows per block (4 per wave)

struct LeafArgs {
  const double* M;        // X (first pass) or XT (second pass), [leaves][c][c]
  const void* coef_in;    // first pass: coefficient image to gather from
  double* y;              // [3][c]: first pass output, second pass input
  void* coef_out;         // second pass: coefficient image to scatter into
  int n, tiles, c, TS;
  int py[3], px[3];
};

template <typename T, bool SECOND>
__global__ __launch_bounds__(256) void k_leaf(LeafArgs a) {
  extern __shared__ double vin[];
  const int lf = blockIdx.y;
  const int py = a.py[lf], px = a.px[lf];
  const double* __restrict__ Mb = a.M + (size_t)(py * a.TS + px) * a.c * a.c;
  for (int k = threadIdx.x; k < a.c; k += 256) {
    if constexpr (!SECOND) {
      const int ky = k / a.tiles, kx = k - ky * a.tiles;
      vin[k] = (double)((const T*)a.coef_in)[((size_t)ky * a.TS + py) * a.n +
                                               (size_t)kx * a.TS + px];
    } else {
      vin[k] = a.y[(size_t)lf * a.c + k];
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int rr = 0; rr < kLeafRows / 4; ++rr) {
    const int i = blockIdx.x * kLeafRows + wave * (kLeafRows / 4) + rr;
    if (i >= a.c) break;   // uniform per wave
    const double* __restrict__ row = Mb + (size_t)i * a.c;
    // X is lower triangular (k <= i), XT upper (k >= i)
    const int k0 = SECOND ? i : 0, k1 = SECOND ? a.c : i + 1;
    double s = 0.0;
    for (int k = k0 + lane; k < k1; k += 64) s = fma(row[k], vin[k], s);
    s = wave_sum(s);
    if (lane == 0) {
      if constexpr (!SECOND) {
        a.y[(size_t)lf * a.c + i] = s;
      } else {
        const int iy = i / a.tiles, ix = i - iy * a.tiles;
        ((T*)a.coef_out)[((size_t)iy * a.TS + py) * a.n + (size_t)ix * a.TS + px] = (T)s;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Set-up kernels (float64)
// ---------------------------------------------------------------------------
// The Galerkin blocks directly in the packet domain.  The basis vector of
// packet p = (py, px) on tile i is the Hadamard pattern (-1)^(popc(qy & py) +
// popc(qx & px)) / TS on the tile's pixels (qy, qx), and these vectors are
// orthonormal, so A_p[i][i'] = <W v_p,i, W v_p,i'> + lambda [i = i'].  Row
// (k, j) of W holds h times the trapezoid weight of each pixel's bin distance
// (the weight of the projectors), so (W v_p,i) at ray (k, j) is h / TS times
// the Hadamard coefficient p of the tile's weights for that ray, and
//   A_p[i][i'] = h^2 / 4^L  sum_k sum_j H_p(i; k, j) H_p(i'; k, j)
// over the rays that meet both tiles.  One group of TS lanes per tile pair
// i <= i' (pairs in row order, so a wave's pairs share i and have
// neighbouring i'): lane y holds row y of each tile's weights, transformed
// along x in registers and along y across the group's lanes (lane y, register
// x ends with coefficient (py, px) = (y, x)); the products are summed over the
// angles in order and the common bins in order.  Every entry is written by
// one group, A_p[i'][i] = A_p[i][i'] beside it.
template <int L>
__global__ __launch_bounds__(256) void k_galerkin_pairs(const BwdAngle* __restrict__ ang,
                                                        double* __restrict__ S, int n, int nb,
                                                        int m, long long npairs, double scale,
                                                        double lambda) {
  constexpr int Tt = 1 << L;
  constexpr int PPW = 64 / Tt;   // pairs per wave
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long pq = ((long long)blockIdx.x * 4 + wv) * PPW + lane / Tt;
  const int y = lane & (Tt - 1);
  const int tiles = n / Tt, c = tiles * tiles;
  const bool active = pq < npairs;
  // pair index -> (a, b), a <= b: row a starts at a c - a (a - 1) / 2
  long long a = 0, b = 0;
  if (active) {
    const double cc2 = 2.0 * c + 1.0;
    a = (long long)((cc2 - sqrt(cc2 * cc2 - 8.0 * (double)pq)) * 0.5);
    auto start = [&](long long r) { return r * c - r * (r - 1) / 2; };
    while (a > 0 && start(a) > pq) --a;
    while (a + 1 < c && start(a + 1) <= pq) ++a;
    b = pq - start(a) + a;
  }
  const double hc = 0.5 * (n - 1), hb = 0.5 * (nb - 1);
  const int tya = (int)(a / tiles), txa = (int)(a % tiles);
  const int tyb = (int)(b / tiles), txb = (int)(b % tiles);
  const double Xa = txa * Tt + 0.5 * (Tt - 1) - hc, Ya = tya * Tt + 0.5 * (Tt - 1) - hc;
  const double Xb = txb * Tt + 0.5 * (Tt - 1) - hc, Yb = tyb * Tt + 0.5 * (Tt - 1) - hc;
  const double dY = y - 0.5 * (Tt - 1);
  double sgn[L > 0 ? L : 1];   // y stage q: +1 keeps u + v (low lane), -1 gives u - v (high lane)
#pragma unroll
  for (int q = 0; q < L; ++q) sgn[q] = ((y >> q) & 1) ? -1.0 : 1.0;
  double acc[Tt];
#pragma unroll
  for (int x = 0; x < Tt; ++x) acc[x] = 0.0;
  // Hadamard coefficients of the weights of bin j on the tile whose row y has
  // bin coordinates J[x]
  auto coeffs = [&](const double (&J)[Tt], int j, double inv_uv, double cc, double wm,
                    double (&w)[Tt]) {
#pragma unroll
    for (int x = 0; x < Tt; ++x) w[x] = fmin(fmax(fma(-fabs((double)j - J[x]), inv_uv, cc), 0.0), wm);
#pragma unroll
    for (int q = 0; q < L; ++q) {   // along x, in registers
#pragma unroll
      for (int x = 0; x < Tt; ++x) {
        if (!(x & (1 << q))) {
          const double u = w[x], v = w[x | (1 << q)];
          w[x] = u + v;
          w[x | (1 << q)] = u - v;
        }
      }
    }
    // along y, across the group's lanes
    if constexpr (L > 0) {
#pragma unroll
      for (int x = 0; x < Tt; ++x) w[x] = fma(sgn[0], w[x], xor_lane<1>(w[x]));
    }
    if constexpr (L > 1) {
#pragma unroll
      for (int x = 0; x < Tt; ++x) w[x] = fma(sgn[1], w[x], xor_lane<2>(w[x]));
    }
    if constexpr (L > 2) {
#pragma unroll
      for (int x = 0; x < Tt; ++x) w[x] = fma(sgn[2], w[x], xor_lane<4>(w[x]));
    }
  };
  if (active) {
    for (int k = 0; k < m; ++k) {
      const BwdAngle A = ang[k];
      const double Jca = fma(Xa, A.c, fma(Ya, A.s, hb));
      const double Jcb = fma(Xb, A.c, fma(Yb, A.s, hb));
      // bins with nonzero weight on a tile: |j - J| < Tt (u + v) / 2 around its centre
      const double reach = Tt * A.half_u_plus_v;
      const int jlo = max(max((int)floor(Jca - reach), (int)floor(Jcb - reach)), 0);
      const int jhi = min(min((int)ceil(Jca + reach), (int)ceil(Jcb + reach)), nb - 1);
      if (jlo > jhi) continue;   // uniform within the pair's lanes
      double Ja[Tt], Jb[Tt];
      const double bya = fma(dY, A.s, Jca), byb = fma(dY, A.s, Jcb);
#pragma unroll
      for (int x = 0; x < Tt; ++x) {
        const double dX = x - 0.5 * (Tt - 1);
        Ja[x] = fma(dX, A.c, bya);
        Jb[x] = fma(dX, A.c, byb);
      }
      for (int j = jlo; j <= jhi; ++j) {
        double wa[Tt], wb[Tt];
        coeffs(Ja, j, A.inv_uv_d, A.cc_d, A.Wmax, wa);
        coeffs(Jb, j, A.inv_uv_d, A.cc_d, A.Wmax, wb);
#pragma unroll
        for (int x = 0; x < Tt; ++x) acc[x] = fma(wa[x], wb[x], acc[x]);
      }
    }
#pragma unroll
    for (int x = 0; x < Tt; ++x) {
      const long long p = (long long)y * Tt + x;
      const double v = scale * acc[x] + (a == b ? lambda : 0.0);
      S[(p * c + a) * c + b] = v;
      if (a != b) S[(p * c + b) * c + a] = v;
    }
  }
}

// thr = kHybridDropRel * (largest diagonal entry of all blocks); one block.
__global__ __launch_bounds__(256) void k_drop_threshold(const double* __restrict__ S, int c,
                                                        int leaves, double* thr) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (long long t = threadIdx.x; t < (long long)c * leaves; t += 256) {
    const long long l = t / c, i = t - l * c;
    mx = fmax(mx, S[(l * c + i) * c + i]);
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *thr = kHybridDropRel * sh[0];
}

// The Cholesky factorisation of every block, right looking and worked in the
// upper triangle (S is formed symmetric, and row k is contiguous where column
// k is strided).  Step k writes the column L[i][k] = S[k][i] / sqrt(S[k][k])
// and updates S[j][i] -= S[k][i] S[k][j] / S[k][k] for k < j <= i, unless the
// pivot is at most thr (dropped: column k of L stays zero, nothing is
// eliminated); row k is final after step k - 1.  The steps go in panels of
// kPanel: k_chol_panel applies a panel's steps to the panel rows, k_chol_trail
// applies them to the rows after it, so every entry takes the same updates in
// the same order as step by step while the trailing matrix is read once per
// panel.
constexpr int kPanel = 16;

// Panel K0 .. K0 + P - 1: one thread per column i >= K0 holds that column of
// the panel rows in registers; the pivots and couplings S[k][j] of the panel
// come from its diagonal block, factorised in LDS by every workgroup alike.
// Grid: x over columns, y over blocks.
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ S,
                                                    double* __restrict__ Lf, int c, int K0,
                                                    const double* __restrict__ thr) {
  __shared__ double D[kPanel][kPanel + 1];
  const size_t off = (size_t)blockIdx.y * c * c;
  const int P = min(kPanel, c - K0);
  const double th = *thr;
  const int t = threadIdx.x, dr = t / kPanel, dq = t % kPanel;
  const bool mine = dr < P && dq < P && dq >= dr;
  if (mine) D[dr][dq] = S[off + (size_t)(K0 + dr) * c + K0 + dq];
  __syncthreads();
  for (int r = 0; r + 1 < P; ++r) {   // writes rows past r, reads row r
    const double piv = D[r][r];
    if (mine && dr > r && piv > th) D[dr][dq] -= D[r][dq] * D[r][dr] / piv;
    __syncthreads();
  }
  const int i = K0 + blockIdx.x * 256 + t;
  if (i >= c) return;
  const int rows = min(P, i - K0 + 1);   // panel rows k <= i
  double v[kPanel];
#pragma unroll
  for (int r = 0; r < kPanel; ++r)
    v[r] = r < rows ? S[off + (size_t)(K0 + r) * c + i] : 0.0;
#pragma unroll
  for (int r = 0; r < kPanel; ++r) {
    if (r >= rows) break;
    const double piv = D[r][r];
    if (!(piv > th)) continue;
    const double sik = v[r];
    Lf[off + (size_t)i * c + K0 + r] = sik / sqrt(piv);
#pragma unroll
    for (int q = r + 1; q < kPanel; ++q)
      if (q < rows) v[q] -= sik * D[r][q] / piv;
  }
#pragma unroll
  for (int r = 0; r < kPanel; ++r)
    if (r < rows) S[off + (size_t)(K0 + r) * c + i] = v[r];
}

// The rows K1 <= j <= i after panel K0 (K1 = K0 + P): 16 x 16 tiles of the
// upper triangle, the panel rows over the tile's columns and rows staged in
// LDS.  Grid: x over column tiles, y over row tiles, z over blocks.
__global__ __launch_bounds__(256) void k_chol_trail(double* __restrict__ S, int c, int K0,
                                                    const double* __restrict__ thr) {
  if (blockIdx.y > blockIdx.x) return;   // below the diagonal throughout
  __shared__ double A[kPanel][16], B[kPanel][16], pv[kPanel];
  const size_t off = (size_t)blockIdx.z * c * c;
  const int P = min(kPanel, c - K0), K1 = K0 + P;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i0 = K1 + (int)blockIdx.x * 16, j0 = K1 + (int)blockIdx.y * 16;
  if (ty < P) {
    A[ty][tx] = i0 + tx < c ? S[off + (size_t)(K0 + ty) * c + i0 + tx] : 0.0;
    B[ty][tx] = j0 + tx < c ? S[off + (size_t)(K0 + ty) * c + j0 + tx] : 0.0;
  }
  if (ty == 0 && tx < P) pv[tx] = S[off + (size_t)(K0 + tx) * c + K0 + tx];
  __syncthreads();
  const int i = i0 + tx, j = j0 + ty;
  if (i >= c || j > i) return;
  const double th = *thr;
  double v = S[off + (size_t)j * c + i];
  for (int r = 0; r < P; ++r) {
    const double piv = pv[r];
    if (piv > th) v -= A[r][tx] * B[r][ty] / piv;
  }
  S[off + (size_t)j * c + i] = v;
}

// X = L^-1 for every block, right looking: T starts as the identity, and
// X[k][j] = T[k][j] / L[k][k] once the rows before k have been eliminated;
// step k then subtracts L[i][k] X[k][j] from T[i][j] for i > k, j <= k (the
// same terms in the same order as X[i][j] = (delta_ij - sum_{j<=m<i} L[i][m]
// X[m][j]) / L[i][i]).  A dropped unknown (L[k][k] = 0) gives a zero row of X
// and subtracts nothing.  In panels as the factorisation: k_trinv_panel
// finishes the panel rows, k_trinv_trail updates the rows after them.

// Panel K0 .. K0 + P - 1: one thread per column j < K1 holds that column of
// the panel rows in registers, runs the panel's steps on them and writes them
// as rows of X.  Grid: x over columns, y over blocks.
__global__ __launch_bounds__(256) void k_trinv_panel(const double* __restrict__ Lf,
                                                     double* __restrict__ T, int c, int K0) {
  __shared__ double D[kPanel][kPanel + 1];   // D[q][r] = L[K0 + q][K0 + r]
  const size_t off = (size_t)blockIdx.y * c * c;
  const int P = min(kPanel, c - K0), K1 = K0 + P;
  const int t = threadIdx.x;
  {
    const int q = t / kPanel, r = t % kPanel;
    if (q < P && r < P) D[q][r] = Lf[off + (size_t)(K0 + q) * c + K0 + r];
  }
  __syncthreads();
  const int j = (int)blockIdx.x * 256 + t;
  if (j >= K1) return;
  double v[kPanel];
#pragma unroll
  for (int r = 0; r < kPanel; ++r) v[r] = r < P ? T[off + (size_t)(K0 + r) * c + j] : 0.0;
#pragma unroll
  for (int r = 0; r < kPanel; ++r) {
    if (r >= P) break;
    if (j > K0 + r) continue;   // X[k][j] = 0 above the diagonal: T stays as it is
    const double lkk = D[r][r];
    if (lkk == 0.0) {
      v[r] = 0.0;
      continue;
    }
    const double x = v[r] / lkk;
    v[r] = x;
#pragma unroll
    for (int q = r + 1; q < kPanel; ++q)
      if (q < P) v[q] -= D[q][r] * x;
  }
#pragma unroll
  for (int r = 0; r < kPanel; ++r)
    if (r < P) T[off + (size_t)(K0 + r) * c + j] = v[r];
}

// The rows i >= K1 after panel K0, columns j < K1, in 16 x 16 tiles: L over
// the tile's rows and the panel's X rows over its columns staged in LDS.
// Grid: x over column tiles, y over row tiles, z over blocks.
__global__ __launch_bounds__(256) void k_trinv_trail(const double* __restrict__ Lf,
                                                     double* __restrict__ T, int c, int K0) {
  __shared__ double A[16][kPanel + 1];   // A[y][r] = L[i0 + y][K0 + r]
  __shared__ double B[kPanel][16];       // B[r][x] = X[K0 + r][j0 + x]
  __shared__ double dg[kPanel];
  const size_t off = (size_t)blockIdx.z * c * c;
  const int P = min(kPanel, c - K0), K1 = K0 + P;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int j0 = (int)blockIdx.x * 16, i0 = K1 + (int)blockIdx.y * 16;
  A[ty][tx] = i0 + ty < c && tx < P ? Lf[off + (size_t)(i0 + ty) * c + K0 + tx] : 0.0;
  B[ty][tx] = ty < P && j0 + tx < K1 ? T[off + (size_t)(K0 + ty) * c + j0 + tx] : 0.0;
  if (ty == 0 && tx < P) dg[tx] = Lf[off + (size_t)(K0 + tx) * c + K0 + tx];
  __syncthreads();
  const int i = i0 + ty, j = j0 + tx;
  if (i >= c || j >= K1) return;
  double v = T[off + (size_t)i * c + j];
  for (int r = 0; r < P; ++r)
    if (j <= K0 + r && dg[r] != 0.0) v -= A[ty][r] * B[r][tx];
  T[off + (size_t)i * c + j] = v;
}

// T = I for every block (the start of the inverse).
__global__ __launch_bounds__(256) void k_identity_blocks(double* __restrict__ T, int c) {
  const size_t off = (size_t)blockIdx.z * c * c;
  const int j = blockIdx.x * 16 + threadIdx.x, i = blockIdx.y * 16 + threadIdx.y;
  if (i < c && j < c) T[off + (size_t)i * c + j] = i == j ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void k_transpose_blocks(const double* __restrict__ X,
                                                          double* __restrict__ XT, int c) {
  const size_t off = (size_t)blockIdx.z * c * c;
  const int k = blockIdx.x * 16 + threadIdx.x, i = blockIdx.y * 16 + threadIdx.y;
  if (i < c && k < c) XT[off + (size_t)k * c + i] = X[off + (size_t)i * c + k];
}

__global__ __launch_bounds__(256) void k_count_dropped(const double* __restrict__ X, int c,
                                                       int leaves, int* out) {
  __shared__ int sh[256];
  int cnt = 0;
  for (long long t = threadIdx.x; t < (long long)c * leaves; t += 256) {
    const long long l = t / c, i = t - l * c;
    cnt += X[(l * c + i) * c + i] == 0.0;
  }
  sh[threadIdx.x] = cnt;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
void dalloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    fail(RECO_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
}

template <typename T>
void launch_wht(const WhtArgs& a, int TS, hipStream_t st) {
  const dim3 grid((unsigned)((a.tiles * a.tiles + 255) / 256));
  switch (TS) {
    case 2: hipLaunchKernelGGL((k_tile_wht<T, 2>), grid, dim3(256), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_tile_wht<T, 4>), grid, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((k_tile_wht<T, 8>), grid, dim3(256), 0, st, a); break;
  }
  HIP_CHECK(hipGetLastError());
}

WhtArgs wht_args(const Geometry& g, int tiles) {
  WhtArgs a{};
  a.n = g.n;
  a.tiles = tiles;
  a.src_ld = a.dst_ld = g.n;
  return a;
}

// Cycle state of one apply.
template <typename T>
struct Cycle {
  const Geometry& g;
  const HybridFactors& f;
  HybridScratch& s;
  hipStream_t st;

  void leaves(const void* in, const int (&py)[3], const int (&px)[3], int count) {
    LeafArgs la{};
    la.M = f.X;
    la.coef_in = in;
    la.y = s.y;
    la.coef_out = s.coefE;
    la.n = g.n;
    la.tiles = f.tiles;
    la.c = f.c;
    la.TS = f.TS;
    for (int i = 0; i < 3; ++i) {
      la.py[i] = py[i];
      la.px[i] = px[i];
    }
    const dim3 grid((unsigned)((f.c + kLeafRows - 1) / kLeafRows), (unsigned)count);
    const size_t lds = sizeof(double) * f.c;
    hipLaunchKernelGGL((k_leaf<T, false>), grid, dim3(256), lds, st, la);
    la.M = f.XT;
    hipLaunchKernelGGL((k_leaf<T, true>), grid, dim3(256), lds, st, la);
    HIP_CHECK(hipGetLastError());
  }

  // r' = in - A_P e_LL on the positions of P's LH, HL and HH children, into
  // coefR[l + 1]; e_LL is the correction on P's LL child's positions.
  void residual_update(int l, int cy, int cx, const void* in) {
    WhtArgs a = wht_args(g, f.tiles);
    a.src = s.coefE;
    a.in_depth = l + 1;
    a.in_cy = cy;
    a.in_cx = cx;
    a.dst = s.P;
    a.dstT = s.TP;
    a.dst_ld = g.ld;
    a.dst_off = kPad;
    launch_wht<T>(a, f.TS, st);
    FwdArgs fa{};
    fa.imgP = s.P;
    fa.imgTP = s.TP;
    fa.out = s.sino;
    launch_forward(g, FWD_PLAIN, fa, st);
    BwdArgs ba{};
    ba.sino = s.sino;
    ba.out = s.img;
    ba.x = s.P;
    ba.x_ld = g.ld;
    ba.x_off = kPad;
    ba.sa = 1.0;
    ba.sx = f.lambda;
    launch_backward(g, BWD_AXPY, ba, st);
    WhtArgs b = wht_args(g, f.tiles);
    b.src = s.img;
    b.dst = s.coefR[l + 1];
    b.base = in;
    b.sub = 1;
    b.out_depth = l;
    b.out_cy = cy;
    b.out_cx = cx;
    launch_wht<T>(b, f.TS, st);
  }

  void run(int l, int cy, int cx, const void* in) {
    if (l == f.L) {
      const int py[3] = {cy, 0, 0}, px[3] = {cx, 0, 0};
      leaves(in, py, px, 1);
      return;
    }
    const int hb = 1 << l;
    run(l + 1, cy, cx, in);   // LL
    residual_update(l, cy, cx, in);
    const void* r2 = s.coefR[l + 1];
    // LH (high along x), HL (high along y), HH
    const int hy[3] = {cy, cy | hb, cy | hb}, hx[3] = {cx | hb, cx, cx | hb};
    if (l + 1 == f.L) {
      leaves(r2, hy, hx, 3);
    } else {
      for (int i = 0; i < 3; ++i) run(l + 1, hy[i], hx[i], r2);
    }
  }
};

template <typename T>
void apply_impl(const Geometry& g, const HybridFactors& f, HybridScratch& s, const void* r,
                void* outP, void* outTP, void* outPlain, hipStream_t st) {
  WhtArgs a = wht_args(g, f.tiles);
  a.src = r;
  a.dst = s.coefR[0];
  launch_wht<T>(a, f.TS, st);
  Cycle<T> cyc{g, f, s, st};
  cyc.run(0, 0, 0, s.coefR[0]);
  if (outP) {
    WhtArgs b = wht_args(g, f.tiles);
    b.src = s.coefE;
    b.dst = outP;
    b.dstT = outTP;
    b.dst_ld = g.ld;
    b.dst_off = kPad;
    launch_wht<T>(b, f.TS, st);
  }
  if (outPlain) {
    WhtArgs b = wht_args(g, f.tiles);
    b.src = s.coefE;
    b.dst = outPlain;
    launch_wht<T>(b, f.TS, st);
  }
}

std::unique_ptr<HybridFactors> build_factors(Geometry& g, double lambda, hipStream_t st) {
  auto f = std::make_unique<HybridFactors>();
  f->L = g.L;
  f->TS = 1 << g.L;
  f->tiles = g.n >> g.L;
  f->c = f->tiles * f->tiles;
  f->leaves = f->TS * f->TS;
  f->lambda = lambda;
  const int c = f->c, TS = f->TS;
  const size_t blk = (size_t)f->leaves * c * c;
  double *S = nullptr, *Lf = nullptr, *thr = nullptr;
  int* cnt = nullptr;
  auto release = [&]() {
    for (void* p : {(void*)S, (void*)Lf, (void*)thr, (void*)cnt})
      if (p) (void)hipFree(p);
  };
  try {
    dalloc((void**)&S, sizeof(double) * blk);
    dalloc((void**)&Lf, sizeof(double) * blk);
    dalloc((void**)&thr, sizeof(double));
    dalloc((void**)&cnt, sizeof(int));
    launch_fill(Lf, blk, true, 0.0, st);
    // Galerkin blocks, every packet and tile pair in one launch (float64)
    const long long npairs = (long long)c * (c + 1) / 2;
    const long long per_block = 4LL * (64 / TS);
    const unsigned grid = (unsigned)((npairs + per_block - 1) / per_block);
    const double scale = g.h * g.h / (double)(TS * TS);
    switch (g.L) {
      case 1:
        hipLaunchKernelGGL(k_galerkin_pairs<1>, dim3(grid), dim3(256), 0, st, g.d_bwd, S, g.n,
                           g.nb, g.m, npairs, scale, lambda);
        break;
      case 2:
        hipLaunchKernelGGL(k_galerkin_pairs<2>, dim3(grid), dim3(256), 0, st, g.d_bwd, S, g.n,
                           g.nb, g.m, npairs, scale, lambda);
        break;
      case 3:
        hipLaunchKernelGGL(k_galerkin_pairs<3>, dim3(grid), dim3(256), 0, st, g.d_bwd, S, g.n,
                           g.nb, g.m, npairs, scale, lambda);
        break;
      default: fail(RECO_EINVAL, "unsupported number of hybrid levels");
    }
    HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_drop_threshold, dim3(1), dim3(256), 0, st, (const double*)S, c,
                       f->leaves, thr);
    for (int K0 = 0; K0 < c; K0 += kPanel) {
      const int rest = c - K0 - std::min(kPanel, c - K0);
      hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)((c - K0 + 255) / 256), f->leaves),
                         dim3(256), 0, st, S, Lf, c, K0, (const double*)thr);
      if (rest > 0) {
        const unsigned side = (unsigned)((rest + 15) / 16);
        hipLaunchKernelGGL(k_chol_trail, dim3(side, side, f->leaves), dim3(16, 16), 0, st, S, c,
                           K0, (const double*)thr);
      }
    }
    HIP_CHECK(hipGetLastError());
    // X = L^-1 into S's storage, then X^T into L's
    double* X = S;
    {
      const unsigned sd = (unsigned)((c + 15) / 16);
      hipLaunchKernelGGL(k_identity_blocks, dim3(sd, sd, f->leaves), dim3(16, 16), 0, st, X, c);
    }
    for (int K0 = 0; K0 < c; K0 += kPanel) {
      const int K1 = K0 + std::min(kPanel, c - K0), rest = c - K1;
      hipLaunchKernelGGL(k_trinv_panel, dim3((unsigned)((K1 + 255) / 256), f->leaves), dim3(256),
                         0, st, (const double*)Lf, X, c, K0);
      if (rest > 0)
        hipLaunchKernelGGL(k_trinv_trail,
                           dim3((unsigned)((K1 + 15) / 16), (unsigned)((rest + 15) / 16), f->leaves),
                           dim3(16, 16), 0, st, (const double*)Lf, X, c, K0);
    }
    HIP_CHECK(hipGetLastError());
    double* XT = Lf;
    const unsigned side = (unsigned)((c + 15) / 16);
    hipLaunchKernelGGL(k_transpose_blocks, dim3(side, side, f->leaves), dim3(16, 16), 0, st,
                       (const double*)X, XT, c);
    hipLaunchKernelGGL(k_count_dropped, dim3(1), dim3(256), 0, st, (const double*)X, c,
                       f->leaves, cnt);
    HIP_CHECK(hipGetLastError());
    int dropped = 0;
    HIP_CHECK(hipMemcpyAsync(&dropped, cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    f->dropped = dropped;
    f->X = X;
    f->XT = XT;
    S = Lf = nullptr;
    release();
  } catch (...) {
    (void)hipStreamSynchronize(st);
    release();
    throw;
  }
  return f;
}

}  // namespace

HybridFactors::~HybridFactors() {
  if (X) (void)hipFree(X);
  if (XT) (void)hipFree(XT);
}

HybridScratch::~HybridScratch() {
  for (void* p : coefR)
    if (p) (void)hipFree(p);
  for (void* p : {coefE, img, P, TP, sino, (void*)y})
    if (p) (void)hipFree(p);
}

void validate_hybrid(const Geometry& g) {
  if (g.L < 1 || g.L > kHybridMaxLevels)
    fail(RECO_EINVAL, "the hybrid cycle needs 2 to 4 WMG levels (wmg_levels)");
  const size_t tiles = (size_t)g.n >> g.L, c = tiles * tiles;
  if (c > 4096)
    fail(RECO_EINVAL, "the hybrid cycle's coarsest problems are limited to 4096 unknowns "
                      "((n / 2^(wmg_levels - 1))^2)");
  const size_t bytes = 2 * sizeof(double) * ((size_t)1 << (2 * g.L)) * c * c;
  if (bytes > kHybridMaxFactorBytes)
    fail(RECO_EINVAL, "the hybrid cycle's coarsest factors would need " + std::to_string(bytes) +
                          " bytes (limit " + std::to_string(kHybridMaxFactorBytes) + ")");
}

const HybridFactors& ensure_hybrid(Geometry& g, double lambda, hipStream_t st) {
  validate_hybrid(g);
  std::lock_guard<std::mutex> lk(g.hyb_mu);
  auto it = g.hyb.find(lambda);
  if (it != g.hyb.end()) return *it->second;
  auto f = build_factors(g, lambda, st);
  const HybridFactors& ref = *f;
  g.hyb.emplace(lambda, std::move(f));
  return ref;
}

HybridScratch& hybrid_scratch(const Geometry& g, Workspace& w, hipStream_t st) {
  if (w.hyb) return *w.hyb;
  std::unique_ptr<HybridScratch> s(new HybridScratch());
  const size_t es = g.esize();
  for (int l = 0; l <= g.L; ++l) dalloc(&s->coefR[l], es * g.N());
  dalloc(&s->coefE, es * g.N());
  dalloc(&s->img, es * g.N());
  dalloc(&s->P, es * g.padded_elems());
  dalloc(&s->TP, es * g.padded_elems());
  dalloc(&s->sino, es * g.M());
  const size_t tiles = (size_t)g.n >> g.L;
  dalloc((void**)&s->y, sizeof(double) * 3 * tiles * tiles);
  // zero padding columns of the padded pair; the transforms write interiors
  launch_fill(s->P, g.padded_elems(), g.f64, 0.0, st);
  launch_fill(s->TP, g.padded_elems(), g.f64, 0.0, st);
  w.hyb = s.release();
  return *w.hyb;
}

void hybrid_apply(const Geometry& g, const HybridFactors& f, HybridScratch& s, const void* r,
                  void* outP, void* outTP, void* outPlain, hipStream_t st) {
  if (g.f64) apply_impl<double>(g, f, s, r, outP, outTP, outPlain, st);
  else apply_impl<float>(g, f, s, r, outP, outTP, outPlain, st);
}

}  // namespace reco
