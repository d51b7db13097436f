// Backprojector s = W^T r (Section 2.1), pixel driven, no atomics.
//
// A block owns a 16 x 16 pixel tile; it holds several angle groups of two
// waves (two pixels per thread), each looping over its contiguous equal share
// of the angles in chunks of 32; their partial sums are added in group order
// at the end (no atomics).  For each angle of a chunk the tile's
// detector footprint (at most 23 bins for a 16-pixel tile) is staged in LDS,
// double buffered: the next chunk's window is fetched into registers while the
// current one is consumed.  The per-angle constants (window start, tile-centre
// bin coordinate, direction cosines, weight coefficients) sit in a three-deep
// LDS ring, filled from angle records fetched two chunks ahead, so no chunk
// waits on them.  Every pixel then reads its two candidate
// bins floor(J) and floor(J)+1, J being the bin coordinate of the pixel
// centre, and weights them with the same weight w(t) the forward projector
// uses (the exact intersection length, a trapezoid in the ray offset t, or
// Joseph's triangle), so the result is the transpose of the forward matrix up
// to rounding.  Pixel coordinates are taken
// relative to the tile centre, whose bin coordinate is computed in float64.
#include "device_common.h"
#include "timing.h"

namespace reco {

namespace {

constexpr int kTile = 16;    // pixels per tile side
constexpr int kThreads = 128; // two pixels per thread: rows ty and ty + 8
constexpr int kChunk = 32;    // angles per LDS stage
constexpr int kWin = 24;      // bins staged per angle: pixel centres lie within
                              // 7.5 (|c| + |s|) <= 7.5 sqrt(2) < 10.61 bins of the
                              // tile centre, so with the window starting kHalf
                              // bins below floor(tile centre) every pixel has
                              // 0.39 < J < 22.61, i.e. 0 <= floor(J), floor(J) + 1 <= 23
constexpr int kHalf = 11;     // window starts kHalf bins below the tile centre
constexpr int kPerThread = kChunk * kWin / kThreads;

template <typename T>
struct BwdK {
  const T* sino;
  T* out;
  const T* q;        // CGLS: projected direction (residual step r - alpha q)
  T* p;              // CGLS: direction
  T* xo;             // CGLS: iterate (updated)
  T* zP;             // CGLS: padded z
  T* zTP;            // CGLS: padded transposed z
  const T* d;        // CGLS: packet diagonal
  int ld, L, identity, fuse;
  const T* xin;      // extra term source (plain or padded layout)
  const T* fin;      // residual form: right-hand side
  const T* C;        // SIRT: inverse column sums
  const BwdAngle* ang;
  const double* fwd_part;   // CGLS: the forward projection's per-block ||q||^2 partials
  int fwd_blocks;
  double* slots;            // CGLS (fused WMG): finisher reduction slots
  SolverState* st;
  RedScratch red;
  int n, nb, m;
  int x_ld, x_off;   // layout of xin
  double h;
  double sa, sx, sf; // out = sa*(W^T r) + sx*xin + sf*fin
};

// Per-angle constants of the current tile, in an LDS ring three chunks deep.
template <typename T>
struct Meta {
  T base;   // bin coordinate of the tile centre minus the window start
  T c, s;   // direction cosines
  T B, C0, C1, Wm;  // weights Wm w0, Wm w1 with w0 = clamp(C0 - f B), w1 = clamp(C1 + f B)
                    // in [0, 1]; Wm multiplies the staged window values
  int jw;   // first bin of the window
};

// The fields of the angle records a chunk's ring entries are filled from,
// fetched by the first wave of each angle group before their use: lane i < 32
// holds the float64 cosines (c, s) of the chunk's angle i, lane 32 + i its
// weight coefficients (B, C0, C1, Wm), in the same registers.
template <typename T>
struct Raw {
  static constexpr int kWords = sizeof(T) == 4 ? 4 : 8;
  unsigned w[kWords];
};

// Called by the group's first wave (t < 64) for the chunk starting at angle k0;
// angles from kend on (the end of the group's share) are not read.
template <typename T>
__device__ __forceinline__ void load_raw(Raw<T>& r, const BwdAngle* __restrict__ ang, int k0,
                                         int t, int kend) {
  const int k = k0 + (t & 31);
  if (k < kend) {
    const BwdAngle& A = ang[k];
    const void* src;
    if constexpr (sizeof(T) == 4) src = t < 32 ? (const void*)&A.c : (const void*)&A.Bf;
    else src = t < 32 ? (const void*)&A.c : (const void*)&A.B;
    const uint2* p = (const uint2*)src;   // 8-byte aligned fields
#pragma unroll
    for (int i = 0; i < Raw<T>::kWords / 2; ++i) {
      const uint2 v = p[i];
      r.w[2 * i] = v.x;
      r.w[2 * i + 1] = v.y;
    }
  }
}

__device__ __forceinline__ double bits_to_double(unsigned lo, unsigned hi) {
  return __hiloint2double((int)hi, (int)lo);
}

// Ring entries of the chunk starting at angle k0 from its records (all lanes
// of the group's first wave take part; lanes t < 32 write entry t, for the
// angles below kend).  The float cosines are the float64 ones rounded to
// nearest, as in the table.
template <typename T>
__device__ __forceinline__ void fill_meta(Meta<T>* __restrict__ ring, const Raw<T>& r, int k0,
                                          int t, int kend, double Xc, double Yc, double hb) {
  Raw<T> up;
#pragma unroll
  for (int i = 0; i < Raw<T>::kWords; ++i) up.w[i] = __shfl_down(r.w[i], 32, 64);
  if (t < kChunk && k0 + t < kend) {
    const double c = bits_to_double(r.w[0], r.w[1]), s = bits_to_double(r.w[2], r.w[3]);
    Meta<T>& M = ring[t];
    const double Jc = fma(Xc, c, fma(Yc, s, hb));
    const double fl = floor(Jc);
    M.jw = (int)fl - kHalf;
    M.base = (T)((Jc - fl) + kHalf);
    M.c = (T)c;
    M.s = (T)s;
    if constexpr (sizeof(T) == 4) {
      M.B = __uint_as_float(up.w[0]);
      M.C0 = __uint_as_float(up.w[1]);
      M.C1 = __uint_as_float(up.w[2]);
      M.Wm = __uint_as_float(up.w[3]);
    } else {
      M.B = bits_to_double(up.w[0], up.w[1]);
      M.C0 = bits_to_double(up.w[2], up.w[3]);
      M.C1 = bits_to_double(up.w[4], up.w[5]);
      M.Wm = bits_to_double(up.w[6], up.w[7]);
    }
  }
}

// The unit clamp, which the compiler folds into the producing FMA's output
// clamp modifier.
__device__ __forceinline__ float clamp01(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 1.0f); }
__device__ __forceinline__ double clamp01(double v) { return fmin(fmax(v, 0.0), 1.0); }

template <typename T>
__device__ __forceinline__ T frac_part(T J) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_fractf(J);
  else return J - floor(J);
}

// One pixel, one angle: the values r0, r1 of the two candidate bins floor(J),
// floor(J)+1 of the window (already multiplied by the angle's plateau Wm),
// weighed by the fraction f = J - floor(J) and accumulated into acc.
template <typename T>
__device__ __forceinline__ T pixel_weigh(T f, T r0, T r1, const Meta<T>& M, T acc) {
  const T w0 = clamp01(fma(f, -M.B, M.C0));
  const T w1 = clamp01(fma(f, M.B, M.C1));
  return fma(w0, r0, fma(w1, r1, acc));
}

// Raw window loads of one chunk.  Thread t stages angle rows t / 8 and
// t / 8 + 16 of the chunk's [kChunk][kWin] window, bins t % 8 + 8 i of each,
// so the lanes of an octet read consecutive bins and a wave's load touches 8
// rows (the cache lines a load touches bound the staging rate); the LDS
// stores of a wave then hit distinct banks.  Bins outside [0, nb) and rows
// past the last angle are read at an offset past the end of the buffer,
// which loads 0; every load is issued unconditionally, so they are all in
// flight together.  In the CGLS modes the projected direction is loaded at
// the same offsets.
constexpr bool kCglsMode(int mode) { return mode == BWD_CGLS || mode == BWD_CGLS_INIT; }
constexpr int kRowLanes = 8;                     // lanes per window row
constexpr int kRowHalf = kChunk / 2;             // the second row of a thread
constexpr int kPerRow = kPerThread / 2;          // elements per row and thread
static_assert(kThreads == kRowLanes * kRowHalf && kWin == kRowLanes * kPerRow,
              "two window rows per octet");

template <typename T, int MODE>
struct Stage {
  T r[kPerThread];
  T q[kCglsMode(MODE) ? kPerThread : 1];
  T wa, wb;   // plateau Wm of the two rows (0 for rows past the last angle)
};

// Buffers of the window loads: the sinogram operand and, in the CGLS modes,
// the projected direction, both [m][nb].
struct StageSrc {
  __amdgpu_buffer_rsrc_t sino, q;
};

template <typename T, int MODE>
__device__ __forceinline__ StageSrc stage_src(const BwdK<T>& a) {
  const size_t bytes = (size_t)a.m * a.nb * sizeof(T);
  StageSrc src;
  src.sino = buffer_rsrc(a.sino, bytes);
  src.q = kCglsMode(MODE) ? buffer_rsrc(a.q, bytes) : src.sino;
  return src;
}

// rowoff = (t / 8) * nb, the offset of the thread's first row within a
// chunk, taken once.  Elements [0, kPerRow) of sg are the first row's,
// [kPerRow, 2 kPerRow) the second's.  Rows from angle kend on (the end of the
// group's share, at most m) load zeros.
template <typename T, int MODE>
__device__ __forceinline__ void stage_load(Stage<T, MODE>& sg, const StageSrc& src,
                                           const Meta<T>* __restrict__ mt, int k0, int kend,
                                           int nb, unsigned rowoff, int t) {
  const int ka = t / kRowLanes, kb = ka + kRowHalf;
  const int ja = mt[ka].jw + (t % kRowLanes), jb = mt[kb].jw + (t % kRowLanes);
  const bool rowa = ka < kend - k0, rowb = kb < kend - k0;
  sg.wa = rowa ? mt[ka].Wm : T(0);
  sg.wb = rowb ? mt[kb].Wm : T(0);
  // byte offsets of bins ja of angle k0 + ka and jb of angle k0 + kb (valid
  // bins lie below 2^31 bytes; rows past the last angle are never read at
  // these offsets)
  const unsigned offa = ((unsigned)k0 * (unsigned)nb + rowoff + (unsigned)ja) * (unsigned)sizeof(T);
  const unsigned offb =
      ((unsigned)(k0 + kRowHalf) * (unsigned)nb + rowoff + (unsigned)jb) * (unsigned)sizeof(T);
  constexpr int kSpan = kRowLanes * (kPerRow - 1);
  const bool full = rowa && rowb && ja >= 0 && ja + kSpan < nb && jb >= 0 && jb + kSpan < nb;
  constexpr unsigned kStep = kRowLanes * sizeof(T);
  if (__builtin_amdgcn_ballot_w64(!full) == 0) {
    // the whole wave's windows lie on the detector (the common case)
#pragma unroll
    for (int i = 0; i < kPerRow; ++i) {
      const unsigned oa = offa + kStep * i, ob = offb + kStep * i;
      sg.r[i] = load_elem(src.sino, oa, 0, T(0));
      sg.r[kPerRow + i] = load_elem(src.sino, ob, 0, T(0));
      if constexpr (kCglsMode(MODE)) {
        sg.q[i] = load_elem(src.q, oa, 0, T(0));
        sg.q[kPerRow + i] = load_elem(src.q, ob, 0, T(0));
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < kPerRow; ++i) {
      unsigned oa = rowa && (unsigned)(ja + kRowLanes * i) < (unsigned)nb ? offa : kOutside;
      unsigned ob = rowb && (unsigned)(jb + kRowLanes * i) < (unsigned)nb ? offb : kOutside;
      // keeps the element's constant offset out of the select, so that it
      // becomes the load's immediate offset
      asm volatile("" : "+v"(oa), "+v"(ob));
      oa += kStep * i;
      ob += kStep * i;
      sg.r[i] = load_elem(src.sino, oa, 0, T(0));
      sg.r[kPerRow + i] = load_elem(src.sino, ob, 0, T(0));
      if constexpr (kCglsMode(MODE)) {
        sg.q[i] = load_elem(src.q, oa, 0, T(0));
        sg.q[kPerRow + i] = load_elem(src.q, ob, 0, T(0));
      }
    }
  }
}

// Window values: the sinogram operand, in the CGLS modes the residual after
// the current step, r - alpha q (the forward projector of the next iteration
// stores the same value up to rounding), times the row's plateau Wm.  In
// float, alpha is split into two floats ah + al (equal to alpha within
// 2^-48 relative): the inner FMA forms r - ah q exactly before its one
// rounding, so the difference, which cancels as the residual shrinks, takes
// only roundings of its own size (alpha rounded to float instead moved
// 5-iteration float32 iterates at 512^2 past 1e-5 of the float64 oracle).
template <typename T, int MODE>
__device__ __forceinline__ void stage_store(const Stage<T, MODE>& sg, T* __restrict__ w,
                                            double alpha, int t) {
  T* row = w + (t / kRowLanes) * kWin + (t % kRowLanes);
  const float ah = (float)alpha, al = (float)(alpha - (double)ah);
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int h = i / kPerRow, e = i % kPerRow;   // row (first or second), element
    const T wm = h ? sg.wb : sg.wa;
    T v;
    if constexpr (kCglsMode(MODE) && sizeof(T) == 4)
      v = fmaf(-al, sg.q[i], fmaf(-ah, sg.q[i], sg.r[i])) * wm;
    else if constexpr (kCglsMode(MODE))
      v = (T)(((double)sg.r[i] - alpha * (double)sg.q[i]) * (double)wm);
    else
      v = sg.r[i] * wm;
    row[h * kRowHalf * kWin + kRowLanes * e] = v;
  }
}

// The WMG apply z = H^T diag(4^-L / (d + lambda)) H s on a 16 x 16 tile (the
// Haar packet transform of every 2^L x 2^L tile is its Walsh-Hadamard
// transform up to the 2^-L scale; 1/0 := 0), by one wave: lane l holds the
// pixels (l % 16, l / 16 + 4 k), k < 4.  Butterflies along x pair lanes
// l and l ^ 2^b (lane moves within rows of 16); along y they pair lanes
// l and l ^ 16 2^b for b < 2 (lane shuffles) and the lane's own values k and
// k ^ 2^(b-2) for b >= 2.  Each butterfly forms u + v and u - v, u the element
// with the lower coordinate; x stages first, then y.
template <typename T, int B>
__device__ __forceinline__ T lane_partner(T v) {
  if constexpr (B < 4) return xor_lane<(1 << B)>(v);
  else return __shfl_xor(v, 1 << B, 64);
}

template <typename T, int B>
__device__ __forceinline__ void butterfly_lanes(T (&v)[4], int lane) {
  const bool upper = (lane >> B) & 1;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T p = lane_partner<T, B>(v[k]);
    v[k] = upper ? p - v[k] : v[k] + p;
  }
}

template <typename T, int B>
__device__ __forceinline__ void butterfly_regs(T (&v)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k & (1 << B)) continue;
    const T u = v[k], w = v[k | (1 << B)];
    v[k] = u + w;
    v[k | (1 << B)] = u - w;
  }
}

template <typename T, int L>
__device__ __forceinline__ void wht_wave(T (&v)[4], int lane) {
  if constexpr (L > 0) butterfly_lanes<T, 0>(v, lane);
  if constexpr (L > 1) butterfly_lanes<T, 1>(v, lane);
  if constexpr (L > 2) butterfly_lanes<T, 2>(v, lane);
  if constexpr (L > 3) butterfly_lanes<T, 3>(v, lane);
  if constexpr (L > 0) butterfly_lanes<T, 4>(v, lane);
  if constexpr (L > 1) butterfly_lanes<T, 5>(v, lane);
  if constexpr (L > 2) butterfly_regs<T, 0>(v);
  if constexpr (L > 3) butterfly_regs<T, 1>(v);
}

// dl[k]: d + lambda of the lane's pixel k (0 outside the image).
template <typename T, int L>
__device__ __forceinline__ void wmg_wave(T (&v)[4], const double (&dl)[4], int lane) {
  wht_wave<T, L>(v, lane);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double inv = dl[k] != 0.0 ? (1.0 / (double)(1u << (2 * L))) / dl[k] : 0.0;
    v[k] = (T)((double)v[k] * inv);
  }
  wht_wave<T, L>(v, lane);
}

// Angle groups per block: group g takes the g-th contiguous share of the
// angles, and the G partial sums of a pixel are added in group order at the
// end.  Two groups amortise a thread's prologue and epilogue over twice the
// angles of four (1% faster at 512^2 and 2048^2 in float; eight were 13%
// slower).
template <typename T>
constexpr int kGroups = 2;

template <typename T, int MODE>
__device__ __forceinline__ void backward_body(const BwdK<T>& a, const BlockPos hw) {
  // the tile of this block: neighbouring tiles on one XCD share sinogram windows in its L2
  const BlockPos pos = xcd_tile(hw);
  constexpr int G = kGroups<T>;
  // Solver state read with vector loads (an opaque zero index keeps them off
  // the scalar path: scalar loads share one out-of-order counter with LDS, so
  // they would be waited for before the first angle records are requested).
  int vzero;
  asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
  // The prologue (loads, barriers, latency bound) runs at the top wave
  // priority: blocks that start late would otherwise wait behind the chunk
  // steps of the blocks already computing, which raise theirs.
  set_priority(3);
  // solver finished: later launches are no-ops (tested once the prologue's
  // first loads are in flight; the flag is the same for every block, and
  // nothing is stored before the test)
  int done_v = 0;
  if (a.st) done_v = (&a.st->done)[vzero];
  // CGLS: the previous direction coefficient (the finisher overwrites beta
  // only after every block has stored its partials, so has read it); this iteration's step length is
  // formed below from the forward projection's partial sums and gamma,
  // lambda and ||p||^2
  double alpha = 0.0, beta = 0.0;
  double alpha_v = 0.0, beta_v = 0.0, gamma_v = 0.0, lambda_v = 0.0, pp_v = 0.0;
  if constexpr (MODE == BWD_CGLS || MODE == BWD_CGLS_INIT) {
    beta_v = (&a.st->beta)[vzero];
    if constexpr (MODE == BWD_CGLS_INIT) alpha_v = (&a.st->alpha)[vzero];  // zero before the first iteration
    if constexpr (MODE == BWD_CGLS) {
      gamma_v = (&a.st->gamma)[vzero];
      lambda_v = (&a.st->lambda)[vzero];
      pp_v = (&a.st->pp)[vzero];
    }
  }
  int degen = 0;           // CGLS: delta not positive and finite (no step)
  __shared__ T win[G][2][kChunk * kWin];
  __shared__ Meta<T> meta[G][3][kChunk];
  __shared__ double qsh[G * 2];   // CGLS: per-wave sums of the ||q||^2 partials
  // the groups' partial sums reuse the window memory once the angle loop is done
  static_assert(G * 2 * kThreads <= G * 2 * kChunk * kWin, "partials must fit in the window");
  T (*part)[2][kThreads] = reinterpret_cast<T (*)[2][kThreads]>(&win[0][0][0]);
  const int grp = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kThreads);
  const int t = threadIdx.x - grp * kThreads;
  const int tx = t & (kTile - 1), ty = t / kTile;          // ty in [0, 8)
  const int ix = pos.x * kTile + tx;
  const int iy0 = pos.y * kTile + ty, iy1 = iy0 + 8;
  const int n = a.n, nb = a.nb, m = a.m;
  const StageSrc src = stage_src<T, MODE>(a);
  unsigned rowoff = (unsigned)(t / kRowLanes) * (unsigned)nb;
  asm volatile("" : "+v"(rowoff));   // kept as is: not refolded into a product per chunk
  const double hc = 0.5 * (n - 1), hb = uniform(0.5 * (nb - 1));
  const double Xc = uniform(pos.x * kTile + 0.5 * (kTile - 1) - hc);
  const double Yc = uniform(pos.y * kTile + 0.5 * (kTile - 1) - hc);
  const T dX = T(tx) - T(0.5 * (kTile - 1)), dY = T(ty) - T(0.5 * (kTile - 1));
  T acc0 = T(0), acc1 = T(0);
  // Group grp takes the contiguous angles [kbeg, kend), an equal share (to
  // one angle) of the m angles, in chunks of kChunk; every group makes the
  // same number of chunk steps, each ending at a block barrier, so equal
  // shares keep the groups from waiting on each other.
  const int kbeg = (int)((long long)grp * m / G), kend = (int)((long long)(grp + 1) * m / G);
  const int steps = ((m + G - 1) / G + kChunk - 1) / kChunk;
  // Records of the chunk two steps ahead (the group's first wave).
  const bool rawwave = t < 64;   // uniform per wave
  Raw<T> ahead;
  // prologue: the ring entries of the first two chunks, the records of the
  // third, then the first chunk's window straight into LDS
  {
    const int k0 = kbeg;
    Raw<T> r0, r1;
    if (rawwave) {
      load_raw<T>(r0, a.ang, k0, t, kend);
      load_raw<T>(r1, a.ang, k0 + kChunk, t, kend);
      load_raw<T>(ahead, a.ang, k0 + 2 * kChunk, t, kend);
    }
    if constexpr (MODE == BWD_CGLS) {
      // ||q||^2 from the forward projection's per-block partial sums (loaded
      // beside the angle records), summed in the same fixed order by every
      // block: per thread over blocks tid, tid + blockDim, ... (eight loads in
      // flight at a time), then per wave (published before the barrier
      // below), then the waves in order
      constexpr int kStride = kThreads * G, kBatch = 8;
      const int nf = a.fwd_blocks;
      double qq = 0.0;
      for (int b0 = threadIdx.x; b0 < nf; b0 += kBatch * kStride) {
        double u[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) u[k] = a.fwd_part[min(b0 + k * kStride, nf - 1)];
#pragma unroll
        for (int k = 0; k < kBatch; ++k)
          if (b0 + k * kStride < nf) qq += u[k];
      }
      qq = wave_sum(qq);
      if ((threadIdx.x & 63) == 0) qsh[threadIdx.x >> 6] = qq;
    }
    if (__builtin_amdgcn_readfirstlane(done_v)) return;   // before any store and barrier
    if constexpr (MODE == BWD_CGLS || MODE == BWD_CGLS_INIT) {
      beta = uniform(beta_v);
      alpha = uniform(alpha_v);
    }
    if (rawwave) {
      fill_meta<T>(meta[grp][0], r0, k0, t, kend, Xc, Yc, hb);
      fill_meta<T>(meta[grp][1], r1, k0 + kChunk, t, kend, Xc, Yc, hb);
    }
    __syncthreads();
    Stage<T, MODE> sg;
    stage_load<T, MODE>(sg, src, meta[grp][0], k0, kend, nb, rowoff, t);
    if constexpr (MODE == BWD_CGLS) {
      // while the first window loads are in flight: delta = ||q||^2 +
      // lambda ||p||^2 and alpha = gamma / delta, the same in every block;
      // block 0 stores them for the next forward projection
      double qq = 0.0;
#pragma unroll
      for (int w = 0; w < G * 2; ++w) qq += qsh[w];
      const double delta = qq + uniform(lambda_v) * uniform(pp_v);
      degen = cgls_degenerate(delta);
      alpha = degen ? 0.0 : uniform(gamma_v) / delta;
      if (pos.id() == 0 && threadIdx.x == 0) {
        a.st->alpha = alpha;
        a.st->delta = delta;
      }
    }
    stage_store<T, MODE>(sg, win[grp][0], alpha, t);
    __syncthreads();
  }
  int mcur = 0;   // ring slot of the current chunk
  for (int st = 0; st < steps; ++st) {
    set_priority(steps - 1 - st);   // chunk steps left
    const int cur = st & 1, nxt = cur ^ 1;
    const int mnext = mcur == 2 ? 0 : mcur + 1, mfill = mnext == 2 ? 0 : mnext + 1;
    const int k0 = kbeg + st * kChunk, kc = max(0, min(kChunk, kend - k0));   // this group's chunk
    const int k1 = k0 + kChunk;                  // its next chunk
    const bool more = st + 1 < steps;
    // start the next chunk's window loads; they are consumed after the
    // current chunk is done
    Stage<T, MODE> pre;
    if (more) stage_load<T, MODE>(pre, src, meta[grp][mnext], k1, kend, nb, rowoff, t);
    // compute the current chunk
    const Meta<T>* __restrict__ mt = meta[grp][mcur];
#pragma unroll 4
    for (int kk = 0; kk < kc; ++kk) {
      const Meta<T> M = mt[kk];
      const T* w = win[grp][cur] + kk * kWin;
      const T Ja = fma(dX, M.c, fma(dY, M.s, M.base));
      const T Jb = fma(T(8), M.s, Ja);
      // J > 0 inside the window: truncation is floor; both pixels' bins are
      // read before either is weighed
      const int ja = (int)Ja, jb = (int)Jb;
      const T ra0 = w[ja], ra1 = w[ja + 1], rb0 = w[jb], rb1 = w[jb + 1];
      acc0 = pixel_weigh<T>(frac_part(Ja), ra0, ra1, M, acc0);
      acc1 = pixel_weigh<T>(frac_part(Jb), rb0, rb1, M, acc1);
    }
    // ring entry of the chunk two steps ahead (its slot held the previous
    // chunk, read before the last barrier), then the next window into LDS,
    // then the records of the chunk three steps ahead
    if (rawwave && k0 + 2 * kChunk < kend)
      fill_meta<T>(meta[grp][mfill], ahead, k0 + 2 * kChunk, t, kend, Xc, Yc, hb);
    if (more) stage_store<T, MODE>(pre, win[grp][nxt], alpha, t);
    if (rawwave && k0 + 3 * kChunk < kend) load_raw<T>(ahead, a.ang, k0 + 3 * kChunk, t, kend);
    mcur = mnext;
    __syncthreads();
  }
  set_priority(3);
  // The records fetched ahead end with the loop (no load into them is still
  // in flight here); taking them now keeps the compiler from waiting on the
  // epilogue's loads when it reuses their registers.
#pragma unroll
  for (int i = 0; i < Raw<T>::kWords; ++i) asm volatile("" ::"v"(ahead.w[i]));
  // CGLS: issue the epilogue's loads before the partial-sum barrier, as
  // buffer loads (pixels outside the image read 0, so no load is predicated
  // and nothing that uses them is pulled ahead of the barrier)
  T z_in[2] = {T(0), T(0)}, p_in[2] = {T(0), T(0)}, x_in[2] = {T(0), T(0)};
  T d_raw[4] = {T(0), T(0), T(0), T(0)};   // d of the first wave's WMG pixels
  if constexpr (MODE == BWD_CGLS || MODE == BWD_CGLS_INIT) {
    const size_t img_bytes = (size_t)n * n * sizeof(T);
    if (grp == 0) {
      const __amdgpu_buffer_rsrc_t rx = buffer_rsrc(a.xo, img_bytes);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int iy = q ? iy1 : iy0;
        const bool in = ix < n && iy < n;
        const unsigned off = in ? (unsigned)(iy * n + ix) * (unsigned)sizeof(T) : kOutside;
        if constexpr (MODE == BWD_CGLS) {
          const __amdgpu_buffer_rsrc_t rz = buffer_rsrc(a.zP, (size_t)n * a.ld * sizeof(T));
          const __amdgpu_buffer_rsrc_t rp = buffer_rsrc(a.p, img_bytes);
          const unsigned offz =
              in ? (unsigned)(iy * a.ld + ix + kPad) * (unsigned)sizeof(T) : kOutside;
          z_in[q] = load_elem(rz, offz, 0, T(0));
          p_in[q] = load_elem(rp, off, 0, T(0));
        }
        x_in[q] = load_elem(rx, off, 0, T(0));
      }
    }
    const int tt = threadIdx.x;
    if (a.fuse && !a.identity && tt < 64) {
      const __amdgpu_buffer_rsrc_t rd = buffer_rsrc(a.d, img_bytes);
      const int ix2 = pos.x * kTile + (tt & (kTile - 1));
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int iy2 = pos.y * kTile + (tt >> 4) + 4 * k;
        const unsigned off =
            ix2 < n && iy2 < n ? (unsigned)(iy2 * n + ix2) * (unsigned)sizeof(T) : kOutside;
        d_raw[k] = load_elem(rd, off, 0, T(0));
      }
    }
  }
  part[grp][0][t] = acc0;
  part[grp][1][t] = acc1;
  __syncthreads();
  if constexpr (MODE == BWD_CGLS || MODE == BWD_CGLS_INIT) {
    // first uses of the epilogue's loads here, after the barrier (otherwise
    // their conversions are placed, with a wait, right after the loads)
#pragma unroll
    for (int q = 0; q < 2; ++q) asm volatile("" : "+v"(z_in[q]), "+v"(p_in[q]), "+v"(x_in[q]));
#pragma unroll
    for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(d_raw[k]));
  }
  double bp[2] = {0.0, 0.0};
  if (grp == 0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      T v = part[0][q][t];
#pragma unroll
      for (int g2 = 1; g2 < G; ++g2) v += part[g2][q][t];
      bp[q] = a.h * (double)v;
    }
  }
  const int iys[2] = {iy0, iy1};
  if constexpr (MODE == BWD_CGLS || MODE == BWD_CGLS_INIT) {
    // s = W^T r - lambda x for the tile's pixels, after p = z + beta p and
    // x += alpha p; then z = M^-1 s on the tile and the four dot products.
    // With the WMG apply fused, the dot products go to the finisher
    // reduction, then p, x and z are stored.
    T* lds = &win[0][0][0] + G * 2 * kThreads;   // past the partial sums
    T (*stile)[kTile + 1] = reinterpret_cast<T (*)[kTile + 1]>(lds);
    T (*ptile)[kTile + 1] = reinterpret_cast<T (*)[kTile + 1]>(lds + kTile * (kTile + 1));
    const double lambda = a.st->lambda;
    const int x0 = pos.x * kTile, y0 = pos.y * kTile;
    T pv_new[2] = {T(0), T(0)}, xn_new[2] = {T(0), T(0)};
    if (grp == 0) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ly = ty + 8 * q, iy = iys[q];
        T sv = T(0), pv = T(0);
        if (ix < n && iy < n) {
          const size_t px = (size_t)iy * n + ix;
          T xn;
          if constexpr (MODE == BWD_CGLS) {
            if (!degen) {
              pv = (T)((double)z_in[q] + beta * (double)p_in[q]);
              xn = (T)((double)x_in[q] + alpha * (double)pv);
            } else {   // no step: direction and iterate stay as they are
              pv = p_in[q];
              xn = x_in[q];
            }
          } else {
            xn = x_in[q];
          }
          pv_new[q] = pv;
          xn_new[q] = xn;
          sv = (T)(bp[q] - lambda * (double)xn);
          if (!a.fuse) {
            if constexpr (MODE == BWD_CGLS) {
              a.p[px] = pv;
              a.xo[px] = xn;
            }
            a.out[px] = sv;
          }
        }
        stile[ly][tx] = sv;
        ptile[ly][tx] = pv;
      }
    }
    if (!a.fuse) return;   // uniform: the WMG apply runs as its own launch
    __syncthreads();
    // the first wave: the WMG apply on the whole tile and the four dot
    // products (its lanes' pixels in order k, then the block sum)
    const int tt = threadIdx.x;
    const int qx = tt & (kTile - 1), qy = tt / kTile;   // pixel of threads tt < 256
    double v[4] = {0.0, 0.0, 0.0, 0.0};   // <s,z>, ||s||^2, ||z||^2, <z,p>
    if (tt < 64) {
      // d + lambda of the lane's pixels, 0 outside the image
      double dl[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool in = x0 + qx < n && y0 + (tt >> 4) + 4 * k < n;
        dl[k] = in ? (double)d_raw[k] + lambda : 0.0;
      }
      T sv[4], zv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) zv[k] = sv[k] = stile[(tt >> 4) + 4 * k][qx];
      if (!a.identity) {
        switch (a.L) {
          case 0: wmg_wave<T, 0>(zv, dl, tt); break;
          case 1: wmg_wave<T, 1>(zv, dl, tt); break;
          case 2: wmg_wave<T, 2>(zv, dl, tt); break;
          case 3: wmg_wave<T, 3>(zv, dl, tt); break;
          default: wmg_wave<T, 4>(zv, dl, tt); break;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int ly = (tt >> 4) + 4 * k;
        const double sd = (double)sv[k], zd = (double)zv[k];
        v[0] += sd * zd;
        v[1] += sd * sd;
        v[2] += zd * zd;
        if (MODE == BWD_CGLS && lambda != 0.0) v[3] += zd * (double)ptile[ly][qx];
        stile[ly][qx] = zv[k];
      }
    }
    __syncthreads();
    T z = T(0), zt = T(0);
    if (tt < kTile * kTile) {
      z = stile[qy][qx];
      zt = stile[qx][qy];
    }
    SolverState* sst = a.st;
    // the finisher reads the state fields of the step before its block sum
    reduce_to_finisher<4, kThreads * G / 64>(
        v, a.slots, pos.count(), pos.id(), [sst]() { return cgls_scalars(sst); },
        [sst, degen](double (&tot)[4], bool late, const CglsScalars& sc) {
          if (late) sst->done = 4;
          else cgls_precond_finish(sst, sc, tot, MODE == BWD_CGLS_INIT, degen);
        });
    if constexpr (MODE == BWD_CGLS) {
      if (grp == 0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (ix < n && iys[q] < n) {
            const size_t px = (size_t)iys[q] * n + ix;
            a.p[px] = pv_new[q];
            a.xo[px] = xn_new[q];
          }
        }
      }
    }
    if (tt < kTile * kTile) {
      if (x0 + qx < n && y0 + qy < n) a.zP[(size_t)(y0 + qy) * a.ld + x0 + qx + kPad] = z;
      // transposed copy: consecutive threads write consecutive addresses
      if (x0 + qy < n && y0 + qx < n) a.zTP[(size_t)(x0 + qy) * a.ld + y0 + qx + kPad] = zt;
    }
    return;
  }
  if constexpr (MODE == BWD_SIRT) {
    double usq = 0.0;
    if (grp == 0) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (ix < n && iys[q] < n) {
          const size_t p = (size_t)iys[q] * n + ix;
          double u = (double)a.C[p] * bp[q];
          const T xn = (T)((double)a.out[p] + u);
          u = (double)xn - (double)a.out[p];
          a.out[p] = xn;
          usq += u * u;
        }
      }
    }
    // x += C W^T r, with r = R (b - W x) from the forward pass
    double v[1] = {usq};
    SolverState* sst = a.st;
    reduce_and_finish<1, kThreads * G / 64>(
        v, a.red, pos.count(), pos.id(),
        [sst](double (&tot)[1]) {
          const double nrm = sqrt(tot[0]);
          if (!sst->init) {
            sst->s0 = nrm;
            sst->init = 1;
            if (nrm == 0.0) {   // b = 0: x = 0 is exact, no iteration
              sst->relres = 0.0;
              sst->done = 1;
              return;
            }
          }
          sst->iter += 1;
          const double rr = sst->s0 > 0.0 ? nrm / sst->s0 : 0.0;
          sst->relres = rr;
          if (sst->hist && sst->iter <= sst->hist_cap) sst->hist[sst->iter - 1] = rr;
          if (!finite(nrm)) sst->done = 3;
          else if (sst->s0 == 0.0) sst->done = 1;
          else if (sst->fixed) { if (sst->iter >= sst->max_iter) sst->done = 1; }
          else if (rr <= sst->tol) sst->done = 1;
          else if (sst->iter >= sst->max_iter) sst->done = 2;
        });
  } else if (grp == 0) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int iy = iys[q];
      if (ix >= n || iy >= n) continue;
      const size_t p = (size_t)iy * n + ix;
      if constexpr (MODE == BWD_PLAIN) {
        a.out[p] = (T)bp[q];
      } else if constexpr (MODE == BWD_AXPY) {
        double v = a.sa * bp[q];
        if (a.sx != 0.0) v += a.sx * (double)a.xin[(size_t)iy * a.x_ld + ix + a.x_off];
        if (a.sf != 0.0) v += a.sf * (double)a.fin[p];
        a.out[p] = (T)v;
      }
    }
  }
}

// Eight float blocks of 4 waves per CU (18.5 KB of LDS each) need 8 waves per
// SIMD: at most 64 VGPRs.
template <typename T>
constexpr int kMinWaves = sizeof(T) == 4 ? 8 : 4;

template <typename T, int MODE>
__global__ __launch_bounds__(kThreads * kGroups<T>, kMinWaves<T>) void k_backward(BwdK<T> a) {
  backward_body<T, MODE>(a, grid_pos());
}

template <typename T, int MODE>
__global__ __launch_bounds__(kThreads * kGroups<T>, kMinWaves<T>) void k_backward_batch(
    const BwdK<T>* __restrict__ args, const int* __restrict__ start, const int* __restrict__ gx,
    int count) {
  const int r = batch_find(start, count, blockIdx.x);
  backward_body<T, MODE>(args[r], batch_pos(start, gx, r));
}

template <typename T>
BwdK<T> bwd_args(const Geometry& g, const BwdArgs& a) {
  BwdK<T> k;
  k.sino = (const T*)a.sino;
  k.out = (T*)a.out;
  k.q = (const T*)a.q;
  k.p = (T*)a.p;
  k.xo = (T*)a.x;
  k.zP = (T*)a.zP;
  k.zTP = (T*)a.zTP;
  k.d = (const T*)g.d_diag;
  k.ld = g.ld;
  k.L = g.L;
  k.identity = a.identity ? 1 : 0;
  k.fuse = backward_fuses_wmg(g) ? 1 : 0;
  k.xin = (const T*)a.x;
  k.fin = (const T*)a.f;
  k.C = (const T*)a.C;
  k.ang = g.d_bwd;
  k.fwd_part = a.fwd_part;
  k.fwd_blocks = a.fwd_blocks;
  k.slots = a.slots;
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
  return k;
}

template <typename T>
void bwd_dispatch(const Geometry& g, BwdMode mode, const BwdArgs& a, hipStream_t st) {
  const BwdK<T> k = bwd_args<T>(g, a);
  dim3 grid((g.n + kTile - 1) / kTile, (g.n + kTile - 1) / kTile);
  const dim3 block(kThreads * kGroups<T>);
  TimedLaunch tl(TK_BACKWARD, st);
  switch (mode) {
    case BWD_PLAIN: hipLaunchKernelGGL((k_backward<T, BWD_PLAIN>), grid, block, 0, st, k); break;
    case BWD_CGLS: hipLaunchKernelGGL((k_backward<T, BWD_CGLS>), grid, block, 0, st, k); break;
    case BWD_SIRT: hipLaunchKernelGGL((k_backward<T, BWD_SIRT>), grid, block, 0, st, k); break;
    case BWD_AXPY: hipLaunchKernelGGL((k_backward<T, BWD_AXPY>), grid, block, 0, st, k); break;
    case BWD_CGLS_INIT:
      hipLaunchKernelGGL((k_backward<T, BWD_CGLS_INIT>), grid, block, 0, st, k);
      break;
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace

bool backward_fuses_wmg(const Geometry& g) { return (1 << g.L) <= kTile; }

int backward_blocks(const Geometry& g) {
  const int t = (g.n + kTile - 1) / kTile;
  return t * t;
}

void launch_backward(const Geometry& g, BwdMode mode, const BwdArgs& a, hipStream_t st) {
  if (g.f64) bwd_dispatch<double>(g, mode, a, st);
  else bwd_dispatch<float>(g, mode, a, st);
}

void prepare_backward_batch(DevTable& t, const std::vector<const Geometry*>& gs,
                            const std::vector<BwdArgs>& as, hipStream_t st) {
  std::vector<BwdK<float>> host(gs.size());
  std::vector<int> blocks(gs.size()), widths(gs.size());
  for (size_t i = 0; i < gs.size(); ++i) {
    if (gs[i]->f64) fail(RECO_EINVAL, "batched solves take float32 geometries");
    host[i] = bwd_args<float>(*gs[i], as[i]);
    widths[i] = (gs[i]->n + kTile - 1) / kTile;
    blocks[i] = widths[i] * widths[i];
  }
  t.upload(host.data(), sizeof(BwdK<float>), blocks, widths, st);
}

void launch_backward_batch(const DevTable& t, BwdMode mode, hipStream_t st) {
  if (t.count == 0) return;
  TimedLaunch tl(TK_BACKWARD, st);
  const auto* args = (const BwdK<float>*)t.args;
  const dim3 block(kThreads * kGroups<float>);
  switch (mode) {
    case BWD_CGLS:
      hipLaunchKernelGGL((k_backward_batch<float, BWD_CGLS>), dim3(t.total_blocks), block, 0, st,
                         args, t.start, t.gx, t.count);
      break;
    case BWD_CGLS_INIT:
      hipLaunchKernelGGL((k_backward_batch<float, BWD_CGLS_INIT>), dim3(t.total_blocks), block, 0,
                         st, args, t.start, t.gx, t.count);
      break;
    case BWD_PLAIN:
      hipLaunchKernelGGL((k_backward_batch<float, BWD_PLAIN>), dim3(t.total_blocks), block, 0, st,
                         args, t.start, t.gx, t.count);
      break;
    default: fail(RECO_EINVAL, "unsupported batched backward mode");
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace reco
