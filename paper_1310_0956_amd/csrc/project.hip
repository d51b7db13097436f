// Forward projector q = W x (Section 2.1, eq. sys), ray driven, matrix free.
//
// Each ray is walked along its major axis: at every row (or column, for angles
// closer to the x axis, via a transposed image copy) the ray overlaps exactly
// two candidate pixels, floor(P) and floor(P)+1, where P is the crossing
// position in pixel units.  With f = P - floor(P) the weights are
//   w0 = (h/u) clamp((1/2 - f) B + 1/2, 0, 1),  w1 = h/u - w0,
// u = |major direction cosine|, from per-angle tables: for the exact
// intersection lengths B = u/v, v = |minor cosine| (the trapezoid of the
// chord length against the ray offset, divided by its plateau h/u), for
// Joseph's kernel B = 1 (w0 = h (1 - f)/u, the linear interpolation); the two
// weights of a row always add up to the row's chord h/u.  A ray sums the
// unit-clamped weights and takes the factor h/u once at its end.  Candidate columns are clamped to
// [-2, n]; the padded image copies carry kPad >= 2 zero columns on each side,
// so a ray outside the image reads zeros.
//
// Work decomposition: a block takes up to 8 neighbouring angles that share the
// walk axis ("group") times 32 neighbouring detector bins, one ray per thread
// (each wave: two angles, interleaved across its lanes); for grids too small
// to fill the GPU, two threads per ray, each walking half of every band.
// It walks the rows in bands: the columns the block's rays cross in a band
// (known from the corner rays, since positions are linear in bin and row) are
// staged in LDS with coalesced loads, double buffered through registers, and
// the rays read their two pixels per row from LDS.  A band wider than the LDS
// window (only for very sparse angle sets) is walked straight from memory.
//
// Positions are walked in 32.32 fixed point (float path) or recomputed in
// float64 (double path), so the geometry error stays far below the float
// weight error.
#include <algorithm>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "timing.h"

namespace reco {

namespace {

constexpr int kSlots = 8;       // angles per block
constexpr int kBins = 32;       // bins per block
constexpr int kStride = 126;    // LDS row stride of a staged band (elements); two
                                // float bands plus the block's other shared data
                                // stay under 32 KB, so five blocks fit in a CU
constexpr int kWinCols = 122;   // widest window staged in LDS; columns past the
                                // window's width read zeros (guard columns)
constexpr int kRays = kSlots * kBins;            // rays per block
constexpr int kLoadCols = 128;                    // staging: threads per row
// H threads per ray ("halves"): with H = 2 each walks half the rows of every
// band, so a block has twice the waves, for grids too small to fill the GPU.
template <int H>
constexpr int kFwdThreads = kRays * H;
template <int H>
constexpr int kStageRows = kFwdThreads<H> / kLoadCols;   // rows loaded per staging pass

template <typename T>
constexpr int kBand = sizeof(T) == 4 ? 32 : 16;   // rows per staged band

template <typename T>
struct FwdK {
  const T* imgP;
  const T* imgTP;
  T* out;
  T* r;                // CGLS: residual, updated with the previous step
  const T* b;
  const T* R;
  const FwdAngle* ang;
  const int2* wins;    // [ngroups * nbx][maxb] column window of each band
  const FwdBlk* blk;   // [ngroups * nbx] the record of each grid position
  int nbx, maxb;
  SolverState* st;
  RedScratch red;
  double* part;        // CGLS: per-block ||q||^2 partial sums
  unsigned long long* count;
  int n, ld, nb, m;
  double h;
};

__device__ __forceinline__ int iclamp(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Weight of the left candidate from the fraction, divided by the plateau
// (float and double forms).  The unit clamp folds into the FMA's output clamp.
__device__ __forceinline__ float left_weight(float f, float B, float C) {
  return __builtin_amdgcn_fmed3f(fmaf(0.5f - f, B, C), 0.0f, 1.0f);
}
__device__ __forceinline__ double left_weight(double f, double B, double C) {
  return fmin(fmax(fma(0.5 - f, B, C), 0.0), 1.0);
}

// Position walker along the rows of one ray.  col() is the column of the left
// candidate relative to an offset set by shift_cols (the current LDS window).
template <typename T>
struct Walk;

template <>
struct Walk<float> {
  unsigned long long p, dp;   // 32.32 fixed point
  __device__ void init(double P, double, long long dP) {
    p = (unsigned long long)__double2ll_rn(P * 4294967296.0);
    dp = (unsigned long long)dP;
  }
  __device__ __forceinline__ int col() const { return (int)(p >> 32); }
  __device__ __forceinline__ float frac() const {
    return (float)(unsigned)(p & 0xffffffffull) * 2.3283064365386963e-10f;
  }
  __device__ __forceinline__ void step() { p += dp; }
  __device__ __forceinline__ void skip(int rows) { p += (unsigned long long)rows * dp; }
  __device__ __forceinline__ void shift_cols(int dc) {
    p -= (unsigned long long)(long long)dc << 32;
  }
};

template <>
struct Walk<double> {
  double P0, slope, cur;
  int r, off;
  __device__ void init(double P, double s, long long) {
    P0 = P;
    slope = s;
    cur = P;
    r = 0;
    off = 0;
  }
  __device__ __forceinline__ int col() const { return (int)floor(cur) - off; }
  __device__ __forceinline__ double frac() const { return cur - floor(cur); }
  __device__ __forceinline__ void step() {
    ++r;
    cur = fma((double)r, slope, P0);
  }
  __device__ __forceinline__ void skip(int rows) {
    r += rows;
    cur = fma((double)r, slope, P0);
  }
  __device__ __forceinline__ void shift_cols(int dc) { off += dc; }
};

template <typename T>
__device__ __forceinline__ T wB(const FwdAngle& a) {
  if constexpr (sizeof(T) == 4) return a.Bf; else return a.B;
}
template <typename T>
__device__ __forceinline__ T wC(const FwdAngle& a) {
  if constexpr (sizeof(T) == 4) return a.Cf; else return a.C;
}
template <typename T>
__device__ __forceinline__ T wM(const FwdAngle& a) {
  if constexpr (sizeof(T) == 4) return a.Wmaxf; else return a.Wmax;
}

// `rows` rows of one ray read from an LDS window (row stride kStride).
// Float path: the walker's column is relative to the window start and is
// clamped as an unsigned value to `width`, so a ray left or right of the
// window (only rays outside the image can be) reads the zero guard columns
// width and width + 1; rays inside the image stay in [0, width - 2].  The left
// weight (over the plateau) is clamp(lo * Bq + Cq, 0, 1) with lo the 32-bit
// fraction of the position, Bq = -B 2^-32 and Cq = C + B/2 (the trapezoid
// (1/2 - f) B + C).
__device__ __forceinline__ void band_lds(const float* __restrict__ w, Walk<float>& wk, int rows,
                                         unsigned width, float Bq, float Cq,
                                         float& acc0, float& acc1) {
  unsigned long long p = wk.p;
  const unsigned long long dp = wk.dp;
  int r = 0;
  for (; r + 3 < rows; r += 4) {
    float w0[4], x0[4], x1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const unsigned c = min((unsigned)(p >> 32), width);
      const float* q = w + (r + u) * kStride + c;
      x0[u] = q[0];
      x1[u] = q[1];
      w0[u] = __builtin_amdgcn_fmed3f(fmaf((float)(unsigned)p, Bq, Cq), 0.0f, 1.0f);
      p += dp;
      asm volatile("" : "+v"(p));   // one position register: keep LLVM from cloning it per row
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc0 = fmaf(w0[u], x0[u] - x1[u], acc0);
      acc1 += x1[u];
    }
  }
  for (; r < rows; ++r) {
    const unsigned c = min((unsigned)(p >> 32), width);
    const float* q = w + r * kStride + c;
    const float x0 = q[0], x1 = q[1];
    const float w0 = __builtin_amdgcn_fmed3f(fmaf((float)(unsigned)p, Bq, Cq), 0.0f, 1.0f);
    acc0 = fmaf(w0, x0 - x1, acc0);
    acc1 += x1;
    p += dp;
  }
  wk.p = p;
}

// Double path: the window-relative column is clamped into [lo_w, hi_w], the
// window images of image columns -2 and n.
__device__ __forceinline__ void band_lds(const double* __restrict__ w, Walk<double>& wk, int rows,
                                         int lo_w, int hi_w, double B, double C,
                                         double& acc0, double& acc1) {
  for (int r = 0; r < rows; ++r) {
    const int c = iclamp(wk.col(), lo_w, hi_w);
    const double* q = w + r * kStride + c;
    const double x0 = q[0], x1 = q[1];
    acc0 = fma(left_weight(wk.frac(), B, C), x0 - x1, acc0);
    acc1 += x1;
    wk.step();
  }
}

// `rows` rows of one ray read straight from the padded image (bands wider than
// the LDS window).  The walker's column is relative to image column c0.
template <typename T>
__device__ __forceinline__ void band_mem(__amdgpu_buffer_rsrc_t rs, int ld, int n, int r0, int rows,
                                         int c0, Walk<T>& wk, T B, T C, T& acc0, T& acc1) {
  for (int r = 0; r < rows; ++r) {
    const int c = iclamp(wk.col() + c0, -2, n) + kPad;
    const int soff = (r0 + r) * ld * (int)sizeof(T);
    const T x0 = load_elem(rs, (unsigned)c * sizeof(T), soff, T(0));
    const T x1 = load_elem(rs, (unsigned)(c + 1) * sizeof(T), soff, T(0));
    acc0 = fma(left_weight(wk.frac(), B, C), x0 - x1, acc0);
    acc1 += x1;
    wk.step();
  }
}

struct Window {
  int c0, c1;
};

// Row range and per-band column windows of every block, computed once per
// geometry (they depend on the geometry only).  Block (g, bx) covers angles
// groups[g][0..8) and bins [32 bx, 32 bx + 31] (clipped to nb).
//  - rows: [lo, hi], covering the rows where any of the block's rays is
//    within 1.5 columns of the image (block_rows);
//  - band b (rows [lo + b*BAND, min(lo + (b+1)*BAND - 1, hi)]): columns
//    [c0, c1], the floor(P) range over the block's corner rays (first and
//    last bin of each angle at the band's first and last row), widened by one
//    column on each side for rounding and clamped to [-2, n+1].
// Positions are linear in bin and row for each angle, so the corner rays
// bound every ray of the block.
// Rows of bins [jf, jl] of one angle: the ray of bin j is within 1.5 columns
// of the image between rows (-1.5 - P0(j)) / slope and (n + 0.5 - P0(j)) /
// slope, bounds linear in j, so their extremes over the bins are those of the
// first and last bin, and the rows are taken from them before clipping to the
// image (a ray between two that miss the image on either side may cross it).
// Axis-parallel rays (slope 0) meet every row or none: the block meets them
// all when its positions P0 reach [-1.5, n + 0.5].  Empty: lo > hi.
__device__ __forceinline__ void block_rows(const FwdAngle& ang, int jf, int jl, int n, int& lo,
                                           int& hi) {
  const double Pf = fma((double)jf, ang.inv, ang.A0), Pl = fma((double)jl, ang.inv, ang.A0);
  lo = n;
  hi = -1;
  if (ang.slope == 0.0) {
    if (fmax(Pf, Pl) >= -1.5 && fmin(Pf, Pl) <= n + 0.5) { lo = 0; hi = n - 1; }
  } else {
    const double a1 = (-1.5 - Pf) / ang.slope, a2 = (n + 0.5 - Pf) / ang.slope;
    const double b1 = (-1.5 - Pl) / ang.slope, b2 = (n + 0.5 - Pl) / ang.slope;
    const double tl = fmin(fmin(a1, a2), fmin(b1, b2)), th = fmax(fmax(a1, a2), fmax(b1, b2));
    lo = (int)fmin(fmax(0.0, ceil(tl)), (double)n);
    hi = (int)fmax(fmin((double)(n - 1), floor(th)), -1.0);
  }
}

__device__ __forceinline__ int corner_col(const FwdAngle& ang, int j, int r) {
  const double P = fma((double)r, ang.slope, fma((double)j, ang.inv, ang.A0));
  return (int)fmin(fmax(floor(P), -1.0e9), 1.0e9);
}

// One thread per (block, band); band index -1 (the first thread of a block's
// row) stores the row range.
__global__ __launch_bounds__(256) void k_fwd_windows(const FwdAngle* __restrict__ ang,
                                                     const int* __restrict__ groups, int ngroups,
                                                     int nbx, int n, int nb, int band, int maxb,
                                                     int2* __restrict__ rows,
                                                     int2* __restrict__ wins) {
  const long long id = blockIdx.x * 256ll + threadIdx.x;
  const long long total = (long long)ngroups * nbx * (maxb + 1);
  if (id >= total) return;
  const int blk = (int)(id / (maxb + 1));
  const int b = (int)(id % (maxb + 1)) - 1;
  const int g = blk / nbx, bx = blk % nbx;
  const int jfirst = bx * kBins, jlast = min(jfirst + kBins - 1, nb - 1);
  int lo = n, hi = -1;
  for (int s = 0; s < kSlots; ++s) {
    const int k = groups[g * kSlots + s];
    if (k < 0) continue;
    int l, h;
    block_rows(ang[k], jfirst, jlast, n, l, h);
    if (h >= l) { lo = min(lo, l); hi = max(hi, h); }
  }
  if (b < 0) {
    rows[blk] = make_int2(lo, hi);
    return;
  }
  const int rb = lo + b * band;
  int c0 = 0, c1 = 0;
  if (hi >= lo && rb <= hi) {
    const int re = min(rb + band - 1, hi);
    int wl = 1 << 30, wh = -(1 << 30);
    for (int s = 0; s < kSlots; ++s) {
      const int k = groups[g * kSlots + s];
      if (k < 0) continue;
      const int cs[4] = {corner_col(ang[k], jfirst, rb), corner_col(ang[k], jfirst, re),
                         corner_col(ang[k], jlast, rb), corner_col(ang[k], jlast, re)};
      for (int i = 0; i < 4; ++i) {
        wl = min(wl, cs[i] - 1);
        wh = max(wh, cs[i] + 1);
      }
    }
    c0 = iclamp(wl, -2, n);
    c1 = iclamp(wh, -2, n) + 1;
  }
  wins[(size_t)blk * maxb + b] = make_int2(c0, c1);
}

template <typename T, int MODE, int H>
__device__ __forceinline__ void forward_body(const FwdK<T>& a, const BlockPos bp) {
  constexpr int BAND = kBand<T>;
  constexpr int NT = kFwdThreads<H>;
  constexpr int SR = kStageRows<H>;
  constexpr int STAGE_PER = BAND / SR;   // loads per thread per band
  // H = 2: every band's rows are summed in two parts, [0, HB) by the ray's
  // first thread and [HB, BAND) by its second, each in row order, and the
  // parts are added at the end (first + second).  H = 1: one pass.
  constexpr int HB = BAND / 2;
  static_assert(H == 1 || H == 2, "one or two threads per ray");
  // The prologue runs at the top wave priority (latency bound; the band
  // loop lowers it with the work left).
  set_priority(3);
  // Loads whose results are wanted later carry an opaque zero held in a
  // vector register: the value then stays in vector registers until it is
  // used, instead of being moved to scalar registers (which would wait for
  // the load) right after it is issued.
  int vzero;
  asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
  // solver finished: later launches are no-ops (tested before the first band
  // is staged, once the block's table loads are in flight)
  int done_v = 0;
  if (a.st) done_v = (&a.st->done)[vzero];
  double alpha_v = 0.0;   // CGLS: the previous iteration's step length
  if constexpr (MODE == FWD_CGLS) alpha_v = (&a.st->alpha)[vzero];
  __shared__ T win[2][BAND * kStride];
  const int t = threadIdx.x;
  const int tr = t % kRays;   // the thread's ray
  const int half = __builtin_amdgcn_readfirstlane(t / kRays);   // its rows: [half HB, half HB + HB)
  const int n = a.n, nb = a.nb;
  // the block's record (setup table, one per grid position): its bins, rows,
  // walking axis and first band windows, then its angles
  const FwdBlk* __restrict__ rec = a.blk + bp.id();
  const int lb = rec->lb;
  const int jfirst = rec->jfirst, jlast = rec->jlast;
  const int k0 = rec->k0;            // first angle: sets the walk axis
  // ray of this thread: a wave holds two angles of the group, interleaved by
  // lane parity, so that each half-wave's LDS reads span about 16 bins' worth
  // of columns (fewer bank conflicts than 32 bins of one angle)
  const int kl = rec->k[((tr >> 6) << 1) + (tr & 1)];
  const int jown = jfirst + ((tr >> 1) & 31);
  const bool valid = kl >= 0 && jown <= jlast;
  // invalid lanes shadow the block's first ray so that they stay in the window
  const int k = valid ? kl : k0;
  const int j = valid ? jown : jfirst;
  const FwdAngle ang = a.ang[k];
  const T* img = rec->major ? a.imgTP : a.imgP;
  const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(img, (size_t)n * a.ld * sizeof(T));
  // rows the block's rays touch and the column window of each band
  const int lo = rec->lo, hi = rec->hi;
  const int nbands = rec->nbands;
  const int2* __restrict__ bandwin = a.wins + (size_t)lb * a.maxb;
  // The window of band b + 1 is loaded during band b - 1 (two bands ahead of
  // its first use, with the opaque zero in its index), so no band waits on
  // the table; those of bands 0 and 1 come with the record (zeros when absent).
  Window wcur{rec->w0x, rec->w0y};
  int2 wahead = make_int2(rec->w1x, rec->w1y);
  // staging: thread loads column (t % kLoadCols) of rows (t / kLoadCols) + SR * i;
  // columns past the window's width are written as zeros (the guard columns);
  // threads with scol >= kStride only idle
  const int scol = t % kLoadCols;
  const bool stager = scol < kStride;
  const int srow = __builtin_amdgcn_readfirstlane(t / kLoadCols);   // uniform per wave
  const int rbytes = a.ld * (int)sizeof(T);
  int cur_shift = 0;   // window start the walker's columns are currently relative to
  // the table loads above are issued before the stop test (left alone, the
  // compiler tests first and issues them only after that load returns)
  asm volatile("" ::: "memory");
  if (__builtin_amdgcn_readfirstlane(done_v)) return;   // before any store and barrier
  // the first band's loads, issued before the ray set-up waits for the
  // angle records
  const bool first_lds = nbands > 0 && wcur.c1 - wcur.c0 + 1 <= kWinCols;
  // columns past the window (and a window not staged) read zeros from an
  // offset past the end of the buffer: one select, then unconditional loads
  const unsigned coff0 = first_lds && scol <= wcur.c1 - wcur.c0
                             ? (unsigned)(wcur.c0 + kPad + scol) * (unsigned)sizeof(T)
                             : kOutside;
  T v0[STAGE_PER];
#pragma unroll
  for (int i = 0; i < STAGE_PER; ++i) v0[i] = load_elem(rs, coff0, (lo + srow + SR * i) * rbytes, T(0));
  // the ray: walker and weight coefficients
  const double P0 = fma((double)j, ang.inv, ang.A0);
  const T B = wB<T>(ang), C = wC<T>(ang), Wm = wM<T>(ang);
  const float Bq = (float)(-ang.B * 2.3283064365386963e-10), Cq = (float)(ang.C + 0.5 * ang.B);
  T acc0 = T(0), acc1 = T(0);     // the thread's sums (its part of every band for H = 2)
  Walk<T> wk;
  wk.init(fma((double)lo, ang.slope, P0), ang.slope, ang.dP);
  // the second part's thread starts HB rows on, by the walker's own steps (the
  // same positions as a walker that walks both parts)
  if (half == 1) wk.skip(HB);
  if (nbands > 0) {
    if (first_lds) {
#pragma unroll
      for (int i = 0; i < STAGE_PER; ++i)
        if (stager) win[0][(srow + SR * i) * kStride + scol] = v0[i];
    }
    __syncthreads();
  }
  for (int bnd = 0; bnd < nbands; ++bnd) {
    set_priority((nbands - bnd) >> 2);   // bands left
    const int cur = bnd & 1, nxt = cur ^ 1;
    const int rb = lo + bnd * BAND;
    const int rows = min(BAND, hi - rb + 1);
    const bool more = bnd + 1 < nbands;
    Window wnext{0, 0};
    T pre[STAGE_PER];
    bool next_lds = false;
    if (more) {
      const int rb2 = rb + BAND;
      const int2 w1 = make_int2(__builtin_amdgcn_readfirstlane(wahead.x),
                                __builtin_amdgcn_readfirstlane(wahead.y));
      if (bnd + 2 < nbands) wahead = bandwin[bnd + 2 + vzero];
      wnext = Window{w1.x, w1.y};
      next_lds = wnext.c1 - wnext.c0 + 1 <= kWinCols;
      if (next_lds) {
        const unsigned coff = scol <= wnext.c1 - wnext.c0
                                  ? (unsigned)(wnext.c0 + kPad + scol) * (unsigned)sizeof(T)
                                  : kOutside;
#pragma unroll
        for (int i = 0; i < STAGE_PER; ++i)
          pre[i] = load_elem(rs, coff, (rb2 + srow + SR * i) * rbytes, T(0));
      }
    }
    // walker columns relative to this band's window start
    wk.shift_cols(wcur.c0 - cur_shift);
    cur_shift = wcur.c0;
    const int width = wcur.c1 - wcur.c0 + 1;
    // rows [r0, r0 + nrows) of the band into the thread's sums
    auto walk = [&](int r0, int nrows) {
      if (width <= kWinCols) {
        const T* wband = win[cur] + r0 * kStride;
        if constexpr (sizeof(T) == 4)
          band_lds(wband, wk, nrows, (unsigned)width, Bq, Cq, acc0, acc1);
        else
          band_lds(wband, wk, nrows, max(-2 - wcur.c0, 0), min(n - wcur.c0, width - 2), B, C,
                   acc0, acc1);
      } else {
        band_mem<T>(rs, a.ld, n, rb + r0, nrows, wcur.c0, wk, B, C, acc0, acc1);
      }
    };
    if constexpr (H == 1) {
      walk(0, rows);
    } else {
      walk(half * HB, max(0, min(HB, rows - half * HB)));   // fewer rows in the last band
      // past the other part's rows (after the last band the walker is not used)
      wk.skip(HB);
    }
    if (next_lds) {
#pragma unroll
      for (int i = 0; i < STAGE_PER; ++i)
        if (stager) win[nxt][(srow + SR * i) * kStride + scol] = pre[i];
    }
    wcur = wnext;
    __syncthreads();
  }
  set_priority(3);
  if constexpr (H == 2) {
    // the second part's sums, added by the thread of the first (the band loop
    // ended with a barrier, so the window memory is free)
    T* xch = &win[0][0];
    if (half == 1) {
      xch[tr] = acc0;
      xch[kRays + tr] = acc1;
    }
    __syncthreads();
    if (half == 0) {
      acc0 += xch[tr];
      acc1 += xch[kRays + tr];
    }
  }
  const bool owner = valid && half == 0;   // the thread that stores its ray
  const T result = (T)a.h * (Wm * (acc0 + acc1));
  const size_t i = (size_t)k * nb + j;   // valid lanes only use it
  if constexpr (MODE == FWD_PLAIN) {
    if (owner) a.out[i] = result;
  } else if constexpr (MODE == FWD_SIRT) {
    if (owner) a.out[i] = (T)((double)a.R[i] * ((double)a.b[i] - (double)result));
  } else if constexpr (MODE == FWD_CGLS) {
    // The residual update of the previous iteration, r -= alpha q_old (alpha
    // of that iteration, stored by the previous backprojection), then
    // q = W z + beta q_old  (q_old = W p_old, so q = W (z + beta p_old) = W p_new)
    // and the block's part of ||q||^2: a plain store, summed by every block of
    // the following backprojection (kernel boundaries make it visible), which
    // forms delta and the step length alpha from it.
    double q = 0.0, r_new = 0.0;
    if (owner) {
      const double q_old = (double)a.out[i];
      r_new = (double)a.r[i] - uniform(alpha_v) * q_old;
      q = (double)(T)((double)result + a.st->beta * q_old);
    }
    __shared__ double sh[NT / 64];
    double v[1] = {q * q};
    block_sum<1, NT / 64>(v, sh);
    if (threadIdx.x == 0) a.part[bp.id()] = v[0];
    if (owner) {
      a.r[i] = (T)r_new;
      a.out[i] = (T)q;
    }
  }
}

template <typename T, int MODE, int H>
__global__ __launch_bounds__(kFwdThreads<H>) void k_forward(FwdK<T> a) {
  forward_body<T, MODE, H>(a, grid_pos());
}

template <typename T, int MODE, int H>
__global__ __launch_bounds__(kFwdThreads<H>) void k_forward_batch(const FwdK<T>* __restrict__ args,
                                                            const int* __restrict__ start,
                                                            const int* __restrict__ gx, int count) {
  const int r = batch_find(start, count, blockIdx.x);
  forward_body<T, MODE, H>(args[r], batch_pos(start, gx, r));
}

// Nonzero count of W: one thread per ray, every row of the image, float64
// weights (no image access).
__global__ __launch_bounds__(256) void k_count(const FwdAngle* __restrict__ angs, int n, int nb,
                                               int m, unsigned long long* count) {
  const size_t ray = blockIdx.x * (size_t)256 + threadIdx.x;
  unsigned long long cnt = 0;
  if (ray < (size_t)m * nb) {
    const int k = (int)(ray / nb), j = (int)(ray % nb);
    const FwdAngle ang = angs[k];
    const double P0 = fma((double)j, ang.inv, ang.A0);
    constexpr double eps = 1e-9;   // of the plateau
    for (int r = 0; r < n; ++r) {
      const double P = fma((double)r, ang.slope, P0);
      if (P < -2.0 || P > n + 1.0) continue;
      const double fl = floor(P);
      const int i0 = (int)fl;
      const double w0 = fmin(fmax(fma(0.5 - (P - fl), ang.B, ang.C), 0.0), 1.0);
      const double w1 = 1.0 - w0;
      cnt += (w0 > eps && i0 >= 0 && i0 < n) ? 1 : 0;
      cnt += (w1 > eps && i0 + 1 >= 0 && i0 + 1 < n) ? 1 : 0;
    }
  }
  double v[1] = {(double)cnt};
  __shared__ double sh[4];
  block_sum256<1>(v, sh);
  if (threadIdx.x == 0) atomicAdd(count, (unsigned long long)v[0]);
}

// x[n][n] -> xP[n][ld] (kPad zero columns on each side) and its transpose xTP.
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
      xP[(size_t)iy * ld + ix + kPad] = v;
    }
    tile[r][tx] = v;
  }
  if (blockIdx.x == 0) {   // zero margins of rows y0..y0+31 of both copies
    for (int e = threadIdx.x; e < 32 * 2 * kPad; e += 256) {
      const int r = e / (2 * kPad), c = e % (2 * kPad);
      const int row = y0 + r;
      const int col = c < kPad ? c : n + c;   // [0, kPad) and [n+kPad, n+2kPad)
      if (row < n) {
        xP[(size_t)row * ld + col] = T(0);
        xTP[(size_t)row * ld + col] = T(0);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ty + 8 * i;
    const int ox = x0 + r, oy = y0 + tx;  // output row = original column
    if (ox < n && oy < n) xTP[(size_t)ox * ld + oy + kPad] = tile[tx][r];
  }
}

template <typename T>
FwdK<T> make_args(const Geometry& g, const FwdArgs& a) {
  FwdK<T> k;
  k.imgP = (const T*)a.imgP;
  k.imgTP = (const T*)a.imgTP;
  k.out = (T*)a.out;
  k.r = (T*)a.r;
  k.b = (const T*)a.b;
  k.R = (const T*)a.R;
  k.ang = g.d_fwd;
  k.wins = (const int2*)g.d_fwd_wins;
  k.blk = (const FwdBlk*)g.d_fwd_blk;
  k.part = a.part;
  k.nbx = (g.nb + kBins - 1) / kBins;
  k.maxb = g.fwd_maxb;
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
  TimedLaunch tl(TK_FORWARD, st);
  if (mode == FWD_COUNT) {
    const size_t rays = g.M();
    hipLaunchKernelGGL(k_count, dim3((unsigned)((rays + 255) / 256)), dim3(256), 0, st, g.d_fwd,
                       g.n, g.nb, g.m, a.count);
    HIP_CHECK(hipGetLastError());
    return;
  }
  dim3 grid((g.nb + kBins - 1) / kBins, g.ngroups);
  FwdK<T> k = make_args<T>(g, a);
  if (g.fwd_halves == 2) {
    const dim3 blk(kFwdThreads<2>);
    switch (mode) {
      case FWD_PLAIN: hipLaunchKernelGGL((k_forward<T, FWD_PLAIN, 2>), grid, blk, 0, st, k); break;
      case FWD_CGLS: hipLaunchKernelGGL((k_forward<T, FWD_CGLS, 2>), grid, blk, 0, st, k); break;
      case FWD_SIRT: hipLaunchKernelGGL((k_forward<T, FWD_SIRT, 2>), grid, blk, 0, st, k); break;
      default: break;
    }
  } else {
    const dim3 blk(kFwdThreads<1>);
    switch (mode) {
      case FWD_PLAIN: hipLaunchKernelGGL((k_forward<T, FWD_PLAIN, 1>), grid, blk, 0, st, k); break;
      case FWD_CGLS: hipLaunchKernelGGL((k_forward<T, FWD_CGLS, 1>), grid, blk, 0, st, k); break;
      case FWD_SIRT: hipLaunchKernelGGL((k_forward<T, FWD_SIRT, 1>), grid, blk, 0, st, k); break;
      default: break;
    }
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace

void build_forward_windows(Geometry& g, hipStream_t st) {
  const int band = g.f64 ? kBand<double> : kBand<float>;
  const int nbx = (g.nb + kBins - 1) / kBins;
  g.fwd_maxb = (g.n + band - 1) / band;
  const size_t nblk = (size_t)g.ngroups * nbx;
  HIP_CHECK(hipMalloc(&g.d_fwd_rows, sizeof(int2) * nblk));
  HIP_CHECK(hipMalloc(&g.d_fwd_wins, sizeof(int2) * nblk * g.fwd_maxb));
  HIP_CHECK(hipMalloc(&g.d_fwd_order, sizeof(int) * nblk));
  const long long total = (long long)nblk * (g.fwd_maxb + 1);
  hipLaunchKernelGGL(k_fwd_windows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     g.d_fwd, g.d_groups, g.ngroups, nbx, g.n, g.nb, band, g.fwd_maxb,
                     (int2*)g.d_fwd_rows, (int2*)g.d_fwd_wins);
  HIP_CHECK(hipGetLastError());
  // Grid order: blocks walk from 1 to n rows depending on how far their bins
  // are from the detector centre.  Sorted by rows (most first) and dealt out
  // in rounds of one block per CU, every run of consecutive grid positions of
  // one CU count holds a similar amount of work; blocks are dispatched in grid
  // order.  Within a round, positions p with p % 8 == x run on XCD x (blocks
  // are dealt to the eight XCDs round-robin): each XCD is given a contiguous
  // run of the round's blocks ordered by bin block, then angle group, so the
  // blocks one XCD holds stage overlapping image strips (the same bins at
  // neighbouring angles) through its L2.
  std::vector<int2> rows(nblk);
  HIP_CHECK(hipMemcpyAsync(rows.data(), g.d_fwd_rows, sizeof(int2) * nblk, hipMemcpyDeviceToHost,
                           st));
  HIP_CHECK(hipStreamSynchronize(st));
  std::vector<int> byrows(nblk);
  for (size_t i = 0; i < nblk; ++i) byrows[i] = (int)i;
  std::stable_sort(byrows.begin(), byrows.end(), [&](int a, int b) {
    return rows[a].y - rows[a].x > rows[b].y - rows[b].x;
  });
  int cus = 0;
  HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g.device));
  const size_t P = (size_t)std::max(cus, 1);
  // Two threads per ray when the grid has fewer than 8 blocks per CU (a few
  // resident blocks per CU, all started at once): twice the waves per SIMD to
  // hide latencies.  Larger grids keep one thread per ray: fewer instructions
  // per update, and their VALU issue is the limit.
  g.fwd_halves = nblk < 8 * P ? 2 : 1;
  std::vector<int> order(nblk);
  constexpr size_t kXcds = 8;
  for (size_t base = 0; base < nblk; base += P) {
    const size_t width = std::min(P, nblk - base);
    std::vector<int> round(byrows.begin() + base, byrows.begin() + base + width);
    // block lb = angle group * nbx + bin block: order by bin block, then group
    std::sort(round.begin(), round.end(), [&](int a, int b) {
      const int ba = a % nbx, bb = b % nbx;
      return ba != bb ? ba < bb : a < b;
    });
    size_t i = 0;
    for (size_t x = 0; x < kXcds && x < width; ++x)
      for (size_t p = x; p < width; p += kXcds) order[base + p] = round[i++];
  }
  HIP_CHECK(hipMemcpyAsync(g.d_fwd_order, order.data(), sizeof(int) * nblk, hipMemcpyHostToDevice,
                           st));
  // per grid position: the block's record (its first two band windows from
  // the table the setup kernel wrote)
  std::vector<int> groups((size_t)g.ngroups * kSlots);
  std::vector<int2> wins(nblk * (size_t)g.fwd_maxb);
  HIP_CHECK(hipMemcpyAsync(groups.data(), g.d_groups, sizeof(int) * groups.size(),
                           hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipMemcpyAsync(wins.data(), g.d_fwd_wins, sizeof(int2) * wins.size(),
                           hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  std::vector<FwdBlk> recs(nblk);
  for (size_t pos = 0; pos < nblk; ++pos) {
    const int lb = order[pos];
    const int gi = lb / nbx, bx = lb - gi * nbx;
    FwdBlk& r = recs[pos];
    std::memset(&r, 0, sizeof(r));
    r.lb = lb;
    r.jfirst = bx * kBins;
    r.jlast = std::min(r.jfirst + kBins - 1, g.nb - 1);
    r.lo = rows[lb].x;
    r.hi = rows[lb].y;
    r.nbands = r.hi >= r.lo ? (r.hi - r.lo + band) / band : 0;
    r.k0 = groups[(size_t)gi * kSlots];
    r.major = g.h_fwd[r.k0].major;
    const int2* wb = wins.data() + (size_t)lb * g.fwd_maxb;
    if (r.nbands > 0) { r.w0x = wb[0].x; r.w0y = wb[0].y; }
    if (r.nbands > 1) { r.w1x = wb[1].x; r.w1y = wb[1].y; }
    for (int s = 0; s < kSlots; ++s) r.k[s] = groups[(size_t)gi * kSlots + s];
  }
  HIP_CHECK(hipMalloc(&g.d_fwd_blk, sizeof(FwdBlk) * nblk));
  HIP_CHECK(hipMemcpyAsync(g.d_fwd_blk, recs.data(), sizeof(FwdBlk) * nblk, hipMemcpyHostToDevice,
                           st));
  HIP_CHECK(hipStreamSynchronize(st));
}

int forward_blocks(const Geometry& g) { return ((g.nb + kBins - 1) / kBins) * g.ngroups; }

void launch_forward(const Geometry& g, FwdMode mode, const FwdArgs& a, hipStream_t st) {
  if (g.f64) fwd_dispatch<double>(g, mode, a, st);
  else fwd_dispatch<float>(g, mode, a, st);
}

void prepare_forward_batch(FwdTables& t, const std::vector<const Geometry*>& gs,
                           const std::vector<FwdArgs>& as, hipStream_t st) {
  for (int h = 1; h <= 2; ++h) {   // the problems' order is kept within each table
    std::vector<FwdK<float>> host;
    std::vector<int> blocks, widths;
    for (size_t i = 0; i < gs.size(); ++i) {
      if (gs[i]->f64) fail(RECO_EINVAL, "batched solves take float32 geometries");
      if (gs[i]->fwd_halves != h) continue;
      host.push_back(make_args<float>(*gs[i], as[i]));
      widths.push_back((gs[i]->nb + kBins - 1) / kBins);
      blocks.push_back(widths.back() * gs[i]->ngroups);
    }
    t.t[h - 1].upload(host.data(), sizeof(FwdK<float>), blocks, widths, st);
  }
}

template <int H>
static void launch_forward_batch_h(const DevTable& t, FwdMode mode, hipStream_t st) {
  if (t.count == 0) return;
  TimedLaunch tl(TK_FORWARD, st);
  const auto* args = (const FwdK<float>*)t.args;
  const dim3 blk(kFwdThreads<H>);
  switch (mode) {
    case FWD_PLAIN:
      hipLaunchKernelGGL((k_forward_batch<float, FWD_PLAIN, H>), dim3(t.total_blocks), blk, 0, st,
                         args, t.start, t.gx, t.count);
      break;
    case FWD_CGLS:
      hipLaunchKernelGGL((k_forward_batch<float, FWD_CGLS, H>), dim3(t.total_blocks), blk, 0, st,
                         args, t.start, t.gx, t.count);
      break;
    default: fail(RECO_EINVAL, "unsupported batched forward mode");
  }
  HIP_CHECK(hipGetLastError());
}

void launch_forward_batch(const FwdTables& t, FwdMode mode, hipStream_t st) {
  launch_forward_batch_h<1>(t.t[0], mode, st);
  launch_forward_batch_h<2>(t.t[1], mode, st);
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
