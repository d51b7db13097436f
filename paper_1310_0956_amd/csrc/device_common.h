// Device helpers shared by the kernels: wave64 reductions, fixed-order block
// reductions, the last-block finalisation pattern and the finisher pattern
// (both deterministic: partials are summed in block order, by whichever block
// finishes last or by the block dispatched last).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace reco {

// Value of lane (lane ^ MASK) for MASK < 16, with DPP lane moves inside a row
// of 16 lanes: xor 1 and 2 by quad permutes, 8 by a row rotation by 8, 7 by a
// half-row mirror, 4 by the half-row mirror followed by the quad permute
// i -> i ^ 3.  Larger masks use a general lane permute.
template <int MASK>
__device__ __forceinline__ int xor_lane_b32(int v) {
  if constexpr (MASK == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
  else if constexpr (MASK == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
  else if constexpr (MASK == 4)
    return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true), 0x1B, 0xF,
                                    0xF, true);
  else if constexpr (MASK == 7) return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);
  else if constexpr (MASK == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);
  else return __shfl_xor(v, MASK, 64);
}

template <int MASK>
__device__ __forceinline__ float xor_lane(float v) {
  return __builtin_bit_cast(float, xor_lane_b32<MASK>(__builtin_bit_cast(int, v)));
}
template <int MASK>
__device__ __forceinline__ double xor_lane(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = xor_lane_b32<MASK>((int)b), hi = xor_lane_b32<MASK>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// A wave-uniform float64 held in scalar registers (vector arithmetic leaves
// its results in vector registers).
__device__ __forceinline__ double uniform(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

// Sum over the 64 lanes, the same value in every lane: butterflies within
// each row of 16 lanes (DPP lane moves; every lane of a row ends with the
// same row sum, each pairwise add being commutative), then the four row sums
// in row order.  All lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += xor_lane<1>(v);
  v += xor_lane<2>(v);
  v += xor_lane<4>(v);
  v += xor_lane<8>(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum W values over a block of NW waves in a fixed order.  Result valid in
// thread 0.  `sh` must hold NW*W doubles.
template <int W, int NW = 4>
__device__ __forceinline__ void block_sum(double (&v)[W], double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < W; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < W; ++i) sh[wv * W + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // in wave order; two waves' values in flight at a time keeps the
    // register count low
    double t[W];
#pragma unroll
    for (int i = 0; i < W; ++i) t[i] = sh[i];
#pragma unroll 2
    for (int w = 1; w < NW; ++w) {
#pragma unroll
      for (int i = 0; i < W; ++i) t[i] += sh[w * W + i];
    }
#pragma unroll
    for (int i = 0; i < W; ++i) v[i] = t[i];
  }
  __syncthreads();
}

// Marks every word of s as read and rewritten here, in vector registers: a
// value loaded earlier is then first used (and waited for) at this point.
template <typename S>
__device__ __forceinline__ void in_vgprs(S& s) {
  static_assert(sizeof(S) % 4 == 0, "whole words");
  unsigned w[sizeof(S) / 4];
  __builtin_memcpy(w, &s, sizeof(S));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) asm volatile("" : "+v"(w[i]));
  __builtin_memcpy(&s, w, sizeof(S));
}

template <int W>
__device__ __forceinline__ void block_sum256(double (&v)[W], double* sh) {
  block_sum<W, 4>(v, sh);
}

// Each block contributes W partial sums; the last block to arrive sums them in
// block order and calls fin(totals) from thread 0.  Returns normally in every
// block; the counter is reset for the next use.  Blocks have NW waves.
//
// Visibility without a full L2 writeback: the partials are written with
// agent-scope atomic stores, which write through to the device-coherent
// level, and the block waits for their completion (vmcnt) before taking its
// ticket; the last block reads them with agent-scope atomic loads.  The wait
// covers every outstanding memory access of thread 0's wave, so callers issue
// their bulk stores after this call.  Results the finisher writes to the
// solver state are read by later launches (kernel boundaries order them).
template <int W, int NW = 4, typename F>
__device__ __forceinline__ void reduce_and_finish(double (&v)[W], const RedScratch& red,
                                                  int nblocks, int block_id, F fin) {
  __shared__ double sh[NW * W];
  __shared__ int am_last;
  block_sum<W, NW>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < W; ++i)
      __hip_atomic_store(&red.partial[(size_t)block_id * W + i], v[i], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const unsigned t =
        __hip_atomic_fetch_add(red.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (t == (unsigned)nblocks - 1u);
  }
  __syncthreads();
  if (!am_last) return;
  double acc[W];
#pragma unroll
  for (int i = 0; i < W; ++i) acc[i] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += NW * 64) {
#pragma unroll
    for (int i = 0; i < W; ++i)
      acc[i] += __hip_atomic_load(&red.partial[(size_t)b * W + i], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum<W, NW>(acc, sh);
  if (threadIdx.x == 0) {
    fin(acc);
    __hip_atomic_store(red.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Buffer resource over a device array of `bytes` < 2^31 bytes (geometry
// validation bounds every image copy and sinogram): loads at byte offsets at
// or past the end read 0 instead of faulting.
constexpr int kBufferFlags = 0x00020000;   // raw 32-bit dword access (gfx9 family)
constexpr unsigned kOutside = 0x80000000u; // an offset past the end of every such buffer

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           kBufferFlags);
}

__device__ __forceinline__ float load_elem(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff, float) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}
__device__ __forceinline__ double load_elem(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff, double) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0);
  const unsigned lo = v[0], hi = v[1];
  return __hiloint2double((int)hi, (int)lo);
}

// A reduction without a ticket, for kernels whose blocks are all dispatched
// before the last one (no block waits for another to start).  Every block
// stores its W partial sums into its slots (component-major: slot i of
// block b at i * nblocks + b, so the finisher's loads are coalesced) with
// write-through stores and goes on without waiting; the block dispatched last (block_id nblocks - 1)
// then polls all slots until none holds the empty mark, sums them in the
// fixed order of reduce_and_finish, marks them empty again for the next use
// and calls fin(totals, late) from thread 0.  The slots must hold the empty
// mark on entry (they are filled with it when allocated).  The blocks it
// waits for hold nothing it needs, so the poll ends; it still gives up after
// kPollTicks of the 100 MHz constant clock and then passes late = true.
// Non-finisher blocks return at once: their bulk stores need no ordering.
// pre() runs in the finisher once the poll is done (loads whose latency
// then overlaps the block sum); its result is passed to fin.
constexpr unsigned long long kPollTicks = 1000000000ull;   // 10 s

template <int W, int NW = 4, typename P, typename F>
__device__ __forceinline__ void reduce_to_finisher(double (&v)[W], double* __restrict__ slots,
                                                   int nblocks, int block_id, P pre, F fin) {
  __shared__ double sh[NW * W];
  __shared__ int late;
  if (threadIdx.x == 0) late = 0;
  block_sum<W, NW>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < W; ++i)
      __hip_atomic_store(&slots[(size_t)i * nblocks + block_id], v[i], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  if (block_id != nblocks - 1) return;
  unsigned long long* bits = reinterpret_cast<unsigned long long*>(slots);
  const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
  double acc[W];
  bool full = false;
  for (;;) {
    // one pass over this thread's slots (blocks tid, tid + stride, ...), in
    // batches of four blocks whose loads are all issued before the first sum
    constexpr int kStride = NW * 64, kBatch = 4;
    full = true;
#pragma unroll
    for (int i = 0; i < W; ++i) acc[i] = 0.0;
    for (int b0 = threadIdx.x; b0 < nblocks; b0 += kBatch * kStride) {
      unsigned long long u[kBatch][W];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        // batch entries past the last block for the whole wave are not loaded
        const bool wave_in = __builtin_amdgcn_readfirstlane(b0 + k * kStride) < nblocks;
        const int b = min(b0 + k * kStride, nblocks - 1);
#pragma unroll
        for (int i = 0; i < W; ++i)
          u[k][i] = wave_in ? __hip_atomic_load(&bits[(size_t)i * nblocks + b], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT)
                            : kSlotEmpty;
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        if (b0 + k * kStride < nblocks) {
#pragma unroll
          for (int i = 0; i < W; ++i) {
            full = full && u[k][i] != kSlotEmpty;
            acc[i] += __builtin_bit_cast(double, u[k][i]);
          }
        }
      }
    }
    if (full || __builtin_amdgcn_s_memrealtime() - t0 > kPollTicks) break;
    __builtin_amdgcn_s_sleep(8);
  }
  const auto snap = pre();
  if (!full) late = 1;
  for (int b = threadIdx.x; b < nblocks; b += NW * 64) {
#pragma unroll
    for (int i = 0; i < W; ++i)
      __hip_atomic_store(&bits[(size_t)i * nblocks + b], kSlotEmpty, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum<W, NW>(acc, sh);
  // the snapshot's first use: left to itself the compiler moved its uniform
  // fields to scalar registers right after the loads, waiting for them
  // before the block sum
  auto snap_v = snap;
  in_vgprs(snap_v);
  if (threadIdx.x == 0) fin(acc, late != 0, snap_v);
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// End of the preconditioning step of a CGLS iteration, run once by the last
// block from the totals t = {<s,z>, ||s||^2, ||z||^2, <z,p>} (p = the current
// direction; only used with lambda > 0).  init: the step before the first
// iteration (z_0 = M^-1 s_0, gamma_0 = <s_0,z_0>, reference norm ||s_0||).
// Otherwise: beta = gamma'/gamma, the squared norm of the next direction
// z + beta p, the relative residual ||s|| / ||s_0|| and the stopping test.
// degen (the iteration's delta = ||q||^2 + lambda ||p||^2 was not positive
// and finite: 1 zero, 3 non-finite): the iteration took no step; the solve
// ends with that code and the iteration is not counted.
__device__ __forceinline__ int cgls_degenerate(double delta) {
  return !finite(delta) ? 3 : (delta <= 0.0 ? 1 : 0);
}
// The state fields the step reads, taken ahead of the totals (a finisher
// loads them before it polls, off the end of the launch's critical path).
struct CglsScalars {
  double gamma, pp, s0, tol;
  int iter, max_iter, fixed, hist_cap;
  double* hist;
};
__device__ __forceinline__ CglsScalars cgls_scalars(const SolverState* st) {
  return CglsScalars{st->gamma, st->pp,       st->s0,    st->tol, st->iter,
                     st->max_iter, st->fixed, st->hist_cap, st->hist};
}
__device__ __forceinline__ void cgls_precond_finish(SolverState* st, const CglsScalars& c,
                                                    const double (&t)[4], bool init,
                                                    int degen = 0) {
  if (degen) {
    st->done = degen;
    return;
  }
  if (init) {
    st->gamma = t[0];
    st->s0 = sqrt(t[1]);
    st->beta = 0.0;
    st->pp = t[2];
    st->relres = 1.0;
    st->iter = 0;
    st->init = 1;
    const double s0 = sqrt(t[1]);
    if (!finite(s0) || !finite(t[0])) st->done = 3;
    else if (s0 == 0.0) { st->done = 1; st->relres = 0.0; }
    return;
  }
  const double g = t[0];
  const double beta = g / c.gamma;
  st->pp = t[2] + 2.0 * beta * t[3] + beta * beta * c.pp;
  st->beta = beta;
  st->gamma = g;
  const int iter = c.iter + 1;
  st->iter = iter;
  const double rr = sqrt(t[1]) / c.s0;
  st->relres = rr;
  if (c.hist && iter <= c.hist_cap) c.hist[iter - 1] = rr;
  if (!finite(rr) || !finite(beta)) st->done = 3;
  else if (c.fixed) { if (iter >= c.max_iter) st->done = 1; }
  else if (rr <= c.tol) st->done = 1;
  else if (iter >= c.max_iter) st->done = 2;
  else if (g == 0.0) st->done = 1;
}
__device__ __forceinline__ void cgls_precond_finish(SolverState* st, const double (&t)[4],
                                                    bool init, int degen = 0) {
  cgls_precond_finish(st, cgls_scalars(st), t, init, degen);
}

// Wave issue priority 0..3 (higher issues first; equal priorities issue
// oldest first).  Blocks that share a CU raise the priority of the ones with
// more work left, so they finish together instead of leaving the last block
// to run alone with too few waves to hide its latencies.
__device__ __forceinline__ void set_priority(int p) {
  switch (p) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
  }
}

// Position of a block within its problem's grid.
// Block coordinates (x, y) in a gx x gy grid and the block's linear dispatch
// index `lin` (its slot in reductions; the highest one is dispatched last).
struct BlockPos {
  int x, y, gx, gy, lin;
  __device__ __forceinline__ int id() const { return lin; }
  __device__ __forceinline__ int count() const { return gx * gy; }
};

__device__ __forceinline__ BlockPos grid_pos() {
  return BlockPos{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y,
                  (int)(blockIdx.y * gridDim.x + blockIdx.x)};
}

// XCD-aware tile order.  Blocks are dealt to the eight XCDs round-robin by
// dispatch index, so the blocks with lin % 8 == x share XCD x's L2.  XCD x is
// given the x-th contiguous run of tiles in an order of 8-tile-wide column
// bands (row-major within a band), so the tiles resident together on one XCD
// are neighbours along both axes and read overlapping data through its L2.
// A bijection of the grid; `lin` is kept.
__device__ __forceinline__ BlockPos xcd_tile(const BlockPos b) {
  constexpr int kBand = 8;
  const int cnt = b.gx * b.gy, q = cnt >> 3, r = cnt & 7, xcd = b.lin & 7, j = b.lin >> 3;
  const int t = xcd * q + min(xcd, r) + j;   // position in the band order
  const int full = b.gx / kBand, span = kBand * b.gy;
  int tx, ty;
  if (t < full * span) {
    const int band = t / span, rem = t - band * span;
    ty = rem / kBand;
    tx = band * kBand + (rem - ty * kBand);
  } else {
    const int rem = t - full * span, w = b.gx - full * kBand;
    ty = rem / w;
    tx = full * kBand + (rem - ty * w);
  }
  return BlockPos{tx, ty, b.gx, b.gy, b.lin};
}

// Problem owning flat block b in a batched launch: the last r with start[r] <= b.
__device__ __forceinline__ int batch_find(const int* __restrict__ start, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ BlockPos batch_pos(const int* __restrict__ start,
                                              const int* __restrict__ gx, int r) {
  const int lb = (int)blockIdx.x - start[r];
  const int w = gx[r];
  return BlockPos{lb % w, lb / w, w, (start[r + 1] - start[r]) / w, lb};
}

}  // namespace reco
