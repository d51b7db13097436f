// The paper's hybrid wavelet multigrid cycle with exact coarsest solves
// (Section 3.1.2, hybrid variant; recursion of Section 3.1.3; Cholesky
// coarsest solves of Section 4.1).  Internal declarations.
#pragma once

#include "internal.h"

namespace reco {

// Pivots of the coarsest Cholesky factorisations at most this fraction of the
// largest coarsest diagonal entry are dropped (zero correction).
constexpr double kHybridDropRel = 1e-12;
// Largest supported hierarchy and factor storage.
constexpr int kHybridMaxLevels = 3;
constexpr size_t kHybridMaxFactorBytes = size_t(8) << 30;

// Inverse Cholesky factors of the 4^L coarsest Galerkin blocks
// A_p = V_p^T (W^T W + lambda I) V_p, one per packet p (tile-local Walsh
// index (py, px), block index py * 2^L + px), each c x c with c = (n / 2^L)^2
// unknowns ordered by tile, row-major.  X = L^-1 (lower triangular) and its
// transpose XT, float64; rows and columns of dropped unknowns are zero, so
// A_p^-1 r = XT (X r) on the kept unknowns and 0 on the dropped ones.
struct HybridFactors {
  int L = 0, TS = 1, tiles = 0, c = 0, leaves = 0;
  double lambda = 0.0;
  double* X = nullptr;    // [leaves][c][c]
  double* XT = nullptr;   // [leaves][c][c]
  int dropped = 0;        // unknowns dropped over all blocks
  ~HybridFactors();
};

// Per-solve buffers of the cycle (owned by a workspace).
struct HybridScratch {
  void* coefR[kHybridMaxLevels + 1] = {};   // residuals per depth, coefficient layout [n][n]
  void* coefE = nullptr;                    // correction, coefficient layout
  void* img = nullptr;                      // [n][n]
  void* P = nullptr;                        // padded pair for the Galerkin applies
  void* TP = nullptr;
  void* sino = nullptr;                     // [m][nb]
  double* y = nullptr;                      // [3 c] leaf intermediate
  ~HybridScratch();
};

// Throws RECO_EINVAL when the geometry cannot hold the hybrid cycle.
void validate_hybrid(const Geometry& g);
// The factors for lambda, built on first use (synchronously on `st`) and
// cached on the geometry per lambda until it is destroyed.
const HybridFactors& ensure_hybrid(Geometry& g, double lambda, hipStream_t st);
HybridScratch& hybrid_scratch(const Geometry& g, Workspace& w, hipStream_t st);
// z = M^-1 r for the hybrid cycle: r an image [n][n] (geometry dtype); the
// result is written to the padded pair (outP, outTP; interiors only) and/or
// the plain image outPlain (each may be null).
void hybrid_apply(const Geometry& g, const HybridFactors& f, HybridScratch& s, const void* r,
                  void* outP, void* outTP, void* outPlain, hipStream_t st);

}  // namespace reco
