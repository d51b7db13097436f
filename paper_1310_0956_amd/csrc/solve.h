// Solver workspaces and driver entry points (internal).
#pragma once

#include "internal.h"

namespace reco {

// Per-solve device buffers, pooled per geometry.
struct Workspace {
  void *r = nullptr, *q = nullptr;            // [M] residual, projected direction
  void *s = nullptr, *p = nullptr;            // [N] normal-equation residual, direction
  void *zP = nullptr, *zTP = nullptr;         // padded preconditioned residual (+ transpose)
  void *xP = nullptr, *xTP = nullptr;         // padded iterate copies (SIRT, GMRES)
  void *tmp = nullptr;                        // [max(N, M)]
  void *fvec = nullptr;                       // [N] right-hand side W^T b (GMRES)
  double* partial = nullptr;                  // reduction partials
  unsigned* counter = nullptr;                // 4 ticket counters
  int red_cap = 0;
  SolverState* st = nullptr;                  // device state
  SolverState* h_st = nullptr;                // pinned host copy
  double* hist = nullptr;
  int hist_cap = 0;
  void* V = nullptr;                          // GMRES basis [(restart+1) x N]
  int v_cap = 0;                              // vectors allocated in V
  double* gm = nullptr;                       // GMRES small dense data
  ~Workspace();
};

Workspace* checkout_workspace(Geometry& g, hipStream_t st);
void return_workspace(Geometry& g, Workspace* w);
void release_workspaces(Geometry& g);
RedScratch red_of(Workspace& w, int slot);

reco_status solve_cgls(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                       reco_solve_info* info, hipStream_t st);
reco_status solve_sirt(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                       reco_solve_info* info, hipStream_t st);
reco_status solve_gmres(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                        reco_solve_info* info, hipStream_t st);

}  // namespace reco
