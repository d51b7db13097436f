// Solver workspaces and driver entry points (internal).
#pragma once

#include "internal.h"

namespace reco {

struct HybridScratch;

// Per-solve device buffers, pooled per geometry.
struct Workspace {
  void *r = nullptr, *q = nullptr;            // [M] residual, projected direction
  void *s = nullptr, *p = nullptr;            // [N] normal-equation residual, direction
  void *zP = nullptr, *zTP = nullptr;         // padded preconditioned residual (+ transpose)
  // allocated on first use by SIRT / GMRES (CGLS needs none of them):
  void *xP = nullptr, *xTP = nullptr;         // padded iterate copies (SIRT, GMRES)
  void *tmp = nullptr;                        // [max(N, M)]
  void *fvec = nullptr;                       // [N] right-hand side W^T b (GMRES)
  double* partial = nullptr;                  // reduction partials [red_cap], then the
                                              // forward projection's CGLS partials [red_cap / 4],
                                              // then the finisher slots [red_cap]
  unsigned* counter = nullptr;                // 4 ticket counters
  int red_cap = 0;
  SolverState* st = nullptr;                  // device state
  SolverState* h_st = nullptr;                // pinned host copy
  double* hist = nullptr;
  int hist_cap = 0;
  void* V = nullptr;                          // GMRES basis [(restart+1) x N]
  int v_cap = 0;                              // vectors allocated in V
  double* gm = nullptr;                       // GMRES / BiCGStab small dense data
  size_t gm_cap = 0;                          // doubles allocated in gm
  bool tainted = false;                       // last solve ended abnormally: never pooled
  HybridScratch* hyb = nullptr;               // hybrid wavelet cycle buffers (first use)
  ~Workspace();
};

Workspace* checkout_workspace(Geometry& g, hipStream_t st);
// Pool w again, or free it (after waiting for the device) when w->tainted or
// its last polled state says a reduction gave up.  True when pooled.
bool return_workspace(Geometry& g, Workspace* w);
void release_workspaces(Geometry& g);
void ensure_aux(Geometry& g, Workspace& w);     // xP, xTP, tmp, fvec
void ensure_history(Workspace& w, int cap);
RedScratch red_of(Workspace& w, int slot);
double* fwd_partials(Workspace& w);             // the forward projection's CGLS partials
double* fin_slots(Workspace& w);                // the backprojection's finisher slots (empty-marked)
// Device bytes of one CGLS workspace / of a geometry's own tables, for the
// geometry described by d (used for admission by memory budget).
size_t cgls_workspace_bytes(const reco_geometry_desc& d);
size_t geometry_bytes(const reco_geometry_desc& d);

void validate_opts(const reco_solve_opts& o, bool gmres);
reco_status status_of(int done);
double now_ms();

reco_status solve_cgls(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                       reco_solve_info* info, hipStream_t st);
// CGLS with every buffer in the library's fixed scratch array (no allocation).
reco_status solve_cgls_noalloc(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                               reco_solve_info* info, hipStream_t st);
reco_status solve_sirt(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                       reco_solve_info* info, hipStream_t st);
reco_status solve_bicgstab(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                           reco_solve_info* info, hipStream_t st);
reco_status solve_gmres(Geometry& g, const void* b, void* x, const reco_solve_opts& o,
                        reco_solve_info* info, hipStream_t st);

}  // namespace reco
