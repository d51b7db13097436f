// Internal declarations of libreco: geometry object, per-angle tables, device
// solver state, kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/reco.h"
#include "pool.h"

namespace reco {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

struct Error {
  reco_status code;
  std::string msg;
};

// Throwing helpers used inside the library; the ABI layer converts them.
[[noreturn]] void fail(reco_status code, const std::string& msg);
void check_hip(hipError_t e, const char* what, const char* file, int line);
#define HIP_CHECK(expr) ::reco::check_hip((expr), #expr, __FILE__, __LINE__)

// ---------------------------------------------------------------------------
// Per-angle tables (host-computed in float64; float copies for the f32 path)
// ---------------------------------------------------------------------------
// Forward projector (ray driven).  For angle k let (a, b) = (cos, sin) when
// |cos| >= |sin| ("major" = 0: the ray is walked row by row over the image),
// else (sin, cos) ("major" = 1: walked column by column over the transposed
// image).  At major index r the ray crosses the minor axis at pixel-index
// position P(j, r) = A0 + j*inv + r*slope; the two pixels floor(P) and
// floor(P)+1 are the only ones with nonzero weight, and with f = P - floor(P)
//   w0/h = Wmax clamp((1/2 - f) * B + C, 0, 1),   w1/h = Wmax - w0/h
// (the weights of one row add up to the row's chord h Wmax = h/|a|; B and C
// are the trapezoid's coefficients divided by its plateau Wmax).
struct FwdAngle {
  double A0, inv, slope;
  long long dP;        // slope in 32.32 fixed point
  int major;
  int pad_;
  double B, C, Wmax;
  float Bf, Cf, Wmaxf, padf_;
};

// Backprojector (pixel driven).  Pixel centre (X, Y) in pixel units from the
// image centre projects to bin coordinate J = X c + Y s + (nb-1)/2; with
// f = J - floor(J) the bins floor(J) and floor(J)+1 carry
//   w0/h = Wmax clamp(C0 - f B, 0, 1),   w1/h = Wmax clamp(C1 + f B, 0, 1)
// (the trapezoid divided by its plateau height Wmax, so that the clamp is the
// unit one).
struct BwdAngle {
  double c, s, B, C0, C1, Wmax;
  float cf, sf, Bf, C0f, C1f, Wmaxf;
  double half_u_plus_v;  // (|c|+|s|)/2: half support of the trapezoid, bins
  double inv_uv_d, cc_d; // 1/(uv) and (u+v)/(2uv) in direct form (setup kernels)
  float inv_uv_f, cc_f, huv_f, padf_;
};

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
struct Workspace;      // solver buffers (solve.hip)
struct HybridFactors;  // coarsest factors of the hybrid wavelet cycle (hybrid.hip)

// Zero columns on each side of the padded image copies read by the forward
// projector (see project.hip).
constexpr int kPad = 4;

// Everything a forward block needs before its first band, gathered per grid
// position at setup so that one load brings it: the 64-byte uniform header,
// then the angle of each of the block's 8 slots (-1 = empty).
struct FwdBlk {
  int lb;                  // block g * (bin blocks) + bin block: its rows and band windows
  int jfirst, jlast;       // bins of the block
  int lo, hi;              // image rows its rays touch
  int major;               // walking axis of its angles
  int k0;                  // first angle (invalid slots shadow it)
  int nbands;
  int w0x, w0y, w1x, w1y;  // column windows of the first two bands
  int pad[4];
  int k[8];
};
static_assert(sizeof(FwdBlk) == 96, "FwdBlk layout");

struct Geometry {
  reco_geometry_desc desc{};
  int n = 0, m = 0, nb = 0, L = 0, T = 1;  // L packet levels, T = 2^L
  int ld = 0;                               // padded row length of image copies (n + 2 kPad)
  double h = 0;
  bool f64 = false;
  int device = 0;

  FwdAngle* d_fwd = nullptr;   // [m]
  int* d_groups = nullptr;     // [ngroups][8] angle groups walked together (forward)
  int ngroups = 0;
  void* d_fwd_rows = nullptr;  // [ngroups * bin blocks] row range of each forward block
  void* d_fwd_wins = nullptr;  // [ngroups * bin blocks][fwd_maxb] band column windows
  int* d_fwd_order = nullptr;  // [ngroups * bin blocks] forward block run at each grid position
  void* d_fwd_blk = nullptr;   // [ngroups * bin blocks] FwdBlk record of each grid position
  int fwd_maxb = 0;
  int fwd_halves = 1;          // threads per ray of the solo forward projector (1 or 2)
  BwdAngle* d_bwd = nullptr;   // [m]
  std::vector<FwdAngle> h_fwd;
  std::vector<BwdAngle> h_bwd;

  // packet diagonal (in-place tile layout, see wmg.hip), float64 always
  double* d_diag64 = nullptr;   // [n*n]
  void* d_diag = nullptr;       // [n*n] in the geometry dtype (for the apply);
                                // max(n*n*esize, diag_sum_bytes) bytes

  // SIRT weights (lazily built): R [M], C [N] in the geometry dtype
  std::mutex sirt_mu;
  void* d_sirtR = nullptr;
  void* d_sirtC = nullptr;

  // pool of solver workspaces
  ReusePool<Workspace> ws_pool;

  // hybrid wavelet cycle: coarsest factors per Tikhonov weight (built on first use)
  std::mutex hyb_mu;
  std::map<double, std::unique_ptr<HybridFactors>> hyb;

  size_t N() const { return (size_t)n * n; }
  size_t M() const { return (size_t)m * nb; }
  size_t esize() const { return f64 ? 8 : 4; }
  size_t padded_elems() const { return (size_t)n * ld; }
  ~Geometry();
};

Geometry* create_geometry(const reco_geometry_desc& d, hipStream_t st);
void build_angle_tables(Geometry& g);

// ---------------------------------------------------------------------------
// Device-side solver state (one per solve; arrays of them for batches)
// ---------------------------------------------------------------------------
struct SolverState {
  double gamma;      // <s, z> of the current iterate
  double beta;       // CG direction coefficient for the next p
  double alpha;
  double delta;
  double pp;         // ||p||^2 of the current direction (Tikhonov term)
  double s0;         // reference norm
  double relres;
  double lambda;
  double tol;
  // (iter, max_iter, fixed, hist_cap and hist are read together by the
  // CGLS scalar step: one aligned 16-byte and one aligned 8-byte load)
  int iter;          // completed iterations
  int max_iter;
  int fixed;         // run exactly max_iter iterations
  int hist_cap;      // capacity of hist
  int done;          // 0 running, 1 converged, 2 cap, 3 non-finite
  int init;          // 1 after the initial step
  double* hist;      // device array of relres per iteration (may be null)
  // GMRES
  int j;             // inner steps done in the current cycle
  int restart;
  double fnorm;      // ||W^T b||
  double wnorm;      // norm of the last orthogonalised vector
};

// Empty mark of the slots of a finisher reduction (partial sums stored
// without a ticket; see reduce_to_finisher): a signalling NaN, a pattern that
// no arithmetic produces.
constexpr unsigned long long kSlotEmpty = 0x7FF4C0FFEE000001ull;

// Reduction scratch handed to kernels that finish with a last-block step.
struct RedScratch {
  double* partial;          // [blocks * width]
  unsigned int* counter;    // zero-initialised ticket counter
  int capacity;             // blocks * width capacity
};

// ---------------------------------------------------------------------------
// Batched launches: one launch covers the blocks of many problems.  A device
// table holds each problem's kernel arguments, the prefix sums of their block
// counts and their grid widths; a block finds its problem by binary search.
// ---------------------------------------------------------------------------
struct DevTable {
  void* args = nullptr;     // [count] kernel argument structs
  int* start = nullptr;     // [count + 1] first flat block of each problem
  int* gx = nullptr;        // [count] grid width of each problem
  int count = 0;
  int total_blocks = 0;
  size_t args_cap = 0, idx_cap = 0;
  void upload(const void* host_args, size_t arg_size, const std::vector<int>& blocks,
              const std::vector<int>& widths, hipStream_t st);
  ~DevTable();
};

// ---------------------------------------------------------------------------
// Kernel launchers (project.hip, backproject.hip, wmg.hip, vec.hip)
// ---------------------------------------------------------------------------
enum FwdMode { FWD_PLAIN = 0, FWD_CGLS = 1, FWD_SIRT = 2, FWD_COUNT = 3 };
enum BwdMode { BWD_PLAIN = 0, BWD_CGLS = 1, BWD_SIRT = 2, BWD_AXPY = 3, BWD_CGLS_INIT = 4 };

struct FwdArgs {
  const void* imgP;    // [n][ld] padded image
  const void* imgTP;   // [n][ld] padded transposed image
  void* out;           // [m][nb]
  void* r;             // CGLS: residual [m][nb] (r -= alpha q_old before q is replaced)
  const void* b;       // SIRT: measured data
  const void* R;       // SIRT: inverse row sums
  SolverState* st;     // CGLS/SIRT: state (may be null)
  RedScratch red;      // unused by the CGLS mode
  double* part;        // CGLS: per-block ||q||^2 partial sums (plain stores; the next
                       // backprojection sums them)
  unsigned long long* count;  // FWD_COUNT: nnz counter
};

struct BwdArgs {
  const void* sino;    // [m][nb] (CGLS: the residual before this iteration's step)
  void* out;           // [n][n] (CGLS: s, written only when the WMG apply is separate)
  const void* x;       // extra-term source (CGLS: current x, updated; AXPY: xin)
  const void* f;       // AXPY: right-hand side term
  const void* C;       // SIRT: inverse column sums
  SolverState* st;
  RedScratch red;
  int x_ld = 0, x_off = 0;       // AXPY: layout of x
  double sa = 1.0, sx = 0.0, sf = 0.0;  // AXPY: out = sa*W^T r + sx*x + sf*f
  // CGLS: the step uses r - alpha q; p = z + beta p and x += alpha p are
  // applied to the tile's pixels, and for 2^L <= 16 the WMG apply of the new
  // s is done in the same launch, writing z to zP / zTP.
  const void* q = nullptr;       // [m][nb] projected direction
  void* p = nullptr;             // [n][n] direction
  void* zP = nullptr;            // padded z (read: previous z; written: new z)
  void* zTP = nullptr;           // padded transposed z (written)
  bool identity = false;         // no preconditioner: z = s
  // CGLS: the preceding forward projection's per-block ||q||^2 partial sums,
  // from which every block forms this iteration's step length
  const double* fwd_part = nullptr;
  int fwd_blocks = 0;
  // CGLS with the WMG apply fused: the finisher reduction's slots [blocks * 4],
  // empty-marked between uses
  double* slots = nullptr;
};
// True when the CGLS backprojection also applies the WMG preconditioner.
bool backward_fuses_wmg(const Geometry& g);

void build_forward_windows(Geometry& g, hipStream_t st);
void launch_pad_transpose(const Geometry& g, const void* x, void* xP, void* xTP,
                          hipStream_t st);
void launch_forward(const Geometry& g, FwdMode mode, const FwdArgs& a, hipStream_t st);
int forward_blocks(const Geometry& g);
void launch_backward(const Geometry& g, BwdMode mode, const BwdArgs& a, hipStream_t st);
int backward_blocks(const Geometry& g);

// WMG apply (wmg.hip)
enum WmgMode { WMG_PLAIN = 0, WMG_CGLS = 1, WMG_CGLS_INIT = 2, WMG_GMRES = 3 };
struct WmgArgs {
  const void* s;        // input image [n][n]
  void* z;              // output plain [n][n] (may be null)
  void* zP;             // output padded (may be null)
  void* zTP;            // output padded transposed (may be null)
  const void* pold;     // CGLS with lambda: previous direction
  double lambda;
  bool identity;        // no preconditioner: z = s
  SolverState* st;
  RedScratch red;
};
void launch_wmg(const Geometry& g, WmgMode mode, const WmgArgs& a, hipStream_t st);
int wmg_blocks(const Geometry& g);
void compute_packet_diagonal(Geometry& g, hipStream_t st);
// Bytes of the packet diagonal's running sums (held, during setup, in the
// memory of the dtype copy of d, which is allocated at least this large).
size_t diag_sum_bytes(int n, int L);

// vector kernels (vec.hip)
void launch_fill(void* p, size_t count, bool f64, double value, hipStream_t st);
void launch_copy(const void* src, void* dst, size_t count, bool f64, hipStream_t st);
void launch_invert(void* v, size_t count, bool f64, hipStream_t st);
// CGLS set-up in one launch: state init, x = p = 0 [N], q = 0 and r = b [M].
void launch_cgls_prepare(SolverState* st, double tol, int max_iter, int fixed, double lambda,
                         double* hist, int hist_cap, void* x, void* p, void* q, void* r,
                         const void* b, size_t N, size_t M, bool f64, hipStream_t s);
void launch_state_init(SolverState* st, double tol, int max_iter, int fixed, double lambda,
                       double* hist, int hist_cap, hipStream_t s);

// batched forms (float problems); the tables are filled by prepare_* and the
// launches may be captured in a HIP graph and replayed.
// The batched forward projection is two launches: the problems whose solo
// launch walks each ray with one thread, and those with two (small grids), so
// that each problem's sums are those of its solo launch.
struct FwdTables {
  DevTable t[2];   // [threads per ray - 1]
};
void prepare_forward_batch(FwdTables& t, const std::vector<const Geometry*>& gs,
                           const std::vector<FwdArgs>& as, hipStream_t st);
void launch_forward_batch(const FwdTables& t, FwdMode mode, hipStream_t st);
void prepare_backward_batch(DevTable& t, const std::vector<const Geometry*>& gs,
                            const std::vector<BwdArgs>& as, hipStream_t st);
void launch_backward_batch(const DevTable& t, BwdMode mode, hipStream_t st);
void prepare_wmg_batch(DevTable& t, const std::vector<const Geometry*>& gs,
                       const std::vector<WmgArgs>& as, hipStream_t st);
void launch_wmg_batch(const DevTable& t, WmgMode mode, hipStream_t st);
struct InitArgs {
  void *x, *p, *q, *r;
  const void* b;
  SolverState* st;
  double tol, lambda;
  double* hist;
  int max_iter, fixed, hist_cap;
};
void prepare_init_batch(DevTable& t, const std::vector<const Geometry*>& gs,
                        const std::vector<InitArgs>& as, hipStream_t st);
void launch_init_batch(const DevTable& t, hipStream_t st);

}  // namespace reco
