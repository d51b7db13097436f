// Geometry object: validation, per-angle tables, device allocations.
//
// Angles theta_k = k*pi/m over 180 degrees (Section 4.1: equiangular over
// 180 degrees); k = 0 and 2k = m are snapped to the axes by index so that
// rays parallel to the grid are exactly parallel.  Bins are one pixel wide and
// centred: ray (k, j) is p.(cos, sin) = (j - (nb-1)/2) h with h = 2/n.
#include <cmath>
#include <cstring>

#include "hybrid.h"
#include "internal.h"

namespace reco {

namespace {
constexpr double kAxisSlope = 1048576.0;  // 2^20: stands in for 1/0 at axis angles

void direction(int k, int m, double& c, double& s) {
  if (k == 0) { c = 1.0; s = 0.0; return; }
  if (2 * k == m) { c = 0.0; s = 1.0; return; }
  const double t = (double)k * M_PI / (double)m;
  c = std::cos(t);
  s = std::sin(t);
}
}  // namespace

// Both kernels weigh, per row (column) crossed, the two pixels nearest to the
// ray with w0 = clamp((1/2 - f) B + C, 0, 1/u), w1 = 1/u - w0 (units of h; f the
// fractional crossing position, u >= v the larger and smaller of |cos|, |sin|).
// Exact lengths: B = 1/v, a trapezoid in the ray offset with plateau (u - v)/2
// and support (u + v)/2.  Joseph's kernel is the same form with v replaced by u
// in the weights (B = 1/u: w0 = (1 - f)/u, the linear interpolation), a
// triangle of support u; the ray directions are unchanged.
void build_angle_tables(Geometry& g) {
  const int n = g.n, m = g.m, nb = g.nb;
  const bool joseph = g.desc.projector == RECO_PROJ_JOSEPH;
  g.h_fwd.resize(m);
  g.h_bwd.resize(m);
  const double hc = 0.5 * (n - 1), hb = 0.5 * (nb - 1);
  for (int k = 0; k < m; ++k) {
    double c, s;
    direction(k, m, c, s);
    // ---- forward: walk the major axis
    FwdAngle f{};
    f.major = (std::fabs(c) >= std::fabs(s)) ? 0 : 1;
    const double a = f.major ? s : c;   // |a| = u >= |b| = v
    const double b = f.major ? c : s;
    const double u = std::fabs(a), v = joseph ? u : std::fabs(b);
    f.A0 = hc + (hc * b - hb) / a;
    f.inv = 1.0 / a;
    f.slope = -b / a;
    f.dP = std::llrint(f.slope * 4294967296.0);
    // the trapezoid's slope 1/v and offset 1/(2u), divided by Wmax = 1/u
    f.B = (v > 0 ? 1.0 / v : kAxisSlope) * u;
    f.C = 0.5;
    f.Wmax = 1.0 / u;
    f.Bf = (float)f.B;
    f.Cf = (float)f.C;
    f.Wmaxf = (float)f.Wmax;
    g.h_fwd[k] = f;
    // ---- backward: trapezoid in bin units
    BwdAngle w{};
    const double uu = std::max(std::fabs(c), std::fabs(s));
    const double vv = joseph ? uu : std::min(std::fabs(c), std::fabs(s));
    w.c = c;
    w.s = s;
    // the trapezoid's slope 1/(uu vv) and offsets, divided by Wmax = 1/uu
    const double Bt = vv > 0 ? 1.0 / (uu * vv) : kAxisSlope;
    const double Cp = 0.5 / uu;
    w.B = Bt * uu;
    w.C0 = (Cp + 0.5 * uu * Bt) * uu;
    w.C1 = (Cp + (0.5 * uu - 1.0) * Bt) * uu;
    w.Wmax = 1.0 / uu;
    w.cf = (float)c;
    w.sf = (float)s;
    w.Bf = (float)w.B;
    w.C0f = (float)w.C0;
    w.C1f = (float)w.C1;
    w.Wmaxf = (float)w.Wmax;
    w.half_u_plus_v = 0.5 * (uu + vv);
    w.inv_uv_d = Bt;
    w.cc_d = vv > 0 ? (uu + vv) / (2.0 * uu * vv) : 0.5 * kAxisSlope + 0.5;
    w.inv_uv_f = (float)w.inv_uv_d;
    w.cc_f = (float)w.cc_d;
    w.huv_f = (float)w.half_u_plus_v;
    g.h_bwd[k] = w;
  }
}

Geometry::~Geometry() {
  auto f = [](void* p) { if (p) (void)hipFree(p); };
  f(d_fwd);
  f(d_groups);
  f(d_fwd_rows);
  f(d_fwd_wins);
  f(d_fwd_order);
  f(d_fwd_blk);
  f(d_bwd);
  f(d_diag64);
  f(d_diag);
  f(d_sirtR);
  f(d_sirtC);
}

void release_workspaces(Geometry& g);

Geometry* create_geometry(const reco_geometry_desc& d, hipStream_t st) {
  if (d.n < 2 || d.n > 65536) fail(RECO_EINVAL, "n must be in [2, 65536]");
  if (d.n_angles < 1) fail(RECO_EINVAL, "n_angles must be >= 1");
  if (d.n_bins < 1) fail(RECO_EINVAL, "n_bins must be >= 1");
  if (d.wmg_levels < 1 || d.wmg_levels > 6) fail(RECO_EINVAL, "wmg_levels must be in [1, 6]");
  if (d.dtype != RECO_F32 && d.dtype != RECO_F64) fail(RECO_EINVAL, "dtype must be RECO_F32 or RECO_F64");
  if (d.projector != RECO_PROJ_EXACT && d.projector != RECO_PROJ_JOSEPH)
    fail(RECO_EINVAL, "projector must be RECO_PROJ_EXACT or RECO_PROJ_JOSEPH");
  const int L = d.wmg_levels - 1;
  if (d.n % (1 << L) != 0) fail(RECO_EINVAL, "n must be divisible by 2^(wmg_levels-1)");
  // The projectors address the padded image copies and the sinogram with
  // 32-bit byte offsets (buffer loads): each must stay below 2^31 bytes, the
  // image copy with 32 rows to spare (a staged band's rows may run past the
  // last row, and an offset past the end plus a row offset must not wrap).
  const double es = d.dtype == RECO_F64 ? 8.0 : 4.0;
  if ((double)(d.n + 32) * (d.n + 2 * kPad) * es >= 2147483648.0)
    fail(RECO_EINVAL, "image too large: a padded image copy and 32 more rows must stay below "
                      "2^31 bytes (n <= 23150 for RECO_F32, 16364 for RECO_F64)");
  if ((double)d.n_angles * d.n_bins * es >= 2147483648.0)
    fail(RECO_EINVAL, "sinogram too large: n_angles * n_bins * element size must stay below 2^31");

  std::unique_ptr<Geometry> g(new Geometry());
  g->desc = d;
  g->n = d.n;
  g->m = d.n_angles;
  g->nb = d.n_bins;
  g->L = L;
  g->T = 1 << L;
  g->ld = d.n + 2 * kPad;
  g->h = 2.0 / d.n;
  g->f64 = d.dtype == RECO_F64;
  HIP_CHECK(hipGetDevice(&g->device));
  build_angle_tables(*g);
  HIP_CHECK(hipMalloc(&g->d_fwd, sizeof(FwdAngle) * g->m));
  HIP_CHECK(hipMalloc(&g->d_bwd, sizeof(BwdAngle) * g->m));
  // forward angle groups: runs of up to 8 consecutive angles with the same walk axis
  std::vector<int> groups;
  for (int k = 0; k < g->m;) {
    const int major = g->h_fwd[k].major;
    int cnt = 0;
    while (k < g->m && cnt < 8 && g->h_fwd[k].major == major) {
      groups.push_back(k++);
      ++cnt;
    }
    while (cnt++ < 8) groups.push_back(-1);
  }
  g->ngroups = (int)groups.size() / 8;
  HIP_CHECK(hipMalloc(&g->d_groups, sizeof(int) * groups.size()));
  HIP_CHECK(hipMemcpyAsync(g->d_groups, groups.data(), sizeof(int) * groups.size(),
                           hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(g->d_fwd, g->h_fwd.data(), sizeof(FwdAngle) * g->m,
                           hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(g->d_bwd, g->h_bwd.data(), sizeof(BwdAngle) * g->m,
                           hipMemcpyHostToDevice, st));
  build_forward_windows(*g, st);
  HIP_CHECK(hipMalloc(&g->d_diag64, sizeof(double) * g->N()));
  HIP_CHECK(hipMalloc(&g->d_diag, std::max(g->esize() * g->N(), diag_sum_bytes(g->n, g->L))));
  compute_packet_diagonal(*g, st);
  HIP_CHECK(hipStreamSynchronize(st));
  return g.release();
}

}  // namespace reco
