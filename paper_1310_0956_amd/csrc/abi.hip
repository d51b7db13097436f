// extern "C" entry points of libreco.  Every call validates its arguments
// before enqueuing work, converts internal failures into status codes and
// records the message for reco_last_error().  Nothing throws across the ABI.
#include <chrono>
#include <cstring>
#include <new>

#include "hybrid.h"
#include "internal.h"
#include "solve.h"

namespace reco {

namespace {
thread_local std::string t_err;
}

void set_error(const std::string& msg) { t_err = msg; }
void clear_error() { t_err.clear(); }

[[noreturn]] void fail(reco_status code, const std::string& msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();
  std::string m = std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" +
                  std::to_string(line) + ")";
  if (e == hipErrorOutOfMemory) throw Error{RECO_ENOMEM, m};
  throw Error{RECO_EDEVICE, m};
}

reco_status solve_batch(int32_t count, const reco_geometry* geoms, const void* const* b,
                        void* const* x, const reco_solve_opts* opts, reco_solve_info* info,
                        hipStream_t st);

}  // namespace reco

using reco::Error;
using reco::Geometry;

template <typename F>
static reco_status guard(F&& body) {
  try {
    reco::clear_error();
    return body();
  } catch (const Error& e) {
    reco::set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    reco::set_error("host allocation failed");
    return RECO_ENOMEM;
  } catch (const std::exception& e) {
    reco::set_error(e.what());
    return RECO_EDEVICE;
  } catch (...) {
    reco::set_error("unknown failure");
    return RECO_EDEVICE;
  }
}
#define RECO_GUARD(...) return guard([&]() -> reco_status __VA_ARGS__);

static Geometry* G(reco_geometry g) {
  if (!g) reco::fail(RECO_EINVAL, "null geometry");
  Geometry* p = reinterpret_cast<Geometry*>(g);
  int dev = -1;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev != p->device) HIP_CHECK(hipSetDevice(p->device));
  return p;
}

static hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

static void need(const void* p, const char* what) {
  if (!p) reco::fail(RECO_EINVAL, std::string("null pointer: ") + what);
}

extern "C" {

const char* reco_last_error(void) { return reco::t_err.c_str(); }

const char* reco_version(void) { return "reco 1.0 (gfx950)"; }

reco_status reco_create_geometry(const reco_geometry_desc* desc, void* stream, reco_geometry* out) {
  RECO_GUARD({
    need(desc, "desc");
    need(out, "out");
    *out = nullptr;
    Geometry* g = reco::create_geometry(*desc, S(stream));
    *out = reinterpret_cast<reco_geometry>(g);
    return RECO_OK;
  })
}

reco_status reco_destroy_geometry(reco_geometry g) {
  RECO_GUARD({
    if (!g) return RECO_OK;
    Geometry* p = G(g);
    reco::release_workspaces(*p);
    delete p;
    return RECO_OK;
  })
}

reco_status reco_geometry_get_desc(reco_geometry g, reco_geometry_desc* desc) {
  RECO_GUARD({
    need(desc, "desc");
    *desc = G(g)->desc;
    return RECO_OK;
  })
}

reco_status reco_packet_diagonal(reco_geometry gh, double* d_host) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(d_host, "d_host");
    const int n = g->n, L = g->L, T = 1 << L;
    std::vector<double> inplace(g->N());
    HIP_CHECK(hipMemcpy(inplace.data(), g->d_diag64, sizeof(double) * g->N(), hipMemcpyDeviceToHost));
    for (int iy = 0; iy < n; ++iy) {
      for (int ix = 0; ix < n; ++ix) {
        const int ly = iy & (T - 1), lx = ix & (T - 1);
        int row = iy >> L, col = ix >> L;
        for (int l = 1; l <= L; ++l) {
          row += ((ly >> (l - 1)) & 1) * (n >> l);
          col += ((lx >> (l - 1)) & 1) * (n >> l);
        }
        d_host[(size_t)row * n + col] = inplace[(size_t)iy * n + ix];
      }
    }
    return RECO_OK;
  })
}

reco_status reco_count_nnz(reco_geometry gh, void* stream, int64_t* nnz) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(nnz, "nnz");
    unsigned long long* d = nullptr;
    HIP_CHECK(hipMalloc(&d, sizeof(unsigned long long)));
    unsigned long long h = 0;
    try {
      HIP_CHECK(hipMemsetAsync(d, 0, sizeof(unsigned long long), S(stream)));
      reco::FwdArgs fa{};
      fa.count = d;
      reco::launch_forward(*g, reco::FWD_COUNT, fa, S(stream));
      HIP_CHECK(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, S(stream)));
      HIP_CHECK(hipStreamSynchronize(S(stream)));
    } catch (...) {
      (void)hipFree(d);
      throw;
    }
    (void)hipFree(d);
    *nnz = (int64_t)h;
    return RECO_OK;
  })
}

reco_status reco_project(reco_geometry gh, const void* x, void* b, void* stream) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(x, "x");
    need(b, "b");
    const size_t bytes = g->esize() * g->padded_elems();
    void* P = nullptr;
    void* PT = nullptr;
    HIP_CHECK(hipMallocAsync(&P, bytes, S(stream)));
    HIP_CHECK(hipMallocAsync(&PT, bytes, S(stream)));
    reco::launch_pad_transpose(*g, x, P, PT, S(stream));
    reco::FwdArgs fa{};
    fa.imgP = P;
    fa.imgTP = PT;
    fa.out = b;
    reco::launch_forward(*g, reco::FWD_PLAIN, fa, S(stream));
    HIP_CHECK(hipFreeAsync(P, S(stream)));
    HIP_CHECK(hipFreeAsync(PT, S(stream)));
    return RECO_OK;
  })
}

reco_status reco_backproject(reco_geometry gh, const void* b, void* x, void* stream) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(x, "x");
    need(b, "b");
    reco::BwdArgs ba{};
    ba.sino = b;
    ba.out = x;
    reco::launch_backward(*g, reco::BWD_PLAIN, ba, S(stream));
    return RECO_OK;
  })
}

reco_status reco_wmg_apply(reco_geometry gh, const void* r, void* z, double lambda, void* stream) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(r, "r");
    need(z, "z");
    if (r == z) reco::fail(RECO_EINVAL, "r and z must not alias");
    if (!(lambda >= 0.0)) reco::fail(RECO_EINVAL, "lambda must be >= 0");
    reco::WmgArgs wa{};
    wa.s = r;
    wa.z = z;
    wa.lambda = lambda;
    reco::launch_wmg(*g, reco::WMG_PLAIN, wa, S(stream));
    return RECO_OK;
  })
}

reco_status reco_wmg_hybrid_apply(reco_geometry gh, const void* r, void* z, double lambda,
                                  void* stream) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(r, "r");
    need(z, "z");
    if (r == z) reco::fail(RECO_EINVAL, "r and z must not alias");
    if (!(lambda >= 0.0)) reco::fail(RECO_EINVAL, "lambda must be >= 0");
    const reco::HybridFactors& f = reco::ensure_hybrid(*g, lambda, S(stream));
    reco::Workspace* w = reco::checkout_workspace(*g, S(stream));
    try {
      reco::HybridScratch& s = reco::hybrid_scratch(*g, *w, S(stream));
      reco::hybrid_apply(*g, f, s, r, nullptr, nullptr, z, S(stream));
      HIP_CHECK(hipStreamSynchronize(S(stream)));
    } catch (...) {
      w->tainted = true;
      reco::return_workspace(*g, w);
      throw;
    }
    reco::return_workspace(*g, w);
    return RECO_OK;
  })
}

reco_status reco_solve_cgls(reco_geometry gh, const void* b, void* x, const reco_solve_opts* opts,
                            reco_solve_info* info, void* stream) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(b, "b");
    need(x, "x");
    need(opts, "opts");
    return reco::solve_cgls(*g, b, x, *opts, info, S(stream));
  })
}

reco_status reco_solve_cgls_noalloc(reco_geometry gh, const void* b, void* x,
                                    const reco_solve_opts* opts, reco_solve_info* info,
                                    void* stream) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(b, "b");
    need(x, "x");
    need(opts, "opts");
    return reco::solve_cgls_noalloc(*g, b, x, *opts, info, S(stream));
  })
}

reco_status reco_solve_gmres(reco_geometry gh, const void* b, void* x, const reco_solve_opts* opts,
                             reco_solve_info* info, void* stream) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(b, "b");
    need(x, "x");
    need(opts, "opts");
    return reco::solve_gmres(*g, b, x, *opts, info, S(stream));
  })
}

reco_status reco_solve_bicgstab(reco_geometry gh, const void* b, void* x,
                                const reco_solve_opts* opts, reco_solve_info* info, void* stream) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(b, "b");
    need(x, "x");
    need(opts, "opts");
    return reco::solve_bicgstab(*g, b, x, *opts, info, S(stream));
  })
}

reco_status reco_solve_sirt(reco_geometry gh, const void* b, void* x, const reco_solve_opts* opts,
                            reco_solve_info* info, void* stream) {
  RECO_GUARD({
    Geometry* g = G(gh);
    need(b, "b");
    need(x, "x");
    need(opts, "opts");
    return reco::solve_sirt(*g, b, x, *opts, info, S(stream));
  })
}

reco_status reco_solve_batch(int32_t count, const reco_geometry* geoms, const void* const* b,
                             void* const* x, const reco_solve_opts* opts, reco_solve_info* info,
                             void* stream) {
  RECO_GUARD({
    if (count < 0) reco::fail(RECO_EINVAL, "count must be >= 0");
    if (count == 0) return RECO_OK;
    need(geoms, "geoms");
    need(b, "b");
    need(x, "x");
    need(opts, "opts");
    return reco::solve_batch(count, geoms, b, x, opts, info, S(stream));
  })
}

double reco_clock(void) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // extern "C"
