// The C ABI of include/bkwd.h: argument checks, lattice set-up, dispatch.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/bkwd.h"
#include "bkwd_internal.h"
#include "blas.h"
#include "solver.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

bool valid_dims(const int dims[4], std::string* why) {
  if (dims == nullptr) {
    *why = "dims is NULL";
    return false;
  }
  long long v = 1;
  for (int k = 0; k < 4; ++k) {
    if (dims[k] < 2) {
      *why = "every lattice extent must be >= 2";
      return false;
    }
    v *= dims[k];
  }
  // site indices are 32-bit; 12 * V * 64 elements must fit the int64 index math
  if (v > (1LL << 30)) {
    *why = "lattice volume too large";
    return false;
  }
  return true;
}

Geom make_geom(const int dims[4]) {
  Geom g;
  g.lx = dims[0];
  g.ly = dims[1];
  g.lz = dims[2];
  g.lt = dims[3];
  g.vol = dims[0] * dims[1] * dims[2] * dims[3];
  return g;
}

// kernel attributes are process-wide: set once, whichever thread creates the
// first lattice
std::once_flag g_attrs_once;

int finish_setup(LatticeImpl* lat, hipStream_t s) {
  hipError_t e = launch_clover_build(*lat, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(BKWD_EDEVICE, std::string("clover build: ") + hipGetErrorString(e));
  return BKWD_OK;
}

}  // namespace

LatticeLayout lattice_layout(const Geom& g, unsigned flags) {
  LatticeLayout l{};
  const size_t V = (size_t)g.vol;
  size_t off = 0;
  l.off_links64 = off; off = align_up(off + V * 36 * sizeof(cpx<double>));
  l.off_links32 = off; off = align_up(off + V * 36 * sizeof(cpx<float>));
  l.off_links32c = off;
  if (flags & BKWD_COMPRESS12) off = align_up(off + V * 24 * sizeof(cpx<float>));
  l.off_clover64 = off; off = align_up(off + V * 72 * sizeof(double));
  l.off_clover32 = off; off = align_up(off + V * 72 * sizeof(float));
  l.off_canon = off; off = align_up(off + V * 36 * sizeof(cpx<double>));
  l.total = off;
  return l;
}

struct bkwd_lattice {
  LatticeImpl impl;
};

extern "C" {

const char* bkwd_last_error(void) { return g_err.c_str(); }

const char* bkwd_version(void) { return "bkwd 0.1 (gfx950)"; }

size_t bkwd_lattice_bytes(const int dims[4], unsigned flags) {
  std::string why;
  if (!valid_dims(dims, &why)) return 0;
  return lattice_layout(make_geom(dims), flags).total;
}

int bkwd_lattice_create(const int dims[4], const double* links_host, double kappa, double csw, unsigned flags,
                        void* dev_buf, size_t dev_buf_bytes, void* stream, bkwd_lattice** out) {
  g_err.clear();
  if (out == nullptr) return fail(BKWD_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!valid_dims(dims, &why)) return fail(BKWD_EINVAL, why);
  if (links_host == nullptr) return fail(BKWD_EINVAL, "links_host is NULL");
  if (dev_buf == nullptr) return fail(BKWD_EINVAL, "dev_buf is NULL");
  if ((reinterpret_cast<uintptr_t>(dev_buf) & 255u) != 0) return fail(BKWD_EINVAL, "dev_buf must be 256-byte aligned");
  if (!std::isfinite(kappa) || !std::isfinite(csw)) return fail(BKWD_EINVAL, "kappa and csw must be finite");
  if ((flags & ~BKWD_COMPRESS12) != 0) return fail(BKWD_EINVAL, "unknown flag");
  const Geom g = make_geom(dims);
  const LatticeLayout ly = lattice_layout(g, flags);
  if (dev_buf_bytes < ly.total) return fail(BKWD_ENOMEM, "dev_buf too small: need " + std::to_string(ly.total));

  hipStream_t s = static_cast<hipStream_t>(stream);
  bkwd_lattice* h = new (std::nothrow) bkwd_lattice;
  if (h == nullptr) return fail(BKWD_ENOMEM, "host allocation failed");
  LatticeImpl& L = h->impl;
  std::memset(&L, 0, sizeof(L));
  L.g = g;
  L.kappa = kappa;
  L.csw = csw;
  L.flags = flags;
  unsigned char* base = static_cast<unsigned char*>(dev_buf);
  L.links64 = reinterpret_cast<cpx<double>*>(base + ly.off_links64);
  L.links32 = reinterpret_cast<cpx<float>*>(base + ly.off_links32);
  L.links32c = (flags & BKWD_COMPRESS12) ? reinterpret_cast<cpx<float>*>(base + ly.off_links32c) : nullptr;
  L.clover64 = reinterpret_cast<double*>(base + ly.off_clover64);
  L.clover32 = reinterpret_cast<float*>(base + ly.off_clover32);
  L.canon = reinterpret_cast<cpx<double>*>(base + ly.off_canon);
  hipError_t e = hipHostMalloc(&L.host_scratch, 65536, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete h;
    return fail(BKWD_EDEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  std::call_once(g_attrs_once, [] {
    // only L > 44 needs more than 64 KiB of LDS; a failure here surfaces as a
    // launch error of those kernels
    (void)blas_set_attributes();
    (void)hipGetLastError();
  });
  const size_t link_bytes = (size_t)g.vol * 36 * sizeof(cpx<double>);
  e = hipMemcpyAsync(L.canon, links_host, link_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_pack_links(L, s);
  if (e != hipSuccess) {
    (void)hipHostFree(L.host_scratch);
    delete h;
    return fail(BKWD_EDEVICE, std::string("link upload: ") + hipGetErrorString(e));
  }
  const int rc = finish_setup(&L, s);
  if (rc != BKWD_OK) {
    (void)hipHostFree(L.host_scratch);
    delete h;
    return rc;
  }
  *out = h;
  return BKWD_OK;
}

int bkwd_lattice_set_params(bkwd_lattice* lat, double kappa, double csw, void* stream) {
  g_err.clear();
  if (lat == nullptr) return fail(BKWD_EINVAL, "lattice is NULL");
  if (!std::isfinite(kappa) || !std::isfinite(csw)) return fail(BKWD_EINVAL, "kappa and csw must be finite");
  lat->impl.kappa = kappa;
  lat->impl.csw = csw;
  return finish_setup(&lat->impl, static_cast<hipStream_t>(stream));
}

int bkwd_lattice_destroy(bkwd_lattice* lat) {
  g_err.clear();
  if (lat == nullptr) return BKWD_OK;
  if (lat->impl.host_scratch) (void)hipHostFree(lat->impl.host_scratch);
  delete lat;
  return BKWD_OK;
}

int bkwd_lattice_info(const bkwd_lattice* lat, int dims_out[4], long long* volume, double* kappa, double* csw) {
  g_err.clear();
  if (lat == nullptr) return fail(BKWD_EINVAL, "lattice is NULL");
  const Geom& g = lat->impl.g;
  if (dims_out) {
    dims_out[0] = g.lx;
    dims_out[1] = g.ly;
    dims_out[2] = g.lz;
    dims_out[3] = g.lt;
  }
  if (volume) *volume = g.vol;
  if (kappa) *kappa = lat->impl.kappa;
  if (csw) *csw = lat->impl.csw;
  return BKWD_OK;
}

int bkwd_apply(bkwd_lattice* lat, int dagger, int L, int prec, const void* X, void* Y, void* stream) {
  return bkwd_apply_layout(lat, dagger, L, prec, BKWD_SITE_MAJOR, X, Y, stream);
}

int bkwd_apply_layout(bkwd_lattice* lat, int dagger, int L, int prec, int layout, const void* X, void* Y,
                      void* stream) {
  g_err.clear();
  if (lat == nullptr) return fail(BKWD_EINVAL, "lattice is NULL");
  if (layout != BKWD_SITE_MAJOR && layout != BKWD_COMPONENT_MAJOR)
    return fail(BKWD_EINVAL, "layout must be BKWD_SITE_MAJOR or BKWD_COMPONENT_MAJOR");
  const bool cm = layout == BKWD_COMPONENT_MAJOR;
  if (L < 1 || L > BKWD_MAX_RHS) return fail(BKWD_EINVAL, "L must be in 1..64");
  if (dagger != 0 && dagger != 1) return fail(BKWD_EINVAL, "dagger must be 0 or 1");
  if (X == nullptr || Y == nullptr) return fail(BKWD_EINVAL, "X and Y must be non-NULL");
  if (X == Y) return fail(BKWD_EINVAL, "X and Y must not overlap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (prec == BKWD_FP64) {
    e = launch_dslash<double>(lat->impl, dagger, L, static_cast<const cpx<double>*>(X), static_cast<cpx<double>*>(Y),
                              nullptr, nullptr, nullptr, cm, s);
  } else if (prec == BKWD_FP32) {
    e = launch_dslash<float>(lat->impl, dagger, L, static_cast<const cpx<float>*>(X), static_cast<cpx<float>*>(Y),
                             nullptr, nullptr, nullptr, cm, s);
  } else {
    return fail(BKWD_EINVAL, "prec must be BKWD_FP64 or BKWD_FP32");
  }
  if (e != hipSuccess) return fail(BKWD_EDEVICE, std::string("apply: ") + hipGetErrorString(e));
  return BKWD_OK;
}

void bkwd_solve_opts_default(bkwd_solve_opts* o) {
  if (o == nullptr) return;
  std::memset(o, 0, sizeof(*o));
  o->method = BKWD_BLOCK_BICGGR;
  o->prec = BKWD_MIXED;
  o->max_iter = 10000;
  o->max_restarts = 20;
  o->use_x0 = 0;
  o->shadow = 0;
  o->check_every = 8;
  o->stagnation = 200;
  o->tol = 1e-12;
  o->inner_tol = 0.0;
  o->seed = 12345;
  o->history = nullptr;
  o->history_len = 0;
  o->profile = 0;
  o->shadow_block = nullptr;
  o->qr_frame = -1;
  o->max_block = 0;
  o->evenodd = 0;
  o->deflate = 0;
  o->dagger = 0;
  o->reliable = 0.0;
}

// qr_frame -1 (by precision): a QR frame for FP32 cycles, which need it to
// converge, the fused one (16 block passes instead of 20; the explicit frame
// with reliable updates, which need it); the listing for FP64, where the
// frame's extra block passes buy no iterations.
static bkwd_solve_opts resolved(const bkwd_solve_opts& o) {
  bkwd_solve_opts r = o;
  if (r.qr_frame == -1) r.qr_frame = r.prec == BKWD_FP64 ? 0 : (r.reliable > 0.0 ? 1 : 2);
  return r;
}

size_t bkwd_solve_workspace_bytes(const bkwd_lattice* lat, int L, const bkwd_solve_opts* o) {
  if (lat == nullptr || o == nullptr || L < 1 || L > BKWD_MAX_RHS) return 0;
  const bkwd_solve_opts ro = resolved(*o);
  WsLayout w;
  std::string why;
  if (!ws_layout(lat->impl, L, ro, &w, &why)) return 0;
  WsLayout r;
  if (!ws_layout(lat->impl, L, ro, &r, &why, true)) return 0;
  return w.total > r.total ? w.total : r.total;
}

int bkwd_block_solve(bkwd_lattice* lat, int L, const void* B, void* X, const bkwd_solve_opts* o, void* workspace,
                     size_t workspace_bytes, bkwd_solve_info* info, void* stream) {
  g_err.clear();
  if (lat == nullptr) return fail(BKWD_EINVAL, "lattice is NULL");
  if (o == nullptr || info == nullptr) return fail(BKWD_EINVAL, "opts and info must be non-NULL");
  std::memset(info, 0, sizeof(*info));
  if (L < 1 || L > BKWD_MAX_RHS) return fail(BKWD_EINVAL, "L must be in 1..64");
  if (B == nullptr || X == nullptr || workspace == nullptr) return fail(BKWD_EINVAL, "B, X and workspace must be non-NULL");
  if (B == X) return fail(BKWD_EINVAL, "B and X must not overlap");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(BKWD_EINVAL, "workspace must be 256-byte aligned");
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(BKWD_EINVAL, "tol must be positive");
  if (o->prec == BKWD_MIXED && (!(o->inner_tol >= 0.0) || !(o->inner_tol < 1.0)))
    return fail(BKWD_EINVAL, "inner_tol must be 0 (by L) or in (0, 1)");
  if (o->max_iter < 0 || o->max_restarts < 0 || o->stagnation < 0) return fail(BKWD_EINVAL, "negative cap");
  if (o->method == BKWD_BLOCK_BICGSTAB || o->method == BKWD_BLOCK_BICGGR || o->method == BKWD_BICGSTAB) {
  } else {
    return fail(BKWD_EINVAL, "unknown method");
  }
  if (o->prec != BKWD_FP64 && o->prec != BKWD_MIXED) return fail(BKWD_EINVAL, "prec must be BKWD_FP64 or BKWD_MIXED");
  if (o->shadow < 0 || o->shadow > 2) return fail(BKWD_EINVAL, "shadow must be 0, 1 or 2");
  if (o->shadow == 2 && o->shadow_block == nullptr) return fail(BKWD_EINVAL, "shadow = 2 needs shadow_block");
  if (o->qr_frame < -1 || o->qr_frame > 2) return fail(BKWD_EINVAL, "qr_frame must be -1, 0, 1 or 2");
  if (o->dagger != 0 && o->dagger != 1) return fail(BKWD_EINVAL, "dagger must be 0 or 1");
  if (!(o->reliable >= 0.0 && o->reliable < 1.0)) return fail(BKWD_EINVAL, "reliable must be in [0, 1)");
  if (o->reliable > 0.0 &&
      !(o->prec == BKWD_MIXED && o->method == BKWD_BLOCK_BICGGR && (o->qr_frame == -1 || o->qr_frame == 1)))
    return fail(BKWD_EINVAL, "reliable updates need MIXED block BiCGGR with qr_frame 1 (or -1)");
  if (o->max_block < 0 || o->max_block > BKWD_MAX_RHS) return fail(BKWD_EINVAL, "max_block must be in 0..64");
  if (o->evenodd != 0 && o->evenodd != 1) return fail(BKWD_EINVAL, "evenodd must be 0 or 1");
  if (o->deflate != 0 && o->deflate != 1) return fail(BKWD_EINVAL, "deflate must be 0 or 1");
  if (o->deflate && o->reliable > 0.0) return fail(BKWD_EINVAL, "deflate does not combine with reliable updates");
  if (o->evenodd) {
    const Geom& g = lat->impl.g;
    if (g.lx % 2 || g.ly % 2 || g.lz % 2 || g.lt % 2)
      return fail(BKWD_EINVAL, "evenodd needs every lattice extent even");
    if (o->reliable > 0.0) return fail(BKWD_EINVAL, "evenodd does not combine with reliable updates");
    if (o->shadow == 2) return fail(BKWD_EINVAL, "evenodd does not take a caller shadow block");
  }
  std::string err;
  const int rc = solve_driver(lat->impl, L, static_cast<const cpx<double>*>(B), static_cast<cpx<double>*>(X),
                              resolved(*o), workspace, workspace_bytes, info, static_cast<hipStream_t>(stream), &err);
  if (rc != BKWD_OK) g_err = err;
  return rc;
}

int bkwd_meson_correlators(bkwd_lattice* lat, const void* X, double* pion, double* rho, void* stream) {
  g_err.clear();
  if (lat == nullptr) return fail(BKWD_EINVAL, "lattice is NULL");
  if (X == nullptr || pion == nullptr || rho == nullptr) return fail(BKWD_EINVAL, "X, pion and rho must be non-NULL");
  const hipError_t e = launch_mesons(lat->impl, static_cast<const cpx<double>*>(X), pion, rho,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(BKWD_EDEVICE, std::string("meson contraction: ") + hipGetErrorString(e));
  return BKWD_OK;
}

int bkwd_true_residual(bkwd_lattice* lat, int L, const void* B, const void* X, double* per_col_host, void* workspace,
                       size_t workspace_bytes, void* stream) {
  g_err.clear();
  if (lat == nullptr) return fail(BKWD_EINVAL, "lattice is NULL");
  if (L < 1 || L > BKWD_MAX_RHS) return fail(BKWD_EINVAL, "L must be in 1..64");
  if (B == nullptr || X == nullptr || per_col_host == nullptr || workspace == nullptr)
    return fail(BKWD_EINVAL, "B, X, per_col_host and workspace must be non-NULL");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(BKWD_EINVAL, "workspace must be 256-byte aligned");
  std::string err;
  const int rc = true_residual_driver(lat->impl, L, static_cast<const cpx<double>*>(B),
                                      static_cast<const cpx<double>*>(X), per_col_host, workspace, workspace_bytes,
                                      static_cast<hipStream_t>(stream), &err);
  if (rc != BKWD_OK) g_err = err;
  return rc;
}

int bkwd_true_residual_noalloc(bkwd_lattice* lat, int L, const void* B, const void* X, double* per_col_host,
                               void* stream) {
  g_err.clear();
  if (lat == nullptr) return fail(BKWD_EINVAL, "lattice is NULL");
  if (L < 1 || L > BKWD_MAX_RHS) return fail(BKWD_EINVAL, "L must be in 1..64");
  if (B == nullptr || X == nullptr || per_col_host == nullptr)
    return fail(BKWD_EINVAL, "B, X and per_col_host must be non-NULL");
  std::string err;
  const int rc = true_residual_noalloc(lat->impl, L, static_cast<const cpx<double>*>(B),
                                       static_cast<const cpx<double>*>(X), per_col_host,
                                       static_cast<hipStream_t>(stream), &err);
  if (rc != BKWD_OK) g_err = err;
  return rc;
}

namespace {

struct GradLayout {
  size_t off_clover, off_w, off_part, off_stage, stage_half, off_out, total;
  int grid;
};

GradLayout grad_layout(const LatticeImpl& lat, int L) {
  GradLayout g{};
  const size_t V = (size_t)lat.g.vol;
  g.grid = 1024;  // upper bound of the grid-stride operator launch
  size_t off = 0;
  g.off_clover = off; off = align_up(off + 72 * V * sizeof(double));
  g.off_w = off; off = align_up(off + 6 * 9 * V * sizeof(cpx<double>));
  g.off_part = off; off = align_up(off + (size_t)g.grid * 4 * sizeof(double));
  g.stage_half = ((size_t)g.grid + 255) / 256 * 4;
  g.off_stage = off; off = align_up(off + 2 * g.stage_half * sizeof(double));
  g.off_out = off; off = align_up(off + 4 * sizeof(double));
  g.total = off;
  (void)L;
  return g;
}

}  // namespace

size_t bkwd_gradients_workspace_bytes(const bkwd_lattice* lat, int L) {
  if (lat == nullptr || L < 1 || L > BKWD_MAX_RHS) return 0;
  return grad_layout(lat->impl, L).total;
}

int bkwd_gradients(bkwd_lattice* lat, int L, const void* X, const void* Lambda, double* grad_kappa,
                   double* grad_csw, void* grad_links, void* workspace, size_t workspace_bytes, void* stream) {
  g_err.clear();
  if (lat == nullptr) return fail(BKWD_EINVAL, "lattice is NULL");
  if (L < 1 || L > BKWD_MAX_RHS) return fail(BKWD_EINVAL, "L must be in 1..64");
  if (X == nullptr || Lambda == nullptr || workspace == nullptr)
    return fail(BKWD_EINVAL, "X, Lambda and workspace must be non-NULL");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(BKWD_EINVAL, "workspace must be 256-byte aligned");
  LatticeImpl& impl = lat->impl;
  const GradLayout gl = grad_layout(impl, L);
  if (workspace_bytes < gl.total)
    return fail(BKWD_ENOMEM, "workspace too small: need " + std::to_string(gl.total) + " bytes");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  const cpx<double>* x = static_cast<const cpx<double>*>(X);
  const cpx<double>* lam = static_cast<const cpx<double>*>(Lambda);
  double* unit = reinterpret_cast<double*>(ws + gl.off_clover);
  cpx<double>* w = reinterpret_cast<cpx<double>*>(ws + gl.off_w);
  hipError_t e = hipSuccess;
  if (grad_kappa != nullptr || grad_csw != nullptr) {
    // blocks of 1 - C (kappa csw = 1), then Re <Lam, (csw C + H) X> and Re <Lam, C X>
    e = launch_clover_build_into(impl, unit, 1.0, s);
    int nblk = 0;
    double* part = reinterpret_cast<double*>(ws + gl.off_part);
    double* out = reinterpret_cast<double*>(ws + gl.off_out);
    if (e == hipSuccess) e = launch_grad_scalars(impl, L, x, lam, unit, impl.csw, part, &nblk, s);
    if (e == hipSuccess)
      e = launch_reduce(part, nblk, 4, reinterpret_cast<double*>(ws + gl.off_stage), gl.stage_half, out, s);
    double* host = reinterpret_cast<double*>(impl.host_scratch);
    if (e == hipSuccess) e = hipMemcpyAsync(host, out, 4 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
      if (grad_kappa) *grad_kappa = host[0];
      if (grad_csw) *grad_csw = impl.kappa * host[1];
    }
  }
  if (e == hipSuccess && grad_links != nullptr) {
    const bool clover = impl.kappa * impl.csw != 0.0;
    if (clover) e = launch_clover_w(impl, L, x, lam, impl.kappa * impl.csw, w, s);
    if (e == hipSuccess)
      e = launch_link_force(impl, L, x, lam, clover ? w : nullptr, static_cast<cpx<double>*>(grad_links), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) return fail(BKWD_EDEVICE, std::string("gradients: ") + hipGetErrorString(e));
  return BKWD_OK;
}

}  // extern "C"
