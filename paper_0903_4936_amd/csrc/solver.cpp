// Host drivers: one Krylov cycle of BiCGSTAB / block BiCGSTAB / block BiCGGR
// (Sec. 3) on device-resident blocks, and the outer loop that restarts it on
// the FP64 residual until the true residual of Sec. 4.3 reaches the target
// (FP64 restarts, or FP32 inner cycles inside FP64 defect correction).
//
// Every coefficient is computed on the device; the host only queues kernels
// and reads a small status record every `check_every` iterations.
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "blas.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }


#define HIP_TRY(...)                                                          \
  do {                                                                        \
    hipError_t e_ = (__VA_ARGS__);                                            \
    if (e_ != hipSuccess) {                                                   \
      if (err) *err = std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_); \
      return BKWD_EDEVICE;                                                    \
    }                                                                         \
  } while (0)

// the fused frame's Gram pass rides in the operator launch (BKWD_NO_GRAM_DSLASH:
// a separate Gram kernel)
#ifdef BKWD_NO_GRAM_DSLASH
constexpr bool kGramDslash = false;
#else
constexpr bool kGramDslash = true;
#endif

struct EventRec {
  hipEvent_t a, b;
  int tag;   // iteration index of the launch (-1: set-up)
  int fp32;
  int kind;  // 0: operator; 1, 2, 3: the U, X/R and P/V update kernels of Block BiCGGR
  int post;  // queued after the iteration's stop test
};

// Everything a solve needs on the host side.
struct Ctx {
  LatticeImpl* lat;
  hipStream_t s;
  const WsLayout* ly;
  unsigned char* ws;
  bool profile;
  int dagger = 0;  // 1: every operator application (and residual) uses D^dagger
  std::vector<EventRec> events;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  int matvecs = 0;
  double dslash_ms = 0.0, dslash_ms32 = 0.0;
  int dslash_calls = 0, dslash_calls32 = 0;
  double update_ms[3] = {0.0, 0.0, 0.0};
  int update_calls[3] = {0, 0, 0};
  int cur_tag = -1;  // iteration being queued (tags the update-kernel events)
  int cur_post = 0;  // the launches being queued follow the iteration's stop test
  bool eo = false;   // even-odd: cycles run on compact even blocks with the Schur operator
  bool deflate = false;  // leave out converged and dependent columns between cycles
  bool gram_operator = false;  // a cycle formed the fused frame's Grams in the operator launch
  std::string* err;

  // sites of the cycles' blocks
  int vol_op() const { return eo ? lat->g.vol / 2 : lat->g.vol; }

  template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
  double* partials() const { return at<double>(ly->off_partials); }
  double* stage() const { return at<double>(ly->off_stage); }
  Control* ctl() const { return at<Control>(ly->off_ctl); }
  Control* host_ctl() const { return reinterpret_cast<Control*>(lat->host_scratch); }
  double* host_norms() const { return reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(lat->host_scratch) + 256); }

  hipEvent_t take_event() {
    if (pool_used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[pool_used++];
  }
  ~Ctx() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// Launch the operator (optionally recording events around it).  With
// gram_rt (8-column FP32 blocks, whole lattice or even-odd Schur) the launch also leaves
// the partial Grams in^H out, out^H out, gram_rt^H out in the partial records
// (nblk of them); it is timed as the fused frame's Gram pass.
template <typename T>
int apply_op(Ctx& c, int L, const cpx<T>* in, cpx<T>* out, double* epi, int* nblk, const Control* ctl, int tag,
             const cpx<T>* gram_rt = nullptr) {
  std::string* err = c.err;
  EventRec rec{};
  if (c.profile) {
    rec.a = c.take_event();
    rec.b = c.take_event();
    rec.tag = tag;
    rec.post = c.cur_post;
    rec.fp32 = std::is_same<T, float>::value ? 1 : 0;
    rec.kind = gram_rt ? 3 : 0;
    if (rec.a && rec.b) HIP_TRY(hipEventRecord(rec.a, c.s));
  }
  if (gram_rt) {
    if constexpr (std::is_same<T, float>::value) {
      if (c.eo) {
        const WsLayout& ly = *c.ly;
        HIP_TRY(launch_schur_gram(*c.lat, c.dagger, in, out, c.at<cpx<float>>(ly.off_eotmp), c.lat->clover32,
                                  c.at<float>(ly.off_cinv32), gram_rt, c.partials(), nblk, ctl, c.s));
      } else {
        HIP_TRY(launch_dslash_gram(*c.lat, c.dagger, in, out, gram_rt, c.partials(), nblk, ctl, c.s));
      }
    } else {
      if (err) *err = "internal: the Gram operator launch is FP32 only";
      return BKWD_EDEVICE;
    }
  } else if (c.eo) {
    const WsLayout& ly = *c.ly;
    const void* clov = std::is_same<T, float>::value ? (const void*)c.lat->clover32 : (const void*)c.lat->clover64;
    const void* cinv = std::is_same<T, float>::value ? (const void*)c.at<float>(ly.off_cinv32)
                                                     : (const void*)c.at<double>(ly.off_cinv64);
    HIP_TRY(launch_schur<T>(*c.lat, c.dagger, L, in, out, c.at<cpx<T>>(ly.off_eotmp), clov, cinv, ctl, c.s));
    if (epi) HIP_TRY(launch_trace2<T>(in, out, 12LL * c.vol_op() * L, epi, nblk, c.s));
  } else {
    HIP_TRY(launch_dslash<T>(*c.lat, c.dagger, L, in, out, epi, nblk, ctl, true, c.s));
  }
  if (c.profile && rec.a && rec.b) {
    HIP_TRY(hipEventRecord(rec.b, c.s));
    c.events.push_back(rec);
  }
  c.matvecs += 1;
  return BKWD_OK;
}

int reduce(Ctx& c, long long nrows, int nv, size_t out_off) {
  std::string* err = c.err;
  HIP_TRY(launch_reduce(c.partials(), nrows, nv, c.stage(), c.ly->stage_half, c.at<double>(out_off), c.s));
  return BKWD_OK;
}

struct CycleResult {
  int state = ST_RUNNING;
  int iterations = 0;
  double resid = 0.0;
  int matvecs = 0;
};

// Blocks of one cycle: E (the cycle's solution), R (holds the cycle's
// right-hand side on entry), P, V, W, U, Y, R~0.  Block BiCGSTAB uses W for
// T and Y for Z.
template <typename T>
struct Blocks {
  cpx<T>* b[8];
  cpx<T>* E() const { return b[0]; }
  cpx<T>* R() const { return b[1]; }
  cpx<T>* P() const { return b[2]; }
  cpx<T>* V() const { return b[3]; }
  cpx<T>* W() const { return b[4]; }
  cpx<T>* U() const { return b[5]; }
  cpx<T>* Y() const { return b[6]; }
  cpx<T>* Rt() const { return b[7]; }
};

template <typename T>
Blocks<T> cycle_blocks(const Ctx& c) {
  Blocks<T> bl{};
  for (int k = 0; k < 8; ++k) bl.b[k] = nullptr;
  for (int k = 0; k < c.ly->nblocks; ++k) bl.b[k] = c.at<cpx<T>>(c.ly->off_blocks + (size_t)k * c.ly->block_bytes);
  if (c.ly->nblocks == 7) {  // BiCGSTAB: no U; R~0 is the 7th block
    bl.b[7] = bl.b[6];
    bl.b[6] = bl.b[5];
    bl.b[5] = nullptr;
  }
  return bl;
}

CoefArgs coef_args(const Ctx& c, int L, bool scalar) {
  CoefArgs a{};
  a.L = L;
  a.scalar = scalar ? 1 : 0;
  a.red_a = c.at<double>(c.ly->off_red_a);
  a.red_b = c.at<double>(c.ly->off_red_b);
  a.red_c = c.at<double>(c.ly->off_red_c);
  cpx<double>* coef = c.at<cpx<double>>(c.ly->off_coef);
  const int L2 = L * L;
  a.GR = coef;
  a.GV = coef + L2;
  a.alpha = coef + 2 * L2;
  a.beta = coef + 3 * L2;
  a.zeta = coef + 4 * L2;
  a.S = coef + 4 * L2 + 1;
  a.Sinv = coef + 5 * L2 + 1;
  a.xi = coef + 6 * L2 + 1;
  a.tmp = coef + 7 * L2 + 1;
  a.mu1 = coef + 8 * L2 + 1;
  a.mu2 = coef + 9 * L2 + 1;
  a.mx1 = coef + 10 * L2 + 1;
  a.eta = coef + 11 * L2 + 1;
  a.weight = c.at<double>(c.ly->off_weight);
  a.ctl = c.ctl();
  a.hist = c.ly->hist_cap ? c.at<double>(c.ly->off_hist) : nullptr;
  return a;
}

template <typename T>
BlasArgs<T> blas_args(const Ctx& c, int L, const Blocks<T>& bl, const CoefArgs& ca) {
  BlasArgs<T> a{};
  a.L = L;
  a.nrows = 12LL * c.vol_op();
  a.x = bl.E(); a.r = bl.R(); a.p = bl.P(); a.v = bl.V(); a.w = bl.W(); a.u = bl.U(); a.y = bl.Y();
  a.rt = bl.Rt();
  a.zeta = ca.zeta;
  a.partials = c.partials();
  a.ctl = c.ctl();
  return a;
}

template <typename T>
int blas(Ctx& c, int op, BlasArgs<T> a, const cpx<double>* m1, int nv, int want_norms, size_t red_off,
         const cpx<double>* m2 = nullptr) {
  std::string* err = c.err;
  a.m1 = m1;
  a.m2 = m2;
  a.nv = nv;
  a.want_norms = want_norms;
  // the fused frame's Gram pass counts as the third update kernel inside the
  // iteration (cur_tag >= 0), not at the start of a cycle
  const int kind = (op == OP_BICGGR_U || op == OP_FU || op == OP_FUX) ? 1
                   : (op == OP_GGRQ_XR || op == OP_FXR || op == OP_FXRT) ? 2
                   : (op == OP_GGRQ_PV || (op == OP_FGRAM && c.cur_tag >= 0)) ? 3 : 0;
  EventRec rec{};
  if (c.profile && kind != 0) {
    rec.a = c.take_event();
    rec.b = c.take_event();
    rec.tag = c.cur_tag;
    rec.post = c.cur_post;
    rec.kind = kind;
    if (rec.a && rec.b) HIP_TRY(hipEventRecord(rec.a, c.s));
  }
  const int grid = blas_launch<T>(op, a, c.s);
  if (c.profile && kind != 0 && rec.a && rec.b) {
    HIP_TRY(hipEventRecord(rec.b, c.s));
    c.events.push_back(rec);
  }
  if (grid < 0) {
    if (err) *err = "internal: unknown block kernel";
    return BKWD_EDEVICE;
  }
  HIP_TRY(hipGetLastError());
  if (nv > 0) return reduce(c, grid, nv, red_off);
  return BKWD_OK;
}

int coef(Ctx& c, int op, const CoefArgs& a) {
  std::string* err = c.err;
  HIP_TRY(launch_coef(op, a, c.s));
  return BKWD_OK;
}

#define TRY(...)                    \
  do {                              \
    int rc_ = (__VA_ARGS__);        \
    if (rc_ != BKWD_OK) return rc_; \
  } while (0)

// One Krylov cycle on blocks of precision T.  R holds the right-hand side.
// Shadow residual of a cycle: mode 0 copies R_0, 1 draws a seeded complex
// Gaussian, 2 converts the caller's FP64 block `shadow64`.
struct Shadow {
  int mode;
  unsigned long long seed;
  const cpx<double>* block;
};

int residual(Ctx& c, int L, const cpx<double>* B, const cpx<double>* X, cpx<double>* R, double* r2, double* b2);
int add_correction(Ctx& c, cpx<double>* X, long long n_elem, int L, bool qr, double sign);

// Reliable updates inside an FP32 QR-frame cycle: whenever the recursive
// residual has dropped by a factor delta since the last anchor, the
// correction so far is added to the FP64 solution, the true residual
// B - D X is recomputed in FP64 and becomes the new frame R = Q' xi', and
// the search blocks P, V are carried over into that frame.  The Krylov
// recurrences continue (no restart); only the drift between the recursive
// and the true residual is removed.
struct Reliable {
  double delta = 0.0;              // 0: off
  const cpx<double>* B = nullptr;  // FP64 right-hand sides and solution (ABI layout)
  cpx<double>* X = nullptr;
  cpx<double>* res64 = nullptr;    // FP64 residual scratch
  double anchor0 = 1.0;            // weighted residual at the cycle start
  double tol = 0.0;                // true-residual target (max relative)
  int updates = 0;
  double true_resid = INFINITY;    // max relative true residual at the last update
};

template <typename T>
int run_cycle(Ctx& c, int L, int method, bool scalar, const bkwd_solve_opts& o, const Shadow& sh,
              double cycle_tol, bool frob, CycleResult* res, Reliable* ru = nullptr) {
  std::string* err = c.err;
  c.cur_tag = -1;  // set per iteration below
  c.cur_post = 0;
  const Blocks<T> bl = cycle_blocks<T>(c);
  const CoefArgs ca = coef_args(c, L, scalar);
  BlasArgs<T> ba = blas_args<T>(c, L, bl, ca);
  const long long n_elem = 12LL * c.vol_op() * L;
  const size_t bytes = (size_t)n_elem * sizeof(cpx<T>);
  const int L2 = L * L;
  const int matvecs0 = c.matvecs;

  // control record
  Control* hc = c.host_ctl();
  std::memset(hc, 0, sizeof(Control));
  hc->state = ST_RUNNING;
  hc->best = INFINITY;
  hc->tol = cycle_tol;
  hc->max_iter = std::max(0, o.max_iter);
  hc->stagnation = std::max(0, o.stagnation);
  hc->hist_cap = (int)c.ly->hist_cap;
  hc->frob = frob ? 1 : 0;
  const bool ru_on = ru != nullptr && ru->delta > 0.0 && std::is_same<T, float>::value &&
                     method == BKWD_BLOCK_BICGGR && o.qr_frame == 1 && !frob;
  hc->ru_delta = ru_on ? ru->delta : 0.0;
  hc->ru_anchor = ru_on ? ru->anchor0 : 0.0;
  HIP_TRY(hipMemcpyAsync(c.ctl(), hc, sizeof(Control), hipMemcpyHostToDevice, c.s));

  HIP_TRY(hipMemsetAsync(bl.E(), 0, bytes, c.s));
  if (sh.mode == 1) HIP_TRY(launch_gaussian<T>(bl.Rt(), n_elem, sh.seed, c.s));
  else if (sh.mode == 2) HIP_TRY(launch_convert<T>(sh.block, bl.Rt(), n_elem, L, c.lat->g.vol, c.s));
  else HIP_TRY(hipMemcpyAsync(bl.Rt(), bl.R(), bytes, hipMemcpyDeviceToDevice, c.s));

  const bool ggr = (method == BKWD_BLOCK_BICGGR);
  const bool qrf = ggr && o.qr_frame != 0;
  // P and V eliminated, Q and W kept unnormalised (small-L register kernels)
  const bool fused = qrf && o.qr_frame == 2 && L <= kSmallL;
  // P_0 = R_0 (the fused frame never reads P)
  if (!fused) HIP_TRY(hipMemcpyAsync(bl.P(), bl.R(), bytes, hipMemcpyDeviceToDevice, c.s));
  const bool fused_x = fused && blas_fused_x(L, sizeof(cpx<T>));
  const bool gram_op = fused_x && kGramDslash &&
                       (c.eo ? schur_gram_supported(*c.lat, L) : dslash_gram_supported(*c.lat, L));
  if (gram_op) c.gram_operator = true;
  const int nv_xr = ggr ? 2 * L2 + L : 4 * L2 + L;
  int nblk = 0;
  if (fused) {
    // T = R_0 in R; [T^H T, R~0^H T]; tau, xi_0, R~0^H Q_0; W' = A T; [T^H W', W'^H W', R~0^H W']
    BlasArgs<T> g = ba;
    g.gl[0] = bl.R();
    g.gl[1] = bl.Rt();
    g.gr = bl.R();
    g.ng = 2;
    TRY(blas<T>(c, OP_FGRAM, g, nullptr, 4 * L2, 0, c.ly->off_red_a));
    TRY(coef(c, COEF_FINIT, ca));
    HIP_TRY(hipMemsetAsync(bl.U(), 0, bytes, c.s));
    HIP_TRY(hipMemsetAsync(bl.Y(), 0, bytes, c.s));
    TRY(apply_op<T>(c, L, bl.R(), bl.W(), nullptr, nullptr, c.ctl(), -1));
    g.gl[0] = bl.R();
    g.gl[1] = bl.W();
    g.gl[2] = bl.Rt();
    g.gr = bl.W();
    g.ng = 3;
    TRY(blas<T>(c, OP_FGRAM, g, nullptr, 6 * L2, 0, c.ly->off_red_b));
  } else if (qrf) {
    // R_0 = Q_0 xi_0 (Cholesky QR), W_0 = A Q_0, P_0 = Q_0, V_0 = W_0
    BlasArgs<T> g = ba;
    g.rt = bl.R();
    g.v = bl.R();
    TRY(blas<T>(c, OP_GRAM, g, nullptr, 2 * L2, 0, c.ly->off_red_a));
    TRY(coef(c, COEF_GGRQ_INIT, ca));
    HIP_TRY(launch_rowmat<T, T, false, 0>(bl.R(), bl.R(), ca.Sinv, 1.0, n_elem / L, L, c.vol_op(), c.s));
    TRY(apply_op<T>(c, L, bl.R(), bl.W(), nullptr, nullptr, c.ctl(), -1));
    HIP_TRY(hipMemcpyAsync(bl.P(), bl.R(), bytes, hipMemcpyDeviceToDevice, c.s));
    HIP_TRY(hipMemcpyAsync(bl.V(), bl.W(), bytes, hipMemcpyDeviceToDevice, c.s));
    // red_b = [R~0^H W, W^H Q, W^H W, R~0^H Q]
    BlasArgs<T> g1 = ba;
    g1.rt = bl.Rt(); g1.v = bl.W(); g1.w = bl.W(); g1.r = bl.R();
    TRY(blas<T>(c, OP_GRAM2, g1, nullptr, 4 * L2, 0, c.ly->off_red_b));
    BlasArgs<T> g2 = ba;
    g2.rt = bl.W(); g2.v = bl.W(); g2.w = bl.Rt(); g2.r = bl.R();
    TRY(blas<T>(c, OP_GRAM2, g2, nullptr, 4 * L2, 0, c.ly->off_red_b + 4 * (size_t)L2 * sizeof(double)));
    TRY(coef(c, COEF_GGRQ_INIT2, ca));
  } else if (ggr) {
    // W_0 = V_0 = A R_0, with Tr(W^H R), Tr(W^H W)
    TRY(apply_op<T>(c, L, bl.R(), bl.W(), c.partials(), &nblk, c.ctl(), -1));
    TRY(reduce(c, nblk, 4, c.ly->off_red_c));
    HIP_TRY(hipMemcpyAsync(bl.V(), bl.W(), bytes, hipMemcpyDeviceToDevice, c.s));
  }
  // R~0^H R_0 and ||r_0||^2, then the iteration-0 stop test
  if (!qrf) {
    BlasArgs<T> g = ba;
    g.v = bl.R();
    TRY(blas<T>(c, OP_GRAM, g, nullptr, 2 * L2 + L, 1, c.ly->off_red_a));
    TRY(coef(c, COEF_INIT, ca));
  }
  if (ggr && !qrf) {
    BlasArgs<T> g = ba;
    g.v = bl.V();
    TRY(blas<T>(c, OP_GRAM, g, nullptr, 2 * L2, 0, c.ly->off_red_b));
  }

  auto iteration = [&](int k) -> int {
    c.cur_tag = k;
    c.cur_post = 0;
    if (fused) {
      TRY(coef(c, COEF_FTOP, ca));
      if (fused_x) {
        // X += T (zeta eta) + U_new xi inside the U pass
        BlasArgs<T> bu = ba;
        bu.m3 = ca.mx1;
        bu.m4 = ca.xi;
        TRY(blas<T>(c, OP_FUX, bu, ca.mu1, 0, 0, 0, ca.mu2));
      } else {
        TRY(blas<T>(c, OP_FU, ba, ca.mu1, 0, 0, 0, ca.mu2));
      }
      TRY(apply_op<T>(c, L, bl.U(), bl.Y(), nullptr, nullptr, c.ctl(), k));
      BlasArgs<T> bx = ba;
      bx.m3 = ca.Sinv;
      TRY(blas<T>(c, fused_x ? OP_FXRT : OP_FXR, bx, ca.mx1, 6 * L2, 0, c.ly->off_red_a, ca.xi));
      TRY(coef(c, COEF_GGRQ_END, ca));
      c.cur_post = 1;
      if (gram_op) {
        // W' = A T with the Grams T^H W', W'^H W', R~0^H W' in the same launch
        TRY(apply_op<T>(c, L, bl.R(), bl.W(), nullptr, &nblk, c.ctl(), k, bl.Rt()));
        TRY(reduce(c, nblk, 6 * L2, c.ly->off_red_b));
      } else {
        TRY(apply_op<T>(c, L, bl.R(), bl.W(), nullptr, nullptr, c.ctl(), k));
        BlasArgs<T> g = ba;
        g.gl[0] = bl.R();
        g.gl[1] = bl.W();
        g.gl[2] = bl.Rt();
        g.gr = bl.W();
        g.ng = 3;
        TRY(blas<T>(c, OP_FGRAM, g, nullptr, 6 * L2, 0, c.ly->off_red_b));
      }
    } else if (qrf) {
      TRY(coef(c, COEF_GGRQ_TOP, ca));
      TRY(blas<T>(c, OP_BICGGR_U, ba, ca.alpha, 0, 0, 0));
      TRY(apply_op<T>(c, L, bl.U(), bl.Y(), nullptr, nullptr, c.ctl(), k));
      TRY(blas<T>(c, OP_GGRQ_XR, ba, ca.xi, 4 * L2, 0, c.ly->off_red_a));
      TRY(apply_op<T>(c, L, bl.R(), bl.W(), nullptr, nullptr, c.ctl(), k));
      TRY(coef(c, COEF_GGRQ_END, ca));
      c.cur_post = 1;
      TRY(blas<T>(c, OP_GGRQ_PV, ba, ca.Sinv, 6 * L2, 0, c.ly->off_red_b, ca.beta));
      if (ru_on) TRY(coef(c, COEF_RU_COMMIT, ca));
    } else if (ggr) {
      TRY(coef(c, COEF_BICGGR_TOP, ca));
      TRY(blas<T>(c, OP_BICGGR_U, ba, ca.alpha, 0, 0, 0));
      TRY(apply_op<T>(c, L, bl.U(), bl.Y(), nullptr, nullptr, c.ctl(), k));
      TRY(blas<T>(c, OP_BICGGR_XR, ba, nullptr, nv_xr, 0, c.ly->off_red_a));
      TRY(apply_op<T>(c, L, bl.R(), bl.W(), c.partials(), &nblk, c.ctl(), k));
      TRY(reduce(c, nblk, 4, c.ly->off_red_c));
      TRY(coef(c, COEF_BICGGR_END, ca));
      c.cur_post = 1;
      TRY(blas<T>(c, OP_BICGGR_PV, ba, ca.beta, 2 * L2, 0, c.ly->off_red_b));
    } else {
      TRY(apply_op<T>(c, L, bl.P(), bl.V(), nullptr, nullptr, c.ctl(), k));
      BlasArgs<T> g = ba;
      g.v = bl.V();
      TRY(blas<T>(c, OP_GRAM, g, nullptr, 2 * L2, 0, c.ly->off_red_b));
      TRY(coef(c, COEF_BICGSTAB_ALPHA, ca));
      TRY(blas<T>(c, OP_BICGSTAB_T, ba, ca.alpha, 0, 0, 0));
      TRY(apply_op<T>(c, L, bl.W(), bl.Y(), c.partials(), &nblk, c.ctl(), k));
      TRY(reduce(c, nblk, 4, c.ly->off_red_c));
      TRY(coef(c, COEF_BICGSTAB_ZETA, ca));
      TRY(blas<T>(c, OP_BICGSTAB_XR, ba, ca.alpha, nv_xr, 0, c.ly->off_red_a));
      TRY(coef(c, COEF_BICGSTAB_BETA, ca));
      TRY(blas<T>(c, OP_BICGSTAB_P, ba, ca.beta, 0, 0, 0));
    }
    return BKWD_OK;
  };

  // timing of the launches that ran: those queued after the stop did
  // nothing, and neither did the last counted iteration's launches after its
  // stop test (the test that ended the cycle)
  auto flush_events = [&](int iters_done) {
    if (!c.profile) return;
    for (const EventRec& r : c.events) {
      if (r.tag >= iters_done) continue;
      if (r.post && r.tag == iters_done - 1) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        if (r.kind != 0) {
          c.update_ms[r.kind - 1] += ms;
          c.update_calls[r.kind - 1] += 1;
          continue;
        }
        c.dslash_ms += ms;
        c.dslash_calls += 1;
        if (r.fp32) {
          c.dslash_ms32 += ms;
          c.dslash_calls32 += 1;
        }
      }
    }
    c.events.clear();
    c.pool_used = 0;
  };

  // reliable update (see Reliable); *done = true when the true residual meets the target
  auto reliable_update = [&](bool* done) -> int {
    *done = false;
    TRY(add_correction(c, ru->X, n_elem, L, false, 1.0));
    HIP_TRY(hipMemsetAsync(bl.E(), 0, bytes, c.s));
    std::vector<double> r2(L), b2(L);
    TRY(residual(c, L, ru->B, ru->X, ru->res64, r2.data(), b2.data()));
    double relmax = 0.0;
    for (int i = 0; i < L; ++i) relmax = std::max(relmax, std::sqrt(r2[i] / b2[i]));
    if (!std::isfinite(relmax)) relmax = INFINITY;
    ru->true_resid = relmax;
    ru->updates += 1;
    if (relmax <= ru->tol) {
      *done = true;
      return BKWD_OK;
    }
    // the kernels below skip their work unless the cycle is running
    hc->state = ST_RUNNING;
    hc->ru_pending = 0;
    HIP_TRY(hipMemcpyAsync(c.ctl(), hc, sizeof(Control), hipMemcpyHostToDevice, c.s));
    HIP_TRY(launch_scale_convert<T, double>(ru->res64, bl.R(), c.at<double>(c.ly->off_scale), n_elem, L,
                                            c.lat->g.vol, c.s));
    BlasArgs<T> g = ba;
    g.rt = bl.R();
    g.v = bl.R();
    TRY(blas<T>(c, OP_GRAM, g, nullptr, 2 * L2, 0, c.ly->off_red_a));
    TRY(coef(c, COEF_RU_FRAME, ca));
    HIP_TRY(launch_rowmat<T, T, false, 0>(bl.R(), bl.R(), ca.Sinv, 1.0, n_elem / L, L, c.lat->g.vol, c.s));
    HIP_TRY(launch_rowmat<T, T, false, 0>(bl.P(), bl.P(), ca.tmp, 1.0, n_elem / L, L, c.lat->g.vol, c.s));
    HIP_TRY(launch_rowmat<T, T, false, 0>(bl.V(), bl.V(), ca.tmp, 1.0, n_elem / L, L, c.lat->g.vol, c.s));
    TRY(apply_op<T>(c, L, bl.R(), bl.W(), nullptr, nullptr, c.ctl(), -1));
    BlasArgs<T> g1 = ba;
    g1.rt = bl.Rt(); g1.v = bl.V(); g1.w = bl.W(); g1.r = bl.R();
    TRY(blas<T>(c, OP_GRAM2, g1, nullptr, 4 * L2, 0, c.ly->off_red_b));
    BlasArgs<T> g2 = ba;
    g2.rt = bl.W(); g2.v = bl.W(); g2.w = bl.Rt(); g2.r = bl.R();
    TRY(blas<T>(c, OP_GRAM2, g2, nullptr, 4 * L2, 0, c.ly->off_red_b + 4 * (size_t)L2 * sizeof(double)));
    TRY(coef(c, COEF_GGRQ_INIT2, ca));
    return BKWD_OK;
  };

  const int batch = std::max(1, o.check_every);
  int queued = 0, wasted_iters = 0;
  for (;;) {
    HIP_TRY(hipMemcpyAsync(hc, c.ctl(), sizeof(Control), hipMemcpyDeviceToHost, c.s));
    HIP_TRY(hipStreamSynchronize(c.s));
    if (hc->state == ST_RELIABLE && ru_on) {
      // iterations queued after the one that asked for the update did nothing
      flush_events(hc->iter);
      wasted_iters += queued - hc->iter;
      queued = hc->iter;
      bool done = false;
      TRY(reliable_update(&done));
      if (done) {
        hc->state = ST_CONVERGED;
        break;
      }
      continue;
    }
    if (hc->state != ST_RUNNING) break;
    // queue up to `batch` iterations, never beyond the cap
    const int todo = std::min(batch, std::max(1, hc->max_iter - hc->iter));
    for (int b = 0; b < todo; ++b) TRY(iteration(queued + b));
    queued += todo;
    if (queued > hc->max_iter + 4 * batch + 8) {  // cannot happen: the device stops at max_iter
      if (err) *err = "internal: iteration control lost";
      return BKWD_EDEVICE;
    }
  }
  res->state = hc->state;
  res->iterations = hc->iter;
  res->resid = hc->resid;
  res->matvecs = (c.matvecs - matvecs0);
  // operator applications queued after the cycle ended (or after a reliable
  // update was asked for) did nothing
  const int wasted = 2 * (queued - hc->iter + wasted_iters);
  res->matvecs -= wasted;
  c.matvecs -= wasted;
  flush_events(hc->iter);
  return BKWD_OK;
}

// Column norms of the FP64 residual R = B - D X (and of B): host arrays.
int residual(Ctx& c, int L, const cpx<double>* B, const cpx<double>* X, cpx<double>* R, double* r2, double* b2) {
  std::string* err = c.err;
  int nblk = 0;
  EventRec rec{};
  if (c.profile) {
    rec.a = c.take_event();
    rec.b = c.take_event();
    if (rec.a && rec.b) HIP_TRY(hipEventRecord(rec.a, c.s));
  }
  HIP_TRY(launch_residual64(*c.lat, c.dagger, L, B, X, R, c.partials(), &nblk, c.s));
  if (c.profile && rec.a && rec.b) HIP_TRY(hipEventRecord(rec.b, c.s));
  c.matvecs += 1;
  TRY(reduce(c, nblk, 2 * L, c.ly->off_red_r));
  double* hn = c.host_norms();
  HIP_TRY(hipMemcpyAsync(hn, c.at<double>(c.ly->off_red_r), 2 * L * sizeof(double), hipMemcpyDeviceToHost, c.s));
  HIP_TRY(hipStreamSynchronize(c.s));
  for (int i = 0; i < L; ++i) {
    r2[i] = hn[i];
    b2[i] = hn[L + i];
  }
  if (c.profile && rec.a && rec.b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, rec.a, rec.b) == hipSuccess) {
      c.dslash_ms += ms;
      c.dslash_calls += 1;
    }
    c.pool_used = 0;
  }
  return BKWD_OK;
}

unsigned long long next_seed(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int upload(Ctx& c, size_t off, const double* host, int n) {
  std::string* err = c.err;
  double* tmp = c.host_norms();
  std::memcpy(tmp, host, n * sizeof(double));
  HIP_TRY(hipMemcpyAsync(c.at<double>(off), tmp, n * sizeof(double), hipMemcpyHostToDevice, c.s));
  // the pinned staging area is reused by the next upload
  HIP_TRY(hipStreamSynchronize(c.s));
  return BKWD_OK;
}

// X += unscale_i * E_i (or X += sign * E S after a thin QR of the cycle's
// right-hand side), E the last cycle's solution block
int add_correction(Ctx& c, cpx<double>* X, long long n_elem, int L, bool qr, double sign) {
  std::string* err = c.err;
  const WsLayout& ly = *c.ly;
  if (qr) {
    const CoefArgs ca = coef_args(c, L, false);
    HIP_TRY(launch_rowmat<double, float, true, 2>(cycle_blocks<float>(c).E(), X, ca.S, sign, n_elem / L, L,
                                                   c.lat->g.vol, c.s));
    return BKWD_OK;
  }
  if (ly.prec == BKWD_MIXED)
    HIP_TRY(launch_accumulate<float>(X, cycle_blocks<float>(c).E(), c.at<double>(ly.off_unscale), n_elem, L,
                                     c.lat->g.vol, c.s));
  else
    HIP_TRY(launch_accumulate<double>(X, cycle_blocks<double>(c).E(), c.at<double>(ly.off_unscale), n_elem, L,
                                      c.lat->g.vol, c.s));
  return BKWD_OK;
}

// Even-odd solves.  Before a cycle: w_o = A_oo^{-1} r_o, w_e = r_e + kappa
// H_eo w_o (the even-site right-hand side of the Schur system), scaled per
// column into the cycle's compact block.  After it: w_e = unscale_i * e_e,
// w_o = A_oo^{-1} (r_o + kappa H_oe w_e), X += w.  w keeps the whole
// correction until the next cycle, so an unhelpful one can be taken back.
template <typename T>
int eo_cycle_rhs(Ctx& c, int L, const cpx<double>* res64) {
  std::string* err = c.err;
  const WsLayout& ly = *c.ly;
  cpx<double>* w = c.at<cpx<double>>(ly.off_eo64);
  HIP_TRY(launch_eo_prepare(*c.lat, c.dagger, L, res64, w, c.at<double>(ly.off_cinv64), c.s));
  HIP_TRY(launch_eo_gather<T>(w, cycle_blocks<T>(c).R(), c.at<double>(ly.off_scale), c.lat->g, L, c.s));
  return BKWD_OK;
}

// (X == nullptr: only form the correction w)
template <typename T>
int eo_correction(Ctx& c, int L, const cpx<double>* res64, cpx<double>* X) {
  std::string* err = c.err;
  const WsLayout& ly = *c.ly;
  cpx<double>* w = c.at<cpx<double>>(ly.off_eo64);
  HIP_TRY(launch_eo_scatter<T>(cycle_blocks<T>(c).E(), w, c.at<double>(ly.off_unscale), c.lat->g, L, c.s));
  HIP_TRY(launch_eo_reconstruct(*c.lat, c.dagger, L, res64, w, c.at<double>(ly.off_cinv64), c.s));
  if (X != nullptr) HIP_TRY(launch_axpy64(X, w, 1.0, 12LL * c.lat->g.vol * L, c.s));
  return BKWD_OK;
}

int eo_undo(Ctx& c, int L, cpx<double>* X) {
  std::string* err = c.err;
  HIP_TRY(launch_axpy64(X, c.at<cpx<double>>(c.ly->off_eo64), -1.0, 12LL * c.lat->g.vol * L, c.s));
  return BKWD_OK;
}

// Thin QR factor of the FP64 block R: Gram matrix, then Cholesky on the
// device.  *ok = false when the Gram matrix is not numerically positive
// definite (the caller then scales columns instead).
int thin_qr(Ctx& c, int L, const cpx<double>* R, bool* ok) {
  std::string* err = c.err;
  BlasArgs<double> g{};
  g.L = L;
  g.nrows = 12LL * c.lat->g.vol;
  g.rt = R;
  g.v = const_cast<cpx<double>*>(R);
  g.partials = c.partials();
  g.ctl = nullptr;
  TRY(blas<double>(c, OP_GRAM, g, nullptr, 2 * L * L, 0, c.ly->off_red_b));
  Control* hc = c.host_ctl();
  std::memset(hc, 0, sizeof(Control));
  HIP_TRY(hipMemcpyAsync(c.ctl(), hc, sizeof(Control), hipMemcpyHostToDevice, c.s));
  TRY(coef(c, COEF_CHOL, coef_args(c, L, false)));
  HIP_TRY(hipMemcpyAsync(hc, c.ctl(), sizeof(Control), hipMemcpyDeviceToHost, c.s));
  HIP_TRY(hipStreamSynchronize(c.s));
  *ok = (hc->state == ST_RUNNING);
  return BKWD_OK;
}

// Deflation between cycles.  Columns whose true residual already meets tol
// are left out.  A pivoted Cholesky factorisation of the others' Gram
// matrix, largest remaining diagonal relative to the column's norm first,
// keeps the columns whose part orthogonal to those kept before is at least
// max(drop ||r_i||, tol ||b_i|| / 10): the independent set I (drop =
// kDeflateDrop64 for FP64 cycles, kDeflateDrop32 for FP32 ones, which need
// better conditioned blocks; the second bound keeps out columns that differ
// only below what the solve resolves, such as duplicated right-hand sides
// whose residuals drift apart by rounding).  Every other active
// column d is r_d ~ R_I c_d with c_d = (R_I^H R_I)^{-1} R_I^H r_d, so its
// correction is E c_d for the cycle's solution E of A E = R_I.  C (|I| x L,
// row-major) maps the cycle's columns back: C[j][I_j] = 1, C[:, d] = c_d,
// zero for converged columns.
constexpr double kDeflateDrop64 = 1e-6;
constexpr double kDeflateDrop32 = 1e-4;

void deflation_plan(int L, const std::vector<std::complex<double>>& G, const std::vector<double>& r2,
                    const std::vector<double>& b2, double tol, double drop, std::vector<int>* I,
                    std::vector<std::complex<double>>* C) {
  using cd = std::complex<double>;
  std::vector<int> active;
  for (int i = 0; i < L; ++i)
    if (std::sqrt(r2[i]) > tol * std::sqrt(b2[i])) active.push_back(i);
  const int na = (int)active.size();
  // Gram matrix of the active columns, eliminated in place; d0: their squared norms
  std::vector<cd> A((size_t)na * na);
  std::vector<double> d0(na), fl(na);
  for (int a = 0; a < na; ++a) {
    for (int b = 0; b < na; ++b) A[(size_t)a * na + b] = G[(size_t)active[a] * L + active[b]];
    d0[a] = std::real(A[(size_t)a * na + a]);
    fl[a] = 0.01 * tol * tol * b2[active[a]];
  }
  auto relrem = [&](int u) { return d0[u] > 0.0 ? std::real(A[(size_t)u * na + u]) / d0[u] : 0.0; };
  std::vector<int> perm(na);
  for (int a = 0; a < na; ++a) perm[a] = a;
  I->clear();
  for (int k = 0; k < na; ++k) {
    int best = k;
    for (int q = k + 1; q < na; ++q)
      if (relrem(perm[q]) > relrem(perm[best])) best = q;
    const int p = perm[best];
    const double piv2 = std::real(A[(size_t)p * na + p]);
    if (!(relrem(p) >= drop * drop) || !(piv2 >= fl[p])) break;
    std::swap(perm[k], perm[best]);
    I->push_back(active[p]);
    std::vector<cd> col(na);
    for (int q = 0; q < na; ++q) col[q] = A[(size_t)q * na + p];
    for (int q = k + 1; q < na; ++q)
      for (int t = k + 1; t < na; ++t) {
        const int u = perm[q], v = perm[t];
        A[(size_t)u * na + v] -= col[u] * std::conj(col[v]) / piv2;
      }
  }
  const int r = (int)I->size();
  C->assign((size_t)r * L, cd(0.0));
  for (int j = 0; j < r; ++j) (*C)[(size_t)j * L + (*I)[j]] = 1.0;
  // c_d = G_II^{-1} G_Id by Gauss-Jordan with partial pivoting (G_II is positive definite)
  for (int d : active) {
    if (std::find(I->begin(), I->end(), d) != I->end()) continue;
    std::vector<cd> M((size_t)r * (r + 1));
    for (int a = 0; a < r; ++a) {
      for (int b = 0; b < r; ++b) M[(size_t)a * (r + 1) + b] = G[(size_t)(*I)[a] * L + (*I)[b]];
      M[(size_t)a * (r + 1) + r] = G[(size_t)(*I)[a] * L + d];
    }
    for (int col = 0; col < r; ++col) {
      int pr = col;
      for (int q = col + 1; q < r; ++q)
        if (std::abs(M[(size_t)q * (r + 1) + col]) > std::abs(M[(size_t)pr * (r + 1) + col])) pr = q;
      for (int b = 0; b <= r; ++b) std::swap(M[(size_t)col * (r + 1) + b], M[(size_t)pr * (r + 1) + b]);
      const cd dv = M[(size_t)col * (r + 1) + col];
      for (int b = 0; b <= r; ++b) M[(size_t)col * (r + 1) + b] /= dv;
      for (int q = 0; q < r; ++q) {
        if (q == col) continue;
        const cd f = M[(size_t)q * (r + 1) + col];
        for (int b = 0; b <= r; ++b) M[(size_t)q * (r + 1) + b] -= f * M[(size_t)col * (r + 1) + b];
      }
    }
    for (int a = 0; a < r; ++a) (*C)[(size_t)a * L + d] = M[(size_t)a * (r + 1) + r];
  }
}

// Gram matrix R^H R of an FP64 site-major block (host copy, row-major L x L)
int residual_gram(Ctx& c, int L, const cpx<double>* R, std::vector<std::complex<double>>* G) {
  std::string* err = c.err;
  BlasArgs<double> g{};
  g.L = L;
  g.nrows = 12LL * c.lat->g.vol;
  g.rt = R;
  g.v = const_cast<cpx<double>*>(R);
  g.partials = c.partials();
  g.ctl = nullptr;
  TRY(blas<double>(c, OP_GRAM, g, nullptr, 2 * L * L, 0, c.ly->off_red_b));
  std::vector<double> h((size_t)2 * L * L);
  HIP_TRY(hipMemcpyAsync(h.data(), c.at<double>(c.ly->off_red_b), h.size() * sizeof(double), hipMemcpyDeviceToHost,
                         c.s));
  HIP_TRY(hipStreamSynchronize(c.s));
  G->resize((size_t)L * L);
  for (size_t e = 0; e < (size_t)L * L; ++e) (*G)[e] = std::complex<double>(h[2 * e], h[2 * e + 1]);
  return BKWD_OK;
}

int upload_bytes(Ctx& c, size_t off, const void* host, size_t n) {
  std::string* err = c.err;
  HIP_TRY(hipMemcpyAsync(c.ws + off, host, n, hipMemcpyHostToDevice, c.s));
  HIP_TRY(hipStreamSynchronize(c.s));
  return BKWD_OK;
}

// The outer loop for L columns held in B, X (FP64 device blocks): compute the
// FP64 true residual, stop if it meets tol, otherwise solve for a correction
// with one Krylov cycle (FP64, or FP32 for MIXED) on the column-scaled
// residual and add it.  A cycle that leaves the true residual no smaller is
// undone and retried with a fresh Gaussian shadow residual (at most twice).
int solve_columns(Ctx& c, int L, const cpx<double>* B, cpx<double>* X, const bkwd_solve_opts& o, bool scalar,
                  bool use_x0, const cpx<double>* shadow64, bkwd_solve_info* info, double** hist_out,
                  int* hist_left) {
  std::string* err = c.err;
  const WsLayout& ly = *c.ly;
  const long long n_elem = 12LL * c.lat->g.vol * L;
  cpx<double>* res64 = (ly.Lc == ly.L) ? c.at<cpx<double>>(ly.off_res64) : c.at<cpx<double>>(ly.off_res64c);
  if (!use_x0) HIP_TRY(hipMemsetAsync(X, 0, n_elem * sizeof(cpx<double>), c.s));

  std::vector<double> r2(L), b2(L), rel(L), scale(L), unscale(L);
  double prev = INFINITY;
  int last_state = ST_CONVERGED;
  int cycles = 0, failures = 0;
  bool have_correction = false, last_qr = false, last_defl = false;
  Shadow sh{o.shadow, o.seed, shadow64};
  int rc = BKWD_ENOCONV;
  // deflated cycles: Lr of the L columns, right-hand side block rhs_sub, the
  // correction mapped back as X += (cycle correction) M, M (Lr x L) in the workspace
  int Lr = L;
  cpx<double>* rhs_sub = ly.deflate ? c.at<cpx<double>>(ly.off_defl_sub) : nullptr;
  const cpx<double>* Mdev = ly.deflate ? c.at<cpx<double>>(ly.off_defl_m) : nullptr;
  auto defl_apply = [&](double sign) -> int {
    const long long nrows = 12LL * c.lat->g.vol;
    if (c.eo)
      HIP_TRY(launch_rowmat_rect<double, false>(c.at<cpx<double>>(ly.off_eo64), X, Mdev, sign, nrows, Lr, L,
                                                c.lat->g.vol, c.s));
    else if (o.prec == BKWD_MIXED)
      HIP_TRY(launch_rowmat_rect<float, true>(cycle_blocks<float>(c).E(), X, Mdev, sign, nrows, Lr, L, c.lat->g.vol,
                                              c.s));
    else
      HIP_TRY(launch_rowmat_rect<double, true>(cycle_blocks<double>(c).E(), X, Mdev, sign, nrows, Lr, L,
                                               c.lat->g.vol, c.s));
    return BKWD_OK;
  };
  for (;;) {
    TRY(residual(c, L, B, X, res64, r2.data(), b2.data()));
    double relmax = 0.0;
    bool finite = true;
    for (int i = 0; i < L; ++i) {
      if (!(b2[i] > 0.0) && cycles == 0) {
        if (err) *err = "column " + std::to_string(i) + " of B is zero";
        return BKWD_EINVAL;
      }
      rel[i] = std::sqrt(r2[i] / b2[i]);
      if (!std::isfinite(rel[i])) finite = false;
      relmax = std::max(relmax, rel[i]);
    }
    if (!finite) relmax = INFINITY;
    if (have_correction && !(relmax < prev)) {
      // the last cycle did not help: take its correction back
      if (last_defl) {
        TRY(defl_apply(-1.0));
      } else if (c.eo) {
        TRY(eo_undo(c, L, X));
      } else {
        for (int i = 0; i < L; ++i) unscale[i] = -unscale[i];
        TRY(upload(c, ly.off_unscale, unscale.data(), L));
        TRY(add_correction(c, X, n_elem, L, last_qr, -1.0));
      }
      have_correction = false;
      failures += 1;
      sh.mode = 1;
      sh.seed = next_seed(sh.seed + (unsigned long long)failures);
      if (failures > 2) {
        info->true_residual_max = prev;
        rc = (last_state == ST_BREAKDOWN) ? BKWD_EBREAKDOWN : BKWD_ENOCONV;
        break;
      }
      continue;  // recompute the residual of the restored X
    }
    info->true_residual_max = relmax;
    if (relmax <= o.tol) {
      rc = BKWD_OK;
      info->converged = 1;
      break;
    }
    if (!finite) {
      rc = BKWD_EBREAKDOWN;
      info->status_detail = 2;
      break;
    }
    if (cycles > o.max_restarts) {
      rc = BKWD_ENOCONV;
      break;
    }
    // deflation: the columns this cycle solves for
    std::vector<int> cols(L);
    for (int i = 0; i < L; ++i) cols[i] = i;
    std::vector<std::complex<double>> Cmap;
    bool defl = false;
    if (c.deflate && L > 1 && !scalar) {
      std::vector<std::complex<double>> G;
      TRY(residual_gram(c, L, res64, &G));
      std::vector<int> I;
      deflation_plan(L, G, r2, b2, o.tol, o.prec == BKWD_MIXED ? kDeflateDrop32 : kDeflateDrop64, &I, &Cmap);
      if ((int)I.size() < L && !I.empty()) {
        defl = true;
        cols = I;
      }
    }
    Lr = (int)cols.size();
    const cpx<double>* rhs64 = res64;
    if (defl) {
      TRY(upload_bytes(c, ly.off_defl_idx, cols.data(), cols.size() * sizeof(int)));
      HIP_TRY(launch_gather_idx(res64, rhs_sub, 12LL * c.lat->g.vol, L, c.at<int>(ly.off_defl_idx), Lr, c.s));
      rhs64 = rhs_sub;
    }
    const long long n_elem_r = 12LL * c.lat->g.vol * Lr;
    std::vector<double> rel_r(Lr);
    for (int j = 0; j < Lr; ++j) {
      const double rn = std::sqrt(r2[cols[j]]);
      scale[j] = rn > 0.0 ? 1.0 / rn : 0.0;
      unscale[j] = rn;
      rel_r[j] = rel[cols[j]];
    }
    if (defl) {
      // the correction of cycle column j goes to column cols[j] and, through
      // Cmap, to the dependent columns (unscaled here unless the even-odd
      // correction already is)
      std::vector<std::complex<double>> M((size_t)Lr * L);
      for (int j = 0; j < Lr; ++j)
        for (int k = 0; k < L; ++k) M[(size_t)j * L + k] = Cmap[(size_t)j * L + k] * (c.eo ? 1.0 : unscale[j]);
      TRY(upload_bytes(c, ly.off_defl_m, M.data(), M.size() * sizeof(std::complex<double>)));
    }
    // weights: the cycle's residual of column i in units of ||b_i||
    TRY(upload(c, ly.off_weight, rel_r.data(), Lr));
    TRY(upload(c, ly.off_scale, scale.data(), Lr));
    TRY(upload(c, ly.off_unscale, unscale.data(), Lr));
    CycleResult cr;
    const int method = scalar ? BKWD_BLOCK_BICGSTAB : o.method;
    bool qr = false;
    if (o.prec == BKWD_MIXED) {
      // FP32 cycles start from an orthonormal block: R = Q S (thin QR from the
      // FP64 Gram matrix); the cycle solves for Q and the correction is E S.
      // A badly conditioned restart block otherwise drives the FP32 block
      // iteration into divergence.
      const bool frame = (method == BKWD_BLOCK_BICGGR && o.qr_frame != 0);
      if (Lr > 1 && !frame && !c.eo && !defl) TRY(thin_qr(c, Lr, rhs64, &qr));
      const Blocks<float> bl = cycle_blocks<float>(c);
      if (c.eo) {
        TRY(eo_cycle_rhs<float>(c, Lr, rhs64));
      } else if (qr) {
        const CoefArgs ca = coef_args(c, Lr, false);
        HIP_TRY(launch_rowmat<float, double, false, 1>(rhs64, bl.R(), ca.Sinv, 1.0, n_elem_r / Lr, Lr,
                                                       c.lat->g.vol, c.s));
        double w0 = relmax;
        TRY(upload(c, ly.off_weight, &w0, 1));
      } else {
        HIP_TRY(launch_scale_convert<float, double>(rhs64, bl.R(), c.at<double>(ly.off_scale), n_elem_r, Lr,
                                                    c.lat->g.vol, c.s));
      }
      Reliable ru;
      const bool use_ru = o.reliable > 0.0 && frame && !scalar && !defl;
      if (use_ru) {
        ru.delta = o.reliable;
        ru.B = B;
        ru.X = X;
        ru.res64 = res64;
        ru.anchor0 = relmax;
        ru.tol = o.tol;
      }
      // with reliable updates one cycle runs to the final target
      const double itol = o.inner_tol > 0.0 ? o.inner_tol : (Lr > kSmallL ? 3e-2 : 1e-5);
      const double ctol = use_ru ? 0.5 * o.tol : std::max(itol * relmax, 0.5 * o.tol);
      TRY(run_cycle<float>(c, Lr, method, scalar, o, sh, ctol, qr, &cr, use_ru ? &ru : nullptr));
      info->reliable_updates += ru.updates;
    } else {
      const Blocks<double> bl = cycle_blocks<double>(c);
      if (c.eo)
        TRY(eo_cycle_rhs<double>(c, Lr, rhs64));
      else
        HIP_TRY(launch_scale_convert<double, double>(rhs64, bl.R(), c.at<double>(ly.off_scale), n_elem_r, Lr,
                                                     c.lat->g.vol, c.s));
      TRY(run_cycle<double>(c, Lr, method, scalar, o, sh, o.tol, false, &cr));
    }
    if (defl) {
      if (c.eo) {
        if (o.prec == BKWD_MIXED) TRY(eo_correction<float>(c, Lr, rhs64, nullptr));
        else TRY(eo_correction<double>(c, Lr, rhs64, nullptr));
      }
      TRY(defl_apply(1.0));
    } else if (c.eo) {
      if (o.prec == BKWD_MIXED) TRY(eo_correction<float>(c, L, res64, X));
      else TRY(eo_correction<double>(c, L, res64, X));
    } else {
      TRY(add_correction(c, X, n_elem, L, qr, 1.0));
    }
    last_defl = defl;
    info->deflated_columns += L - Lr;
    have_correction = true;
    last_qr = qr;
    // history entries of this cycle
    if (ly.hist_cap && *hist_left > 0) {
      const Control* hc = c.host_ctl();
      const int n = std::min(hc->hist_count, *hist_left);
      if (n > 0) {
        HIP_TRY(hipMemcpyAsync(*hist_out, c.at<double>(ly.off_hist), n * sizeof(double), hipMemcpyDeviceToHost, c.s));
        HIP_TRY(hipStreamSynchronize(c.s));
        *hist_out += n;
        *hist_left -= n;
        info->history_written += n;
      }
    }
    info->iterations += cr.iterations;
    info->recursive_residual_max = cr.resid;
    cycles += 1;
    last_state = cr.state;
    if (cr.state == ST_MAXITER) info->status_detail = 1;
    else if (cr.state == ST_BREAKDOWN) info->status_detail = 2;
    else if (cr.state == ST_STAGNATION) info->status_detail = 3;
    prev = relmax;
    if (o.shadow == 1) sh.seed = next_seed(sh.seed);
  }
  info->outer_cycles += cycles;
  if (rc == BKWD_OK) info->status_detail = 0;
  return rc;
}

}  // namespace

// Mixed-precision block solves with opts.max_block 0: up to kMixedOneBlock
// columns run as one block; wider ones as blocks of kMixedMaxBlock columns
// and one with the rest.
// The FP32 block iteration's count grows fast above 16 columns (at 16^3 x 32
// with Z2 sources: 152 at L = 16, 217 to 423 at L = 32, 358 to 782 at L = 64),
// while per block it is nearly flat from 4 to 16 columns, and above 8 columns
// the update kernels turn VALU-bound; 8 is also the narrowest width of the
// LDS-staged operator.  Measured: at 32^3 x 64 (L = 32, 64) blocks of 8 beat
// blocks of 4, 6, 11 and 16; at 24^3 x 48 with 12 point sources 8 + 4 beats
// one block of 12, 6 + 6 and 4 + 4 + 4.
constexpr int kMixedOneBlock = 8;
constexpr int kMixedMaxBlock = 8;
// FP64 block solves with opts.max_block 0: one block up to 16 columns, else
// blocks of 16.  The FP64 block iteration does not lose speed with width, but
// above 16 columns the general update kernels (FP64 register-blocked Grams)
// are VALU-bound: at 16^3 x 32, L = 64 ran at 22 RHS/s as one block and 52 as
// blocks of 16 (50 as blocks of 8).
constexpr int kFp64MaxBlock = 16;

bool ws_layout(const LatticeImpl& lat, int L, const bkwd_solve_opts& o, WsLayout* out, std::string* err,
               bool residual_only) {
  WsLayout w{};
  w.L = L;
  w.method = o.method;
  w.prec = o.prec;
  if (o.method < 0 || o.method > 2) {
    if (err) *err = "unknown method";
    return false;
  }
  if (o.prec != BKWD_FP64 && o.prec != BKWD_MIXED) {
    if (err) *err = "solve precision must be BKWD_FP64 or BKWD_MIXED";
    return false;
  }
  if (o.method == BKWD_BICGSTAB) {
    w.Lc = 1;
  } else {
    // blocks of max_block columns, the last one holding the rest
    const int mb_auto = o.prec == BKWD_MIXED ? (L > kMixedOneBlock ? kMixedMaxBlock : L)
                                             : (L > kFp64MaxBlock ? kFp64MaxBlock : L);
    w.Lc = std::min(L, o.max_block > 0 ? o.max_block : mb_auto);
  }
  w.nblocks = (o.method == BKWD_BLOCK_BICGGR) ? 8 : 7;
  if (residual_only) {
    w.Lc = 1;
    w.nblocks = 0;
  }
  w.elem = (o.prec == BKWD_MIXED) ? sizeof(cpx<float>) : sizeof(cpx<double>);
  w.evenodd = (o.evenodd != 0 && !residual_only) ? 1 : 0;
  const long long nrows = 12LL * lat.g.vol;
  const long long nrows_op = w.evenodd ? nrows / 2 : nrows;  // rows of the cycles' blocks
  const int Lc = w.Lc;
  size_t off = 0;
  w.off_res64 = off; off = align_up(off + (size_t)nrows * L * sizeof(cpx<double>));
  if (Lc != L && !residual_only) {
    const size_t cb = (size_t)nrows * Lc * sizeof(cpx<double>);
    w.off_col_b = off; off = align_up(off + cb);
    w.off_col_x = off; off = align_up(off + cb);
    w.off_col_s = off; off = align_up(off + cb);
    w.off_res64c = off; off = align_up(off + cb);
  }
  w.block_bytes = align_up((size_t)nrows_op * Lc * w.elem);
  w.off_blocks = off; off += (size_t)w.nblocks * w.block_bytes;
  w.deflate = (o.deflate != 0 && !residual_only && o.method != BKWD_BICGSTAB && Lc > 1) ? 1 : 0;
  if (w.deflate) {
    w.off_defl_sub = off; off = align_up(off + (size_t)nrows * Lc * sizeof(cpx<double>));
    w.off_defl_idx = off; off = align_up(off + (size_t)Lc * sizeof(int));
    w.off_defl_m = off; off = align_up(off + (size_t)Lc * Lc * sizeof(cpx<double>));
  }
  if (w.evenodd) {
    w.off_cinv64 = off; off = align_up(off + (size_t)lat.g.vol * 72 * sizeof(double));
    w.off_cinv32 = off; off = align_up(off + (size_t)lat.g.vol * 72 * sizeof(float));
    w.off_eo64 = off; off = align_up(off + (size_t)nrows * Lc * sizeof(cpx<double>));
    w.off_eotmp = off; off = align_up(off + (size_t)nrows_op * Lc * w.elem);
  }
  // partial records
  const size_t nv_max = 8 * (size_t)Lc * Lc + Lc;
  const size_t dblk = (size_t)dslash_launch_grid(lat.g, Lc);
  const size_t rblk = (size_t)residual_grid(lat.g.vol, L);
  const size_t upd_rows = (size_t)std::max(kUpdBlocks, kUpdBlocksSmall);
  const size_t gblk = (size_t)std::max(dslash_launch_grid(lat.g, 8), schur_gram_grid(lat.g));
  w.n_partials = std::max({upd_rows * nv_max, dblk * 4, rblk * 2 * (size_t)L, gblk * 384});
  w.off_partials = off; off = align_up(off + w.n_partials * sizeof(double));
  w.stage_half = std::max({(upd_rows + 255) / 256 * nv_max, (dblk + 255) / 256 * 4, (rblk + 255) / 256 * 2 * (size_t)L, (gblk + 255) / 256 * 384});
  w.off_stage = off; off = align_up(off + 2 * w.stage_half * sizeof(double));
  w.off_red_a = off; off = align_up(off + nv_max * sizeof(double));
  w.off_red_b = off; off = align_up(off + nv_max * sizeof(double));
  w.off_red_c = off; off = align_up(off + 4 * sizeof(double));
  w.off_red_r = off; off = align_up(off + 2 * (size_t)L * sizeof(double));
  w.off_coef = off; off = align_up(off + (12 * (size_t)Lc * Lc + 1) * sizeof(cpx<double>));
  w.off_weight = off; off = align_up(off + L * sizeof(double));
  w.off_scale = off; off = align_up(off + L * sizeof(double));
  w.off_unscale = off; off = align_up(off + L * sizeof(double));
  w.off_ctl = off; off = align_up(off + sizeof(Control));
  w.hist_cap = (o.history != nullptr && o.history_len > 0) ? (size_t)std::max(0, o.max_iter) + 1 : 0;
  w.off_hist = off; off = align_up(off + w.hist_cap * sizeof(double));
  w.total = off;
  *out = w;
  return true;
}

int solve_driver(LatticeImpl& lat, int L, const cpx<double>* B, cpx<double>* X, const bkwd_solve_opts& o, void* ws,
                 size_t ws_bytes, bkwd_solve_info* info, hipStream_t s, std::string* err) {
  const auto t0 = std::chrono::steady_clock::now();
  WsLayout ly;
  if (!ws_layout(lat, L, o, &ly, err)) return BKWD_EINVAL;
  if (ws_bytes < ly.total) {
    if (err) *err = "workspace too small: need " + std::to_string(ly.total) + " bytes";
    return BKWD_ENOMEM;
  }
  std::memset(info, 0, sizeof(*info));
  Ctx c;
  c.lat = &lat;
  c.s = s;
  c.ly = &ly;
  c.ws = static_cast<unsigned char*>(ws);
  c.profile = o.profile != 0;
  c.dagger = o.dagger;
  c.err = err;
  c.eo = ly.evenodd != 0;
  c.deflate = ly.deflate != 0;
  if (c.eo) {
    hipError_t e = launch_clover_inverse(lat, c.at<double>(ly.off_cinv64), c.at<float>(ly.off_cinv32), s);
    if (e != hipSuccess) {
      if (err) *err = std::string("clover inverse: ") + hipGetErrorString(e);
      return BKWD_EDEVICE;
    }
  }
  double* hist = o.history;
  int hist_left = (o.history != nullptr) ? std::max(0, o.history_len) : 0;
  int rc = BKWD_OK;
  info->main_width = ly.Lc;
  if (ly.Lc == L) {
    rc = solve_columns(c, L, B, X, o, o.method == BKWD_BICGSTAB, o.use_x0 != 0,
                       static_cast<const cpx<double>*>(o.shadow_block), info, &hist, &hist_left);
  } else {
    // BiCGSTAB one column at a time, or the block methods on blocks of at
    // most ly.Lc columns: each block is gathered into contiguous buffers,
    // solved on its own and scattered back.
    const long long nrows = 12LL * lat.g.vol;
    cpx<double>* bcol = c.at<cpx<double>>(ly.off_col_b);
    cpx<double>* xcol = c.at<cpx<double>>(ly.off_col_x);
    cpx<double>* scol = c.at<cpx<double>>(ly.off_col_s);
    const bool scalar = o.method == BKWD_BICGSTAB;
    double worst = 0.0;
    int worst_rc = BKWD_OK;
    bool all_conv = true;
    for (int i = 0, blk = 0; i < L; i += ly.Lc, ++blk) {
      const int n = std::min(ly.Lc, L - i);
      hipError_t e = launch_gather_cols(B, bcol, nrows, L, i, n, s);
      if (e == hipSuccess && o.use_x0) e = launch_gather_cols(X, xcol, nrows, L, i, n, s);
      if (e == hipSuccess && o.shadow == 2)
        e = launch_gather_cols(static_cast<const cpx<double>*>(o.shadow_block), scol, nrows, L, i, n, s);
      if (e != hipSuccess) {
        if (err) *err = std::string("gather: ") + hipGetErrorString(e);
        return BKWD_EDEVICE;
      }
      bkwd_solve_info ci;
      std::memset(&ci, 0, sizeof(ci));
      // timing of the full-width blocks only
      const double d0 = c.dslash_ms32;
      const int n0 = c.dslash_calls32;
      double u0[3];
      int k0[3];
      for (int q = 0; q < 3; ++q) {
        u0[q] = c.update_ms[q];
        k0[q] = c.update_calls[q];
      }
      bkwd_solve_opts oc = o;
      oc.seed = next_seed(o.seed + (unsigned long long)blk);
      const int r = solve_columns(c, n, bcol, xcol, oc, scalar, o.use_x0 != 0, scol, &ci, &hist, &hist_left);
      if (r == BKWD_EINVAL || r == BKWD_EDEVICE) return r;
      if (n == ly.Lc) {
        info->dslash_ms_fp32_main += c.dslash_ms32 - d0;
        info->dslash_calls_fp32_main += c.dslash_calls32 - n0;
        for (int q = 0; q < 3; ++q) {
          info->update_ms_main[q] += c.update_ms[q] - u0[q];
          info->update_calls_main[q] += c.update_calls[q] - k0[q];
        }
      }
      e = launch_scatter_cols(X, xcol, nrows, L, i, n, s);
      if (e != hipSuccess) {
        if (err) *err = std::string("scatter: ") + hipGetErrorString(e);
        return BKWD_EDEVICE;
      }
      info->iterations += ci.iterations;
      info->outer_cycles += ci.outer_cycles;
      info->history_written += ci.history_written;
      info->reliable_updates += ci.reliable_updates;
      info->deflated_columns += ci.deflated_columns;
      info->recursive_residual_max = std::max(info->recursive_residual_max, ci.recursive_residual_max);
      worst = std::max(worst, ci.true_residual_max);
      if (r != BKWD_OK) {
        all_conv = false;
        worst_rc = r;
        info->status_detail = ci.status_detail;
      }
    }
    info->true_residual_max = worst;
    info->converged = all_conv ? 1 : 0;
    rc = worst_rc;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    if (err) *err = std::string("solve: ") + hipGetErrorString(e);
    return BKWD_EDEVICE;
  }
  info->matvecs = c.matvecs;
  info->gram_operator = c.gram_operator ? 1 : 0;
  info->dslash_ms = c.dslash_ms;
  info->dslash_calls = c.dslash_calls;
  info->dslash_ms_fp32 = c.dslash_ms32;
  info->dslash_calls_fp32 = c.dslash_calls32;
  for (int q = 0; q < 3; ++q) {
    info->update_ms[q] = c.update_ms[q];
    info->update_calls[q] = c.update_calls[q];
  }
  if (ly.Lc == L) {
    info->dslash_ms_fp32_main = c.dslash_ms32;
    info->dslash_calls_fp32_main = c.dslash_calls32;
    for (int q = 0; q < 3; ++q) {
      info->update_ms_main[q] = c.update_ms[q];
      info->update_calls_main[q] = c.update_calls[q];
    }
  }
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rc == BKWD_ENOCONV && err) *err = "not converged";
  if (rc == BKWD_EBREAKDOWN && err) *err = "breakdown (singular L x L system or non-finite scalar)";
  return rc;
}

int true_residual_driver(LatticeImpl& lat, int L, const cpx<double>* B, const cpx<double>* X, double* per_col,
                         void* ws, size_t ws_bytes, hipStream_t s, std::string* err) {
  bkwd_solve_opts o;
  bkwd_solve_opts_default(&o);
  o.method = BKWD_BLOCK_BICGGR;
  o.prec = BKWD_FP64;
  o.history = nullptr;
  WsLayout ly;
  if (!ws_layout(lat, L, o, &ly, err, true)) return BKWD_EINVAL;
  Ctx c;
  c.lat = &lat;
  c.s = s;
  c.ly = &ly;
  c.ws = static_cast<unsigned char*>(ws);
  c.profile = false;
  c.err = err;
  if (ws_bytes < ly.total) {
    if (err) *err = "workspace too small";
    return BKWD_ENOMEM;
  }
  std::vector<double> r2(L), b2(L);
  int rc = residual(c, L, B, X, c.at<cpx<double>>(ly.off_res64), r2.data(), b2.data());
  if (rc != BKWD_OK) return rc;
  for (int i = 0; i < L; ++i) per_col[i] = b2[i] > 0.0 ? std::sqrt(r2[i] / b2[i]) : INFINITY;
  return BKWD_OK;
}
