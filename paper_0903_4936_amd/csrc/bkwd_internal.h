// Internal declarations shared by the HIP kernels and the host drivers.
#pragma once

#include <string>

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>
#include <stddef.h>

// ----------------------------------------------------------------- complex
template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) cpx {
  T re, im;
};

template <typename T> __host__ __device__ __forceinline__ cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a) { return {-a.re, -a.im}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
// a * b^*
template <typename T> __host__ __device__ __forceinline__ cpx<T> mul_conj(cpx<T> a, cpx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// a^* * b
template <typename T> __host__ __device__ __forceinline__ cpx<T> conj_mul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a and -i * a
template <typename T> __host__ __device__ __forceinline__ cpx<T> times_i(cpx<T> a) { return {-a.im, a.re}; }
template <typename T> __host__ __device__ __forceinline__ cpx<T> times_mi(cpx<T> a) { return {a.im, -a.re}; }
// acc += a * b
template <typename T> __host__ __device__ __forceinline__ void cmac(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename T> __host__ __device__ __forceinline__ void cmac_conj(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}

template <typename To, typename Ti> __host__ __device__ __forceinline__ cpx<To> cast(cpx<Ti> a) {
  return {static_cast<To>(a.re), static_cast<To>(a.im)};
}

// ----------------------------------------------------------------- geometry
struct Geom {
  int lx, ly, lz, lt;
  int vol;
};

// ----------------------------------------------------------------- lattice
struct LatticeImpl {
  Geom g;
  double kappa, csw;
  unsigned flags;
  // device regions (inside the caller's buffer)
  cpx<double>* links64;   // [4][9][V]  structure of arrays: entry (mu, 3a+b) of every site
  cpx<float>* links32;    // [4][9][V]
  cpx<float>* links32c;   // [4][6][V]  two rows, only with BKWD_COMPRESS12
  double* clover64;       // [36][V][2] A+/2, A-/2 packed Hermitian 6x6: the 72 reals of a
                          //            site as 36 pairs, pair q of all sites contiguous
  float* clover32;        // [18][V][4] the same as 18 four-vectors
  cpx<double>* canon;     // [4][V][3][3] copy of the input links
  // pinned host scratch for status read-back
  void* host_scratch;
};

// Bytes of each region, 256-aligned.
struct LatticeLayout {
  size_t off_links64, off_links32, off_links32c, off_clover64, off_clover32, off_canon, total;
};
LatticeLayout lattice_layout(const Geom& g, unsigned flags);

// ----------------------------------------------------------------- solver control
// Device-resident state of one Krylov cycle.  Every iteration kernel reads
// `state` first and does nothing once it is non-zero, so the host may queue
// iterations ahead of knowing whether the cycle has ended.
struct Control {
  int state;        // 0 running, 1 converged, 2 max_iter, 3 breakdown, 4 stagnation
  int iter;         // completed iterations
  int best_iter;    // iteration of the smallest max residual so far
  int hist_count;   // entries written to the device history
  double resid;     // max_i ||r_i|| / ||b_i|| at iteration `iter`
  double best;      // smallest value of resid so far
  double tol;       // stop threshold of this cycle
  int max_iter;
  int stagnation;
  int hist_cap;
  int frob;         // 1: resid = weight[0] * ||R||_F (orthonormalised right-hand side)
  int ru_pending;   // reliable update asked for by the stop test of this iteration
  double ru_delta;  // > 0: ask for a reliable update when resid < ru_delta * ru_anchor
  double ru_anchor; // resid at the last reliable update (or the cycle start)
};

enum { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXITER = 2, ST_BREAKDOWN = 3, ST_STAGNATION = 4, ST_RELIABLE = 5 };

// ----------------------------------------------------------------- launchers
// setup
hipError_t launch_pack_links(const LatticeImpl& lat, hipStream_t s);
hipError_t launch_clover_build(const LatticeImpl& lat, hipStream_t s);
hipError_t launch_clover_build_into(const LatticeImpl& lat, double* c64, double kc, hipStream_t s);
// Re <Lam, (csw C + H) X> and Re <Lam, C X> per workgroup (partials[4 * blk + {0, 1}]);
// unit_clover holds the blocks of 1 - C
// pion[t], rho[t] (device, Lt doubles) from the 12 point-source solutions X
hipError_t launch_mesons(const LatticeImpl& lat, const cpx<double>* X, double* pion, double* rho, hipStream_t s);

hipError_t launch_grad_scalars(const LatticeImpl& lat, int L, const cpx<double>* x, const cpx<double>* lam,
                               const double* unit_clover, double csw, double* partials, int* nblk_out, hipStream_t s);
// W^{mu nu}(n) for the six planes mu < nu, and the link gradient
hipError_t launch_clover_w(const LatticeImpl& lat, int L, const cpx<double>* x, const cpx<double>* lam, double kc,
                           cpx<double>* w, hipStream_t s);
hipError_t launch_link_force(const LatticeImpl& lat, int L, const cpx<double>* x, const cpx<double>* lam,
                             const cpx<double>* w, cpx<double>* grad, hipStream_t s);

// Dirac operator.  `epi` optionally receives per-workgroup partial sums of
// Tr(Y^H X) and Tr(Y^H Y) for the operator's own input X and output Y
// (4 doubles per workgroup, laid out [nblk][4]); returns the number of
// workgroups written through *nblk_out.  When `ctl` is non-null the kernel
// does nothing once ctl->state != 0.
// comp_major: blocks in the Krylov-workspace layout [spin*3+colour][site][rhs]
// instead of the ABI layout [site][spin*3+colour][rhs].
template <typename T>
hipError_t launch_dslash(const LatticeImpl& lat, int dagger, int L, const cpx<T>* in, cpx<T>* out,
                         double* epi, int* nblk_out, const Control* ctl, bool comp_major, hipStream_t s);

// r = b - D x in FP64 with per-workgroup partial ||r_i||^2 and ||b_i||^2
// ([nblk][2L] doubles); at most kResidualBlocks workgroups.
constexpr int kResidualBlocks = 1024;
int residual_grid(long long vol, int L);
// workgroups of a one-pass operator launch (the t-slice grid); the trace
// epilogue writes one partial record per workgroup
int dslash_launch_grid(const Geom& g, int L);
// W' = A T for an 8-column FP32 component-major block with the per-workgroup
// Grams T^H W', W'^H W', R~0^H W' ([nblk][384] doubles in partials)
bool dslash_gram_supported(const LatticeImpl& lat, int L);
hipError_t launch_dslash_gram(const LatticeImpl& lat, int dagger, const cpx<float>* in, cpx<float>* out,
                              const cpx<float>* rt, double* partials, int* nblk_out, const Control* ctl,
                              hipStream_t s);
hipError_t launch_residual_norms64(const LatticeImpl& lat, int dagger, int L, const cpx<double>* b,
                                   const cpx<double>* x, double* partials, int* nblk_out, hipStream_t s);
// even-odd solve (csrc/dslash.hip, csrc/setup.hip): the inverse site-local
// blocks, the Schur operator on compact even blocks (component-major, site / 2),
// and the FP64 preparation / reconstruction on whole-lattice site-major blocks
hipError_t launch_clover_inverse(const LatticeImpl& lat, double* i64, float* i32, hipStream_t s);
template <typename T>
hipError_t launch_schur(const LatticeImpl& lat, int dagger, int L, const cpx<T>* in, cpx<T>* out, cpx<T>* tmp,
                        const void* clover, const void* cinv, const Control* ctl, hipStream_t s);
// The Schur operator of launch_schur on 8-column FP32 compact blocks whose second
// launch also leaves the partial Grams in^H out, out^H out, rt^H out in nblk
// partial records (schur_gram_grid of them)
bool schur_gram_supported(const LatticeImpl& lat, int L);
int schur_gram_grid(const Geom& g);
hipError_t launch_schur_gram(const LatticeImpl& lat, int dagger, const cpx<float>* in, cpx<float>* out,
                             cpx<float>* tmp, const void* clover, const void* cinv, const cpx<float>* rt,
                             double* partials, int* nblk_out, const Control* ctl, hipStream_t s);
hipError_t launch_eo_prepare(const LatticeImpl& lat, int dagger, int L, const cpx<double>* r, cpx<double>* w,
                             const double* cinv64, hipStream_t s);
hipError_t launch_eo_reconstruct(const LatticeImpl& lat, int dagger, int L, const cpx<double>* r, cpx<double>* w,
                                 const double* cinv64, hipStream_t s);

// bkwd_true_residual_noalloc (csrc/noalloc.hip)
int true_residual_noalloc(LatticeImpl& lat, int L, const cpx<double>* B, const cpx<double>* X, double* per_col,
                          hipStream_t s, std::string* err);
hipError_t launch_residual64(const LatticeImpl& lat, int dagger, int L, const cpx<double>* b, const cpx<double>* x,
                             cpx<double>* r, double* partials, int* nblk_out, hipStream_t s);
