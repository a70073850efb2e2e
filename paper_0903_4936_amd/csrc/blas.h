// Block kernels of the Krylov solvers: argument structs and launchers.
#pragma once

#include "bkwd_internal.h"

// Streaming block kernels use at most this many workgroups (grid-stride),
// so per-workgroup partial records stay few.
#ifndef BKWD_UPD_BLOCKS
#define BKWD_UPD_BLOCKS 2048
#endif
constexpr int kUpdBlocks = BKWD_UPD_BLOCKS;
// L <= kSmallL uses the register-column kernels with more workgroups
constexpr int kSmallL = 16;
#ifndef BKWD_UPD_BLOCKS_SMALL
#define BKWD_UPD_BLOCKS_SMALL 2048
#endif
constexpr int kUpdBlocksSmall = BKWD_UPD_BLOCKS_SMALL;

enum BlasOp {
  OP_BICGGR_U = 0,     // U = (P - zeta V) m1
  OP_BICGGR_XR = 1,    // X += zeta R + U; R -= zeta W + Y; [R~0^H R, ||r||^2]
  OP_BICGGR_PV = 2,    // P = R + U m1; V = W + Y m1; [R~0^H V]
  OP_BICGSTAB_T = 3,   // W(=T) = R - V m1
  OP_BICGSTAB_XR = 4,  // X += P m1 + zeta W(=T); R = T - zeta Y(=Z); [R~0^H R, R~0^H Z, ||r||^2]
  OP_BICGSTAB_P = 5,   // P = R + (P - zeta V) m1
  OP_GRAM = 6,         // [R~0^H V, ||v||^2 if want_norms]
  OP_GRAM2 = 7,        // [rt^H v, w^H r]
  OP_GGRQ_XR = 8,      // QR frame: X += (zeta Q + U) m1; T = Q - zeta W - Y; [T^H T, R~0^H T]
  OP_GGRQ_PV = 9,      // QR frame: Q = T m1; W = W m1; P = Q + U m2; V = W + Y m2; [R~0^H V, W^H Q, W^H W]
  // QR frame with P and V eliminated (L <= kSmallL); r holds T (Q = T tau^-1), w holds W' = A T
  OP_FU = 10,          // U = (T - zeta W') m1 + (U - zeta Y) m2   (in place)
  OP_FXR = 11,         // X += T m1 + U m2; T = (T - zeta W') m3 - Y; [T^H T, R~0^H T, R~0^H Y]
  OP_FGRAM = 12,       // [gl0^H gr, gl1^H gr, gl2^H gr] for the first ng left operands
  // the same frame with the solution update moved into the U pass (8-column
  // FP32 blocks, blas_fused_x): 7 + 5 passes instead of 5 + 8
  OP_FUX = 13,         // U = (T - zeta W') m1 + (U - zeta Y) m2; X += T m3 + U_new m4
  OP_FXRT = 14         // T = (T - zeta W') m3 - Y; [T^H T, R~0^H T, R~0^H Y]
};

template <typename T>
struct BlasArgs {
  int L;
  int nv;            // doubles per workgroup partial record
  int want_norms;
  long long nrows;   // N = 12 V
  cpx<T>* x;
  cpx<T>* r;
  cpx<T>* p;
  cpx<T>* v;
  cpx<T>* w;
  cpx<T>* u;
  cpx<T>* y;
  const cpx<T>* rt;
  const cpx<double>* m1;    // L x L coefficient matrix (FP64)
  const cpx<double>* m2;    // second L x L matrix (FP64)
  const cpx<double>* m3;    // third L x L matrix (FP64)
  const cpx<double>* m4;    // fourth L x L matrix (FP64, OP_FUX)
  const cpx<T>* gl[3];      // OP_FGRAM: left operands
  const cpx<T>* gr;         // OP_FGRAM: right operand
  int ng;                   // OP_FGRAM: number of left operands (1..3)
  const cpx<double>* zeta;  // scalar (FP64)
  double* partials;
  const Control* ctl;
};

enum CoefOp {
  COEF_INIT = 0,
  COEF_BICGGR_TOP = 1,
  COEF_BICGGR_END = 2,
  COEF_BICGSTAB_ALPHA = 3,
  COEF_BICGSTAB_ZETA = 4,
  COEF_BICGSTAB_BETA = 5,
  COEF_CHOL = 6,
  COEF_GGRQ_INIT = 7,
  COEF_GGRQ_INIT2 = 8,
  COEF_GGRQ_TOP = 9,
  COEF_GGRQ_END = 10,
  COEF_FINIT = 11,
  COEF_FTOP = 12,
  COEF_RU_FRAME = 13,  // reliable update: new frame from the true residual's Gram
  COEF_RU_COMMIT = 14  // end of an iteration: a pending reliable update stops the queue
};

struct CoefArgs {
  int L;
  int scalar;            // BiCGSTAB with the scalar beta formula (L = 1)
  const double* red_a;   // reduced record of the last update kernel
  const double* red_b;   // reduced R~0^H V
  const double* red_c;   // reduced traces (Re, Im of Tr(Y^H X), Tr(Y^H Y))
  cpx<double>* GR;       // R~0^H R_k
  cpx<double>* GV;       // R~0^H V_k
  cpx<double>* alpha;
  cpx<double>* beta;     // beta (BiCGSTAB) or gamma (BiCGGR)
  cpx<double>* zeta;
  cpx<double>* S;        // thin-QR factor of the cycle's right-hand side
  cpx<double>* Sinv;
  cpx<double>* xi;       // QR frame: R_k = Q_k xi_k
  cpx<double>* tmp;
  cpx<double>* mu1;      // fused QR frame: tau^-1 alpha
  cpx<double>* mu2;      // fused QR frame: gamma_{k-1} alpha
  cpx<double>* mx1;      // fused QR frame: zeta eta
  cpx<double>* eta;      // fused QR frame: tau^-1 xi (= xi of the previous iteration)
  const double* weight;  // per-column weights of the stop test
  Control* ctl;
  double* hist;
};

size_t blas_smem_bytes(int L, size_t elem);
int blas_grid(long long nrows, int L);
template <typename T>
int blas_launch(int op, const BlasArgs<T>& a, hipStream_t s);
// whether OP_FUX / OP_FXRT exist for blocks of L columns of this element size
bool blas_fused_x(int L, size_t elem);
hipError_t launch_reduce(const double* in, long long nrows, int nv, double* stage, size_t stage_half, double* out,
                         hipStream_t s);
hipError_t launch_coef(int op, const CoefArgs& c, hipStream_t s);
template <typename T>
hipError_t launch_gaussian(cpx<T>* out, long long n, unsigned long long seed, hipStream_t s);
// Conversions between the ABI block layout (site-major, FP64) of the outer
// loop and the component-major layout of the Krylov cycle blocks.
template <typename To, typename Ti>
hipError_t launch_scale_convert(const cpx<Ti>* in, cpx<To>* out, const double* scale, long long n, int L, int vol,
                                hipStream_t s);
template <typename Ti>
hipError_t launch_accumulate(cpx<double>* x, const cpx<Ti>* e, const double* scale, long long n, int L, int vol,
                             hipStream_t s);
template <typename To>
hipError_t launch_convert(const cpx<double>* in, cpx<To>* out, long long n, int L, int vol, hipStream_t s);
template <typename To, typename Ti, bool ACC, int PERM>
hipError_t launch_rowmat(const cpx<Ti>* in, cpx<To>* out, const cpx<double>* M, double sign, long long nrows, int L,
                         int vol, hipStream_t s);
// columns c0 .. c0 + n - 1 of an nrows x L block <-> a contiguous nrows x n block
hipError_t launch_gather_cols(const cpx<double>* X, cpx<double>* x, long long nrows, int L, int c0, int n,
                              hipStream_t s);
hipError_t launch_scatter_cols(cpx<double>* X, const cpx<double>* x, long long nrows, int L, int c0, int n,
                               hipStream_t s);
hipError_t blas_set_attributes();
// even-odd blocks: the even sites of an FP64 site-major block <-> a compact
// even block (component-major, position site / 2), with per-column scaling;
// x += sign * w over FP64 blocks
template <typename To>
hipError_t launch_eo_gather(const cpx<double>* in, cpx<To>* out, const double* scale, const Geom& g, int L,
                            hipStream_t s);
template <typename Ti>
hipError_t launch_eo_scatter(const cpx<Ti>* in, cpx<double>* out, const double* unscale, const Geom& g, int L,
                             hipStream_t s);
hipError_t launch_axpy64(cpx<double>* x, const cpx<double>* w, double sign, long long n, hipStream_t s);
// per-workgroup [Re Tr(Y^H X), Im Tr(Y^H X), Tr(Y^H Y), 0] over n elements (at most 1024 workgroups)
template <typename T>
hipError_t launch_trace2(const cpx<T>* x, const cpx<T>* y, long long n, double* partials, int* nblk, hipStream_t s);
// deflation: columns idx[0..n) of an nrows x L block into a contiguous nrows x n
// block; out (site-major, Lout columns) += sign * in (Lin columns, component-
// major if CM) times the Lin x Lout FP64 matrix M
hipError_t launch_gather_idx(const cpx<double>* src, cpx<double>* dst, long long nrows, int L, const int* idx, int n,
                             hipStream_t s);
template <typename Ti, bool CM>
hipError_t launch_rowmat_rect(const cpx<Ti>* in, cpx<double>* out, const cpx<double>* M, double sign, long long nrows,
                              int Lin, int Lout, int vol, hipStream_t s);
