// Tall-skinny block kernels of the Krylov solvers of Sec. 3: the fused block
// updates with their (N x L)(L x L) products, the Gram matrices R~0^H M
// (L x L), column norms, a deterministic reduction of per-workgroup partial
// sums, and the single-workgroup FP64 kernels that solve the L x L systems
// and decide whether the iteration continues.
//
// Thread mapping of the streaming kernels: a workgroup of 256 threads covers
// a tile of R = 256 / L consecutive rows; thread t owns element
// (row = tile*R + t/L, column t%L), so element loads and stores are
// contiguous.  Operands that enter a row product are staged in LDS.  Gram
// contributions are accumulated in FP64 by threads that own (i, j) entries.
#include "blas.h"
#include "mfma16.h"

#include <algorithm>
#include <type_traits>

namespace {

constexpr int kBT = 256;

template <typename T>
struct TileMap {
  int L, R, nact, rl, j;
  bool act;
  __device__ __forceinline__ explicit TileMap(int L_) : L(L_) {
    R = kBT / L;
    nact = R * L;
    rl = threadIdx.x / L;
    j = threadIdx.x - rl * L;
    act = (int)threadIdx.x < nact;
  }
};

template <typename T>
__device__ __forceinline__ bool running(const Control* ctl) {
  return ctl == nullptr || ctl->state == ST_RUNNING;
}

// Load an L x L FP64 matrix into LDS in precision T.
template <typename T>
__device__ __forceinline__ void load_matrix(cpx<T>* sM, const cpx<double>* __restrict__ M, int L) {
  for (int e = threadIdx.x; e < L * L; e += kBT) sM[e] = cast<T>(M[e]);
}

// out = sum_i S[rl][i] M[i][j]  (S, M in LDS)
template <typename T>
__device__ __forceinline__ cpx<T> row_product(const cpx<T>* sS, const cpx<T>* sM, int rl, int j, int L) {
  cpx<T> acc = mk(T(0), T(0));
  const cpx<T>* srow = sS + rl * L;
  for (int i = 0; i < L; ++i) cmac(acc, srow[i], sM[i * L + j]);
  return acc;
}

// Gram accumulation over the rows of one staged tile: acc[k] for entry
// e = threadIdx.x + k*256 (i = e / L, j = e % L) += sum_r conj(A[r][i]) B[r][j].
template <typename T, int NE>
__device__ __forceinline__ void gram_tile(cpx<double> acc[NE], const cpx<T>* sA, const cpx<T>* sB, int rows, int L) {
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = threadIdx.x + k * kBT;
    if (e < L * L) {
      const int i = e / L, jj = e - (e / L) * L;
      for (int r = 0; r < rows; ++r) {
        const cpx<T> a = sA[r * L + i], b = sB[r * L + jj];
        cmac_conj(acc[k], cast<double>(a), cast<double>(b));
      }
    }
  }
}

template <int NE>
__device__ __forceinline__ void gram_store(const cpx<double> acc[NE], double* out, int L) {
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = threadIdx.x + k * kBT;
    if (e < L * L) {
      out[2 * e] = acc[k].re;
      out[2 * e + 1] = acc[k].im;
    }
  }
}

// Gram accumulators of the general-L kernels.  Every product and sum is FP64
// (the products of FP32 operands are exact): the QR frame's Cholesky of
// T^H T and the solves with R~0^H T need that accuracy once the residual
// block is badly conditioned, which at L = 64 it becomes.
//
// Layout code NE: 1 = one entry per thread (L <= 16); 4, 9, 16 = a B x B
// register block per thread (B = 2, 3, 4); -NT = FP64 MFMA with L = 8 NT.

// Register-blocked Gram accumulation for 16 < L <= 16 B, NE = B^2: thread t
// owns the B x B block of entries with rows i = B (t / 16) + p and columns
// j = B (t % 16) + q, acc[p B + q] += sum_r conj(A[r][i]) B[r][j].  Each LDS
// value read feeds B products.  Where 16 B > L the block runs past the row
// into the next one (or past the tile, still inside the workgroup's LDS);
// those entries have i >= L or j >= L and are never stored.
template <typename T, int B>
__device__ __forceinline__ void gram_blk(cpx<double>* acc, const cpx<T>* sA, const cpx<T>* sB, int rows, int L) {
  const int i0 = (threadIdx.x >> 4) * B, j0 = (threadIdx.x & 15) * B;
  for (int r = 0; r < rows; ++r) {
    cpx<double> a[B], b[B];
#pragma unroll
    for (int p = 0; p < B; ++p) a[p] = cast<double>(sA[r * L + i0 + p]);
#pragma unroll
    for (int q = 0; q < B; ++q) b[q] = cast<double>(sB[r * L + j0 + q]);
#pragma unroll
    for (int p = 0; p < B; ++p)
#pragma unroll
      for (int q = 0; q < B; ++q) cmac_conj(acc[p * B + q], a[p], b[q]);
  }
}

template <int B>
__device__ __forceinline__ void gram_store_blk(const cpx<double>* acc, double* out, int L) {
  const int i0 = (threadIdx.x >> 4) * B, j0 = (threadIdx.x & 15) * B;
#pragma unroll
  for (int p = 0; p < B; ++p)
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (i0 + p < L && j0 + q < L) {
        const int e = (i0 + p) * L + j0 + q;
        out[2 * e] = acc[p * B + q].re;
        out[2 * e + 1] = acc[p * B + q].im;
      }
    }
}

// FP64 MFMA Gram for L = 8 NT (NT <= 4).  The tile's rows are read as real
// rows of 2L values (re, im interleaved), so that P = A'^T B' (2L x 2L, real,
// summed over rows) holds G = A^H B in its 2 x 2 blocks:
//   G_ij = (P[2i][2j] + P[2i+1][2j+1]) + i (P[2i][2j+1] - P[2i+1][2j]).
// Wave w < NT owns the 16-row band w of P, as NT tiles of 16 x 16, each one
// v_mfma_f64_16x16x4f64 per 4 rows of the tile.  Operands: lane l supplies
// A[m][k] and B[k][n] with k = l / 16 and m, n = l % 16; output register v of
// lane l is D[l / 16 + 4 v][l % 16].  The A operand's row m is taken from real
// row 4 (m % 4) + m / 4 of the band, so that lane l holds band rows
// 4 (l / 16) + v: re and im of one complex row in registers v, v + 1.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <typename T, int NT>
__device__ __forceinline__ void gram_mfma(mfma_d4 acc[NT], const cpx<T>* sA, const cpx<T>* sB, int rows, int L) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (w >= NT) return;  // uniform over the wave
  const T* rA = reinterpret_cast<const T*>(sA);
  const T* rB = reinterpret_cast<const T*>(sB);
  const int m = l & 15, kq = l >> 4;
  const int ca = w * 16 + 4 * (m & 3) + (m >> 2);
  for (int k0 = 0; k0 < rows; k0 += 4) {
    const int r = k0 + kq;
    const bool ok = r < rows;
    const double a = ok ? (double)rA[r * 2 * L + ca] : 0.0;
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      const double b = ok ? (double)rB[r * 2 * L + tj * 16 + m] : 0.0;
      acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[tj], 0, 0, 0);
    }
  }
}

template <int NT>
__device__ __forceinline__ void gram_mfma_store(const mfma_d4 acc[NT], double* out, int L) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (w >= NT) return;
  const int m = l & 15, kq = l >> 4;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj) {
    double nb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) nb[v] = __shfl_xor(acc[tj][v], 1);
    if ((m & 1) == 0) {
      const int j = tj * 8 + (m >> 1);
#pragma unroll
      for (int v = 0; v < 4; v += 2) {
        const int i = w * 8 + 2 * kq + (v >> 1);
        const int e = i * L + j;
        out[2 * e] = acc[tj][v] + nb[v + 1];
        out[2 * e + 1] = nb[v] - acc[tj][v + 1];
      }
    }
  }
}

template <int NE>
struct GBlock;
template <> struct GBlock<4> { static constexpr int B = 2; };
template <> struct GBlock<9> { static constexpr int B = 3; };
template <> struct GBlock<16> { static constexpr int B = 4; };

template <typename T, int NE, bool MFMA = (NE < 0)>
struct Gram {
  cpx<double> v[NE];
  __device__ Gram() {
#pragma unroll
    for (int k = 0; k < NE; ++k) v[k] = mk(0.0, 0.0);
  }
  // += sum over the tile's rows of conj(A[r][i]) B[r][j]
  __device__ void add(const cpx<T>* sA, const cpx<T>* sB, int rows, int L) {
    if constexpr (NE == 1) gram_tile<T, 1>(v, sA, sB, rows, L);
    else gram_blk<T, GBlock<NE>::B>(v, sA, sB, rows, L);
  }
  // this workgroup's partial Gram: out[2 (i L + j)] = re, out[2 (i L + j) + 1] = im
  __device__ void store(double* out, int L) const {
    if constexpr (NE == 1) gram_store<1>(v, out, L);
    else gram_store_blk<GBlock<NE>::B>(v, out, L);
  }
};

template <typename T, int NE>
struct Gram<T, NE, true> {
  static constexpr int NT = -NE;
  mfma_d4 v[NT];
  __device__ Gram() {
#pragma unroll
    for (int k = 0; k < NT; ++k) v[k] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  }
  __device__ void add(const cpx<T>* sA, const cpx<T>* sB, int rows, int L) { gram_mfma<T, NT>(v, sA, sB, rows, L); }
  __device__ void store(double* out, int L) const { gram_mfma_store<NT>(v, out, L); }
};

// Per-column sum of a per-thread value, fixed order; threads j < L write out[j].
__device__ __forceinline__ void column_store(double v, double* red, double* out, int L, int nact) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  if ((int)threadIdx.x < L) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nact; k += L) s += red[k];
    out[threadIdx.x] = s;
  }
}

template <typename T>
__device__ __forceinline__ double abs2(cpx<T> v) {
  return (double)v.re * (double)v.re + (double)v.im * (double)v.im;
}

// ------------------------------------------------------------------ LDS carving
template <typename T>
struct Smem {
  cpx<T>* M1;
  cpx<T>* M2;
  cpx<T>* t0;
  cpx<T>* t1;
  cpx<T>* t2;
  cpx<T>* t3;
  cpx<T>* t4;
  double* red;
};

template <typename T>
__device__ __forceinline__ Smem<T> carve(unsigned char* base, int L) {
  Smem<T> s;
  cpx<T>* p = reinterpret_cast<cpx<T>*>(base);
  s.M1 = p; p += L * L;
  s.M2 = p; p += L * L;
  s.t0 = p; p += kBT;
  s.t1 = p; p += kBT;
  s.t2 = p; p += kBT;
  s.t3 = p; p += kBT;
  s.t4 = p; p += kBT;
  s.red = reinterpret_cast<double*>(p);
  return s;
}

}  // namespace

size_t blas_smem_bytes(int L, size_t elem) {
  return (size_t)(2 * L * L + 5 * kBT) * 2 * elem + kBT * sizeof(double);
}

namespace {

// ------------------------------------------------------------------ BiCGGR
// U = (P - zeta V) alpha
template <typename T>
__global__ void __launch_bounds__(kBT) k_bicggr_u(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  load_matrix(sm.M1, a.m1, L);
  const cpx<T> z = cast<T>(a.zeta[0]);
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * tm.R + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    __syncthreads();
    if (valid) {
      const cpx<T> p = a.p[e], v = a.v[e];
      sm.t0[threadIdx.x] = p - z * v;
    }
    __syncthreads();
    if (valid) a.u[e] = row_product(sm.t0, sm.M1, tm.rl, tm.j, L);
  }
}

// X += zeta R + U;  R <- R - zeta W - Y;  partials: R~0^H R (L^2), ||r_i||^2 (L)
template <typename T, int NE>
__global__ void __launch_bounds__(kBT) k_bicggr_xr(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  const cpx<T> z = cast<T>(a.zeta[0]);
  Gram<T, NE> acc;
  double nrm = 0.0;
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row0 = tile * tm.R;
    const long long row = row0 + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    const int rows = (int)min((long long)tm.R, a.nrows - row0);
    __syncthreads();
    if (valid) {
      const cpx<T> r = a.r[e];
      const cpx<T> x = a.x[e] + z * r + a.u[e];
      const cpx<T> rn = r - z * a.w[e] - a.y[e];
      a.x[e] = x;
      a.r[e] = rn;
      sm.t0[threadIdx.x] = a.rt[e];
      sm.t1[threadIdx.x] = rn;
      nrm += abs2(rn);
    }
    __syncthreads();
    acc.add(sm.t0, sm.t1, rows, L);
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  acc.store(out, L);
  column_store(nrm, sm.red, out + 2 * L * L, L, tm.nact);
}

// P = R + U gamma;  V = W + Y gamma;  partials: R~0^H V (L^2)
template <typename T, int NE>
__global__ void __launch_bounds__(kBT) k_bicggr_pv(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  load_matrix(sm.M1, a.m1, L);
  Gram<T, NE> acc;
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row0 = tile * tm.R;
    const long long row = row0 + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    const int rows = (int)min((long long)tm.R, a.nrows - row0);
    __syncthreads();
    if (valid) {
      sm.t0[threadIdx.x] = a.u[e];
      sm.t1[threadIdx.x] = a.y[e];
      sm.t2[threadIdx.x] = a.rt[e];
    }
    __syncthreads();
    cpx<T> v = mk(T(0), T(0));
    if (valid) {
      const cpx<T> p = a.r[e] + row_product(sm.t0, sm.M1, tm.rl, tm.j, L);
      v = a.w[e] + row_product(sm.t1, sm.M1, tm.rl, tm.j, L);
      a.p[e] = p;
      a.v[e] = v;
    }
    __syncthreads();
    if (valid) sm.t0[threadIdx.x] = v;
    __syncthreads();
    acc.add(sm.t2, sm.t0, rows, L);
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  acc.store(out, L);
}

// ------------------------------------------------------------------ BiCGSTAB
// T = R - V alpha
template <typename T>
__global__ void __launch_bounds__(kBT) k_bicgstab_t(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  load_matrix(sm.M1, a.m1, L);
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * tm.R + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    __syncthreads();
    if (valid) sm.t0[threadIdx.x] = a.v[e];
    __syncthreads();
    if (valid) a.w[e] = a.r[e] - row_product(sm.t0, sm.M1, tm.rl, tm.j, L);
  }
}

// X += P alpha + zeta T;  R = T - zeta Z;
// partials: R~0^H R (L^2), R~0^H Z (L^2), ||r_i||^2 (L)
template <typename T, int NE>
__global__ void __launch_bounds__(kBT) k_bicgstab_xr(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  load_matrix(sm.M1, a.m1, L);
  const cpx<T> z = cast<T>(a.zeta[0]);
  Gram<T, NE> acc1, acc2;
  double nrm = 0.0;
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row0 = tile * tm.R;
    const long long row = row0 + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    const int rows = (int)min((long long)tm.R, a.nrows - row0);
    __syncthreads();
    if (valid) {
      sm.t0[threadIdx.x] = a.p[e];
      sm.t1[threadIdx.x] = a.rt[e];
    }
    __syncthreads();
    cpx<T> rn = mk(T(0), T(0)), zz = mk(T(0), T(0));
    if (valid) {
      const cpx<T> t = a.w[e];
      zz = a.y[e];
      a.x[e] = a.x[e] + row_product(sm.t0, sm.M1, tm.rl, tm.j, L) + z * t;
      rn = t - z * zz;
      a.r[e] = rn;
      nrm += abs2(rn);
    }
    __syncthreads();
    if (valid) {
      sm.t0[threadIdx.x] = rn;
      sm.t2[threadIdx.x] = zz;
    }
    __syncthreads();
    acc1.add(sm.t1, sm.t0, rows, L);
    acc2.add(sm.t1, sm.t2, rows, L);
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  acc1.store(out, L);
  acc2.store(out + 2 * L * L, L);
  column_store(nrm, sm.red, out + 4 * L * L, L, tm.nact);
}

// P = R + (P - zeta V) beta
template <typename T>
__global__ void __launch_bounds__(kBT) k_bicgstab_p(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  load_matrix(sm.M1, a.m1, L);
  const cpx<T> z = cast<T>(a.zeta[0]);
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * tm.R + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    __syncthreads();
    if (valid) sm.t0[threadIdx.x] = a.p[e] - z * a.v[e];
    __syncthreads();
    if (valid) a.p[e] = a.r[e] + row_product(sm.t0, sm.M1, tm.rl, tm.j, L);
  }
}

// ------------------------------------------------------------------ one column
// L = 1 (BiCGSTAB solving one column at a time): plain streaming kernels, one
// element per thread and grid stride, the 1 x 1 coefficients as scalars, the
// sums of a workgroup in a fixed order (FP64): record layouts as above.

// sum over the workgroup of NV per-thread values into out[0..NV)
template <int NV>
__device__ __forceinline__ void k1_store(double (&v)[NV], double* out) {
  __shared__ double red[NV][kBT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double x = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[q][w] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double x = 0.0;
#pragma unroll
    for (int k = 0; k < kBT / 64; ++k) x += red[threadIdx.x][k];
    out[threadIdx.x] = x;
  }
}

// W(=T) = R - V alpha
template <typename T>
__global__ void __launch_bounds__(kBT) k1_bicgstab_t(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  const cpx<T> al = cast<T>(a.m1[0]);
  for (long long e = (long long)blockIdx.x * kBT + threadIdx.x; e < a.nrows; e += (long long)gridDim.x * kBT)
    a.w[e] = a.r[e] - a.v[e] * al;
}

// X += P alpha + zeta T;  R = T - zeta Z;  [r~^H r, r~^H z, ||r||^2]
template <typename T>
__global__ void __launch_bounds__(kBT) k1_bicgstab_xr(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  const cpx<T> al = cast<T>(a.m1[0]);
  const cpx<T> z = cast<T>(a.zeta[0]);
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long e = (long long)blockIdx.x * kBT + threadIdx.x; e < a.nrows; e += (long long)gridDim.x * kBT) {
    const cpx<T> t = a.w[e], zz = a.y[e], rt = a.rt[e];
    a.x[e] = a.x[e] + a.p[e] * al + z * t;
    const cpx<T> rn = t - z * zz;
    a.r[e] = rn;
    const cpx<double> r8 = cast<double>(rn), z8 = cast<double>(zz), t8 = cast<double>(rt);
    v[0] += t8.re * r8.re + t8.im * r8.im;
    v[1] += t8.re * r8.im - t8.im * r8.re;
    v[2] += t8.re * z8.re + t8.im * z8.im;
    v[3] += t8.re * z8.im - t8.im * z8.re;
    v[4] += r8.re * r8.re + r8.im * r8.im;
  }
  k1_store<5>(v, a.partials + (long long)blockIdx.x * a.nv);
}

// P = R + (P - zeta V) beta
template <typename T>
__global__ void __launch_bounds__(kBT) k1_bicgstab_p(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  const cpx<T> be = cast<T>(a.m1[0]);
  const cpx<T> z = cast<T>(a.zeta[0]);
  for (long long e = (long long)blockIdx.x * kBT + threadIdx.x; e < a.nrows; e += (long long)gridDim.x * kBT)
    a.p[e] = a.r[e] + (a.p[e] - z * a.v[e]) * be;
}

// [r~^H v] and, if a.want_norms, ||v||^2
template <typename T>
__global__ void __launch_bounds__(kBT) k1_gram(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  double v[3] = {0.0, 0.0, 0.0};
  for (long long e = (long long)blockIdx.x * kBT + threadIdx.x; e < a.nrows; e += (long long)gridDim.x * kBT) {
    const cpx<double> t8 = cast<double>(a.rt[e]), v8 = cast<double>(a.v[e]);
    v[0] += t8.re * v8.re + t8.im * v8.im;
    v[1] += t8.re * v8.im - t8.im * v8.re;
    v[2] += v8.re * v8.re + v8.im * v8.im;
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  if (a.want_norms) {
    k1_store<3>(v, out);
  } else {
    double u[2] = {v[0], v[1]};
    k1_store<2>(u, out);
  }
}

// ------------------------------------------------------------------ Gram + norms
// partials: R~0^H M (L^2) and, if a.want_norms, ||m_i||^2 (L)
template <typename T, int NE>
__global__ void __launch_bounds__(kBT) k_gram(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  Gram<T, NE> acc;
  double nrm = 0.0;
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row0 = tile * tm.R;
    const long long row = row0 + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    const int rows = (int)min((long long)tm.R, a.nrows - row0);
    __syncthreads();
    if (valid) {
      const cpx<T> m = a.v[e];
      sm.t0[threadIdx.x] = a.rt[e];
      sm.t1[threadIdx.x] = m;
      nrm += abs2(m);
    }
    __syncthreads();
    acc.add(sm.t0, sm.t1, rows, L);
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  acc.store(out, L);
  if (a.want_norms) column_store(nrm, sm.red, out + 2 * L * L, L, tm.nact);
}

// ------------------------------------------------------------------ BiCGGR, QR frame
// The residual is carried as R_k = Q_k xi_k with Q_k orthonormal (N x L,
// precision T) and xi_k an FP64 L x L factor; P, V, W, U, Y are kept in the
// same frame.  The iterates equal those of the listing in exact arithmetic.

// X += (zeta Q + U) xi;  T = Q - zeta W - Y (into the Q block);
// partials: T^H T (L^2), R~0^H T (L^2)
template <typename T, int NE>
__global__ void __launch_bounds__(kBT) k_ggrq_xr(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  load_matrix(sm.M1, a.m1, L);
  const cpx<T> z = cast<T>(a.zeta[0]);
  Gram<T, NE> acc1, acc2;
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row0 = tile * tm.R;
    const long long row = row0 + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    const int rows = (int)min((long long)tm.R, a.nrows - row0);
    __syncthreads();
    if (valid) {
      const cpx<T> q = a.r[e];
      sm.t0[threadIdx.x] = z * q + a.u[e];
      const cpx<T> t = q - z * a.w[e] - a.y[e];
      a.r[e] = t;
      sm.t1[threadIdx.x] = t;
      sm.t2[threadIdx.x] = a.rt[e];
    }
    __syncthreads();
    if (valid) a.x[e] = a.x[e] + row_product(sm.t0, sm.M1, tm.rl, tm.j, L);
    acc1.add(sm.t1, sm.t1, rows, L);
    acc2.add(sm.t2, sm.t1, rows, L);
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  acc1.store(out, L);
  acc2.store(out + 2 * L * L, L);
}

// Q = T tau^-1 (in place);  W = W' tau^-1 (in place);  P = Q + U gamma;
// V = W + Y gamma;  partials: R~0^H V, W^H Q, W^H W (L^2 each)
template <typename T, int NE>
__global__ void __launch_bounds__(kBT) k_ggrq_pv(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  load_matrix(sm.M1, a.m1, L);
  load_matrix(sm.M2, a.m2, L);
  Gram<T, NE> acc1, acc2, acc3;
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row0 = tile * tm.R;
    const long long row = row0 + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    const int rows = (int)min((long long)tm.R, a.nrows - row0);
    __syncthreads();
    if (valid) {
      sm.t0[threadIdx.x] = a.r[e];
      sm.t1[threadIdx.x] = a.w[e];
      sm.t2[threadIdx.x] = a.u[e];
      sm.t3[threadIdx.x] = a.y[e];
      sm.t4[threadIdx.x] = a.rt[e];
    }
    __syncthreads();
    cpx<T> q = mk(T(0), T(0)), w = q, v = q;
    if (valid) {
      q = row_product(sm.t0, sm.M1, tm.rl, tm.j, L);
      w = row_product(sm.t1, sm.M1, tm.rl, tm.j, L);
      const cpx<T> p = q + row_product(sm.t2, sm.M2, tm.rl, tm.j, L);
      v = w + row_product(sm.t3, sm.M2, tm.rl, tm.j, L);
      a.r[e] = q;
      a.w[e] = w;
      a.p[e] = p;
      a.v[e] = v;
    }
    __syncthreads();
    if (valid) {
      sm.t0[threadIdx.x] = q;
      sm.t1[threadIdx.x] = w;
      sm.t2[threadIdx.x] = v;
    }
    __syncthreads();
    acc1.add(sm.t4, sm.t2, rows, L);
    acc2.add(sm.t1, sm.t0, rows, L);
    acc3.add(sm.t1, sm.t1, rows, L);
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  acc1.store(out, L);
  acc2.store(out + 2 * L * L, L);
  acc3.store(out + 4 * L * L, L);
}

// Two Gram matrices: partials A1^H B1, A2^H B2 (a.rt/a.v and a.w/a.r)
template <typename T, int NE>
__global__ void __launch_bounds__(kBT) k_gram2(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int L = a.L;
  Smem<T> sm = carve<T>(smem_raw, L);
  TileMap<T> tm(L);
  Gram<T, NE> acc1, acc2;
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row0 = tile * tm.R;
    const long long row = row0 + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    const int rows = (int)min((long long)tm.R, a.nrows - row0);
    __syncthreads();
    if (valid) {
      sm.t0[threadIdx.x] = a.rt[e];
      sm.t1[threadIdx.x] = a.v[e];
      sm.t2[threadIdx.x] = a.w[e];
      sm.t3[threadIdx.x] = a.r[e];
    }
    __syncthreads();
    acc1.add(sm.t0, sm.t1, rows, L);
    acc2.add(sm.t2, sm.t3, rows, L);
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  acc1.store(out, L);
  acc2.store(out + 2 * L * L, L);
}

// ------------------------------------------------------------------ small-L kernels
// For L <= 16 every thread (row slot rl, column j) keeps column j of the
// L x L coefficient matrices in registers and accumulates column j of each
// Gram matrix over the rows it visits (LB >= L accumulators); one LDS
// reduction over the row slots runs at the end.  The per-thread partial sums
// are in the accumulator type A (FP32 for FP32 blocks: each thread adds at
// most a few hundred terms), the workgroup and grid sums in FP64.

template <typename T>
struct AccT;
template <>
struct AccT<float> {
  using type = float;
};
template <>
struct AccT<double> {
  using type = double;
};

template <typename T, int LB>
__device__ __forceinline__ void load_column(cpx<T> col[LB], const cpx<double>* __restrict__ M, int L, int j) {
#pragma unroll
  for (int i = 0; i < LB; ++i) col[i] = (i < L) ? cast<T>(M[i * L + j]) : mk(T(0), T(0));
}

// The LDS row tiles of the small-L kernels have a compile-time row stride
// LB >= L; the entries of a row past L are zero (set once at kernel start,
// never written afterwards), and so are the entries of the coefficient
// columns past L.  The unrolled loops below then run over all LB entries
// with no per-entry branch, and the padding adds zeros.
template <int LB>
struct SmallTile {
  // most rows a tile can hold: 256 / L with L > LB - 4 (L >= 1 for LB = 4)
  static constexpr int rows = LB == 4 ? kBT : kBT / (LB - 3);
  static constexpr int size = rows * LB;
};

template <typename T, int LB>
__device__ __forceinline__ void zero_tile(cpx<T>* t) {
  for (int e = threadIdx.x; e < SmallTile<LB>::size; e += kBT) t[e] = mk(T(0), T(0));
}

// sum_i S[rl][i] col[i]
template <typename T, int LB>
__device__ __forceinline__ cpx<T> row_col(const cpx<T>* sS, const cpx<T> col[LB], int rl) {
  cpx<T> acc = mk(T(0), T(0));
  const cpx<T>* srow = sS + rl * LB;
#pragma unroll
  for (int i = 0; i < LB; ++i) cmac(acc, srow[i], col[i]);
  return acc;
}

// g[i] += conj(S[rl][i]) * b
template <typename T, typename A, int LB>
__device__ __forceinline__ void gram_col(cpx<A> g[LB], const cpx<T>* sS, cpx<T> b, int rl) {
  const cpx<T>* srow = sS + rl * LB;
  const cpx<A> bb = cast<A>(b);
#pragma unroll
  for (int i = 0; i < LB; ++i) cmac_conj(g[i], cast<A>(srow[i]), bb);
}

// Write column sums of g over the row slots: out[2*(i*L + j)] (re, im), FP64.
template <typename A, int LB>
__device__ __forceinline__ void gram_col_store(const cpx<A> g[LB], cpx<double>* red, double* out, int L, int R) {
  const int rl = threadIdx.x / L, j = threadIdx.x - (threadIdx.x / L) * L;
  const bool act = rl < R;
#pragma unroll
  for (int i = 0; i < LB; ++i) {
    // i < L is uniform over the workgroup
    if (i < L) {
      __syncthreads();
      red[threadIdx.x] = act ? cast<double>(g[i]) : mk(0.0, 0.0);
      __syncthreads();
      if ((int)threadIdx.x < L) {
        cpx<double> s = mk(0.0, 0.0);
        for (int r = 0; r < R; ++r) s = s + red[r * L + threadIdx.x];
        out[2 * (i * L + threadIdx.x)] = s.re;
        out[2 * (i * L + threadIdx.x) + 1] = s.im;
      }
    }
  }
}

// U = (P - zeta V) alpha
template <typename T, int LB>
__global__ void __launch_bounds__(kBT) k_s_bicggr_u(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  __shared__ cpx<T> t0[SmallTile<LB>::size];
  const int L = a.L;
  TileMap<T> tm(L);
  zero_tile<T, LB>(t0);
  cpx<T> m1[LB];
  load_column<T, LB>(m1, a.m1, L, tm.j);
  const cpx<T> z = cast<T>(a.zeta[0]);
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * tm.R + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    cpx<T> pv = mk(T(0), T(0));
    if (valid) pv = a.p[e] - z * a.v[e];
    __syncthreads();
    if (tm.act) t0[tm.rl * LB + tm.j] = pv;
    __syncthreads();
    if (valid) a.u[e] = row_col<T, LB>(t0, m1, tm.rl);
  }
}

// QR frame: X += (zeta Q + U) xi;  T = Q - zeta W - Y (into Q);  [T^H T, R~0^H T]
template <typename T, int LB>
__global__ void __launch_bounds__(kBT) k_s_ggrq_xr(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  using A = typename AccT<T>::type;
  __shared__ cpx<T> t0[SmallTile<LB>::size], t1[SmallTile<LB>::size], t2[SmallTile<LB>::size];
  __shared__ cpx<double> red[kBT];
  const int L = a.L;
  TileMap<T> tm(L);
  zero_tile<T, LB>(t0);
  zero_tile<T, LB>(t1);
  zero_tile<T, LB>(t2);
  cpx<T> xi[LB];
  load_column<T, LB>(xi, a.m1, L, tm.j);
  const cpx<T> z = cast<T>(a.zeta[0]);
  cpx<A> g1[LB], g2[LB];
#pragma unroll
  for (int i = 0; i < LB; ++i) g1[i] = g2[i] = mk(A(0), A(0));
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * tm.R + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    cpx<T> s = mk(T(0), T(0)), t = s, rt = s;
    if (valid) {
      const cpx<T> q = a.r[e];
      s = z * q + a.u[e];
      t = q - z * a.w[e] - a.y[e];
      rt = a.rt[e];
      a.r[e] = t;
    }
    __syncthreads();
    if (tm.act) t0[tm.rl * LB + tm.j] = s;
    if (tm.act) t1[tm.rl * LB + tm.j] = t;
    if (tm.act) t2[tm.rl * LB + tm.j] = rt;
    __syncthreads();
    if (valid) {
      a.x[e] = a.x[e] + row_col<T, LB>(t0, xi, tm.rl);
      gram_col<T, A, LB>(g1, t1, t, tm.rl);
      gram_col<T, A, LB>(g2, t2, t, tm.rl);
    }
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  gram_col_store<A, LB>(g1, red, out, L, tm.R);
  gram_col_store<A, LB>(g2, red, out + 2 * L * L, L, tm.R);
}

// QR frame: Q = T tau^-1;  W = W' tau^-1;  P = Q + U gamma;  V = W + Y gamma;
// [R~0^H V, W^H Q, W^H W]
template <typename T, int LB>
__global__ void __launch_bounds__(kBT) k_s_ggrq_pv(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  using A = typename AccT<T>::type;
  __shared__ cpx<T> t0[SmallTile<LB>::size], t1[SmallTile<LB>::size], t2[SmallTile<LB>::size],
      t3[SmallTile<LB>::size], t4[SmallTile<LB>::size];
  __shared__ cpx<double> red[kBT];
  const int L = a.L;
  TileMap<T> tm(L);
  zero_tile<T, LB>(t0);
  zero_tile<T, LB>(t1);
  zero_tile<T, LB>(t2);
  zero_tile<T, LB>(t3);
  zero_tile<T, LB>(t4);
  cpx<T> m1[LB], m2[LB];
  load_column<T, LB>(m1, a.m1, L, tm.j);
  load_column<T, LB>(m2, a.m2, L, tm.j);
  cpx<A> g1[LB], g2[LB], g3[LB];
#pragma unroll
  for (int i = 0; i < LB; ++i) g1[i] = g2[i] = g3[i] = mk(A(0), A(0));
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * tm.R + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    cpx<T> vt = mk(T(0), T(0)), vw = vt, vu = vt, vy = vt, vr = vt;
    if (valid) {
      vt = a.r[e];
      vw = a.w[e];
      vu = a.u[e];
      vy = a.y[e];
      vr = a.rt[e];
    }
    __syncthreads();
    if (tm.act) t0[tm.rl * LB + tm.j] = vt;
    if (tm.act) t1[tm.rl * LB + tm.j] = vw;
    if (tm.act) t2[tm.rl * LB + tm.j] = vu;
    if (tm.act) t3[tm.rl * LB + tm.j] = vy;
    if (tm.act) t4[tm.rl * LB + tm.j] = vr;
    __syncthreads();
    cpx<T> q = mk(T(0), T(0)), w = q, v = q;
    if (valid) {
      q = row_col<T, LB>(t0, m1, tm.rl);
      w = row_col<T, LB>(t1, m1, tm.rl);
      const cpx<T> p = q + row_col<T, LB>(t2, m2, tm.rl);
      v = w + row_col<T, LB>(t3, m2, tm.rl);
      a.r[e] = q;
      a.w[e] = w;
      a.p[e] = p;
      a.v[e] = v;
      gram_col<T, A, LB>(g1, t4, v, tm.rl);
    }
    __syncthreads();
    if (tm.act) t1[tm.rl * LB + tm.j] = w;
    __syncthreads();
    if (valid) {
      gram_col<T, A, LB>(g2, t1, q, tm.rl);
      gram_col<T, A, LB>(g3, t1, w, tm.rl);
    }
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  gram_col_store<A, LB>(g1, red, out, L, tm.R);
  gram_col_store<A, LB>(g2, red, out + 2 * L * L, L, tm.R);
  gram_col_store<A, LB>(g3, red, out + 4 * L * L, L, tm.R);
}


// ------------------------------------------------------------------ fused QR frame (L <= kSmallL)
// The QR-frame iteration with P = Q + U_{k-1} gamma_{k-1} and
// V = W + Y_{k-1} gamma_{k-1} never formed, and Q = T tau^-1, W = W' tau^-1
// kept as the raw blocks T and W' = A T with tau^-1 folded into the
// coefficient matrices (16 block passes per iteration instead of 20).

// U = (T - zeta W') m1 + (U - zeta Y) m2, in place
template <typename T, int LB>
__global__ void __launch_bounds__(kBT) k_s_fu(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  __shared__ cpx<T> t0[SmallTile<LB>::size], t1[SmallTile<LB>::size];
  const int L = a.L;
  TileMap<T> tm(L);
  zero_tile<T, LB>(t0);
  zero_tile<T, LB>(t1);
  cpx<T> m1[LB], m2[LB];
  load_column<T, LB>(m1, a.m1, L, tm.j);
  load_column<T, LB>(m2, a.m2, L, tm.j);
  const cpx<T> z = cast<T>(a.zeta[0]);
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * tm.R + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    cpx<T> d1 = mk(T(0), T(0)), d2 = d1;
    if (valid) {
      d1 = a.r[e] - z * a.w[e];
      d2 = a.u[e] - z * a.y[e];
    }
    __syncthreads();
    if (tm.act) {
      t0[tm.rl * LB + tm.j] = d1;
      t1[tm.rl * LB + tm.j] = d2;
    }
    __syncthreads();
    if (valid) a.u[e] = row_col<T, LB>(t0, m1, tm.rl) + row_col<T, LB>(t1, m2, tm.rl);
  }
}

// X += T m1 + U m2;  T_new = (T - zeta W') m3 - Y (in place);
// [T_new^H T_new, R~0^H T_new, R~0^H Y]
template <typename T, int LB>
__global__ void __launch_bounds__(kBT) k_s_fxr(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  using A = typename AccT<T>::type;
  __shared__ cpx<T> t0[SmallTile<LB>::size], t1[SmallTile<LB>::size], t2[SmallTile<LB>::size],
      t3[SmallTile<LB>::size];
  __shared__ cpx<double> red[kBT];
  const int L = a.L;
  TileMap<T> tm(L);
  zero_tile<T, LB>(t0);
  zero_tile<T, LB>(t1);
  zero_tile<T, LB>(t2);
  zero_tile<T, LB>(t3);
  cpx<T> m1[LB], m2[LB], m3[LB];
  load_column<T, LB>(m1, a.m1, L, tm.j);
  load_column<T, LB>(m2, a.m2, L, tm.j);
  load_column<T, LB>(m3, a.m3, L, tm.j);
  const cpx<T> z = cast<T>(a.zeta[0]);
  cpx<A> g1[LB], g2[LB], g3[LB];
#pragma unroll
  for (int i = 0; i < LB; ++i) g1[i] = g2[i] = g3[i] = mk(A(0), A(0));
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * tm.R + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    cpx<T> vt = mk(T(0), T(0)), vu = vt, d = vt, vy = vt, vr = vt;
    if (valid) {
      vt = a.r[e];
      vu = a.u[e];
      d = vt - z * a.w[e];
      vy = a.y[e];
      vr = a.rt[e];
    }
    __syncthreads();
    if (tm.act) {
      t0[tm.rl * LB + tm.j] = vt;
      t1[tm.rl * LB + tm.j] = vu;
      t2[tm.rl * LB + tm.j] = d;
      t3[tm.rl * LB + tm.j] = vr;
    }
    __syncthreads();
    cpx<T> tn = mk(T(0), T(0));
    if (valid) {
      a.x[e] = a.x[e] + row_col<T, LB>(t0, m1, tm.rl) + row_col<T, LB>(t1, m2, tm.rl);
      tn = row_col<T, LB>(t2, m3, tm.rl) - vy;
      a.r[e] = tn;
      gram_col<T, A, LB>(g2, t3, tn, tm.rl);
      gram_col<T, A, LB>(g3, t3, vy, tm.rl);
    }
    __syncthreads();
    if (tm.act) t0[tm.rl * LB + tm.j] = tn;
    __syncthreads();
    if (valid) gram_col<T, A, LB>(g1, t0, tn, tm.rl);
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
  gram_col_store<A, LB>(g1, red, out, L, tm.R);
  gram_col_store<A, LB>(g2, red, out + 2 * L * L, L, tm.R);
  gram_col_store<A, LB>(g3, red, out + 4 * L * L, L, tm.R);
}

// [gl0^H gr, gl1^H gr, gl2^H gr] (the first ng of them)
template <typename T, int LB, int NG>
__device__ __forceinline__ void fgram_body(const BlasArgs<T>& a) {
  using A = typename AccT<T>::type;
  __shared__ cpx<T> tl[NG][SmallTile<LB>::size];
  __shared__ cpx<double> red[kBT];
  const int L = a.L;
  TileMap<T> tm(L);
#pragma unroll
  for (int q = 0; q < NG; ++q) zero_tile<T, LB>(tl[q]);
  cpx<A> g[NG][LB];
#pragma unroll
  for (int q = 0; q < NG; ++q)
#pragma unroll
    for (int i = 0; i < LB; ++i) g[q][i] = mk(A(0), A(0));
  const long long ntiles = (a.nrows + tm.R - 1) / tm.R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * tm.R + tm.rl;
    const bool valid = tm.act && row < a.nrows;
    const long long e = row * L + tm.j;
    cpx<T> vl[NG], vr = mk(T(0), T(0));
#pragma unroll
    for (int q = 0; q < NG; ++q) vl[q] = mk(T(0), T(0));
    if (valid) {
#pragma unroll
      for (int q = 0; q < NG; ++q) vl[q] = a.gl[q][e];
      vr = a.gr[e];
    }
    __syncthreads();
    if (tm.act) {
#pragma unroll
      for (int q = 0; q < NG; ++q) tl[q][tm.rl * LB + tm.j] = vl[q];
    }
    __syncthreads();
    if (valid) {
#pragma unroll
      for (int q = 0; q < NG; ++q) gram_col<T, A, LB>(g[q], tl[q], vr, tm.rl);
    }
  }
  double* out = a.partials + (long long)blockIdx.x * a.nv;
#pragma unroll
  for (int q = 0; q < NG; ++q) gram_col_store<A, LB>(g[q], red, out + 2 * q * L * L, L, tm.R);
}

template <typename T, int LB>
__global__ void __launch_bounds__(kBT) k_s_fgram2(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  fgram_body<T, LB, 2>(a);
}

template <typename T, int LB>
__global__ void __launch_bounds__(kBT) k_s_fgram3(BlasArgs<T> a) {
  if (!running<T>(a.ctl)) return;
  fgram_body<T, LB, 3>(a);
}

// ------------------------------------------------------------------ fused QR frame, FP32, 8 columns
// Lane-per-real kernels for 8-column FP32 blocks.  One row of a block is 8
// complex = 16 floats = 64 bytes, and the 16 lanes of a DPP row hold the 16
// reals of one block row (lane m = 2 j + part: column j, real or imaginary
// part).  A wave covers 4 rows with one dword per lane, so a tile of 16 rows
// is 4 registers per block, each register one contiguous 256-byte run.
//
// * (N x 8)(8 x 8) row products: lane m forms sum_{m'} S[m'] M'[m'][m] with
//   M' the real 16 x 16 form of the complex 8 x 8 matrix.  S[m'] comes from
//   the other lanes of the DPP row by row_ror rotations; the coefficient a
//   lane needs for rotation k is M'[source lane][m], and the source lane is
//   found by rotating the lane index itself, so no lane order is assumed.
// * Gram matrices A^H B: one v_mfma_f32_16x16x4f32 per register pair; the
//   instruction's K = 4 runs over the 4 rows held by the register (lanes
//   16 k .. 16 k + 15 hold row k of both operands), so it accumulates the
//   real product P = A'^T B' (16 x 16) whose 2 x 2 blocks give
//   (A^H B)[a][b] = (P[2a][2b] + P[2a+1][2b+1]) + i (P[2a][2b+1] - P[2a+1][2b]).
//   Which (i, j) of P each lane's accumulator registers hold is found at run
//   time with two MFMAs on index-coded operands.  The FP32 accumulators are
//   added into FP64 every kL8Flush tiles.
// * No LDS and no barrier in the row loop; the workgroup's four waves sum
//   their FP64 P in LDS at the end, in a fixed order.


template <int K>
__device__ __forceinline__ float l8_ror(float v) {
  if constexpr (K == 0) return v;
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x120 + K, 0xf, 0xf,
                                                                   true));
}

template <int K>
__device__ __forceinline__ int l8_ror_i(int v) {
  if constexpr (K == 0) return v;
  else return __builtin_amdgcn_update_dpp(0, v, 0x120 + K, 0xf, 0xf, true);
}

// value of the partner lane (re <-> im of the same complex entry)
__device__ __forceinline__ float l8_swap_pair(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xf, 0xf, true));
}

// Real 16 x 16 form of a complex 8 x 8 matrix M (row-major, FP64), written
// to LDS by the whole workgroup: M'[2i + q][2j + p] is Re M[i][j] for
// q = p, Im M[i][j] for (q, p) = (0, 1) and -Im M[i][j] for (1, 0).
__device__ __forceinline__ void l8_stage_mreal(const cpx<double>* __restrict__ M, float* __restrict__ sm) {
  const int e = threadIdx.x;  // 256 threads, one entry each
  const int mp = e >> 4, m = e & 15;
  const cpx<double> v = M[(mp >> 1) * 8 + (m >> 1)];
  const int q = mp & 1, p = m & 1;
  sm[e] = (float)(q == p ? v.re : (q == 0 ? v.im : -v.im));
}

struct L8Coef {
  float c[16];
};

// coefficient of rotation step K for lane part m: M'[source lane][m], where
// the source lane after K single-lane rotations is found by rotating the
// lane index the same way (no assumption on the rotation's direction)
__device__ __forceinline__ void l8_load_coef(L8Coef& cf, const float* __restrict__ sm, int m) {
  int src = m;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    cf.c[k] = sm[src * 16 + m];
    src = l8_ror_i<1>(src);
  }
}

// the NM coefficient matrices of a kernel, through LDS
template <int NM>
__device__ __forceinline__ void l8_load_coefs(L8Coef (&cf)[NM], const cpx<double>* const (&M)[NM], int m) {
  __shared__ float sm[NM][256];
#pragma unroll
  for (int k = 0; k < NM; ++k) l8_stage_mreal(M[k], sm[k]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NM; ++k) l8_load_coef(cf[k], sm[k], m);
}

// acc + sum_k S[source lane k] M'[source lane k][m]: the row product, one
// single-lane rotation per step
__device__ __forceinline__ float l8_prod(float s, const L8Coef& cf, float acc) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    acc = __builtin_fmaf(s, cf.c[k], acc);
    if (k < 15) s = l8_ror<1>(s);
  }
  return acc;
}

// z * v for the complex scalar z: lane part p holds Re (p = 0) or Im (p = 1)
struct L8Scalar {
  float re, im_signed;  // im_signed = -Im z on real lanes, +Im z on imaginary lanes
};

__device__ __forceinline__ float l8_scale(float v, const L8Scalar& z) {
  return z.re * v + z.im_signed * l8_swap_pair(v);
}

constexpr int kL8Flush = 16;  // tiles between FP64 flushes of the Gram accumulators

// FP32 MFMA accumulator of one Gram and its FP64 running sum, which lives in
// the workgroup's LDS (each lane owns its 4 entries: no synchronisation).
struct L8Gram {
  f32x4 acc;
  double* d;  // LDS, 4 doubles of this lane
};

__device__ __forceinline__ void l8_gram_init(L8Gram& g, double* lane_slot) {
  g.acc = f32x4{0.f, 0.f, 0.f, 0.f};
  g.d = lane_slot;
#pragma unroll
  for (int v = 0; v < 4; ++v) g.d[v] = 0.0;
}

__device__ __forceinline__ void l8_gram_add(L8Gram& g, float a, float b) {
  g.acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, g.acc, 0, 0, 0);
}

__device__ __forceinline__ void l8_gram_flush(L8Gram& g) {
#pragma unroll
  for (int v = 0; v < 4; ++v) g.d[v] += (double)g.acc[v];
  g.acc = f32x4{0.f, 0.f, 0.f, 0.f};
}

// LDS of the Gram kernels: FP64 running sums [wave][gram][lane][4], reused by
// the final sum as [wave][gram][16 x 16]
template <int NG>
struct L8Smem {
  double d[4][NG][256];
};

template <int NG>
__device__ __forceinline__ void l8_grams_init(L8Gram (&g)[NG], L8Smem<NG>& sm) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < NG; ++q) l8_gram_init(g[q], &sm.d[w][q][4 * lane]);
}

// Sum the NG Grams of the workgroup's waves (fixed order) and write the
// complex 8 x 8 results at out[q * 128 + 2 (a * 8 + b)] (re, im).
template <int NG>
__device__ __forceinline__ void l8_gram_store(L8Gram (&g)[NG], L8Smem<NG>& sm, const L8Layout& ly,
                                              double* __restrict__ out) {
  const int w = threadIdx.x >> 6;
  double vals[NG][4];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    l8_gram_flush(g[q]);
#pragma unroll
    for (int v = 0; v < 4; ++v) vals[q][v] = g[q].d[v];
  }
  // every lane has read its own running sums before any is overwritten
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NG; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) sm.d[w][q][ly.i[v] * 16 + ly.j[v]] = vals[q][v];
  __syncthreads();
  const double (*P)[NG][256] = sm.d;
  for (int e = threadIdx.x; e < NG * 64; e += kBT) {
    const int q = e >> 6, a = (e >> 3) & 7, b = e & 7;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) {
      const double* p = P[ww][q];
      re += p[(2 * a) * 16 + 2 * b] + p[(2 * a + 1) * 16 + 2 * b + 1];
      im += p[(2 * a) * 16 + 2 * b + 1] - p[(2 * a + 1) * 16 + 2 * b];
    }
    out[q * 128 + 2 * (a * 8 + b)] = re;
    out[q * 128 + 2 * (a * 8 + b) + 1] = im;
  }
}

// Row walk of the lane-per-real kernels: wave w of workgroup b takes the
// 16-row tiles b * 4 + w, + 4 * gridDim.x, ...; group q of the wave (one
// register of rows) is rows 16 t + 4 (q % 4) + lane / 16 of its (q / 4)-th
// tile, lane part m = lane % 16.  The next group's loads are issued before
// the current group is computed.
struct L8Walk {
  long long nrows, tile0, stride;
  int g, m, ngroups;
  __device__ __forceinline__ explicit L8Walk(long long nrows_) : nrows(nrows_) {
    const int lane = threadIdx.x & 63;
    g = lane >> 4;
    m = lane & 15;
    tile0 = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    stride = (long long)gridDim.x * 4;
    const long long ntiles = (nrows + 15) / 16;
    ngroups = tile0 < ntiles ? (int)(4 * ((ntiles - tile0 + stride - 1) / stride)) : 0;
  }
  __device__ __forceinline__ long long row(int q) const { return (tile0 + (q >> 2) * stride) * 16 + 4 * (q & 3) + g; }
};

// one value per lane of NB blocks at a row; rows past the end read the last
// row (always in bounds) and are zeroed
template <int NB>
struct L8Vals {
  float v[NB];
};

template <int NB>
__device__ __forceinline__ L8Vals<NB> l8_load(const cpx<float>* const (&p)[NB], long long row, const L8Walk& wk) {
  const long long r = row < wk.nrows ? row : wk.nrows - 1;
  const long long off = r * 16 + wk.m;
  L8Vals<NB> o;
#pragma unroll
  for (int b = 0; b < NB; ++b) o.v[b] = reinterpret_cast<const float*>(p[b])[off];
  return o;
}

template <int NB>
__device__ __forceinline__ void l8_mask(L8Vals<NB>& o, bool ok) {
#pragma unroll
  for (int b = 0; b < NB; ++b) o.v[b] = ok ? o.v[b] : 0.f;
}

__device__ __forceinline__ void l8_st(cpx<float>* p, long long row, int m, bool ok, float v) {
  if (ok) reinterpret_cast<float*>(p)[row * 16 + m] = v;
}

__device__ __forceinline__ L8Scalar l8_zeta(const cpx<double>* zeta, int m) {
  const cpx<double> z = zeta[0];
  return L8Scalar{(float)z.re, (float)((m & 1) ? z.im : -z.im)};
}

// Streams the wave's groups through body(vals, row, ok) with loads issued
// ahead: TILE = false keeps the next DEPTH (1 or 2) 4-row groups in flight
// (the update kernels, whose registers hold coefficient matrices), TILE =
// true the next whole tile of 4 groups (the Gram pass, which has registers
// to spare).  Every kL8Flush tiles it calls flush().
template <int NB, bool TILE, int DEPTH = 1, class Body, class Flush>
__device__ __forceinline__ void l8_stream(const L8Walk& wk, const cpx<float>* const (&p)[NB], Body body, Flush flush) {
  if (wk.ngroups == 0) return;
  if constexpr (TILE) {
    const int nt = wk.ngroups >> 2;
    L8Vals<NB> cur[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) cur[v] = l8_load<NB>(p, wk.row(v), wk);
    for (int t = 0; t < nt; ++t) {
      const int tn = t + 1 < nt ? t + 1 : t;
      L8Vals<NB> nxt[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) nxt[v] = l8_load<NB>(p, wk.row(4 * tn + v), wk);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long long row = wk.row(4 * t + v);
        const bool ok = row < wk.nrows;
        l8_mask<NB>(cur[v], ok);
        body(cur[v], row, ok);
      }
      if (t % kL8Flush == kL8Flush - 1) flush();
#pragma unroll
      for (int v = 0; v < 4; ++v) cur[v] = nxt[v];
    }
  } else {
    static_assert(DEPTH == 1 || DEPTH == 2, "one or two groups ahead");
    L8Vals<NB> cur = l8_load<NB>(p, wk.row(0), wk);
    L8Vals<NB> nx1;
    if constexpr (DEPTH == 2) nx1 = l8_load<NB>(p, wk.row(1 < wk.ngroups ? 1 : 0), wk);
    for (int q = 0; q < wk.ngroups; ++q) {
      // the last group is loaded again past the end (in bounds, unused)
      const int qn = q + DEPTH < wk.ngroups ? q + DEPTH : wk.ngroups - 1;
      const L8Vals<NB> nxt = l8_load<NB>(p, wk.row(qn), wk);
      const long long row = wk.row(q);
      const bool ok = row < wk.nrows;
      l8_mask<NB>(cur, ok);
      body(cur, row, ok);
      if ((q & (4 * kL8Flush - 1)) == 4 * kL8Flush - 1) flush();
      if constexpr (DEPTH == 2) {
        cur = nx1;
        nx1 = nxt;
      } else {
        cur = nxt;
      }
    }
  }
}

// U_new = (T - zeta W') m1 + (U - zeta Y) m2;  X += T m3 + U_new m4
// (the solution update of the iteration, done where T and the new U are in
// registers, so that the X/R pass no longer reads U and X)
__global__ void __launch_bounds__(kBT) k_l8_fux(BlasArgs<float> a) {
  if (!running<float>(a.ctl)) return;
  const L8Walk wk(a.nrows);
  L8Coef cf[4];
  l8_load_coefs<4>(cf, {a.m1, a.m2, a.m3, a.m4}, wk.m);
  const L8Scalar z = l8_zeta(a.zeta, wk.m);
  const cpx<float>* const src[5] = {a.r, a.w, a.u, a.y, a.x};
  l8_stream<5, false>(wk, src, [&](const L8Vals<5>& c, long long row, bool ok) {
    const float tv = c.v[0];
    const float d1 = tv - l8_scale(c.v[1], z);
    const float d2 = c.v[2] - l8_scale(c.v[3], z);
    const float un = l8_prod(d2, cf[1], l8_prod(d1, cf[0], 0.f));
    const float xn = l8_prod(un, cf[3], l8_prod(tv, cf[2], c.v[4]));
    l8_st(a.u, row, wk.m, ok, un);
    l8_st(a.x, row, wk.m, ok, xn);
  }, [] {});
}

// T_new = (T - zeta W') m3 - Y (in place); [T_new^H T_new, R~0^H T_new, R~0^H Y]
__global__ void __launch_bounds__(kBT) k_l8_fxrt(BlasArgs<float> a) {
  if (!running<float>(a.ctl)) return;
  const L8Walk wk(a.nrows);
  const L8Layout ly = l8_layout();
  L8Coef cf[1];
  l8_load_coefs<1>(cf, {a.m3}, wk.m);
  const L8Scalar z = l8_zeta(a.zeta, wk.m);
  __shared__ L8Smem<3> sm;
  L8Gram g[3];
  l8_grams_init<3>(g, sm);
  const cpx<float>* const src[4] = {a.r, a.w, a.y, a.rt};
  // two groups ahead (one ahead measured 4 % slower here; in k_l8_fux, whose
  // coefficient registers leave none to spare, two ahead was 4 % slower)
  l8_stream<4, false, 2>(wk, src, [&](const L8Vals<4>& c, long long row, bool ok) {
    const float tv = c.v[0], wv = c.v[1], yv = c.v[2], rtv = c.v[3];
    const float tn = l8_prod(tv - l8_scale(wv, z), cf[0], -yv);
    l8_st(a.r, row, wk.m, ok, tn);
    l8_gram_add(g[0], tn, tn);
    l8_gram_add(g[1], rtv, tn);
    l8_gram_add(g[2], rtv, yv);
  }, [&] {
#pragma unroll
    for (int q = 0; q < 3; ++q) l8_gram_flush(g[q]);
  });
  l8_gram_store<3>(g, sm, ly, a.partials + (long long)blockIdx.x * a.nv);
}

// [gl0^H gr, gl1^H gr, gl2^H gr] (the first NG of them)
template <int NG>
__global__ void __launch_bounds__(kBT) k_l8_fgram(BlasArgs<float> a) {
  if (!running<float>(a.ctl)) return;
  const L8Walk wk(a.nrows);
  const L8Layout ly = l8_layout();
  __shared__ L8Smem<NG> sm;
  L8Gram g[NG];
  l8_grams_init<NG>(g, sm);
  cpx<float> const* src[NG + 1];
#pragma unroll
  for (int q = 0; q < NG; ++q) src[q] = a.gl[q];
  src[NG] = a.gr;
  const cpx<float>* const (&srcc)[NG + 1] = src;
  l8_stream<NG + 1, true>(wk, srcc, [&](const L8Vals<NG + 1>& c, long long, bool) {
#pragma unroll
    for (int q = 0; q < NG; ++q) l8_gram_add(g[q], c.v[q], c.v[NG]);
  }, [&] {
#pragma unroll
    for (int q = 0; q < NG; ++q) l8_gram_flush(g[q]);
  });
  l8_gram_store<NG>(g, sm, ly, a.partials + (long long)blockIdx.x * a.nv);
}

// ------------------------------------------------------------------ reductions
// out[s][v] = sum over rows [s*rows_per, (s+1)*rows_per) of in[row][v], fixed order.
__global__ void __launch_bounds__(1024) k_reduce(const double* __restrict__ in, long long nrows, int nv,
                                                  int rows_per, double* __restrict__ out) {
  __shared__ double red[16][64];
  const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
  const int v = blockIdx.x * 64 + lane;
  const long long r0 = (long long)blockIdx.y * rows_per;
  const long long r1 = min(nrows, r0 + rows_per);
  double acc = 0.0;
  if (v < nv)
    for (long long r = r0 + slice; r < r1; r += 16) acc += in[r * nv + v];
  red[slice][lane] = acc;
  __syncthreads();
  if (slice == 0 && v < nv) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += red[k][lane];
    out[(long long)blockIdx.y * nv + v] = s;
  }
}

// ------------------------------------------------------------------ elementwise
template <typename T>
__global__ void k_gaussian(cpx<T>* out, long long n, unsigned long long seed) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // splitmix64 counter hash -> two uniforms -> Box-Muller
  auto mix = [](unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const unsigned long long h1 = mix(seed ^ (2ull * (unsigned long long)i));
  const unsigned long long h2 = mix(seed ^ (2ull * (unsigned long long)i + 1ull));
  const double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
  const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586 * u2;
  out[i] = mk((T)(rad * cos(ang)), (T)(rad * sin(ang)));
}

// Row r of a component-major block ([spin*3+colour][site][rhs]) is row
// site*12 + spin*3 + colour of the site-major (ABI) block.
__device__ __forceinline__ long long cm_to_sm_row(long long r, int vol) {
  const long long sc = r / vol;
  return (r - sc * vol) * 12 + sc;
}

// out (component-major)[e] = (To)(in (site-major) * scale[col])
template <typename To, typename Ti>
__global__ void k_scale_convert(const cpx<Ti>* __restrict__ in, cpx<To>* __restrict__ out,
                                const double* __restrict__ scale, long long n, int L, int vol) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long row = i / L;
  const int col = (int)(i - row * L);
  const double s = scale[col];
  const cpx<Ti> v = in[cm_to_sm_row(row, vol) * L + col];
  out[i] = mk((To)((double)v.re * s), (To)((double)v.im * s));
}

// x (site-major) += scale[col] * (double) e (component-major)
template <typename Ti>
__global__ void k_accumulate(cpx<double>* __restrict__ x, const cpx<Ti>* __restrict__ e,
                             const double* __restrict__ scale, long long n, int L, int vol) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long row = i / L;
  const int col = (int)(i - row * L);
  const double s = scale[col];
  const cpx<Ti> v = e[i];
  const long long o = cm_to_sm_row(row, vol) * L + col;
  cpx<double> xv = x[o];
  xv.re += s * (double)v.re;
  xv.im += s * (double)v.im;
  x[o] = xv;
}

// out (component-major) = (To) in (site-major)
template <typename To, typename Ti>
__global__ void k_convert(const cpx<Ti>* __restrict__ in, cpx<To>* __restrict__ out, long long n, int L, int vol) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long row = i / L;
  const int col = (int)(i - row * L);
  out[i] = cast<To>(in[cm_to_sm_row(row, vol) * L + col]);
}

// Columns c0 .. c0 + n - 1 of an nrows x L block <-> an nrows x n block.
__global__ void k_gather_cols(const cpx<double>* __restrict__ X, cpx<double>* __restrict__ x, long long nrows, int L,
                              int c0, int n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nrows * n) {
    const long long r = e / n;
    x[e] = X[r * L + c0 + (e - r * n)];
  }
}

__global__ void k_scatter_cols(cpx<double>* __restrict__ X, const cpx<double>* __restrict__ x, long long nrows, int L,
                               int c0, int n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nrows * n) {
    const long long r = e / n;
    X[r * L + c0 + (e - r * n)] = x[e];
  }
}

// ------------------------------------------------------------------ deflation
// dst (nrows x n, rows in the order of src) = columns idx[0..n) of src (nrows x L)
__global__ void k_gather_idx(const cpx<double>* __restrict__ src, cpx<double>* __restrict__ dst, long long nrows,
                             int L, const int* __restrict__ idx, int n) {
  const long long tot = nrows * n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const long long row = e / n;
    const int j = (int)(e - row * n);
    dst[e] = src[row * L + idx[j]];
  }
}

// out (site-major, nrows x Lout) += sign * in (nrows x Lin) M (Lin x Lout, FP64);
// CM: `in` is component-major (a Krylov block), else site-major
template <typename Ti, bool CM>
__global__ void k_rowmat_rect(const cpx<Ti>* __restrict__ in, cpx<double>* __restrict__ out,
                              const cpx<double>* __restrict__ M, double sign, long long nrows, int Lin, int Lout,
                              int vol) {
  const long long tot = nrows * Lout;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const long long row = e / Lout;  // site-major row of out
    const int k = (int)(e - row * Lout);
    long long rin = row;
    if constexpr (CM) {
      const long long site = row / 12, sc = row - site * 12;
      rin = sc * vol + site;
    }
    cpx<double> acc = mk(0.0, 0.0);
    for (int j = 0; j < Lin; ++j) cmac(acc, cast<double>(in[rin * Lin + j]), M[j * Lout + k]);
    out[e] = out[e] + sign * acc;
  }
}

// ------------------------------------------------------------------ even-odd blocks
// Position c of a compact block of parity p is site eo_pos_site(c, p) (Lx even).
__device__ __forceinline__ int eo_pos_site(int lx, int ly, int lz, int c, int p) {
  const int half = lx >> 1;
  const int r = c / half;
  const int k = c - r * half;
  const int y = r % ly;
  const int rz = r / ly;
  const int x = 2 * k + ((p + y + rz % lz + rz / lz) & 1);
  return x + lx * r;
}

// out (compact even, component-major)[(sc * Vh + c) * L + l] = (To) scale[l] * in (site-major)
template <typename To>
__global__ void k_eo_gather(const cpx<double>* __restrict__ in, cpx<To>* __restrict__ out,
                            const double* __restrict__ scale, int lx, int ly, int lz, int vh, int L) {
  const long long n = 12LL * vh * L;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int l = (int)(e % L);
    const long long q = e / L;
    const int c = (int)(q % vh);
    const int sc = (int)(q / vh);
    const int site = eo_pos_site(lx, ly, lz, c, 0);
    out[e] = cast<To>(scale[l] * in[((long long)site * 12 + sc) * L + l]);
  }
}

// out (site-major, even sites) = unscale[l] * in (compact even, component-major)
template <typename Ti>
__global__ void k_eo_scatter(const cpx<Ti>* __restrict__ in, cpx<double>* __restrict__ out,
                             const double* __restrict__ unscale, int lx, int ly, int lz, int vh, int L) {
  const long long n = 12LL * vh * L;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int l = (int)(e % L);
    const long long q = e / L;
    const int c = (int)(q % vh);
    const int sc = (int)(q / vh);
    const int site = eo_pos_site(lx, ly, lz, c, 0);
    out[((long long)site * 12 + sc) * L + l] = unscale[l] * cast<double>(in[e]);
  }
}

// Per-workgroup partial sums of Tr(Y^H X) (Re, Im) and Tr(Y^H Y), fixed
// order: the trace epilogue of the operator, for operators without one
template <typename T>
__global__ void __launch_bounds__(256) k_trace2(const cpx<T>* __restrict__ x, const cpx<T>* __restrict__ y, long long n,
                                                double* __restrict__ partials) {
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const cpx<double> xv = cast<double>(x[e]), yv = cast<double>(y[e]);
    e0 += yv.re * xv.re + yv.im * xv.im;
    e1 += yv.re * xv.im - yv.im * xv.re;
    e2 += yv.re * yv.re + yv.im * yv.im;
  }
  __shared__ double red[3][256];
  red[0][threadIdx.x] = e0;
  red[1][threadIdx.x] = e1;
  red[2][threadIdx.x] = e2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) partials[(long long)blockIdx.x * 4 + threadIdx.x] = threadIdx.x < 3 ? red[threadIdx.x][0] : 0.0;
}

// x += sign * w (FP64)
__global__ void k_axpy64(cpx<double>* __restrict__ x, const cpx<double>* __restrict__ w, double sign, long long n) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    x[e] = x[e] + sign * w[e];
}

// ------------------------------------------------------------------ row transforms
// out[row][j] (+)= sign * sum_i in[row][i] M[i][j]   (M: L x L, FP64).  Rows
// are enumerated in component-major order; PERM = 1: `in` is site-major,
// PERM = 2: `out` is site-major, PERM = 0: neither.
template <typename To, typename Ti, bool ACC, int PERM>
__global__ void __launch_bounds__(kBT) k_rowmat(const cpx<Ti>* __restrict__ in, cpx<To>* __restrict__ out,
                                                 const cpx<double>* __restrict__ M, double sign, long long nrows,
                                                 int L, int vol) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<double>* sM = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* sT = sM + L * L;
  for (int e = threadIdx.x; e < L * L; e += kBT) sM[e] = M[e];
  const int R = kBT / L, rl = threadIdx.x / L, j = threadIdx.x - (threadIdx.x / L) * L;
  const bool act = (int)threadIdx.x < R * L;
  const long long ntiles = (nrows + R - 1) / R;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long row = tile * R + rl;
    const bool valid = act && row < nrows;
    const long long e = row * L + j;
    const long long e_sm = (PERM != 0 && valid) ? cm_to_sm_row(row, vol) * L + j : e;
    __syncthreads();
    if (valid) sT[threadIdx.x] = cast<double>(in[PERM == 1 ? e_sm : e]);
    __syncthreads();
    if (valid) {
      cpx<double> acc = mk(0.0, 0.0);
      for (int i = 0; i < L; ++i) cmac(acc, sT[rl * L + i], sM[i * L + j]);
      acc = sign * acc;
      const long long eo = (PERM == 2) ? e_sm : e;
      if constexpr (ACC) out[eo] = cast<To>(cast<double>(out[eo]) + acc);
      else out[eo] = cast<To>(acc);
    }
  }
}

// ------------------------------------------------------------------ L x L solves
// Solve A X = B in place (A: L x L, B: L x nb, both in LDS, row-major) by
// Gauss-Jordan elimination with partial pivoting, FP64, one workgroup.
// Returns false (uniformly) if a pivot is zero, tiny relative to the
// matrix, or not finite.
__device__ bool solve_gj(cpx<double>* A, cpx<double>* B, int L, int nb, int* s_int, double* s_dbl) {
  const int t = threadIdx.x, nt = blockDim.x;
  // matrix scale for the pivot test
  if (t == 0) {
    double mx = 0.0;
    for (int e = 0; e < L * L; ++e) mx = fmax(mx, fabs(A[e].re) + fabs(A[e].im));
    s_dbl[0] = mx;
    s_int[1] = 1;
  }
  __syncthreads();
  const double thresh = s_dbl[0] * 64.0 * 2.220446049250313e-16;
  for (int k = 0; k < L; ++k) {
    if (t == 0) {
      int p = k;
      double best = -1.0;
      for (int r = k; r < L; ++r) {
        const double m = fabs(A[r * L + k].re) + fabs(A[r * L + k].im);
        if (m > best) { best = m; p = r; }
      }
      s_int[0] = p;
      if (!(best > thresh) || !isfinite(best)) s_int[1] = 0;
    }
    __syncthreads();
    if (!s_int[1]) return false;
    const int p = s_int[0];
    if (p != k) {
      for (int c = t; c < L + nb; c += nt) {
        if (c < L) { cpx<double> tmp = A[k * L + c]; A[k * L + c] = A[p * L + c]; A[p * L + c] = tmp; }
        else { const int cc = c - L; cpx<double> tmp = B[k * nb + cc]; B[k * nb + cc] = B[p * nb + cc]; B[p * nb + cc] = tmp; }
      }
    }
    __syncthreads();
    // normalise row k
    if (t == 0) {
      const cpx<double> piv = A[k * L + k];
      const double d = piv.re * piv.re + piv.im * piv.im;
      s_dbl[1] = piv.re / d;
      s_dbl[2] = -piv.im / d;
    }
    __syncthreads();
    const cpx<double> inv = mk(s_dbl[1], s_dbl[2]);
    for (int c = t; c < L + nb; c += nt) {
      if (c < L) { if (c > k) A[k * L + c] = A[k * L + c] * inv; }
      else B[k * nb + (c - L)] = B[k * nb + (c - L)] * inv;
    }
    __syncthreads();
    // eliminate column k from every other row (columns > k of A, all of B)
    const int w = (L - k - 1) + nb;
    for (int idx = t; idx < L * w; idx += nt) {
      const int r = idx / w, c = idx - (idx / w) * w;
      if (r == k) continue;
      const cpx<double> f = A[r * L + k];
      if (c < L - k - 1) {
        const int cc = k + 1 + c;
        A[r * L + cc] = A[r * L + cc] - f * A[k * L + cc];
      } else {
        const int cc = c - (L - k - 1);
        B[r * nb + cc] = B[r * nb + cc] - f * B[k * nb + cc];
      }
    }
    __syncthreads();
  }
  // finite result?
  if (t == 0) {
    for (int e = 0; e < L * nb; ++e)
      if (!isfinite(B[e].re) || !isfinite(B[e].im)) s_int[1] = 0;
  }
  __syncthreads();
  return s_int[1] != 0;
}

__device__ __forceinline__ void load_reduced(cpx<double>* dst, const double* src, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = mk(src[2 * e], src[2 * e + 1]);
}

// Record the residual of iteration ctl->iter and decide whether to go on.
// resid = max_i weight_i * sqrt(norm2_i).
__device__ int control_check(Control* ctl, double* hist, const double* norm2, const double* weight, int L) {
  __shared__ int s_state;
  if (threadIdx.x == 0) {
    double res = 0.0;
    bool bad = false;
    if (ctl->frob) {
      // orthonormalised right-hand side: bound every column of the original
      // block by weight[0] * ||R||_F
      double f = 0.0;
      for (int i = 0; i < L; ++i) f += norm2[i];
      res = weight[0] * sqrt(f);
      bad = !isfinite(res);
    } else {
      for (int i = 0; i < L; ++i) {
        const double v = weight[i] * sqrt(norm2[i]);
        if (!isfinite(v)) bad = true;
        res = fmax(res, v);
      }
    }
    ctl->resid = res;
    if (hist != nullptr && ctl->hist_count < ctl->hist_cap) hist[ctl->hist_count++] = res;
    if (bad) {
      ctl->state = ST_BREAKDOWN;
    } else if (res <= ctl->tol) {
      ctl->state = ST_CONVERGED;
    } else {
      if (res < ctl->best) {
        ctl->best = res;
        ctl->best_iter = ctl->iter;
      }
      if (ctl->iter >= ctl->max_iter) ctl->state = ST_MAXITER;
      else if (ctl->stagnation > 0 && ctl->iter - ctl->best_iter >= ctl->stagnation) ctl->state = ST_STAGNATION;
      else if (res > 1e5 * ctl->best) ctl->state = ST_STAGNATION;  // diverging
      else if (ctl->ru_delta > 0.0 && res < ctl->ru_delta * ctl->ru_anchor) ctl->ru_pending = 1;
    }
    s_state = ctl->state;
  }
  __syncthreads();
  return s_state;
}

// Cholesky factor of a Hermitian positive definite G (in A, LDS): on return
// A holds the upper-triangular S with G = S^H S and B holds S^-1.  Returns
// false (uniformly) if G is not numerically positive definite.
__device__ bool chol_inv(cpx<double>* A, cpx<double>* B, int L, int* s_int, double* s_dbl) {
  if (threadIdx.x == 0) s_int[1] = 1;
  __syncthreads();
  for (int j = 0; j < L; ++j) {
    if (threadIdx.x == 0) {
      double d = A[j * L + j].re;
      for (int k = 0; k < j; ++k) d -= A[k * L + j].re * A[k * L + j].re + A[k * L + j].im * A[k * L + j].im;
      if (!(d > 1e-28 * fabs(A[j * L + j].re)) || !isfinite(d)) s_int[1] = 0;
      s_dbl[0] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double sjj = s_dbl[0];
    for (int i = j + 1 + threadIdx.x; i < L; i += blockDim.x) {
      cpx<double> v = A[j * L + i];
      for (int k = 0; k < j; ++k) v = v - conj(A[k * L + j]) * A[k * L + i];
      A[j * L + i] = (1.0 / sjj) * v;
    }
    __syncthreads();
    if (threadIdx.x == 0) A[j * L + j] = mk(sjj, 0.0);
    __syncthreads();
  }
  const bool ok = s_int[1] != 0;
  __syncthreads();
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    const int i = e / L, j = e - (e / L) * L;
    if (i > j) A[e] = mk(0.0, 0.0);
    B[e] = mk(0.0, 0.0);
  }
  __syncthreads();
  if (!ok) return false;
  // S^-1 (upper): column j by back substitution, one thread per column
  for (int j = threadIdx.x; j < L; j += blockDim.x) {
    for (int i = j; i >= 0; --i) {
      cpx<double> v = mk(i == j ? 1.0 : 0.0, 0.0);
      for (int k = i + 1; k <= j; ++k) v = v - A[i * L + k] * B[k * L + j];
      const double d = A[i * L + i].re;
      B[i * L + j] = (1.0 / d) * v;
    }
  }
  __syncthreads();
  return true;
}

// Thin QR of an N x L block R from its Gram matrix G = R^H R (red_b):
// upper-triangular S with G = S^H S (Cholesky, FP64) and S^-1, so that
// Q = R S^-1 has orthonormal columns.  Failure (G not numerically positive
// definite) is reported through ctl->state = ST_BREAKDOWN.
__global__ void __launch_bounds__(256) k_coef_chol(CoefArgs c) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  const int L = c.L;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  load_reduced(A, c.red_b, L * L);
  __syncthreads();
  const bool ok = chol_inv(A, B, L, s_int, s_dbl);
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) c.S[e] = A[e];
  if (!ok) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) c.Sinv[e] = B[e];
  if (threadIdx.x == 0) c.ctl->state = ST_RUNNING;
}

// column norms^2 of an L x L matrix in LDS -> nrm[0..L)
__device__ __forceinline__ void col_norms2(const cpx<double>* M, int L, double* nrm) {
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < L; ++j) s += M[j * L + i].re * M[j * L + i].re + M[j * L + i].im * M[j * L + i].im;
    nrm[i] = s;
  }
  __syncthreads();
}

// QR frame, set-up: tau from the Gram matrix T^H T of the cycle's right-hand
// side (red_a); xi_0 = tau, tau^-1 for Q_0 = T tau^-1; iteration-0 stop test.
__global__ void __launch_bounds__(256) k_coef_ggrq_init(CoefArgs c) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  __shared__ double nrm[64];
  const int L = c.L;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  load_reduced(A, c.red_a, L * L);
  __syncthreads();
  const bool ok = chol_inv(A, B, L, s_int, s_dbl);
  if (!ok) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    c.xi[e] = A[e];
    c.Sinv[e] = B[e];
  }
  col_norms2(A, L, nrm);
  control_check(c.ctl, c.hist, nrm, c.weight, L);
}

// QR frame, set-up after the Gram kernels: R~0^H Q_0 from red_b[6L^2..8L^2).
__global__ void __launch_bounds__(256) k_coef_ggrq_init2(CoefArgs c) {
  const int L = c.L;
  load_reduced(c.GR, c.red_b + 6 * L * L, L * L);
}

// QR frame, top of iteration: alpha = (R~0^H V)^-1 R~0^H Q and the listing's
// zeta = Tr(W_k^H R_k) / Tr(W_k^H W_k) = Tr(xi^H (W^H Q) xi) / Tr(xi^H (W^H W) xi);
// red_b = [R~0^H V, W^H Q, W^H W].
__global__ void __launch_bounds__(256) k_coef_ggrq_top(CoefArgs c) {
  if (c.ctl->state != ST_RUNNING) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  __shared__ double part[3][256];
  const int L = c.L;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  // zeta: A <- xi, then sum_{j,i} conj(xi_ji) (G xi)_ji for G = W^H Q and W^H W
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) A[e] = c.xi[e];
  __syncthreads();
  double n_re = 0.0, n_im = 0.0, d_re = 0.0;
  const double* gwq = c.red_b + 2 * L * L;
  const double* gww = c.red_b + 4 * L * L;
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    const int j = e / L, i = e - (e / L) * L;
    cpx<double> m1 = mk(0.0, 0.0), m2 = mk(0.0, 0.0);
    for (int k = 0; k < L; ++k) {
      const cpx<double> x = A[k * L + i];
      cmac(m1, mk(gwq[2 * (j * L + k)], gwq[2 * (j * L + k) + 1]), x);
      cmac(m2, mk(gww[2 * (j * L + k)], gww[2 * (j * L + k) + 1]), x);
    }
    const cpx<double> xji = A[j * L + i];
    const cpx<double> t1 = conj(xji) * m1, t2 = conj(xji) * m2;
    n_re += t1.re;
    n_im += t1.im;
    d_re += t2.re;
  }
  part[0][threadIdx.x] = n_re;
  part[1][threadIdx.x] = n_im;
  part[2][threadIdx.x] = d_re;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k = 0; k < (int)blockDim.x; ++k) {
      a0 += part[0][k];
      a1 += part[1][k];
      a2 += part[2][k];
    }
    s_dbl[1] = a0 / a2;
    s_dbl[2] = a1 / a2;
    s_dbl[3] = a2;
    c.zeta[0] = mk(a0 / a2, a1 / a2);
  }
  __syncthreads();
  if (!(s_dbl[3] > 0.0) || !isfinite(s_dbl[1]) || !isfinite(s_dbl[2])) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  // alpha
  load_reduced(A, c.red_b, L * L);
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) B[e] = c.GR[e];
  __syncthreads();
  if (!solve_gj(A, B, L, L, s_int, s_dbl)) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) c.alpha[e] = B[e];
}

// QR frame, end of iteration: red_a = [T^H T, R~0^H T].  T = Q_{k+1} tau,
// xi_{k+1} = tau xi_k; count the iteration and test ||r_i|| = ||xi e_i||;
// R~0^H Q_{k+1} = (R~0^H T) tau^-1; gamma = (R~0^H Q_k)^-1 (R~0^H Q_{k+1}) / zeta.
__global__ void __launch_bounds__(256) k_coef_ggrq_end(CoefArgs c) {
  if (c.ctl->state != ST_RUNNING) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  __shared__ double nrm[64];
  const int L = c.L;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  if (threadIdx.x == 0) c.ctl->iter += 1;
  load_reduced(A, c.red_a, L * L);
  __syncthreads();
  if (!chol_inv(A, B, L, s_int, s_dbl)) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  // tau^-1 for the next update kernel, and R~0^H Q_{k+1} = (R~0^H T) tau^-1
  // into tmp (each thread later reads back only the entries it wrote)
  const double* gtt = c.red_a + 2 * L * L;
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    const int i = e / L, j = e - (e / L) * L;
    c.Sinv[e] = B[e];
    cpx<double> v = mk(0.0, 0.0);
    for (int k = 0; k <= j; ++k) cmac(v, mk(gtt[2 * (i * L + k)], gtt[2 * (i * L + k) + 1]), B[k * L + j]);
    c.tmp[e] = v;
  }
  __syncthreads();
  // xi_{k+1} = tau xi_k
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    const int i = e / L, j = e - (e / L) * L;
    cpx<double> v = mk(0.0, 0.0);
    for (int k = i; k < L; ++k) cmac(v, A[i * L + k], c.xi[k * L + j]);
    B[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    c.eta[e] = c.xi[e];  // tau_{k+1}^-1 xi_{k+1} = xi_k
    c.xi[e] = B[e];
  }
  col_norms2(B, L, nrm);
  if (control_check(c.ctl, c.hist, nrm, c.weight, L) != ST_RUNNING) return;
  const cpx<double> z = c.zeta[0];
  const double zd = z.re * z.re + z.im * z.im;
  const cpx<double> zi = mk(z.re / zd, -z.im / zd);
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    A[e] = c.GR[e];
    B[e] = c.tmp[e] * zi;
  }
  __syncthreads();
  if (!solve_gj(A, B, L, L, s_int, s_dbl)) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    c.beta[e] = B[e];
    c.GR[e] = c.tmp[e];
  }
}

// Fused QR frame, set-up: red_a = [T^H T, R~0^H T] of the cycle's
// right-hand side T = R_0.  tau = chol(T^H T); xi_0 = tau, tau^-1,
// eta = I, gamma_{-1} = 0, R~0^H Q_0 = (R~0^H T) tau^-1; iteration-0 stop test.
__global__ void __launch_bounds__(256) k_coef_finit(CoefArgs c) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  __shared__ double nrm[64];
  const int L = c.L;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  load_reduced(A, c.red_a, L * L);
  __syncthreads();
  if (!chol_inv(A, B, L, s_int, s_dbl)) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  const double* grt = c.red_a + 2 * L * L;
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    const int i = e / L, j = e - (e / L) * L;
    c.xi[e] = A[e];
    c.Sinv[e] = B[e];
    c.eta[e] = mk(i == j ? 1.0 : 0.0, 0.0);
    c.beta[e] = mk(0.0, 0.0);
    cpx<double> v = mk(0.0, 0.0);
    for (int k = 0; k <= j; ++k) cmac(v, mk(grt[2 * (i * L + k)], grt[2 * (i * L + k) + 1]), B[k * L + j]);
    c.GR[e] = v;
  }
  col_norms2(A, L, nrm);
  control_check(c.ctl, c.hist, nrm, c.weight, L);
}

// Fused QR frame, top of iteration k.  red_b = [T^H W', W'^H W', R~0^H W'],
// red_a[4L^2..6L^2) = R~0^H Y_{k-1} (k > 0).  With eta = tau^-1 xi:
//   zeta = Tr(eta^H (W'^H T) eta) / Tr(eta^H (W'^H W') eta)   (= Tr(W_k^H R_k) / Tr(W_k^H W_k)),
//   R~0^H V_k = (R~0^H W') tau^-1 + (R~0^H Y_{k-1}) gamma_{k-1},
//   alpha = (R~0^H V_k)^-1 R~0^H Q_k,
//   mu1 = tau^-1 alpha, mu2 = gamma_{k-1} alpha, mx1 = zeta eta.
__global__ void __launch_bounds__(256) k_coef_ftop(CoefArgs c) {
  if (c.ctl->state != ST_RUNNING) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  __shared__ double part[3][256];
  const int L = c.L, L2 = L * L;
  const bool first = c.ctl->iter == 0;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L2;
  cpx<double>* E = B + L2;  // eta
  for (int e = threadIdx.x; e < L2; e += blockDim.x) E[e] = c.eta[e];
  __syncthreads();
  // traces: sum_{a,i} conj(eta_ai) (M eta)_ai for M = W'^H T (conj-transpose of T^H W') and W'^H W'
  const double* gtw = c.red_b;
  const double* gww = c.red_b + 2 * L2;
  double n_re = 0.0, n_im = 0.0, d_re = 0.0;
  for (int e = threadIdx.x; e < L2; e += blockDim.x) {
    const int a = e / L, i = e - (e / L) * L;
    cpx<double> m1 = mk(0.0, 0.0), m2 = mk(0.0, 0.0);
    for (int b = 0; b < L; ++b) {
      const cpx<double> x = E[b * L + i];
      // (W'^H T)_ab = conj((T^H W')_ba)
      cmac(m1, mk(gtw[2 * (b * L + a)], -gtw[2 * (b * L + a) + 1]), x);
      cmac(m2, mk(gww[2 * (a * L + b)], gww[2 * (a * L + b) + 1]), x);
    }
    const cpx<double> ea = E[a * L + i];
    const cpx<double> t1 = conj(ea) * m1, t2 = conj(ea) * m2;
    n_re += t1.re;
    n_im += t1.im;
    d_re += t2.re;
  }
  part[0][threadIdx.x] = n_re;
  part[1][threadIdx.x] = n_im;
  part[2][threadIdx.x] = d_re;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k = 0; k < (int)blockDim.x; ++k) {
      a0 += part[0][k];
      a1 += part[1][k];
      a2 += part[2][k];
    }
    s_dbl[1] = a0 / a2;
    s_dbl[2] = a1 / a2;
    s_dbl[3] = a2;
  }
  __syncthreads();
  if (!(s_dbl[3] > 0.0) || !isfinite(s_dbl[1]) || !isfinite(s_dbl[2])) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  const cpx<double> z = mk(s_dbl[1], s_dbl[2]);
  // A = R~0^H V_k, B = R~0^H Q_k
  const double* grw = c.red_b + 4 * L2;
  const double* gry = c.red_a + 4 * L2;
  for (int e = threadIdx.x; e < L2; e += blockDim.x) {
    const int i = e / L, j = e - (e / L) * L;
    cpx<double> v = mk(0.0, 0.0);
    for (int k = 0; k <= j; ++k) cmac(v, mk(grw[2 * (i * L + k)], grw[2 * (i * L + k) + 1]), c.Sinv[k * L + j]);
    if (!first)
      for (int k = 0; k < L; ++k) cmac(v, mk(gry[2 * (i * L + k)], gry[2 * (i * L + k) + 1]), c.beta[k * L + j]);
    A[e] = v;
    B[e] = c.GR[e];
  }
  __syncthreads();
  if (!solve_gj(A, B, L, L, s_int, s_dbl)) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  // B = alpha
  for (int e = threadIdx.x; e < L2; e += blockDim.x) {
    const int i = e / L, j = e - (e / L) * L;
    cpx<double> v1 = mk(0.0, 0.0), v2 = mk(0.0, 0.0);
    for (int k = i; k < L; ++k) cmac(v1, c.Sinv[i * L + k], B[k * L + j]);
    if (!first)
      for (int k = 0; k < L; ++k) cmac(v2, c.beta[i * L + k], B[k * L + j]);
    c.alpha[e] = B[e];
    c.mu1[e] = v1;
    c.mu2[e] = v2;
    c.mx1[e] = z * E[e];
  }
  if (threadIdx.x == 0) c.zeta[0] = z;
}

// Reliable update, new frame: red_a[0..L^2) = R^H R of the true residual R
// (cycle units).  tau = chol(R^H R): the new frame is Q' = R tau^-1 with
// xi' = tau; the search blocks are carried over as P' = P M, V' = V M with
// M = xi_old tau^-1 (so that P' xi' = P xi_old), M into tmp.  The control
// record restarts from the true residual, and the queue runs again.
__global__ void __launch_bounds__(256) k_coef_ru_frame(CoefArgs c) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  __shared__ double nrm[64];
  const int L = c.L;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  load_reduced(A, c.red_a, L * L);
  __syncthreads();
  if (!chol_inv(A, B, L, s_int, s_dbl)) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    const int i = e / L, j = e - (e / L) * L;
    cpx<double> v = mk(0.0, 0.0);
    for (int k = 0; k <= j; ++k) cmac(v, c.xi[i * L + k], B[k * L + j]);
    c.tmp[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    c.xi[e] = A[e];
    c.Sinv[e] = B[e];
  }
  col_norms2(A, L, nrm);
  if (threadIdx.x == 0) {
    double res = 0.0;
    if (c.ctl->frob) {
      double f = 0.0;
      for (int i = 0; i < L; ++i) f += nrm[i];
      res = c.weight[0] * sqrt(f);
    } else {
      for (int i = 0; i < L; ++i) res = fmax(res, c.weight[i] * sqrt(nrm[i]));
    }
    c.ctl->resid = res;
    c.ctl->ru_anchor = res;
    c.ctl->ru_pending = 0;
    c.ctl->state = ST_RUNNING;
  }
}

// End of an iteration: a reliable update asked for by its stop test stops
// the iterations queued after it.
__global__ void k_coef_ru_commit(CoefArgs c) {
  if (threadIdx.x == 0 && c.ctl->state == ST_RUNNING && c.ctl->ru_pending) {
    c.ctl->ru_pending = 0;
    c.ctl->state = ST_RELIABLE;
  }
}

// Iteration 0: G_R = R~0^H R_0 from the reduced record (Gram + norms).
__global__ void __launch_bounds__(256) k_coef_init(CoefArgs c) {
  load_reduced(c.GR, c.red_a, c.L * c.L);
  __syncthreads();
  control_check(c.ctl, c.hist, c.red_a + 2 * c.L * c.L, c.weight, c.L);
}

// BiCGGR top of iteration: solve (R~0^H V) alpha = R~0^H R; zeta = Tr(W^H R)/Tr(W^H W)
__global__ void __launch_bounds__(256) k_coef_bicggr_top(CoefArgs c) {
  if (c.ctl->state != ST_RUNNING) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  const int L = c.L;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  load_reduced(A, c.red_b, L * L);          // R~0^H V
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) B[e] = c.GR[e];
  __syncthreads();
  const bool ok = solve_gj(A, B, L, L, s_int, s_dbl);
  const double t0 = c.red_c[0], t1 = c.red_c[1], t2 = c.red_c[2];
  if (!ok || !(t2 > 0.0) || !isfinite(t0) || !isfinite(t1)) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) c.alpha[e] = B[e];
  if (threadIdx.x == 0) c.zeta[0] = mk(t0 / t2, t1 / t2);
}

// BiCGGR end of iteration: count it, check R_{k+1}, then
// solve (R~0^H R_k) gamma = R~0^H R_{k+1} / zeta and keep R~0^H R_{k+1}.
__global__ void __launch_bounds__(256) k_coef_bicggr_end(CoefArgs c) {
  if (c.ctl->state != ST_RUNNING) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  const int L = c.L;
  if (threadIdx.x == 0) c.ctl->iter += 1;
  __syncthreads();
  if (control_check(c.ctl, c.hist, c.red_a + 2 * L * L, c.weight, L) != ST_RUNNING) return;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  const cpx<double> z = c.zeta[0];
  const double zd = z.re * z.re + z.im * z.im;
  const cpx<double> zi = mk(z.re / zd, -z.im / zd);
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    A[e] = c.GR[e];
    B[e] = mk(c.red_a[2 * e], c.red_a[2 * e + 1]) * zi;
  }
  __syncthreads();
  const bool ok = zd > 0.0 && solve_gj(A, B, L, L, s_int, s_dbl);
  if (!ok) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    c.beta[e] = B[e];
    c.GR[e] = mk(c.red_a[2 * e], c.red_a[2 * e + 1]);
  }
}

// BiCGSTAB: solve (R~0^H V) alpha = R~0^H R, keep R~0^H V for the beta solve
__global__ void __launch_bounds__(256) k_coef_bicgstab_alpha(CoefArgs c) {
  if (c.ctl->state != ST_RUNNING) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  const int L = c.L;
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  load_reduced(A, c.red_b, L * L);
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    B[e] = c.GR[e];
    c.GV[e] = mk(c.red_b[2 * e], c.red_b[2 * e + 1]);
  }
  __syncthreads();
  if (!solve_gj(A, B, L, L, s_int, s_dbl)) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) c.alpha[e] = B[e];
}

// BiCGSTAB: zeta = Tr(Z^H T) / Tr(Z^H Z); zeta = 0 when Z = 0 exactly
__global__ void k_coef_bicgstab_zeta(CoefArgs c) {
  if (c.ctl->state != ST_RUNNING) return;
  if (threadIdx.x == 0) {
    const double t0 = c.red_c[0], t1 = c.red_c[1], t2 = c.red_c[2];
    if (!isfinite(t0) || !isfinite(t1) || !isfinite(t2)) c.ctl->state = ST_BREAKDOWN;
    else c.zeta[0] = (t2 == 0.0) ? mk(0.0, 0.0) : mk(t0 / t2, t1 / t2);
  }
}

// BiCGSTAB end of iteration: count it, check R_{k+1}, then beta.
// Block: (R~0^H V) beta = -R~0^H Z.  Scalar listing (L = 1, scalar = 1):
// beta = (alpha / zeta) (r~0, r_{k+1}) / (r~0, r_k).
__global__ void __launch_bounds__(256) k_coef_bicgstab_beta(CoefArgs c) {
  if (c.ctl->state != ST_RUNNING) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_int[2];
  __shared__ double s_dbl[4];
  const int L = c.L;
  if (threadIdx.x == 0) c.ctl->iter += 1;
  __syncthreads();
  if (control_check(c.ctl, c.hist, c.red_a + 4 * L * L, c.weight, L) != ST_RUNNING) return;
  if (c.scalar) {
    if (threadIdx.x == 0) {
      const cpx<double> z = c.zeta[0];
      const cpx<double> rho_new = mk(c.red_a[0], c.red_a[1]);
      const cpx<double> rho_old = c.GR[0];
      cpx<double> beta = mk(0.0, 0.0);
      if (z.re != 0.0 || z.im != 0.0) {
        const cpx<double> num = c.alpha[0] * rho_new;
        const cpx<double> den = z * rho_old;
        const double dd = den.re * den.re + den.im * den.im;
        beta = mk((num.re * den.re + num.im * den.im) / dd, (num.im * den.re - num.re * den.im) / dd);
      }
      if (!isfinite(beta.re) || !isfinite(beta.im)) c.ctl->state = ST_BREAKDOWN;
      c.beta[0] = beta;
      c.GR[0] = rho_new;
    }
    return;
  }
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* B = A + L * L;
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    A[e] = c.GV[e];
    B[e] = mk(-c.red_a[2 * L * L + 2 * e], -c.red_a[2 * L * L + 2 * e + 1]);
  }
  __syncthreads();
  if (!solve_gj(A, B, L, L, s_int, s_dbl)) {
    if (threadIdx.x == 0) c.ctl->state = ST_BREAKDOWN;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    c.beta[e] = B[e];
    c.GR[e] = mk(c.red_a[2 * e], c.red_a[2 * e + 1]);
  }
}

int upd_grid(long long nrows, int L) {
  const int R = kBT / L;
  const long long ntiles = (nrows + R - 1) / R;
  return (int)std::min<long long>(ntiles, L <= kSmallL ? kUpdBlocksSmall : kUpdBlocks);
}

}  // namespace

// ------------------------------------------------------------------ launchers
// Grams on FP64 MFMA at L = 24, where the 2 x 2 VALU blocks would compute a
// 32 x 32 Gram.  At L = 32 the MFMA form measured slower: on this chip the
// FP64 matrix rate equals the FP64 vector rate, and its accumulators cost
// occupancy in these latency-bound kernels.
#ifdef BKWD_NO_MFMA_GRAM
constexpr bool kMfmaGram = false;
#else
constexpr bool kMfmaGram = true;
#endif

#define LAUNCH_NE(KERNEL, T, L, grid, smem, s, args)                                         \
  do {                                                                                       \
    if ((L) * (L) <= kBT) hipLaunchKernelGGL((KERNEL<T, 1>), dim3(grid), dim3(kBT), smem, s, args); \
    else if (kMfmaGram && (L) == 24) hipLaunchKernelGGL((KERNEL<T, -3>), dim3(grid), dim3(kBT), smem, s, args); \
    else if ((L) <= 32) hipLaunchKernelGGL((KERNEL<T, 4>), dim3(grid), dim3(kBT), smem, s, args);    \
    else if ((L) <= 48) hipLaunchKernelGGL((KERNEL<T, 9>), dim3(grid), dim3(kBT), smem, s, args);    \
    else hipLaunchKernelGGL((KERNEL<T, 16>), dim3(grid), dim3(kBT), smem, s, args);                  \
  } while (0)

#define LAUNCH_LB(KERNEL, T, L, grid, s, args)                                                    \
  do {                                                                                            \
    if ((L) <= 4) hipLaunchKernelGGL((KERNEL<T, 4>), dim3(grid), dim3(kBT), 0, s, args);          \
    else if ((L) <= 8) hipLaunchKernelGGL((KERNEL<T, 8>), dim3(grid), dim3(kBT), 0, s, args);     \
    else if ((L) <= 12) hipLaunchKernelGGL((KERNEL<T, 12>), dim3(grid), dim3(kBT), 0, s, args);   \
    else hipLaunchKernelGGL((KERNEL<T, 16>), dim3(grid), dim3(kBT), 0, s, args);                  \
  } while (0)

// The lane-per-real kernels serve the fused frame's 8-column FP32 blocks.
#ifdef BKWD_NO_L8_KERNELS
constexpr bool kL8Kernels = false;
#else
constexpr bool kL8Kernels = true;
#endif

template <typename T>
bool l8_lane_kernels(const BlasArgs<T>& a) {
  return kL8Kernels && std::is_same<T, float>::value && a.L == 8;
}

// the FP32 kernels' argument type (only reached when T is float)
template <typename T>
const BlasArgs<float>& as_f32(const BlasArgs<T>& a) {
  return *reinterpret_cast<const BlasArgs<float>*>(&a);
}

template <typename T>
int blas_launch(int op, const BlasArgs<T>& a, hipStream_t s) {
  const int grid = upd_grid(a.nrows, a.L);
  const size_t smem = blas_smem_bytes(a.L, sizeof(T));
  if (a.L <= kSmallL) {
    switch (op) {
      case OP_BICGGR_U: LAUNCH_LB(k_s_bicggr_u, T, a.L, grid, s, a); return grid;
      case OP_GGRQ_XR: LAUNCH_LB(k_s_ggrq_xr, T, a.L, grid, s, a); return grid;
      case OP_GGRQ_PV: LAUNCH_LB(k_s_ggrq_pv, T, a.L, grid, s, a); return grid;
      case OP_FU: LAUNCH_LB(k_s_fu, T, a.L, grid, s, a); return grid;
      case OP_FXR: LAUNCH_LB(k_s_fxr, T, a.L, grid, s, a); return grid;
      case OP_FUX:
        if (!l8_lane_kernels(a)) return -1;
        hipLaunchKernelGGL(k_l8_fux, dim3(grid), dim3(kBT), 0, s, as_f32(a));
        return grid;
      case OP_FXRT:
        if (!l8_lane_kernels(a)) return -1;
        hipLaunchKernelGGL(k_l8_fxrt, dim3(grid), dim3(kBT), 0, s, as_f32(a));
        return grid;
      case OP_FGRAM:
        if (l8_lane_kernels(a)) {
          if (a.ng == 2) hipLaunchKernelGGL(k_l8_fgram<2>, dim3(grid), dim3(kBT), 0, s, as_f32(a));
          else hipLaunchKernelGGL(k_l8_fgram<3>, dim3(grid), dim3(kBT), 0, s, as_f32(a));
        } else if (a.ng == 2) {
          LAUNCH_LB(k_s_fgram2, T, a.L, grid, s, a);
        } else {
          LAUNCH_LB(k_s_fgram3, T, a.L, grid, s, a);
        }
        return grid;
      default: break;
    }
  }
  switch (op) {
    case OP_BICGGR_U: hipLaunchKernelGGL(k_bicggr_u<T>, dim3(grid), dim3(kBT), smem, s, a); break;
    case OP_BICGGR_XR: LAUNCH_NE(k_bicggr_xr, T, a.L, grid, smem, s, a); break;
    case OP_BICGGR_PV: LAUNCH_NE(k_bicggr_pv, T, a.L, grid, smem, s, a); break;
    case OP_BICGSTAB_T:
      if (a.L == 1) hipLaunchKernelGGL(k1_bicgstab_t<T>, dim3(grid), dim3(kBT), 0, s, a);
      else hipLaunchKernelGGL(k_bicgstab_t<T>, dim3(grid), dim3(kBT), smem, s, a);
      break;
    case OP_BICGSTAB_XR:
      if (a.L == 1) hipLaunchKernelGGL(k1_bicgstab_xr<T>, dim3(grid), dim3(kBT), 0, s, a);
      else LAUNCH_NE(k_bicgstab_xr, T, a.L, grid, smem, s, a);
      break;
    case OP_BICGSTAB_P:
      if (a.L == 1) hipLaunchKernelGGL(k1_bicgstab_p<T>, dim3(grid), dim3(kBT), 0, s, a);
      else hipLaunchKernelGGL(k_bicgstab_p<T>, dim3(grid), dim3(kBT), smem, s, a);
      break;
    case OP_GRAM:
      if (a.L == 1) hipLaunchKernelGGL(k1_gram<T>, dim3(grid), dim3(kBT), 0, s, a);
      else LAUNCH_NE(k_gram, T, a.L, grid, smem, s, a);
      break;
    case OP_GRAM2: LAUNCH_NE(k_gram2, T, a.L, grid, smem, s, a); break;
    case OP_GGRQ_XR: LAUNCH_NE(k_ggrq_xr, T, a.L, grid, smem, s, a); break;
    case OP_GGRQ_PV: LAUNCH_NE(k_ggrq_pv, T, a.L, grid, smem, s, a); break;
    default: return -1;
  }
  return grid;
}

template int blas_launch<float>(int, const BlasArgs<float>&, hipStream_t);
template int blas_launch<double>(int, const BlasArgs<double>&, hipStream_t);

int blas_grid(long long nrows, int L) { return upd_grid(nrows, L); }

bool blas_fused_x(int L, size_t elem) { return kL8Kernels && elem == sizeof(cpx<float>) && L == 8; }

hipError_t launch_reduce(const double* in, long long nrows, int nv, double* stage, size_t stage_half, double* out,
                         hipStream_t s) {
  // stage 1..k: at most 256 rows per workgroup
  const double* src = in;
  long long rows = nrows;
  double* bufs[2] = {stage, stage + stage_half};
  int which = 0;
  while (rows > 256) {
    const long long nsplit = (rows + 255) / 256;
    double* dst = bufs[which];
    hipLaunchKernelGGL(k_reduce, dim3((nv + 63) / 64, (unsigned)nsplit), dim3(1024), 0, s, src, rows, nv, 256, dst);
    src = dst;
    rows = nsplit;
    which ^= 1;
  }
  hipLaunchKernelGGL(k_reduce, dim3((nv + 63) / 64, 1), dim3(1024), 0, s, src, rows, nv, (int)rows, out);
  return hipGetLastError();
}

hipError_t launch_coef(int op, const CoefArgs& c, hipStream_t s) {
  const size_t smem = (size_t)2 * c.L * c.L * sizeof(cpx<double>);
  switch (op) {
    case COEF_INIT: hipLaunchKernelGGL(k_coef_init, dim3(1), dim3(256), 0, s, c); break;
    case COEF_BICGGR_TOP: hipLaunchKernelGGL(k_coef_bicggr_top, dim3(1), dim3(256), smem, s, c); break;
    case COEF_BICGGR_END: hipLaunchKernelGGL(k_coef_bicggr_end, dim3(1), dim3(256), smem, s, c); break;
    case COEF_BICGSTAB_ALPHA: hipLaunchKernelGGL(k_coef_bicgstab_alpha, dim3(1), dim3(256), smem, s, c); break;
    case COEF_BICGSTAB_ZETA: hipLaunchKernelGGL(k_coef_bicgstab_zeta, dim3(1), dim3(64), 0, s, c); break;
    case COEF_BICGSTAB_BETA: hipLaunchKernelGGL(k_coef_bicgstab_beta, dim3(1), dim3(256), smem, s, c); break;
    case COEF_CHOL: hipLaunchKernelGGL(k_coef_chol, dim3(1), dim3(256), smem, s, c); break;
    case COEF_GGRQ_INIT: hipLaunchKernelGGL(k_coef_ggrq_init, dim3(1), dim3(256), smem, s, c); break;
    case COEF_GGRQ_INIT2: hipLaunchKernelGGL(k_coef_ggrq_init2, dim3(1), dim3(256), 0, s, c); break;
    case COEF_GGRQ_TOP: hipLaunchKernelGGL(k_coef_ggrq_top, dim3(1), dim3(256), smem, s, c); break;
    case COEF_GGRQ_END: hipLaunchKernelGGL(k_coef_ggrq_end, dim3(1), dim3(256), smem, s, c); break;
    case COEF_FINIT: hipLaunchKernelGGL(k_coef_finit, dim3(1), dim3(256), smem, s, c); break;
    case COEF_FTOP:
      hipLaunchKernelGGL(k_coef_ftop, dim3(1), dim3(256), (size_t)3 * c.L * c.L * sizeof(cpx<double>), s, c);
      break;
    case COEF_RU_FRAME: hipLaunchKernelGGL(k_coef_ru_frame, dim3(1), dim3(256), smem, s, c); break;
    case COEF_RU_COMMIT: hipLaunchKernelGGL(k_coef_ru_commit, dim3(1), dim3(64), 0, s, c); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gaussian(cpx<T>* out, long long n, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(k_gaussian<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, seed);
  return hipGetLastError();
}
template hipError_t launch_gaussian<float>(cpx<float>*, long long, unsigned long long, hipStream_t);
template hipError_t launch_gaussian<double>(cpx<double>*, long long, unsigned long long, hipStream_t);

template <typename To, typename Ti>
hipError_t launch_scale_convert(const cpx<Ti>* in, cpx<To>* out, const double* scale, long long n, int L, int vol,
                                hipStream_t s) {
  hipLaunchKernelGGL((k_scale_convert<To, Ti>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, scale,
                     n, L, vol);
  return hipGetLastError();
}
template hipError_t launch_scale_convert<float, double>(const cpx<double>*, cpx<float>*, const double*, long long,
                                                        int, int, hipStream_t);
template hipError_t launch_scale_convert<double, double>(const cpx<double>*, cpx<double>*, const double*, long long,
                                                         int, int, hipStream_t);

template <typename Ti>
hipError_t launch_accumulate(cpx<double>* x, const cpx<Ti>* e, const double* scale, long long n, int L, int vol,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate<Ti>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, e, scale, n, L, vol);
  return hipGetLastError();
}
template hipError_t launch_accumulate<float>(cpx<double>*, const cpx<float>*, const double*, long long, int, int,
                                             hipStream_t);
template hipError_t launch_accumulate<double>(cpx<double>*, const cpx<double>*, const double*, long long, int, int,
                                              hipStream_t);

template <typename To>
hipError_t launch_convert(const cpx<double>* in, cpx<To>* out, long long n, int L, int vol, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<To, double>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n, L, vol);
  return hipGetLastError();
}
template hipError_t launch_convert<float>(const cpx<double>*, cpx<float>*, long long, int, int, hipStream_t);
template hipError_t launch_convert<double>(const cpx<double>*, cpx<double>*, long long, int, int, hipStream_t);

template <typename To, typename Ti, bool ACC, int PERM>
hipError_t launch_rowmat(const cpx<Ti>* in, cpx<To>* out, const cpx<double>* M, double sign, long long nrows, int L,
                         int vol, hipStream_t s) {
  const int R = kBT / L;
  const long long ntiles = (nrows + R - 1) / R;
  const int grid = (int)std::min<long long>(ntiles, 4096);
  const size_t smem = (size_t)(L * L + kBT) * sizeof(cpx<double>);
  hipLaunchKernelGGL((k_rowmat<To, Ti, ACC, PERM>), dim3(grid), dim3(kBT), smem, s, in, out, M, sign, nrows, L, vol);
  return hipGetLastError();
}
template hipError_t launch_rowmat<float, double, false, 1>(const cpx<double>*, cpx<float>*, const cpx<double>*, double,
                                                           long long, int, int, hipStream_t);
template hipError_t launch_rowmat<double, float, true, 2>(const cpx<float>*, cpx<double>*, const cpx<double>*, double,
                                                          long long, int, int, hipStream_t);
template hipError_t launch_rowmat<float, float, false, 0>(const cpx<float>*, cpx<float>*, const cpx<double>*, double,
                                                          long long, int, int, hipStream_t);
template hipError_t launch_rowmat<double, double, false, 0>(const cpx<double>*, cpx<double>*, const cpx<double>*,
                                                            double, long long, int, int, hipStream_t);

hipError_t launch_gather_cols(const cpx<double>* X, cpx<double>* x, long long nrows, int L, int c0, int n,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((nrows * n + 255) / 256)), dim3(256), 0, s, X, x, nrows, L, c0, n);
  return hipGetLastError();
}

hipError_t launch_scatter_cols(cpx<double>* X, const cpx<double>* x, long long nrows, int L, int c0, int n,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_cols, dim3((unsigned)((nrows * n + 255) / 256)), dim3(256), 0, s, X, x, nrows, L, c0, n);
  return hipGetLastError();
}

// The entry layouts whose LDS can pass 64 KiB (L > 32).
template <auto K9, auto K16, typename F>
void set_ne(F& set, int bytes) {
  set((const void*)K9, bytes);
  set((const void*)K16, bytes);
}

hipError_t blas_set_attributes() {
  // dynamic LDS above 64 KiB: coefficient kernels at L = 64 hold two 64 x 64
  // complex-double matrices (128 KiB); FP64 streaming kernels at L = 64 need
  // about 78 KiB.
  hipError_t e = hipSuccess;
  auto set = [&](const void* f, int bytes) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (r != hipSuccess) e = r;
  };
  const int coef_bytes = 2 * 64 * 64 * (int)sizeof(cpx<double>);
  const int blas_bytes = (int)blas_smem_bytes(64, sizeof(cpx<double>) / 2);
  set((const void*)k_coef_bicggr_top, coef_bytes);
  set((const void*)k_coef_bicggr_end, coef_bytes);
  set((const void*)k_coef_bicgstab_alpha, coef_bytes);
  set((const void*)k_coef_bicgstab_beta, coef_bytes);
  set((const void*)k_coef_chol, coef_bytes);
  set((const void*)k_coef_ggrq_init, coef_bytes);
  set((const void*)k_coef_ggrq_top, coef_bytes);
  set((const void*)k_coef_ggrq_end, coef_bytes);
  set((const void*)k_coef_finit, coef_bytes);
  set((const void*)k_coef_ftop, coef_bytes);
  set((const void*)k_coef_ru_frame, coef_bytes);
  set_ne<k_gram2<double, 9>, k_gram2<double, 16>>(set, blas_bytes);
  set_ne<k_ggrq_xr<double, 9>, k_ggrq_xr<double, 16>>(set, blas_bytes);
  set_ne<k_ggrq_pv<double, 9>, k_ggrq_pv<double, 16>>(set, blas_bytes);
  set_ne<k_gram2<float, 9>, k_gram2<float, 16>>(set, blas_bytes);
  set_ne<k_ggrq_xr<float, 9>, k_ggrq_xr<float, 16>>(set, blas_bytes);
  set_ne<k_ggrq_pv<float, 9>, k_ggrq_pv<float, 16>>(set, blas_bytes);
  set((const void*)k_rowmat<float, double, false, 1>, coef_bytes);
  set((const void*)k_rowmat<double, float, true, 2>, coef_bytes);
  set((const void*)k_rowmat<float, float, false, 0>, coef_bytes);
  set((const void*)k_rowmat<double, double, false, 0>, coef_bytes);
  set((const void*)k_bicggr_u<double>, blas_bytes);
  set_ne<k_bicggr_xr<double, 9>, k_bicggr_xr<double, 16>>(set, blas_bytes);
  set_ne<k_bicggr_pv<double, 9>, k_bicggr_pv<double, 16>>(set, blas_bytes);
  set((const void*)k_bicgstab_t<double>, blas_bytes);
  set_ne<k_bicgstab_xr<double, 9>, k_bicgstab_xr<double, 16>>(set, blas_bytes);
  set((const void*)k_bicgstab_p<double>, blas_bytes);
  set_ne<k_gram<double, 9>, k_gram<double, 16>>(set, blas_bytes);
  return e;
}

template <typename To>
hipError_t launch_eo_gather(const cpx<double>* in, cpx<To>* out, const double* scale, const Geom& g, int L,
                            hipStream_t s) {
  const long long n = 6LL * g.vol * L;
  const int grid = (int)std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_eo_gather<To>, dim3(grid), dim3(256), 0, s, in, out, scale, g.lx, g.ly, g.lz, g.vol / 2, L);
  return hipGetLastError();
}
template hipError_t launch_eo_gather<float>(const cpx<double>*, cpx<float>*, const double*, const Geom&, int,
                                            hipStream_t);
template hipError_t launch_eo_gather<double>(const cpx<double>*, cpx<double>*, const double*, const Geom&, int,
                                             hipStream_t);

template <typename Ti>
hipError_t launch_eo_scatter(const cpx<Ti>* in, cpx<double>* out, const double* unscale, const Geom& g, int L,
                             hipStream_t s) {
  const long long n = 6LL * g.vol * L;
  const int grid = (int)std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_eo_scatter<Ti>, dim3(grid), dim3(256), 0, s, in, out, unscale, g.lx, g.ly, g.lz, g.vol / 2,
                     L);
  return hipGetLastError();
}
template hipError_t launch_eo_scatter<float>(const cpx<float>*, cpx<double>*, const double*, const Geom&, int,
                                             hipStream_t);
template hipError_t launch_eo_scatter<double>(const cpx<double>*, cpx<double>*, const double*, const Geom&, int,
                                              hipStream_t);

hipError_t launch_axpy64(cpx<double>* x, const cpx<double>* w, double sign, long long n, hipStream_t s) {
  const int grid = (int)std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_axpy64, dim3(grid), dim3(256), 0, s, x, w, sign, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trace2(const cpx<T>* x, const cpx<T>* y, long long n, double* partials, int* nblk, hipStream_t s) {
  const int grid = (int)std::min<long long>((n + 255) / 256, 1024);
  *nblk = grid;
  hipLaunchKernelGGL(k_trace2<T>, dim3(grid), dim3(256), 0, s, x, y, n, partials);
  return hipGetLastError();
}
template hipError_t launch_trace2<float>(const cpx<float>*, const cpx<float>*, long long, double*, int*, hipStream_t);
template hipError_t launch_trace2<double>(const cpx<double>*, const cpx<double>*, long long, double*, int*,
                                          hipStream_t);

hipError_t launch_gather_idx(const cpx<double>* src, cpx<double>* dst, long long nrows, int L, const int* idx, int n,
                             hipStream_t s) {
  const int grid = (int)std::min<long long>((nrows * n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_gather_idx, dim3(grid), dim3(256), 0, s, src, dst, nrows, L, idx, n);
  return hipGetLastError();
}

template <typename Ti, bool CM>
hipError_t launch_rowmat_rect(const cpx<Ti>* in, cpx<double>* out, const cpx<double>* M, double sign, long long nrows,
                              int Lin, int Lout, int vol, hipStream_t s) {
  const int grid = (int)std::min<long long>((nrows * Lout + 255) / 256, 8192);
  hipLaunchKernelGGL((k_rowmat_rect<Ti, CM>), dim3(grid), dim3(256), 0, s, in, out, M, sign, nrows, Lin, Lout, vol);
  return hipGetLastError();
}
template hipError_t launch_rowmat_rect<float, true>(const cpx<float>*, cpx<double>*, const cpx<double>*, double,
                                                    long long, int, int, int, hipStream_t);
template hipError_t launch_rowmat_rect<double, true>(const cpx<double>*, cpx<double>*, const cpx<double>*, double,
                                                     long long, int, int, int, hipStream_t);
template hipError_t launch_rowmat_rect<double, false>(const cpx<double>*, cpx<double>*, const cpx<double>*, double,
                                                      long long, int, int, int, hipStream_t);
