// Multi-right-hand-side O(a)-improved Wilson-Dirac operator (Sec. 2, Eq. (1)):
//
//   (D X)(n) = A(n) X(n) - kappa sum_mu [ (1 - gamma_mu) U_mu(n) X(n + mu)
//                                        + (1 + gamma_mu) U_mu^dagger(n - mu) X(n - mu) ]
//
// for every column of an N x L block stored [site][spin][colour][rhs].
// One thread computes one (site, rhs) pair; the L threads of a site read the
// same gauge links and clover blocks, so each link fetched from memory is
// reused for all L right-hand sides.  Each hop projects the neighbour's four
// spin components onto two (the projectors 1 -/+ gamma_mu have rank 2),
// multiplies the two colour vectors by the link and rebuilds four.
// D^dagger = gamma_5 D gamma_5 swaps the two projectors.
#include "bkwd_internal.h"

#include <algorithm>

namespace {

constexpr int kThreads = 256;

enum EpiMode { EPI_PLAIN = 0, EPI_TRACE = 1, EPI_RESID = 2 };

template <typename T>
struct DslashArgs {
  const cpx<T>* in;
  cpx<T>* out;
  const cpx<T>* links;       // [V][4][3][3]
  const cpx<T>* links_c;     // [V][4][2][3] (compressed) or null
  const T* clover;           // [V][2][36]
  const cpx<T>* b;           // EPI_RESID: right-hand side
  double* partials;          // per-workgroup partial sums
  const Control* ctl;
  Geom g;
  int L;
  T kappa;
};

template <typename T>
struct Half {
  cpx<T> h[2][3];
};

// rows 0..2 of a link; compressed links rebuild row 2 = conj(row0 x row1)
template <typename T, bool COMP>
__device__ __forceinline__ void load_link(const DslashArgs<T>& a, int site, int mu, cpx<T> u[3][3]) {
  if constexpr (COMP) {
    const cpx<T>* p = a.links_c + ((long long)site * 4 + mu) * 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      u[0][k] = p[k];
      u[1][k] = p[3 + k];
    }
    u[2][0] = conj(u[0][1] * u[1][2] - u[0][2] * u[1][1]);
    u[2][1] = conj(u[0][2] * u[1][0] - u[0][0] * u[1][2]);
    u[2][2] = conj(u[0][0] * u[1][1] - u[0][1] * u[1][0]);
  } else {
    const cpx<T>* p = a.links + ((long long)site * 4 + mu) * 9;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) u[i][k] = p[i * 3 + k];
  }
}

// spin component s (all 3 colours) of column l at site
template <typename T>
__device__ __forceinline__ void load_spin(const cpx<T>* __restrict__ f, int site, int s, int l, int L,
                                          cpx<T> v[3]) {
  const cpx<T>* p = f + ((long long)site * 12 + s * 3) * L + l;
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = p[c * L];
}

// Projection with (1 - gamma_mu) (MINUS) or (1 + gamma_mu) onto two colour
// vectors, gamma matrices of Sec. 2 (0-based spins):
//   x: h1 = psi0 -/+ ... see the case bodies; t-direction projectors are
//   diagonal, so only two spin components are read.
template <typename T, int MU, bool MINUS>
__device__ __forceinline__ void project(const cpx<T>* __restrict__ f, int site, int l, int L, Half<T>& h) {
  cpx<T> a[3], b[3];
  if constexpr (MU == 3) {
    // (1 - gamma_4) = diag(0,0,2,2), (1 + gamma_4) = diag(2,2,0,0)
    load_spin(f, site, MINUS ? 2 : 0, l, L, a);
    load_spin(f, site, MINUS ? 3 : 1, l, L, b);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      h.h[0][c] = T(2) * a[c];
      h.h[1][c] = T(2) * b[c];
    }
  } else {
    cpx<T> p0[3], p1[3];
    load_spin(f, site, 0, l, L, p0);
    load_spin(f, site, 1, l, L, p1);
    if constexpr (MU == 0) {
      // minus: h1 = psi0 + i psi3, h2 = psi1 + i psi2;  plus: -i instead of +i
      load_spin(f, site, 3, l, L, a);
      load_spin(f, site, 2, l, L, b);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        h.h[0][c] = MINUS ? p0[c] + times_i(a[c]) : p0[c] + times_mi(a[c]);
        h.h[1][c] = MINUS ? p1[c] + times_i(b[c]) : p1[c] + times_mi(b[c]);
      }
    } else if constexpr (MU == 1) {
      // minus: h1 = psi0 + psi3, h2 = psi1 - psi2;  plus: h1 = psi0 - psi3, h2 = psi1 + psi2
      load_spin(f, site, 3, l, L, a);
      load_spin(f, site, 2, l, L, b);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        h.h[0][c] = MINUS ? p0[c] + a[c] : p0[c] - a[c];
        h.h[1][c] = MINUS ? p1[c] - b[c] : p1[c] + b[c];
      }
    } else {
      // MU == 2. minus: h1 = psi0 + i psi2, h2 = psi1 - i psi3;  plus: signs of i flipped
      load_spin(f, site, 2, l, L, a);
      load_spin(f, site, 3, l, L, b);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        h.h[0][c] = MINUS ? p0[c] + times_i(a[c]) : p0[c] + times_mi(a[c]);
        h.h[1][c] = MINUS ? p1[c] + times_mi(b[c]) : p1[c] + times_i(b[c]);
      }
    }
  }
}

// acc += reconstruction of the two multiplied colour vectors g into 4 spins
template <typename T, int MU, bool MINUS>
__device__ __forceinline__ void reconstruct(cpx<T> acc[4][3], const Half<T>& g) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cpx<T> g1 = g.h[0][c], g2 = g.h[1][c];
    if constexpr (MU == 3) {
      if constexpr (MINUS) {
        acc[2][c] = acc[2][c] + g1;
        acc[3][c] = acc[3][c] + g2;
      } else {
        acc[0][c] = acc[0][c] + g1;
        acc[1][c] = acc[1][c] + g2;
      }
    } else {
      acc[0][c] = acc[0][c] + g1;
      acc[1][c] = acc[1][c] + g2;
      if constexpr (MU == 0) {
        // minus: rows 2,3 = -i g2, -i g1;  plus: +i g2, +i g1
        acc[2][c] = acc[2][c] + (MINUS ? times_mi(g2) : times_i(g2));
        acc[3][c] = acc[3][c] + (MINUS ? times_mi(g1) : times_i(g1));
      } else if constexpr (MU == 1) {
        // minus: rows 2,3 = -g2, g1;  plus: g2, -g1
        acc[2][c] = MINUS ? acc[2][c] - g2 : acc[2][c] + g2;
        acc[3][c] = MINUS ? acc[3][c] + g1 : acc[3][c] - g1;
      } else {
        // minus: rows 2,3 = -i g1, +i g2;  plus: +i g1, -i g2
        acc[2][c] = acc[2][c] + (MINUS ? times_mi(g1) : times_i(g1));
        acc[3][c] = acc[3][c] + (MINUS ? times_i(g2) : times_mi(g2));
      }
    }
  }
}

// One hop.  FWD: from n + mu with U_mu(n); else from n - mu with U_mu(n-mu)^dagger.
// The forward projector is (1 - gamma_mu) for D and (1 + gamma_mu) for D^dagger.
template <typename T, int MU, bool FWD, bool DAG, bool COMP>
__device__ __forceinline__ void hop(const DslashArgs<T>& a, int nbr, int link_site, int l, cpx<T> acc[4][3]) {
  constexpr bool MINUS = (FWD != DAG);
  Half<T> h, g;
  project<T, MU, MINUS>(a.in, nbr, l, a.L, h);
  cpx<T> u[3][3];
  load_link<T, COMP>(a, link_site, MU, u);
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cpx<T> v = mk(T(0), T(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if constexpr (FWD) cmac(v, u[i][k], h.h[s][k]);
        else cmac_conj(v, u[k][i], h.h[s][k]);
      }
      g.h[s][i] = v;
    }
  reconstruct<T, MU, MINUS>(acc, g);
}

// y = A_blk x for one packed Hermitian 6x6 block (6 real diagonals, then the
// 15 complex upper entries in row-major order).
template <typename T>
__device__ __forceinline__ void herm6(const T* __restrict__ c, const cpx<T> x[6], cpx<T> y[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) y[i] = c[i] * x[i];
  int k = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j, ++k) {
      const cpx<T> aij = mk(c[6 + 2 * k], c[7 + 2 * k]);
      cmac(y[i], aij, x[j]);
      cmac_conj(y[j], aij, x[i]);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// (D X) at one (site, column); the epilogue mode decides what is stored and
// which partial sums are accumulated.
template <typename T, bool DAG, bool COMP, int EPI>
__device__ __forceinline__ void site_rhs(const DslashArgs<T>& a, int site, int l, double& e0, double& e1,
                                         double& e2) {
  const Geom g = a.g;
  const int L = a.L;
  int r = site;
  const int x = r % g.lx; r /= g.lx;
  const int y = r % g.ly; r /= g.ly;
  const int z = r % g.lz;
  const int t = r / g.lz;
  const int sx = 1, sy = g.lx, sz = g.lx * g.ly, st = g.lx * g.ly * g.lz;
  const int xp = (x + 1 == g.lx) ? site - (g.lx - 1) * sx : site + sx;
  const int xm = (x == 0) ? site + (g.lx - 1) * sx : site - sx;
  const int yp = (y + 1 == g.ly) ? site - (g.ly - 1) * sy : site + sy;
  const int ym = (y == 0) ? site + (g.ly - 1) * sy : site - sy;
  const int zp = (z + 1 == g.lz) ? site - (g.lz - 1) * sz : site + sz;
  const int zm = (z == 0) ? site + (g.lz - 1) * sz : site - sz;
  const int tp = (t + 1 == g.lt) ? site - (g.lt - 1) * st : site + st;
  const int tm = (t == 0) ? site + (g.lt - 1) * st : site - st;

  cpx<T> acc[4][3];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[s][c] = mk(T(0), T(0));

  hop<T, 0, true, DAG, COMP>(a, xp, site, l, acc);
  hop<T, 0, false, DAG, COMP>(a, xm, xm, l, acc);
  hop<T, 1, true, DAG, COMP>(a, yp, site, l, acc);
  hop<T, 1, false, DAG, COMP>(a, ym, ym, l, acc);
  hop<T, 2, true, DAG, COMP>(a, zp, site, l, acc);
  hop<T, 2, false, DAG, COMP>(a, zm, zm, l, acc);
  hop<T, 3, true, DAG, COMP>(a, tp, site, l, acc);
  hop<T, 3, false, DAG, COMP>(a, tm, tm, l, acc);

  // site-local term on phi_+- = psi_{0,1} +- psi_{2,3}
  cpx<T> psi[4][3];
#pragma unroll
  for (int s = 0; s < 4; ++s) load_spin(a.in, site, s, l, L, psi[s]);
  cpx<T> pp[6], pm[6], qp[6], qm[6];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pp[3 * s + c] = psi[s][c] + psi[s + 2][c];
      pm[3 * s + c] = psi[s][c] - psi[s + 2][c];
    }
  const T* cl = a.clover + (long long)site * 72;
  herm6(cl, pp, qp);
  herm6(cl + 36, pm, qm);

  const T kap = a.kappa;
  cpx<T>* op = a.out + (long long)site * 12 * L + l;
  const cpx<T>* bp = (EPI == EPI_RESID) ? a.b + (long long)site * 12 * L + l : nullptr;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cpx<T> loc = (s < 2) ? qp[3 * s + c] + qm[3 * s + c] : qp[3 * (s - 2) + c] - qm[3 * (s - 2) + c];
      cpx<T> res = mk(loc.re - kap * acc[s][c].re, loc.im - kap * acc[s][c].im);
      if constexpr (EPI == EPI_TRACE) {
        // Tr(Y^H X) and Tr(Y^H Y) with Y = D X
        const cpx<T> xin = psi[s][c];
        e0 += (double)res.re * (double)xin.re + (double)res.im * (double)xin.im;
        e1 += (double)res.re * (double)xin.im - (double)res.im * (double)xin.re;
        e2 += (double)res.re * (double)res.re + (double)res.im * (double)res.im;
      } else if constexpr (EPI == EPI_RESID) {
        const cpx<T> bv = bp[(s * 3 + c) * L];
        res = bv - res;
        e0 += (double)res.re * (double)res.re + (double)res.im * (double)res.im;
        e1 += (double)bv.re * (double)bv.re + (double)bv.im * (double)bv.im;
      }
      op[(s * 3 + c) * L] = res;
    }
}

// Grid-stride over (site, column) pairs.  For EPI_RESID the stride is a
// multiple of L, so every thread keeps one column.
template <typename T, bool DAG, bool COMP, int EPI>
__global__ void __launch_bounds__(kThreads) k_dslash(DslashArgs<T> a) {
  if (a.ctl != nullptr && a.ctl->state != ST_RUNNING) return;
  const int L = a.L;
  const long long total = (long long)a.g.vol * L;
  const long long stride = (long long)gridDim.x * kThreads;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;  // epilogue partial sums
  for (long long base = (long long)blockIdx.x * kThreads; base < total; base += stride) {
    const long long tid = base + threadIdx.x;
    if (tid < total) {
      const int site = (int)(tid / L);
      const int l = (int)(tid - (long long)site * L);
      site_rhs<T, DAG, COMP, EPI>(a, site, l, e0, e1, e2);
    }
  }

  if constexpr (EPI == EPI_TRACE) {
    __shared__ double red[kThreads / 64][3];
    e0 = wave_sum(e0);
    e1 = wave_sum(e1);
    e2 = wave_sum(e2);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
      red[w][0] = e0;
      red[w][1] = e1;
      red[w][2] = e2;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      double v = 0.0;
      if (threadIdx.x < 3)
        for (int k = 0; k < kThreads / 64; ++k) v += red[k][threadIdx.x];
      a.partials[(long long)blockIdx.x * 4 + threadIdx.x] = v;
    }
  } else if constexpr (EPI == EPI_RESID) {
    // per-column sums: thread of global index tid holds column tid % L
    __shared__ double red[2][kThreads];
    red[0][threadIdx.x] = e0;
    red[1][threadIdx.x] = e1;
    __syncthreads();
    if (threadIdx.x < L) {
      const long long base = (long long)blockIdx.x * kThreads;
      const int first = (int)((L - (int)(base % L) + threadIdx.x) % L);  // first local index with column tid
      double v0 = 0.0, v1 = 0.0;
      for (int k = first; k < kThreads; k += L) {
        v0 += red[0][k];
        v1 += red[1][k];
      }
      a.partials[(long long)blockIdx.x * 2 * L + threadIdx.x] = v0;
      a.partials[(long long)blockIdx.x * 2 * L + L + threadIdx.x] = v1;
    }
  }
}

template <typename T>
DslashArgs<T> make_args(const LatticeImpl& lat, int L, const cpx<T>* in, cpx<T>* out, const Control* ctl);

template <>
DslashArgs<double> make_args<double>(const LatticeImpl& lat, int L, const cpx<double>* in, cpx<double>* out,
                                     const Control* ctl) {
  DslashArgs<double> a{};
  a.in = in; a.out = out; a.links = lat.links64; a.links_c = nullptr; a.clover = lat.clover64;
  a.ctl = ctl; a.g = lat.g; a.L = L; a.kappa = lat.kappa;
  return a;
}

template <>
DslashArgs<float> make_args<float>(const LatticeImpl& lat, int L, const cpx<float>* in, cpx<float>* out,
                                   const Control* ctl) {
  DslashArgs<float> a{};
  a.in = in; a.out = out; a.links = lat.links32; a.links_c = lat.links32c; a.clover = lat.clover32;
  a.ctl = ctl; a.g = lat.g; a.L = L; a.kappa = (float)lat.kappa;
  return a;
}

template <typename T, int EPI>
hipError_t dispatch(const DslashArgs<T>& a, int dagger, bool comp, int grid, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (comp) {
      if (dagger) hipLaunchKernelGGL((k_dslash<T, true, true, EPI>), dim3(grid), dim3(kThreads), 0, s, a);
      else hipLaunchKernelGGL((k_dslash<T, false, true, EPI>), dim3(grid), dim3(kThreads), 0, s, a);
      return hipGetLastError();
    }
  }
  if (dagger) hipLaunchKernelGGL((k_dslash<T, true, false, EPI>), dim3(grid), dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((k_dslash<T, false, false, EPI>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_dslash(const LatticeImpl& lat, int dagger, int L, const cpx<T>* in, cpx<T>* out, double* epi,
                         int* nblk_out, const Control* ctl, hipStream_t s) {
  DslashArgs<T> a = make_args<T>(lat, L, in, out, ctl);
  const long long total = (long long)lat.g.vol * L;
  const int grid = (int)((total + kThreads - 1) / kThreads);
  const bool comp = (lat.flags & 1u) && lat.links32c != nullptr;
  if (nblk_out) *nblk_out = grid;
  if (epi) {
    a.partials = epi;
    return dispatch<T, EPI_TRACE>(a, dagger, comp, grid, s);
  }
  return dispatch<T, EPI_PLAIN>(a, dagger, comp, grid, s);
}

template hipError_t launch_dslash<double>(const LatticeImpl&, int, int, const cpx<double>*, cpx<double>*, double*,
                                          int*, const Control*, hipStream_t);
template hipError_t launch_dslash<float>(const LatticeImpl&, int, int, const cpx<float>*, cpx<float>*, double*,
                                         int*, const Control*, hipStream_t);

int residual_grid(long long vol, int L) {
  // at most kResidualBlocks workgroups, a multiple of L / gcd(L, 256)
  int g = L, b = kThreads;
  while (b) { const int t = g % b; g = b; b = t; }
  const int m = L / g;
  const long long need = (vol * L + kThreads - 1) / kThreads;
  long long grid = std::min<long long>(need, (kResidualBlocks / m) * m);
  if (grid < 1) grid = 1;
  return (int)grid;
}

hipError_t launch_residual64(const LatticeImpl& lat, int L, const cpx<double>* b, const cpx<double>* x,
                             cpx<double>* r, double* partials, int* nblk_out, hipStream_t s) {
  DslashArgs<double> a = make_args<double>(lat, L, x, r, nullptr);
  a.b = b;
  a.partials = partials;
  const int grid = residual_grid(lat.g.vol, L);
  if (nblk_out) *nblk_out = grid;
  hipLaunchKernelGGL((k_dslash<double, false, false, EPI_RESID>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
