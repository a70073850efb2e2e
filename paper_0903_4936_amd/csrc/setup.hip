// Operator set-up on the device: gauge-link repacking and the site-local
// clover blocks of the O(a)-improved Wilson-Dirac operator (Sec. 2, Eq. (1)).
#include "bkwd_internal.h"

namespace {

constexpr int kSetupThreads = 256;

// canonical [4][V][3][3] -> structure of arrays [4][9][V] (FP64, FP32) and
// the two-row FP32 form [4][6][V].
__global__ void __launch_bounds__(kSetupThreads)
k_pack_links(const cpx<double>* __restrict__ canon, cpx<double>* __restrict__ l64,
             cpx<float>* __restrict__ l32, cpx<float>* __restrict__ l32c, int vol) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // (mu, site)
  if (idx >= 4LL * vol) return;
  const int mu = (int)(idx / vol);
  const int site = (int)(idx - (long long)mu * vol);
  const cpx<double>* src = canon + ((long long)mu * vol + site) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const cpx<double> u = src[k];
    const long long o = ((long long)mu * 9 + k) * vol + site;
    l64[o] = u;
    l32[o] = cast<float>(u);
  }
  if (l32c) {
#pragma unroll
    for (int k = 0; k < 6; ++k) l32c[((long long)mu * 6 + k) * vol + site] = cast<float>(src[k]);
  }
}

struct M3 {
  cpx<double> m[3][3];
};

__device__ __forceinline__ M3 load_link(const cpx<double>* __restrict__ l64, int vol, int site, int mu) {
  M3 r;
  const cpx<double>* p = l64 + (long long)mu * 9 * vol + site;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) r.m[a][b] = p[(long long)(a * 3 + b) * vol];
  return r;
}

__device__ __forceinline__ M3 dagger(const M3& a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.m[i][j] = conj(a.m[j][i]);
  return r;
}

__device__ __forceinline__ M3 mul(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<double> s = mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cmac(s, a.m[i][k], b.m[k][j]);
      r.m[i][j] = s;
    }
  return r;
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

struct Coord {
  int c[4];
};

__device__ __forceinline__ int site_of(const Geom& g, const Coord& x) {
  return x.c[0] + g.lx * (x.c[1] + g.ly * (x.c[2] + g.lz * x.c[3]));
}

// site of n + a*mu_hat + b*nu_hat
__device__ __forceinline__ int displaced(const Geom& g, Coord n, int mu, int a, int nu, int b) {
  const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
  n.c[mu] = wrap(n.c[mu] + a, ext[mu]);
  n.c[nu] = wrap(n.c[nu] + b, ext[nu]);
  return site_of(g, n);
}

// F_{mu nu}(n) = (1/4) sum of the four clover leaves' anti-Hermitian parts
// divided by 2i (Sec. 2, definition of F_{mu nu}); the leaves are the four
// plaquettes around n in the (mu, nu) plane, traversed counter-clockwise.
__device__ M3 field_strength(const cpx<double>* __restrict__ l64, const Geom& g, const Coord& n, int mu, int nu) {
  const int s0 = site_of(g, n);
  const int s_pm = displaced(g, n, mu, +1, nu, 0);    // n + mu
  const int s_pn = displaced(g, n, mu, 0, nu, +1);    // n + nu
  const int s_mm = displaced(g, n, mu, -1, nu, 0);    // n - mu
  const int s_mn = displaced(g, n, mu, 0, nu, -1);    // n - nu
  const int s_mm_pn = displaced(g, n, mu, -1, nu, +1);  // n - mu + nu
  const int s_mm_mn = displaced(g, n, mu, -1, nu, -1);  // n - mu - nu
  const int s_pm_mn = displaced(g, n, mu, +1, nu, -1);  // n + mu - nu

  const M3 umu_n = load_link(l64, g.vol, s0, mu), unu_n = load_link(l64, g.vol, s0, nu);
  // leaf 1: n -> n+mu -> n+mu+nu -> n+nu -> n
  M3 q = mul(mul(umu_n, load_link(l64, g.vol, s_pm, nu)), mul(dagger(load_link(l64, g.vol, s_pn, mu)), dagger(unu_n)));
  // leaf 2: n -> n+nu -> n-mu+nu -> n-mu -> n
  M3 p2 = mul(mul(unu_n, dagger(load_link(l64, g.vol, s_mm_pn, mu))),
              mul(dagger(load_link(l64, g.vol, s_mm, nu)), load_link(l64, g.vol, s_mm, mu)));
  // leaf 3: n -> n-mu -> n-mu-nu -> n-nu -> n
  M3 p3 = mul(mul(dagger(load_link(l64, g.vol, s_mm, mu)), dagger(load_link(l64, g.vol, s_mm_mn, nu))),
              mul(load_link(l64, g.vol, s_mm_mn, mu), load_link(l64, g.vol, s_mn, nu)));
  // leaf 4: n -> n-nu -> n-nu+mu -> n+mu -> n
  M3 p4 = mul(mul(dagger(load_link(l64, g.vol, s_mn, nu)), load_link(l64, g.vol, s_mn, mu)),
              mul(load_link(l64, g.vol, s_pm_mn, nu), dagger(umu_n)));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) q.m[i][j] = q.m[i][j] + p2.m[i][j] + p3.m[i][j] + p4.m[i][j];
  // F = (Q - Q^dagger) / (8 i) = -i (Q - Q^dagger) / 8
  M3 f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const cpx<double> d = q.m[i][j] - conj(q.m[j][i]);
      f.m[i][j] = 0.125 * times_mi(d);
    }
  return f;
}

// The site-local term 1 - kappa csw sum_{mu,nu} (i/2) sigma_{mu nu} F_{mu nu}
// of Eq. (1) is block-diagonal for the spin combinations
// phi_+- = psi_{spins 0,1} +- psi_{spins 2,3}.  On each block (index
// 3*s + colour, s = 0, 1) it is the Hermitian 6x6 matrix
//   A_+- = 1 + kappa csw [ sigma_1 (x) G1 + sigma_2 (x) G2 + sigma_3 (x) G3 ]
// with Pauli matrices sigma_k and (1-based planes)
//   G1 = F23 +- F14,  G2 = -F13 +- F24,  G3 = F12 +- F34,
// which follows from the gamma matrices of Sec. 2.  Each block is stored
// halved (the back-transform to psi then needs no factor 1/2) and packed as
// 6 real diagonal entries followed by the 15 complex entries above the
// diagonal in row-major order: 36 reals per block, 72 per site, stored as a
// structure of small vectors over sites.
__global__ void __launch_bounds__(kSetupThreads)
k_clover_build(const cpx<double>* __restrict__ l64, double* __restrict__ c64, float* __restrict__ c32,
               Geom g, double kc) {
  const int site = blockIdx.x * blockDim.x + threadIdx.x;
  if (site >= g.vol) return;
  Coord n;
  int r = site;
  n.c[0] = r % g.lx; r /= g.lx;
  n.c[1] = r % g.ly; r /= g.ly;
  n.c[2] = r % g.lz;
  n.c[3] = r / g.lz;

  const M3 f01 = field_strength(l64, g, n, 0, 1);
  const M3 f02 = field_strength(l64, g, n, 0, 2);
  const M3 f03 = field_strength(l64, g, n, 0, 3);
  const M3 f12 = field_strength(l64, g, n, 1, 2);
  const M3 f13 = field_strength(l64, g, n, 1, 3);
  const M3 f23 = field_strength(l64, g, n, 2, 3);

  for (int blk = 0; blk < 2; ++blk) {
    const double sg = blk == 0 ? 1.0 : -1.0;
    cpx<double> A[6][6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const cpx<double> G1 = f12.m[a][b] + sg * f03.m[a][b];
        const cpx<double> G2 = -f02.m[a][b] + sg * f13.m[a][b];
        const cpx<double> G3 = f01.m[a][b] + sg * f23.m[a][b];
        const double d = (a == b) ? 1.0 : 0.0;
        A[a][b] = mk(d, 0.0) + kc * G3;
        A[a][3 + b] = kc * (G1 - times_i(G2));
        A[3 + a][b] = kc * (G1 + times_i(G2));
        A[3 + a][3 + b] = mk(d, 0.0) - kc * G3;
      }
    // real number r (0..71) of the site: FP64 pair r/2 of [36][V][2],
    // FP32 four-vector r/4 of [18][V][4]
    auto put = [&](int r, double v) {
      c64[((long long)(r >> 1) * g.vol + site) * 2 + (r & 1)] = v;
      if (c32) c32[((long long)(r >> 2) * g.vol + site) * 4 + (r & 3)] = (float)v;
    };
    const int base = blk * 36;
    for (int i = 0; i < 6; ++i) put(base + i, 0.5 * A[i][i].re);
    int k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j, ++k) {
        put(base + 6 + 2 * k, 0.5 * A[i][j].re);
        put(base + 7 + 2 * k, 0.5 * A[i][j].im);
      }
  }
}

// Inverse of the site-local term, in the same packed form.  The site-local
// term acts as A_+ on phi_+ and A_- on phi_-, so its inverse acts as A_+^{-1}
// and A_-^{-1}; with the blocks stored halved (S = A / 2) the stored inverse
// blocks are A^{-1} / 2 = S^{-1} / 4.  Each 6 x 6 block is inverted in FP64 by
// Gauss-Jordan elimination with partial pivoting (one thread per site).
__global__ void __launch_bounds__(kSetupThreads)
k_clover_inverse(const double* __restrict__ c64, double* __restrict__ i64, float* __restrict__ i32, int vol) {
  const int site = blockIdx.x * blockDim.x + threadIdx.x;
  if (site >= vol) return;
  auto get = [&](int r) { return c64[((long long)(r >> 1) * vol + site) * 2 + (r & 1)]; };
  auto put = [&](int r, double v) {
    i64[((long long)(r >> 1) * vol + site) * 2 + (r & 1)] = v;
    i32[((long long)(r >> 2) * vol + site) * 4 + (r & 3)] = (float)v;
  };
  for (int blk = 0; blk < 2; ++blk) {
    const int base = blk * 36;
    cpx<double> a[6][6], inv[6][6];
    for (int i = 0; i < 6; ++i) {
      a[i][i] = mk(get(base + i), 0.0);
      for (int j = 0; j < 6; ++j) inv[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
    }
    int k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j, ++k) {
        a[i][j] = mk(get(base + 6 + 2 * k), get(base + 7 + 2 * k));
        a[j][i] = conj(a[i][j]);
      }
    for (int c = 0; c < 6; ++c) {
      int piv = c;
      double best = a[c][c].re * a[c][c].re + a[c][c].im * a[c][c].im;
      for (int r = c + 1; r < 6; ++r) {
        const double m = a[r][c].re * a[r][c].re + a[r][c].im * a[r][c].im;
        if (m > best) {
          best = m;
          piv = r;
        }
      }
      if (piv != c)
        for (int j = 0; j < 6; ++j) {
          const cpx<double> t = a[c][j];
          a[c][j] = a[piv][j];
          a[piv][j] = t;
          const cpx<double> u = inv[c][j];
          inv[c][j] = inv[piv][j];
          inv[piv][j] = u;
        }
      const cpx<double> d = a[c][c];
      const double dn = d.re * d.re + d.im * d.im;
      const cpx<double> di = mk(d.re / dn, -d.im / dn);
      for (int j = 0; j < 6; ++j) {
        a[c][j] = a[c][j] * di;
        inv[c][j] = inv[c][j] * di;
      }
      for (int r = 0; r < 6; ++r) {
        if (r == c) continue;
        const cpx<double> f = a[r][c];
        for (int j = 0; j < 6; ++j) {
          a[r][j] = a[r][j] - f * a[c][j];
          inv[r][j] = inv[r][j] - f * inv[c][j];
        }
      }
    }
    // S^{-1} / 4, Hermitian: diagonal reals and the upper triangle
    for (int i = 0; i < 6; ++i) put(base + i, 0.25 * inv[i][i].re);
    k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j, ++k) {
        put(base + 6 + 2 * k, 0.25 * inv[i][j].re);
        put(base + 7 + 2 * k, 0.25 * inv[i][j].im);
      }
  }
}

}  // namespace

hipError_t launch_pack_links(const LatticeImpl& lat, hipStream_t s) {
  const long long n = 4LL * lat.g.vol;
  const int grid = (int)((n + kSetupThreads - 1) / kSetupThreads);
  hipLaunchKernelGGL(k_pack_links, dim3(grid), dim3(kSetupThreads), 0, s, lat.canon, lat.links64, lat.links32,
                     lat.links32c, lat.g.vol);
  return hipGetLastError();
}

hipError_t launch_clover_build(const LatticeImpl& lat, hipStream_t s) {
  const int grid = (lat.g.vol + kSetupThreads - 1) / kSetupThreads;
  hipLaunchKernelGGL(k_clover_build, dim3(grid), dim3(kSetupThreads), 0, s, lat.links64, lat.clover64,
                     lat.clover32, lat.g, lat.kappa * lat.csw);
  return hipGetLastError();
}

// FP64 clover blocks for an arbitrary kappa * csw into caller memory
// (kc = 1 gives the blocks of 1 - C with C = sum (i/2) sigma F, used by the
// gradient with respect to c_SW)
hipError_t launch_clover_build_into(const LatticeImpl& lat, double* c64, double kc, hipStream_t s) {
  const int grid = (lat.g.vol + kSetupThreads - 1) / kSetupThreads;
  hipLaunchKernelGGL(k_clover_build, dim3(grid), dim3(kSetupThreads), 0, s, lat.links64, c64, (float*)nullptr, lat.g,
                     kc);
  return hipGetLastError();
}

// inverse of the site-local term (packed like the clover blocks) into caller memory
hipError_t launch_clover_inverse(const LatticeImpl& lat, double* i64, float* i32, hipStream_t s) {
  const int grid = (lat.g.vol + kSetupThreads - 1) / kSetupThreads;
  hipLaunchKernelGGL(k_clover_inverse, dim3(grid), dim3(kSetupThreads), 0, s, lat.clover64, i64, i32, lat.g.vol);
  return hipGetLastError();
}
