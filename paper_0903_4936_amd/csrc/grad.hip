// Gradients of a solve X = D_W^{-1} B with respect to the gauge links
// (derived from Eq. (1) of Sec. 2), FP64.  With Lam = D_W^{-H} G the
// gradient of the loss is that of f(U) = -Re <Lam, D_W(U) X>; for a link
// U_mu(n) (gradient convention g = dl/dRe U + i dl/dIm U):
//
//   hopping:  g += kappa (conj(A) + B^T),
//             A_ab = sum_{l, alpha} conj(Lam_{alpha a l}(n)) ((1 - gamma_mu) X(n + mu))_{alpha b l},
//             B_ab = sum_{l, alpha} conj(Lam_{alpha a l}(n + mu)) ((1 + gamma_mu) X(n))_{alpha b l};
//   clover:   with F = (Q - Q^dagger) / (8i), Q the sum of the four leaves,
//             and W^{mu nu} = kappa c_SW / (4i) (K + K^H),
//             K_ab = sum_{l, alpha, beta} conj(Lam_{alpha a l}) ((i/2) sigma_{mu nu})_{alpha beta} X_{beta b l},
//             every leaf through the link contributes (the link is the
//             bottom edge of the plaquette at n and the top edge of the one
//             at n - nu, in each plane (mu, nu); a leaf at corner c is that
//             plaquette traversed counter-clockwise from c):
//             link as a factor:          g += M^H,  M = (links after) W^T(c) (links before),
//             link daggered in the loop: g += M.
//   For nu < mu the plane is the (nu, mu) plane seen in the other
//   orientation: its leaves are the daggered ones, and W changes sign.
#include "bkwd_internal.h"

namespace {

constexpr int kGradThreads = 256;

// gamma_1..gamma_4 of Sec. 2: one non-zero per row, at column gcol[mu][row]
// with value gval[mu][row] (re, im).
__constant__ int gcol[4][4] = {{3, 2, 1, 0}, {3, 2, 1, 0}, {2, 3, 0, 1}, {0, 1, 2, 3}};
__constant__ double gval[4][4][2] = {
    {{0, -1}, {0, -1}, {0, 1}, {0, 1}},    // gamma_1
    {{-1, 0}, {1, 0}, {1, 0}, {-1, 0}},    // gamma_2
    {{0, -1}, {0, 1}, {0, 1}, {0, -1}},    // gamma_3
    {{1, 0}, {1, 0}, {-1, 0}, {-1, 0}}};   // gamma_4

struct M3 {
  cpx<double> e[3][3];
};

__device__ __forceinline__ M3 zero3() {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[i][j] = mk(0.0, 0.0);
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
      for (int k = 0; k < 3; ++k) cmac(s, a.e[i][k], b.e[k][j]);
      r.e[i][j] = s;
    }
  return r;
}

__device__ __forceinline__ M3 dag(const M3& a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[i][j] = conj(a.e[j][i]);
  return r;
}

__device__ __forceinline__ void add_to(M3& acc, const M3& a) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc.e[i][j] = acc.e[i][j] + a.e[i][j];
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

struct Site {
  int c[4];
};

__device__ __forceinline__ Site coords(const Geom& g, int site) {
  Site s;
  s.c[0] = site % g.lx;
  s.c[1] = (site / g.lx) % g.ly;
  s.c[2] = (site / (g.lx * g.ly)) % g.lz;
  s.c[3] = site / (g.lx * g.ly * g.lz);
  return s;
}

// flat index of n + a mu_hat + b nu_hat
__device__ __forceinline__ int moved(const Geom& g, Site n, int mu, int a, int nu, int b) {
  const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
  n.c[mu] = wrap(n.c[mu] + a, ext[mu]);
  n.c[nu] = wrap(n.c[nu] + b, ext[nu]);
  return n.c[0] + g.lx * (n.c[1] + g.ly * (n.c[2] + g.lz * n.c[3]));
}

__device__ __forceinline__ M3 load_link(const cpx<double>* __restrict__ canon, int vol, int mu, int site) {
  M3 r;
  const cpx<double>* p = canon + ((long long)mu * vol + site) * 9;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[i][j] = p[i * 3 + j];
  return r;
}

// W^T of plane p at a site, times sign
__device__ __forceinline__ M3 load_wt(const cpx<double>* __restrict__ w, int vol, int p, int site, double sign) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[j][i] = sign * w[((long long)p * 9 + i * 3 + j) * vol + site];
  return r;
}

// plane index of mu < nu: (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__device__ __forceinline__ int plane_of(int mu, int nu) {
  const int a = mu < nu ? mu : nu, b = mu < nu ? nu : mu;
  return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

__device__ __forceinline__ long long elem(int site, int spin, int col, int l, int L) {
  return (((long long)site * 4 + spin) * 3 + col) * L + l;
}

// W^{mu nu}(n) = kc / (4i) (K + K^H), one thread per (site, plane)
__global__ void __launch_bounds__(kGradThreads) k_clover_w(const cpx<double>* __restrict__ x,
                                                           const cpx<double>* __restrict__ lam, cpx<double>* w, Geom g,
                                                           int L, double kc) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 6LL * g.vol) return;
  const int p = (int)(idx / g.vol);
  const int site = (int)(idx - (long long)p * g.vol);
  const int mus[6] = {0, 0, 0, 1, 1, 2}, nus[6] = {1, 2, 3, 2, 3, 3};
  const int mu = mus[p], nu = nus[p];
  // (i/2) sigma_{mu nu} = (i/2) gamma_mu gamma_nu (mu != nu): one non-zero per row
  int scol[4];
  cpx<double> sval[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int c1 = gcol[mu][r];
    scol[r] = gcol[nu][c1];
    const cpx<double> v = mk(gval[mu][r][0], gval[mu][r][1]) * mk(gval[nu][c1][0], gval[nu][c1][1]);
    sval[r] = mk(-0.5 * v.im, 0.5 * v.re);  // (i/2) v
  }
  M3 K = zero3();
  for (int l = 0; l < L; ++l) {
#pragma unroll
    for (int al = 0; al < 4; ++al) {
      const int be = scol[al];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const cpx<double> cl = conj(lam[elem(site, al, a, l, L)]) * sval[al];
#pragma unroll
        for (int b = 0; b < 3; ++b) cmac(K.e[a][b], cl, x[elem(site, be, b, l, L)]);
      }
    }
  }
  // kc / (4i) = -i kc / 4
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const cpx<double> h = K.e[a][b] + conj(K.e[b][a]);
      w[((long long)p * 9 + a * 3 + b) * g.vol + site] = mk(0.25 * kc * h.im, -0.25 * kc * h.re);
    }
}

// one thread per link (rho, m)
__global__ void __launch_bounds__(kGradThreads) k_link_force(const cpx<double>* __restrict__ x,
                                                             const cpx<double>* __restrict__ lam,
                                                             const cpx<double>* __restrict__ canon,
                                                             const cpx<double>* __restrict__ w, cpx<double>* grad,
                                                             Geom g, int L, double kappa) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 4LL * g.vol) return;
  const int rho = (int)(idx / g.vol);
  const int m = (int)(idx - (long long)rho * g.vol);
  const Site n = coords(g, m);
  const int mp = moved(g, n, rho, 1, rho, 0);  // m + rho

  // hopping part
  M3 A = zero3(), B = zero3();
  for (int l = 0; l < L; ++l) {
#pragma unroll
    for (int al = 0; al < 4; ++al) {
      const int gc = gcol[rho][al];
      const cpx<double> gv = mk(gval[rho][al][0], gval[rho][al][1]);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        // ((1 - gamma) X(m + rho))_{alpha b} and ((1 + gamma) X(m))_{alpha b}
        const cpx<double> xf = x[elem(mp, al, b, l, L)], xfg = x[elem(mp, gc, b, l, L)];
        const cpx<double> xb = x[elem(m, al, b, l, L)], xbg = x[elem(m, gc, b, l, L)];
        const cpx<double> y1 = xf - gv * xfg, y2 = xb + gv * xbg;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          cmac_conj(A.e[a][b], lam[elem(m, al, a, l, L)], y1);
          cmac_conj(B.e[a][b], lam[elem(mp, al, a, l, L)], y2);
        }
      }
    }
  }
  M3 gr;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) gr.e[a][b] = kappa * (conj(A.e[a][b]) + B.e[b][a]);

  // clover part
  if (w != nullptr) {
    M3 P = zero3(), N = zero3();  // sums of the M of undaggered and daggered occurrences
    for (int nu = 0; nu < 4; ++nu) {
      if (nu == rho) continue;
      const int p = plane_of(rho, nu);
      const double sign = rho < nu ? 1.0 : -1.0;
      const int s_pn = moved(g, n, rho, 1, nu, 1);    // m + rho + nu
      const int s_n = moved(g, n, rho, 0, nu, 1);     // m + nu
      const int s_mn = moved(g, n, rho, 0, nu, -1);   // m - nu
      const int s_pmn = moved(g, n, rho, 1, nu, -1);  // m + rho - nu
      const M3 u_nu_p = load_link(canon, g.vol, nu, mp);       // U_nu(m + rho)
      const M3 u_rho_n = load_link(canon, g.vol, rho, s_n);    // U_rho(m + nu)
      const M3 u_nu_m = load_link(canon, g.vol, nu, m);        // U_nu(m)
      const M3 u_nu_mn = load_link(canon, g.vol, nu, s_mn);    // U_nu(m - nu)
      const M3 u_rho_mn = load_link(canon, g.vol, rho, s_mn);  // U_rho(m - nu)
      const M3 u_nu_pmn = load_link(canon, g.vol, nu, s_pmn);  // U_nu(m + rho - nu)
      const M3 wt_m = load_wt(w, g.vol, p, m, sign);
      const M3 wt_p = load_wt(w, g.vol, p, mp, sign);
      // plaquette at m (link undaggered): loop m -> m+rho -> m+rho+nu -> m+nu -> m
      const M3 d_rho_n = dag(u_rho_n), d_nu_m = dag(u_nu_m);
      const M3 tail = mul(d_rho_n, d_nu_m);        // m+rho+nu -> m
      const M3 staple = mul(u_nu_p, tail);         // m+rho -> m
      add_to(P, mul(staple, wt_m));
      add_to(P, mul(wt_p, staple));
      add_to(P, mul(mul(u_nu_p, load_wt(w, g.vol, p, s_pn, sign)), tail));
      add_to(P, mul(mul(mul(u_nu_p, d_rho_n), load_wt(w, g.vol, p, s_n, sign)), d_nu_m));
      // plaquette at m - nu (link daggered): loop m-nu -> m-nu+rho -> m+rho -> m -> m-nu
      const M3 d_nu_mn = dag(u_nu_mn);
      const M3 head = mul(u_rho_mn, u_nu_pmn);     // m-nu -> m+rho
      const M3 staple2 = mul(d_nu_mn, head);       // m -> m+rho
      add_to(N, mul(wt_m, staple2));
      add_to(N, mul(mul(d_nu_mn, load_wt(w, g.vol, p, s_mn, sign)), head));
      add_to(N, mul(mul(mul(d_nu_mn, u_rho_mn), load_wt(w, g.vol, p, s_pmn, sign)), u_nu_pmn));
      add_to(N, mul(staple2, wt_p));
    }
    add_to(gr, dag(P));
    add_to(gr, N);
  }
  cpx<double>* out = grad + ((long long)rho * g.vol + m) * 9;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) out[a * 3 + b] = gr.e[a][b];
}

}  // namespace

hipError_t launch_clover_w(const LatticeImpl& lat, int L, const cpx<double>* x, const cpx<double>* lam, double kc,
                           cpx<double>* w, hipStream_t s) {
  const long long n = 6LL * lat.g.vol;
  const int grid = (int)((n + kGradThreads - 1) / kGradThreads);
  hipLaunchKernelGGL(k_clover_w, dim3(grid), dim3(kGradThreads), 0, s, x, lam, w, lat.g, L, kc);
  return hipGetLastError();
}

hipError_t launch_link_force(const LatticeImpl& lat, int L, const cpx<double>* x, const cpx<double>* lam,
                             const cpx<double>* w, cpx<double>* grad, hipStream_t s) {
  const long long n = 4LL * lat.g.vol;
  const int grid = (int)((n + kGradThreads - 1) / kGradThreads);
  hipLaunchKernelGGL(k_link_force, dim3(grid), dim3(kGradThreads), 0, s, x, lam, lat.canon, w, grad, lat.g, L,
                     lat.kappa);
  return hipGetLastError();
}
