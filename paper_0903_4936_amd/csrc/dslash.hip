// Multi-right-hand-side O(a)-improved Wilson-Dirac operator (Sec. 2, Eq. (1)):
//
//   (D X)(n) = A(n) X(n) - kappa sum_mu [ (1 - gamma_mu) U_mu(n) X(n + mu)
//                                        + (1 + gamma_mu) U_mu^dagger(n - mu) X(n - mu) ]
//
// for every column of an N x L block.  One thread computes one (site, rhs)
// pair; the L threads of a site read the same gauge links and clover blocks,
// so each link fetched from memory serves all L right-hand sides.  Each hop
// projects the neighbour's four spin components onto two (the projectors
// 1 -/+ gamma_mu have rank 2), multiplies the two colour vectors by the link
// and rebuilds four.  D^dagger = gamma_5 D gamma_5 swaps the two projectors.
//
// Memory layouts (every wave-wide access below is a contiguous run):
//   links   [mu][3x3 entry][site]          (structure of arrays)
//   clover  [vector q][site], q over the 72 reals of a site's two blocks
//   blocks  site-major [site][spin*3+colour][rhs] (the ABI layout), or
//           component-major [spin*3+colour][site][rhs] (Krylov workspace):
//           one spin-colour component of consecutive (site, rhs) threads is
//           then one contiguous run.
#include "bkwd_internal.h"
#include "mfma16.h"

#include <algorithm>
#include <type_traits>

namespace {

constexpr int kThreads = 256;

enum EpiMode { EPI_PLAIN = 0, EPI_TRACE = 1, EPI_RESID = 2, EPI_GRAD = 3, EPI_NORMS = 4 };

template <typename T>
struct CloverVec;
template <>
struct CloverVec<float> {
  using type = float4;
  static constexpr int n = 18;  // 72 reals in 18 four-vectors
};
template <>
struct CloverVec<double> {
  using type = double2;
  static constexpr int n = 36;
};

template <typename T>
struct DslashArgs {
  const cpx<T>* in;
  cpx<T>* out;
  const cpx<T>* links;       // [4][9][V]
  const cpx<T>* links_c;     // [4][6][V] (two rows) or null
  const typename CloverVec<T>::type* clover;  // [n][V]
  const cpx<T>* b;           // EPI_RESID: right-hand side
  double* partials;          // per-workgroup partial sums
  const Control* ctl;
  Geom g;
  int L;
  int wpx;                   // > 0: one-pass t-slice grid, workgroups per XCD per slice
  int spw;                   // staged kernel: sites per workgroup
  T kappa;
  T aux;                     // EPI_GRAD: c_SW
};

template <typename T>
struct Half {
  cpx<T> h[2][3];
};

// rows 0..2 of a link; compressed links rebuild row 2 = conj(row0 x row1)
template <typename T, bool COMP>
__device__ __forceinline__ void load_link(const DslashArgs<T>& a, int site, int mu, cpx<T> u[3][3]) {
  const long long V = a.g.vol;
  if constexpr (COMP) {
    const cpx<T>* p = a.links_c + (long long)mu * 6 * V + site;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      u[0][k] = p[k * V];
      u[1][k] = p[(3 + k) * V];
    }
    u[2][0] = conj(u[0][1] * u[1][2] - u[0][2] * u[1][1]);
    u[2][1] = conj(u[0][2] * u[1][0] - u[0][0] * u[1][2]);
    u[2][2] = conj(u[0][0] * u[1][1] - u[0][1] * u[1][0]);
  } else {
    const cpx<T>* p = a.links + (long long)mu * 9 * V + site;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) u[i][k] = p[(i * 3 + k) * V];
  }
}

// Links and clover blocks either straight from the structure-of-arrays
// copies in global memory (GlobalSrc) or from the workgroup's LDS copy
// (LdsSrc), loaded once per site for all of the site's L threads.
template <typename T>
struct LinkRows {
  static constexpr int full = 9;
};

template <typename T, bool COMP>
__device__ __forceinline__ void finish_link(cpx<T> u[3][3]) {
  if constexpr (COMP) {
    u[2][0] = conj(u[0][1] * u[1][2] - u[0][2] * u[1][1]);
    u[2][1] = conj(u[0][2] * u[1][0] - u[0][0] * u[1][2]);
    u[2][2] = conj(u[0][0] * u[1][1] - u[0][1] * u[1][0]);
  }
}

template <typename T, bool COMP>
struct GlobalSrc {
  const DslashArgs<T>* a;
  int site;
  __device__ __forceinline__ void fwd(int mu, cpx<T> u[3][3]) const { load_link<T, COMP>(*a, site, mu, u); }
  __device__ __forceinline__ void bwd(int mu, int nb, cpx<T> u[3][3]) const { load_link<T, COMP>(*a, nb, mu, u); }
  __device__ __forceinline__ void clover(T cl[72]) const {
    using VecT = typename CloverVec<T>::type;
    constexpr int NV = CloverVec<T>::n;
    constexpr int W = 72 / NV;
    const VecT* cp = a->clover + site;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const VecT v = cp[(long long)q * a->g.vol];
      const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int w = 0; w < W; ++w) cl[q * W + w] = pv[w];
    }
  }
};

template <typename T, bool COMP>
struct LdsSrc {
  static constexpr int NC = COMP ? 6 : 9;
  using VecT = typename CloverVec<T>::type;
  static constexpr int NV = CloverVec<T>::n;
  const cpx<T>* lf;  // [S][4][NC] links U_mu(n) of the workgroup's sites
  const cpx<T>* lb;  // [S][4][NC] links U_mu(n - mu)
  const VecT* lc;    // [S][NV] clover vectors
  __device__ __forceinline__ void get(const cpx<T>* p, int mu, cpx<T> u[3][3]) const {
#pragma unroll
    for (int e = 0; e < NC; ++e) u[e / 3][e % 3] = p[mu * NC + e];
    finish_link<T, COMP>(u);
  }
  __device__ __forceinline__ void fwd(int mu, cpx<T> u[3][3]) const { get(lf, mu, u); }
  __device__ __forceinline__ void bwd(int mu, int, cpx<T> u[3][3]) const { get(lb, mu, u); }
  __device__ __forceinline__ void clover(T cl[72]) const {
    constexpr int W = 72 / NV;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const VecT v = lc[q];
      const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int w = 0; w < W; ++w) cl[q * W + w] = pv[w];
    }
  }
};

// offset of (site, spin*3 + colour, rhs) in a block; CM: component-major
template <bool CM>
__device__ __forceinline__ long long elem(int site, int sc, int l, int L, int V) {
  if constexpr (CM) return ((long long)sc * V + site) * L + l;
  else return ((long long)site * 12 + sc) * L + l;
}

// NR consecutive columns of one element, loaded as one vector when NR = 2
template <typename T, int NR>
struct __attribute__((aligned(NR * 2 * sizeof(T)))) Cols {
  cpx<T> v[NR];
};

template <typename T, int NR>
__device__ __forceinline__ Cols<T, NR> load_cols(const cpx<T>* __restrict__ p) {
  return *reinterpret_cast<const Cols<T, NR>*>(p);
}

template <typename T, int NR>
__device__ __forceinline__ void store_cols(cpx<T>* __restrict__ p, const Cols<T, NR>& c) {
  *reinterpret_cast<Cols<T, NR>*>(p) = c;
}

// Addressing of element (site, spin*3 + colour, column) in a block that
// starts at `base`.  Addr64: either layout, 64-bit element offsets.
template <bool CM>
struct Addr64 {
  int L, V;
  template <class P>
  __device__ __forceinline__ P* at(P* base, int site, int sc, int l) const {
    return base + elem<CM>(site, sc, l, L, V);
  }
};

// Component-major blocks whose components span less than 4 GiB each: the
// component's start (base + sc * V * L) is the same for the whole
// workgroup and is computed on the scalar unit, and the position inside the
// component is a 32-bit byte offset, so a load needs no per-thread 64-bit
// address arithmetic.
struct AddrCM32 {
  long long cs;  // V * L
  int L;
  template <class P>
  __device__ __forceinline__ P* at(P* base, int site, int sc, int l) const {
    using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
    const unsigned bo = ((unsigned)site * (unsigned)L + (unsigned)l) * (unsigned)sizeof(P);
    return reinterpret_cast<P*>(reinterpret_cast<C*>(base + sc * cs) + bo);
  }
};

// spin component s (all 3 colours) of columns l0 .. l0+NR-1 at site
template <typename T, int NR, class Ad>
__device__ __forceinline__ void load_spin(const cpx<T>* __restrict__ f, const Ad& ad, int site, int s, int l0,
                                          cpx<T> v[3][NR]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cols<T, NR> x = load_cols<T, NR>(ad.at(f, site, s * 3 + c, l0));
#pragma unroll
    for (int r = 0; r < NR; ++r) v[c][r] = x.v[r];
  }
}

// Projection with (1 - gamma_mu) (MINUS) or (1 + gamma_mu) onto two colour
// vectors, gamma matrices of Sec. 2 (0-based spins); the t-direction
// projectors are diagonal, so only two spin components are read.
template <typename T, int MU, bool MINUS, int NR, class Ad>
__device__ __forceinline__ void project(const cpx<T>* __restrict__ f, const Ad& ad, int site, int l0,
                                        cpx<T> h[2][3][NR]) {
  cpx<T> a[3][NR], b[3][NR];
  if constexpr (MU == 3) {
    // (1 - gamma_4) = diag(0,0,2,2), (1 + gamma_4) = diag(2,2,0,0)
    load_spin<T, NR>(f, ad, site, MINUS ? 2 : 0, l0, a);
    load_spin<T, NR>(f, ad, site, MINUS ? 3 : 1, l0, b);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        h[0][c][r] = T(2) * a[c][r];
        h[1][c][r] = T(2) * b[c][r];
      }
  } else {
    cpx<T> p0[3][NR], p1[3][NR];
    load_spin<T, NR>(f, ad, site, 0, l0, p0);
    load_spin<T, NR>(f, ad, site, 1, l0, p1);
    if constexpr (MU == 0) {
      // minus: h1 = psi0 + i psi3, h2 = psi1 + i psi2;  plus: -i instead of +i
      load_spin<T, NR>(f, ad, site, 3, l0, a);
      load_spin<T, NR>(f, ad, site, 2, l0, b);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          h[0][c][r] = MINUS ? p0[c][r] + times_i(a[c][r]) : p0[c][r] + times_mi(a[c][r]);
          h[1][c][r] = MINUS ? p1[c][r] + times_i(b[c][r]) : p1[c][r] + times_mi(b[c][r]);
        }
    } else if constexpr (MU == 1) {
      // minus: h1 = psi0 + psi3, h2 = psi1 - psi2;  plus: h1 = psi0 - psi3, h2 = psi1 + psi2
      load_spin<T, NR>(f, ad, site, 3, l0, a);
      load_spin<T, NR>(f, ad, site, 2, l0, b);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          h[0][c][r] = MINUS ? p0[c][r] + a[c][r] : p0[c][r] - a[c][r];
          h[1][c][r] = MINUS ? p1[c][r] - b[c][r] : p1[c][r] + b[c][r];
        }
    } else {
      // MU == 2. minus: h1 = psi0 + i psi2, h2 = psi1 - i psi3;  plus: signs of i flipped
      load_spin<T, NR>(f, ad, site, 2, l0, a);
      load_spin<T, NR>(f, ad, site, 3, l0, b);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          h[0][c][r] = MINUS ? p0[c][r] + times_i(a[c][r]) : p0[c][r] + times_mi(a[c][r]);
          h[1][c][r] = MINUS ? p1[c][r] + times_mi(b[c][r]) : p1[c][r] + times_i(b[c][r]);
        }
    }
  }
}

// acc += reconstruction of the two multiplied colour vectors g into 4 spins
template <typename T, int MU, bool MINUS, int NR>
__device__ __forceinline__ void reconstruct(cpx<T> acc[4][3][NR], const cpx<T> g[2][3][NR]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const cpx<T> g1 = g[0][c][r], g2 = g[1][c][r];
      if constexpr (MU == 3) {
        if constexpr (MINUS) {
          acc[2][c][r] = acc[2][c][r] + g1;
          acc[3][c][r] = acc[3][c][r] + g2;
        } else {
          acc[0][c][r] = acc[0][c][r] + g1;
          acc[1][c][r] = acc[1][c][r] + g2;
        }
      } else {
        acc[0][c][r] = acc[0][c][r] + g1;
        acc[1][c][r] = acc[1][c][r] + g2;
        if constexpr (MU == 0) {
          // minus: rows 2,3 = -i g2, -i g1;  plus: +i g2, +i g1
          acc[2][c][r] = acc[2][c][r] + (MINUS ? times_mi(g2) : times_i(g2));
          acc[3][c][r] = acc[3][c][r] + (MINUS ? times_mi(g1) : times_i(g1));
        } else if constexpr (MU == 1) {
          // minus: rows 2,3 = -g2, g1;  plus: g2, -g1
          acc[2][c][r] = MINUS ? acc[2][c][r] - g2 : acc[2][c][r] + g2;
          acc[3][c][r] = MINUS ? acc[3][c][r] + g1 : acc[3][c][r] - g1;
        } else {
          // minus: rows 2,3 = -i g1, +i g2;  plus: +i g1, -i g2
          acc[2][c][r] = acc[2][c][r] + (MINUS ? times_mi(g1) : times_i(g1));
          acc[3][c][r] = acc[3][c][r] + (MINUS ? times_i(g2) : times_mi(g2));
        }
      }
    }
}

// One hop.  FWD: from n + mu with U_mu(n); else from n - mu with U_mu(n-mu)^dagger.
// The forward projector is (1 - gamma_mu) for D and (1 + gamma_mu) for D^dagger.
// The link is loaded once and applied to all NR columns of the thread.
template <typename T, int MU, bool FWD, bool DAG, int NR, class Src, class Ad>
__device__ __forceinline__ void hop(const DslashArgs<T>& a, const Src& src, const Ad& ad, int nbr, int l0,
                                    cpx<T> acc[4][3][NR]) {
  constexpr bool MINUS = (FWD != DAG);
  cpx<T> h[2][3][NR], g[2][3][NR];
  project<T, MU, MINUS, NR>(a.in, ad, nbr, l0, h);
  cpx<T> u[3][3];
  if constexpr (FWD) src.fwd(MU, u);
  else src.bwd(MU, nbr, u);
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        cpx<T> v = mk(T(0), T(0));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if constexpr (FWD) cmac(v, u[i][k], h[sp][k][r]);
          else cmac_conj(v, u[k][i], h[sp][k][r]);
        }
        g[sp][i][r] = v;
      }
  reconstruct<T, MU, MINUS, NR>(acc, g);
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
// Keep the scheduler from hoisting the next hop's loads above this point:
// bounds the live registers to about one hop's operands.
#ifdef BKWD_SCHED_FENCE
#define SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define SCHED_FENCE() (void)0
#endif

template <typename T, bool DAG, int EPI, int NR, class Src, class Ad>
__device__ __forceinline__ void site_rhs(const DslashArgs<T>& a, const Src& src, const Ad& ad, int site, int l0,
                                         double& e0, double& e1, double& e2) {
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

  cpx<T> acc[4][3][NR];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[s][c][q] = mk(T(0), T(0));

  hop<T, 0, true, DAG, NR>(a, src, ad, xp, l0, acc);
  SCHED_FENCE();
  hop<T, 0, false, DAG, NR>(a, src, ad, xm, l0, acc);
  SCHED_FENCE();
  hop<T, 1, true, DAG, NR>(a, src, ad, yp, l0, acc);
  SCHED_FENCE();
  hop<T, 1, false, DAG, NR>(a, src, ad, ym, l0, acc);
  SCHED_FENCE();
  hop<T, 2, true, DAG, NR>(a, src, ad, zp, l0, acc);
  SCHED_FENCE();
  hop<T, 2, false, DAG, NR>(a, src, ad, zm, l0, acc);
  SCHED_FENCE();
  hop<T, 3, true, DAG, NR>(a, src, ad, tp, l0, acc);
  SCHED_FENCE();
  hop<T, 3, false, DAG, NR>(a, src, ad, tm, l0, acc);

  // site-local term on phi_+- = psi_{0,1} +- psi_{2,3}
  cpx<T> psi[4][3][NR];
#pragma unroll
  for (int s = 0; s < 4; ++s) load_spin<T, NR>(a.in, ad, site, s, l0, psi[s]);
  T cl[72];
  src.clover(cl);
  const T kap = a.kappa;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    cpx<T> pp[6], pm[6], qp[6], qm[6];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pp[3 * s + c] = psi[s][c][q] + psi[s + 2][c][q];
        pm[3 * s + c] = psi[s][c][q] - psi[s + 2][c][q];
      }
    herm6(cl, pp, qp);
    herm6(cl + 36, pm, qm);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cpx<T> loc = (s < 2) ? qp[3 * s + c] + qm[3 * s + c] : qp[3 * (s - 2) + c] - qm[3 * (s - 2) + c];
        cpx<T> res = mk(loc.re - kap * acc[s][c][q].re, loc.im - kap * acc[s][c][q].im);
        if constexpr (EPI == EPI_TRACE) {
          // Tr(Y^H X) and Tr(Y^H Y) with Y = D X
          const cpx<T> xin = psi[s][c][q];
          e0 += (double)res.re * (double)xin.re + (double)res.im * (double)xin.im;
          e1 += (double)res.re * (double)xin.im - (double)res.im * (double)xin.re;
          e2 += (double)res.re * (double)res.re + (double)res.im * (double)res.im;
        } else if constexpr (EPI == EPI_GRAD) {
          // b = Lam; the clover blocks are those of 1 - C, so C X = X - loc and
          // acc = H X:  e0 += Re conj(lam) (csw C X + H X),  e1 += Re conj(lam) C X
          const cpx<T> lam = *ad.at(a.b, site, s * 3 + c, l0 + q);
          const cpx<T> cx = psi[s][c][q] - loc;
          const cpx<T> hx = acc[s][c][q];
          const T tr = a.aux * cx.re + hx.re, ti = a.aux * cx.im + hx.im;
          e0 += (double)lam.re * (double)tr + (double)lam.im * (double)ti;
          e1 += (double)lam.re * (double)cx.re + (double)lam.im * (double)cx.im;
        } else if constexpr (EPI == EPI_RESID || EPI == EPI_NORMS) {
          const cpx<T> bv = *ad.at(a.b, site, s * 3 + c, l0 + q);
          res = bv - res;
          e0 += (double)res.re * (double)res.re + (double)res.im * (double)res.im;
          e1 += (double)bv.re * (double)bv.re + (double)bv.im * (double)bv.im;
        }
        acc[s][c][q] = res;
      }
  }
  if constexpr (EPI == EPI_GRAD || EPI == EPI_NORMS) return;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Cols<T, NR> o;
#pragma unroll
      for (int q = 0; q < NR; ++q) o.v[q] = acc[s][c][q];
      store_cols<T, NR>(ad.at(a.out, site, s * 3 + c, l0), o);
    }
}

// Workgroup sums of the trace epilogue -> partials[blk][0..3]
__device__ __forceinline__ void trace_store(double* partials, int blk, double e0, double e1, double e2) {
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
    partials[(long long)blk * 4 + threadIdx.x] = v;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  For a one-pass launch the grid is laid out as t-slices: workgroup g
// runs on XCD g % 8 and, as the k = g / 8-th workgroup of that XCD, covers
// part (g % 8) of time slice k / wpx.  All XCDs then sweep the lattice in t
// together, each over its own eighth of every slice, so the +-t neighbour
// of a site was loaded about one slice-eighth earlier by the same XCD and
// the +-x, +-y, +-z neighbours even more recently.
__device__ __forceinline__ long long slab_base(int wpx, long long per_slice) {
  const int g = blockIdx.x;
  const int xcd = g & 7;
  const int k = g >> 3;
  const int t = k / wpx;
  const int part = xcd * wpx + (k - t * wpx);
  const long long off = (long long)part * kThreads;
  if (off >= per_slice) return -1;  // padding workgroup
  return (long long)t * per_slice + off;
}

// grid-stride launches (the residual) keep a plain contiguous split over XCDs
__device__ __forceinline__ int xcd_block() {
  const int n = gridDim.x, b = blockIdx.x;
  if (n % 8 != 0) return b;
  return (b % 8) * (n / 8) + b / 8;
}

// minimum waves per SIMD requested from the register allocator
#ifndef BKWD_DSLASH_MINWAVES_F32
#define BKWD_DSLASH_MINWAVES_F32 1
#endif
#ifndef BKWD_DSLASH_MINWAVES_F64
#define BKWD_DSLASH_MINWAVES_F64 1
#endif
template <typename T>
struct MinWaves {
  static constexpr int value = sizeof(T) == 4 ? BKWD_DSLASH_MINWAVES_F32 : BKWD_DSLASH_MINWAVES_F64;
};

template <typename T, bool DAG, bool COMP, int EPI, bool CM, int NR>
__global__ void __launch_bounds__(kThreads, MinWaves<T>::value) k_dslash(DslashArgs<T> a) {
  if (a.ctl != nullptr && a.ctl->state != ST_RUNNING) return;
  const int L = a.L;
  const int LT = L / NR;  // threads per site
  const long long total = (long long)a.g.vol * LT;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;  // epilogue partial sums
  int blk;
  if (a.wpx > 0) {
    // one pass, t-slice layout of the grid
    blk = blockIdx.x;
    const long long per_slice = total / a.g.lt;
    const long long base = slab_base(a.wpx, per_slice);
    if (base >= 0) {
      const long long slice_end = base - base % per_slice + per_slice;
      const long long tid = base + threadIdx.x;
      if (tid < slice_end) {
        const int site = (int)(tid / LT);
        const int l0 = (int)(tid - (long long)site * LT) * NR;
        site_rhs<T, DAG, EPI, NR>(a, GlobalSrc<T, COMP>{&a, site}, Addr64<CM>{L, a.g.vol}, site, l0, e0, e1, e2);
      }
    }
  } else {
    const long long stride = (long long)gridDim.x * kThreads;
    blk = xcd_block();
    for (long long base = (long long)blk * kThreads; base < total; base += stride) {
      const long long tid = base + threadIdx.x;
      if (tid < total) {
        const int site = (int)(tid / LT);
        const int l0 = (int)(tid - (long long)site * LT) * NR;
        site_rhs<T, DAG, EPI, NR>(a, GlobalSrc<T, COMP>{&a, site}, Addr64<CM>{L, a.g.vol}, site, l0, e0, e1, e2);
      }
    }
  }

  if constexpr (EPI == EPI_TRACE || EPI == EPI_GRAD) {
    trace_store(a.partials, blk, e0, e1, e2);
  } else if constexpr (EPI == EPI_RESID || EPI == EPI_NORMS) {
    // per-column sums: thread of global index tid holds column tid % L
    __shared__ double red[2][kThreads];
    red[0][threadIdx.x] = e0;
    red[1][threadIdx.x] = e1;
    __syncthreads();
    if (threadIdx.x < L) {
      const long long base = (long long)blk * kThreads;
      const int first = (int)((L - (int)(base % L) + threadIdx.x) % L);  // first local index with column tid
      double v0 = 0.0, v1 = 0.0;
      for (int k = first; k < kThreads; k += L) {
        v0 += red[0][k];
        v1 += red[1][k];
      }
      a.partials[(long long)blk * 2 * L + threadIdx.x] = v0;
      a.partials[(long long)blk * 2 * L + L + threadIdx.x] = v1;
    }
  }
}


// One-pass operator with the workgroup's links (U_mu(n) and U_mu(n - mu))
// and clover blocks staged in LDS: a workgroup owns S = 256 / L whole sites,
// thread (j, l) computes column l of site j, and the S sites' link and
// clover data are read from memory once instead of once per column.  The
// grid uses the same t-slice layout as the direct kernel, at site
// granularity: workgroup g runs on XCD g % 8 and covers S sites of part
// (g % 8) of time slice (g / 8) / wpx.
template <typename T, bool DAG, bool COMP, int EPI, bool CM>
__global__ void __launch_bounds__(kThreads, MinWaves<T>::value) k_dslash_st(DslashArgs<T> a) {
  if (a.ctl != nullptr && a.ctl->state != ST_RUNNING) return;
  constexpr int NC = COMP ? 6 : 9;
  using VecT = typename CloverVec<T>::type;
  constexpr int NV = CloverVec<T>::n;
  const Geom g = a.g;
  const int L = a.L, S = a.spw, V = g.vol;
  const int sps = g.lx * g.ly * g.lz;
  const int b = blockIdx.x;
  const int k = b >> 3;
  const int t = k / a.wpx;
  const int part = (b & 7) * a.wpx + (k - t * a.wpx);
  const int first = part * S;
  const int nsites = min(S, sps - first);  // <= 0: padding workgroup
  const int site0 = t * sps + first;

  // LDS, site-major so that a thread's reads sit at fixed offsets from its
  // site's record: clover [S][NV], links U_mu(n) [S][4][NC], U_mu(n-mu) [S][4][NC]
  extern __shared__ __align__(16) unsigned char smem_raw[];
  VecT* lc = reinterpret_cast<VecT*>(smem_raw);
  cpx<T>* lf = reinterpret_cast<cpx<T>*>(lc + NV * S);
  cpx<T>* lb = lf + 4 * NC * S;
  const cpx<T>* links = COMP ? a.links_c : a.links;

  if (nsites > 0) {
    for (int idx = threadIdx.x; idx < 4 * NC * nsites; idx += kThreads) {
      const int me = idx / nsites;  // mu * NC + e
      const int jj = idx - me * nsites;
      const int mu = me / NC;
      const int site = site0 + jj;
      int c[4] = {site % g.lx, (site / g.lx) % g.ly, (site / (g.lx * g.ly)) % g.lz, t};
      const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
      c[mu] = (c[mu] == 0) ? ext[mu] - 1 : c[mu] - 1;
      const int nb = c[0] + g.lx * (c[1] + g.ly * (c[2] + g.lz * c[3]));
      const long long arr = (long long)me * V;
      lf[jj * 4 * NC + me] = links[arr + site];
      lb[jj * 4 * NC + me] = links[arr + nb];
    }
    for (int idx = threadIdx.x; idx < NV * nsites; idx += kThreads) {
      const int q = idx / nsites;
      const int jj = idx - q * nsites;
      lc[jj * NV + q] = a.clover[(long long)q * V + site0 + jj];
    }
  }
  __syncthreads();
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  const int j = threadIdx.x / L;
  const int l = threadIdx.x - j * L;
  if (j < nsites) {
    const LdsSrc<T, COMP> src{lf + j * 4 * NC, lb + j * 4 * NC, lc + j * NV};
    if constexpr (CM) site_rhs<T, DAG, EPI, 1>(a, src, AddrCM32{(long long)V * L, L}, site0 + j, l, e0, e1, e2);
    else site_rhs<T, DAG, EPI, 1>(a, src, Addr64<false>{L, V}, site0 + j, l, e0, e1, e2);
  }
  if constexpr (EPI == EPI_TRACE) trace_store(a.partials, b, e0, e1, e2);
}

// Staged operator with the hopping factors folded into the links, for the
// plain epilogue (every FP32 application of the solver's inner iteration).
// Per workgroup of S = 256 / L whole sites, LDS holds one record per site:
// the links U_mu(n) and U_mu(n - mu) multiplied by -kappa (by -2 kappa in t,
// which absorbs the factor 2 of the diagonal t projectors), the two clover
// blocks and the eight neighbour indices.  Each thread (site j, column l)
// starts its accumulator with the site-local term A(n) X(n) and adds the
// eight hops, so no value other than the accumulator survives from one phase
// to the next.  Records are padded to a dword stride of 4 mod 64 so that the
// different sites of a wave read distinct LDS banks.
template <typename T>
struct SrRec {
  static constexpr int off_lf = 0;                                   // [4][9] cpx<T>
  static constexpr int off_lb = 36 * (int)sizeof(cpx<T>);            // [4][9] cpx<T>
  static constexpr int off_cl = 72 * (int)sizeof(cpx<T>);            // 72 T (A+/2, A-/2)
  static constexpr int off_nb = off_cl + 72 * (int)sizeof(T);        // 8 int: +x -x +y -y +z -z +t -t
  static constexpr int raw_dw = (off_nb + 32) / 4;
  static constexpr int stride = 4 * (((raw_dw + 27) / 32) * 32 + 4);  // bytes, dwords = 4 mod 32
};

// One hop of the folded-link operator, split into the loads of the
// neighbour's spin rows and the arithmetic on them, so that a hop's loads can
// be in flight while the previous hop is computed.  Rows kept per hop: for x,
// y, z spins 0 and 1 and the two that the projector pairs with them; in t the
// two spins that the diagonal (1 -/+ gamma_4)/2 keeps (the factor 2 of the
// projector lives in the staged link).
template <typename T>
struct HopRows {
  cpx<T> r[4][3][1];
};

template <typename T, int MU, bool FWD, bool DAG, class Ad>
__device__ __forceinline__ void fetch_sr(const cpx<T>* __restrict__ in, const Ad& ad, int nbr, int l,
                                         HopRows<T>& q) {
  constexpr bool MINUS = (FWD != DAG);
  if constexpr (MU == 3) {
    load_spin<T, 1>(in, ad, nbr, MINUS ? 2 : 0, l, q.r[0]);
    load_spin<T, 1>(in, ad, nbr, MINUS ? 3 : 1, l, q.r[1]);
  } else {
    load_spin<T, 1>(in, ad, nbr, 0, l, q.r[0]);
    load_spin<T, 1>(in, ad, nbr, 1, l, q.r[1]);
    // the spins combined with 0 and 1: (3, 2) in x and y, (2, 3) in z
    load_spin<T, 1>(in, ad, nbr, MU == 2 ? 2 : 3, l, q.r[2]);
    load_spin<T, 1>(in, ad, nbr, MU == 2 ? 3 : 2, l, q.r[3]);
  }
}

template <typename T, int MU, bool FWD, bool DAG>
__device__ __forceinline__ void apply_sr(const unsigned char* rec, const HopRows<T>& q, cpx<T> acc[4][3][1]) {
  constexpr bool MINUS = (FWD != DAG);
  cpx<T> h[2][3][1], g[2][3][1];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cpx<T> p0 = q.r[0][c][0], p1 = q.r[1][c][0];
    if constexpr (MU == 3) {
      h[0][c][0] = p0;
      h[1][c][0] = p1;
    } else {
      const cpx<T> a = q.r[2][c][0], b = q.r[3][c][0];
      if constexpr (MU == 0) {
        // minus: h1 = psi0 + i psi3, h2 = psi1 + i psi2;  plus: -i instead of +i
        h[0][c][0] = MINUS ? p0 + times_i(a) : p0 + times_mi(a);
        h[1][c][0] = MINUS ? p1 + times_i(b) : p1 + times_mi(b);
      } else if constexpr (MU == 1) {
        // minus: h1 = psi0 + psi3, h2 = psi1 - psi2;  plus: h1 = psi0 - psi3, h2 = psi1 + psi2
        h[0][c][0] = MINUS ? p0 + a : p0 - a;
        h[1][c][0] = MINUS ? p1 - b : p1 + b;
      } else {
        // minus: h1 = psi0 + i psi2, h2 = psi1 - i psi3;  plus: signs of i flipped
        h[0][c][0] = MINUS ? p0 + times_i(a) : p0 + times_mi(a);
        h[1][c][0] = MINUS ? p1 + times_mi(b) : p1 + times_i(b);
      }
    }
  }
  const cpx<T>* u = reinterpret_cast<const cpx<T>*>(rec + (FWD ? SrRec<T>::off_lf : SrRec<T>::off_lb)) + MU * 9;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cpx<T> v = mk(T(0), T(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if constexpr (FWD) cmac(v, u[i * 3 + k], h[sp][k][0]);
        else cmac_conj(v, u[k * 3 + i], h[sp][k][0]);
      }
      g[sp][i][0] = v;
    }
  reconstruct<T, MU, MINUS, 1>(acc, g);
}

// The eight hops in the order +x -x +y -y +z -z +t -t, each hop's rows
// loaded before the previous hop is computed (about 14 more registers per
// lane than one hop after the other); q0 holds the rows of +x, already
// requested by the caller.
template <typename T, bool DAG, class Ad>
__device__ __forceinline__ void hops_sr(const cpx<T>* __restrict__ in, const unsigned char* rec, const Ad& ad,
                                        const int* nb, int l, HopRows<T>& q0, cpx<T> acc[4][3][1]) {
  HopRows<T> q1;
  fetch_sr<T, 0, false, DAG>(in, ad, nb[1], l, q1);
  apply_sr<T, 0, true, DAG>(rec, q0, acc);
  fetch_sr<T, 1, true, DAG>(in, ad, nb[2], l, q0);
  apply_sr<T, 0, false, DAG>(rec, q1, acc);
  fetch_sr<T, 1, false, DAG>(in, ad, nb[3], l, q1);
  apply_sr<T, 1, true, DAG>(rec, q0, acc);
  fetch_sr<T, 2, true, DAG>(in, ad, nb[4], l, q0);
  apply_sr<T, 1, false, DAG>(rec, q1, acc);
  fetch_sr<T, 2, false, DAG>(in, ad, nb[5], l, q1);
  apply_sr<T, 2, true, DAG>(rec, q0, acc);
  fetch_sr<T, 3, true, DAG>(in, ad, nb[6], l, q0);
  apply_sr<T, 2, false, DAG>(rec, q1, acc);
  fetch_sr<T, 3, false, DAG>(in, ad, nb[7], l, q1);
  apply_sr<T, 3, true, DAG>(rec, q0, acc);
  apply_sr<T, 3, false, DAG>(rec, q1, acc);
}

// (D in)(site) for column l, stored to a.out; with KEEP the result is also
// returned in own_out[sc], sc = spin * 3 + colour
template <typename T, bool DAG, bool KEEP, class Ad>
__device__ __forceinline__ void site_sr_core(const DslashArgs<T>& a, const unsigned char* rec, const Ad& ad, int site,
                                             int l, cpx<T>* own_out) {
  cpx<T> acc[4][3][1];
  const int* nb = reinterpret_cast<const int*>(rec + SrRec<T>::off_nb);
  HopRows<T> q0;
  {
    // site-local term on phi_+- = psi_{0,1} +- psi_{2,3} (halved blocks A+-/2),
    // with the rows of the first hop in flight
    cpx<T> psi[4][3][1];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) load_spin<T, 1>(a.in, ad, site, sp, l, psi[sp]);
    fetch_sr<T, 0, true, DAG>(a.in, ad, nb[0], l, q0);
    cpx<T> pp[6], pm[6], qp[6], qm[6];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pp[3 * sp + c] = psi[sp][c][0] + psi[sp + 2][c][0];
        pm[3 * sp + c] = psi[sp][c][0] - psi[sp + 2][c][0];
      }
    const T* cl = reinterpret_cast<const T*>(rec + SrRec<T>::off_cl);
    herm6(cl, pp, qp);
    herm6(cl + 36, pm, qm);
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[sp][c][0] = qp[3 * sp + c] + qm[3 * sp + c];
        acc[sp + 2][c][0] = qp[3 * sp + c] - qm[3 * sp + c];
      }
  }
  hops_sr<T, DAG>(a.in, rec, ad, nb, l, q0, acc);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      *ad.at(a.out, site, sp * 3 + c, l) = acc[sp][c][0];
      if constexpr (KEEP) own_out[sp * 3 + c] = acc[sp][c][0];
    }
}

template <typename T, bool DAG, class Ad>
__device__ __forceinline__ void site_sr(const DslashArgs<T>& a, const unsigned char* rec, const Ad& ad, int site,
                                        int l) {
  site_sr_core<T, DAG, false>(a, rec, ad, site, l, nullptr);
}

// The slice part of workgroup index b: workgroup b runs on XCD b mod 8, and
// XCD x takes the x-th eighth of every time slice (wpx parts per XCD and
// slice); nsites <= 0 marks a padding part.
struct SrPart {
  int t, first, nsites, site0;
};

template <typename T>
__device__ __forceinline__ SrPart sr_part(const DslashArgs<T>& a, int b) {
  const int sps = a.g.lx * a.g.ly * a.g.lz;
  const int k = b >> 3;
  SrPart p;
  p.t = k / a.wpx;
  const int part = (b & 7) * a.wpx + (k - p.t * a.wpx);
  p.first = part * a.spw;
  p.nsites = min(a.spw, sps - p.first);
  p.site0 = p.t * sps + p.first;
  return p;
}

// Site records of a part in LDS: neighbour indices, links scaled by -kappa
// (-2 kappa in t) for U_mu(n) and U_mu(n - mu), the two clover blocks.
// Called by the whole workgroup with p.nsites > 0.
template <typename T>
__device__ __forceinline__ void sr_stage(const DslashArgs<T>& a, unsigned char* smem_raw, const SrPart& p) {
  using VecT = typename CloverVec<T>::type;
  constexpr int NV = CloverVec<T>::n;
  constexpr int RS = SrRec<T>::stride;
  const Geom g = a.g;
  const int V = g.vol, nsites = p.nsites, first = p.first, site0 = p.site0, t = p.t;
  for (int idx = threadIdx.x; idx < 8 * nsites; idx += kThreads) {
    const int jj = idx >> 3, d = idx & 7, mu = d >> 1;
    const int sp = first + jj;
    int c[4] = {sp % g.lx, (sp / g.lx) % g.ly, sp / (g.lx * g.ly), t};
    const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
    c[mu] = (d & 1) ? (c[mu] == 0 ? ext[mu] - 1 : c[mu] - 1) : (c[mu] + 1 == ext[mu] ? 0 : c[mu] + 1);
    reinterpret_cast<int*>(smem_raw + jj * RS + SrRec<T>::off_nb)[d] =
        c[0] + g.lx * (c[1] + g.ly * (c[2] + g.lz * c[3]));
  }
  __syncthreads();
  const T kap = a.kappa;
  for (int idx = threadIdx.x; idx < 36 * nsites; idx += kThreads) {
    const int me = idx / nsites;  // mu * 9 + e
    const int jj = idx - me * nsites;
    const int mu = me / 9;
    const T f = (mu == 3) ? T(-2) * kap : -kap;
    const int nbm = reinterpret_cast<const int*>(smem_raw + jj * RS + SrRec<T>::off_nb)[2 * mu + 1];
    const long long arr = (long long)me * V;
    const cpx<T> uf = a.links[arr + site0 + jj], ub = a.links[arr + nbm];
    reinterpret_cast<cpx<T>*>(smem_raw + jj * RS + SrRec<T>::off_lf)[me] = mk(f * uf.re, f * uf.im);
    reinterpret_cast<cpx<T>*>(smem_raw + jj * RS + SrRec<T>::off_lb)[me] = mk(f * ub.re, f * ub.im);
  }
  for (int idx = threadIdx.x; idx < NV * nsites; idx += kThreads) {
    const int q = idx / nsites;
    const int jj = idx - q * nsites;
    reinterpret_cast<VecT*>(smem_raw + jj * RS + SrRec<T>::off_cl)[q] = a.clover[(long long)q * V + site0 + jj];
  }
}

template <typename T, bool DAG, bool CM>
__global__ void __launch_bounds__(kThreads) k_dslash_sr(DslashArgs<T> a) {
  if (a.ctl != nullptr && a.ctl->state != ST_RUNNING) return;
  constexpr int RS = SrRec<T>::stride;
  const int L = a.L, V = a.g.vol;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const SrPart p = sr_part(a, blockIdx.x);
  if (p.nsites > 0) sr_stage(a, smem_raw, p);
  __syncthreads();
  const int j = threadIdx.x / L;
  const int l = threadIdx.x - j * L;
  if (j < p.nsites) {
    const unsigned char* rec = smem_raw + j * RS;
    if constexpr (CM) site_sr<T, DAG>(a, rec, AddrCM32{(long long)V * L, L}, p.site0 + j, l);
    else site_sr<T, DAG>(a, rec, Addr64<false>{L, V}, p.site0 + j, l);
  }
}

// ------------------------------------------------------------------ W' = A T with its Grams
// The fused frame's Gram pass, folded into the operator launch that makes
// W' = A T (8-column FP32 blocks, component-major): besides storing W', each
// workgroup sums T^H W', W'^H W' and R~0^H W' over the sites it applies the
// operator to.  Per spin-colour row, the lane of (site, column) holds one
// complex value; ds_bpermute spreads it to the layout of the lane-per-real
// block kernels (16 lanes = the 16 reals of one block row, four sites per
// register), and one v_mfma_f32_16x16x4f32 per Gram and register adds the
// real 16 x 16 product whose 2 x 2 blocks are the complex Gram.  One
// workgroup per slice part, on the XCD of the plain launch (a grid-stride
// walk over the parts lost L2 locality: 2290 against 2155 us per launch at
// 32^3 x 64), each writing one FP64 partial record that k_reduce sums.

// lane 16 k + m of register h takes part m % 2 of column m / 2 at site
// 4 h + k of the wave: the value held by lane 32 h + lane / 2
__device__ __forceinline__ float realify(const cpx<float>& v, int h, int lane) {
  const int src = (32 * h + (lane >> 1)) << 2;
  const float re = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v.re)));
  const float im = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v.im)));
  return (lane & 1) ? im : re;
}

// The three Grams of a wave's 8 sites x 8 columns, row by row: the lane of
// (site, column) holds W' (wout), and T and R~0 of its element are read at
// (site, l); acc = the real 16 x 16 forms of T^H W', W'^H W' and R~0^H W'.
// Lanes with act false add zeros.
template <class Ad>
__device__ __forceinline__ void gram3_rows(const cpx<float>* __restrict__ t, const cpx<float>* __restrict__ rt,
                                           const Ad& ad, int site, int l, bool act, const cpx<float> wout[12],
                                           f32x4 acc[3]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 3; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int sc = 0; sc < 12; ++sc) {
    const cpx<float> tv = act ? *ad.at(t, site, sc, l) : mk(0.f, 0.f);
    const cpx<float> rv = act ? *ad.at(rt, site, sc, l) : mk(0.f, 0.f);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float wv = realify(wout[sc], h, lane);
      acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(realify(tv, h, lane), wv, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv, wv, acc[1], 0, 0, 0);
      acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(realify(rv, h, lane), wv, acc[2], 0, 0, 0);
    }
  }
}

// The workgroup's four waves' sums in a fixed order, through LDS (at least
// 4 x 3 x 256 doubles, free for reuse), to one FP64 partial record:
// out[q * 128 + 2 (i * 8 + k)] = (T^H W', W'^H W', R~0^H W')[i][k]
__device__ __forceinline__ void gram3_flush(const f32x4 acc[3], unsigned char* smem_raw, double* out) {
  const int w = threadIdx.x >> 6;
  const L8Layout ly = l8_layout();
  double* P = reinterpret_cast<double*>(smem_raw);  // [wave][gram][16 x 16]
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) P[(w * 3 + q) * 256 + ly.i[v] * 16 + ly.j[v]] = (double)acc[q][v];
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * 64; e += kThreads) {
    const int q = e >> 6, r = (e >> 3) & 7, c = e & 7;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) {
      const double* pp = P + (ww * 3 + q) * 256;
      re += pp[(2 * r) * 16 + 2 * c] + pp[(2 * r + 1) * 16 + 2 * c + 1];
      im += pp[(2 * r) * 16 + 2 * c + 1] - pp[(2 * r + 1) * 16 + 2 * c];
    }
    out[q * 128 + 2 * (r * 8 + c)] = re;
    out[q * 128 + 2 * (r * 8 + c) + 1] = im;
  }
}

// The Gram accumulators are formed after the hops, so that they take no
// registers while the hops' loads are in flight; at most 102 registers per
// lane, so that five workgroups fit per CU (as many as the site records' LDS
// allows).
template <bool DAG>
__global__ void __launch_bounds__(kThreads, 5) k_dslash_srg(DslashArgs<float> a) {
  if (a.ctl != nullptr && a.ctl->state != ST_RUNNING) return;
  constexpr int RS = SrRec<float>::stride;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int V = a.g.vol;
  const int j = threadIdx.x >> 3, l = threadIdx.x & 7;
  const AddrCM32 ad{(long long)V * 8, 8};
  // one slice part per workgroup (the grid is the part count)
  const SrPart p = sr_part(a, blockIdx.x);
  if (p.nsites > 0) sr_stage(a, smem_raw, p);
  __syncthreads();
  const bool act = j < p.nsites;
  const int site = p.site0 + (act ? j : 0);
  cpx<float> wout[12];
  if (act) {
    site_sr_core<float, DAG, true>(a, smem_raw + j * RS, ad, site, l, wout);
  } else {
#pragma unroll
    for (int sc = 0; sc < 12; ++sc) wout[sc] = mk(0.f, 0.f);
  }
  f32x4 acc[3];
  gram3_rows(a.in, a.b, ad, site, l, act, wout, acc);
  // the records are no longer read: the LDS takes the sums
  __syncthreads();
  gram3_flush(acc, smem_raw, a.partials + (long long)blockIdx.x * 384);
}

// ------------------------------------------------------------------ even-odd
// With every extent even, each hop joins sites of opposite parity
// (x + y + z + t even or odd).  The even-odd solve needs, for the sites n of
// one parity,
//   out(n) = POST( CEN in_c(n) + f sum_mu [hops of Eq. (1) from in_h] ),
// CEN: nothing, the identity, the site-local term A or its inverse; POST: the
// identity or A^{-1}; the hop factor f (-kappa, +kappa) is folded into the
// staged links as in k_dslash_sr (2 f in t).  Blocks are either compact
// (the sites of one parity only, component-major, position site / 2 with Lx
// even) or whole-lattice site-major.
enum { EO_CEN_NONE = 0, EO_CEN_ID = 1, EO_CEN_A = 2, EO_CEN_AINV = 3 };

template <typename T>
struct EoArgs {
  const cpx<T>* in_c;   // centre input (CEN != NONE)
  const cpx<T>* in_h;   // hop input (hops != 0)
  cpx<T>* out;
  const cpx<T>* links;  // [4][9][V]
  const typename CloverVec<T>::type* clov;  // A or A^{-1} blocks, whichever CEN / POST use
  const Control* ctl;
  const cpx<T>* rt;     // R~0 of the Gram launch (compact, like in_c)
  double* partials;     // its partial records
  Geom g;
  int L, par, spw, hops;
  T f;                  // hop factor
};

// compact component-major block of one parity: position site / 2
struct AddrHalf {
  long long cs;  // (V / 2) * L
  int L;
  template <class P>
  __device__ __forceinline__ P* at(P* base, int site, int sc, int l) const {
    using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
    const unsigned bo = ((unsigned)(site >> 1) * (unsigned)L + (unsigned)l) * (unsigned)sizeof(P);
    return reinterpret_cast<P*>(reinterpret_cast<C*>(base + sc * cs) + bo);
  }
};

// site index of position c among the sites of parity p (Lx even)
__device__ __forceinline__ int eo_site(const Geom& g, int c, int p) {
  const int half = g.lx >> 1;
  const int r = c / half;
  const int k = c - r * half;
  const int y = r % g.ly;
  const int rz = r / g.ly;
  const int z = rz % g.lz;
  const int t = rz / g.lz;
  const int x = 2 * k + ((p + y + z + t) & 1);
  return x + g.lx * r;
}

// psi -> A psi (or A^{-1} psi) with the packed halved blocks at cl
template <typename T>
__device__ __forceinline__ void local_packed(const T* cl, cpx<T> v[4][3][1]) {
  cpx<T> pp[6], pm[6], qp[6], qm[6];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pp[3 * sp + c] = v[sp][c][0] + v[sp + 2][c][0];
      pm[3 * sp + c] = v[sp][c][0] - v[sp + 2][c][0];
    }
  herm6(cl, pp, qp);
  herm6(cl + 36, pm, qm);
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[sp][c][0] = qp[3 * sp + c] + qm[3 * sp + c];
      v[sp + 2][c][0] = qp[3 * sp + c] - qm[3 * sp + c];
    }
}

// out(site) for column l; with KEEP it is also returned in own_out[sc]
template <typename T, bool DAG, int CEN, bool POST, class Ad, bool KEEP = false>
__device__ __forceinline__ void site_eo(const EoArgs<T>& a, const unsigned char* rec, const Ad& ad, int site, int l,
                                        cpx<T>* own_out = nullptr) {
  cpx<T> acc[4][3][1];
  const int* nb = reinterpret_cast<const int*>(rec + SrRec<T>::off_nb);
  HopRows<T> q0;
  // the rows of the first hop are in flight while the centre term is formed
  if (a.hops) fetch_sr<T, 0, true, DAG>(a.in_h, ad, nb[0], l, q0);
  if constexpr (CEN == EO_CEN_NONE) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[sp][c][0] = mk(T(0), T(0));
  } else {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) load_spin<T, 1>(a.in_c, ad, site, sp, l, acc[sp]);
    if constexpr (CEN == EO_CEN_A || CEN == EO_CEN_AINV)
      local_packed<T>(reinterpret_cast<const T*>(rec + SrRec<T>::off_cl), acc);
  }
  if (a.hops) hops_sr<T, DAG>(a.in_h, rec, ad, nb, l, q0, acc);
  if constexpr (POST) local_packed<T>(reinterpret_cast<const T*>(rec + SrRec<T>::off_cl), acc);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      *ad.at(a.out, site, sp * 3 + c, l) = acc[sp][c][0];
      if constexpr (KEEP) own_out[sp * 3 + c] = acc[sp][c][0];
    }
}

// Site records of the workgroup's sites c0 .. c0 + nsites - 1 of parity
// a.par (compact positions) in LDS: neighbour indices, the links scaled by
// the hop factor (twice it in t) when the launch hops, the CLOV blocks.
// Called by the whole workgroup with nsites > 0.
template <typename T, bool CLOV>
__device__ __forceinline__ void eo_stage(const EoArgs<T>& a, unsigned char* smem_raw, int c0, int nsites) {
  using VecT = typename CloverVec<T>::type;
  constexpr int NV = CloverVec<T>::n;
  constexpr int RS = SrRec<T>::stride;
  const Geom g = a.g;
  const int V = g.vol;
  for (int idx = threadIdx.x; idx < 8 * nsites; idx += blockDim.x) {
    const int jj = idx >> 3, d = idx & 7, mu = d >> 1;
    const int site = eo_site(g, c0 + jj, a.par);
    int r = site;
    int c[4];
    c[0] = r % g.lx; r /= g.lx;
    c[1] = r % g.ly; r /= g.ly;
    c[2] = r % g.lz;
    c[3] = r / g.lz;
    const int ext[4] = {g.lx, g.ly, g.lz, g.lt};
    c[mu] = (d & 1) ? (c[mu] == 0 ? ext[mu] - 1 : c[mu] - 1) : (c[mu] + 1 == ext[mu] ? 0 : c[mu] + 1);
    reinterpret_cast<int*>(smem_raw + jj * RS + SrRec<T>::off_nb)[d] =
        c[0] + g.lx * (c[1] + g.ly * (c[2] + g.lz * c[3]));
  }
  __syncthreads();
  if (a.hops) {
    for (int idx = threadIdx.x; idx < 36 * nsites; idx += blockDim.x) {
      const int me = idx / nsites;  // mu * 9 + e
      const int jj = idx - me * nsites;
      const int mu = me / 9;
      const T f = (mu == 3) ? T(2) * a.f : a.f;
      const int site = eo_site(g, c0 + jj, a.par);
      const int nbm = reinterpret_cast<const int*>(smem_raw + jj * RS + SrRec<T>::off_nb)[2 * mu + 1];
      const long long arr = (long long)me * V;
      const cpx<T> uf = a.links[arr + site], ub = a.links[arr + nbm];
      reinterpret_cast<cpx<T>*>(smem_raw + jj * RS + SrRec<T>::off_lf)[me] = mk(f * uf.re, f * uf.im);
      reinterpret_cast<cpx<T>*>(smem_raw + jj * RS + SrRec<T>::off_lb)[me] = mk(f * ub.re, f * ub.im);
    }
  }
  if constexpr (CLOV) {
    for (int idx = threadIdx.x; idx < NV * nsites; idx += blockDim.x) {
      const int q = idx / nsites;
      const int jj = idx - q * nsites;
      reinterpret_cast<VecT*>(smem_raw + jj * RS + SrRec<T>::off_cl)[q] =
          a.clov[(long long)q * V + eo_site(g, c0 + jj, a.par)];
    }
  }
}

// the workgroup's first compact position: consecutive workgroups on one XCD
// cover consecutive positions
__device__ __forceinline__ int eo_first(int S) {
  const int nb = gridDim.x, b = blockIdx.x;
  const int blk = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  return blk * S;
}

template <typename T, bool DAG, int CEN, bool POST, bool COMPACT>
__global__ void __launch_bounds__(kThreads) k_eo(EoArgs<T> a) {
  if (a.ctl != nullptr && a.ctl->state != ST_RUNNING) return;
  constexpr int RS = SrRec<T>::stride;
  constexpr bool CLOV = (CEN == EO_CEN_A || CEN == EO_CEN_AINV || POST);
  const Geom g = a.g;
  const int L = a.L, S = a.spw, V = g.vol, Vh = V >> 1;
  const int c0 = eo_first(S);
  const int nsites = min(S, Vh - c0);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (nsites > 0) eo_stage<T, CLOV>(a, smem_raw, c0, nsites);
  __syncthreads();
  const int j = threadIdx.x / L;
  const int l = threadIdx.x - j * L;
  if (j < nsites) {
    const unsigned char* rec = smem_raw + j * RS;
    const int site = eo_site(g, c0 + j, a.par);
    if constexpr (COMPACT) site_eo<T, DAG, CEN, POST>(a, rec, AddrHalf{(long long)Vh * L, L}, site, l);
    else site_eo<T, DAG, CEN, POST>(a, rec, Addr64<false>{L, V}, site, l);
  }
}

// The second launch of the Schur operator on 8-column FP32 blocks, W' =
// A_ee T - kappa H_eo tmp on the compact even sites, which also sums the
// fused frame's Grams T^H W', W'^H W' and R~0^H W' over its sites into one
// FP64 partial record per workgroup (in_c = T and rt = R~0, both compact),
// as k_dslash_srg does on the whole lattice.
template <bool DAG>
__global__ void __launch_bounds__(kThreads, 5) k_eo_gram(EoArgs<float> a) {
  if (a.ctl != nullptr && a.ctl->state != ST_RUNNING) return;
  constexpr int RS = SrRec<float>::stride;
  const int Vh = a.g.vol >> 1;
  const int c0 = eo_first(a.spw);
  const int nsites = min(a.spw, Vh - c0);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (nsites > 0) eo_stage<float, true>(a, smem_raw, c0, nsites);
  __syncthreads();
  const int j = threadIdx.x >> 3, l = threadIdx.x & 7;
  const AddrHalf ad{(long long)Vh * 8, 8};
  const bool act = j < nsites;
  const int site = act ? eo_site(a.g, c0 + j, a.par) : 0;
  cpx<float> wout[12];
  if (act) {
    site_eo<float, DAG, EO_CEN_A, false, AddrHalf, true>(a, smem_raw + j * RS, ad, site, l, wout);
  } else {
#pragma unroll
    for (int sc = 0; sc < 12; ++sc) wout[sc] = mk(0.f, 0.f);
  }
  f32x4 acc[3];
  gram3_rows(a.in_c, a.rt, ad, site, l, act, wout, acc);
  // the records are no longer read: the LDS takes the sums
  __syncthreads();
  gram3_flush(acc, smem_raw, a.partials + (long long)blockIdx.x * 384);
}

template <typename T>
DslashArgs<T> make_args(const LatticeImpl& lat, int L, const cpx<T>* in, cpx<T>* out, const Control* ctl);

template <>
DslashArgs<double> make_args<double>(const LatticeImpl& lat, int L, const cpx<double>* in, cpx<double>* out,
                                     const Control* ctl) {
  DslashArgs<double> a{};
  a.in = in; a.out = out; a.links = lat.links64; a.links_c = nullptr;
  a.clover = reinterpret_cast<const double2*>(lat.clover64);
  a.ctl = ctl; a.g = lat.g; a.L = L; a.kappa = lat.kappa;
  return a;
}

template <>
DslashArgs<float> make_args<float>(const LatticeImpl& lat, int L, const cpx<float>* in, cpx<float>* out,
                                   const Control* ctl) {
  DslashArgs<float> a{};
  a.in = in; a.out = out; a.links = lat.links32; a.links_c = lat.links32c;
  a.clover = reinterpret_cast<const float4*>(lat.clover32);
  a.ctl = ctl; a.g = lat.g; a.L = L; a.kappa = (float)lat.kappa;
  return a;
}

template <typename T, int EPI, bool CM, int NR>
hipError_t dispatch(const DslashArgs<T>& a, int dagger, bool comp, int grid, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (comp) {
      if (dagger) hipLaunchKernelGGL((k_dslash<T, true, true, EPI, CM, NR>), dim3(grid), dim3(kThreads), 0, s, a);
      else hipLaunchKernelGGL((k_dslash<T, false, true, EPI, CM, NR>), dim3(grid), dim3(kThreads), 0, s, a);
      return hipGetLastError();
    }
  }
  if (dagger) hipLaunchKernelGGL((k_dslash<T, true, false, EPI, CM, NR>), dim3(grid), dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((k_dslash<T, false, false, EPI, CM, NR>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

// columns per thread: 2 for even L (one 16-byte load covers a thread's two
// FP32 columns), else 1
#ifndef BKWD_DSLASH_NR
#define BKWD_DSLASH_NR 1
#endif
int cols_per_thread(int L) { return (L % 2 == 0) ? BKWD_DSLASH_NR : 1; }

// the staged kernel serves L >= kStageMinL (for smaller L a workgroup would
// hold too many sites' links in LDS: 64 sites, 55 KB, at L = 4; 221 KB at
// L = 1).  At L = 4 it beats the direct kernel by about a third per column.
#ifndef BKWD_STAGE_MIN_L
#define BKWD_STAGE_MIN_L 4
#endif
constexpr int kStageMinL = BKWD_STAGE_MIN_L;

template <typename T>
size_t staged_smem(int S, bool comp) {
  const int NC = comp ? 6 : 9;
  return (size_t)CloverVec<T>::n * S * sizeof(typename CloverVec<T>::type) + (size_t)8 * NC * S * sizeof(cpx<T>);
}

template <typename T, bool CM>
hipError_t dispatch_sr(const DslashArgs<T>& a, int dagger, int grid, hipStream_t s) {
  const size_t smem = (size_t)SrRec<T>::stride * a.spw;
  if (dagger) hipLaunchKernelGGL((k_dslash_sr<T, true, CM>), dim3(grid), dim3(kThreads), smem, s, a);
  else hipLaunchKernelGGL((k_dslash_sr<T, false, CM>), dim3(grid), dim3(kThreads), smem, s, a);
  return hipGetLastError();
}

// the folded-link record kernel serves the plain epilogue with full links
#ifdef BKWD_NO_SR_DSLASH
constexpr bool kSrDslash = false;
#else
constexpr bool kSrDslash = true;
#endif

template <typename T, int EPI, bool CM>
hipError_t dispatch_staged(const DslashArgs<T>& a, int dagger, bool comp, int grid, hipStream_t s) {
  if constexpr (EPI == EPI_PLAIN) {
    if (kSrDslash && !comp) return dispatch_sr<T, CM>(a, dagger, grid, s);
  }
  const size_t smem = staged_smem<T>(a.spw, comp);
  if constexpr (std::is_same<T, float>::value) {
    if (comp) {
      if (dagger) hipLaunchKernelGGL((k_dslash_st<T, true, true, EPI, CM>), dim3(grid), dim3(kThreads), smem, s, a);
      else hipLaunchKernelGGL((k_dslash_st<T, false, true, EPI, CM>), dim3(grid), dim3(kThreads), smem, s, a);
      return hipGetLastError();
    }
  }
  if (dagger) hipLaunchKernelGGL((k_dslash_st<T, true, false, EPI, CM>), dim3(grid), dim3(kThreads), smem, s, a);
  else hipLaunchKernelGGL((k_dslash_st<T, false, false, EPI, CM>), dim3(grid), dim3(kThreads), smem, s, a);
  return hipGetLastError();
}

template <typename T, int EPI, bool CM>
hipError_t dispatch_nr(const DslashArgs<T>& a, int dagger, bool comp, int nr, int grid, hipStream_t s) {
#if BKWD_DSLASH_NR == 2
  if (nr == 2) return dispatch<T, EPI, CM, 2>(a, dagger, comp, grid, s);
#endif
  (void)nr;
  return dispatch<T, EPI, CM, 1>(a, dagger, comp, grid, s);
}

// one-pass grid in the t-slice layout: Lt slices x 8 XCDs x wpx workgroups
int slab_wpx(const Geom& g, int L) {
  const long long per_slice = (long long)g.lx * g.ly * g.lz * (L / cols_per_thread(L));
  return (int)((per_slice + 8LL * kThreads - 1) / (8LL * kThreads));
}

}  // namespace

// staged grid: whole sites per workgroup
int staged_spw(int L) { return kThreads / L; }
int staged_wpx(const Geom& g, int L) {
  const int sps = g.lx * g.ly * g.lz;
  const int wg_per_slice = (sps + staged_spw(L) - 1) / staged_spw(L);
  return (wg_per_slice + 7) / 8;
}

// upper bound on the workgroups of a one-pass launch (sizes the partial sums)
int dslash_launch_grid(const Geom& g, int L) {
  return g.lt * 8 * std::max(L >= kStageMinL ? staged_wpx(g, L) : 0, slab_wpx(g, L));
}

template <typename T>
hipError_t launch_dslash(const LatticeImpl& lat, int dagger, int L, const cpx<T>* in, cpx<T>* out, double* epi,
                         int* nblk_out, const Control* ctl, bool comp_major, hipStream_t s) {
  DslashArgs<T> a = make_args<T>(lat, L, in, out, ctl);
  const bool comp = (lat.flags & 1u) && lat.links32c != nullptr;
  const bool off32 = (unsigned long long)lat.g.vol * L * sizeof(cpx<T>) < (1ull << 32);
  if (L >= kStageMinL && (off32 || !comp_major)) {
    a.spw = staged_spw(L);
    a.wpx = staged_wpx(lat.g, L);
    const int grid = lat.g.lt * 8 * a.wpx;
    if (nblk_out) *nblk_out = grid;
    if (epi) {
      a.partials = epi;
      return comp_major ? dispatch_staged<T, EPI_TRACE, true>(a, dagger, comp, grid, s)
                        : dispatch_staged<T, EPI_TRACE, false>(a, dagger, comp, grid, s);
    }
    return comp_major ? dispatch_staged<T, EPI_PLAIN, true>(a, dagger, comp, grid, s)
                      : dispatch_staged<T, EPI_PLAIN, false>(a, dagger, comp, grid, s);
  }
  a.wpx = slab_wpx(lat.g, L);
  const int grid = lat.g.lt * 8 * a.wpx;
  if (nblk_out) *nblk_out = grid;
  const int nr = cols_per_thread(L);
  if (epi) {
    a.partials = epi;
    return comp_major ? dispatch_nr<T, EPI_TRACE, true>(a, dagger, comp, nr, grid, s)
                      : dispatch_nr<T, EPI_TRACE, false>(a, dagger, comp, nr, grid, s);
  }
  return comp_major ? dispatch_nr<T, EPI_PLAIN, true>(a, dagger, comp, nr, grid, s)
                    : dispatch_nr<T, EPI_PLAIN, false>(a, dagger, comp, nr, grid, s);
}

// W' = A T (dagger: A^dagger T) for an 8-column FP32 component-major block,
// with the partial Grams T^H W', W'^H W', R~0^H W' of every workgroup in
// partials ([nblk][384] doubles)
bool dslash_gram_supported(const LatticeImpl& lat, int L) {
  const bool comp = (lat.flags & 1u) && lat.links32c != nullptr;
  return kSrDslash && L == 8 && !comp && (unsigned long long)lat.g.vol * 8 * sizeof(cpx<float>) < (1ull << 32);
}

hipError_t launch_dslash_gram(const LatticeImpl& lat, int dagger, const cpx<float>* in, cpx<float>* out,
                              const cpx<float>* rt, double* partials, int* nblk_out, const Control* ctl,
                              hipStream_t s) {
  if (!dslash_gram_supported(lat, 8)) return hipErrorInvalidValue;
  DslashArgs<float> a = make_args<float>(lat, 8, in, out, ctl);
  a.b = rt;
  a.partials = partials;
  a.spw = staged_spw(8);
  a.wpx = staged_wpx(lat.g, 8);
  const int nparts = lat.g.lt * 8 * a.wpx;
  const int grid = nparts;  // = dslash_launch_grid(lat.g, 8): the workspace's partial records
  const size_t smem = (size_t)SrRec<float>::stride * a.spw;
  static_assert((size_t)SrRec<float>::stride * (kThreads / 8) >= 4 * 3 * 256 * sizeof(double),
                "the cross-wave Gram sums reuse the site records' LDS");
  if (nblk_out) *nblk_out = grid;
  if (dagger) hipLaunchKernelGGL(k_dslash_srg<true>, dim3(grid), dim3(kThreads), smem, s, a);
  else hipLaunchKernelGGL(k_dslash_srg<false>, dim3(grid), dim3(kThreads), smem, s, a);
  return hipGetLastError();
}

template hipError_t launch_dslash<double>(const LatticeImpl&, int, int, const cpx<double>*, cpx<double>*, double*,
                                          int*, const Control*, bool, hipStream_t);
template hipError_t launch_dslash<float>(const LatticeImpl&, int, int, const cpx<float>*, cpx<float>*, double*,
                                         int*, const Control*, bool, hipStream_t);

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

hipError_t launch_residual64(const LatticeImpl& lat, int dagger, int L, const cpx<double>* b, const cpx<double>* x,
                             cpx<double>* r, double* partials, int* nblk_out, hipStream_t s) {
  DslashArgs<double> a = make_args<double>(lat, L, x, r, nullptr);
  a.b = b;
  a.partials = partials;
  const int grid = residual_grid(lat.g.vol, L);
  if (nblk_out) *nblk_out = grid;
  if (dagger) hipLaunchKernelGGL((k_dslash<double, true, false, EPI_RESID, false, 1>), dim3(grid), dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((k_dslash<double, false, false, EPI_RESID, false, 1>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

// ||b_i - D x_i||^2 and ||b_i||^2 per column only (nothing else is stored):
// per-workgroup partial sums [nblk][2L] into `partials`
hipError_t launch_residual_norms64(const LatticeImpl& lat, int dagger, int L, const cpx<double>* b,
                                   const cpx<double>* x, double* partials, int* nblk_out, hipStream_t s) {
  DslashArgs<double> a = make_args<double>(lat, L, x, nullptr, nullptr);
  a.b = b;
  a.partials = partials;
  const int grid = residual_grid(lat.g.vol, L);
  if (nblk_out) *nblk_out = grid;
  if (dagger) hipLaunchKernelGGL((k_dslash<double, true, false, EPI_NORMS, false, 1>), dim3(grid), dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((k_dslash<double, false, false, EPI_NORMS, false, 1>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_grad_scalars(const LatticeImpl& lat, int L, const cpx<double>* x, const cpx<double>* lam,
                               const double* unit_clover, double csw, double* partials, int* nblk_out, hipStream_t s) {
  DslashArgs<double> a = make_args<double>(lat, L, x, nullptr, nullptr);
  a.clover = reinterpret_cast<const double2*>(unit_clover);
  a.b = lam;
  a.aux = csw;
  a.partials = partials;
  const int grid = residual_grid(lat.g.vol, L);
  if (nblk_out) *nblk_out = grid;
  hipLaunchKernelGGL((k_dslash<double, false, false, EPI_GRAD, false, 1>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

// workgroup shape of the even-odd kernels: S sites x L columns, with the
// site records within 64 KiB of LDS and at most 256 threads
template <typename T>
static int eo_spw(int L) { return std::min(65536 / SrRec<T>::stride, kThreads / L); }

template <typename T, bool DAG, int CEN, bool POST, bool COMPACT>
static hipError_t eo_go(const EoArgs<T>& a, hipStream_t s) {
  const int Vh = a.g.vol / 2;
  const int grid = (Vh + a.spw - 1) / a.spw;
  const size_t smem = (size_t)SrRec<T>::stride * a.spw;
  hipLaunchKernelGGL((k_eo<T, DAG, CEN, POST, COMPACT>), dim3(grid), dim3(a.spw * a.L), smem, s, a);
  return hipGetLastError();
}

template <typename T, int CEN, bool POST, bool COMPACT>
static hipError_t eo_dag(const EoArgs<T>& a, int dagger, hipStream_t s) {
  return dagger ? eo_go<T, true, CEN, POST, COMPACT>(a, s) : eo_go<T, false, CEN, POST, COMPACT>(a, s);
}

template <typename T>
static EoArgs<T> eo_args(const LatticeImpl& lat, int L, int par, const Control* ctl);

template <>
EoArgs<double> eo_args<double>(const LatticeImpl& lat, int L, int par, const Control* ctl) {
  EoArgs<double> a{};
  a.links = lat.links64;
  a.g = lat.g; a.L = L; a.par = par; a.spw = eo_spw<double>(L); a.ctl = ctl;
  return a;
}

template <>
EoArgs<float> eo_args<float>(const LatticeImpl& lat, int L, int par, const Control* ctl) {
  EoArgs<float> a{};
  a.links = lat.links32;
  a.g = lat.g; a.L = L; a.par = par; a.spw = eo_spw<float>(L); a.ctl = ctl;
  return a;
}

// Schur operator on compact even blocks: out = A_ee in - kappa^2 H_eo A_oo^{-1} H_oe in,
// as tmp = A_oo^{-1} (kappa H_oe in), then out = A_ee in - kappa H_eo tmp
template <typename T>
hipError_t launch_schur(const LatticeImpl& lat, int dagger, int L, const cpx<T>* in, cpx<T>* out, cpx<T>* tmp,
                        const void* clover, const void* cinv, const Control* ctl, hipStream_t s) {
  using VecT = typename CloverVec<T>::type;
  EoArgs<T> a = eo_args<T>(lat, L, 1, ctl);
  a.in_h = in; a.out = tmp; a.hops = 1; a.f = (T)lat.kappa;
  a.clov = static_cast<const VecT*>(cinv);
  hipError_t e = eo_dag<T, EO_CEN_NONE, true, true>(a, dagger, s);
  if (e != hipSuccess) return e;
  EoArgs<T> b = eo_args<T>(lat, L, 0, ctl);
  b.in_c = in; b.in_h = tmp; b.out = out; b.hops = 1; b.f = (T)(-lat.kappa);
  b.clov = static_cast<const VecT*>(clover);
  return eo_dag<T, EO_CEN_A, false, true>(b, dagger, s);
}

template hipError_t launch_schur<float>(const LatticeImpl&, int, int, const cpx<float>*, cpx<float>*, cpx<float>*,
                                        const void*, const void*, const Control*, hipStream_t);
template hipError_t launch_schur<double>(const LatticeImpl&, int, int, const cpx<double>*, cpx<double>*, cpx<double>*,
                                         const void*, const void*, const Control*, hipStream_t);

bool schur_gram_supported(const LatticeImpl& lat, int L) {
  return L == 8 && eo_spw<float>(8) * 8 == kThreads &&
         (unsigned long long)(lat.g.vol / 2) * 8 * sizeof(cpx<float>) < (1ull << 32);
}

int schur_gram_grid(const Geom& g) {
  const int S = eo_spw<float>(8);
  return (g.vol / 2 + S - 1) / S;
}

hipError_t launch_schur_gram(const LatticeImpl& lat, int dagger, const cpx<float>* in, cpx<float>* out,
                             cpx<float>* tmp, const void* clover, const void* cinv, const cpx<float>* rt,
                             double* partials, int* nblk_out, const Control* ctl, hipStream_t s) {
  using VecT = CloverVec<float>::type;
  if (!schur_gram_supported(lat, 8)) return hipErrorInvalidValue;
  EoArgs<float> a = eo_args<float>(lat, 8, 1, ctl);
  a.in_h = in; a.out = tmp; a.hops = 1; a.f = (float)lat.kappa;
  a.clov = static_cast<const VecT*>(cinv);
  hipError_t e = eo_dag<float, EO_CEN_NONE, true, true>(a, dagger, s);
  if (e != hipSuccess) return e;
  EoArgs<float> b = eo_args<float>(lat, 8, 0, ctl);
  b.in_c = in; b.in_h = tmp; b.out = out; b.hops = 1; b.f = (float)(-lat.kappa);
  b.clov = static_cast<const VecT*>(clover);
  b.rt = rt; b.partials = partials;
  const int grid = schur_gram_grid(lat.g);
  const size_t smem = (size_t)SrRec<float>::stride * b.spw;
  static_assert((size_t)SrRec<float>::stride * (kThreads / 8) >= 4 * 3 * 256 * sizeof(double),
                "the cross-wave Gram sums reuse the site records' LDS");
  if (nblk_out) *nblk_out = grid;
  if (dagger) hipLaunchKernelGGL(k_eo_gram<true>, dim3(grid), dim3(kThreads), smem, s, b);
  else hipLaunchKernelGGL(k_eo_gram<false>, dim3(grid), dim3(kThreads), smem, s, b);
  return hipGetLastError();
}

// FP64 whole-lattice site-major steps of the even-odd solve:
//   eo_prepare:     w_o = A_oo^{-1} r_o, then w_e = r_e + kappa H_eo w_o
//   eo_reconstruct: w_o = A_oo^{-1} (r_o + kappa H_oe w_e)   (w_e holds x_e)
hipError_t launch_eo_prepare(const LatticeImpl& lat, int dagger, int L, const cpx<double>* r, cpx<double>* w,
                             const double* cinv64, hipStream_t s) {
  EoArgs<double> a = eo_args<double>(lat, L, 1, nullptr);
  a.in_c = r; a.out = w; a.hops = 0;
  a.clov = reinterpret_cast<const double2*>(cinv64);
  hipError_t e = eo_dag<double, EO_CEN_AINV, false, false>(a, dagger, s);
  if (e != hipSuccess) return e;
  EoArgs<double> b = eo_args<double>(lat, L, 0, nullptr);
  b.in_c = r; b.in_h = w; b.out = w; b.hops = 1; b.f = lat.kappa;
  return eo_dag<double, EO_CEN_ID, false, false>(b, dagger, s);
}

hipError_t launch_eo_reconstruct(const LatticeImpl& lat, int dagger, int L, const cpx<double>* r, cpx<double>* w,
                                 const double* cinv64, hipStream_t s) {
  EoArgs<double> a = eo_args<double>(lat, L, 1, nullptr);
  a.in_c = r; a.in_h = w; a.out = w; a.hops = 1; a.f = lat.kappa;
  a.clov = reinterpret_cast<const double2*>(cinv64);
  return eo_dag<double, EO_CEN_ID, true, false>(a, dagger, s);
}
