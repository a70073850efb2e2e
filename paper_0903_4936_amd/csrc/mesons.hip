// Pion and rho two-point functions contracted from the 12 point-source
// solutions (the downstream use of the L = 12 solves: the columns of X are
// the quark propagator from the origin).
//
// With S(x) the 12 x 12 propagator at site x (rows and columns ordered
// 3 * spin + colour, column i = colour + 3 * spin of the point source of
// Sec. 2) and gamma_5-hermiticity S(0, x) = gamma_5 S(x, 0)^dagger gamma_5,
// the Wick contraction of psibar G psi is, per time slice t,
//   C_G(t) = - sum_x Re Tr[A S(x) B S(x)^dagger],  A = gamma_5 G,
//   B = gamma_4 G^dagger gamma_4 gamma_5,
// trace over spin and colour.  Every gamma matrix of Sec. 2 has one non-zero
// per row, so A and B are monomial and, for one colour pair (a, b),
//   Tr_spin = sum_{alpha, beta} A[alpha] B[beta]
//             s[pa(alpha)][beta] conj(s[alpha][pb(beta)]),
//   s[alpha][beta] = S[(alpha, a), (beta, b)].
// Pion: G = gamma_5.  Rho: G = gamma_k, averaged over k = 1, 2, 3.
#include "bkwd_internal.h"

namespace {

constexpr int kMesonThreads = 512;

// a 4 x 4 matrix with one non-zero per row: row r holds v[r] at column c[r]
struct Mono {
  int c[4];
  double re[4], im[4];
};

constexpr Mono mono_mul(const Mono& x, const Mono& y) {  // x y
  Mono p{};
  for (int r = 0; r < 4; ++r) {
    const int k = x.c[r];
    p.c[r] = y.c[k];
    p.re[r] = x.re[r] * y.re[k] - x.im[r] * y.im[k];
    p.im[r] = x.re[r] * y.im[k] + x.im[r] * y.re[k];
  }
  return p;
}

constexpr Mono mono_dag(const Mono& x) {
  Mono d{};
  for (int r = 0; r < 4; ++r) {
    d.c[x.c[r]] = r;
    d.re[x.c[r]] = x.re[r];
    d.im[x.c[r]] = -x.im[r];
  }
  return d;
}

// the gamma matrices of Sec. 2 (rows and columns 0-based)
constexpr Mono kGamma[4] = {
    {{3, 2, 1, 0}, {0, 0, 0, 0}, {-1, -1, 1, 1}},    // gamma_1
    {{3, 2, 1, 0}, {-1, 1, 1, -1}, {0, 0, 0, 0}},    // gamma_2
    {{2, 3, 0, 1}, {0, 0, 0, 0}, {-1, 1, 1, -1}},    // gamma_3
    {{0, 1, 2, 3}, {1, 1, -1, -1}, {0, 0, 0, 0}},    // gamma_4
};
constexpr Mono kGamma5 = {{2, 3, 0, 1}, {1, 1, 1, 1}, {0, 0, 0, 0}};

// the four channels: pion and rho_1..3
struct MesonTab {
  int pa[4][4], pb[4][4];
  double ar[4][4], ai[4][4], br[4][4], bi[4][4];
};

constexpr MesonTab meson_tables() {
  MesonTab t{};
  const Mono G[4] = {kGamma5, kGamma[0], kGamma[1], kGamma[2]};
  for (int ch = 0; ch < 4; ++ch) {
    const Mono A = mono_mul(kGamma5, G[ch]);
    const Mono B = mono_mul(mono_mul(mono_mul(kGamma[3], mono_dag(G[ch])), kGamma[3]), kGamma5);
    for (int r = 0; r < 4; ++r) {
      t.pa[ch][r] = A.c[r];
      t.ar[ch][r] = A.re[r];
      t.ai[ch][r] = A.im[r];
      t.pb[ch][r] = B.c[r];
      t.br[ch][r] = B.re[r];
      t.bi[ch][r] = B.im[r];
    }
  }
  return t;
}

// compile-time tables: after unrolling every index into s[][] is a constant
constexpr MesonTab kTab = meson_tables();

// One workgroup per time slice t (sites t Vs .. (t + 1) Vs - 1); each thread
// takes sites in a stride, each site once per colour pair.  Fixed-order LDS
// reduction; thread 0 writes pion[t] and rho[t].
__global__ void __launch_bounds__(kMesonThreads) k_mesons(const cpx<double>* __restrict__ X, int vs,
                                                          double* __restrict__ pion, double* __restrict__ rho) {
  __shared__ double red[2][kMesonThreads];
  const int t = blockIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int xs = threadIdx.x; xs < vs; xs += kMesonThreads) {
    const cpx<double>* Sx = X + ((long long)t * vs + xs) * 144;  // [4][3][12]
#pragma unroll 1
    for (int a = 0; a < 3; ++a) {
#pragma unroll 1
      for (int b = 0; b < 3; ++b) {
        cpx<double> s[4][4];
#pragma unroll
        for (int al = 0; al < 4; ++al)
#pragma unroll
          for (int be = 0; be < 4; ++be) s[al][be] = Sx[(al * 3 + a) * 12 + be * 3 + b];
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
          double sre = 0.0;
#pragma unroll
          for (int al = 0; al < 4; ++al) {
#pragma unroll
            for (int be = 0; be < 4; ++be) {
              const cpx<double> u = s[kTab.pa[ch][al]][be];
              const cpx<double> v = s[al][kTab.pb[ch][be]];
              // c = A[al] B[be];  Re(c u conj(v))
              const double cr = kTab.ar[ch][al] * kTab.br[ch][be] - kTab.ai[ch][al] * kTab.bi[ch][be];
              const double ci = kTab.ar[ch][al] * kTab.bi[ch][be] + kTab.ai[ch][al] * kTab.br[ch][be];
              const double wr = u.re * v.re + u.im * v.im;  // u conj(v)
              const double wi = u.im * v.re - u.re * v.im;
              sre += cr * wr - ci * wi;
            }
          }
          acc[ch] -= sre;
        }
      }
    }
  }
  red[0][threadIdx.x] = acc[0];
  red[1][threadIdx.x] = (acc[1] + acc[2] + acc[3]) / 3.0;
  __syncthreads();
  for (int h = kMesonThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pion[t] = red[0][0];
    rho[t] = red[1][0];
  }
}

}  // namespace

hipError_t launch_mesons(const LatticeImpl& lat, const cpx<double>* X, double* pion, double* rho, hipStream_t s) {
  const int vs = lat.g.lx * lat.g.ly * lat.g.lz;
  hipLaunchKernelGGL(k_mesons, dim3(lat.g.lt), dim3(kMesonThreads), 0, s, X, vs, pion, rho);
  return hipGetLastError();
}
