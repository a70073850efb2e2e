/*
 * The oracle's operator D_W (Sec. 2, Eq. (1)) written out in plain C, FP64,
 * site by site, for whole-lattice residual checks at lattice sizes where the
 * NumPy oracle (oracle/dirac.py) takes too long.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/ through oracle/native.py,
 * never by the HIP library.  It shares no code with the library.  It is
 * checked against oracle/dirac.py and against the closed forms the NumPy
 * oracle is pinned by (tests/test_oracle_native.py).
 *
 * Layouts (those of the NumPy oracle, flattened):
 *   links U: [4][V][3][3] complex, U[mu][site][a][b] = U_mu(n, a, b);
 *   fields:  [V][4][3][L] complex, spin alpha, colour a, column l;
 *   local matrix M: [V][12][12] complex, row and column 3 * alpha + a;
 * with site = x + Lx * (y + Ly * (z + Lz * t)), periodic in every direction.
 * Complex values are pairs of doubles (re, im).
 *
 * Readings (the same as the NumPy oracle's): the first and fourth clover
 * leaves are the closed plaquettes (third factor of P_1 is U_mu^dagger(n+nu),
 * second factor of P_4 is U_mu(n-nu)); F_{mu nu} keeps its trace; the clover
 * sum runs over all ordered pairs (mu, nu).
 *
 * Arithmetic is written as plain loops in the order of the definitions; the
 * only parallelism is an OpenMP loop over sites.
 */
#include <complex.h>
#include <string.h>

typedef double complex cplx;

/* Euclidean gamma matrices of Sec. 2 (0-based rows and columns). */
static cplx gam[4][4][4];

static void set_gammas(void) {
  memset(gam, 0, sizeof(gam));
  /* gamma_1 */
  gam[0][0][3] = -I; gam[0][1][2] = -I; gam[0][2][1] = I; gam[0][3][0] = I;
  /* gamma_2 */
  gam[1][0][3] = -1; gam[1][1][2] = 1; gam[1][2][1] = 1; gam[1][3][0] = -1;
  /* gamma_3 */
  gam[2][0][2] = -I; gam[2][1][3] = I; gam[2][2][0] = I; gam[2][3][1] = -I;
  /* gamma_4 */
  gam[3][0][0] = 1; gam[3][1][1] = 1; gam[3][2][2] = -1; gam[3][3][3] = -1;
}

typedef struct {
  int d[4];  /* Lx, Ly, Lz, Lt */
  long long vol;
} geom;

static geom make_geom(const int dims[4]) {
  geom g;
  g.vol = 1;
  for (int k = 0; k < 4; ++k) {
    g.d[k] = dims[k];
    g.vol *= dims[k];
  }
  return g;
}

static void coords(const geom* g, long long site, int c[4]) {
  for (int k = 0; k < 4; ++k) {
    c[k] = (int)(site % g->d[k]);
    site /= g->d[k];
  }
}

/* site index of c + s * e_mu + s2 * e_nu, periodic */
static long long index_of(const geom* g, const int c[4], int mu, int s, int nu, int s2) {
  int cc[4] = {c[0], c[1], c[2], c[3]};
  cc[mu] += s;
  cc[nu] += s2;
  long long idx = 0;
  for (int k = 3; k >= 0; --k) idx = idx * g->d[k] + ((cc[k] % g->d[k]) + g->d[k]) % g->d[k];
  return idx;
}

static const cplx* link(const cplx* U, const geom* g, int mu, long long site) {
  return U + ((long long)mu * g->vol + site) * 9;
}

/* c = a * b, or with a and/or b conjugate-transposed */
static void mul3(const cplx* a, int adag, const cplx* b, int bdag, cplx* c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = 0;
      for (int k = 0; k < 3; ++k) {
        const cplx x = adag ? conj(a[k * 3 + i]) : a[i * 3 + k];
        const cplx y = bdag ? conj(b[j * 3 + k]) : b[k * 3 + j];
        s += x * y;
      }
      c[i * 3 + j] = s;
    }
}

/* product of four links, each optionally daggered */
static void loop4(const cplx* l0, int d0, const cplx* l1, int d1, const cplx* l2, int d2, const cplx* l3, int d3,
                  cplx* out) {
  cplx t1[9], t2[9];
  mul3(l0, d0, l1, d1, t1);
  mul3(t1, 0, l2, d2, t2);
  mul3(t2, 0, l3, d3, out);
}

/* F_{mu nu}(n) = 1/4 sum_i (P_i - P_i^dagger) / (2i), leaves of Sec. 2 */
static void field_strength(const cplx* U, const geom* g, long long site, int mu, int nu, cplx F[9]) {
  int c[4];
  coords(g, site, c);
  cplx P[4][9];
  /* P_1 = U_mu(n) U_nu(n+mu) U_mu^+(n+nu) U_nu^+(n) */
  loop4(link(U, g, mu, site), 0, link(U, g, nu, index_of(g, c, mu, 1, nu, 0)), 0,
        link(U, g, mu, index_of(g, c, nu, 1, mu, 0)), 1, link(U, g, nu, site), 1, P[0]);
  /* P_2 = U_nu(n) U_mu^+(n-mu+nu) U_nu^+(n-mu) U_mu(n-mu) */
  loop4(link(U, g, nu, site), 0, link(U, g, mu, index_of(g, c, mu, -1, nu, 1)), 1,
        link(U, g, nu, index_of(g, c, mu, -1, nu, 0)), 1, link(U, g, mu, index_of(g, c, mu, -1, nu, 0)), 0, P[1]);
  /* P_3 = U_mu^+(n-mu) U_nu^+(n-mu-nu) U_mu(n-mu-nu) U_nu(n-nu) */
  loop4(link(U, g, mu, index_of(g, c, mu, -1, nu, 0)), 1, link(U, g, nu, index_of(g, c, mu, -1, nu, -1)), 1,
        link(U, g, mu, index_of(g, c, mu, -1, nu, -1)), 0, link(U, g, nu, index_of(g, c, nu, -1, mu, 0)), 0, P[2]);
  /* P_4 = U_nu^+(n-nu) U_mu(n-nu) U_nu(n+mu-nu) U_mu^+(n) */
  loop4(link(U, g, nu, index_of(g, c, nu, -1, mu, 0)), 1, link(U, g, mu, index_of(g, c, nu, -1, mu, 0)), 0,
        link(U, g, nu, index_of(g, c, mu, 1, nu, -1)), 0, link(U, g, mu, site), 1, P[3]);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cplx s = 0;
      for (int i = 0; i < 4; ++i) s += (P[i][a * 3 + b] - conj(P[i][b * 3 + a])) / (2.0 * I);
      F[a * 3 + b] = s / 4.0;
    }
}

/* M(n) = 1 - kappa csw sum_{mu,nu} (i/2) sigma_{mu nu} (x) F_{mu nu}(n),
   sigma_{mu nu} = (gamma_mu gamma_nu - gamma_nu gamma_mu) / 2 */
int oracle_local_matrix(const int dims[4], const double* Ud, double kappa, double csw, double* Md) {
  set_gammas();
  const geom g = make_geom(dims);
  const cplx* U = (const cplx*)Ud;
  cplx* M = (cplx*)Md;
  cplx sigma[4][4][4][4];
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu)
      for (int r = 0; r < 4; ++r)
        for (int s = 0; s < 4; ++s) {
          cplx v = 0;
          for (int k = 0; k < 4; ++k) v += gam[mu][r][k] * gam[nu][k][s] - gam[nu][r][k] * gam[mu][k][s];
          sigma[mu][nu][r][s] = v / 2.0;
        }
#pragma omp parallel for schedule(static)
  for (long long site = 0; site < g.vol; ++site) {
    cplx C[12][12];
    memset(C, 0, sizeof(C));
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = 0; nu < 4; ++nu) {
        if (mu == nu) continue;
        cplx F[9];
        field_strength(U, &g, site, mu, nu, F);
        for (int r = 0; r < 4; ++r)
          for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b) C[3 * r + a][3 * s + b] += 0.5 * I * sigma[mu][nu][r][s] * F[a * 3 + b];
      }
    cplx* m = M + site * 144;
    for (int i = 0; i < 12; ++i)
      for (int j = 0; j < 12; ++j) m[i * 12 + j] = (i == j ? 1.0 : 0.0) - kappa * csw * C[i][j];
  }
  return 0;
}

/* (D X)(n) for all L columns into y[12][L] (dagger: D^dagger, for which the
   projectors (1 -/+ gamma_mu) swap and M, being Hermitian, stays) */
static void apply_site(const geom* g, const cplx* U, const cplx* M, double kappa, int L, const cplx* X, long long site,
                       int dagger, cplx* y, cplx* v) {
  int c[4];
  coords(g, site, c);
  const cplx* x0 = X + site * 12 * L;
  const cplx* m = M + site * 144;
  for (int i = 0; i < 12; ++i)
    for (int l = 0; l < L; ++l) {
      cplx s = 0;
      for (int j = 0; j < 12; ++j) s += m[i * 12 + j] * x0[j * L + l];
      y[i * L + l] = s;
    }
  const double sgn = dagger ? -1.0 : 1.0;
  for (int mu = 0; mu < 4; ++mu)
    for (int dir = 0; dir < 2; ++dir) {
      /* dir 0: (1 - sgn gamma_mu) U_mu(n) X(n + mu);  dir 1: (1 + sgn gamma_mu) U_mu^+(n - mu) X(n - mu) */
      const long long nb = index_of(g, c, mu, dir == 0 ? 1 : -1, mu, 0);
      const cplx* u = link(U, g, mu, dir == 0 ? site : nb);
      const cplx* xn = X + nb * 12 * L;
      /* colour: v[s][a][l] = sum_b u(a,b) x(s,b,l) or conj(u(b,a)) x(s,b,l) */
      for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a)
          for (int l = 0; l < L; ++l) {
            cplx acc = 0;
            for (int b = 0; b < 3; ++b) acc += (dir == 0 ? u[a * 3 + b] : conj(u[b * 3 + a])) * xn[(3 * s + b) * L + l];
            v[(3 * s + a) * L + l] = acc;
          }
      const double ps = dir == 0 ? -sgn : sgn;  /* spin matrix 1 + ps gamma_mu */
      for (int r = 0; r < 4; ++r)
        for (int s = 0; s < 4; ++s) {
          const cplx p = (r == s ? 1.0 : 0.0) + ps * gam[mu][r][s];
          if (p == 0) continue;
          for (int a = 0; a < 3; ++a)
            for (int l = 0; l < L; ++l) y[(3 * r + a) * L + l] -= kappa * p * v[(3 * s + a) * L + l];
        }
    }
}

/* Y = D X (or D^dagger X) for fields of L <= 64 columns */
int oracle_apply(const int dims[4], const double* Ud, const double* Md, double kappa, int L, const double* Xd,
                 double* Yd, int dagger) {
  if (L < 1 || L > 64) return -1;
  set_gammas();
  const geom g = make_geom(dims);
#pragma omp parallel
  {
    cplx v[12 * 64];
#pragma omp for schedule(static)
    for (long long site = 0; site < g.vol; ++site)
      apply_site(&g, (const cplx*)Ud, (const cplx*)Md, kappa, L, (const cplx*)Xd, site, dagger,
                 (cplx*)Yd + site * 12 * L, v);
  }
  return 0;
}

/* Per column l: r2[l] = ||b_l - D x_l||^2 and b2[l] = ||b_l||^2 over the
   whole lattice, the quantities of the true residual of Sec. 4.3. */
int oracle_residual(const int dims[4], const double* Ud, const double* Md, double kappa, int L, const double* Xd,
                    const double* Bd, int dagger, double* r2, double* b2) {
  if (L < 1 || L > 64) return -1;
  set_gammas();
  const geom g = make_geom(dims);
  for (int l = 0; l < L; ++l) r2[l] = b2[l] = 0.0;
#pragma omp parallel
  {
    cplx v[12 * 64], y[12 * 64];
    double pr[64], pb[64];
    for (int l = 0; l < L; ++l) pr[l] = pb[l] = 0.0;
#pragma omp for schedule(static)
    for (long long site = 0; site < g.vol; ++site) {
      apply_site(&g, (const cplx*)Ud, (const cplx*)Md, kappa, L, (const cplx*)Xd, site, dagger, y, v);
      const cplx* b = (const cplx*)Bd + site * 12 * L;
      for (int i = 0; i < 12; ++i)
        for (int l = 0; l < L; ++l) {
          const cplx r = b[i * L + l] - y[i * L + l];
          pr[l] += creal(r) * creal(r) + cimag(r) * cimag(r);
          pb[l] += creal(b[i * L + l]) * creal(b[i * L + l]) + cimag(b[i * L + l]) * cimag(b[i * L + l]);
        }
    }
#pragma omp critical
    for (int l = 0; l < L; ++l) {
      r2[l] += pr[l];
      b2[l] += pb[l];
    }
  }
  return 0;
}
