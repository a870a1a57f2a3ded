/*
 * oracle.c -- TEST INFRASTRUCTURE, not part of the product (see oracle.h).
 *
 * Plain FP64 C, IEEE arithmetic, no fast-math.  Each function follows one
 * passage of "Smoothing algorithms for projected center-vortex gauge fields"
 * (arXiv:2203.09764), cited by section and equation label.  OpenMP is used only
 * across links that the method treats as independent (all links of a smearing
 * step; the links of one masked subset of an annealing step), so the result is
 * the same for any thread count.
 *
 * Readings of points where the paper is silent (each also listed in the design
 * notes of the repository):
 *  - sector boundaries and Tr U = 0 in the Z(3) projection are "undefined";
 *  - the annealing subset of link (x, mu) is c = (2 x_mu + sum_{nu != mu} x_nu)
 *    mod 4, visited for mu = 0..3 and, inside each mu, c = 0, 2, 1, 3;
 *  - MaxReTr skips an SU(2) hit whose k = sqrt(det T) vanishes (k <= 1e-12 (|L|+1)),
 *    the case Sec. III.A shows to be undefined;
 *  - over-improved stout uses Omega = Sigma^OI U^dagger with the weights of
 *    Eq. (over-improvement); eps = 1 is plain stout.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef double complex cplx;
typedef struct {
  cplx a[3][3];
} mat3;

/* ------------------------------------------------------------------ lattice */

typedef struct {
  int L[4];
  int64_t V;
  int64_t *nb; /* nb[8*s + 2*mu + 0] = s - mu, nb[8*s + 2*mu + 1] = s + mu */
} lattice;

static int lat_init(lattice *g, const int32_t dims[4]) {
  if (!dims) return ORA_E_NULL;
  g->V = 1;
  for (int d = 0; d < 4; ++d) {
    if (dims[d] < 1) return ORA_E_DIMS;
    g->L[d] = dims[d];
    g->V *= dims[d];
  }
  g->nb = (int64_t *)malloc(sizeof(int64_t) * 8 * (size_t)g->V);
  if (!g->nb) return ORA_E_PARAM;
  for (int64_t s = 0; s < g->V; ++s) {
    int c[4];
    int64_t r = s;
    for (int d = 0; d < 4; ++d) {
      c[d] = (int)(r % g->L[d]);
      r /= g->L[d];
    }
    for (int mu = 0; mu < 4; ++mu) {
      for (int dir = 0; dir < 2; ++dir) {
        int e[4] = {c[0], c[1], c[2], c[3]};
        e[mu] = (e[mu] + (dir ? 1 : g->L[mu] - 1)) % g->L[mu];
        g->nb[8 * s + 2 * mu + dir] =
            e[0] + (int64_t)g->L[0] * (e[1] + (int64_t)g->L[1] * (e[2] + (int64_t)g->L[2] * e[3]));
      }
    }
  }
  return ORA_OK;
}

static void lat_free(lattice *g) { free(g->nb); }

static int64_t fwd(const lattice *g, int64_t s, int mu) { return g->nb[8 * s + 2 * mu + 1]; }
static int64_t bwd(const lattice *g, int64_t s, int mu) { return g->nb[8 * s + 2 * mu + 0]; }

static int coord(const lattice *g, int64_t s, int d) {
  for (int k = 0; k < d; ++k) s /= g->L[k];
  return (int)(s % g->L[d]);
}

/* ------------------------------------------------------------ 3x3 algebra */

static mat3 m_load(const double *p) {
  mat3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.a[i][j] = p[2 * (3 * i + j)] + I * p[2 * (3 * i + j) + 1];
  return r;
}

static void m_store(const mat3 *m, double *p) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      p[2 * (3 * i + j)] = creal(m->a[i][j]);
      p[2 * (3 * i + j) + 1] = cimag(m->a[i][j]);
    }
}

static mat3 m_link(const double *links, const lattice *g, int mu, int64_t s) {
  return m_load(links + 18 * ((size_t)mu * g->V + s));
}

static mat3 m_zero(void) {
  mat3 r;
  memset(&r, 0, sizeof r);
  return r;
}

static mat3 m_ident(void) {
  mat3 r = m_zero();
  for (int i = 0; i < 3; ++i) r.a[i][i] = 1.0;
  return r;
}

static mat3 m_mul(const mat3 *x, const mat3 *y) {
  mat3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx acc = 0;
      for (int k = 0; k < 3; ++k) acc += x->a[i][k] * y->a[k][j];
      r.a[i][j] = acc;
    }
  return r;
}

static mat3 m_dag(const mat3 *x) {
  mat3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.a[i][j] = conj(x->a[j][i]);
  return r;
}

static mat3 m_add(const mat3 *x, const mat3 *y) {
  mat3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.a[i][j] = x->a[i][j] + y->a[i][j];
  return r;
}

static mat3 m_sub(const mat3 *x, const mat3 *y) {
  mat3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.a[i][j] = x->a[i][j] - y->a[i][j];
  return r;
}

static mat3 m_scale(const mat3 *x, cplx c) {
  mat3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.a[i][j] = c * x->a[i][j];
  return r;
}

static cplx m_trace(const mat3 *x) { return x->a[0][0] + x->a[1][1] + x->a[2][2]; }

/* -------------------------------------------------- centre projection, Sec. I */

/* Eq. (centre_element): n = 0, +1, -1 for arg Tr U in (-pi/3, pi/3), (pi/3, pi),
 * (-pi, -pi/3).  The open intervals leave the boundaries and Tr U = 0 undefined.
 * The open end at +-pi is decided by the sign of Im Tr U (arg < pi exactly when
 * Im > 0), because atan2 rounds arguments within an ulp of pi to pi itself. */
int ora_sector(double re, double im) {
  if (!isfinite(re) || !isfinite(im) || (re == 0.0 && im == 0.0)) return ORA_UNDEF;
  double phi = atan2(im, re);
  const double third = M_PI / 3.0;
  if (phi > -third && phi < third) return 0;
  if (phi > third && im > 0.0) return 1;
  if (phi < -third && im < 0.0) return -1;
  return ORA_UNDEF;
}

static int sector_of(const mat3 *u) {
  cplx t = m_trace(u);
  return ora_sector(creal(t), cimag(t));
}

/* Z(3) element e^{i 2 pi n / 3} (Eq. centre_project). */
static cplx z3(int n) { return cexp(I * (2.0 * M_PI / 3.0) * (double)n); }

int ora_sectors(const int32_t dims[4], const double *links, int8_t *out) {
  if (!links || !out) return ORA_E_NULL;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  for (int mu = 0; mu < 4; ++mu)
    for (int64_t s = 0; s < g.V; ++s) {
      mat3 u = m_link(links, &g, mu, s);
      out[(size_t)mu * g.V + s] = (int8_t)sector_of(&u);
    }
  lat_free(&g);
  return ORA_OK;
}

/* ------------------------------------------------------------ field ingest */

int ora_z3_field(const int32_t dims[4], const int8_t *n, double *links) {
  if (!n || !links) return ORA_E_NULL;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  for (int mu = 0; mu < 4; ++mu)
    for (int64_t s = 0; s < g.V; ++s) {
      int k = n[(size_t)mu * g.V + s];
      if (k < -1 || k > 1) {
        lat_free(&g);
        return ORA_E_PARAM;
      }
      mat3 one = m_ident();
      mat3 u = m_scale(&one, z3(k));
      m_store(&u, links + 18 * ((size_t)mu * g.V + s));
    }
  lat_free(&g);
  return ORA_OK;
}

/* ----------------------------------------------- centrifuge, Sec. IV */

/* The staple phase sigma_mu(x) of Sec. IV built from the non-compact phases
 * lambda = 2 pi n / 3, with the integer m of Sec. IV.A defined by
 * sigma = m 2 pi / 18.  Each link gets (Eqs. lambda_j, lambda_k)
 *   lambda^j = (1 - omega) lambda + omega sigma,
 *   lambda^k = (1 + omega) lambda - omega sigma,
 * the third phase unchanged; the preservation condition Eq. (expcon),
 * -2pi/3 < omega (sigma - lambda) < 2pi/3, is checked for every link. */
int ora_centrifuge(const int32_t dims[4], const int8_t *n, const int8_t *pair, double omega,
                   double *links, int32_t *m_out) {
  if (!n || !pair || !links) return ORA_E_NULL;
  if (!isfinite(omega)) return ORA_E_PARAM;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  const int64_t V = g.V;
  const double unit = 2.0 * M_PI / 3.0;
  int bad = 0;
  for (int mu = 0; mu < 4; ++mu) {
    for (int64_t s = 0; s < V; ++s) {
      int64_t xm = fwd(&g, s, mu);
      double sig = 0.0;
      int m = 0;
      for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int64_t xn = fwd(&g, s, nu), xmn = bwd(&g, s, nu), xmnm = fwd(&g, xmn, mu);
        int t1 = n[(size_t)nu * V + s], t2 = n[(size_t)mu * V + xn], t3 = n[(size_t)nu * V + xm];
        int t4 = n[(size_t)nu * V + xmn], t5 = n[(size_t)mu * V + xmn], t6 = n[(size_t)nu * V + xmnm];
        sig += unit * t1 + unit * t2 - unit * t3 - unit * t4 + unit * t5 + unit * t6;
        m += t1 + t2 - t3 - t4 + t5 + t6;
      }
      sig /= 6.0;
      int nn = n[(size_t)mu * V + s];
      int pc = pair[(size_t)mu * V + s];
      if (nn < -1 || nn > 1 || pc < 0 || pc > 2) {
        bad = 1;
        continue;
      }
      double lam = unit * nn;
      double arg = omega * (sig - lam);
      if (!(arg > -unit && arg < unit)) bad = 1;
      int j = pc, k = (pc + 1) % 3;
      double ph[3] = {lam, lam, lam};
      ph[j] = (1.0 - omega) * lam + omega * sig;
      ph[k] = (1.0 + omega) * lam - omega * sig;
      mat3 u = m_zero();
      for (int i = 0; i < 3; ++i) u.a[i][i] = cexp(I * ph[i]);
      m_store(&u, links + 18 * ((size_t)mu * V + s));
      if (m_out) m_out[(size_t)mu * V + s] = m;
    }
  }
  lat_free(&g);
  return bad ? ORA_E_PARAM : ORA_OK;
}

/* ------------------------------------------------ gauge transform, Sec. V.C */

/* U^G_mu(x) = G(x) U_mu(x) G^dagger(x + mu). */
int ora_gauge_transform(const int32_t dims[4], const double *links, const double *gauge,
                        double *out) {
  if (!links || !gauge || !out) return ORA_E_NULL;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  for (int mu = 0; mu < 4; ++mu)
    for (int64_t s = 0; s < g.V; ++s) {
      mat3 G = m_load(gauge + 18 * (size_t)s);
      mat3 Gp = m_load(gauge + 18 * (size_t)fwd(&g, s, mu));
      mat3 Gpd = m_dag(&Gp);
      mat3 u = m_link(links, &g, mu, s);
      mat3 t = m_mul(&G, &u);
      mat3 r = m_mul(&t, &Gpd);
      m_store(&r, out + 18 * ((size_t)mu * g.V + s));
    }
  lat_free(&g);
  return ORA_OK;
}

/* ------------------------------------------------------------ staples */

/* Product of links along a path that starts at site s.  Step +(d+1) moves one
 * site forward along direction d and multiplies U_d(y); step -(d+1) moves one
 * site back along d and multiplies U_d(y - d)^dagger. */
static mat3 path_product(const lattice *g, const double *links, int64_t s, const int *steps,
                         int n) {
  mat3 acc = m_ident();
  int64_t y = s;
  for (int i = 0; i < n; ++i) {
    int d = abs(steps[i]) - 1;
    mat3 u;
    if (steps[i] > 0) {
      u = m_link(links, g, d, y);
      y = fwd(g, y, d);
    } else {
      y = bwd(g, y, d);
      mat3 w = m_link(links, g, d, y);
      u = m_dag(&w);
    }
    acc = m_mul(&acc, &u);
  }
  return acc;
}

/* Sigma_mu(x): the weighted sum of all paths from x to x + mu of Eq. (plaq_staples)
 * and Eq. (over-improvement).  The over-improvement diagrams are drawn for
 * Sigma^dagger (paths from x + mu back to x); the paths below are those diagrams
 * reversed.  For every nu != mu and both orientations of nu:
 *   plaquette staple    (5 - 2 eps)/3          : +nu, +mu, -nu
 *   1x2 rectangle       (eps - 1)/(12 u0^2)    : +nu, +nu, +mu, -nu, -nu
 *   2x1, x at the left  (eps - 1)/(12 u0^2)    : +nu, +mu, +mu, -nu, -mu
 *   2x1, x in the middle(eps - 1)/(12 u0^2)    : -mu, +nu, +mu, +mu, -nu
 * With eps = 1 the rectangle weight vanishes and the plaquette weight is 1: the
 * plain staple sum of Eq. (plaq_staples). */
static mat3 staple_sum(const lattice *g, const double *links, int mu, int64_t s, double eps,
                       double u0) {
  const double cp = (5.0 - 2.0 * eps) / 3.0;
  const double cr = (eps - 1.0) / (12.0 * u0 * u0);
  const int m = mu + 1;
  mat3 plaq = m_zero(), rect = m_zero();
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    for (int sg = -1; sg <= 1; sg += 2) {
      const int n = sg * (nu + 1);
      const int p_st[3] = {n, m, -n};
      mat3 t = path_product(g, links, s, p_st, 3);
      plaq = m_add(&plaq, &t);
      if (cr != 0.0) {
        const int r12[5] = {n, n, m, -n, -n};
        const int r21l[5] = {n, m, m, -n, -m};
        const int r21m[5] = {-m, n, m, m, -n};
        mat3 a = path_product(g, links, s, r12, 5);
        mat3 b = path_product(g, links, s, r21l, 5);
        mat3 c = path_product(g, links, s, r21m, 5);
        rect = m_add(&rect, &a);
        rect = m_add(&rect, &b);
        rect = m_add(&rect, &c);
      }
    }
  }
  mat3 sp = m_scale(&plaq, cp);
  mat3 sr = m_scale(&rect, cr);
  return m_add(&sp, &sr);
}

int ora_staple(const int32_t dims[4], const double *links, int32_t mu, int64_t site, double eps,
               double u0, double *sigma) {
  if (!links || !sigma) return ORA_E_NULL;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  if (mu < 0 || mu > 3 || site < 0 || site >= g.V || u0 == 0.0) {
    lat_free(&g);
    return ORA_E_PARAM;
  }
  mat3 S = staple_sum(&g, links, mu, site, eps, u0);
  m_store(&S, sigma);
  lat_free(&g);
  return ORA_OK;
}

/* ------------------------------------------------------- Q, Eq. (generator) */

/* Q = 1/2 [Omega - Omega^dagger] - 1/6 Tr[Omega - Omega^dagger] 1 */
static mat3 generator(const mat3 *om) {
  mat3 od = m_dag(om);
  mat3 d = m_sub(om, &od);
  mat3 q = m_scale(&d, 0.5);
  cplx tr = m_trace(&d) / 6.0;
  for (int i = 0; i < 3; ++i) q.a[i][i] -= tr;
  return q;
}

void ora_generator(const double *omega, double *q) {
  mat3 om = m_load(omega);
  mat3 r = generator(&om);
  m_store(&r, q);
}

/* ------------------------------------------------------------ exponential */

/* exp(X) by scaling and squaring of the Taylor series: X is divided by 2^s so
 * that its 1-norm is at most 1/2, the series is summed to order 20 (remainder
 * below 1e-26), and the result is squared s times.  This is a textbook route
 * chosen on purpose to differ from the Cayley-Hamilton form used on the GPU. */
static mat3 expm(const mat3 *x) {
  double nrm = 0.0;
  for (int j = 0; j < 3; ++j) {
    double c = 0.0;
    for (int i = 0; i < 3; ++i) c += cabs(x->a[i][j]);
    if (c > nrm) nrm = c;
  }
  int sq = 0;
  double scale = 1.0;
  while (nrm * scale > 0.5) {
    scale *= 0.5;
    ++sq;
  }
  mat3 y = m_scale(x, scale);
  mat3 e = m_ident(), term = m_ident();
  for (int k = 1; k <= 20; ++k) {
    mat3 t = m_mul(&term, &y);
    term = m_scale(&t, 1.0 / (double)k);
    e = m_add(&e, &term);
  }
  for (int i = 0; i < sq; ++i) e = m_mul(&e, &e);
  return e;
}

void ora_expm(const double *x, double *e) {
  mat3 xm = m_load(x);
  mat3 r = expm(&xm);
  m_store(&r, e);
}

/* ------------------------------------------------- MaxReTr, Sec. III */

/* Cabibbo-Marinari maximisation of Re Tr[U V^dagger] (Eq. maxReTr): for each of
 * the subgroups (1,2), (2,3), (1,3), in that order, L = U V^dagger (Eq. def_L1),
 * T is built from L's 2x2 block as in Eq. (def_T1), k = sqrt(det T), and
 * U <- T^c U with [T^c] = [T^dagger]/k embedded in SU(3).  The three subgroups
 * are looped over `loops` times.  A hit with k = 0 is undefined (Sec. III.A);
 * it is skipped when k <= 1e-12 (|L|_F + 1). */
static mat3 maxretr(const mat3 *u0, const mat3 *v, int loops) {
  static const int sub[3][2] = {{0, 1}, {1, 2}, {0, 2}};
  mat3 u = *u0;
  mat3 vd = m_dag(v);
  for (int it = 0; it < loops; ++it) {
    for (int h = 0; h < 3; ++h) {
      const int p = sub[h][0], q = sub[h][1];
      mat3 L = m_mul(&u, &vd);
      cplx t00 = 0.5 * (L.a[p][p] + conj(L.a[q][q]));
      cplx t01 = 0.5 * (L.a[p][q] - conj(L.a[q][p]));
      cplx t10 = 0.5 * (L.a[q][p] - conj(L.a[p][q]));
      cplx t11 = 0.5 * (conj(L.a[p][p]) + L.a[q][q]);
      double det = creal(t00 * t11 - t01 * t10);
      double lf = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) lf += creal(L.a[i][j] * conj(L.a[i][j]));
      lf = sqrt(lf);
      double k = sqrt(det > 0.0 ? det : 0.0);
      if (!(k > 1e-12 * (lf + 1.0))) continue;
      mat3 tc = m_ident();
      tc.a[p][p] = conj(t00) / k;
      tc.a[p][q] = conj(t10) / k;
      tc.a[q][p] = conj(t01) / k;
      tc.a[q][q] = conj(t11) / k;
      u = m_mul(&tc, &u);
    }
  }
  return u;
}

void ora_maxretr(const double *u, const double *v, int32_t loops, double *out) {
  mat3 um = m_load(u), vm = m_load(v);
  mat3 r = maxretr(&um, &vm, loops);
  m_store(&r, out);
}

/* Eigen-decomposition A = Q diag(lam) Q^dagger of a Hermitian 3x3 matrix by
 * cyclic Jacobi rotations, each zeroing one off-diagonal pair (the complex
 * Hermitian form of the classical method, Golub & Van Loan Sec. 8.5). */
static void herm_eig(const mat3 *A, double lam[3], mat3 *Q) {
  mat3 a = *A, q = m_ident();
  static const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double m = creal(a.a[i][j] * conj(a.a[i][j]));
        tot += m;
        if (i != j) off += m;
      }
    if (off <= 1e-30 * tot) break;
    for (int k = 0; k < 3; ++k) {
      const int p = pairs[k][0], r = pairs[k][1];
      const double mag = cabs(a.a[p][r]);
      if (mag == 0.0) continue;
      const cplx ph = a.a[p][r] / mag;
      const double tau = (creal(a.a[r][r]) - creal(a.a[p][p])) / (2.0 * mag);
      const double t = fabs(tau) > 1e150 ? 0.5 / tau
                                         : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
      mat3 J = m_ident();
      J.a[p][p] = c;
      J.a[p][r] = sn * ph;
      J.a[r][p] = -sn * conj(ph);
      J.a[r][r] = c;
      mat3 Jd = m_dag(&J), t1 = m_mul(&Jd, &a);
      a = m_mul(&t1, &J);
      q = m_mul(&q, &J);
    }
  }
  for (int i = 0; i < 3; ++i) lam[i] = creal(a.a[i][i]);
  *Q = q;
}

/* Unit circle projection (Sec. II.C, Eq. W): W = V (V^dagger V)^{-1/2}, then
 * W / cbrt(det W) with the principal cube root (arg det W in (-pi, pi], so the
 * root's phase lies in (-pi/3, pi/3]).  The inverse square root is taken from
 * the eigen-decomposition of V^dagger V. */
static mat3 unit_circle_projection(const mat3 *v) {
  mat3 vd = m_dag(v), A = m_mul(&vd, v), Q;
  double lam[3];
  herm_eig(&A, lam, &Q);
  mat3 D = m_zero();
  for (int i = 0; i < 3; ++i) D.a[i][i] = 1.0 / sqrt(lam[i]);
  mat3 Qd = m_dag(&Q), t = m_mul(&Q, &D), isq = m_mul(&t, &Qd);
  mat3 W = m_mul(v, &isq);
  const cplx det = W.a[0][0] * (W.a[1][1] * W.a[2][2] - W.a[1][2] * W.a[2][1]) -
                   W.a[0][1] * (W.a[1][0] * W.a[2][2] - W.a[1][2] * W.a[2][0]) +
                   W.a[0][2] * (W.a[1][0] * W.a[2][1] - W.a[1][1] * W.a[2][0]);
  const cplx root = cpow(cabs(det), 1.0 / 3.0) * cexp(I * carg(det) / 3.0);
  return m_scale(&W, 1.0 / root);
}

void ora_unit_circle_projection(const double *v, double *out) {
  mat3 vm = m_load(v);
  mat3 r = unit_circle_projection(&vm);
  m_store(&r, out);
}

/* ------------------------------------------------------- link update */

typedef struct {
  int update, vp;
  double rho, eps, u0, alpha;
  int loops;
} params;

/* Candidate for link (x, mu) from the current field, then the vortex-preserving
 * accept/reject of Sec. VI.  Stout (Eq. stout): U' = exp(rho Q) U with Q from
 * Omega = Sigma U^dagger.  MaxReTr (Sec. III, Eq. V): the blocked matrix
 * V = (1 - alpha) U + (alpha/6) Sigma, then U' = MaxReTr(U, V); alpha = 1 is
 * cooling.  APE (Sec. II.C): the same V returned to SU(3) by the unit circle
 * projection.  With vp on, U' is accepted only if it projects to the original
 * centre element n0, after undoing the gauge transform when one is given:
 * P_Z3{G^dagger(x) U' G(x + mu)} = Z.  Returns 1 if accepted. */
static int update_link(const lattice *g, const double *links, const int8_t *n0,
                       const double *gauge, const params *pr, int mu, int64_t s, mat3 *out) {
  mat3 u = m_link(links, g, mu, s);
  mat3 S = staple_sum(g, links, mu, s, pr->eps, pr->u0);
  mat3 cand;
  if (pr->update == ORA_STOUT) {
    mat3 ud = m_dag(&u);
    mat3 om = m_mul(&S, &ud);
    mat3 q = generator(&om);
    mat3 x = m_scale(&q, pr->rho);
    mat3 e = expm(&x);
    cand = m_mul(&e, &u);
  } else {
    mat3 a = m_scale(&u, 1.0 - pr->alpha);
    mat3 b = m_scale(&S, pr->alpha / 6.0);
    mat3 v = m_add(&a, &b);
    if (pr->update == ORA_APE)
      cand = unit_circle_projection(&v);
    else
      cand = maxretr(&u, &v, pr->loops);
  }
  if (pr->vp) {
    mat3 test = cand;
    if (gauge) {
      mat3 G = m_load(gauge + 18 * (size_t)s);
      mat3 Gp = m_load(gauge + 18 * (size_t)fwd(g, s, mu));
      mat3 Gd = m_dag(&G);
      mat3 t = m_mul(&Gd, &cand);
      test = m_mul(&t, &Gp);
    }
    if (sector_of(&test) != n0[(size_t)mu * g->V + s]) {
      *out = u;
      return 0;
    }
  }
  *out = cand;
  return 1;
}

static int check_params(const params *pr) {
  if (pr->update != ORA_STOUT && pr->update != ORA_MAXRETR && pr->update != ORA_APE) return 0;
  if (!isfinite(pr->rho) || !isfinite(pr->eps) || !isfinite(pr->u0) || pr->u0 == 0.0) return 0;
  if (!isfinite(pr->alpha) || pr->loops < 0) return 0;
  return 1;
}

int ora_update_link(const int32_t dims[4], const double *links, const int8_t *n0,
                    const double *gauge, int32_t update, int32_t vp, double rho, double eps,
                    double u0, double alpha, int32_t su2_loops, int32_t mu, int64_t site,
                    double *out, int32_t *accepted) {
  if (!links || !out || (vp && !n0)) return ORA_E_NULL;
  params pr = {update, vp, rho, eps, u0, alpha, su2_loops};
  if (!check_params(&pr)) return ORA_E_PARAM;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  if (mu < 0 || mu > 3 || site < 0 || site >= g.V) {
    lat_free(&g);
    return ORA_E_PARAM;
  }
  mat3 r;
  int acc = update_link(&g, links, n0, gauge, &pr, mu, site, &r);
  m_store(&r, out);
  if (accepted) *accepted = acc;
  lat_free(&g);
  return ORA_OK;
}

int ora_update_links(const int32_t dims[4], const double *links, const int8_t *n0,
                     const double *gauge, int32_t update, int32_t vp, double rho, double eps,
                     double u0, double alpha, int32_t su2_loops, int64_t count, const int32_t *mus,
                     const int64_t *sites, double *out, int32_t *accepted) {
  if (!links || !out || !mus || !sites || (vp && !n0)) return ORA_E_NULL;
  params pr = {update, vp, rho, eps, u0, alpha, su2_loops};
  if (!check_params(&pr) || count < 0) return ORA_E_PARAM;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  for (int64_t i = 0; i < count; ++i)
    if (mus[i] < 0 || mus[i] > 3 || sites[i] < 0 || sites[i] >= g.V) {
      lat_free(&g);
      return ORA_E_PARAM;
    }
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < count; ++i) {
    mat3 r;
    const int acc = update_link(&g, links, n0, gauge, &pr, mus[i], sites[i], &r);
    m_store(&r, out + 18 * i);
    if (accepted) accepted[i] = acc;
  }
  lat_free(&g);
  return ORA_OK;
}

/* ---------------------------------------------------------- schedules */

/* Masked subset of the annealing schedule (Sec. III.A: annealing updates links
 * one at a time, and can be run in parallel with a suitable mask). */
static int colour_of(const lattice *g, int mu, int64_t s) {
  int c = 0;
  for (int d = 0; d < 4; ++d) c += (d == mu ? 2 : 1) * coord(g, s, d);
  return c % 4;
}

int ora_colour(const int32_t dims[4], int32_t mu, int64_t site) {
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  int c = colour_of(&g, mu, site);
  lat_free(&g);
  return c;
}

/* One masked annealing step: every link (x, mu) of subset `colour` is replaced,
 * in place, by its update computed from the current field.  No link of the
 * subset enters another's staple, so the in-place order does not matter. */
static int64_t anneal_subset(const lattice *g, double *links, const int8_t *n0,
                             const double *gauge, const params *pr, int mu, int colour) {
  int64_t rej = 0;
#pragma omp parallel for schedule(static) reduction(+ : rej)
  for (int64_t s = 0; s < g->V; ++s) {
    if (colour_of(g, mu, s) != colour) continue;
    mat3 r;
    if (!update_link(g, links, n0, gauge, pr, mu, s, &r)) ++rej;
    m_store(&r, links + 18 * ((size_t)mu * g->V + s));
  }
  return rej;
}

int ora_pass(const int32_t dims[4], double *links, const int8_t *n0, const double *gauge,
             int32_t update, int32_t vp, double rho, double eps, double u0, double alpha,
             int32_t su2_loops, int32_t mu, int32_t colour, int64_t *rejected) {
  if (!links || (vp && !n0)) return ORA_E_NULL;
  params pr = {update, vp, rho, eps, u0, alpha, su2_loops};
  if (!check_params(&pr) || mu < 0 || mu > 3 || colour < 0 || colour > 3) return ORA_E_PARAM;
  for (int d = 0; d < 4; ++d)
    if (!dims || dims[d] % 4) return ORA_E_DIMS;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  int64_t rej = anneal_subset(&g, links, n0, gauge, &pr, mu, colour);
  if (rejected) *rejected = rej;
  lat_free(&g);
  return ORA_OK;
}

static int measure(const lattice *g, const double *links, const int8_t *n0, const double *gauge,
                   ora_stats *out, int8_t *flux);

/* n_sweeps sweeps.  JACOBI (smearing, Sec. III.A): every link is updated from
 * the field of the previous sweep.  ANNEALED: for mu = 0..3, subsets 0, 2, 1, 3
 * (each lattice extent must be a multiple of 4 for the subsets to be
 * independent).  After every `measure_every`-th sweep a record is written. */
int ora_smooth(const int32_t dims[4], double *links, const int8_t *n0, const double *gauge,
               int32_t n_sweeps, int32_t order, int32_t update, int32_t vp, double rho,
               double eps, double u0, double alpha, int32_t su2_loops, int32_t measure_every,
               ora_stats *stats) {
  if (!links || ((vp || (measure_every > 0)) && !n0)) return ORA_E_NULL;
  if (measure_every > 0 && !stats) return ORA_E_NULL;
  params pr = {update, vp, rho, eps, u0, alpha, su2_loops};
  if (!check_params(&pr) || n_sweeps < 0 || (order != ORA_JACOBI && order != ORA_ANNEALED))
    return ORA_E_PARAM;
  if (!dims) return ORA_E_NULL;
  for (int d = 0; d < 4; ++d) {
    if (dims[d] < 1) return ORA_E_DIMS;
    if (order == ORA_ANNEALED && dims[d] % 4) return ORA_E_DIMS;
  }
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  const int64_t V = g.V;
  double *old = NULL;
  if (order == ORA_JACOBI) {
    old = (double *)malloc(sizeof(double) * 18 * 4 * (size_t)V);
    if (!old) {
      lat_free(&g);
      return ORA_E_PARAM;
    }
  }
  static const int colours[4] = {0, 2, 1, 3};
  int64_t rej_since = 0;
  int rec = 0;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    if (order == ORA_JACOBI) {
      memcpy(old, links, sizeof(double) * 18 * 4 * (size_t)V);
      int64_t rej = 0;
#pragma omp parallel for schedule(static) reduction(+ : rej) collapse(2)
      for (int mu = 0; mu < 4; ++mu)
        for (int64_t s = 0; s < V; ++s) {
          mat3 r;
          if (!update_link(&g, old, n0, gauge, &pr, mu, s, &r)) ++rej;
          m_store(&r, links + 18 * ((size_t)mu * V + s));
        }
      rej_since += rej;
    } else {
      for (int mu = 0; mu < 4; ++mu)
        for (int c = 0; c < 4; ++c)
          rej_since += anneal_subset(&g, links, n0, gauge, &pr, mu, colours[c]);
    }
    if (measure_every > 0 && (sw + 1) % measure_every == 0) {
      measure(&g, links, n0, gauge, &stats[rec], NULL);
      stats[rec].rejected = rej_since;
      rej_since = 0;
      ++rec;
    }
  }
  free(old);
  lat_free(&g);
  return ORA_OK;
}

/* ------------------------------------------------------- Wilson flow */

/* Z(W)_mu(x) = eps Q_mu(x)[W]: the flow generator of Sec. II.B (the stout
 * generator of Eq. generator, with plain or over-improved staples), times the
 * step, for every link of W. */
static void flow_generators(const lattice *g, const double *w, double eps, double eps_oi, double u0,
                            mat3 *z) {
  const int64_t V = g->V;
#pragma omp parallel for schedule(static) collapse(2)
  for (int mu = 0; mu < 4; ++mu)
    for (int64_t s = 0; s < V; ++s) {
      mat3 u = m_link(w, g, mu, s);
      mat3 S = staple_sum(g, w, mu, s, eps_oi, u0);
      mat3 ud = m_dag(&u), om = m_mul(&S, &ud), q = generator(&om);
      z[(size_t)mu * V + s] = m_scale(&q, eps);
    }
}

/* W <- exp(X) W for every link, X = a Z + b Y (Y may be NULL). */
static void flow_apply(const lattice *g, double *w, const mat3 *z, double a, const mat3 *y, double b) {
  const int64_t V = g->V;
#pragma omp parallel for schedule(static) collapse(2)
  for (int mu = 0; mu < 4; ++mu)
    for (int64_t s = 0; s < V; ++s) {
      const size_t k = (size_t)mu * V + s;
      mat3 x = m_scale(&z[k], a);
      if (y) {
        mat3 t = m_scale(&y[k], b);
        x = m_add(&x, &t);
      }
      mat3 e = expm(&x), u = m_link(w, g, mu, s), r = m_mul(&e, &u);
      m_store(&r, w + 18 * k);
    }
}

/* n_steps steps of the Wilson flow dU/dtau = Q[U] U (Sec. II.B) of size eps,
 * every link at once.  integrator 0: Euler, U <- exp(eps Q[U]) U (the
 * simultaneous form of the stout step, Sec. V.B).  integrator 1: the
 * third-order Runge-Kutta scheme the paper mentions (Sec. V.B; Luscher 2010):
 *   W1 = exp(Z0/4) W0,  W2 = exp(8/9 Z1 - 17/36 Z0) W1,
 *   U(tau + eps) = exp(3/4 Z2 - 8/9 Z1 + 17/36 Z0) W2,  Z_i = eps Q[W_i]. */
int ora_flow(const int32_t dims[4], double *links, int32_t n_steps, double eps, double eps_oi, double u0,
             int32_t integrator) {
  if (!links) return ORA_E_NULL;
  if (n_steps < 0 || !isfinite(eps) || !isfinite(eps_oi) || !isfinite(u0) || u0 == 0.0 ||
      (integrator != 0 && integrator != 1))
    return ORA_E_PARAM;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  const size_t n = 4 * (size_t)g.V;
  mat3 *z0 = (mat3 *)malloc(sizeof(mat3) * n);
  mat3 *z1 = integrator ? (mat3 *)malloc(sizeof(mat3) * n) : NULL;
  mat3 *z2 = integrator ? (mat3 *)malloc(sizeof(mat3) * n) : NULL;
  if (!z0 || (integrator && (!z1 || !z2))) {
    free(z0);
    free(z1);
    free(z2);
    lat_free(&g);
    return ORA_E_PARAM;
  }
  for (int st = 0; st < n_steps; ++st) {
    flow_generators(&g, links, eps, eps_oi, u0, z0);
    if (!integrator) {
      flow_apply(&g, links, z0, 1.0, NULL, 0.0);
      continue;
    }
    flow_apply(&g, links, z0, 0.25, NULL, 0.0);
    flow_generators(&g, links, eps, eps_oi, u0, z1);
    flow_apply(&g, links, z1, 8.0 / 9.0, z0, -17.0 / 36.0);
    flow_generators(&g, links, eps, eps_oi, u0, z2);
    /* 3/4 Z2 - 8/9 Z1 + 17/36 Z0 */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
      mat3 a = m_scale(&z1[k], -8.0 / 9.0), b = m_scale(&z0[k], 17.0 / 36.0);
      z1[k] = m_add(&a, &b);
    }
    flow_apply(&g, links, z2, 0.75, z1, 1.0);
  }
  free(z0);
  free(z1);
  free(z2);
  lat_free(&g);
  return ORA_OK;
}

/* ------------------------------------------------------- measurement */

/* Neumaier's compensated summation, in long double. */
typedef struct {
  long double sum, comp;
} ksum;

static void ks_add(ksum *k, long double v) {
  long double t = k->sum + v;
  if (fabsl(k->sum) >= fabsl(v))
    k->comp += (k->sum - t) + v;
  else
    k->comp += (v - t) + k->sum;
  k->sum = t;
}

/* Plaquette P_{mu nu}(x) = U_mu(x) U_nu(x+mu) U_mu^dag(x+nu) U_nu^dag(x) (Sec. I);
 * the Wilson action density S(x) = beta/(2 n_c n_d (n_d-1)) sum_{mu != nu}
 * Re Tr[1 - P_{mu nu}(x)] (Sec. V), reported as <S>/beta with n_c = 3, n_d = 4
 * and the ordered sum written as twice the sum over mu < nu; the vortex flux
 * p_{mu nu}(x) of the projected plaquette (Sec. I) from the centre projections
 * of the current links, compared with the flux of the original charges n0.
 * The charges n0 belong to the field in maximal centre gauge; when the field
 * lives in a random gauge G (Sec. V.C), a link's centre projection is taken
 * after undoing it, from G^dagger(x) U G(x + mu), as the vortex-preserving test
 * of Sec. VI does. */
static int measure(const lattice *g, const double *links, const int8_t *n0, const double *gauge,
                   ora_stats *out, int8_t *flux) {
  const int64_t V = g->V;
  long double *site_p = (long double *)malloc(sizeof(long double) * (size_t)V);
  long double *site_s = (long double *)malloc(sizeof(long double) * (size_t)V);
  int8_t *sec = (int8_t *)malloc((size_t)(4 * V));
  if (!site_p || !site_s || !sec) {
    free(site_p);
    free(site_s);
    free(sec);
    return ORA_E_PARAM;
  }
  double maxu = 0.0;
  int64_t undef = 0, nonfin = 0;
#pragma omp parallel for schedule(static) reduction(max : maxu) reduction(+ : undef, nonfin) collapse(2)
  for (int mu = 0; mu < 4; ++mu)
    for (int64_t s = 0; s < V; ++s) {
      mat3 u = m_link(links, g, mu, s);
      int fin = 1;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          if (!isfinite(creal(u.a[i][j])) || !isfinite(cimag(u.a[i][j]))) fin = 0;
      if (!fin) ++nonfin;
      mat3 ud = m_dag(&u);
      mat3 uu = m_mul(&ud, &u);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double dv = cabs(uu.a[i][j] - (i == j ? 1.0 : 0.0));
          if (dv > maxu) maxu = dv;
        }
      mat3 mcg = u;
      if (gauge) {
        mat3 G = m_load(gauge + 18 * (size_t)s);
        mat3 Gp = m_load(gauge + 18 * (size_t)fwd(g, s, mu));
        mat3 Gd = m_dag(&G);
        mat3 t = m_mul(&Gd, &u);
        mcg = m_mul(&t, &Gp);
      }
      int sc = sector_of(&mcg);
      if (sc == ORA_UNDEF) ++undef;
      sec[(size_t)mu * V + s] = (int8_t)sc;
    }
  int64_t mism = 0;
#pragma omp parallel for schedule(static) reduction(+ : mism)
  for (int64_t s = 0; s < V; ++s) {
    long double sp = 0.0L, ss = 0.0L;
    int plane = 0;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
        int64_t xm = fwd(g, s, mu), xn = fwd(g, s, nu);
        mat3 a = m_link(links, g, mu, s);
        mat3 b = m_link(links, g, nu, xm);
        mat3 c = m_link(links, g, mu, xn);
        mat3 d = m_link(links, g, nu, s);
        mat3 cd = m_dag(&c), dd = m_dag(&d);
        mat3 t1 = m_mul(&a, &b);
        mat3 t2 = m_mul(&t1, &cd);
        mat3 P = m_mul(&t2, &dd);
        mat3 one = m_ident();
        mat3 one_minus_p = m_sub(&one, &P);
        sp += (long double)creal(m_trace(&P));
        ss += (long double)creal(m_trace(&one_minus_p));
        int q1 = sec[(size_t)mu * V + s], q2 = sec[(size_t)nu * V + xm];
        int q3 = sec[(size_t)mu * V + xn], q4 = sec[(size_t)nu * V + s];
        int o = n0[(size_t)mu * V + s] + n0[(size_t)nu * V + xm] - n0[(size_t)mu * V + xn] -
                n0[(size_t)nu * V + s];
        o = ((o % 3) + 3) % 3;
        int pv;
        if (q1 == ORA_UNDEF || q2 == ORA_UNDEF || q3 == ORA_UNDEF || q4 == ORA_UNDEF) {
          pv = ORA_UNDEF;
          ++mism;
        } else {
          int r = (((q1 + q2 - q3 - q4) % 3) + 3) % 3;
          if (r != o) ++mism;
          pv = r == 2 ? -1 : r;
        }
        if (flux) flux[(size_t)plane * V + s] = (int8_t)pv;
      }
    site_p[s] = sp;
    site_s[s] = ss;
  }
  ksum kp = {0, 0}, kss = {0, 0};
  for (int64_t s = 0; s < V; ++s) {
    ks_add(&kp, site_p[s]);
    ks_add(&kss, site_s[s]);
  }
  out->plaq = (double)((kp.sum + kp.comp) / (18.0L * (long double)V));
  out->action = (double)((kss.sum + kss.comp) / (36.0L * (long double)V));
  out->max_unitarity = maxu;
  out->reserved = 0.0;
  out->flux_mismatch = mism;
  out->undefined_sector = undef;
  out->rejected = 0;
  out->nonfinite = nonfin;
  free(site_p);
  free(site_s);
  free(sec);
  return ORA_OK;
}

/* The 1x1 clover term C_{mu nu}(x): the mean of the four plaquettes of the
 * (mu, nu) plane that start and end at x, each taken in the mu -> nu sense. */
static mat3 clover(const lattice *g, const double *links, int64_t x, int mu, int nu) {
  const int64_t xpm = fwd(g, x, mu), xpn = fwd(g, x, nu);
  const int64_t xmm = bwd(g, x, mu), xmn = bwd(g, x, nu);
  const int64_t xmm_pn = fwd(g, xmm, nu), xmm_mn = bwd(g, xmm, nu), xpm_mn = fwd(g, xmn, mu);
  mat3 leaf[4];
  {
    /* U_mu(x) U_nu(x+mu) U_mu^dag(x+nu) U_nu^dag(x) */
    mat3 a = m_link(links, g, mu, x), b = m_link(links, g, nu, xpm);
    mat3 c = m_link(links, g, mu, xpn), d = m_link(links, g, nu, x);
    mat3 cd = m_dag(&c), dd = m_dag(&d), t = m_mul(&a, &b), t2 = m_mul(&t, &cd);
    leaf[0] = m_mul(&t2, &dd);
  }
  {
    /* U_nu(x) U_mu^dag(x-mu+nu) U_nu^dag(x-mu) U_mu(x-mu) */
    mat3 a = m_link(links, g, nu, x), b = m_link(links, g, mu, xmm_pn);
    mat3 c = m_link(links, g, nu, xmm), d = m_link(links, g, mu, xmm);
    mat3 bd = m_dag(&b), cd = m_dag(&c), t = m_mul(&a, &bd), t2 = m_mul(&t, &cd);
    leaf[1] = m_mul(&t2, &d);
  }
  {
    /* U_mu^dag(x-mu) U_nu^dag(x-mu-nu) U_mu(x-mu-nu) U_nu(x-nu) */
    mat3 a = m_link(links, g, mu, xmm), b = m_link(links, g, nu, xmm_mn);
    mat3 c = m_link(links, g, mu, xmm_mn), d = m_link(links, g, nu, xmn);
    mat3 ad = m_dag(&a), bd = m_dag(&b), t = m_mul(&ad, &bd), t2 = m_mul(&t, &c);
    leaf[2] = m_mul(&t2, &d);
  }
  {
    /* U_nu^dag(x-nu) U_mu(x-nu) U_nu(x+mu-nu) U_mu^dag(x) */
    mat3 a = m_link(links, g, nu, xmn), b = m_link(links, g, mu, xmn);
    mat3 c = m_link(links, g, nu, xpm_mn), d = m_link(links, g, mu, x);
    mat3 ad = m_dag(&a), dd = m_dag(&d), t = m_mul(&ad, &b), t2 = m_mul(&t, &c);
    leaf[3] = m_mul(&t2, &dd);
  }
  mat3 s01 = m_add(&leaf[0], &leaf[1]), s23 = m_add(&leaf[2], &leaf[3]), sum = m_add(&s01, &s23);
  return m_scale(&sum, 0.25);
}

/* Sec. V, Eqs. (1LFST), (1LTopQ) and the reconstructed action of Sec. V.A, with
 * g = 1:  F_{mu nu} = (C - C^dag)/(2i) (no trace removed, as written),
 * q(x) = 1/(32 pi^2) eps_{mu nu rho sigma} Tr[F_{mu nu} F_{rho sigma}] summed
 * over all 24 orderings, and S_R(x)/beta = 1/(2 n_c n_d (n_d - 1)) times the sum
 * of Tr[F F] over the six planes (mu < nu: the reading under which S_R tends to
 * S for smooth fields).  out = {<S_R>/beta, Q = sum_x q(x), <S>/beta}; sdens and
 * qdens (may be NULL) receive S(x)/beta and q(x). */
int ora_clover(const int32_t dims[4], const double *links, double *out, double *sdens, double *qdens) {
  if (!links || !out) return ORA_E_NULL;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  const int64_t V = g.V;
  long double *sr = (long double *)malloc(sizeof(long double) * (size_t)V);
  long double *qq = (long double *)malloc(sizeof(long double) * (size_t)V);
  long double *ss = (long double *)malloc(sizeof(long double) * (size_t)V);
  if (!sr || !qq || !ss) {
    free(sr);
    free(qq);
    free(ss);
    lat_free(&g);
    return ORA_E_PARAM;
  }
  static const int perm4[24][4] = {
      {0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 1, 3}, {0, 2, 3, 1}, {0, 3, 1, 2}, {0, 3, 2, 1},
      {1, 0, 2, 3}, {1, 0, 3, 2}, {1, 2, 0, 3}, {1, 2, 3, 0}, {1, 3, 0, 2}, {1, 3, 2, 0},
      {2, 0, 1, 3}, {2, 0, 3, 1}, {2, 1, 0, 3}, {2, 1, 3, 0}, {2, 3, 0, 1}, {2, 3, 1, 0},
      {3, 0, 1, 2}, {3, 0, 2, 1}, {3, 1, 0, 2}, {3, 1, 2, 0}, {3, 2, 0, 1}, {3, 2, 1, 0}};
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < V; ++x) {
    mat3 F[4][4];
    for (int mu = 0; mu < 4; ++mu) F[mu][mu] = m_zero();
    long double s_r = 0.0L, s_w = 0.0L;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        mat3 C = clover(&g, links, x, mu, nu);
        mat3 Cd = m_dag(&C);
        mat3 diff = m_sub(&C, &Cd);
        F[mu][nu] = m_scale(&diff, 1.0 / (2.0 * I));
        mat3 neg = m_scale(&F[mu][nu], -1.0);
        F[nu][mu] = neg;
        mat3 ff = m_mul(&F[mu][nu], &F[mu][nu]);
        s_r += (long double)creal(m_trace(&ff));
        /* the plaquette at x, for S(x): both orders of the plane */
        mat3 a = m_link(links, &g, mu, x), b = m_link(links, &g, nu, fwd(&g, x, mu));
        mat3 c = m_link(links, &g, mu, fwd(&g, x, nu)), d = m_link(links, &g, nu, x);
        mat3 cd = m_dag(&c), dd = m_dag(&d), t = m_mul(&a, &b), t2 = m_mul(&t, &cd);
        mat3 P = m_mul(&t2, &dd);
        s_w += 2.0L * (3.0L - (long double)creal(m_trace(&P)));
      }
    long double q = 0.0L;
    for (int k = 0; k < 24; ++k) {
      const int *pm = perm4[k];
      /* sign of the permutation: count inversions */
      int inv = 0;
      for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
          if (pm[i] > pm[j]) ++inv;
      mat3 prod = m_mul(&F[pm[0]][pm[1]], &F[pm[2]][pm[3]]);
      q += (inv % 2 ? -1.0L : 1.0L) * (long double)creal(m_trace(&prod));
    }
    const long double norm = 1.0L / (2.0L * 3.0L * 4.0L * 3.0L);
    sr[x] = s_r * norm;
    ss[x] = s_w * norm;
    qq[x] = q / (32.0L * (long double)M_PI * (long double)M_PI);
  }
  ksum ksr = {0, 0}, kq = {0, 0}, ks = {0, 0};
  for (int64_t x = 0; x < V; ++x) {
    ks_add(&ksr, sr[x]);
    ks_add(&kq, qq[x]);
    ks_add(&ks, ss[x]);
    if (sdens) sdens[x] = (double)ss[x];
    if (qdens) qdens[x] = (double)qq[x];
  }
  out[0] = (double)((ksr.sum + ksr.comp) / (long double)V);
  out[1] = (double)(kq.sum + kq.comp);
  out[2] = (double)((ks.sum + ks.comp) / (long double)V);
  free(sr);
  free(qq);
  free(ss);
  lat_free(&g);
  return ORA_OK;
}

/* Sec. VII, Eq. (correlation_s): <a b> / sqrt(<a^2> <b^2>) over n values. */
double ora_correlation(int64_t n, const double *a, const double *b) {
  ksum ab = {0, 0}, aa = {0, 0}, bb = {0, 0};
  for (int64_t i = 0; i < n; ++i) {
    ks_add(&ab, (long double)a[i] * b[i]);
    ks_add(&aa, (long double)a[i] * a[i]);
    ks_add(&bb, (long double)b[i] * b[i]);
  }
  const long double sab = ab.sum + ab.comp, saa = aa.sum + aa.comp, sbb = bb.sum + bb.comp;
  return (double)(sab / sqrtl(saa * sbb));
}

int ora_measure(const int32_t dims[4], const double *links, const int8_t *n0, const double *gauge,
                ora_stats *out, int8_t *flux) {
  if (!links || !n0 || !out) return ORA_E_NULL;
  lattice g;
  int rc = lat_init(&g, dims);
  if (rc) return rc;
  rc = measure(&g, links, n0, gauge, out, flux);
  lat_free(&g);
  return rc;
}

int ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
