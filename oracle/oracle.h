/*
 * oracle.h -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, FP64 CPU implementation of the smoothing path of
 * "Smoothing algorithms for projected center-vortex gauge fields"
 * (A. Virgili, W. Kamleh, D. Leinweber, arXiv:2203.09764).  Tests, the smoke
 * check and the CPU-baseline leg of the benchmark are the only users.  It
 * shares no code, header, table or constant with the HIP library.
 *
 * Interchange layout (all arrays host memory, caller-owned):
 *   site s = x + Lx*(y + Ly*(z + Lz*t)), direction mu = 0..3 = (x, y, z, t);
 *   links   : complex128 [4][V][3][3], row-major 3x3 (re, im interleaved doubles);
 *   charges : int8 [4][V] in {-1, 0, 1};
 *   pairs   : int8 [4][V] in {0, 1, 2} = centrifuge pair (1,2), (2,3), (3,1);
 *   gauge   : complex128 [V][3][3] or NULL;
 *   flux    : int8 [6][V], planes (01, 02, 03, 12, 13, 23), values in {-1,0,1},
 *             ORA_UNDEF where a link sector is undefined.
 *
 * Parity status: every function below is pinned by the CPU test-suite against
 * closed forms, invariants or brute force, except the long trajectories of the
 * annealed over-improved stout sweep, for which the paper prints no values
 * ("parity unpinned" beyond agreement with the HIP path and the invariants).
 */
#ifndef VSM_ORACLE_H
#define VSM_ORACLE_H

#include <stdint.h>

#define ORA_OK 0
#define ORA_E_DIMS (-1)
#define ORA_E_PARAM (-2)
#define ORA_E_NULL (-3)
#define ORA_UNDEF (-128)

#define ORA_JACOBI 0
#define ORA_ANNEALED 1
#define ORA_STOUT 0
#define ORA_MAXRETR 1
#define ORA_APE 2

typedef struct {
  double plaq;          /* <P> = (1/18V) sum_x sum_{mu<nu} Re Tr P_{mu nu}(x)      */
  double action;        /* <S>/beta = (1/36V) sum_x sum_{mu<nu} Re Tr[1 - P]        */
  double max_unitarity; /* max over links and entries of |U^dag U - 1|              */
  double reserved;
  int64_t flux_mismatch;    /* plaquettes whose flux differs from the original   */
  int64_t undefined_sector; /* links whose trace lies on a sector boundary / 0    */
  int64_t rejected;         /* vortex-preservation rejections since last record   */
  int64_t nonfinite;        /* links with a non-finite entry                      */
} ora_stats;

int ora_set_threads(int n);
int ora_sector(double re, double im);
int ora_colour(const int32_t dims[4], int32_t mu, int64_t site);

int ora_z3_field(const int32_t dims[4], const int8_t *n, double *links);
int ora_centrifuge(const int32_t dims[4], const int8_t *n, const int8_t *pair, double omega,
                   double *links, int32_t *m_out);
int ora_gauge_transform(const int32_t dims[4], const double *links, const double *gauge,
                        double *out);

int ora_staple(const int32_t dims[4], const double *links, int32_t mu, int64_t site,
               double eps, double u0, double *sigma);
void ora_generator(const double *omega, double *q);
void ora_expm(const double *x, double *e);
void ora_maxretr(const double *u, const double *v, int32_t loops, double *out);
void ora_unit_circle_projection(const double *v, double *out);

int ora_update_link(const int32_t dims[4], const double *links, const int8_t *n0,
                    const double *gauge, int32_t update, int32_t vp, double rho, double eps,
                    double u0, double alpha, int32_t su2_loops, int32_t mu, int64_t site,
                    double *out, int32_t *accepted);

/* The same update for `count` links at once, (mus[i], sites[i]) -> out + 18 i
 * (one call sets the lattice up once; for sampled checks of large lattices). */
int ora_update_links(const int32_t dims[4], const double *links, const int8_t *n0,
                     const double *gauge, int32_t update, int32_t vp, double rho, double eps,
                     double u0, double alpha, int32_t su2_loops, int64_t count, const int32_t *mus,
                     const int64_t *sites, double *out, int32_t *accepted);
int ora_pass(const int32_t dims[4], double *links, const int8_t *n0, const double *gauge,
             int32_t update, int32_t vp, double rho, double eps, double u0, double alpha,
             int32_t su2_loops, int32_t mu, int32_t colour, int64_t *rejected);
int ora_smooth(const int32_t dims[4], double *links, const int8_t *n0, const double *gauge,
               int32_t n_sweeps, int32_t order, int32_t update, int32_t vp, double rho,
               double eps, double u0, double alpha, int32_t su2_loops, int32_t measure_every,
               ora_stats *stats);
int ora_measure(const int32_t dims[4], const double *links, const int8_t *n0, const double *gauge,
                ora_stats *out, int8_t *flux);
int ora_sectors(const int32_t dims[4], const double *links, int8_t *out);

/* n_steps Wilson-flow steps of size eps on every link at once; integrator 0 =
 * Euler, 1 = third-order Runge-Kutta.  eps_oi: staple over-improvement. */
int ora_flow(const int32_t dims[4], double *links, int32_t n_steps, double eps, double eps_oi, double u0,
             int32_t integrator);

/* Reconstructed action and topological charge from the 1x1 clover field
 * strength: out = {<S_R>/beta, Q, <S>/beta}; sdens, qdens (nullable) receive
 * S(x)/beta and q(x), canonical site order. */
int ora_clover(const int32_t dims[4], const double *links, double *out, double *sdens, double *qdens);
/* <a b> / sqrt(<a^2> <b^2>). */
double ora_correlation(int64_t n, const double *a, const double *b);

#endif
