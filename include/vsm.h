/*
 * vsm.h -- C ABI of the MI355X (gfx950) library for smoothing Z(3)
 * centre-vortex gauge fields, after "Smoothing algorithms for projected
 * center-vortex gauge fields" (A. Virgili, W. Kamleh, D. Leinweber,
 * arXiv:2203.09764).
 *
 * The calls follow the paper's statement of the problem: take a Z(3) field
 * (Sec. I), precondition it (Sec. IV), smooth it with stout / over-improved stout
 * or MaxReTr (cooling) updates, annealed or smeared, with or without vortex
 * preservation (Sec. II, III, V, VI), and measure it (Sec. I, V.A).
 *
 * Conventions for every call
 *   dims[4]   lattice extents (Lx, Ly, Lz, Lt), host array.  Every extent must be
 *             >= 4 and a multiple of 4 (the annealing subsets need it).
 *             6 * (V + 64) * sizeof(entry) must stay below 2^31 bytes
 *             (V < 22.3M sites in FP64, < 44.7M in FP32).
 *   site      s = x + Lx*(y + Ly*(z + Lz*t)); direction mu = 0..3 = (x, y, z, t).
 *   precision VSM_FP64 (all arithmetic and storage FP64) or VSM_FP32_BULK
 *             (links stored and staples / products computed in FP32; the
 *             Cayley-Hamilton coefficients, reunitarisation, MaxReTr and all
 *             measurement sums in FP64).
 *   pointers  "device" means memory of the current HIP device (for example a
 *             torch CUDA tensor's data_ptr()); the library never allocates,
 *             frees or keeps caller buffers.
 *   links     device buffer of vsm_links_bytes(dims, precision) bytes in the
 *             library's internal layout; only the calls below read or write it.
 *             Links must be SU(3): the library stores rows 0 and 1 and
 *             rebuilds row 2 as conj(row0 x row1).
 *   stream    hipStream_t passed as void* (NULL = default stream).  Every call
 *             is asynchronous on that stream; none synchronises the host.
 *   status    0 (VSM_OK) on success, a negative VSM_E_* code otherwise.  On an
 *             error nothing has been enqueued.  Numerical anomalies (NaN links,
 *             traces on a sector boundary) are not errors: they are counted in
 *             vsm_stats.
 */
#ifndef VSM_H
#define VSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VSM_OK 0
#define VSM_E_DIMS (-1)      /* extents not allowed for the layout or schedule       */
#define VSM_E_PARAM (-2)     /* a parameter outside its domain                       */
#define VSM_E_NULL (-3)      /* a required pointer is NULL                           */
#define VSM_E_WORKSPACE (-4) /* workspace smaller than vsm_workspace_bytes          */
#define VSM_E_BUDGET (-5)    /* serving: job larger than the whole memory budget     */
#define VSM_E_HIP (-6)       /* a HIP call failed; see vsm_last_hip_error()          */
#define VSM_E_STATE (-7)     /* serving: unknown job, or the job cannot do this now   */
#define VSM_E_TIMEOUT (-8)   /* serving: the wait ended before the job finished       */

#define VSM_FP64 0
#define VSM_FP32_BULK 1

#define VSM_JACOBI 0   /* smearing: every link from the previous sweep (Sec. III.A)   */
#define VSM_ANNEALED 1 /* annealing: masked subsets updated in place (Sec. III.A)    */

#define VSM_STOUT 0    /* U' = exp(rho Q) U (Eq. stout, Eq. generator)                */
#define VSM_MAXRETR 1  /* MaxReTr of V = (1-alpha) U + alpha/6 Sigma (Sec. III);
                          alpha = 1 is cooling                                        */
#define VSM_APE 2      /* APE: the same V returned to SU(3) by the unit circle
                          projection V (V^dag V)^{-1/2} / cbrt(det) (Sec. II.C)        */

/* How a sweep updates links. */
typedef struct {
  int32_t order;     /* VSM_JACOBI or VSM_ANNEALED                                    */
  int32_t update;    /* VSM_STOUT or VSM_MAXRETR                                      */
  int32_t vp;        /* 1: vortex-preserving accept/reject of Sec. VI                 */
  int32_t su2_loops; /* MaxReTr: loops over the three SU(2) subgroups (paper: 3)      */
  double u0;         /* mean link in the rectangle weight of Eq. (over-improvement)  */
  double alpha;      /* MaxReTr and APE: blocking fraction of Eq. (V)                 */
} vsm_schedule;

/* One measurement record (64 bytes, host or device). */
typedef struct {
  double plaq;              /* <P> = (1/18V) sum_x sum_{mu<nu} Re Tr P_{mu nu}(x)         */
  double action;            /* <S>/beta = (1/36V) sum_x sum_{mu<nu} Re Tr[1 - P_{mu nu}]  */
  double max_unitarity;     /* max over links and entries of |U^dag U - 1|               */
  double sweep;             /* sweeps done when the record was taken                    */
  int64_t flux_mismatch;    /* plaquettes whose vortex flux differs from the original   */
  int64_t undefined_sector; /* links whose trace lies on a sector boundary or is 0      */
  int64_t rejected;         /* vortex-preservation rejections since the last record     */
  int64_t nonfinite;        /* links with a non-finite entry                            */
} vsm_stats;

/* Library version string; never NULL. */
const char *vsm_version(void);
/* Text of a status code; never NULL. */
const char *vsm_strerror(int status);
/* hipError_t of the last VSM_E_HIP returned on this thread (0 if none). */
int vsm_last_hip_error(void);

/* 0 if dims are allowed for `order` (VSM_JACOBI or VSM_ANNEALED) and precision,
 * otherwise VSM_E_DIMS or VSM_E_NULL.  Host only. */
int vsm_check_dims(const int32_t dims[4], int32_t order, int32_t precision);
/* Bytes of the internal link buffer (0 for invalid arguments). */
size_t vsm_links_bytes(const int32_t dims[4], int32_t precision);
/* Bytes of device workspace that vsm_smooth / vsm_measure / vsm_pass need for
 * this order: counters, reduction slots and a copy of the charges in the
 * internal layout (4V bytes), plus a second link buffer for VSM_JACOBI.  0 for
 * invalid arguments. */
size_t vsm_workspace_bytes(const int32_t dims[4], int32_t precision, int32_t order);

/* Copy links in from / out to the canonical interchange layout:
 * canon = device complex128 [4][V][3][3] (row-major 3x3, re/im interleaved).
 * FP32_BULK rounds on the way in and widens exactly on the way out. */
int vsm_set_links(const int32_t dims[4], int32_t precision, const double *canon_dev, void *links_dev,
                  void *stream);
int vsm_get_links(const int32_t dims[4], int32_t precision, const void *links_dev, double *canon_dev,
                  void *stream);

/* Sec. I, Eq. (centre_project): U_mu(x) = e^{2 pi i n_mu(x)/3} 1 from the charges
 * z3_dev = device int8 [4][V] with values in {-1, 0, 1}.  Values outside that set
 * are not checked on the device (they are treated as the nearest valid one). */
int vsm_load_z3(const int32_t dims[4], int32_t precision, const int8_t *z3_dev, void *links_dev,
                void *stream);

/* Sec. IV: centrifuge preconditioning of the Z(3) field with charges z3_dev.
 * For every link, with lambda = 2 pi n/3 and the staple phase sigma = 2 pi m/18
 * (m the integer sum over the six staples of the neighbouring charges),
 * lambda^j = (1-omega) lambda + omega sigma, lambda^k = (1+omega) lambda - omega sigma
 * (Eqs. lambda_j, lambda_k), the third phase unchanged.  pair_dev = device int8
 * [4][V] with the random pair per link, 0, 1, 2 = (j,k) = (1,2), (2,3), (3,1).
 * |omega| must be below 1/4 (Sec. IV.A): then omega |m - 6n| < 6 holds for every
 * link and the centre sector of every link is kept.  m_dev (device int32 [4][V])
 * receives m when not NULL.  Overwrites links_dev. */
int vsm_precondition(const int32_t dims[4], int32_t precision, const int8_t *z3_dev,
                     const int8_t *pair_dev, double omega, void *links_dev, int32_t *m_dev,
                     void *stream);

/* Sec. V.C: U_mu(x) -> G(x) U_mu(x) G^dagger(x + mu) in place, gauge_dev = device
 * complex128 [V][3][3], canonical site order.  Test and recipe utility. */
int vsm_gauge_transform(const int32_t dims[4], int32_t precision, void *links_dev,
                        const double *gauge_dev, void *stream);

/* n_sweeps sweeps of the update chosen by *sched (host pointer) on links_dev.
 *   rho  stout step (flow-time step of the Euler integration, Sec. V.B).
 *   eps  over-improvement parameter of Eq. (over-improvement): staple weights
 *        (5 - 2 eps)/3 and (eps - 1)/(12 u0^2); eps = 1 gives the plain staples
 *        of Eq. (plaq_staples).
 *   VSM_ANNEALED: per sweep, for mu = 0..3, the subsets c = 0, 2, 1, 3 with
 *        c = (2 x_mu + sum_{nu != mu} x_nu) mod 4 (no two links of a subset share a
 *        staple path), each updated in place.  VSM_JACOBI: every link from the
 *        previous sweep's field.
 *   vp   with sched->vp, a candidate is kept only if its Z(3) projection equals
 *        the original charge z3_dev (Sec. VI); with gauge_dev != NULL the test
 *        projects G^dagger(x) U' G(x + mu) (the field is in that random gauge).
 *   measure_every > 0: after every measure_every-th sweep a vsm_stats record is
 *        written to stats_dev (device, n_sweeps / measure_every records).
 *   workspace_dev: device, at least vsm_workspace_bytes(dims, precision, order).
 * z3_dev is required when vp or measurement is on. */
int vsm_smooth(const int32_t dims[4], int32_t precision, void *links_dev, const int8_t *z3_dev,
               const double *gauge_dev, void *workspace_dev, size_t workspace_bytes,
               int32_t n_sweeps, double rho, double eps, const vsm_schedule *sched,
               int32_t measure_every, vsm_stats *stats_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): vsm_smooth
 * with every argument as there except the workspace, which is a static device
 * array of VSM_NOALLOC_SCRATCH_BYTES (64 MiB) inside the library, one per device
 * that the library runs on, held until the process ends.  The call allocates
 * nothing; the caller still passes links, charges, gauge and stats.  Enough
 * for annealed sweeps with measurement up to about 15.5M sites (48^3 x 96 fits)
 * and for smearing up to 170k sites in FP64 (340k in FP32-bulk); larger
 * lattices return VSM_E_WORKSPACE before anything is enqueued.  The first call
 * on a device looks up that device's array (hipGetSymbolAddress) with the
 * device current.  Every call on a device shares its array (counters, charges,
 * reduction slots, the smearing buffer), and each call re-initialises what it
 * reads: calls that overlap on one device (two streams, two threads) race and
 * must be serialised by the caller. */
#define VSM_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
size_t vsm_noalloc_scratch_bytes(void);
int vsm_smooth_noalloc(const int32_t dims[4], int32_t precision, void *links_dev, const int8_t *z3_dev,
                       const double *gauge_dev, int32_t n_sweeps, double rho, double eps,
                       const vsm_schedule *sched, int32_t measure_every, vsm_stats *stats_dev, void *stream);

/* One annealing subset (direction mu, subset colour) of the update chosen by
 * *sched, in place; the building block of an annealed sweep.  The rejection
 * count accumulates in the workspace until the next measurement. */
int vsm_pass(const int32_t dims[4], int32_t precision, void *links_dev, const int8_t *z3_dev,
             const double *gauge_dev, void *workspace_dev, size_t workspace_bytes, int32_t mu,
             int32_t colour, double rho, double eps, const vsm_schedule *sched, void *stream);

/* Sec. I, V.A: one vsm_stats record of links_dev into stats_dev (device); the
 * vortex flux p_{mu nu}(x) in {-1, 0, 1} of the current links' centre projections
 * into flux_dev (device int8 [6][V], planes 01, 02, 03, 12, 13, 23; -128 where a
 * sector is undefined) when not NULL.  gauge_dev (nullable, as for vsm_smooth):
 * the field lives in that random gauge (Sec. V.C), and a link's centre
 * projection is taken from G^dagger(x) U G(x + mu), where the original charges
 * z3_dev live.  The rejected field reports the count accumulated in the
 * workspace since the last record and clears it. */
int vsm_measure(const int32_t dims[4], int32_t precision, const void *links_dev, const int8_t *z3_dev,
                const double *gauge_dev, void *workspace_dev, size_t workspace_bytes, vsm_stats *stats_dev,
                int8_t *flux_dev, void *stream);

/* Sec. II.B, V.B: n_steps steps of size eps of the Wilson flow
 * dU/dtau = Q[U] U, every link at once (Q the stout generator with staples of
 * over-improvement eps_oi, u0 as for vsm_smooth).  VSM_EULER: U <- exp(eps Q) U
 * (the simultaneous stout step).  VSM_RK3: the third-order Runge-Kutta scheme
 * W1 = exp(Z0/4) W0, W2 = exp(8/9 Z1 - 17/36 Z0) W1,
 * U(tau + eps) = exp(3/4 Z2 - 8/9 Z1 + 17/36 Z0) W2 with Z_i = eps Q[W_i].
 * workspace_dev: at least vsm_flow_workspace_bytes (a second link buffer, and
 * for RK3 an FP64 accumulator of 8 reals per link). */
#define VSM_EULER 0
#define VSM_RK3 1
size_t vsm_flow_workspace_bytes(const int32_t dims[4], int32_t precision, int32_t integrator);
int vsm_flow(const int32_t dims[4], int32_t precision, void *links_dev, void *workspace_dev,
             size_t workspace_bytes, int32_t n_steps, double eps, double eps_oi, double u0, int32_t integrator,
             void *stream);

/* Sec. V, Eqs. (1LFST), (1LTopQ) and the reconstructed action of Sec. V.A,
 * with g = 1: the 1x1 clover C_{mu nu}(x) (mean of the four plaquettes of the
 * plane that start and end at x), F_{mu nu} = (C - C^dag)/(2i) (no trace
 * removed, as written), q(x) = eps_{mu nu rho sigma} Tr[F_{mu nu} F_{rho sigma}] /
 * (32 pi^2), S_R(x)/beta = sum over the six planes of Tr[F F] / 72.
 * out_dev (device, 4 doubles) = {<S_R>/beta, Q = sum_x q(x), <S>/beta, 0};
 * the smoothness condition of Sec. V.A compares <S_R> with <S>.  sdens_dev and
 * qdens_dev (device float64 [V], canonical site order, nullable) receive
 * S(x)/beta and q(x).  Arithmetic in FP64 for both precisions.  Uses the
 * reduction slots of the workspace. */
int vsm_measure_clover(const int32_t dims[4], int32_t precision, const void *links_dev, void *workspace_dev,
                       size_t workspace_bytes, double *out_dev, double *sdens_dev, double *qdens_dev,
                       void *stream);

/* Sec. VII, Eq. (correlation_s): out_dev (device, 4 doubles) =
 * {<a b>/sqrt(<a^2> <b^2>), sum a b, sum a^2, sum b^2} over n device doubles
 * (for example two action or charge densities).  n > 0. */
int vsm_correlate(int64_t n, const double *a_dev, const double *b_dev, double *out_dev, void *stream);

/* ------------------------------------------------------------------ serving
 *
 * A server smooths a stream of independent jobs (Z(3) fields of any allowed
 * size) on one GPU with continuous batching.  It owns one worker thread, one
 * HIP stream, one device memory pool of hbm_budget_bytes and one pinned host
 * pool of host_budget_bytes, all allocated by vsm_server_create and released by
 * vsm_server_destroy; nothing else allocates on the device while it runs.
 *
 * A submitted job waits in a FIFO queue until its footprint
 * (vsm_server_job_bytes) fits in the free device pool and a slot is free; it is
 * then admitted: its charges (and centrifuge pairs) are uploaded, the field is
 * built (Sec. I ingest, or Sec. IV preconditioning) and stays resident until
 * the job ends.  Every scheduler step is one kernel launch that runs the next
 * annealing subset pass (Sec. III.A order: mu = 0..3, subsets 0, 2, 1, 3) of
 * every resident job, so jobs that arrive while others run join at the next
 * step and small lattices share launches.  Measurement records follow the
 * rules of vsm_smooth, plus one final record after the last sweep when
 * n_sweeps is not a multiple of measure_every (or measure_every = 0).  A job's
 * links and records are bit-identical whatever other jobs run beside it; they
 * equal vsm_smooth's up to the rounding of the same arithmetic in another
 * kernel.  Only VSM_ANNEALED stout schedules are served, without a gauge.
 *
 * Job states: QUEUED -> RUNNING -> DONE, or FAILED (a HIP error, or the server
 * was destroyed first).  Times are seconds on the server's steady clock
 * (vsm_server_clock).  All server calls are thread-safe. */

#define VSM_JOB_QUEUED 0
#define VSM_JOB_RUNNING 1
#define VSM_JOB_DONE 2
#define VSM_JOB_FAILED 3

typedef struct {
  size_t hbm_budget_bytes;  /* device pool for resident jobs (> 0)                       */
  size_t host_budget_bytes; /* pinned host pool for uploads and results (> 0)            */
  int32_t max_slots;        /* jobs resident at once, 1..256                             */
  int32_t max_inflight;     /* scheduler steps queued ahead of the GPU, 1..64            */
  int32_t device;           /* HIP device ordinal                                        */
  int32_t reserved;
} vsm_server_config;

typedef struct {
  int32_t dims[4];          /* as for every call; the field's extents                    */
  int32_t precision;        /* VSM_FP64 or VSM_FP32_BULK                                  */
  int32_t n_sweeps;         /* >= 0                                                       */
  double rho, eps;          /* as for vsm_smooth                                          */
  double omega;             /* centrifuge parameter, |omega| < 1/4 (unused without pairs) */
  vsm_schedule sched;       /* order VSM_ANNEALED, update VSM_STOUT                       */
  int32_t measure_every;    /* >= 0, as for vsm_smooth                                    */
  int32_t want_links;       /* 1: keep the final links (canonical layout) for fetch       */
  const int8_t *z3_host;    /* host int8 [4][V] charges; copied by submit                 */
  const int8_t *pair_host;  /* host int8 [4][V] centrifuge pairs, copied by submit, or
                               NULL for the plain Z(3) field                              */
} vsm_job;

typedef struct {
  int32_t state;            /* VSM_JOB_*                                                  */
  int32_t status;           /* VSM_OK, or the error that failed the job                   */
  int32_t n_records;        /* vsm_stats records the job produces                         */
  int32_t sweeps_done;      /* sweeps enqueued so far                                     */
  double t_submit, t_admit, t_done; /* server clock; -1 until reached                    */
  size_t footprint_bytes;   /* device pool bytes the job holds while resident            */
} vsm_job_info;

typedef struct {
  int64_t steps;            /* scheduler steps (batched launches) enqueued               */
  int64_t launches;         /* kernel launches of those steps                            */
  int64_t jobs_submitted, jobs_done, jobs_failed;
  int64_t link_updates;     /* link updates enqueued over all jobs                       */
  int64_t peak_resident_jobs;
  size_t peak_pool_bytes;   /* high-water mark of the device pool                        */
  double busy_seconds;      /* worker time with at least one job resident                */
} vsm_server_counters;

/* Device pool bytes one job needs (links, charges, pairs, workspace, records,
 * and the canonical link buffer when want_links); 0 if the job is invalid. */
size_t vsm_server_job_bytes(const vsm_job *job);
/* Pinned host pool bytes one job needs (uploads and results). */
size_t vsm_server_host_bytes(const vsm_job *job);

/* Creates a server; *srv receives its handle.  VSM_E_HIP if a pool cannot be
 * allocated. */
int vsm_server_create(const vsm_server_config *cfg, void **srv);
/* Validates and enqueues a job; *job_id receives its id.  VSM_E_BUDGET if the
 * job can never fit the pools; VSM_E_PARAM for a schedule the server does not
 * serve; VSM_E_STATE after destroy has begun. */
int vsm_server_submit(void *srv, const vsm_job *job, uint64_t *job_id);
/* Current state of a job into *info (host); does not block. */
int vsm_server_poll(void *srv, uint64_t job_id, vsm_job_info *info);
/* Blocks until the job is DONE or FAILED (VSM_OK) or timeout_s seconds have
 * passed (VSM_E_TIMEOUT; timeout_s < 0 waits without limit); *info as poll. */
int vsm_server_wait(void *srv, uint64_t job_id, double timeout_s, vsm_job_info *info);
/* Copies a DONE job's results to host memory and forgets the job:
 * records_host receives up to max_records vsm_stats, links_host (complex128
 * [4][V][3][3], may be NULL) the final links if the job kept them.  A FAILED
 * job is forgotten and its status returned.  VSM_E_STATE if not finished. */
int vsm_server_fetch(void *srv, uint64_t job_id, vsm_stats *records_host, int32_t max_records,
                     double *links_host);
/* Seconds on the server's steady clock. */
double vsm_server_clock(void *srv);
/* Scheduler counters into *out (host). */
int vsm_server_get_counters(void *srv, vsm_server_counters *out);
/* Stops admitting, lets the device finish what is enqueued, fails the jobs
 * not finished, joins the worker and releases the pools and the handle. */
int vsm_server_destroy(void *srv);

#ifdef __cplusplus
}
#endif

#endif /* VSM_H */
