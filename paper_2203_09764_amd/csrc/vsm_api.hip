// vsm_api.hip -- the C ABI of include/vsm.h: validation, workspace layout and the
// launch sequences of the smoothing path.  No entry point allocates memory.
#include <math.h>
#include <string.h>

#include "vsm.h"
#include "vsm_host.h"
#include "vsm_launch.h"

using namespace vsm;

namespace {
thread_local int g_last_hip = 0;
}  // namespace

namespace vsm {

int note_hip_error(hipError_t e) {
  if (e == hipSuccess) return VSM_OK;
  g_last_hip = (int)e;
  return VSM_E_HIP;
}

int hip_status() { return note_hip_error(hipGetLastError()); }

}  // namespace vsm

extern "C" {

const char* vsm_version(void) { return "vsm 1.0 (gfx950)"; }

const char* vsm_strerror(int status) {
  switch (status) {
    case VSM_OK: return "ok";
    case VSM_E_DIMS: return "lattice extents not allowed (each >= 4 and a multiple of 4, 6*V*entry < 2^31)";
    case VSM_E_PARAM: return "parameter outside its domain";
    case VSM_E_NULL: return "required pointer is NULL";
    case VSM_E_WORKSPACE: return "workspace too small";
    case VSM_E_BUDGET: return "job exceeds the memory budget";
    case VSM_E_HIP: return "HIP call failed (see vsm_last_hip_error)";
    case VSM_E_STATE: return "unknown job or server state";
    case VSM_E_TIMEOUT: return "timed out waiting for the job";
    default: return "unknown status";
  }
}

int vsm_last_hip_error(void) { return g_last_hip; }

int vsm_check_dims(const int32_t dims[4], int32_t order, int32_t precision) {
  return check_dims_impl(dims, order, precision);
}

size_t vsm_links_bytes(const int32_t dims[4], int32_t precision) {
  if (check_dims_impl(dims, VSM_JACOBI, precision) != VSM_OK) return 0;
  const Geo g = make_geo(dims);
  return 24ull * g.es * entry_bytes(precision);
}

size_t vsm_workspace_bytes(const int32_t dims[4], int32_t precision, int32_t order) {
  if (check_dims_impl(dims, order, precision) != VSM_OK) return 0;
  return ws_layout(dims, precision, order).total;
}

int vsm_set_links(const int32_t dims[4], int32_t precision, const double* canon_dev, void* links_dev,
                  void* stream) {
  int rc = check_dims_impl(dims, VSM_JACOBI, precision);
  if (rc) return rc;
  if (!canon_dev || !links_dev) return VSM_E_NULL;
  launch_set_links(precision, make_geo(dims), canon_dev, links_dev, (hipStream_t)stream);
  return hip_status();
}

int vsm_get_links(const int32_t dims[4], int32_t precision, const void* links_dev, double* canon_dev,
                  void* stream) {
  int rc = check_dims_impl(dims, VSM_JACOBI, precision);
  if (rc) return rc;
  if (!canon_dev || !links_dev) return VSM_E_NULL;
  launch_get_links(precision, make_geo(dims), links_dev, canon_dev, (hipStream_t)stream);
  return hip_status();
}

int vsm_load_z3(const int32_t dims[4], int32_t precision, const int8_t* z3_dev, void* links_dev,
                void* stream) {
  int rc = check_dims_impl(dims, VSM_JACOBI, precision);
  if (rc) return rc;
  if (!z3_dev || !links_dev) return VSM_E_NULL;
  launch_load_z3(precision, make_geo(dims), z3_dev, links_dev, (hipStream_t)stream);
  return hip_status();
}

int vsm_precondition(const int32_t dims[4], int32_t precision, const int8_t* z3_dev,
                     const int8_t* pair_dev, double omega, void* links_dev, int32_t* m_dev,
                     void* stream) {
  int rc = check_dims_impl(dims, VSM_JACOBI, precision);
  if (rc) return rc;
  if (!z3_dev || !pair_dev || !links_dev) return VSM_E_NULL;
  if (!is_fin(omega) || !(fabs(omega) < 0.25)) return VSM_E_PARAM;
  launch_centrifuge(precision, make_geo(dims), z3_dev, pair_dev, omega, links_dev, m_dev,
                    (hipStream_t)stream);
  return hip_status();
}

int vsm_gauge_transform(const int32_t dims[4], int32_t precision, void* links_dev,
                        const double* gauge_dev, void* stream) {
  int rc = check_dims_impl(dims, VSM_JACOBI, precision);
  if (rc) return rc;
  if (!links_dev || !gauge_dev) return VSM_E_NULL;
  launch_gauge(precision, make_geo(dims), links_dev, gauge_dev, (hipStream_t)stream);
  return hip_status();
}

}  // extern "C"

namespace vsm {

int smooth_impl(const int32_t dims[4], int32_t precision, void* links_dev, const int8_t* z3_dev,
                const double* gauge_dev, char* ws, size_t ws_bytes, int32_t n_sweeps, double rho, double eps,
                const vsm_schedule* sched, int32_t measure_every, vsm_stats* stats_dev, hipStream_t st) {
  int rc = check_sched(sched);
  if (rc) return rc;
  rc = check_dims_impl(dims, sched->order, precision);
  if (rc) return rc;
  if (!links_dev || !ws) return VSM_E_NULL;
  if (n_sweeps < 0 || measure_every < 0 || !is_fin(rho) || !is_fin(eps)) return VSM_E_PARAM;
  if ((sched->vp || measure_every > 0) && !z3_dev) return VSM_E_NULL;
  if (measure_every > 0 && !stats_dev) return VSM_E_NULL;
  const WsLayout w = ws_layout(dims, precision, sched->order);
  if (ws_bytes < w.total) return VSM_E_WORKSPACE;
  const Geo g = make_geo(dims);
  const UpdParams p = make_params(rho, eps, sched);
  unsigned long long* rej = (unsigned long long*)(ws + w.counters);
  VsmStatsDev* out = (VsmStatsDev*)stats_dev;
  // the measurement reads the charges in the internal layout
  int8_t* z3i = nullptr;
  if (measure_every > 0) {
    z3i = (int8_t*)(ws + w.charges);
    launch_charges(g, z3_dev, z3i, 0, 4, st);
  }
  launch_zero_u64(rej, 1, st);
  void* cur = links_dev;
  void* other = ws + w.field;
  int rec = 0;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    if (sched->order == VSM_JACOBI) {
      for (int mu = 0; mu < 4; ++mu)
        launch_update(precision, g, cur, other, z3_dev, gauge_dev, p, g.perm[mu], 0, 1, rej, st);
      void* t = cur;
      cur = other;
      other = t;
    } else {
      for (int mu = 0; mu < 4; ++mu)
        for (int c = 0; c < 4; ++c)
          launch_update(precision, g, links_dev, links_dev, z3_dev, gauge_dev, p, g.perm[mu], kColours[c], 0,
                        rej, st);
    }
    if (measure_every > 0 && (sw + 1) % measure_every == 0) {
      launch_measure(precision, g, cur, z3i, gauge_dev, ws + w.partials, nullptr, rej, out + rec, sw + 1, st);
      ++rec;
    }
  }
  if (cur != links_dev) {
    const hipError_t e =
        hipMemcpyAsync(links_dev, cur, 24ull * g.es * entry_bytes(precision), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return note_hip_error(e);
  }
  return hip_status();
}

}  // namespace vsm

extern "C" {

int vsm_smooth(const int32_t dims[4], int32_t precision, void* links_dev, const int8_t* z3_dev,
               const double* gauge_dev, void* workspace_dev, size_t workspace_bytes,
               int32_t n_sweeps, double rho, double eps, const vsm_schedule* sched,
               int32_t measure_every, vsm_stats* stats_dev, void* stream) {
  return smooth_impl(dims, precision, links_dev, z3_dev, gauge_dev, (char*)workspace_dev, workspace_bytes, n_sweeps,
                     rho, eps, sched, measure_every, stats_dev, (hipStream_t)stream);
}

int vsm_pass(const int32_t dims[4], int32_t precision, void* links_dev, const int8_t* z3_dev,
             const double* gauge_dev, void* workspace_dev, size_t workspace_bytes, int32_t mu,
             int32_t colour, double rho, double eps, const vsm_schedule* sched, void* stream) {
  int rc = check_sched(sched);
  if (rc) return rc;
  rc = check_dims_impl(dims, VSM_ANNEALED, precision);
  if (rc) return rc;
  if (!links_dev || !workspace_dev) return VSM_E_NULL;
  if (sched->vp && !z3_dev) return VSM_E_NULL;
  if (mu < 0 || mu > 3 || colour < 0 || colour > 3 || !is_fin(rho) || !is_fin(eps)) return VSM_E_PARAM;
  const WsLayout w = ws_layout(dims, precision, VSM_ANNEALED);
  if (workspace_bytes < w.total) return VSM_E_WORKSPACE;
  const UpdParams p = make_params(rho, eps, sched);
  unsigned long long* rej = (unsigned long long*)((char*)workspace_dev + w.counters);
  const Geo g = make_geo(dims);
  launch_update(precision, g, links_dev, links_dev, z3_dev, gauge_dev, p, g.perm[mu], colour, 0, rej,
                (hipStream_t)stream);
  return hip_status();
}

int vsm_measure(const int32_t dims[4], int32_t precision, const void* links_dev, const int8_t* z3_dev,
                const double* gauge_dev, void* workspace_dev, size_t workspace_bytes, vsm_stats* stats_dev,
                int8_t* flux_dev, void* stream) {
  int rc = check_dims_impl(dims, VSM_JACOBI, precision);
  if (rc) return rc;
  if (!links_dev || !z3_dev || !workspace_dev || !stats_dev) return VSM_E_NULL;
  const WsLayout w = ws_layout(dims, precision, VSM_ANNEALED);
  if (workspace_bytes < w.total) return VSM_E_WORKSPACE;
  char* ws = (char*)workspace_dev;
  const Geo g = make_geo(dims);
  hipStream_t st = (hipStream_t)stream;
  launch_charges(g, z3_dev, (int8_t*)(ws + w.charges), 0, 4, st);
  launch_measure(precision, g, links_dev, (const int8_t*)(ws + w.charges), gauge_dev, ws + w.partials, flux_dev,
                 (unsigned long long*)(ws + w.counters), (VsmStatsDev*)stats_dev, -1, st);
  return hip_status();
}

size_t vsm_flow_workspace_bytes(const int32_t dims[4], int32_t precision, int32_t integrator) {
  if (check_dims_impl(dims, VSM_JACOBI, precision) != VSM_OK) return 0;
  if (integrator != VSM_EULER && integrator != VSM_RK3) return 0;
  const WsLayout w = ws_layout(dims, precision, VSM_JACOBI);
  const Geo g = make_geo(dims);
  return w.total + (integrator == VSM_RK3 ? align256(8ull * 4ull * g.V * sizeof(double)) : 0);
}

int vsm_flow(const int32_t dims[4], int32_t precision, void* links_dev, void* workspace_dev, size_t workspace_bytes,
             int32_t n_steps, double eps, double eps_oi, double u0, int32_t integrator, void* stream) {
  int rc = check_dims_impl(dims, VSM_JACOBI, precision);
  if (rc) return rc;
  if (!links_dev || !workspace_dev) return VSM_E_NULL;
  if (n_steps < 0 || !is_fin(eps) || !is_fin(eps_oi) || !is_fin(u0) || u0 == 0.0) return VSM_E_PARAM;
  if (integrator != VSM_EULER && integrator != VSM_RK3) return VSM_E_PARAM;
  if (workspace_bytes < vsm_flow_workspace_bytes(dims, precision, integrator)) return VSM_E_WORKSPACE;
  const WsLayout w = ws_layout(dims, precision, VSM_JACOBI);
  const Geo g = make_geo(dims);
  hipStream_t st = (hipStream_t)stream;
  const double cp = (5.0 - 2.0 * eps_oi) / 3.0, cr = (eps_oi - 1.0) / (12.0 * u0 * u0);
  char* ws = (char*)workspace_dev;
  double* acc = integrator == VSM_RK3 ? (double*)(ws + w.total) : nullptr;
  void* cur = links_dev;
  void* other = ws + w.field;
  for (int k = 0; k < n_steps; ++k) {
    const int stages = integrator == VSM_RK3 ? 3 : 1;
    for (int sg = 0; sg < stages; ++sg) {
      launch_flow(precision, g, cur, other, acc, integrator == VSM_RK3 ? sg + 1 : 0, eps, cp, cr, st);
      void* t = cur;
      cur = other;
      other = t;
    }
  }
  if (cur != links_dev) {
    const hipError_t e =
        hipMemcpyAsync(links_dev, cur, 24ull * g.es * entry_bytes(precision), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return note_hip_error(e);
  }
  return hip_status();
}

int vsm_measure_clover(const int32_t dims[4], int32_t precision, const void* links_dev, void* workspace_dev,
                       size_t workspace_bytes, double* out_dev, double* sdens_dev, double* qdens_dev,
                       void* stream) {
  int rc = check_dims_impl(dims, VSM_JACOBI, precision);
  if (rc) return rc;
  if (!links_dev || !workspace_dev || !out_dev) return VSM_E_NULL;
  const WsLayout w = ws_layout(dims, precision, VSM_ANNEALED);
  if (workspace_bytes < w.total) return VSM_E_WORKSPACE;
  launch_clover(precision, make_geo(dims), links_dev, (char*)workspace_dev + w.partials, out_dev, sdens_dev,
                qdens_dev, (hipStream_t)stream);
  return hip_status();
}

int vsm_correlate(int64_t n, const double* a_dev, const double* b_dev, double* out_dev, void* stream) {
  if (!a_dev || !b_dev || !out_dev) return VSM_E_NULL;
  if (n <= 0) return VSM_E_PARAM;
  launch_correlate((long long)n, a_dev, b_dev, out_dev, (hipStream_t)stream);
  return hip_status();
}

}  // extern "C"
