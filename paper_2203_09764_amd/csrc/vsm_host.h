// vsm_host.h -- host-side helpers shared by the C-ABI entry points and the
// serving scheduler: argument validation, the internal lattice geometry, the
// workspace layout and the per-launch update parameters.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "vsm.h"
#include "vsm_launch.h"

namespace vsm {

// Records e as this thread's last HIP error; VSM_E_HIP if e is an error.
int note_hip_error(hipError_t e);
// note_hip_error(hipGetLastError()).
int hip_status();

inline size_t entry_bytes(int32_t precision) { return precision == VSM_FP64 ? 16 : 8; }

inline bool valid_precision(int32_t p) { return p == VSM_FP64 || p == VSM_FP32_BULK; }

inline bool is_fin(double v) { return isfinite(v) != 0; }

inline size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

inline int check_dims_impl(const int32_t dims[4], int32_t order, int32_t precision) {
  if (!dims) return VSM_E_NULL;
  if (!valid_precision(precision)) return VSM_E_PARAM;
  if (order != VSM_JACOBI && order != VSM_ANNEALED) return VSM_E_PARAM;
  uint64_t V = 1;
  for (int d = 0; d < 4; ++d) {
    if (dims[d] < 4 || dims[d] % 4) return VSM_E_DIMS;
    V *= (uint64_t)dims[d];
  }
  if (6ull * (V + kEntryPad) * entry_bytes(precision) >= (1ull << 31)) return VSM_E_DIMS;
  return VSM_OK;
}

// Internal axis 0 (blocked by 4, fastest in memory) is the longest user axis,
// preferring one whose rows of L/4 FP64 entries fill whole 128-byte lines; the
// other user axes follow in their own order.  Directions are relabelled with
// the axes, which leaves the annealing subsets unchanged.
inline Geo make_geo(const int32_t dims[4]) {
  int a0 = 0;
  auto score = [&](int d) { return (long)dims[d] * 2 + (((dims[d] / 4) * 16) % 128 == 0 ? 1 : 0); };
  for (int d = 1; d < 4; ++d)
    if (score(d) > score(a0)) a0 = d;
  Geo g;
  g.perm[a0] = 0;
  g.uperm[0] = a0;
  int k = 1;
  for (int d = 0; d < 4; ++d)
    if (d != a0) {
      g.perm[d] = k;
      g.uperm[k] = d;
      ++k;
    }
  uint32_t cstride[4];
  uint32_t acc = 1;
  for (int d = 0; d < 4; ++d) {
    cstride[d] = acc;
    acc *= (uint32_t)dims[d];
  }
  for (int i = 0; i < 4; ++i) {
    g.L[i] = dims[g.uperm[i]];
    g.cst[i] = cstride[g.uperm[i]];
  }
  g.Xq = g.L[0] / 4;
  g.V = acc;
  g.V4 = g.V / 4;
  g.es = g.V + kEntryPad;
  g.jst[0] = 1;
  g.jst[1] = (uint32_t)g.Xq;
  g.jst[2] = (uint32_t)g.Xq * (uint32_t)g.L[1];
  g.jst[3] = (uint32_t)g.Xq * (uint32_t)g.L[1] * (uint32_t)g.L[2];
  // traversal tiles (see tile_rows): the largest even divisor of L1 up to 16
  // and the largest divisors of L2 and L3 up to 8, the best measured on 48^3x96
  g.T1 = 2;
  for (int t = 16; t >= 2; t -= 2)
    if (g.L[1] % t == 0) {
      g.T1 = t;
      break;
    }
  g.T2 = 1;
  for (int t = 8; t >= 1; --t)
    if (g.L[2] % t == 0) {
      g.T2 = t;
      break;
    }
  g.T3 = 1;
  for (int t = 8; t >= 1; --t)
    if (g.L[3] % t == 0) {
      g.T3 = t;
      break;
    }
  // Lattices of at most 2^19 sites (the serving sizes) take their rows in plain
  // order, one tile: with many of them in one serving step this measured 5%
  // faster than tiles, and a single such lattice runs as fast either way.
  if (g.V <= (1u << 19)) {
    g.T1 = g.L[1];
    g.T2 = g.L[2];
    g.T3 = g.L[3];
  }
  return g;
}

// Workspace: [0, 256) counters (rejections at 0); the measurement block
// partials; the original charges in the internal layout (4V bytes); then, for
// the smearing schedule, a second link buffer.
struct WsLayout {
  size_t counters, partials, charges, field, total;
};

inline WsLayout ws_layout(const int32_t dims[4], int32_t precision, int32_t order) {
  const Geo g = make_geo(dims);
  WsLayout w;
  w.counters = 0;
  w.partials = 256;
  w.charges = align256(w.partials + (size_t)measure_blocks(g) * partial_bytes());
  w.field = align256(w.charges + 4ull * g.V);
  w.total = w.field;
  if (order == VSM_JACOBI) w.total += align256(24ull * g.es * entry_bytes(precision));
  return w;
}

inline int check_sched(const vsm_schedule* s) {
  if (!s) return VSM_E_NULL;
  if (s->order != VSM_JACOBI && s->order != VSM_ANNEALED) return VSM_E_PARAM;
  if (s->update != VSM_STOUT && s->update != VSM_MAXRETR && s->update != VSM_APE) return VSM_E_PARAM;
  if (!is_fin(s->u0) || s->u0 == 0.0) return VSM_E_PARAM;
  if (s->update == VSM_MAXRETR && (!is_fin(s->alpha) || s->su2_loops < 0)) return VSM_E_PARAM;
  if (s->update == VSM_APE && !is_fin(s->alpha)) return VSM_E_PARAM;
  return VSM_OK;
}

// Staple weights of the over-improved action: c_p = (5 - 2 eps)/3 and
// c_r = (eps - 1)/(12 u0^2); eps = 1 leaves the plain plaquette staples.
inline UpdParams make_params(double rho, double eps, const vsm_schedule* s) {
  UpdParams p;
  p.cp = (5.0 - 2.0 * eps) / 3.0;
  p.cr = (eps - 1.0) / (12.0 * s->u0 * s->u0);
  p.rho = rho;
  p.alpha = s->alpha;
  // rounding level of Q: the staple sum adds 6 plaquette and 18 rectangle
  // paths of SU(3) matrices (entries at most 1) with weights c_p and c_r, each
  // carrying a few roundings; 2^-48 (32 units of FP64 rounding) times the sum of
  // the weights.  A centre field's Q stays below it; a generator that small
  // moves a link by less than 1e-13.
  p.qfloor = 3.552713678800501e-15 * (6.0 * fabs(p.cp) + 18.0 * fabs(p.cr));
  p.update = s->update == VSM_MAXRETR ? 1 : (s->update == VSM_APE ? 2 : 0);
  p.oi = p.cr != 0.0 ? 1 : 0;
  p.vp = s->vp ? 1 : 0;
  p.loops = s->su2_loops;
  return p;
}

// Subset order of one direction in an annealed sweep.
constexpr int kColours[4] = {0, 2, 1, 3};

// The sweeps of vsm_smooth (validation included) on a device workspace of
// ws_bytes bytes at ws.
int smooth_impl(const int32_t dims[4], int32_t precision, void* links_dev, const int8_t* z3_dev,
                const double* gauge_dev, char* ws, size_t ws_bytes, int32_t n_sweeps, double rho, double eps,
                const vsm_schedule* sched, int32_t measure_every, vsm_stats* stats_dev, hipStream_t st);

}  // namespace vsm
