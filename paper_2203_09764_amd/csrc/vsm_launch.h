// vsm_launch.h -- internal interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "vsm_device.h"

namespace vsm {

// Parameters of one update step, uniform over the launch.
struct UpdParams {
  double cp;     // plaquette-staple weight (5 - 2 eps)/3
  double cr;     // rectangle weight (eps - 1)/(12 u0^2)
  double rho;    // stout step
  double alpha;  // APE blocking fraction (MaxReTr)
  double qfloor; // stout: |Q|_F at or below which Q counts as 0 (rounding level)
  int update;    // 0 stout, 1 MaxReTr, 2 APE with unit circle projection
  int oi;        // rectangles present (eps != 1)
  int vp;        // vortex-preserving accept/reject
  int loops;     // MaxReTr subgroup loops
};

// Device image of vsm_stats (same field order and sizes).
struct VsmStatsDev {
  double plaq, action, max_unitarity, sweep;
  long long flux_mismatch, undefined_sector, rejected, nonfinite;
};

// A job resident on the device under the serving scheduler: its geometry,
// buffers and update parameters, written once when the job is admitted.
struct ServeJob {
  Geo g;
  void* links;
  const int8_t* z3;  // original charges, canonical layout
  unsigned long long* rej;  // the job's rejection counter
  UpdParams p;
};

// One step of the serving scheduler: one annealing subset pass of each listed
// job, all in one launch.  Job i owns blocks [first_block[i], first_block[i+1])
// (the last one up to the grid size) and runs subset `colour[i]` of internal
// direction mu[i] on jobs[slot[i]].
constexpr int kBatchMax = 64;
struct BatchStep {
  uint32_t first_block[kBatchMax];
  uint32_t slot[kBatchMax];
  uint8_t mu[kBatchMax];
  uint8_t colour[kBatchMax];
  uint32_t njobs;
};

// One step of the small-lattice serving path: each listed job runs `sweeps[i]`
// whole annealed sweeps (all 16 subset passes of each) inside one workgroup,
// the passes separated by workgroup barriers; job i is jobs[slot[i]].
constexpr int kSmallMax = 128;
struct SmallStep {
  uint16_t slot[kSmallMax];
  uint16_t sweeps[kSmallMax];
  uint32_t njobs;
};
// Lattices of at most this many sites are served by the small-lattice path: a
// workgroup of 256 threads then takes at most 8 rounds per subset pass, faster
// than a pass per batched step; larger lattices are faster spread over many
// workgroups, one pass per step.
constexpr uint32_t kSmallSites = 8192;

void launch_set_links(int prec, const Geo& g, const void* canon, void* links, hipStream_t st);
void launch_get_links(int prec, const Geo& g, const void* links, void* canon, hipStream_t st);
void launch_load_z3(int prec, const Geo& g, const int8_t* z3, void* links, hipStream_t st);
void launch_centrifuge(int prec, const Geo& g, const int8_t* z3, const int8_t* pair, double omega,
                       void* links, int32_t* m_out, hipStream_t st);
void launch_gauge(int prec, const Geo& g, void* links, const void* gauge, hipStream_t st);
void launch_update(int prec, const Geo& g, const void* src, void* dst, const int8_t* z3,
                   const void* gauge, const UpdParams& p, int mu, int colour, int jacobi,
                   unsigned long long* rej, hipStream_t st);
uint32_t measure_blocks(const Geo& g);
size_t partial_bytes();
// gauge: the field's random gauge G (canonical complex128 [V][3][3]) or null;
// with it the link sectors are those of G^dagger(x) U G(x + mu).
void launch_measure(int prec, const Geo& g, const void* links, const int8_t* z3, const void* gauge,
                    void* partials, int8_t* flux, unsigned long long* rej, VsmStatsDev* out, long long sweep,
                    hipStream_t st);
// Blocks of 256 threads one annealing pass of g takes.
inline uint32_t pass_blocks(const Geo& g) { return (g.V4 + 255u) / 256u; }
// One serving step: every job of `step` (stout updates, annealed, in place).
void launch_update_batch(int prec, const ServeJob* jobs_dev, const BatchStep& step, uint32_t nblocks,
                         hipStream_t st);
// One small-lattice serving step (stout updates, annealed, in place), one
// workgroup per job of `step`.
void launch_serve_small(int prec, const ServeJob* jobs_dev, const SmallStep& step, hipStream_t st);
// Charges z3 (canonical layout) into out (internal layout, 4V bytes) for the
// internal directions d0 .. d0 + nd - 1.
void launch_charges(const Geo& g, const int8_t* z3, int8_t* out, int d0, int nd, hipStream_t st);
// One Wilson-flow stage (0 Euler, 1..3 Runge-Kutta) of all four directions
// from src into dst; acc: the FP64 accumulator, 8 x 4V doubles.
void launch_flow(int prec, const Geo& g, const void* src, void* dst, double* acc, int stage, double eps,
                 double cp, double cr, hipStream_t st);
// Clover field strength: {<S_R>/beta, Q, <S>/beta, 0} into out (device), the
// densities S(x)/beta and q(x) (canonical order) when not null.
void launch_clover(int prec, const Geo& g, const void* links, void* partials, double* out, double* sdens,
                   double* qdens, hipStream_t st);
// {<ab>/sqrt(<a^2><b^2>), <ab>, <a^2>, <b^2>} (sums, not means) into out.
void launch_correlate(long long n, const double* a, const double* b, double* out, hipStream_t st);
void launch_zero_u64(unsigned long long* p, int n, hipStream_t st);

}  // namespace vsm
