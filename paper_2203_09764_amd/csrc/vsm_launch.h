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
  int update;    // 0 stout, 1 MaxReTr
  int oi;        // rectangles present (eps != 1)
  int vp;        // vortex-preserving accept/reject
  int loops;     // MaxReTr subgroup loops
};

// Device image of vsm_stats (same field order and sizes).
struct VsmStatsDev {
  double plaq, action, max_unitarity, sweep;
  long long flux_mismatch, undefined_sector, rejected, nonfinite;
};

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
void launch_measure(int prec, const Geo& g, const void* links, const int8_t* z3, void* partials,
                    int8_t* flux, unsigned long long* rej, VsmStatsDev* out, long long sweep,
                    hipStream_t st);
void launch_zero_u64(unsigned long long* p, int n, hipStream_t st);

}  // namespace vsm
