// vsm_kernels.hip -- precision dispatch of the kernel launchers, and the small
// kernels that do not depend on the precision.
#include "vsm_launch.h"

namespace vsm {

template <typename R>
void launch_set_links_t(const Geo&, const void*, void*, hipStream_t);
template <typename R>
void launch_get_links_t(const Geo&, const void*, void*, hipStream_t);
template <typename R>
void launch_load_z3_t(const Geo&, const int8_t*, void*, hipStream_t);
template <typename R>
void launch_centrifuge_t(const Geo&, const int8_t*, const int8_t*, double, void*, int32_t*, hipStream_t);
template <typename R>
void launch_gauge_t(const Geo&, void*, const void*, hipStream_t);
template <typename R>
void launch_update_t(const Geo&, const void*, void*, const int8_t*, const void*, const UpdParams&, int,
                     int, int, unsigned long long*, hipStream_t);
template <typename R>
void launch_update_batch_t(const ServeJob*, const BatchStep&, uint32_t, hipStream_t);
template <typename R>
void launch_serve_small_t(const ServeJob*, const SmallStep&, hipStream_t);
template <typename R>
void launch_clover_t(const Geo&, const void*, void*, double*, double*, double*, hipStream_t);
template <typename R>
void launch_flow_t(const Geo&, const void*, void*, double*, int, double, double, double, hipStream_t);
template <typename R>
void launch_measure_t(const Geo&, const void*, const int8_t*, const void*, void*, int8_t*, unsigned long long*,
                      VsmStatsDev*, long long, hipStream_t);

// Clears n 64-bit counters (a kernel rather than a memset, so that the call can
// sit inside a captured graph).
__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Charges from the canonical layout (user direction, canonical site) to the
// internal one (internal direction d, internal site index) for directions
// d0 .. d0 + nd - 1, so that the update and measurement kernels read them with
// the same coalesced index as the links.
__global__ void k_charges(Geo g, const int8_t* __restrict__ z3, int8_t* __restrict__ out, int d0,
                          int nd) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (size_t)nd * g.V) return;
  const int d = d0 + (int)(tid / g.V);
  const uint32_t idx = (uint32_t)(tid % g.V);
  int c[4];
  coords_of_index(g, idx, c);
  out[(size_t)d * g.V + idx] = z3[(size_t)g.uperm[d] * g.V + canonical_index(g, c)];
}

void launch_charges(const Geo& g, const int8_t* z3, int8_t* out, int d0, int nd, hipStream_t st) {
  const size_t n = (size_t)nd * g.V;
  hipLaunchKernelGGL(k_charges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, z3, out, d0, nd);
}

void launch_zero_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, p, n);
}

void launch_set_links(int prec, const Geo& g, const void* canon, void* links, hipStream_t st) {
  if (prec == 0) launch_set_links_t<double>(g, canon, links, st);
  else launch_set_links_t<float>(g, canon, links, st);
}

void launch_get_links(int prec, const Geo& g, const void* links, void* canon, hipStream_t st) {
  if (prec == 0) launch_get_links_t<double>(g, links, canon, st);
  else launch_get_links_t<float>(g, links, canon, st);
}

void launch_load_z3(int prec, const Geo& g, const int8_t* z3, void* links, hipStream_t st) {
  if (prec == 0) launch_load_z3_t<double>(g, z3, links, st);
  else launch_load_z3_t<float>(g, z3, links, st);
}

void launch_centrifuge(int prec, const Geo& g, const int8_t* z3, const int8_t* pair, double omega,
                       void* links, int32_t* m_out, hipStream_t st) {
  if (prec == 0) launch_centrifuge_t<double>(g, z3, pair, omega, links, m_out, st);
  else launch_centrifuge_t<float>(g, z3, pair, omega, links, m_out, st);
}

void launch_gauge(int prec, const Geo& g, void* links, const void* gauge, hipStream_t st) {
  if (prec == 0) launch_gauge_t<double>(g, links, gauge, st);
  else launch_gauge_t<float>(g, links, gauge, st);
}

void launch_update(int prec, const Geo& g, const void* src, void* dst, const int8_t* z3,
                   const void* gauge, const UpdParams& p, int mu, int colour, int jacobi,
                   unsigned long long* rej, hipStream_t st) {
  if (prec == 0) launch_update_t<double>(g, src, dst, z3, gauge, p, mu, colour, jacobi, rej, st);
  else launch_update_t<float>(g, src, dst, z3, gauge, p, mu, colour, jacobi, rej, st);
}

void launch_update_batch(int prec, const ServeJob* jobs_dev, const BatchStep& step, uint32_t nblocks,
                         hipStream_t st) {
  if (prec == 0) launch_update_batch_t<double>(jobs_dev, step, nblocks, st);
  else launch_update_batch_t<float>(jobs_dev, step, nblocks, st);
}

void launch_serve_small(int prec, const ServeJob* jobs_dev, const SmallStep& step, hipStream_t st) {
  if (prec == 0) launch_serve_small_t<double>(jobs_dev, step, st);
  else launch_serve_small_t<float>(jobs_dev, step, st);
}

void launch_flow(int prec, const Geo& g, const void* src, void* dst, double* acc, int stage, double eps,
                 double cp, double cr, hipStream_t st) {
  if (prec == 0) launch_flow_t<double>(g, src, dst, acc, stage, eps, cp, cr, st);
  else launch_flow_t<float>(g, src, dst, acc, stage, eps, cp, cr, st);
}

void launch_clover(int prec, const Geo& g, const void* links, void* partials, double* out, double* sdens,
                   double* qdens, hipStream_t st) {
  if (prec == 0) launch_clover_t<double>(g, links, partials, out, sdens, qdens, st);
  else launch_clover_t<float>(g, links, partials, out, sdens, qdens, st);
}

// <a b> / sqrt(<a^2> <b^2>) with Neumaier sums: one block, a fixed stride per
// thread and a fixed-order tree, so the result does not depend on scheduling.
__device__ __forceinline__ void nsum(double& s, double& c, double v) {
  const double t = s + v;
  if (fabs(s) >= fabs(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

__global__ void __launch_bounds__(1024) k_correlate(long long n, const double* __restrict__ a,
                                                    const double* __restrict__ b, double* out) {
  double v[6] = {0, 0, 0, 0, 0, 0};  // ab, aa, bb sums and compensations
  for (long long i = threadIdx.x; i < n; i += blockDim.x) {
    const double x = a[i], y = b[i];
    nsum(v[0], v[1], x * y);
    nsum(v[2], v[3], x * x);
    nsum(v[4], v[5], y * y);
  }
  __shared__ double sh[6][1024];
#pragma unroll
  for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int stride = 512; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) {
#pragma unroll
      for (int k = 0; k < 6; k += 2) {
        double s = sh[k][threadIdx.x], c = sh[k + 1][threadIdx.x];
        nsum(s, c, sh[k][threadIdx.x + stride]);
        c += sh[k + 1][threadIdx.x + stride];
        sh[k][threadIdx.x] = s;
        sh[k + 1][threadIdx.x] = c;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ab = sh[0][0] + sh[1][0], aa = sh[2][0] + sh[3][0], bb = sh[4][0] + sh[5][0];
    out[0] = ab / sqrt(aa * bb);
    out[1] = ab;
    out[2] = aa;
    out[3] = bb;
  }
}

void launch_correlate(long long n, const double* a, const double* b, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_correlate, dim3(1), dim3(1024), 0, st, n, a, b, out);
}

// Block partials written by the measurement kernel: 10 eight-byte fields.
uint32_t measure_blocks(const Geo& g) { return (g.V + 255u) / 256u; }
size_t partial_bytes() { return 80; }

void launch_measure(int prec, const Geo& g, const void* links, const int8_t* z3, const void* gauge,
                    void* partials, int8_t* flux, unsigned long long* rej, VsmStatsDev* out, long long sweep,
                    hipStream_t st) {
  if (prec == 0) launch_measure_t<double>(g, links, z3, gauge, partials, flux, rej, out, sweep, st);
  else launch_measure_t<float>(g, links, z3, gauge, partials, flux, rej, out, sweep, st);
}

}  // namespace vsm
