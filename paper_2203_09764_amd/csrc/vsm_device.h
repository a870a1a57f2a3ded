// vsm_device.h -- device-side building blocks of the smoothing kernels (gfx950).
//
//  * 3x3 complex matrices in registers, templated on the storage/arithmetic type
//    R (double for the FP64 form, float for the FP32-bulk form);
//  * the internal link layout and its buffer-resource loads;
//  * the Cayley-Hamilton exponential (Morningstar & Peardon, Phys. Rev. D 69,
//    054501 (2004), the stout reference of Sec. II.A) with FP64 coefficients;
//  * reunitarisation and the Z(3) sector test of Eq. (centre_element).
//
// Internal layout.  The lattice axes are relabelled so that internal axis 0 is
// the longest one; every extent is a multiple of 4.  A site with internal
// coordinates (c0, c1, c2, c3) has the sublattice s = (c0 + c1 + c2 + c3) mod 4
// and the position j = (c0 >> 2) + Xq * (c1 + L1 * (c2 + L2 * c3)), Xq = L0 / 4,
// and lives at idx = s * V/4 + j.  The links of one annealing subset of a
// direction mu != 0 then fill long contiguous runs of j (the subset is
// s = (colour - c_mu) mod 4), and so does every neighbour of them.
// Links are SU(3), so only rows 0 and 1 are stored; row 2 is rebuilt on load as
// conj(row0 x row1).  The six stored entries (e = 3 * row + column, rows 0
// and 1) go into 16-byte words: one entry per word in FP64 ({re, im}), two in
// FP32 ({re, im} of entries 2w and 2w + 1).  Each direction owns one array of
// V words per word of a link (6 in FP64, 3 in FP32):
//   word w of link (mu, idx) lives at element (mu * W + w) * V + idx,
// so that a wave reads 64 consecutive idx of one word in one 1 KiB request,
// 16 bytes per lane, in either form.  A link costs 96 B (FP64) or 48 B (FP32).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace vsm {

constexpr int kUndef = -128;
// 16-byte words per stored link (rows 0 and 1): 6 in FP64, 3 in FP32.
template <typename R>
constexpr uint32_t kLinkWords = (uint32_t)(12 * sizeof(R) / 16);
// Gap after each word array, in words.  Without it, at extents such as
// 48^3 x 96 the arrays start 2^21-byte multiples apart, and a wave's six word
// loads of one link fall on the same L2 channels; 64 words measured best.
constexpr uint32_t kEntryPad = 64;
constexpr uint32_t kRsrcWord3 = 0x00020000u;  // gfx9-family raw buffer descriptor

// ------------------------------------------------------------------ complex

template <typename R>
struct Cx {
  R re, im;
};

template <typename R>
struct M3 {
  Cx<R> a[9];
};

template <typename R>
__device__ __forceinline__ Cx<R> cx(R re, R im) {
  return Cx<R>{re, im};
}

// acc += x * y
template <typename R>
__device__ __forceinline__ void cfma(Cx<R>& acc, const Cx<R>& x, const Cx<R>& y) {
  acc.re = fma(x.re, y.re, acc.re);
  acc.re = fma(-x.im, y.im, acc.re);
  acc.im = fma(x.re, y.im, acc.im);
  acc.im = fma(x.im, y.re, acc.im);
}
// acc += x * conj(y)
template <typename R>
__device__ __forceinline__ void cfma_c2(Cx<R>& acc, const Cx<R>& x, const Cx<R>& y) {
  acc.re = fma(x.re, y.re, acc.re);
  acc.re = fma(x.im, y.im, acc.re);
  acc.im = fma(x.im, y.re, acc.im);
  acc.im = fma(-x.re, y.im, acc.im);
}
// acc += conj(x) * y
template <typename R>
__device__ __forceinline__ void cfma_c1(Cx<R>& acc, const Cx<R>& x, const Cx<R>& y) {
  acc.re = fma(x.re, y.re, acc.re);
  acc.re = fma(x.im, y.im, acc.re);
  acc.im = fma(x.re, y.im, acc.im);
  acc.im = fma(-x.im, y.re, acc.im);
}

// ------------------------------------------------------------------ 3x3 algebra

template <typename R>
__device__ __forceinline__ M3<R> mzero() {
  M3<R> r;
#pragma unroll
  for (int e = 0; e < 9; ++e) r.a[e] = cx<R>(R(0), R(0));
  return r;
}

// x * y
template <typename R>
__device__ __forceinline__ M3<R> mul_nn(const M3<R>& x, const M3<R>& y) {
  M3<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Cx<R> acc = cx<R>(R(0), R(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma(acc, x.a[3 * i + k], y.a[3 * k + j]);
      r.a[3 * i + j] = acc;
    }
  return r;
}

// x * y^dagger
template <typename R>
__device__ __forceinline__ M3<R> mul_nd(const M3<R>& x, const M3<R>& y) {
  M3<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Cx<R> acc = cx<R>(R(0), R(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma_c2(acc, x.a[3 * i + k], y.a[3 * j + k]);
      r.a[3 * i + j] = acc;
    }
  return r;
}

// x^dagger * y
template <typename R>
__device__ __forceinline__ M3<R> mul_dn(const M3<R>& x, const M3<R>& y) {
  M3<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Cx<R> acc = cx<R>(R(0), R(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma_c1(acc, x.a[3 * k + i], y.a[3 * k + j]);
      r.a[3 * i + j] = acc;
    }
  return r;
}

// Rows 0 and 1 of x * y, x * y^dagger, x^dagger * y (row 2 of the result is
// left unset).  For SU(3) operands the product is SU(3), so row 2 can be rebuilt
// afterwards with rebuild_row2 at a third of the cost of computing it.
template <typename R>
__device__ __forceinline__ M3<R> mul2_nn(const M3<R>& x, const M3<R>& y) {
  M3<R> r;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Cx<R> acc = cx<R>(R(0), R(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma(acc, x.a[3 * i + k], y.a[3 * k + j]);
      r.a[3 * i + j] = acc;
    }
  return r;
}

template <typename R>
__device__ __forceinline__ M3<R> mul2_nd(const M3<R>& x, const M3<R>& y) {
  M3<R> r;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Cx<R> acc = cx<R>(R(0), R(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma_c2(acc, x.a[3 * i + k], y.a[3 * j + k]);
      r.a[3 * i + j] = acc;
    }
  return r;
}

template <typename R>
__device__ __forceinline__ M3<R> mul2_dn(const M3<R>& x, const M3<R>& y) {
  M3<R> r;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Cx<R> acc = cx<R>(R(0), R(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma_c1(acc, x.a[3 * k + i], y.a[3 * k + j]);
      r.a[3 * i + j] = acc;
    }
  return r;
}

// Rows 0 and 1 of x^dagger y^dagger = (y x)^dagger.
template <typename R>
__device__ __forceinline__ M3<R> mul2_dd(const M3<R>& x, const M3<R>& y) {
  M3<R> r;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      // (x^dag y^dag)_ij = conj((y x)_ji) = conj(sum_k y_jk x_ki)
      Cx<R> acc = cx<R>(R(0), R(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma(acc, y.a[3 * j + k], x.a[3 * k + i]);
      r.a[3 * i + j] = cx<R>(acc.re, -acc.im);
    }
  return r;
}

// acc += c * x (real c)
template <typename R>
__device__ __forceinline__ void maxpy(M3<R>& acc, R c, const M3<R>& x) {
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    acc.a[e].re = fma(c, x.a[e].re, acc.a[e].re);
    acc.a[e].im = fma(c, x.a[e].im, acc.a[e].im);
  }
}

template <typename R>
__device__ __forceinline__ M3<R> madj(const M3<R>& x) {
  M3<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[3 * i + j] = cx<R>(x.a[3 * j + i].re, -x.a[3 * j + i].im);
  return r;
}

template <typename R>
__device__ __forceinline__ Cx<R> mtrace(const M3<R>& x) {
  return cx<R>(x.a[0].re + x.a[4].re + x.a[8].re, x.a[0].im + x.a[4].im + x.a[8].im);
}

template <typename D, typename S>
__device__ __forceinline__ M3<D> mconvert(const M3<S>& x) {
  M3<D> r;
#pragma unroll
  for (int e = 0; e < 9; ++e) r.a[e] = cx<D>(D(x.a[e].re), D(x.a[e].im));
  return r;
}

// ------------------------------------------------------------------ geometry

struct Geo {
  int L[4];        // internal extents; axis 0 is blocked by 4 and fastest in memory
  int Xq;          // L[0] / 4
  uint32_t V;      // sites
  uint32_t V4;     // V / 4
  uint32_t jst[4]; // j stride of internal axes 1..3 (jst[0] unused)
  uint32_t cst[4]; // canonical-index stride of internal axis d
  int perm[4];     // internal axis of user axis mu
  int uperm[4];    // user axis of internal axis d
  int T1, T2, T3;  // traversal tiles: rows of axis 1 (T1) with rows of axis 2 (T2) or axis 3 (T3)
  uint32_t es;     // entries from one entry array of a direction to the next: V + kEntryPad
};

// Axes 1..3 of the r-th row (x1, x2, x3) in traversal order (a row is the
// run of x0 positions one j-range covers).  The lattice is cut into tiles of
// T1 rows of axis 1 by T2 rows of axis 2, and each tile is swept through the
// whole of axis 3 before the next (SW = 3), so that the neighbours along the
// tile axes and the sweep axis of what a pass is updating were read a short
// time before.  With SW = 2 the roles of axes 2 and 3 swap (tiles T1 x T3,
// swept along axis 2): a pass of direction 3 reaches further along its own
// axis, which is then a tile axis.  With half = 1 the row index counts axis-1
// pairs (x1 = 2 y + p): the caller passes y back in c[1].
template <int SW = 3>
__device__ __forceinline__ void tile_rows(const Geo& g, uint32_t r, int c[4], int half) {
  constexpr int B = SW == 3 ? 2 : 3;
  const uint32_t L1 = (uint32_t)(g.L[1] >> half), T1 = (uint32_t)(g.T1 >> half);
  const uint32_t T2 = (uint32_t)(SW == 3 ? g.T2 : g.T3), LS = (uint32_t)g.L[SW];
  const uint32_t inner = T1 * T2 * LS;
  const uint32_t tile = r / inner;
  uint32_t q = r - tile * inner;
  const uint32_t a = q % T1;
  q /= T1;
  const uint32_t b = q % T2;
  const uint32_t xs = q / T2;
  const uint32_t n1 = L1 / T1;
  const uint32_t t2 = tile / n1;
  const uint32_t t1 = tile - t2 * n1;
  c[1] = (int)(t1 * T1 + a);
  c[B] = (int)(t2 * T2 + b);
  c[SW] = (int)xs;
}

__device__ __forceinline__ uint32_t site_index(const Geo& g, const int c[4]) {
  const uint32_t s = (uint32_t)(c[0] + c[1] + c[2] + c[3]) & 3u;
  const uint32_t j = (uint32_t)(c[0] >> 2) + (uint32_t)c[1] * g.jst[1] + (uint32_t)c[2] * g.jst[2] +
                     (uint32_t)c[3] * g.jst[3];
  return s * g.V4 + j;
}

__device__ __forceinline__ void coords_of_index(const Geo& g, uint32_t idx, int c[4]) {
  const uint32_t s = idx / g.V4;
  const uint32_t j = idx - s * g.V4;
  const uint32_t xi = j % (uint32_t)g.Xq;
  uint32_t r = j / (uint32_t)g.Xq;
  c[1] = (int)(r % (uint32_t)g.L[1]);
  r /= (uint32_t)g.L[1];
  c[2] = (int)(r % (uint32_t)g.L[2]);
  c[3] = (int)(r / (uint32_t)g.L[2]);
  c[0] = (int)(4 * xi) + (int)((s - (uint32_t)(c[1] + c[2] + c[3])) & 3u);
}

// Canonical site index s = x + Lx (y + Ly (z + Lz t)) of internal coordinates.
__device__ __forceinline__ uint32_t canonical_index(const Geo& g, const int c[4]) {
  return (uint32_t)c[0] * g.cst[0] + (uint32_t)c[1] * g.cst[1] + (uint32_t)c[2] * g.cst[2] +
         (uint32_t)c[3] * g.cst[3];
}

__device__ __forceinline__ int pick4(const int v[4], int i) {
  return i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
}

// Internal coordinates of canonical site s.
__device__ __forceinline__ void coords_of_canonical(const Geo& g, uint32_t s, int c[4]) {
  int u[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t Lu = (uint32_t)g.L[g.perm[k]];
    u[k] = (int)(s % Lu);
    s /= Lu;
  }
#pragma unroll
  for (int d = 0; d < 4; ++d) c[d] = pick4(u, g.uperm[d]);
}

__device__ __forceinline__ int wrap_add(int v, int k, int L) {
  int w = v + k;
  if (w < 0) w += L;
  if (w >= L) w -= L;
  return w;
}

// Change of j for a step of k (|k| <= 2) along internal axis d from coordinate v.
// The sublattice of the neighbour is (s + k) mod 4: wraps move by L = 0 mod 4.
__device__ __forceinline__ int jdelta(const Geo& g, int d, int v, int k) {
  const int w = wrap_add(v, k, g.L[d]);
  return d == 0 ? (w >> 2) - (v >> 2) : (w - v) * (int)g.jst[d];
}

// ------------------------------------------------------------------ link access

// One direction's word arrays as a raw buffer resource: voffset = idx * 16 in
// a VGPR, soffset = w * es * 16 in an SGPR.
template <typename R>
struct DirBuf {
  __amdgpu_buffer_rsrc_t rs;
  uint32_t estride;  // bytes between word arrays = es * 16
};

template <typename R>
__device__ __forceinline__ DirBuf<R> dir_buf(const void* links, const Geo& g, int mu) {
  const uint32_t es = g.es * 16u;
  const char* base = (const char*)links + (size_t)mu * kLinkWords<R> * (size_t)es;
  DirBuf<R> b;
  b.rs = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(kLinkWords<R> * es),
                                           (int)kRsrcWord3);
  b.estride = es;
  return b;
}

// Rows 0 and 1 of the link at voffset voff into m.a[0..5].
__device__ __forceinline__ void ld_words(const DirBuf<double>& b, uint32_t voff, M3<double>& m) {
#pragma unroll
  for (int w = 0; w < 6; ++w) {
    auto v = __builtin_amdgcn_raw_buffer_load_b128(b.rs, voff, (int)(w * b.estride), 0);
    double2 d;
    __builtin_memcpy(&d, &v, sizeof d);
    m.a[w] = cx<double>(d.x, d.y);
  }
}

__device__ __forceinline__ void ld_words(const DirBuf<float>& b, uint32_t voff, M3<float>& m) {
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    auto v = __builtin_amdgcn_raw_buffer_load_b128(b.rs, voff, (int)(w * b.estride), 0);
    float4 d;
    __builtin_memcpy(&d, &v, sizeof d);
    m.a[2 * w] = cx<float>(d.x, d.y);
    m.a[2 * w + 1] = cx<float>(d.z, d.w);
  }
}

// Row 2 of an SU(3) matrix from rows 0 and 1: r2 = conj(r0 x r1).
template <typename R>
__device__ __forceinline__ void rebuild_row2(M3<R>& m) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
    const Cx<R>& a1 = m.a[k1];
    const Cx<R>& a2 = m.a[k2];
    const Cx<R>& b1 = m.a[3 + k1];
    const Cx<R>& b2 = m.a[3 + k2];
    R re = a1.re * b2.re;
    re = fma(-a1.im, b2.im, re);
    re = fma(-a2.re, b1.re, re);
    re = fma(a2.im, b1.im, re);
    R im = a1.re * b2.im;
    im = fma(a1.im, b2.re, im);
    im = fma(-a2.re, b1.im, im);
    im = fma(-a2.im, b1.re, im);
    m.a[6 + k] = cx<R>(re, -im);
  }
}

template <typename R>
__device__ __forceinline__ M3<R> ld_link(const DirBuf<R>& b, uint32_t idx) {
  M3<R> m;
  ld_words(b, idx * 16u, m);
  rebuild_row2(m);
  return m;
}

// Rows 0 and 1 of a stored link as they are in memory (row 2 left zero and
// never read): a link held across several uses costs two thirds of the
// registers; full() rebuilds row 2 where a product needs it.
template <typename R>
__device__ __forceinline__ M3<R> ld_rows(const DirBuf<R>& b, uint32_t idx) {
  M3<R> m;
  ld_words(b, idx * 16u, m);
#pragma unroll
  for (int e = 6; e < 9; ++e) m.a[e] = cx<R>(R(0), R(0));
  return m;
}

// Keeps the compiler from treating two rebuilds of the same rows as one value
// (which would hold the rebuilt row live between the uses).
__device__ __forceinline__ void opaque(double& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void opaque(float& v) { asm volatile("" : "+v"(v)); }

template <typename R>
__device__ __forceinline__ M3<R> full(const M3<R>& m) {
  M3<R> f;
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    f.a[e] = m.a[e];
    opaque(f.a[e].re);
    opaque(f.a[e].im);
  }
  rebuild_row2(f);
  return f;
}

__device__ __forceinline__ void st_words(double2* p, size_t es, const M3<double>& m) {
#pragma unroll
  for (int w = 0; w < 6; ++w) p[(size_t)w * es] = make_double2(m.a[w].re, m.a[w].im);
}

__device__ __forceinline__ void st_words(float4* p, size_t es, const M3<float>& m) {
#pragma unroll
  for (int w = 0; w < 3; ++w)
    p[(size_t)w * es] = make_float4(m.a[2 * w].re, m.a[2 * w].im, m.a[2 * w + 1].re, m.a[2 * w + 1].im);
}

template <typename R>
__device__ __forceinline__ void st_link(void* links, const Geo& g, int mu, uint32_t idx, const M3<R>& m) {
  using W = typename std::conditional<sizeof(R) == 8, double2, float4>::type;
  W* p = (W*)links + (size_t)mu * kLinkWords<R> * g.es + idx;
  st_words(p, g.es, m);
}

// ------------------------------------------------------------------ centre sector

// Eq. (centre_element) written without arg(): for t = a + i b,
//   n = 0  iff a > 0 and b^2 < 3 a^2          (|arg t| < pi/3)
//   n = +1 iff b > 0 and (a <= 0 or b^2 > 3 a^2)  (arg t in (pi/3, pi))
//   n = -1 iff b < 0 and (a <= 0 or b^2 > 3 a^2)  (arg t in (-pi, -pi/3))
// and undefined on the boundaries and at t = 0.
__device__ __forceinline__ int z3_sector(double a, double b) {
  if (!(isfinite(a) && isfinite(b))) return kUndef;
  const double a3 = 3.0 * a * a, b2 = b * b;
  if (a > 0.0 && b2 < a3) return 0;
  const bool outside = (a <= 0.0) || (b2 > a3);
  if (b > 0.0 && outside) return 1;
  if (b < 0.0 && outside) return -1;
  return kUndef;
}

// The Z(3) element e^{2 pi i n/3} with the exact real part -1/2 for n = +-1.
__device__ __forceinline__ Cx<double> z3_elem(int n) {
  const double s = 0.86602540378443864676;  // sqrt(3)/2
  if (n == 0) return cx<double>(1.0, 0.0);
  return cx<double>(-0.5, n > 0 ? s : -s);
}

// ------------------------------------------------------------------ exponential

// exp(X) for X traceless anti-Hermitian, as exp(iH) = f0 + f1 H + f2 H^2 with
// H = -i X Hermitian traceless, c0 = det H, c1 = Tr H^2 / 2 (Cayley-Hamilton:
// H^3 = c1 H + c0).  Coefficients f_j in FP64:
//  * c1 < 0.5 (all eigenvalues below 0.82 in size): the Taylor series of
//    exp(iH) reduced with H^3 = c1 H + c0, summed to order 20 (remainder below
//    1e-19) -- no cancellation as c1 -> 0, where the closed form is 0/0;
//  * otherwise the closed form of Morningstar & Peardon with theta, u, w and the
//    symmetry f_j(-c0) = (-1)^j conj f_j(c0).
struct CHCoef {
  Cx<double> f0, f1, f2;
};

__device__ __forceinline__ CHCoef ch_coefficients(double c0, double c1) {
  CHCoef r;
  if (c1 < 0.5) {
    // H^k = a_k + b_k H + c_k H^2; (a,b,c)_{k+1} = (c0 c_k, a_k + c1 c_k, b_k); with
    // the 1/k! folded in.  i^k cycles through 1, i, -1, -i.
    double a = 1.0, b = 0.0, c = 0.0;
    double f0r = 1.0, f0i = 0.0, f1r = 0.0, f1i = 0.0, f2r = 0.0, f2i = 0.0;
#pragma unroll
    for (int k = 1; k <= 20; ++k) {
      const double inv = 1.0 / (double)k;
      const double na = c0 * c * inv;
      const double nb = fma(c1, c, a) * inv;
      const double nc = b * inv;
      a = na;
      b = nb;
      c = nc;
      switch (k & 3) {
        case 0: f0r += a; f1r += b; f2r += c; break;
        case 1: f0i += a; f1i += b; f2i += c; break;
        case 2: f0r -= a; f1r -= b; f2r -= c; break;
        default: f0i -= a; f1i -= b; f2i -= c; break;
      }
    }
    r.f0 = cx<double>(f0r, f0i);
    r.f1 = cx<double>(f1r, f1i);
    r.f2 = cx<double>(f2r, f2i);
    return r;
  }
  const bool neg = c0 < 0.0;
  const double c0a = fabs(c0);
  const double c0max = 2.0 * c1 / 3.0 * sqrt(c1 / 3.0);
  double ratio = c0a / c0max;
  ratio = ratio > 1.0 ? 1.0 : ratio;
  const double theta = acos(ratio);
  const double u = sqrt(c1 / 3.0) * cos(theta / 3.0);
  const double w = sqrt(c1) * sin(theta / 3.0);
  const double u2 = u * u, w2 = w * w;
  double xi0;
  if (fabs(w) < 0.05)
    xi0 = 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0));
  else
    xi0 = sin(w) / w;
  const double cw = cos(w);
  double s2u, c2u, su, cu;
  sincos(2.0 * u, &s2u, &c2u);
  sincos(u, &su, &cu);
  // e^{-iu} * (p + i q)
  auto emiu = [&](double p, double q) { return cx<double>(cu * p + su * q, cu * q - su * p); };
  const Cx<double> t0 = emiu(8.0 * u2 * cw, 2.0 * u * (3.0 * u2 + w2) * xi0);
  const Cx<double> t1 = emiu(2.0 * u * cw, -(3.0 * u2 - w2) * xi0);
  const Cx<double> t2 = emiu(cw, 3.0 * u * xi0);
  const double den = 1.0 / (9.0 * u2 - w2);
  Cx<double> h0 = cx<double>((u2 - w2) * c2u + t0.re, (u2 - w2) * s2u + t0.im);
  Cx<double> h1 = cx<double>(2.0 * u * c2u - t1.re, 2.0 * u * s2u - t1.im);
  Cx<double> h2 = cx<double>(c2u - t2.re, s2u - t2.im);
  r.f0 = cx<double>(h0.re * den, h0.im * den);
  r.f1 = cx<double>(h1.re * den, h1.im * den);
  r.f2 = cx<double>(h2.re * den, h2.im * den);
  if (neg) {
    r.f0 = cx<double>(r.f0.re, -r.f0.im);
    r.f1 = cx<double>(-r.f1.re, r.f1.im);
    r.f2 = cx<double>(r.f2.re, -r.f2.im);
  }
  return r;
}

// H = -i X for X anti-Hermitian: H_ij = (Im X_ij, -Re X_ij).  Returns c0, c1 in FP64.
template <typename R>
__device__ __forceinline__ void ch_invariants(const M3<R>& h, double& c0, double& c1) {
  const double h00 = h.a[0].re, h11 = h.a[4].re, h22 = h.a[8].re;
  const double x01r = h.a[1].re, x01i = h.a[1].im;
  const double x02r = h.a[2].re, x02i = h.a[2].im;
  const double x12r = h.a[5].re, x12i = h.a[5].im;
  const double n01 = x01r * x01r + x01i * x01i;
  const double n02 = x02r * x02r + x02i * x02i;
  const double n12 = x12r * x12r + x12i * x12i;
  c1 = 0.5 * (h00 * h00 + h11 * h11 + h22 * h22) + n01 + n02 + n12;
  // det H = h00 h11 h22 + 2 Re(h01 h12 h20) - h00 |h12|^2 - h11 |h02|^2 - h22 |h01|^2
  // with h20 = conj(h02)
  const double pr = x01r * x12r - x01i * x12i;
  const double pi = x01r * x12i + x01i * x12r;
  const double re3 = pr * x02r + pi * x02i;
  c0 = h00 * h11 * h22 + 2.0 * re3 - h00 * n12 - h11 * n02 - h22 * n01;
}

// ------------------------------------------------------------------ reunitarise

// Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): the nearest SU(3)
// matrix to first order, exact structure for diagonal input.  FP64.
__device__ __forceinline__ void reunitarise(M3<double>& u) {
  double n0 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) n0 += u.a[k].re * u.a[k].re + u.a[k].im * u.a[k].im;
  const double i0 = 1.0 / sqrt(n0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    u.a[k].re *= i0;
    u.a[k].im *= i0;
  }
  Cx<double> ip = cx<double>(0.0, 0.0);  // <r0, r1> = sum conj(r0_k) r1_k
#pragma unroll
  for (int k = 0; k < 3; ++k) cfma_c1(ip, u.a[k], u.a[3 + k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    // r1 -= ip * r0
    u.a[3 + k].re -= ip.re * u.a[k].re - ip.im * u.a[k].im;
    u.a[3 + k].im -= ip.re * u.a[k].im + ip.im * u.a[k].re;
  }
  double n1 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) n1 += u.a[3 + k].re * u.a[3 + k].re + u.a[3 + k].im * u.a[3 + k].im;
  const double i1 = 1.0 / sqrt(n1);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    u.a[3 + k].re *= i1;
    u.a[3 + k].im *= i1;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
    // (r0 x r1)_k = r0_k1 r1_k2 - r0_k2 r1_k1 ; row 2 = conj of that
    const Cx<double>& a1 = u.a[k1];
    const Cx<double>& a2 = u.a[k2];
    const Cx<double>& b1 = u.a[3 + k1];
    const Cx<double>& b2 = u.a[3 + k2];
    const double re = (a1.re * b2.re - a1.im * b2.im) - (a2.re * b1.re - a2.im * b1.im);
    const double im = (a1.re * b2.im + a1.im * b2.re) - (a2.re * b1.im + a2.im * b1.re);
    u.a[6 + k] = cx<double>(re, -im);
  }
}

}  // namespace vsm
