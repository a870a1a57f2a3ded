// vsm_kernels_impl.h -- HIP kernels of the vortex-field smoothing path (gfx950).
// Included once per precision by vsm_k_f64.hip and vsm_k_f32.hip.
//
// Kernels (all launched by vsm_api.hip on the caller's stream):
//   k_set_links / k_get_links : canonical complex128 [4][V][3][3] <-> internal layout
//   k_load_z3                 : Z(3) charges -> centre-element links (Eq. centre_project)
//   k_centrifuge              : centrifuge preconditioning (Sec. IV)
//   k_gauge                   : U -> G(x) U G^dagger(x + mu) (Sec. V.C)
//   k_update<R, MU, OI, UPD>  : one annealing subset or one smearing step of
//                               stout (Eq. stout), MaxReTr (Sec. III) or APE with
//                               unit circle projection (Sec. III) updates, with the
//                               vortex-preserving test (Sec. VI)
//   k_update_batch            : one serving step: a subset pass of every resident job
//   k_flow                    : one Euler or Runge-Kutta stage of the Wilson flow (Sec. II.B)
//   k_measure / k_finalize    : plaquette, Wilson action, vortex flux (Sec. I, V.A)
//   k_clover / k_clover_finalize : clover F, reconstructed action, topological charge (Sec. V)
//
// Site orders: subset passes take their sites by subset_site (rows in tiles,
// swept along an axis other than the pass direction); kernels that visit every
// site take them by chunk_site (one sublattice per wave, four per block).  Both
// hand blocks to the XCDs in contiguous ranges (xcd_block).
#pragma once

#include "vsm_device.h"
#include "vsm_launch.h"

namespace vsm {

// ------------------------------------------------------------------ layout

// Threads run over (user direction mu, canonical site s); the link goes to
// internal direction perm[mu] at site_index(c).
template <typename R>
__global__ void k_set_links(Geo g, const double2* __restrict__ canon, void* links) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 4u * g.V) return;
  const int mu = (int)(tid / g.V);
  const uint32_t s = tid - (uint32_t)mu * g.V;
  int c[4];
  coords_of_canonical(g, s, c);
  const double2* src = canon + ((size_t)mu * g.V + s) * 9;
  M3<R> m;
#pragma unroll
  for (int e = 0; e < 9; ++e) m.a[e] = cx<R>((R)src[e].x, (R)src[e].y);
  st_link<R>(links, g, g.perm[mu], site_index(g, c), m);
}

template <typename R>
__global__ void k_get_links(Geo g, const void* links, double2* __restrict__ canon) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 4u * g.V) return;
  const int mu = (int)(tid / g.V);
  const uint32_t s = tid - (uint32_t)mu * g.V;
  int c[4];
  coords_of_canonical(g, s, c);
  const M3<R> m = ld_link<R>(dir_buf<R>(links, g, g.perm[mu]), site_index(g, c));
  double2* dst = canon + ((size_t)mu * g.V + s) * 9;
#pragma unroll
  for (int e = 0; e < 9; ++e) dst[e] = make_double2((double)m.a[e].re, (double)m.a[e].im);
}

// ------------------------------------------------------------------ ingest

template <typename R>
__global__ void k_load_z3(Geo g, const int8_t* __restrict__ z3, void* links) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 4u * g.V) return;
  const int mu = (int)(tid / g.V);
  const uint32_t s = tid - (uint32_t)mu * g.V;
  int c[4];
  coords_of_canonical(g, s, c);
  const Cx<double> z = z3_elem(z3[tid]);
  M3<R> m = mzero<R>();
  m.a[0] = m.a[4] = m.a[8] = cx<R>((R)z.re, (R)z.im);
  st_link<R>(links, g, g.perm[mu], site_index(g, c), m);
}

// ------------------------------------------------------------------ centrifuge

// Sec. IV: with lambda = 2 pi n/3 and the staple phase sigma = 2 pi m/18,
//   lambda^j = lambda + omega (sigma - lambda),  lambda^k = lambda - omega (sigma - lambda),
// i.e. e^{i lambda^j} = z(n) e^{+i d}, e^{i lambda^k} = z(n) e^{-i d} with
// d = omega (2 pi / 18) (m - 6 n), and the third phase stays lambda.  m is the
// exact integer sum of the 18 neighbouring charges of the six staples.  Threads
// run over the internal layout (internal direction dmu, link index idx), so that
// a wave's link stores are contiguous; the charges, the pair and m are read and
// written in the canonical order of user direction mu and site s.
template <typename R>
__global__ void k_centrifuge(Geo g, const int8_t* __restrict__ z3, const int8_t* __restrict__ pair,
                             double omega, void* links, int32_t* __restrict__ m_out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 4u * g.V) return;
  const int dmu = (int)(tid / g.V);
  const uint32_t idx = tid - (uint32_t)dmu * g.V;
  int c[4];
  coords_of_index(g, idx, c);
  const int mu = g.uperm[dmu];
  const uint32_t s = canonical_index(g, c);
  const uint32_t lk = (uint32_t)mu * g.V + s;  // the link in canonical order
  // charge of user direction d at the site shifted by (i along mu, k along nu)
  auto nat = [&](int d, int i, int k, int dnu) -> int {
    int e[4] = {c[0], c[1], c[2], c[3]};
    e[dmu] = wrap_add(e[dmu], i, g.L[dmu]);
    e[dnu] = wrap_add(e[dnu], k, g.L[dnu]);
    return (int)z3[(size_t)d * g.V + canonical_index(g, e)];
  };
  int m = 0;
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    const int dnu = g.perm[nu];
    m += nat(nu, 0, 0, dnu) + nat(mu, 0, 1, dnu) - nat(nu, 1, 0, dnu);     // upper staple
    m += -nat(nu, 0, -1, dnu) + nat(mu, 0, -1, dnu) + nat(nu, 1, -1, dnu);  // lower staple
  }
  const int n = z3[lk];
  const double d = omega * (2.0 * 3.14159265358979323846 / 18.0) * (double)(m - 6 * n);
  double sd, cd;
  sincos(d, &sd, &cd);
  const Cx<double> z = z3_elem(n);
  const Cx<double> zp = cx<double>(z.re * cd - z.im * sd, z.re * sd + z.im * cd);
  const Cx<double> zm = cx<double>(z.re * cd + z.im * sd, z.im * cd - z.re * sd);
  const int j = pair[lk];
  const int k = (j + 1) % 3;
  M3<R> u = mzero<R>();
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const Cx<double> v = (i == j) ? zp : ((i == k) ? zm : z);
    u.a[4 * i] = cx<R>((R)v.re, (R)v.im);
  }
  st_link<R>(links, g, dmu, idx, u);
  if (m_out) m_out[lk] = m;
}

// ------------------------------------------------------------------ gauge transform

// U_mu(x) -> G(x) U_mu(x) G^dagger(x + mu); threads over (internal direction, idx).
template <typename R>
__global__ void k_gauge(Geo g, void* links, const double2* __restrict__ gauge) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 4u * g.V) return;
  const int d = (int)(tid / g.V);
  const uint32_t idx = tid - (uint32_t)d * g.V;
  int c[4];
  coords_of_index(g, idx, c);
  const uint32_t s = canonical_index(g, c);
  int cp[4] = {c[0], c[1], c[2], c[3]};
  cp[d] = wrap_add(cp[d], 1, g.L[d]);
  const uint32_t sp = canonical_index(g, cp);
  M3<double> G, Gp;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    G.a[e] = cx<double>(gauge[(size_t)s * 9 + e].x, gauge[(size_t)s * 9 + e].y);
    Gp.a[e] = cx<double>(gauge[(size_t)sp * 9 + e].x, gauge[(size_t)sp * 9 + e].y);
  }
  const M3<double> u = mconvert<double>(ld_link<R>(dir_buf<R>(links, g, d), idx));
  const M3<double> r = mul_nd(mul_nn(G, u), Gp);
  st_link<R>(links, g, d, idx, mconvert<R>(r));
}

// ------------------------------------------------------------------ staples

// Staple paths as chains of link products (Eq. plaq_staples and the
// over-improvement diagrams).  Links are loaded as rows 0 and 1 and completed
// (row 2 rebuilt) where a product needs them; running products keep only rows
// 0 and 1 too (a product of SU(3) links), and chain_add rebuilds row 2 before a
// path is added to Sigma.  The compiler-only memory fence after a group of
// loads fixes how far ahead of their use loads are issued: without it the
// compiler hoists every load of the staple and spills.
__device__ __forceinline__ void load_fence() { asm volatile("" ::: "memory"); }

template <typename R>
__device__ __forceinline__ void chain_add(M3<R>& S, R c, M3<R> w) {
  rebuild_row2(w);
  maxpy(S, c, w);
}

// Neighbours of the thread's site x: x + a mu + b nu has sublattice
// (S + a + b) mod 4 and position j + dm[a + 1] + dn[b + 2].
struct Nb {
  uint32_t j;
  int S;
  int dm[4];  // a = -1, 0, 1, 2
  int dn[5];  // b = -2 .. 2
};

__device__ __forceinline__ uint32_t nbi(const Geo& g, const Nb& o, int a, int b) {
  return (uint32_t)((o.S + a + b) & 3) * g.V4 + (uint32_t)((int)o.j + o.dm[a + 1] + o.dn[b + 2]);
}

// The staple paths of one nu and one orientation, from x to x + mu
// (a step -d multiplies the adjoint of the link it walks back along):
//   +nu: plaquette  +nu +mu -nu          : U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
//        1x2        +nu +nu +mu -nu -nu  : U_nu(x) U_nu(x+nu) U_mu(x+2nu) U_nu(x+mu+nu)^dag U_nu(x+mu)^dag
//        2x1 left   +nu +mu +mu -nu -mu  : U_nu(x) U_mu(x+nu) U_mu(x+mu+nu) U_nu(x+2mu)^dag U_mu(x+mu)^dag
//        2x1 middle -mu +nu +mu +mu -nu  : U_mu(x-mu)^dag U_nu(x-mu) U_mu(x-mu+nu) U_mu(x+nu) U_nu(x+mu)^dag
//   -nu: the same paths with nu reversed.
// Weights: (5 - 2 eps)/3 for the plaquette staple, (eps - 1)/(12 u0^2) for rectangles.
//
// The order in which an orientation's ten distinct links are loaded, as
// (direction mu?, a, b for +nu, b for -nu) in x + a mu + b nu:
//   D = U_nu(x+nu)  E = U_mu(x+2nu)  F = U_nu(x+mu+nu)  B = U_mu(x+nu)  A = U_nu(x)
//   H = U_nu(x+2mu)  N = U_mu(x-mu+nu)  G = U_mu(x+mu+nu)  M = U_nu(x-mu)  C = U_nu(x+mu)
// (for -nu, the b of take_bd: the same paths with nu reversed).  The update
// of x + 2mu, in the same subset and two rows of the traversal away, needs
// x's H, G, C as its A, N, M: loading each such pair back to back lets the
// two updates' requests for the same line meet in the L2.  A model of one
// XCD's L2 replaying the loads of the blocks in flight puts this order 13-17%
// below the order of first use in fetched lines; measured on 48^3x96 in FP64,
// a pass fetches 8% less (10.9 to 10.1 GB).
__host__ __device__ constexpr bool take_mu(int k) {
  constexpr bool t[10] = {false, true, false, true, false, false, true, true, false, false};
  return t[k];
}
__host__ __device__ constexpr int take_a(int k) {
  constexpr int t[10] = {0, 0, 1, 0, 0, 2, -1, 1, -1, 1};
  return t[k];
}
__host__ __device__ constexpr int take_bu(int k) {
  constexpr int t[10] = {1, 2, 1, 1, 0, 0, 1, 1, 0, 0};
  return t[k];
}
__host__ __device__ constexpr int take_bd(int k) {
  constexpr int t[10] = {-2, -2, -2, -1, -1, -1, -1, -1, -1, -1};
  return t[k];
}

template <int K>
struct Take {
  static constexpr int value = K;
};

// S += x y^dagger (DAG) or S += x y, with all three rows of x.
template <typename R, bool DAG>
__device__ __forceinline__ void madd_prod(M3<R>& S, const M3<R>& x, const M3<R>& y) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (DAG)
          cfma_c2(S.a[3 * i + j], x.a[3 * i + k], y.a[3 * j + k]);
        else
          cfma(S.a[3 * i + j], x.a[3 * i + k], y.a[3 * k + j]);
      }
}

// The four paths of one orientation, added to S with every distinct link
// loaded once (10 loads instead of 18) and the links shared by several paths
// multiplied once:
//   - the plaquette, the 1x2 and the 2x1 middle path all end in the step back
//     along nu at x + mu (C^dag for +nu, C for -nu), so they are summed first,
//       Z = cp A B + cr A (D E F^dag) + cr L^dag M (N B),   S += Z C^dag;
//   - the plaquette's A B starts the 2x1 left path, A B G (H^dag K^dag).
// (For -nu: A, D, F, H, M walked backwards.)  Every factor is formed as soon
// as the load order above has delivered its links, so that few are held:
// ten 2-row products and one 3-row product, against thirteen 2-row products
// path by path.  Each path and partial product is a product of SU(3) links, so
// its row 2 is rebuilt from rows 0 and 1 where it is needed.  get(Take<k>())
// returns rows 0 and 1 of link k of the load order; K = U_mu(x+mu) and
// L = U_mu(x-mu) (rows 0 and 1) are common to all nu.  The FP64 form's route.
template <typename R, bool UP, typename Get>
__device__ __forceinline__ void orient_paths(M3<R>& S, R cp, R cr, const M3<R>& K, const M3<R>& L, Get&& get) {
  // 1x2: P = D E F^dag (+nu), D^dag E F (-nu)
  const M3<R> D = get(Take<0>());
  const M3<R> E = get(Take<1>());
  M3<R> P = UP ? mul2_nn(D, full(E)) : mul2_dn(full(D), full(E));
  const M3<R> F = get(Take<2>());
  P = UP ? mul2_nd(P, full(F)) : mul2_nn(P, full(F));
  const M3<R> Bf = full(get(Take<3>()));
  const M3<R> A = get(Take<4>());
  M3<R> Af;
  if (!UP) Af = full(A);
  // the plaquette's T = A B and the 1x2 path A P open the sum Z
  M3<R> T = UP ? mul2_nn(A, Bf) : mul2_dn(Af, Bf);
  rebuild_row2(T);
  M3<R> w = UP ? mul2_nn(A, full(P)) : mul2_dn(Af, full(P));
  rebuild_row2(w);
  M3<R> Z;
#pragma unroll
  for (int e = 0; e < 9; ++e) Z.a[e] = cx<R>(cr * w.a[e].re, cr * w.a[e].im);
  maxpy(Z, cp, T);
  // 2x1 left: T G Q with Q = H^dag K^dag (+nu), H K^dag (-nu)
  const M3<R> H = get(Take<5>());
  const M3<R> Q = UP ? mul2_dd(full(H), full(K)) : mul2_nd(H, full(K));
  // 2x1 middle: N B, formed now so that B need not be held further
  const M3<R> NB = mul2_nn(get(Take<6>()), Bf);
  const M3<R> G = get(Take<7>());
  w = mul2_nn(T, full(G));
  w = mul2_nn(w, full(Q));
  chain_add(S, cr, w);
  const M3<R> M = get(Take<8>());
  w = UP ? mul2_dn(full(L), full(M)) : mul2_dd(full(L), full(M));
  w = mul2_nn(w, full(NB));
  rebuild_row2(w);
  maxpy(Z, cr, w);
  madd_prod<R, UP>(S, Z, full(get(Take<9>())));
}

// orient_paths with ordinary loads into registers, each issued two links
// ahead of its use.
template <typename R, bool UP>
__device__ __forceinline__ void staple_dir_loads(M3<R>& S, const DirBuf<R>& bm, const DirBuf<R>& bn,
                                                 const Geo& g, const Nb& o, R cp, R cr, const M3<R>& K,
                                                 const M3<R>& L) {
  M3<R> q[3];
  auto ld = [&](int k) {
    return ld_rows(take_mu(k) ? bm : bn, nbi(g, o, take_a(k), UP ? take_bu(k) : take_bd(k)));
  };
  auto get = [&](auto pos) {
    constexpr int k = decltype(pos)::value;
    if constexpr (k == 0) {
      q[0] = ld(0);
      q[1] = ld(1);
      load_fence();
    }
    if constexpr (k + 2 < 10) {
      q[(k + 2) % 3] = ld(k + 2);
      load_fence();
    }
    return q[k % 3];
  };
  orient_paths<R, UP>(S, cp, cr, K, L, get);
}

// The FP32 form's staples: the grouping of orient_paths with the 2x1 left
// path multiplied out in full and the links loaded in the order of their
// first use (A D E F B G H M N C),
//   Z = cp A B + cr A D E F^dag + cr L^dag M N B,   S += Z C^dag + cr A B G H^dag K^dag
// (for -nu: A, D, F, H, M walked backwards): ten 2-row products and one 3-row
// product, and no partial product beyond the paths needs its row 2.  FP32's
// pass is bound by its arithmetic as much as by its reads.  orient_paths saves
// 4% of the FP32 reads but takes more instructions and 70 more registers, and
// measured 3% slower on 48^3x96; issuing this path's loads with the pairs of
// orient_paths' order together (A H D E F B N G M C) saved 3% of the reads at
// the same instruction count, and measured 5% slower on 32^3x64.
template <typename R, bool UP>
__device__ __forceinline__ void staple_dir_factored(M3<R>& S, const DirBuf<R>& bm, const DirBuf<R>& bn,
                                                    const Geo& g, const Nb& o, R cp, R cr,
                                                    const M3<R>& Kf, const M3<R>& Lf) {
  auto I = [&](int a, int b) { return nbi(g, o, a, b); };
  const int sg = UP ? 1 : -1;
  // 1x2: A D E F^dag
  const M3<R> Ar = ld_rows(bn, I(0, UP ? 0 : -1));
  const M3<R> Dr = ld_rows(bn, I(0, UP ? 1 : -2));
  const M3<R> Er = ld_rows(bm, I(0, 2 * sg));
  load_fence();
  const M3<R> Fr = ld_rows(bn, I(1, UP ? 1 : -2));
  load_fence();
  M3<R> Af;
  if (!UP) Af = full(Ar);
  M3<R> w = UP ? mul2_nn(Ar, full(Dr)) : mul2_dd(Af, full(Dr));
  const M3<R> Br = ld_rows(bm, I(0, sg));
  load_fence();
  w = mul2_nn(w, full(Er));
  const M3<R> Gr = ld_rows(bm, I(1, sg));
  load_fence();
  w = UP ? mul2_nd(w, full(Fr)) : mul2_nn(w, full(Fr));
  rebuild_row2(w);
  M3<R> Z;
#pragma unroll
  for (int e = 0; e < 9; ++e) Z.a[e] = cx<R>(cr * w.a[e].re, cr * w.a[e].im);
  // plaquette A B, and 2x1 left A B G H^dag K^dag, share T = A B
  const M3<R> Hr = ld_rows(bn, I(2, UP ? 0 : -1));
  load_fence();
  const M3<R> Bf = full(Br);
  M3<R> T = UP ? mul2_nn(Ar, Bf) : mul2_dn(Af, Bf);
  rebuild_row2(T);
  maxpy(Z, cp, T);
  const M3<R> Mr = ld_rows(bn, I(-1, UP ? 0 : -1));
  load_fence();
  T = mul2_nn(T, full(Gr));
  const M3<R> Nr = ld_rows(bm, I(-1, sg));
  load_fence();
  T = UP ? mul2_nd(T, full(Hr)) : mul2_nn(T, full(Hr));
  const M3<R> Cr = ld_rows(bn, I(1, UP ? 0 : -1));
  load_fence();
  chain_add(S, cr, mul2_nd(T, Kf));
  // 2x1 middle: L^dag M N B
  w = UP ? mul2_dn(Lf, full(Mr)) : mul2_dd(Lf, full(Mr));
  w = mul2_nn(w, full(Nr));
  w = mul2_nn(w, Bf);
  rebuild_row2(w);
  maxpy(Z, cr, w);
  madd_prod<R, UP>(S, Z, full(Cr));
}

// ------------------------------------------------------------------ LDS ring

// Over-improved staples with the link loads staged through LDS.  A buffer load
// with the lds flag writes each lane's bytes straight into LDS (at M0 + lane
// times the load size), so a link in flight holds no registers; the link is
// read back just before its first use, and each such use issues the load kRing
// links ahead into the slot it has just emptied.  The waits are explicit:
// vector memory loads complete in order, so when a link is taken at most the
// loads issued after it (kRing - 1 links) may still be in flight.  The links of
// one nu are taken in the load order of orient_paths (take_*), 20 per nu, a
// multiple of kRing, so that every take has a fixed slot.  After the last nu
// the own link U is issued once, at position 20, and the last takes wait for
// exactly the loads issued after them.
// FP64 only: an entry (16 B) is one dwordx4 load, and a wave's slot is 6 entries
// of 64 x 16 B.  (When FP32 links were stored one entry per 8-byte word, an
// FP32 ring took 12 loads per link and measured a third slower than FP32 loads
// into registers.  FP32 now stores 16-byte words as well, but it takes the
// staples of staple_dir_factored, whose fewer instructions and registers matter
// more to its pass than a deeper prefetch, and the serving kernels share that
// path with the single-field pass.)
constexpr int kRing = 5;
static_assert(20 % kRing == 0, "the 20 takes of one nu must fill whole turns of the ring");

template <typename R>
struct RingGeom;
template <>
struct RingGeom<double> {
  static constexpr uint32_t slot = 6u * 64u * 16u;  // one link of a wave
  static constexpr int loads = 6;                   // loads per link
};
template <typename R>
constexpr uint32_t kRingWave = (uint32_t)kRing * RingGeom<R>::slot;  // a wave's ring
template <typename R>
constexpr uint32_t kRingBytes = 4u * kRingWave<R>;  // a block of four waves: 120 KiB
static_assert(RingGeom<double>::loads * (kRing - 1) == 24, "a take waits for vmcnt(24)");

typedef __attribute__((address_space(3))) void lds_void_t;

// The loads of link idx of direction buffer b into the wave's slot at LDS byte
// offset slot (uniform over the wave).
__device__ __forceinline__ void ring_issue(const DirBuf<double>& b, uint32_t idx, uint32_t slot) {
  const uint32_t voff = idx * 16u;
#pragma unroll
  for (int e = 0; e < 6; ++e)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(b.rs, (lds_void_t*)(uintptr_t)(slot + (uint32_t)e * 1024u), 16,
                                             voff, (int)((uint32_t)e * b.estride), 0, 0);
}

// Waits until at most N vector loads are outstanding: those issued after the
// link about to be taken, which is then the oldest in flight and has landed.
template <int N>
__device__ __forceinline__ void ring_wait() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Rows 0 and 1 of the link in slot SLOT of the lane's ring, once ring_wait has
// seen it land.  The LDS reads wait for themselves in the same block.
// lane_ring: the LDS byte offset of the lane's first entry word in slot 0.
template <int SLOT>
__device__ __forceinline__ M3<double> ring_take(uint32_t lane_ring, double) {
  double2 v0, v1, v2, v3, v4, v5;
  asm volatile(
      "ds_read_b128 %0, %6 offset:%7\n\t"
      "ds_read_b128 %1, %6 offset:%8\n\t"
      "ds_read_b128 %2, %6 offset:%9\n\t"
      "ds_read_b128 %3, %6 offset:%10\n\t"
      "ds_read_b128 %4, %6 offset:%11\n\t"
      "ds_read_b128 %5, %6 offset:%12\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(v0), "=&v"(v1), "=&v"(v2), "=&v"(v3), "=&v"(v4), "=&v"(v5)
      : "v"(lane_ring), "n"(SLOT * 6144), "n"(SLOT * 6144 + 1024), "n"(SLOT * 6144 + 2048),
        "n"(SLOT * 6144 + 3072), "n"(SLOT * 6144 + 4096), "n"(SLOT * 6144 + 5120)
      : "memory");
  M3<double> m;
  m.a[0] = cx<double>(v0.x, v0.y);
  m.a[1] = cx<double>(v1.x, v1.y);
  m.a[2] = cx<double>(v2.x, v2.y);
  m.a[3] = cx<double>(v3.x, v3.y);
  m.a[4] = cx<double>(v4.x, v4.y);
  m.a[5] = cx<double>(v5.x, v5.y);
#pragma unroll
  for (int e = 6; e < 9; ++e) m.a[e] = cx<double>(0.0, 0.0);
  return m;
}

// orient_paths with the links taken from the ring in the load order; each
// take issues the load kRing links ahead into the slot it has just emptied
// (issue(q) loads the link of take position q: this nu 0-19, the next 20-24).
// After the last nu only the own link follows (position 20), so there the
// takes of positions 17-19 wait for the 3, 2, 1 links issued after them.
template <typename R, bool UP, bool LAST, typename Issue>
__device__ __forceinline__ void ring_orient(M3<R>& S, R cp, R cr, const M3<R>& K, const M3<R>& L,
                                            uint32_t lane_ring, Issue&& issue) {
  constexpr int q0 = UP ? 0 : 10;
  auto get = [&](auto pos) {
    constexpr int k = decltype(pos)::value;
    constexpr int q = q0 + k;
    constexpr int after = LAST && q > 20 - kRing ? 20 - q : kRing - 1;  // links issued after q
    ring_wait<RingGeom<R>::loads * after>();
    const M3<R> m = ring_take<k % kRing>(lane_ring, R());
    if constexpr (!LAST || q + kRing <= 20) issue(q + kRing);
    return m;
  };
  orient_paths<R, UP>(S, cp, cr, K, L, get);
}

// The over-improved staple sum of U_MU(x) (as staple_sum) and the own link U,
// every link but K = U_mu(x+mu) and L = U_mu(x-mu) through the LDS ring.  The
// block's dynamic LDS must hold kRingBytes<R>.
template <typename R, int MU>
__device__ __forceinline__ void staple_ring(const Geo& g, const void* src, const int c[4], uint32_t x, R cp, R cr,
                                            M3<R>& S, M3<R>& U) {
  const DirBuf<R> bm = dir_buf<R>(src, g, MU);
  Nb o;
  o.S = (c[0] + c[1] + c[2] + c[3]) & 3;
  o.dn[0] = o.dn[1] = o.dn[2] = o.dn[3] = o.dn[4] = 0;  // b = 0 (K, L) before a nu is set
  o.j = x - (uint32_t)o.S * g.V4;
  o.dm[0] = jdelta(g, MU, c[MU], -1);
  o.dm[1] = 0;
  o.dm[2] = jdelta(g, MU, c[MU], 1);
  o.dm[3] = jdelta(g, MU, c[MU], 2);
  const uint32_t ring = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * kRingWave<R>;
  const uint32_t lane_ring = ring + (threadIdx.x & 63u) * (sizeof(R) == 8 ? 16u : 4u);
  // K and L, held through every orientation: ordinary loads, issued first
  const M3<R> K = ld_rows(bm, nbi(g, o, 1, 0));
  const M3<R> L = ld_rows(bm, nbi(g, o, -1, 0));
  load_fence();
  auto set_nu = [&](int n) {
    o.dn[0] = jdelta(g, n, c[n], -2);
    o.dn[1] = jdelta(g, n, c[n], -1);
    o.dn[2] = 0;
    o.dn[3] = jdelta(g, n, c[n], 1);
    o.dn[4] = jdelta(g, n, c[n], 2);
  };
  {
    // the first five links of the first nu
    const int n0 = MU == 0 ? 1 : 0;
    set_nu(n0);
    const DirBuf<R> b0 = dir_buf<R>(src, g, n0);
#pragma unroll
    for (int q = 0; q < kRing; ++q)
      ring_issue(take_mu(q) ? bm : b0, nbi(g, o, take_a(q), take_bu(q)), ring + (uint32_t)q * RingGeom<R>::slot);
  }
  S = mzero<R>();
#pragma unroll 1
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == MU) continue;
    set_nu(nu);
    const DirBuf<R> bn = dir_buf<R>(src, g, nu);
    // the next nu, whose first five links are issued from the end of this one;
    // after the last nu the own link is issued instead
    int nn = nu + 1;
    if (nn == MU) ++nn;
    const bool last = nn > 3;
    const int nx = last ? nu : nn;  // a valid axis on the last nu (its offsets go unused)
    const int dn1 = jdelta(g, nx, c[nx], 1), dn2 = jdelta(g, nx, c[nx], 2);
    const DirBuf<R> bnn = dir_buf<R>(src, g, nx);
    auto issue = [&](int q) {
      // the ring base is read again at each issue (an empty asm that may change
      // it), so that the compiler forms the LDS addresses where they are used
      // instead of holding all of them in scalar registers through the loop
      uint32_t rg = ring;
      asm volatile("" : "+s"(rg));
      const uint32_t slot = rg + (uint32_t)(q % kRing) * RingGeom<R>::slot;
      if (q < 20) {
        const int k = q % 10;
        ring_issue(take_mu(k) ? bm : bn, nbi(g, o, take_a(k), q < 10 ? take_bu(k) : take_bd(k)), slot);
      } else if (last) {
        ring_issue(bm, x, slot);
      } else {
        const int k = q - 20;
        const int b = take_bu(k);
        const uint32_t nidx = (uint32_t)((o.S + take_a(k) + b) & 3) * g.V4 +
                              (uint32_t)((int)o.j + o.dm[take_a(k) + 1] + (b == 0 ? 0 : (b == 1 ? dn1 : dn2)));
        ring_issue(take_mu(k) ? bm : bnn, nidx, slot);
      }
    };
    ring_orient<R, true, false>(S, cp, cr, K, L, lane_ring, issue);
    if (last)
      ring_orient<R, false, true>(S, cp, cr, K, L, lane_ring, issue);
    else
      ring_orient<R, false, false>(S, cp, cr, K, L, lane_ring, issue);
  }
  // the own link went into the slot of take position 20 (slot 0); wait for
  // every load issued after it too, so that no write into LDS is pending when
  // the wave moves on
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  U = ring_take<0>(lane_ring, R());
  rebuild_row2(U);
}

// k_update, whose launch allocates kRingBytes<double> of dynamic LDS in FP64,
// takes the FP64 over-improved staples through the ring.  The serving step
// kernel does not: with the bodies of all four directions in one kernel the
// ring's code left it with a thousand spilled registers.
template <typename R, bool OI>
constexpr bool kUseRing = OI && sizeof(R) == 8;

// ------------------------------------------------------------------ updates

// H = -i rho Q for the stout generator Q of Omega = Sigma U^dag: Hermitian and
// traceless, the diagonal from differences (exactly 0 for Omega proportional
// to 1).
template <typename R>
__device__ __forceinline__ M3<R> stout_h(const M3<R>& S, const M3<R>& U, double rho) {
  const M3<R> om = mul_nd(S, U);
  // A = (Omega - Omega^dag)/2 ; Q_ij = A_ij off the diagonal; diagonal A_ii is i*a_i
  const R a0 = om.a[0].im, a1 = om.a[4].im, a2 = om.a[8].im;
  const R q0 = ((a0 - a1) + (a0 - a2)) / R(3);
  const R q1 = ((a1 - a0) + (a1 - a2)) / R(3);
  const R q2 = ((a2 - a0) + (a2 - a1)) / R(3);
  // H = -i rho Q: H_ii = rho q_i ; H_ij = -i rho A_ij with A_ij = (om_ij - conj om_ji)/2
  M3<R> H;
  const R r = (R)rho;
  H.a[0] = cx<R>(r * q0, R(0));
  H.a[4] = cx<R>(r * q1, R(0));
  H.a[8] = cx<R>(r * q2, R(0));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i + 1; j < 3; ++j) {
      const R ar = R(0.5) * (om.a[3 * i + j].re - om.a[3 * j + i].re);
      const R ai = R(0.5) * (om.a[3 * i + j].im + om.a[3 * j + i].im);
      // -i (ar + i ai) = ai - i ar
      H.a[3 * i + j] = cx<R>(r * ai, -r * ar);
      H.a[3 * j + i] = cx<R>(r * ai, r * ar);
    }
  return H;
}

// out = exp(i H) U for Hermitian traceless H, by Cayley-Hamilton with FP64
// coefficients, then FP64 reunitarisation.  Returns false (U unchanged) when
// c1 = Tr H^2 / 2 does not exceed c1_floor: H = 0, or H below the rounding
// level its caller states.
template <typename R>
__device__ __forceinline__ bool exp_apply(const M3<R>& H, const M3<R>& U, M3<double>& out, double c1_floor = 0.0) {
  double c0, c1;
  ch_invariants(H, c0, c1);
  if (c1 <= c1_floor) return false;  // a NaN carries on, so that it is counted
  const CHCoef f = ch_coefficients(c0, c1);
  // E = f0 + f1 H + f2 H^2 in the working precision
  const M3<R> H2 = mul_nn(H, H);
  M3<R> E;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    Cx<R> v = cx<R>(R(0), R(0));
    cfma(v, cx<R>((R)f.f1.re, (R)f.f1.im), H.a[e]);
    cfma(v, cx<R>((R)f.f2.re, (R)f.f2.im), H2.a[e]);
    E.a[e] = v;
  }
  E.a[0].re += (R)f.f0.re;
  E.a[0].im += (R)f.f0.im;
  E.a[4].re += (R)f.f0.re;
  E.a[4].im += (R)f.f0.im;
  E.a[8].re += (R)f.f0.re;
  E.a[8].im += (R)f.f0.im;
  out = mconvert<double>(mul_nn(E, U));
  reunitarise(out);
  return true;
}

// Stout (Eq. stout, Eq. generator): Omega = Sigma U^dag, Q its traceless
// anti-Hermitian part, X = rho Q, U' = exp(X) U.  Q = 0 returns U unchanged
// (Sec. II.A: a centre field, whose staples are proportional to 1, does not
// move).  Q counts as 0 when |Q|_F <= q_floor (UpdParams::qfloor, a few dozen
// FP64 roundings of the staple sum's terms): a stored link's row 2 is rebuilt
// from rows 0 and 1 with a rounding error, so for a centre field Omega is
// proportional to 1 only up to the rounding of the paths summed into Sigma.
template <typename R>
__device__ __forceinline__ bool stout_candidate(const M3<R>& S, const M3<R>& U, double rho, double q_floor,
                                                M3<double>& out) {
  const M3<R> H = stout_h(S, U, rho);
  // c1 = |H|_F^2 / 2 = rho^2 |Q|_F^2 / 2
  const double rq = rho * q_floor;
  return exp_apply(H, U, out, 0.5 * rq * rq);
}

// MaxReTr (Eq. maxReTr, def_L1, def_T1): V = (1 - alpha) U + (alpha/6) Sigma,
// L = U V^dag; for loops x subgroups (0,1), (1,2), (0,2): T from L's 2x2 block,
// k = sqrt(det T), T^c = T^dag / k, U <- T^c U and L <- T^c L.  A hit with
// k <= 1e-12 (|L|_F + 1) is skipped (k = 0 leaves the hit undefined).  FP64.
template <typename R>
__device__ __forceinline__ bool maxretr_candidate(const M3<R>& S, const M3<R>& U0, double alpha,
                                                  int loops, M3<double>& out) {
  M3<double> U = mconvert<double>(U0);
  M3<double> Vb;
  const M3<double> Sd = mconvert<double>(S);
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    Vb.a[e].re = (1.0 - alpha) * U.a[e].re + alpha / 6.0 * Sd.a[e].re;
    Vb.a[e].im = (1.0 - alpha) * U.a[e].im + alpha / 6.0 * Sd.a[e].im;
  }
  M3<double> L = mul_nd(U, Vb);
  double lf = 0.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) lf += L.a[e].re * L.a[e].re + L.a[e].im * L.a[e].im;
  lf = sqrt(lf);
  const double thr = 1e-12 * (lf + 1.0);
  bool moved = false;
  for (int it = 0; it < loops; ++it) {
#pragma unroll
    for (int h = 0; h < 3; ++h) {
      const int p = (h == 1) ? 1 : 0;
      const int q = (h == 0) ? 1 : 2;
      const Cx<double> Lpp = L.a[4 * p], Lqq = L.a[4 * q], Lpq = L.a[3 * p + q], Lqp = L.a[3 * q + p];
      // T = [[a, b], [-conj b, conj a]] with a = (Lpp + conj Lqq)/2, b = (Lpq - conj Lqp)/2
      const double ar = 0.5 * (Lpp.re + Lqq.re), ai = 0.5 * (Lpp.im - Lqq.im);
      const double br = 0.5 * (Lpq.re - Lqp.re), bi = 0.5 * (Lpq.im + Lqp.im);
      const double det = ar * ar + ai * ai + br * br + bi * bi;
      const double k = sqrt(det);
      if (!(k > thr)) continue;
      const double ik = 1.0 / k;
      // T^c = T^dag / k = [[conj a, -b], [conj b, a]] / k
      const Cx<double> t00 = cx<double>(ar * ik, -ai * ik), t01 = cx<double>(-br * ik, -bi * ik);
      const Cx<double> t10 = cx<double>(br * ik, -bi * ik), t11 = cx<double>(ar * ik, ai * ik);
#pragma unroll
      for (int col = 0; col < 3; ++col) {
        Cx<double> up = cx<double>(0.0, 0.0), uq = cx<double>(0.0, 0.0);
        cfma(up, t00, U.a[3 * p + col]);
        cfma(up, t01, U.a[3 * q + col]);
        cfma(uq, t10, U.a[3 * p + col]);
        cfma(uq, t11, U.a[3 * q + col]);
        U.a[3 * p + col] = up;
        U.a[3 * q + col] = uq;
        Cx<double> lp = cx<double>(0.0, 0.0), lq = cx<double>(0.0, 0.0);
        cfma(lp, t00, L.a[3 * p + col]);
        cfma(lp, t01, L.a[3 * q + col]);
        cfma(lq, t10, L.a[3 * p + col]);
        cfma(lq, t11, L.a[3 * q + col]);
        L.a[3 * p + col] = lp;
        L.a[3 * q + col] = lq;
      }
      moved = true;
    }
  }
  out = U;
  return moved;
}

// APE (Sec. II.C, Eqs. V, W): the blocked matrix V = (1 - alpha) U +
// (alpha/6) Sigma in FP64, returned to SU(3) by the unit circle projection:
// its unitary polar factor W, by the scaled Newton iteration
// X <- (z X + X^{-dagger}/z)/2 with z = sqrt(|X^{-1}|_F / |X|_F) (Higham), then
// W / cbrt(det W) with the principal root (phase in (-pi/3, pi/3]), and an
// FP64 Gram-Schmidt clean-up.  A singular V has no projection (NaN, counted as
// non-finite by the measurement).
template <typename R>
__device__ __forceinline__ bool ape_candidate(const M3<R>& S, const M3<R>& U0, double alpha, M3<double>& out) {
  const M3<double> U = mconvert<double>(U0);
  const M3<double> Sd = mconvert<double>(S);
  M3<double> X;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    X.a[e].re = (1.0 - alpha) * U.a[e].re + alpha / 6.0 * Sd.a[e].re;
    X.a[e].im = (1.0 - alpha) * U.a[e].im + alpha / 6.0 * Sd.a[e].im;
  }
  auto cmul = [](Cx<double> a, Cx<double> b) { return cx<double>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); };
  auto adj_det = [&](const M3<double>& m, M3<double>& adj) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const Cx<double> p = cmul(m.a[3 * ((j + 1) % 3) + (i + 1) % 3], m.a[3 * ((j + 2) % 3) + (i + 2) % 3]);
        const Cx<double> q = cmul(m.a[3 * ((j + 1) % 3) + (i + 2) % 3], m.a[3 * ((j + 2) % 3) + (i + 1) % 3]);
        adj.a[3 * i + j] = cx<double>(p.re - q.re, p.im - q.im);
      }
    Cx<double> d = cx<double>(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const Cx<double> t = cmul(m.a[j], adj.a[3 * j]);
      d.re += t.re;
      d.im += t.im;
    }
    return d;
  };
  auto fro = [](const M3<double>& m) {
    double r = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) r += m.a[e].re * m.a[e].re + m.a[e].im * m.a[e].im;
    return sqrt(r);
  };
#pragma unroll 1
  for (int it = 0; it < 20; ++it) {
    M3<double> adj;
    const Cx<double> d = adj_det(X, adj);
    const double dd = d.re * d.re + d.im * d.im;
    // X^{-1} = adj / d; X^{-dagger} = adj^dagger / conj(d) = adj^dagger d / |d|^2
    const double nx = fro(X), ni = fro(adj) / sqrt(dd);
    const double z = sqrt(ni / nx);
    double diff = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const Cx<double> a = adj.a[3 * j + i];  // (adj^dagger)_ij = conj(adj_ji)
        const Cx<double> inv_dag = cmul(cx<double>(a.re, -a.im), d);
        const Cx<double> x = X.a[3 * i + j];
        const Cx<double> y = cx<double>(0.5 * (z * x.re + inv_dag.re / (z * dd)),
                                        0.5 * (z * x.im + inv_dag.im / (z * dd)));
        diff += (y.re - x.re) * (y.re - x.re) + (y.im - x.im) * (y.im - x.im);
        X.a[3 * i + j] = y;
      }
    if (!(diff > 1e-28 * 3.0)) break;  // |X|_F = sqrt 3 at convergence; NaN stops too
  }
  M3<double> adj;
  const Cx<double> d = adj_det(X, adj);
  const double r = cbrt(sqrt(d.re * d.re + d.im * d.im));
  const double ph = atan2(d.im, d.re) / 3.0;
  const Cx<double> inv_root = cx<double>(cos(ph) / r, -sin(ph) / r);
#pragma unroll
  for (int e = 0; e < 9; ++e) X.a[e] = cmul(X.a[e], inv_root);
  reunitarise(X);
  out = X;
  return true;
}

// Tr[G^dagger(x) U G(x + mu)]: the trace the vortex-preservation test projects
// when the field lives in the random gauge G (Sec. VI).
__device__ __noinline__ Cx<double> gauge_undone_trace(const double2* __restrict__ gauge, uint32_t s0,
                                                     uint32_t s1, M3<double> u) {
  M3<double> G, Gp;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    G.a[e] = cx<double>(gauge[(size_t)s0 * 9 + e].x, gauge[(size_t)s0 * 9 + e].y);
    Gp.a[e] = cx<double>(gauge[(size_t)s1 * 9 + e].x, gauge[(size_t)s1 * 9 + e].y);
  }
  return mtrace(mul_nn(mul_dn(G, u), Gp));
}

// The FP32 form holds K and L completed through all nu (12 registers more,
// two row rebuilds per orientation fewer); FP64, short of registers, holds
// rows 0 and 1, and takes its staples through orient_paths whether the LDS
// ring or ordinary loads bring the links in, so that every FP64 kernel gives
// the same links.
template <typename R>
constexpr bool kFullKL = sizeof(R) == 4;

// Sigma of link (x, MU) from the field src (Eq. plaq_staples; with OI the
// over-improved sum of Eq. over-improvement, in the factored form with
// U_mu(x +- mu) loaded once).
template <typename R, int MU, bool OI>
__device__ __forceinline__ M3<R> staple_sum(const Geo& g, const void* src, const int c[4], uint32_t x, R cp,
                                            R cr) {
  const DirBuf<R> bm = dir_buf<R>(src, g, MU);
  Nb o;
  o.S = (c[0] + c[1] + c[2] + c[3]) & 3;
  o.dn[0] = o.dn[1] = o.dn[2] = o.dn[3] = o.dn[4] = 0;  // b = 0 (K, L) before a nu is set
  o.j = x - (uint32_t)o.S * g.V4;
  o.dm[0] = jdelta(g, MU, c[MU], -1);
  o.dm[1] = 0;
  o.dm[2] = jdelta(g, MU, c[MU], 1);
  o.dm[3] = jdelta(g, MU, c[MU], 2);
  M3<R> S = mzero<R>();
  M3<R> K, Lm;
  if (OI) {
    K = ld_rows(bm, nbi(g, o, 1, 0));
    load_fence();
    Lm = ld_rows(bm, nbi(g, o, -1, 0));
    load_fence();
    if (kFullKL<R>) {
      K = full(K);
      Lm = full(Lm);
    }
  }
#pragma unroll 1
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == MU) continue;
    o.dn[0] = jdelta(g, nu, c[nu], -2);
    o.dn[1] = jdelta(g, nu, c[nu], -1);
    o.dn[2] = 0;
    o.dn[3] = jdelta(g, nu, c[nu], 1);
    o.dn[4] = jdelta(g, nu, c[nu], 2);
    const DirBuf<R> bn = dir_buf<R>(src, g, nu);
    if constexpr (OI && sizeof(R) == 4) {
      staple_dir_factored<R, true>(S, bm, bn, g, o, cp, cr, K, Lm);
      staple_dir_factored<R, false>(S, bm, bn, g, o, cp, cr, K, Lm);
    } else if constexpr (OI) {
      staple_dir_loads<R, true>(S, bm, bn, g, o, cp, cr, K, Lm);
      staple_dir_loads<R, false>(S, bm, bn, g, o, cp, cr, K, Lm);
    } else {
      // the six links of the two plaquette staples, loaded together:
      // U_nu(x) U_mu(x+nu) U_nu^dag(x+mu) and U_nu^dag(x-nu) U_mu(x-nu) U_nu(x+mu-nu)
      const M3<R> Au = ld_rows(bn, nbi(g, o, 0, 0)), Bu = ld_rows(bm, nbi(g, o, 0, 1)),
                  Cu = ld_rows(bn, nbi(g, o, 1, 0));
      const M3<R> Ad = ld_rows(bn, nbi(g, o, 0, -1)), Bd = ld_rows(bm, nbi(g, o, 0, -1)),
                  Cd = ld_rows(bn, nbi(g, o, 1, -1));
      load_fence();
      M3<R> w = mul2_nn(Au, full(Bu));
      w = mul2_nd(w, full(Cu));
      chain_add(S, cp, w);
      w = mul2_dn(full(Ad), full(Bd));
      w = mul2_nn(w, full(Cd));
      chain_add(S, cp, w);
    }
  }
  return S;
}

// The thread's link of an annealing subset (Sec. III.A masking).  Subset c of
// direction mu holds the sites with (2 x_mu + sum_{nu != mu} x_nu) mod 4 = c,
// i.e. with sublattice (x0 + x1 + x2 + x3) mod 4 = (c - x_mu) mod 4 (internal axes).
//   mu != 0: every position j has exactly one such site, in sublattice
//            (c - x_mu) mod 4, so thread t takes j = t;
//   mu == 0: only rows with x1 + x2 + x3 of the parity of c take part, each with
//            the two residues x0 mod 4 = h, h + 2, h = ((c - x1 - x2 - x3) mod 4) / 2.
// The sweep axis of the traversal (tile_rows): never MU itself, whose
// neighbours the staples reach furthest; for the FP32 form (twice the blocks in
// flight) axis 2 otherwise, for FP64 axis 3 (both chosen with a model of the L2
// and confirmed by timing on 48^3x96).
template <typename R, int MU>
constexpr int sweep_axis() {
  return MU == 3 ? 2 : (MU == 2 ? 3 : (sizeof(R) == 4 ? 2 : 3));
}

template <int MU, int SW>
__device__ __forceinline__ void subset_site(const Geo& g, int colour, uint32_t t, int c[4]) {
  if (MU != 0) {
    const uint32_t xi = t % (uint32_t)g.Xq;
    tile_rows<SW>(g, t / (uint32_t)g.Xq, c, 0);
    const int s = (colour - c[MU]) & 3;
    c[0] = (int)(4 * xi) + ((s - c[1] - c[2] - c[3]) & 3);
  } else {
    const uint32_t two = 2u * (uint32_t)g.Xq;
    const uint32_t k = t / two;
    const uint32_t rem = t - k * two;
    const uint32_t which = rem / (uint32_t)g.Xq;
    const uint32_t xi = rem - which * (uint32_t)g.Xq;
    tile_rows<SW>(g, k, c, 1);
    c[1] = 2 * c[1] + ((colour - c[2] - c[3]) & 1);
    const int S = c[1] + c[2] + c[3];
    const int h = ((colour - S) & 3) >> 1;
    c[0] = (int)(4 * xi) + h + 2 * (int)which;
  }
}

// XCD-aware block order: consecutive hardware blocks go round-robin to the 8
// XCDs; this gives each XCD one contiguous range of the lattice (when the grid
// is a multiple of 8 blocks), so that neighbouring blocks share an L2.
__device__ __forceinline__ uint32_t xcd_block() {
  const uint32_t b = blockIdx.x, nb = gridDim.x;
  return (nb & 7u) == 0u ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
}

// Site of thread t of a kernel that visits every site (measurement, Jacobi
// smearing, flow), in blocks of 256.  Block t / 256 takes a chunk of 64
// positions j (rows of internal axis 0 in the tile order of the update) and
// its four waves take the four sublattices of that chunk: a wave's loads of a
// link entry are one contiguous run, and the neighbour x + mu of a site (the
// next sublattice) is read by another wave of the same block.  Returns false
// for threads past the end of the lattice.
__device__ __forceinline__ bool chunk_site(const Geo& g, uint32_t t, int c[4]) {
  const uint32_t tj = (t >> 8) * 64u + (t & 63u);
  if (tj >= g.V4) return false;
  const uint32_t s = (t >> 6) & 3u;
  const uint32_t row = tj / (uint32_t)g.Xq;
  const uint32_t xi = tj - row * (uint32_t)g.Xq;
  tile_rows(g, row, c, 0);
  c[0] = (int)(4u * xi) + (int)((s - (uint32_t)(c[1] + c[2] + c[3])) & 3u);
  return true;
}

// One link update of direction MU for thread t: jacobi = 0, the t-th link of
// annealing subset `colour` (subset_site), in place (src == dst); jacobi = 1,
// the link of direction MU at chunk_site(t), from src into dst (smearing).
// UPD = 0 stout, 1 MaxReTr, 2 APE with unit circle projection.  With
// vp, a candidate is kept only if its centre sector (after undoing the gauge
// transform, when one is given) equals the original charge (z3, canonical
// layout: one byte per update, not worth a relayout).  Returns whether a
// candidate was rejected.
template <typename R, int MU, bool OI, int UPD, bool RING>
__device__ __forceinline__ bool update_one(const Geo& g, const void* src, void* dst,
                                           const int8_t* __restrict__ z3,
                                           const double2* __restrict__ gauge, const UpdParams& p,
                                           int colour, int jacobi, uint32_t t, uint32_t nthreads) {
  const bool active = t < nthreads;
  int c[4] = {0, 0, 0, 0};
  if (active) {
    if (jacobi)
      chunk_site(g, t, c);
    else
      subset_site<MU, sweep_axis<R, MU>()>(g, colour, t, c);
  }
  bool rej = false;
  if (active) {
    const uint32_t x = site_index(g, c);
    M3<R> S, U;
    if constexpr (RING) {
      static_assert(OI, "the LDS ring serves the over-improved staples");
      staple_ring<R, MU>(g, src, c, x, (R)p.cp, (R)p.cr, S, U);
    } else {
      S = staple_sum<R, MU, OI>(g, src, c, x, (R)p.cp, (R)p.cr);
      U = ld_link(dir_buf<R>(src, g, MU), x);
    }
    M3<double> cand;
    bool moved;
    if (UPD == 0)
      moved = stout_candidate<R>(S, U, p.rho, p.qfloor, cand);
    else if (UPD == 1)
      moved = maxretr_candidate<R>(S, U, p.alpha, p.loops, cand);
    else
      moved = ape_candidate<R>(S, U, p.alpha, cand);
    // the candidate exactly as a later load will see it: rows 0 and 1 rounded
    // to the storage precision, row 2 rebuilt from them
    M3<R> cr_ = mconvert<R>(cand);
    rebuild_row2(cr_);
    bool accept = moved;
    if (moved && p.vp) {
      // sector of the stored candidate, evaluated in FP64 as the measurement does
      Cx<double> tr;
      if (gauge) {
        int cp1[4] = {c[0], c[1], c[2], c[3]};
        cp1[MU] = (cp1[MU] + 1 == g.L[MU]) ? 0 : cp1[MU] + 1;
        tr = gauge_undone_trace(gauge, canonical_index(g, c), canonical_index(g, cp1), mconvert<double>(cr_));
      } else {
        tr = mtrace(mconvert<double>(cr_));
      }
      const int n0 = z3[(size_t)g.uperm[MU] * g.V + canonical_index(g, c)];
      accept = (z3_sector(tr.re, tr.im) == n0);
    }
    rej = moved && !accept;
    if (jacobi || accept) {
      // Chosen entry by entry: an if/else assigning whole matrices here made the
      // gfx950 build of the vortex-preserving, gauge-undoing path store two
      // entries of the old link (seen in the generated code and on the device).
      // The random-gauge vortex-preservation tests cover this path.
      M3<R> outl;
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        outl.a[e].re = accept ? cr_.a[e].re : U.a[e].re;
        outl.a[e].im = accept ? cr_.a[e].im : U.a[e].im;
      }
      st_link<R>(dst, g, MU, x, outl);
    }
  }
  return rej;
}

// One update step for direction MU over the whole lattice (see update_one);
// rejections are counted per wave into *rejected.
template <typename R, int MU, bool OI, int UPD>
__global__ void __launch_bounds__(256) k_update(Geo g, const void* src, void* dst,
                                                const int8_t* __restrict__ z3,
                                                const double2* __restrict__ gauge, UpdParams p,
                                                int colour, int jacobi, uint32_t nthreads,
                                                unsigned long long* __restrict__ rejected) {
  const uint32_t t = xcd_block() * blockDim.x + threadIdx.x;
  const bool rej = update_one<R, MU, OI, UPD, kUseRing<R, OI>>(g, src, dst, z3, gauge, p, colour, jacobi, t,
                                                               nthreads);
  if (rejected) {
    const unsigned long long m = __ballot(rej);
    if ((threadIdx.x & 63u) == 0u && m) atomicAdd(rejected, (unsigned long long)__popcll(m));
  }
}

// One serving step (see BatchStep): each block belongs to one job, found from
// the step's block ranges; its threads run that job's subset pass with exactly
// the per-link code of k_update, so a job's links do not depend on which other
// jobs share the launch.  Stout updates only.
template <typename R, int MU, bool OI, bool RING>
__device__ __forceinline__ bool batch_one(const ServeJob& J, int colour, uint32_t t) {
  return update_one<R, MU, OI, 0, RING>(J.g, J.links, J.links, J.z3, nullptr, J.p, colour, 0, t, J.g.V4);
}

template <typename R>
__global__ void __launch_bounds__(256) k_update_batch(const ServeJob* __restrict__ jobs, BatchStep st) {
  // blocks in XCD ranges, so that a job's neighbouring blocks share an L2; the
  // grid is padded to a multiple of 8 and the padding blocks fall past the end
  // of the last job (t >= its thread count: nothing to do)
  const uint32_t b = xcd_block();
  uint32_t fb = st.first_block[0], slot = st.slot[0];
  int mu = st.mu[0], colour = st.colour[0];
#pragma unroll
  for (int k = 1; k < kBatchMax; ++k) {
    if ((uint32_t)k < st.njobs && b >= st.first_block[k]) {
      fb = st.first_block[k];
      slot = st.slot[k];
      mu = st.mu[k];
      colour = st.colour[k];
    }
  }
  const ServeJob& J = jobs[slot];
  const uint32_t t = (b - fb) * blockDim.x + threadIdx.x;
  bool rej;
  if (J.p.oi) {
    switch (mu) {
      case 0: rej = batch_one<R, 0, true, false>(J, colour, t); break;
      case 1: rej = batch_one<R, 1, true, false>(J, colour, t); break;
      case 2: rej = batch_one<R, 2, true, false>(J, colour, t); break;
      default: rej = batch_one<R, 3, true, false>(J, colour, t); break;
    }
  } else {
    switch (mu) {
      case 0: rej = batch_one<R, 0, false, false>(J, colour, t); break;
      case 1: rej = batch_one<R, 1, false, false>(J, colour, t); break;
      case 2: rej = batch_one<R, 2, false, false>(J, colour, t); break;
      default: rej = batch_one<R, 3, false, false>(J, colour, t); break;
    }
  }
  const unsigned long long m = __ballot(rej);
  if ((threadIdx.x & 63u) == 0u && m) atomicAdd(J.rej, (unsigned long long)__popcll(m));
}

// Small-lattice serving step (see SmallStep): workgroup b runs sweeps[b] whole
// annealed sweeps of job slot[b] -- for mu = 0..3 (user order), subsets 0, 2,
// 1, 3, each pass over all V/4 links of the subset with the per-link code of
// k_update (batch_one), its threads striding over the subset -- with a
// workgroup barrier after every pass, so the next pass reads the links this one
// stored (all waves of a workgroup share one CU and its L1).  No device-wide
// wait: the job lives in one workgroup.  Rejections are counted per wave into
// the job's counter.
template <typename R>
constexpr unsigned kSmallThreads = sizeof(R) == 4 ? 512u : 256u;  // FP32 fits two waves per SIMD

template <typename R>
__global__ void __launch_bounds__(kSmallThreads<R>) k_serve_small(const ServeJob* __restrict__ jobs, SmallStep st) {
  if (blockIdx.x >= st.njobs) return;
  const ServeJob& J = jobs[st.slot[blockIdx.x]];
  const int nsw = st.sweeps[blockIdx.x];
  const uint32_t V4 = J.g.V4;
  unsigned long long rej = 0;
  for (int sw = 0; sw < nsw; ++sw) {
    for (int d = 0; d < 4; ++d) {
      const int mu = J.g.perm[d];
      for (int k = 0; k < 4; ++k) {
        const int colour = k == 1 ? 2 : (k == 2 ? 1 : k);
        for (uint32_t t0 = 0; t0 < V4; t0 += blockDim.x) {
          const uint32_t t = t0 + threadIdx.x;
          bool r;
          if (J.p.oi) {
            switch (mu) {
              case 0: r = batch_one<R, 0, true, false>(J, colour, t); break;
              case 1: r = batch_one<R, 1, true, false>(J, colour, t); break;
              case 2: r = batch_one<R, 2, true, false>(J, colour, t); break;
              default: r = batch_one<R, 3, true, false>(J, colour, t); break;
            }
          } else {
            switch (mu) {
              case 0: r = batch_one<R, 0, false, false>(J, colour, t); break;
              case 1: r = batch_one<R, 1, false, false>(J, colour, t); break;
              case 2: r = batch_one<R, 2, false, false>(J, colour, t); break;
              default: r = batch_one<R, 3, false, false>(J, colour, t); break;
            }
          }
          rej += r ? 1ull : 0ull;
        }
        __syncthreads();
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) rej += __shfl_xor(rej, off);
  if ((threadIdx.x & 63u) == 0u && rej) atomicAdd(J.rej, rej);
}

// ------------------------------------------------------------------ Wilson flow

// One stage of the Wilson flow (Sec. II.B, V.B) for every link of direction MU,
// from the field src into dst (all links at once).  H_Z = -i eps Q[src] is the
// step's generator (the stout generator with rho = eps); acc holds the
// Runge-Kutta accumulator H_A (FP64, 8 reals per link: H_00, H_11 and the
// upper triangle).  Stage 0: Euler, H = H_Z.  Stages 1-3: the third-order
// scheme W1 = exp(Z0/4) W0, W2 = exp(8/9 Z1 - 17/36 Z0) W1,
// W3 = exp(3/4 Z2 - 8/9 Z1 + 17/36 Z0) W2, kept with one accumulator:
// stage 1 H = H_Z/4, A <- H; stage 2 H = 8/9 H_Z - 17/9 A, A <- H;
// stage 3 H = 3/4 H_Z - A.  dst = exp(i H) src, reunitarised.
template <typename R, int MU, bool OI>
__global__ void __launch_bounds__(256) k_flow(Geo g, const void* src, void* dst, double* __restrict__ acc,
                                              int stage, double eps, double cp, double cr) {
  int c[4];
  if (!chunk_site(g, xcd_block() * 256u + threadIdx.x, c)) return;
  const uint32_t t = site_index(g, c);
  const M3<R> S = staple_sum<R, MU, OI>(g, src, c, t, (R)cp, (R)cr);
  const M3<R> U = ld_link(dir_buf<R>(src, g, MU), t);
  const M3<R> Hz = stout_h(S, U, eps);
  M3<R> H = Hz;
  if (stage > 0) {
    double* a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = acc + ((size_t)k * 4 + MU) * g.V + t;
    double hz[8] = {(double)Hz.a[0].re, (double)Hz.a[4].re, (double)Hz.a[1].re, (double)Hz.a[1].im,
                    (double)Hz.a[2].re, (double)Hz.a[2].im, (double)Hz.a[5].re, (double)Hz.a[5].im};
    double h[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (stage == 1)
        h[k] = 0.25 * hz[k];
      else if (stage == 2)
        h[k] = (8.0 / 9.0) * hz[k] - (17.0 / 9.0) * *a[k];
      else
        h[k] = 0.75 * hz[k] - *a[k];
      if (stage < 3) *a[k] = h[k];
    }
    H.a[0] = cx<R>((R)h[0], R(0));
    H.a[4] = cx<R>((R)h[1], R(0));
    H.a[8] = cx<R>((R)(-h[0] - h[1]), R(0));
    H.a[1] = cx<R>((R)h[2], (R)h[3]);
    H.a[3] = cx<R>((R)h[2], (R)(-h[3]));
    H.a[2] = cx<R>((R)h[4], (R)h[5]);
    H.a[6] = cx<R>((R)h[4], (R)(-h[5]));
    H.a[5] = cx<R>((R)h[6], (R)h[7]);
    H.a[7] = cx<R>((R)h[6], (R)(-h[7]));
  }
  M3<double> out;
  if (!exp_apply(H, U, out)) out = mconvert<double>(U);
  st_link<R>(dst, g, MU, t, mconvert<R>(out));
}

// ------------------------------------------------------------------ measurement

// Neumaier/TwoSum accumulation of a double.
struct KSum {
  double s, c;
};
__device__ __forceinline__ void kadd(KSum& k, double v) {
  const double t = k.s + v;
  if (fabs(k.s) >= fabs(v))
    k.c += (k.s - t) + v;
  else
    k.c += (v - t) + k.s;
  k.s = t;
}
__device__ __forceinline__ void kmerge(KSum& k, const KSum& o) {
  kadd(k, o.s);
  k.c += o.c;
}

struct Partial {  // 80 bytes; partial_bytes() in vsm_kernels.hip must match
  double plaq_s, plaq_c, act_s, act_c, max_unit, pad;
  long long mism, undef, nonfin, pad2;
};
static_assert(sizeof(Partial) == 80, "partial record size is part of the workspace layout");

__device__ __forceinline__ int link_sector(const M3<double>& u) {
  const Cx<double> t = mtrace(u);
  return z3_sector(t.re, t.im);
}

// Centre sector of the link u = U_d(x) (internal direction d, site c) in
// maximal centre gauge: with a gauge field G (the field lives in that random
// gauge, Sec. V.C) the sector of G^dagger(x) u G(x + d), as the vortex-preserving
// test of Sec. VI takes it; without one, the sector of u itself.
template <bool GAUGE>
__device__ __forceinline__ int mcg_sector(const Geo& g, const double2* __restrict__ gauge, const M3<double>& u,
                                          const int c[4], int d) {
  if (!GAUGE) return link_sector(u);
  int cp[4] = {c[0], c[1], c[2], c[3]};
  cp[d] = wrap_add(cp[d], 1, g.L[d]);
  const Cx<double> t = gauge_undone_trace(gauge, canonical_index(g, c), canonical_index(g, cp), u);
  return z3_sector(t.re, t.im);
}

// Per site: the six plaquettes P_{mu nu}(x), mu < nu (Sec. I), summed as
// Re Tr P and Re Tr[1 - P] (Sec. V.A); the sectors of the four links at x;
// the vortex flux of every plaquette from the link sectors compared with the
// flux of the original charges; unitarity and finiteness of the own links.
// Sites by chunk_site, blocks in XCD ranges, so the neighbours x + mu of a
// site are read by the same or a nearby block and come from cache.
// Planes use user axes; the original charges z3 are in the internal layout
// (k_charges).  Block partials go to fixed slots; k_finalize sums them in a
// fixed order, so the result does not depend on the scheduling.  With GAUGE,
// link sectors are taken after undoing the gauge field (mcg_sector).
template <typename R, bool GAUGE>
__global__ void __launch_bounds__(256) k_measure(Geo g, const void* links, const int8_t* __restrict__ z3,
                                                 const double2* __restrict__ gauge, Partial* __restrict__ part,
                                                 int8_t* __restrict__ flux) {
  const uint32_t blk = xcd_block();
  KSum kp = {0.0, 0.0}, ka = {0.0, 0.0};
  double maxu2 = 0.0;  // largest |(U^dag U - 1)_ij|^2; its root is taken once per thread
  long long mism = 0, undef = 0, nonfin = 0;
  int c[4];
  if (chunk_site(g, blk * 256u + threadIdx.x, c)) {
    const uint32_t x = site_index(g, c);
    const uint32_t s = canonical_index(g, c);
    // original charges of the four links at x (user directions), one byte each;
    // their sectors are filled in as the links are first read
    uint32_t secb = 0, n0b = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) n0b |= (uint32_t)(z3[(size_t)g.perm[mu] * g.V + x] & 0xff) << (8 * mu);
    auto byte_at = [](uint32_t w, int i) { return (int)(int8_t)((w >> (8 * i)) & 0xffu); };
    // sector, finiteness and unitarity of an own link, once per link
    // (U^dag U is Hermitian: its three diagonal entries and three entries above)
    auto own_checks = [&](const M3<double>& U, int mu) {
      const int sc = mcg_sector<GAUGE>(g, gauge, U, c, g.perm[mu]);
      secb |= (uint32_t)(sc & 0xff) << (8 * mu);
      bool fin = true;
#pragma unroll
      for (int e = 0; e < 9; ++e) fin = fin && isfinite(U.a[e].re) && isfinite(U.a[e].im);
      if (!fin) ++nonfin;
      if (sc == kUndef) ++undef;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double d = -1.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) d = fma(U.a[3 * i + j].re, U.a[3 * i + j].re, fma(U.a[3 * i + j].im, U.a[3 * i + j].im, d));
        maxu2 = fmax(maxu2, d * d);
#pragma unroll
        for (int k = j + 1; k < 3; ++k) {
          Cx<double> o = cx<double>(0.0, 0.0);
#pragma unroll
          for (int i = 0; i < 3; ++i) cfma_c1(o, U.a[3 * i + j], U.a[3 * i + k]);
          maxu2 = fmax(maxu2, fma(o.re, o.re, o.im * o.im));
        }
      }
    };
    // <a, b> = sum_k a_k conj(b_k) of rows of two matrices
    auto rdot = [](const M3<double>& a, int ra, const M3<double>& b, int rb) {
      Cx<double> v = cx<double>(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) cfma_c2(v, a.a[3 * ra + k], b.a[3 * rb + k]);
      return v;
    };
    // Planes in the order 01, 02, 03, 13, 12, 23 (user axes), so that each plane
    // after the first shares an own link of x with the plane before: that link
    // is held over (held), the plane loads the other own link and its two
    // neighbour links together (rows 0 and 1), and one memory latency is
    // exposed per plane.  An own link read again after more planes would have
    // left the L2 by then; in this order x's own links are read 7 times instead
    // of 12.
    // P = A B C^dag D^dag = X Y^dag with X = A B and Y = D C, both SU(3): rows 0
    // and 1 of X and Y are products of two-row links with completed right
    // factors, and the diagonal of X Y^dag is <x_i, y_i>, the third entry by
    // the Binet-Cauchy identity <x0 x x1, y0 x y1> = <x0,y0><x1,y1> - <x0,y1><x1,y0>
    // (row 2 of an SU(3) matrix is conj(row0 x row1)).
    M3<R> held = mzero<R>();
#pragma unroll 1
    for (int q = 0; q < 6; ++q) {
      // plane q of this order: (mu, nu), its index in the flux array, and
      // which own link comes from the plane before (1: U_mu, 2: U_nu) and is
      // kept for the next (1: U_mu, 2: U_nu)
      const int mu = q < 3 ? 0 : (q < 5 ? 1 : 2);
      const int nu = q < 3 ? q + 1 : (q == 3 ? 3 : (q == 4 ? 2 : 3));
      const int p = q == 3 ? 4 : (q == 4 ? 3 : q);
      const int from = q == 0 ? 0 : (q == 3 ? 2 : 1);
      const int keep = (q == 2 || q == 4) ? 2 : 1;
      const int dm = g.perm[mu], dn = g.perm[nu];
      const DirBuf<R> bmu = dir_buf<R>(links, g, dm), bnu = dir_buf<R>(links, g, dn);
      int cm[4] = {c[0], c[1], c[2], c[3]};
      cm[dm] = wrap_add(cm[dm], 1, g.L[dm]);
      int cn[4] = {c[0], c[1], c[2], c[3]};
      cn[dn] = wrap_add(cn[dn], 1, g.L[dn]);
      const uint32_t xm = site_index(g, cm), xn = site_index(g, cn);
      M3<R> Ar = held, Dr = held;
      if (from != 1) Ar = ld_rows(bmu, x);
      const M3<R> Br = ld_rows(bnu, xm);
      const M3<R> Cr = ld_rows(bmu, xn);
      if (from != 2) Dr = ld_rows(bnu, x);
      load_fence();
      held = keep == 1 ? Ar : Dr;
      if (q == 0) own_checks(mconvert<double>(full(Ar)), 0);
      if (mu == 0) own_checks(mconvert<double>(full(Dr)), nu);
      const M3<double> B = mconvert<double>(full(Br));
      const int sb = mcg_sector<GAUGE>(g, gauge, B, cm, dn);
      const M3<double> X = mul2_nn(mconvert<double>(Ar), B);
      const M3<double> Cm = mconvert<double>(full(Cr));
      const int sc = mcg_sector<GAUGE>(g, gauge, Cm, cn, dm);
      const M3<double> Y = mul2_nn(mconvert<double>(Dr), Cm);
      const Cx<double> p00 = rdot(X, 0, Y, 0), p11 = rdot(X, 1, Y, 1);
      const Cx<double> p01 = rdot(X, 0, Y, 1), p10 = rdot(X, 1, Y, 0);
      double d2 = p00.re * p11.re;
      d2 = fma(-p00.im, p11.im, d2);
      d2 = fma(-p01.re, p10.re, d2);
      d2 = fma(p01.im, p10.im, d2);
      const double rt = p00.re + p11.re + d2;
      const double ra = (1.0 - p00.re) + (1.0 - p11.re) + (1.0 - d2);
      kadd(kp, rt);
      kadd(ka, ra);
      const int smu = byte_at(secb, mu), snu = byte_at(secb, nu);
      const int o = byte_at(n0b, mu) + (int)z3[(size_t)dn * g.V + xm] - (int)z3[(size_t)dm * g.V + xn] -
                    byte_at(n0b, nu);
      const int orig = ((o % 3) + 3) % 3;
      int pv;
      if (smu == kUndef || sb == kUndef || sc == kUndef || snu == kUndef) {
        ++mism;
        pv = kUndef;
      } else {
        const int r = (((smu + sb - sc - snu) % 3) + 3) % 3;
        if (r != orig) ++mism;
        pv = (r == 2) ? -1 : r;
      }
      if (flux) flux[(size_t)p * g.V + s] = (int8_t)pv;
    }
  }
  double maxu = sqrt(maxu2);
  // wave reduction (fixed butterfly), then a fixed-order pass over the 4 waves
  for (int off = 32; off > 0; off >>= 1) {
    KSum op = {__shfl_xor(kp.s, off), __shfl_xor(kp.c, off)};
    KSum oa = {__shfl_xor(ka.s, off), __shfl_xor(ka.c, off)};
    kmerge(kp, op);
    kmerge(ka, oa);
    maxu = fmax(maxu, __shfl_xor(maxu, off));
    mism += __shfl_xor(mism, off);
    undef += __shfl_xor(undef, off);
    nonfin += __shfl_xor(nonfin, off);
  }
  __shared__ Partial w[4];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    w[wave] = Partial{kp.s, kp.c, ka.s, ka.c, maxu, 0.0, mism, undef, nonfin, 0};
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Partial r = w[0];
    KSum a = {r.plaq_s, r.plaq_c}, bsum = {r.act_s, r.act_c};
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      kmerge(a, KSum{w[i].plaq_s, w[i].plaq_c});
      kmerge(bsum, KSum{w[i].act_s, w[i].act_c});
      r.max_unit = fmax(r.max_unit, w[i].max_unit);
      r.mism += w[i].mism;
      r.undef += w[i].undef;
      r.nonfin += w[i].nonfin;
    }
    r.plaq_s = a.s;
    r.plaq_c = a.c;
    r.act_s = bsum.s;
    r.act_c = bsum.c;
    part[blk] = r;
  }
}

// One block of 256: fixed-order reduction of the block partials into a record,
// plus the rejection counter (read, then cleared for the next interval).
template <typename R>
__global__ void __launch_bounds__(256) k_finalize(const Partial* __restrict__ part, uint32_t nparts,
                                                  double inv18v, double inv36v,
                                                  unsigned long long* rejected, VsmStatsDev* out,
                                                  long long sweep) {
  KSum a = {0.0, 0.0}, b = {0.0, 0.0};
  double mu = 0.0;
  long long mism = 0, undef = 0, nonfin = 0;
  for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x) {
    kmerge(a, KSum{part[i].plaq_s, part[i].plaq_c});
    kmerge(b, KSum{part[i].act_s, part[i].act_c});
    mu = fmax(mu, part[i].max_unit);
    mism += part[i].mism;
    undef += part[i].undef;
    nonfin += part[i].nonfin;
  }
  __shared__ Partial sh[256];
  sh[threadIdx.x] = Partial{a.s, a.c, b.s, b.c, mu, 0.0, mism, undef, nonfin, 0};
  __syncthreads();
  for (int stride = 128; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) {
      Partial& x = sh[threadIdx.x];
      const Partial& y = sh[threadIdx.x + stride];
      KSum pa = {x.plaq_s, x.plaq_c}, pb = {x.act_s, x.act_c};
      kmerge(pa, KSum{y.plaq_s, y.plaq_c});
      kmerge(pb, KSum{y.act_s, y.act_c});
      x.plaq_s = pa.s;
      x.plaq_c = pa.c;
      x.act_s = pb.s;
      x.act_c = pb.c;
      x.max_unit = fmax(x.max_unit, y.max_unit);
      x.mism += y.mism;
      x.undef += y.undef;
      x.nonfin += y.nonfin;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const Partial& r = sh[0];
    out->plaq = (r.plaq_s + r.plaq_c) * inv18v;
    out->action = (r.act_s + r.act_c) * inv36v;
    out->max_unitarity = r.max_unit;
    out->sweep = (double)sweep;
    out->flux_mismatch = r.mism;
    out->undefined_sector = r.undef;
    out->nonfinite = r.nonfin;
    if (rejected) {
      out->rejected = (long long)*rejected;
      *rejected = 0ull;
    } else {
      out->rejected = 0;
    }
  }
}

// ------------------------------------------------------------------ field strength

// The 1x1 clover C_{mu nu}(x) (internal directions dm, dn): the mean of the
// four plaquettes of the plane that start and end at x, each in the mu -> nu
// sense; FP64.  The first leaf is the plaquette P_{mu nu}(x) itself; wilson
// receives Re Tr[1 - P] of it.
template <typename R>
__device__ __forceinline__ M3<double> clover_at(const Geo& g, const void* links, const int c[4], int dm,
                                                int dn, double& wilson) {
  const DirBuf<R> bm = dir_buf<R>(links, g, dm), bn = dir_buf<R>(links, g, dn);
  auto at = [&](int a, int b) {
    int e[4] = {c[0], c[1], c[2], c[3]};
    e[dm] = wrap_add(e[dm], a, g.L[dm]);
    e[dn] = wrap_add(e[dn], b, g.L[dn]);
    return site_index(g, e);
  };
  auto F = [&](const M3<R>& r) { return mconvert<double>(full(r)); };
  // full 3x3 products: links stored in FP32 are unitary only to FP32 rounding,
  // so a row rebuilt from two others would not be the product's own.  The four
  // links of a leaf are loaded together.
  M3<double> C = mzero<double>();
  M3<double> t;
  {
    // U_mu(x) U_nu(x+mu) U_mu^dag(x+nu) U_nu^dag(x)
    const M3<R> a = ld_rows(bm, at(0, 0)), b = ld_rows(bn, at(1, 0)), c_ = ld_rows(bm, at(0, 1)),
                d = ld_rows(bn, at(0, 0));
    load_fence();
    t = mul_nn(F(a), F(b));
    t = mul_nd(t, F(c_));
    t = mul_nd(t, F(d));
  }
  wilson = (1.0 - t.a[0].re) + (1.0 - t.a[4].re) + (1.0 - t.a[8].re);
  maxpy(C, 0.25, t);
  {
    // U_nu(x) U_mu^dag(x-mu+nu) U_nu^dag(x-mu) U_mu(x-mu)
    const M3<R> a = ld_rows(bn, at(0, 0)), b = ld_rows(bm, at(-1, 1)), c_ = ld_rows(bn, at(-1, 0)),
                d = ld_rows(bm, at(-1, 0));
    load_fence();
    t = mul_nd(F(a), F(b));
    t = mul_nd(t, F(c_));
    t = mul_nn(t, F(d));
  }
  maxpy(C, 0.25, t);
  {
    // U_mu^dag(x-mu) U_nu^dag(x-mu-nu) U_mu(x-mu-nu) U_nu(x-nu)
    const M3<R> a = ld_rows(bn, at(-1, -1)), b = ld_rows(bm, at(-1, 0)), c_ = ld_rows(bm, at(-1, -1)),
                d = ld_rows(bn, at(0, -1));
    load_fence();
    t = madj(mul_nn(F(a), F(b)));
    t = mul_nn(t, F(c_));
    t = mul_nn(t, F(d));
  }
  maxpy(C, 0.25, t);
  {
    // U_nu^dag(x-nu) U_mu(x-nu) U_nu(x+mu-nu) U_mu^dag(x)
    const M3<R> a = ld_rows(bn, at(0, -1)), b = ld_rows(bm, at(0, -1)), c_ = ld_rows(bn, at(1, -1)),
                d = ld_rows(bm, at(0, 0));
    load_fence();
    t = mul_dn(F(a), F(b));
    t = mul_nn(t, F(c_));
    t = mul_nd(t, F(d));
  }
  maxpy(C, 0.25, t);
  return C;
}

// F = (C - C^dag) / (2i), Hermitian (no trace removed).
__device__ __forceinline__ M3<double> field_strength(const M3<double>& C) {
  M3<double> F;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const Cx<double> a = C.a[3 * i + j], b = C.a[3 * j + i];
      F.a[3 * i + j] = cx<double>(0.5 * (a.im + b.im), -0.5 * (a.re - b.re));
    }
  return F;
}

// Re Tr[F G].
__device__ __forceinline__ double retr_prod(const M3<double>& F, const M3<double>& G) {
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      r = fma(F.a[3 * i + j].re, G.a[3 * j + i].re, r);
      r = fma(-F.a[3 * i + j].im, G.a[3 * j + i].im, r);
    }
  return r;
}

struct ClovPartial {  // 80 bytes, the size of a measurement partial
  double sr_s, sr_c, q_s, q_c, s_s, s_c, pad[4];
};
static_assert(sizeof(ClovPartial) == 80, "clover partials share the measurement slots");

// Per site (Sec. V, Eqs. 1LFST, 1LTopQ; the reconstructed action of Sec. V.A):
// F for the six planes from the clover, S_R(x)/beta = (1/72) sum_{mu<nu}
// Tr[F F], q(x) = 1/(32 pi^2) eps Tr[F F] = (1/4 pi^2) Re Tr[F01 F23 - F02 F13
// + F03 F12] (user axes), and S(x)/beta = (2/72) sum_{mu<nu} Re Tr[1 - P]
// with P the first clover leaf.  Densities (canonical order) when asked for;
// fixed-slot block partials as in k_measure.
template <typename R>
__global__ void __launch_bounds__(256) k_clover(Geo g, const void* links, ClovPartial* __restrict__ part,
                                                double* __restrict__ sdens, double* __restrict__ qdens) {
  // sites in the order of k_measure
  const uint32_t blk = xcd_block();
  KSum ksr = {0.0, 0.0}, kq = {0.0, 0.0}, ks = {0.0, 0.0};
  int c[4];
  if (chunk_site(g, blk * 256u + threadIdx.x, c)) {
    double sr = 0.0, q = 0.0, sw = 0.0;
    // plane pairs (01, 23), (02, 13), (03, 12) with signs +, -, +; together
    // they visit all six planes once, so the Wilson density comes from the
    // first clover leaves
#pragma unroll 1
    for (int pr = 0; pr < 3; ++pr) {
      const int a0 = 0, a1 = pr + 1;
      const int b0 = pr == 0 ? 2 : 1, b1 = pr == 2 ? 2 : 3;
      double wa, wb;
      const M3<double> Fa = field_strength(clover_at<R>(g, links, c, g.perm[a0], g.perm[a1], wa));
      const M3<double> Fb = field_strength(clover_at<R>(g, links, c, g.perm[b0], g.perm[b1], wb));
      sr += retr_prod(Fa, Fa) + retr_prod(Fb, Fb);
      q += (pr == 1 ? -1.0 : 1.0) * retr_prod(Fa, Fb);
      sw += wa + wb;
    }
    const double norm = 1.0 / 72.0;
    sr *= norm;
    sw *= 2.0 * norm;
    q *= 1.0 / (4.0 * 3.14159265358979323846 * 3.14159265358979323846);
    kadd(ksr, sr);
    kadd(kq, q);
    kadd(ks, sw);
    const uint32_t s = canonical_index(g, c);
    if (sdens) sdens[s] = sw;
    if (qdens) qdens[s] = q;
  }
  for (int off = 32; off > 0; off >>= 1) {
    kmerge(ksr, KSum{__shfl_xor(ksr.s, off), __shfl_xor(ksr.c, off)});
    kmerge(kq, KSum{__shfl_xor(kq.s, off), __shfl_xor(kq.c, off)});
    kmerge(ks, KSum{__shfl_xor(ks.s, off), __shfl_xor(ks.c, off)});
  }
  __shared__ ClovPartial w[4];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) w[wave] = ClovPartial{ksr.s, ksr.c, kq.s, kq.c, ks.s, ks.c, {0, 0, 0, 0}};
  __syncthreads();
  if (threadIdx.x == 0) {
    KSum a = {w[0].sr_s, w[0].sr_c}, b = {w[0].q_s, w[0].q_c}, d = {w[0].s_s, w[0].s_c};
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      kmerge(a, KSum{w[i].sr_s, w[i].sr_c});
      kmerge(b, KSum{w[i].q_s, w[i].q_c});
      kmerge(d, KSum{w[i].s_s, w[i].s_c});
    }
    part[blk] = ClovPartial{a.s, a.c, b.s, b.c, d.s, d.c, {0, 0, 0, 0}};
  }
}

// Fixed-order reduction of the clover partials into {<S_R>/beta, Q, <S>/beta}.
template <typename R>
__global__ void __launch_bounds__(256) k_clover_finalize(const ClovPartial* __restrict__ part, uint32_t nparts,
                                                         double inv_v, double* out) {
  KSum a = {0.0, 0.0}, b = {0.0, 0.0}, d = {0.0, 0.0};
  for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x) {
    kmerge(a, KSum{part[i].sr_s, part[i].sr_c});
    kmerge(b, KSum{part[i].q_s, part[i].q_c});
    kmerge(d, KSum{part[i].s_s, part[i].s_c});
  }
  __shared__ KSum sh[3][256];
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = d;
  __syncthreads();
  for (int stride = 128; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride)
#pragma unroll
      for (int k = 0; k < 3; ++k) kmerge(sh[k][threadIdx.x], sh[k][threadIdx.x + stride]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = (sh[0][0].s + sh[0][0].c) * inv_v;
    out[1] = sh[1][0].s + sh[1][0].c;
    out[2] = (sh[2][0].s + sh[2][0].c) * inv_v;
    out[3] = 0.0;
  }
}

// ------------------------------------------------------------------ launchers

inline unsigned blocks_for(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename R>
void launch_set_links_t(const Geo& g, const void* canon, void* links, hipStream_t st) {
  hipLaunchKernelGGL(k_set_links<R>, dim3(blocks_for(4ull * g.V, 256)), dim3(256), 0, st, g,
                     (const double2*)canon, links);
}

template <typename R>
void launch_get_links_t(const Geo& g, const void* links, void* canon, hipStream_t st) {
  hipLaunchKernelGGL(k_get_links<R>, dim3(blocks_for(4ull * g.V, 256)), dim3(256), 0, st, g, links,
                     (double2*)canon);
}

template <typename R>
void launch_load_z3_t(const Geo& g, const int8_t* z3, void* links, hipStream_t st) {
  hipLaunchKernelGGL(k_load_z3<R>, dim3(blocks_for(4ull * g.V, 256)), dim3(256), 0, st, g, z3, links);
}

template <typename R>
void launch_centrifuge_t(const Geo& g, const int8_t* z3, const int8_t* pair, double omega, void* links,
                         int32_t* m_out, hipStream_t st) {
  hipLaunchKernelGGL(k_centrifuge<R>, dim3(blocks_for(4ull * g.V, 256)), dim3(256), 0, st, g, z3, pair,
                     omega, links, m_out);
}

template <typename R>
void launch_gauge_t(const Geo& g, void* links, const void* gauge, hipStream_t st) {
  hipLaunchKernelGGL(k_gauge<R>, dim3(blocks_for(4ull * g.V, 256)), dim3(256), 0, st, g, links,
                     (const double2*)gauge);
}

template <typename R, int MU>
void launch_update_mu(const Geo& g, const void* src, void* dst, const int8_t* z3, const void* gauge,
                      const UpdParams& p, int colour, int jacobi, unsigned long long* rej,
                      hipStream_t st) {
  const uint32_t n = jacobi ? g.V : g.V4;
  const unsigned nb = blocks_for(n, 256);
  const double2* gp = (const double2*)gauge;
  // Occupancy: fewer resident blocks per CU keep more of the links' reuse in
  // L2.  Dynamic LDS (160 KB per CU) caps the blocks per CU: 1 for FP64 (4
  // waves; the LDS is the staples' load ring), 2 for FP32 (8 waves, unused
  // LDS), the best measured on the 48^3x96 pass.
  const unsigned lds = p.oi ? (sizeof(R) == 8 ? kRingBytes<double> : 54u * 1024u) : 0u;
  if (p.oi) {
    if (p.update == 0)
      hipLaunchKernelGGL((k_update<R, MU, true, 0>), dim3(nb), dim3(256), lds, st, g, src, dst, z3, gp, p,
                         colour, jacobi, n, rej);
    else if (p.update == 1)
      hipLaunchKernelGGL((k_update<R, MU, true, 1>), dim3(nb), dim3(256), lds, st, g, src, dst, z3, gp, p,
                         colour, jacobi, n, rej);
    else
      hipLaunchKernelGGL((k_update<R, MU, true, 2>), dim3(nb), dim3(256), lds, st, g, src, dst, z3, gp, p,
                         colour, jacobi, n, rej);
  } else {
    if (p.update == 0)
      hipLaunchKernelGGL((k_update<R, MU, false, 0>), dim3(nb), dim3(256), lds, st, g, src, dst, z3, gp, p,
                         colour, jacobi, n, rej);
    else if (p.update == 1)
      hipLaunchKernelGGL((k_update<R, MU, false, 1>), dim3(nb), dim3(256), lds, st, g, src, dst, z3, gp, p,
                         colour, jacobi, n, rej);
    else
      hipLaunchKernelGGL((k_update<R, MU, false, 2>), dim3(nb), dim3(256), lds, st, g, src, dst, z3, gp, p,
                         colour, jacobi, n, rej);
  }
}

template <typename R>
void launch_update_t(const Geo& g, const void* src, void* dst, const int8_t* z3, const void* gauge,
                     const UpdParams& p, int mu, int colour, int jacobi, unsigned long long* rej,
                     hipStream_t st) {
  switch (mu) {
    case 0: launch_update_mu<R, 0>(g, src, dst, z3, gauge, p, colour, jacobi, rej, st); break;
    case 1: launch_update_mu<R, 1>(g, src, dst, z3, gauge, p, colour, jacobi, rej, st); break;
    case 2: launch_update_mu<R, 2>(g, src, dst, z3, gauge, p, colour, jacobi, rej, st); break;
    default: launch_update_mu<R, 3>(g, src, dst, z3, gauge, p, colour, jacobi, rej, st); break;
  }
}

template <typename R>
void launch_update_batch_t(const ServeJob* jobs, const BatchStep& step, uint32_t nblocks, hipStream_t st) {
  // the same cap on resident blocks per CU as for single-field passes (unused
  // dynamic LDS)
  const unsigned lds = sizeof(R) == 8 ? 96u * 1024u : 54u * 1024u;
  const uint32_t nb8 = (nblocks + 7u) & ~7u;
  hipLaunchKernelGGL(k_update_batch<R>, dim3(nb8), dim3(256), lds, st, jobs, step);
}

template <typename R>
void launch_serve_small_t(const ServeJob* jobs, const SmallStep& step, hipStream_t st) {
  if (step.njobs == 0) return;
  hipLaunchKernelGGL(k_serve_small<R>, dim3(step.njobs), dim3(kSmallThreads<R>), 0, st, jobs, step);
}

template <typename R, int MU>
void launch_flow_mu(const Geo& g, const void* src, void* dst, double* acc, int stage, double eps, double cp,
                    double cr, hipStream_t st) {
  const unsigned nb = blocks_for(g.V, 256);
  if (cr != 0.0) {
    const unsigned lds = sizeof(R) == 8 ? 96u * 1024u : 54u * 1024u;
    hipLaunchKernelGGL((k_flow<R, MU, true>), dim3(nb), dim3(256), lds, st, g, src, dst, acc, stage, eps, cp, cr);
  } else {
    hipLaunchKernelGGL((k_flow<R, MU, false>), dim3(nb), dim3(256), 0, st, g, src, dst, acc, stage, eps, cp, cr);
  }
}

template <typename R>
void launch_flow_t(const Geo& g, const void* src, void* dst, double* acc, int stage, double eps, double cp,
                   double cr, hipStream_t st) {
  launch_flow_mu<R, 0>(g, src, dst, acc, stage, eps, cp, cr, st);
  launch_flow_mu<R, 1>(g, src, dst, acc, stage, eps, cp, cr, st);
  launch_flow_mu<R, 2>(g, src, dst, acc, stage, eps, cp, cr, st);
  launch_flow_mu<R, 3>(g, src, dst, acc, stage, eps, cp, cr, st);
}

template <typename R>
void launch_clover_t(const Geo& g, const void* links, void* partials, double* out, double* sdens,
                     double* qdens, hipStream_t st) {
  const unsigned nb = blocks_for(g.V, 256);
  hipLaunchKernelGGL(k_clover<R>, dim3(nb), dim3(256), 0, st, g, links, (ClovPartial*)partials, sdens, qdens);
  hipLaunchKernelGGL(k_clover_finalize<R>, dim3(1), dim3(256), 0, st, (const ClovPartial*)partials, nb,
                     1.0 / (double)g.V, out);
}

template <typename R>
void launch_measure_t(const Geo& g, const void* links, const int8_t* z3, const void* gauge, void* partials,
                      int8_t* flux, unsigned long long* rej, VsmStatsDev* out, long long sweep, hipStream_t st) {
  const unsigned nb = blocks_for(g.V, 256);
  if (gauge)
    hipLaunchKernelGGL((k_measure<R, true>), dim3(nb), dim3(256), 0, st, g, links, z3, (const double2*)gauge,
                       (Partial*)partials, flux);
  else
    hipLaunchKernelGGL((k_measure<R, false>), dim3(nb), dim3(256), 0, st, g, links, z3, nullptr,
                       (Partial*)partials, flux);
  hipLaunchKernelGGL(k_finalize<R>, dim3(1), dim3(256), 0, st, (const Partial*)partials, nb,
                     1.0 / (18.0 * (double)g.V), 1.0 / (36.0 * (double)g.V), rej, out, sweep);
}

}  // namespace vsm
