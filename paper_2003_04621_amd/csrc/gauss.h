// gauss.h -- the Edwards-Anderson model with Gaussian couplings (Sec. 2.1:
// couplings drawn from a standard normal distribution; the 2D Gaussian
// workload of Sec. 4.2), device side shared by the Gaussian kernels.
//
// Couplings live on a fixed-point grid, J = n 2^-16 with |n| <= 2^19 (the
// float32 values the caller passes must lie on it), and are held as the
// integers n.  Local fields and energies are then exact integers of 2^-16
// units whatever the summation order, and the chain is decided by integer
// data plus one real comparison per move: a Metropolis flip with energy
// change dE > 0 (or an exchange with D > 0) is accepted iff the move's 32-bit
// Philox word r satisfies r < 2^32 exp(-beta dE 2^-16) (Eq. (5) and the
// Metropolis rule of Sec. 2.2, with beta the inverse temperature or the
// difference of the two inverse temperatures).  That comparison is decided
// exactly, in three tiers: float32 with a certified error margin, then
// double, then double-double (about 2^-98 relative), each tier deciding only
// where its error bound cannot change the answer.
//
// Per-site coupling data, grouped by the four same-colour sites of one
// Philox call (group gi of colour c: word w = gi mod NW, field f and group q
// of that field from gi / NW = f Gp + q, sites b = 4q + j, j < 4, of field f;
// Gp = ceil(H/4)): int4 Jg[S][2][2d+1][NGc], entry k < 2d the value -2 n of
// the bond in direction k (+x0, -x0, +x1, -x1, +x2, -x2) of each of the four
// sites, entry 2d the sum of the site's 2d couplings.  With a_k = 1 where
// the site and its neighbour in direction k are antiparallel,
// x = s_i h_i = sum_k n_k (1 - 2 a_k) = Hs + sum_k a_k (-2 n_k).
#pragma once
#include "device.h"

namespace ptsg {

constexpr int kGaussUnitBits = 16;       // J = n 2^-16
constexpr int32_t kGaussMaxUnits = 1 << 19;  // |J| <= 8

// Groups of four same-colour sites per colour of a lattice.
__host__ __device__ constexpr int gauss_groups(const Geo& g) {
  return g.NW * g.P * ((g.H + 3) / 4);
}

// ---------------------------------------------------------------------------
// Double-double arithmetic (Dekker's error-free sum and product; the product
// through a fused multiply-add).
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};
__host__ __device__ inline dd dd_two_sum(double a, double b) {
  const double s = a + b, bb = s - a;
  return dd{s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ inline dd dd_fast_sum(double a, double b) {  // |a| >= |b|
  const double s = a + b;
  return dd{s, b - (s - a)};
}
__host__ __device__ inline dd dd_two_prod(double a, double b) {
  const double p = a * b;
  return dd{p, fma(a, b, -p)};
}
__host__ __device__ inline dd dd_add(dd a, dd b) {
  dd s = dd_two_sum(a.hi, b.hi);
  const dd t = dd_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_fast_sum(s.hi, s.lo);
  s.lo += t.lo;
  return dd_fast_sum(s.hi, s.lo);
}
__host__ __device__ inline dd dd_mul(dd a, dd b) {
  dd p = dd_two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return dd_fast_sum(p.hi, p.lo);
}
__host__ __device__ inline dd dd_mul_d(dd a, double b) {
  dd p = dd_two_prod(a.hi, b);
  p.lo += a.lo * b;
  return dd_fast_sum(p.hi, p.lo);
}
// a / b for a double b: the quotient's leading part, then the exact remainder
// divided once more.
__host__ __device__ inline dd dd_div_d(dd a, double b) {
  const double q1 = a.hi / b;
  const dd p = dd_two_prod(q1, b);
  const double r = ((a.hi - p.hi) - p.lo) + a.lo;
  return dd_fast_sum(q1, r / b);
}

// ln 2 as a double-double (the double nearest ln 2 and the remainder).
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;
constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;

// r < 2^32 exp(-b u 2^-16) for b > 0 and u > 0, in double-double: y = b u
// 2^-16 exactly (an error-free product, then a power-of-two scale), reduced
// as y = k ln 2 + f with |f| <= ln(2)/2 + 2^-40, exp(-f) by its Taylor series
// (24 terms, Horner form; the remainder is below 2^-110), and t = exp(-f)
// 2^(32 - k).  r = 0 is always accepted (t > 0); for r >= 1 acceptance needs
// t > 1, i.e. y < 32 ln 2 = 22.18...
__host__ __device__ inline bool gauss_accept_dd(uint32_t r, double b, int64_t u) {
  if (r == 0u) return true;
  dd y = dd_two_prod(b, (double)u);
  y.hi *= 0x1p-16;
  y.lo *= 0x1p-16;
  if (y.hi > 22.25) return false;
  const int k = (int)rint(y.hi / kLn2Hi);
  const dd f = dd_add(y, dd_mul_d(dd{-kLn2Hi, -kLn2Lo}, (double)k));
  const dd mf{-f.hi, -f.lo};
  dd s{1.0, 0.0};
  for (int n = 24; n >= 1; --n) s = dd_add(dd{1.0, 0.0}, dd_div_d(dd_mul(s, mf), (double)n));
  s.hi = ldexp(s.hi, 32 - k);
  s.lo = ldexp(s.lo, 32 - k);
  // r < s.hi + s.lo  <=>  r - s.hi < s.lo; the difference is exact where it
  // matters (Sterbenz) and has the right sign elsewhere.
  return (double)r - s.hi < s.lo;
}

// The float32 tier's per-temperature constant, b log2(e) 2^-16 rounded to
// float (host and device compute it with the same double operations).
__host__ __device__ inline float gauss_cz(double b) {
  return (float)(b * 1.4426950408889634 / 65536.0);
}

// The double tier: y = b u 2^-16 rounded once (relative error 2^-53), exp in
// double (within a few ulp); together well inside the 2^-40 margin.  Cases
// inside the margin go to the double-double tier.
__device__ inline bool gauss_accept_d(uint32_t r, double b, int64_t u) {
  const double y = b * (double)u * 0x1p-16;
  if (y > 22.25) return r == 0u;
  const double t = ldexp(exp(-y), 32);
  const double rd = (double)r;
  if (rd < t * (1.0 - 0x1p-40)) return true;
  if (rd > t * (1.0 + 0x1p-40)) return false;
  return gauss_accept_dd(r, b, u);
}

// The Metropolis decision for u = 2x energy units (2 <= u < 2^24), with
// cz = float(b log2(e) 2^-16) from the host: z = u cz carries a relative
// error below 2^-23, so for z < 33 the float32 threshold 2^32 2^-z
// (v_exp_f32) is within 2^-18 of the true one; a word outside a 2^-15 band
// around it is decided here, the rest by the double tier.  For z >= 33 the
// threshold is below 1 and only r = 0 accepts.
// The float32 tier alone, without branches: 1 accept, 0 reject, -1
// undecided (inside the band).  For z >= 33 the threshold is below 1/2 (or
// flushed to 0): every r >= 1 is rejected and r = 0 is accepted or, if the
// threshold underflowed, left to the double tier, which accepts it.
__device__ __forceinline__ int gauss_metro_f32(uint32_t r, float cz, uint32_t u) {
  const float z = (float)u * cz;
  const float t = __builtin_amdgcn_exp2f(-z) * 4294967296.0f;
  const float rf = (float)r;
  return rf < t * (1.0f - 0x1p-15f) ? 1 : (rf > t * (1.0f + 0x1p-15f) ? 0 : -1);
}
__device__ inline bool gauss_accept_metro(uint32_t r, float cz, double b, uint32_t u) {
  const int f = gauss_metro_f32(r, cz, u);
  return f >= 0 ? f != 0 : gauss_accept_d(r, b, (int64_t)u);
}

// ---------------------------------------------------------------------------
// Site groups of the Gaussian kernels.
// ---------------------------------------------------------------------------
// Decodes group gi of a colour: word w, field f, group q.
struct GroupPos {
  int w, f, q, shift, nv;
};
__device__ __forceinline__ GroupPos group_pos(const Geo& g, int gi) {
  const int Gp = (g.H + 3) / 4;
  GroupPos p;
  p.w = gi % g.NW;
  const int fg = gi / g.NW;
  p.f = fg / Gp;
  p.q = fg - p.f * Gp;
  p.shift = p.f * g.H + 4 * p.q;
  p.nv = min(4, g.H - 4 * p.q);
  return p;
}

__device__ __forceinline__ int lane_of(const int4& v, int j) {
  return j == 0 ? v.x : j == 1 ? v.y : j == 2 ? v.z : v.w;
}
__device__ __forceinline__ uint32_t word_of(const Ctr4& v, int j) {
  return j == 0 ? v.x : j == 1 ? v.y : j == 2 ? v.z : v.w;
}

// Bit j of a sign-extended to a mask (0 or -1), one v_bfe_i32.  Written as
// an instruction so that the compiler keeps the mask-and-add form (its own
// canonical form, a compare and a select per term, costs one more).
template <int J>
__device__ __forceinline__ int bit_mask(uint32_t a) {
  int r;
  asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(r) : "v"(a), "i"(J));
  return r;
}

// x = s_i h_i of the four sites of a group from the antiparallel words a[k]
// (already shifted to the group) and the group's coupling data: bit j of a[k]
// as a mask selects the term.
template <int D>
__device__ __forceinline__ void group_fields(const uint32_t (&a)[2 * D], const int4 (&m)[2 * D],
                                             const int4& hs, int (&x)[4]) {
  x[0] = hs.x;
  x[1] = hs.y;
  x[2] = hs.z;
  x[3] = hs.w;
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) {
    x[0] += m[k].x & bit_mask<0>(a[k]);
    x[1] += m[k].y & bit_mask<1>(a[k]);
    x[2] += m[k].z & bit_mask<2>(a[k]);
    x[3] += m[k].w & bit_mask<3>(a[k]);
  }
}

// The Metropolis decisions of one group of four same-colour sites (the first
// nv valid) whose Philox words are r, in two parts so that a caller can
// interleave two groups: gauss_group_fast computes the local fields and the
// float32 tier for the four sites without branches (x <= 0 flips at once):
// the flip bits F and the undecided bits und; gauss_group_finish decides the
// rare undecided sites by the exact tiers and adds the flips' energy change
// 2x to dE.
template <int D>
__device__ __forceinline__ void gauss_group_fast(const uint32_t (&a)[2 * D], const int4 (&m)[2 * D],
                                                 const int4& hs, int nv, const Ctr4& r, float cz,
                                                 int (&x)[4], uint32_t& F, uint32_t& und) {
  group_fields<D>(a, m, hs, x);
  F = 0;
  und = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int xj = x[j];
    int f = gauss_metro_f32(word_of(r, j), cz, 2u * (uint32_t)(xj > 0 ? xj : 0));
    f = xj <= 0 ? 1 : f;
    f = j < nv ? f : 0;
    F |= (uint32_t)(f > 0) << j;
    und |= (uint32_t)(f < 0) << j;
  }
}
__device__ __forceinline__ uint32_t gauss_group_finish(const int (&x)[4], const Ctr4& r, double beta,
                                                       uint32_t F, uint32_t und, int& dE) {
  while (und) {
    const int j = __builtin_ctz(und);
    und &= und - 1u;
    if (gauss_accept_d(word_of(r, j), beta, (int64_t)(2 * x[j]))) F |= 1u << j;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) dE += ((F >> j) & 1u) ? 2 * x[j] : 0;
  return F;
}
template <int D>
__device__ __forceinline__ uint32_t gauss_group_flips(const uint32_t (&a)[2 * D], const int4 (&m)[2 * D],
                                                      const int4& hs, int nv, const Ctr4& r, float cz,
                                                      double beta, int& dE) {
  int x[4];
  uint32_t F, und;
  gauss_group_fast<D>(a, m, hs, nv, r, cz, x, F, und);
  return gauss_group_finish(x, r, beta, F, und, dE);
}

// Energy change of replica a when the cluster C (both colours' words) is
// exchanged with replica b: the sum over bonds leaving C of 2 n s_i^a s_j^a,
// taken from the colour-0 end of every bond (with m = -2n, m (2 a - 1) where a
// = 1 if the bond's two spins of replica a are antiparallel).  Threads t of T
// share the groups; each returns its part.
template <int D>
__device__ inline int64_t gauss_cluster_delta(const Geo& g, const uint32_t* C, const uint32_t* A,
                                              const int4* __restrict__ J0, int t, int T) {
  const int NW = g.NW, NGc = gauss_groups(g);
  int64_t dl = 0;
  for (int gi = t; gi < NGc; gi += T) {
    const GroupPos gp = group_pos(g, gi);
    const WordNb nb = word_nb(g, gp.w);
    const uint32_t vmask = (1u << gp.nv) - 1u;
    uint32_t nc[2 * D], X[2 * D];
    neighbour_words<D>(g, C + NW, gp.w, nb, nb.par, nc);
    const uint32_t C0 = C[gp.w];
    uint32_t any = 0;
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
      X[k] = ((C0 ^ nc[k]) >> gp.shift) & vmask;
      any |= X[k];
    }
    if (!any) continue;
    uint32_t na[2 * D];
    neighbour_words<D>(g, A + NW, gp.w, nb, nb.par, na);
    const uint32_t A0 = A[gp.w];
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
      if (!X[k]) continue;
      const uint32_t a = (A0 ^ na[k]) >> gp.shift;
      const int4 m = J0[(size_t)k * NGc + gi];
      for (int j = 0; j < 4; ++j)
        if ((X[k] >> j) & 1u) dl += ((a >> j) & 1u) ? lane_of(m, j) : -lane_of(m, j);
    }
  }
  return dl;
}

// (hi, lo) += (vhi, vlo) as one 128-bit integer held in two int64 words.
__device__ __forceinline__ void add128(int64_t* lo, int64_t* hi, uint64_t vlo, uint64_t vhi) {
  const uint64_t l = (uint64_t)*lo + vlo;
  *lo = (int64_t)l;
  *hi = (int64_t)((uint64_t)*hi + vhi + (l < vlo ? 1u : 0u));
}

}  // namespace ptsg
