// rowops.h -- the Metropolis update of one colour-c row word (Sec. 2.2),
// shared by the per-lattice sweep kernel and the fused Monte Carlo step.
//
// Per row word (H = L/2 sites of one colour) the 2d "unsatisfied bond" words
// U = s_i ^ s_j ^ J_ij (bit set <=> J_ij s_i s_j = -1) are added bit-sliced
// into u = number of unsatisfied bonds.  With x = s_i h_i = 2d - 2u: u >= d
// (x <= 0) always flips; otherwise the site flips iff its Philox word
// r < thr[k][x/2 - 1].  The comparison results are gathered as bit planes C1
// (x = 2), C2 (x = 4), C3 (x = 6), so the flip word is
//   F = [u >= d] | [u = d-1] & C1 | [u = d-2] & C2 | [u = d-3] & C3.
// Energy change per flip is 2x = 4(d - u), summed with popcounts.
#pragma once
#include "device.h"

namespace ptsg {

template <int D>
__device__ __forceinline__ void sweep_row(const Geo& g, uint32_t* W, const uint32_t* __restrict__ jw,
                                          int c, int R, int slot, int s, uint32_t tcount,
                                          uint32_t th2, uint32_t th4, uint32_t th6, int& dE) {
  const RowNb q = row_nb(g, R);
  const int p = (c + q.x1 + q.x2) & 1;
  const uint32_t* Wo = W + (1 - c) * g.NR;
  const uint32_t Wc = W[c * g.NR + R];
  uint32_t n0, n1;
  x0_neighbours(g, Wo[R], p, n0, n1);
  const size_t js = (size_t)g.NR;
  const uint32_t U0 = Wc ^ n0 ^ jw[0 * js + R];
  const uint32_t U1 = Wc ^ n1 ^ jw[1 * js + R];
  const uint32_t U2 = Wc ^ Wo[q.r1p] ^ jw[2 * js + R];
  const uint32_t U3 = Wc ^ Wo[q.r1m] ^ jw[3 * js + R];

  uint32_t u0, u1, u2;
  if (D == 3) {
    const uint32_t U4 = Wc ^ Wo[q.r2p] ^ jw[4 * js + R];
    const uint32_t U5 = Wc ^ Wo[q.r2m] ^ jw[5 * js + R];
    const uint32_t t1 = U0 ^ U1, s1 = t1 ^ U2, c1 = (U0 & U1) | (U2 & t1);
    const uint32_t t2 = U3 ^ U4, s2 = t2 ^ U5, c2 = (U3 & U4) | (U5 & t2);
    u0 = s1 ^ s2;
    const uint32_t k = s1 & s2, t3 = c1 ^ c2;
    u1 = t3 ^ k;
    u2 = (c1 & c2) | (k & t3);
  } else {
    const uint32_t t1 = U0 ^ U1, s1 = t1 ^ U2, c1 = (U0 & U1) | (U2 & t1);
    u0 = s1 ^ U3;
    const uint32_t k = s1 & U3;
    u1 = c1 ^ k;
    u2 = c1 & k;
  }

  // comparison planes, one Philox call per four sites of the row word
  uint32_t C1 = 0, C2 = 0, C3 = 0;
  const uint32_t c1w = 2u * tcount + (uint32_t)c;
  const uint32_t c3w = (kTagMetro << 28) | (uint32_t)s;
  for (int grp = 0; grp < g.G; ++grp) {
    const Ctr4 r = philox10(Ctr4{(uint32_t)(R * g.G + grp), c1w, (uint32_t)slot, c3w}, g.key0, g.key1);
    const uint32_t b1 = (uint32_t)(r.x < th2) | ((uint32_t)(r.y < th2) << 1) |
                        ((uint32_t)(r.z < th2) << 2) | ((uint32_t)(r.w < th2) << 3);
    const uint32_t b2 = (uint32_t)(r.x < th4) | ((uint32_t)(r.y < th4) << 1) |
                        ((uint32_t)(r.z < th4) << 2) | ((uint32_t)(r.w < th4) << 3);
    C1 |= b1 << (4 * grp);
    C2 |= b2 << (4 * grp);
    if (D == 3) {
      const uint32_t b3 = (uint32_t)(r.x < th6) | ((uint32_t)(r.y < th6) << 1) |
                          ((uint32_t)(r.z < th6) << 2) | ((uint32_t)(r.w < th6) << 3);
      C3 |= b3 << (4 * grp);
    }
  }

  uint32_t F;
  if (D == 3) {
    const uint32_t A = u2 | (u1 & u0);
    const uint32_t T0 = u1 & ~u0 & ~u2;
    const uint32_t T1 = u0 & ~u1 & ~u2;
    const uint32_t T2 = ~(u0 | u1 | u2);
    F = (A | (T0 & C1) | (T1 & C2) | (T2 & C3)) & g.maskH;
  } else {
    const uint32_t A = u1 | u2;
    const uint32_t T0 = u0 & ~A;
    const uint32_t T1 = ~u0 & ~A;
    F = (A | (T0 & C1) | (T1 & C2)) & g.maskH;
  }
  dE += 4 * (D * __popc(F) - (__popc(F & u0) + 2 * __popc(F & u1) + 4 * __popc(F & u2)));
  W[c * g.NR + R] = Wc ^ F;
}

}  // namespace ptsg
