// rowops.h -- the Metropolis update of one colour-c word (Sec. 2.2), shared
// by the per-lattice sweep kernel and the fused Monte Carlo step.
//
// The 2d "unsatisfied bond" words U = s_i ^ s_j ^ J_ij (bit set <=>
// J_ij s_i s_j = -1) are added bit-sliced into u = number of unsatisfied bonds
// of every site of the word.  With x = s_i h_i = 2d - 2u: u >= d (x <= 0)
// always flips; otherwise the site flips iff its Philox word r <
// thr[k][x/2 - 1].  The comparison results are gathered as bit planes C1
// (x = 2), C2 (x = 4), C3 (x = 6), so the flip word is
//   F = [u >= d] | [u = d-1] & C1 | [u = d-2] & C2 | [u = d-3] & C3.
// Three-input logic uses gfx950's v_bitop3_b32.
// Energy change per flip is 2x = 4(d - u), summed with popcounts.
#pragma once
#include "device.h"

namespace ptsg {

// jv: the word's 2d coupling words (colour c, direction-major).
template <int D>
__device__ __forceinline__ void sweep_word_j(const Geo& g, uint32_t* W, const uint32_t (&jv)[2 * D],
                                             int c, int w, int slot, int s, uint32_t tcount,
                                             uint32_t th2, uint32_t th4, uint32_t th6, int& dE,
                                             int* nflip = nullptr) {
  const WordNb q = word_nb(g, w);
  const int p = (c + q.par) & 1;
  const uint32_t* Wo = W + (1 - c) * g.NW;
  const uint32_t Wc = W[c * g.NW + w];
  uint32_t n[2 * D];
  neighbour_words<D>(g, Wo, w, q, p, n);
  // unsatisfied-bond words and their bit-sliced count u = 4 u2 + 2 u1 + u0
  const uint32_t U0 = bop3<kXor3>(Wc, n[0], jv[0]);
  const uint32_t U1 = bop3<kXor3>(Wc, n[1], jv[1]);
  const uint32_t U2 = bop3<kXor3>(Wc, n[2], jv[2]);
  const uint32_t U3 = bop3<kXor3>(Wc, n[3], jv[3]);
  uint32_t u0, u1, u2;
  if (D == 3) {
    const uint32_t U4 = bop3<kXor3>(Wc, n[4], jv[4]);
    const uint32_t U5 = bop3<kXor3>(Wc, n[5], jv[5]);
    const uint32_t s1 = bop3<kXor3>(U0, U1, U2), c1 = bop3<kMaj3>(U0, U1, U2);
    const uint32_t s2 = bop3<kXor3>(U3, U4, U5), c2 = bop3<kMaj3>(U3, U4, U5);
    u0 = s1 ^ s2;
    const uint32_t k = s1 & s2;
    u1 = bop3<kXor3>(c1, c2, k);
    u2 = bop3<kMaj3>(c1, c2, k);
  } else {
    const uint32_t s1 = bop3<kXor3>(U0, U1, U2), c1 = bop3<kMaj3>(U0, U1, U2);
    u0 = s1 ^ U3;
    const uint32_t k = s1 & U3;
    u1 = c1 ^ k;
    u2 = c1 & k;
  }

  // Comparison planes: one Philox call per four sites of a row field.  Bits
  // are shifted in from the top site of the top field down, so that bit
  // f*H + b ends up holding site b of field f.  In 3D the three nested
  // threshold tests come from two compares per site (shift_in_k_pair).
  uint32_t C1 = 0, C2 = 0, C3 = 0;  // 2D: [r < th2], [r < th4]; 3D: K1, K0 (below)
  const uint32_t c1w = 2u * tcount + (uint32_t)c;
  const uint32_t c3w = (kTagMetro << 28) | (uint32_t)s;
  if ((g.H & 3) == 0) {
    // every call serves four sites (L a multiple of 8): no partial groups
    for (int f = g.P - 1; f >= 0; --f) {
      const uint32_t R = (uint32_t)word_row(g, q, f);
      for (int grp = g.G - 1; grp >= 0; --grp) {
        const Ctr4 r = philox10_u(Ctr4{R * (uint32_t)g.G + (uint32_t)grp, c1w, (uint32_t)slot, c3w},
                                g.key0, g.key1);
        if (D == 3) {
          shift_in_k_pair(C1, C2, r.w, r.z, th2, th4, th6);
          shift_in_k_pair(C1, C2, r.y, r.x, th2, th4, th6);
        } else {
          C1 = shift_in_less(C1, r.w, th2);
          C2 = shift_in_less(C2, r.w, th4);
          C1 = shift_in_less(C1, r.z, th2);
          C2 = shift_in_less(C2, r.z, th4);
          C1 = shift_in_less(C1, r.y, th2);
          C2 = shift_in_less(C2, r.y, th4);
          C1 = shift_in_less(C1, r.x, th2);
          C2 = shift_in_less(C2, r.x, th4);
        }
      }
    }
  } else {
  for (int f = g.P - 1; f >= 0; --f) {
    const uint32_t R = (uint32_t)word_row(g, q, f);
    for (int grp = g.G - 1; grp >= 0; --grp) {
      const Ctr4 r = philox10_u(Ctr4{R * (uint32_t)g.G + (uint32_t)grp, c1w, (uint32_t)slot, c3w},
                              g.key0, g.key1);
      const int nv = g.H - 4 * grp;  // sites of this row field served by the call
      if (D == 3) {
        if (nv >= 4) {
          shift_in_k_pair(C1, C2, r.w, r.z, th2, th4, th6);
        } else if (nv == 3) {
          shift_in_k_one(C1, C2, r.z, th2, th4, th6);
        }
        if (nv >= 2)
          shift_in_k_pair(C1, C2, r.y, r.x, th2, th4, th6);
        else
          shift_in_k_one(C1, C2, r.x, th2, th4, th6);
      } else {
        if (nv >= 4) {
          C1 = shift_in_less(C1, r.w, th2);
          C2 = shift_in_less(C2, r.w, th4);
        }
        if (nv >= 3) {
          C1 = shift_in_less(C1, r.z, th2);
          C2 = shift_in_less(C2, r.z, th4);
        }
        if (nv >= 2) {
          C1 = shift_in_less(C1, r.y, th2);
          C2 = shift_in_less(C2, r.y, th4);
        }
        C1 = shift_in_less(C1, r.x, th2);
        C2 = shift_in_less(C2, r.x, th4);
      }
    }
  }
  }
  if (D == 3) {
    // K1 = [r < th4] and K0 as above: [r < th2] = K1 | K0, [r < th6] = K1 & K0
    const uint32_t K1 = C1, K0 = C2;
    C1 = K1 | K0;
    C2 = K1;
    C3 = K1 & K0;
  }

  // Truth tables over (u2, u1, u0) are indexed by u itself.  The planes are
  // nested (th6 <= th4 <= th2, so C3 <= C2 <= C1), hence
  //   3D: F = [u>=3] | [u>=2] & C1 | [u>=1] & C2 | C3
  //   2D: F = [u>=2] | [u>=1] & C1 | C2
  uint32_t F;
  if (D == 3) {
    const uint32_t A = bop3<0xF8>(u2, u1, u0);
    const uint32_t G1 = bop3<0xFC>(u2, u1, u0);
    const uint32_t G2 = bop3<0xFE>(u2, u1, u0);
    F = bop3<kAndOr>(G2, C2, bop3<kAndOr>(G1, C1, A | C3)) & g.maskW;
  } else {
    const uint32_t A = bop3<0xFC>(u2, u1, u0);
    const uint32_t G1 = bop3<0xFE>(u2, u1, u0);
    F = bop3<kAndOr>(G1, C1, A | C2) & g.maskW;
  }
  dE += 4 * (D * __popc(F) - (__popc(F & u0) + 2 * __popc(F & u1) + 4 * __popc(F & u2)));
  if (nflip) *nflip += __popc(F);
  W[c * g.NW + w] = Wc ^ F;
}

// The same with the coupling words loaded here (their loads overlap the
// neighbour loads).
template <int D>
__device__ __forceinline__ void sweep_word(const Geo& g, uint32_t* W, const uint32_t* __restrict__ jw,
                                           int c, int w, int slot, int s, uint32_t tcount,
                                           uint32_t th2, uint32_t th4, uint32_t th6, int& dE,
                                           int* nflip = nullptr) {
  const size_t js = (size_t)g.NW;
  uint32_t jv[2 * D];
#pragma unroll
  for (int dir = 0; dir < 2 * D; ++dir) jv[dir] = jw[dir * js + w];
  sweep_word_j<D>(g, W, jv, c, w, slot, s, tcount, th2, th4, th6, dE, nflip);
}

// Number of unsatisfied bonds of the colour-0 word w (every bond has exactly
// one colour-0 end when L is even).  jw0 = the colour-0 direction words.
template <int D>
__device__ __forceinline__ int unsatisfied_word(const Geo& g, const uint32_t* W,
                                                const uint32_t* __restrict__ jw0, int w) {
  const WordNb q = word_nb(g, w);
  const int p = q.par;  // p(0, word)
  uint32_t n[2 * D];
  neighbour_words<D>(g, W + g.NW, w, q, p, n);
  const uint32_t Wc = W[w];
  int u = 0;
#pragma unroll
  for (int dir = 0; dir < 2 * D; ++dir) u += __popc(Wc ^ n[dir] ^ jw0[(size_t)dir * g.NW + w]);
  return u;
}

}  // namespace ptsg
