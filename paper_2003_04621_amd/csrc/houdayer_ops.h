// houdayer_ops.h -- word operations of the Houdayer cluster move (Sec. 2.4,
// Eq. (10)) shared by the per-pair kernel and the fused Monte Carlo step.
// Q = overlap words (bit set <=> q_i = -1), C = cluster words, A = replica a;
// each is 2*NW words, colour c at offset c*NW.
#pragma once
#include "device.h"

namespace ptsg {

// Number of q = -1 sites in row R.
__device__ __forceinline__ uint32_t row_minus_count(const Geo& g, const uint32_t* Q, int R) {
  int w, f;
  row_word(g, R, w, f);
  return __popc((Q[w] >> (f * g.H)) & g.maskH) + __popc((Q[g.NW + w] >> (f * g.H)) & g.maskH);
}

// Plants the seed: the q = -1 site of rank m (increasing site order) among
// rows [r_begin, r_end) becomes the only cluster bit.
__device__ __forceinline__ void seed_in_rows(const Geo& g, const uint32_t* Q, uint32_t* C, int r_begin,
                                             int r_end, uint32_t m) {
  for (int R = r_begin; R < r_end; ++R) {
    const uint32_t cr = row_minus_count(g, Q, R);
    if (m >= cr) {
      m -= cr;
      continue;
    }
    int w, f, c, b;
    row_word(g, R, w, f);
    select_in_row(g, R, Q[w], Q[g.NW + w], f, m, c, b);
    if (c >= 0) C[c * g.NW + w] = 1u << (f * g.H + b);
    return;
  }
}

// One flood-fill update of the colour-c cluster word w; true if it grew.
template <int D>
__device__ __forceinline__ bool grow_word(const Geo& g, uint32_t* C, const uint32_t* Q, int c, int w) {
  const uint32_t qw = Q[c * g.NW + w];
  if (!qw) return false;
  const WordNb q = word_nb(g, w);
  const int p = (c + q.par) & 1;
  uint32_t n[2 * D];
  neighbour_words<D>(g, C + (1 - c) * g.NW, w, q, p, n);
  uint32_t nb = n[0] | n[1] | n[2] | n[3];
  if (D == 3) nb |= n[4] | n[5];
  const uint32_t old = C[c * g.NW + w];
  const uint32_t nw = old | (qw & nb);
  if (nw == old) return false;
  C[c * g.NW + w] = nw;
  return true;
}

// Energy change of replica a from negating it on the cluster: 2 J_ij s_i s_j
// summed over the bonds leaving the cluster, from the colour-0 word w.
template <int D>
__device__ __forceinline__ int cluster_delta_word(const Geo& g, const uint32_t* C, const uint32_t* A,
                                                  const uint32_t* __restrict__ jw0, int w) {
  const WordNb q = word_nb(g, w);
  const int p = q.par;  // p(0, word)
  uint32_t nc[2 * D], na[2 * D];
  neighbour_words<D>(g, C + g.NW, w, q, p, nc);
  neighbour_words<D>(g, A + g.NW, w, q, p, na);
  const uint32_t C0 = C[w], A0 = A[w];
  int cross = 0, cross_u = 0;
#pragma unroll
  for (int dir = 0; dir < 2 * D; ++dir) {
    const uint32_t X = C0 ^ nc[dir];
    const uint32_t U = A0 ^ na[dir] ^ jw0[(size_t)dir * g.NW + w];
    cross += __popc(X);
    cross_u += __popc(X & U);
  }
  return 2 * (cross - 2 * cross_u);
}

}  // namespace ptsg
