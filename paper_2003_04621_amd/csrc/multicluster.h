// multicluster.h -- the multi-cluster variant of the Houdayer move (Sec. 3 and
// Sec. 5 propose it to remove the load imbalance of single clusters): every
// nearest-neighbour cluster of q = -1 sites of a pair is exchanged,
// independently, with probability 1/2.  A cluster is named by its lowest
// site m (site i = x0 + L x1 + L^2 x2) and is exchanged iff bit m mod 128 of
// the Philox output for counter (m / 128, v, k, 6 << 28 | sample) is set (bit
// j = bit j mod 32 of word j / 32).
//
// Connected components by union-find over a team of threads (one wavefront
// in the fused step, one workgroup in the per-pair kernel), with a 32-bit
// parent label per site in LDS, natural site order:
//   1. each row's q = -1 sites form runs along x0 (periodically); every site
//      starts pointing at its run's lowest site, the run's root;
//   2. every pair of runs overlapping along x1 (or x2) is united once, at the
//      first site of each overlap segment: the two roots are found (following
//      parents, each step also pointing the site passed at its grandparent)
//      and the larger is hooked under the smaller with an LDS atomic minimum;
//      if it had been hooked meanwhile, its new parent's root is united next;
//   3. every site takes its root, which is then its component's lowest site
//      (parents only ever point to lower sites of the same component, and
//      nothing hooks a component's lowest site);
//   4. the coins of all sites (one Philox call per 128 sites) and, for each
//      q = -1 site, the coin of its root give the exchanged sites.
// Concurrent finds and hooks only ever replace a parent by a lower ancestor
// in the same component, so every value read is valid and every find ends.
#pragma once
#include "device.h"

namespace ptsg {

constexpr uint32_t kTagHouMulti = 6u;

// Sites a team's labels can name (the per-pair kernel's LDS holds them).
constexpr int kMultiMaxSites = 32768;

// LDS words of one team's scratch for geometry g: overlap and cluster words
// (2 NW each), row masks (64-bit per row), coins (one bit per site, 128-bit
// blocks) and labels (32-bit per site).
__host__ __device__ constexpr int multi_scratch_words(int N, int NR, int NW) {
  return 4 * NW + 2 * NR + 4 * ((N + 127) / 128) + N;
}

// Bit b of x moved to bit 2b (x < 2^32).
__device__ __forceinline__ uint64_t spread_bits(uint32_t x) {
  uint64_t v = x;
  v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
  v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
  v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  v = (v | (v << 1)) & 0x5555555555555555ull;
  return v;
}

// The q = -1 sites of row R as an L-bit mask in x0 order.
__device__ __forceinline__ uint64_t row_q_mask(const Geo& g, const uint32_t* Q, int R) {
  int w, f;
  row_word(g, R, w, f);
  const int p0 = row_parity(g, R);  // colour of the even-x0 sites
  const uint32_t e = (Q[p0 * g.NW + w] >> (f * g.H)) & g.maskH;
  const uint32_t o = (Q[(1 - p0) * g.NW + w] >> (f * g.H)) & g.maskH;
  return spread_bits(e) | (spread_bits(o) << 1);
}

// Rows next to row R in the positive x1 and (3D) x2 directions.
__device__ __forceinline__ void rows_up(const Geo& g, int R, int* up) {
  if (g.d == 3) {
    const int x2 = (int)divL(g, (uint32_t)R), x1 = R - x2 * g.L;
    up[0] = x1 == g.L - 1 ? R - (g.L - 1) : R + 1;
    up[1] = x2 == g.L - 1 ? R - (g.L - 1) * g.L : R + g.L;
  } else {
    up[0] = R == g.L - 1 ? 0 : R + 1;
  }
}

// Root of site x: follows parents (each lower than its child; a root is its
// own parent), pointing every site passed at its grandparent.
__device__ __forceinline__ uint32_t uf_root(uint32_t* lab, uint32_t x) {
  uint32_t cur = lab[x];
  if (cur != x) {
    uint32_t prev = x, next;
    while (cur > (next = lab[cur])) {
      lab[prev] = next;
      prev = cur;
      cur = next;
    }
  }
  return cur;
}

// Unites the components of sites i and j.
__device__ __forceinline__ void uf_unite(uint32_t* lab, uint32_t i, uint32_t j) {
  uint32_t a = uf_root(lab, i), b = uf_root(lab, j);
  while (a != b) {
    if (a > b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    const uint32_t old = atomicMin(&lab[b], a);  // hooks b under a if b is still a root
    if (old == b) break;
    b = uf_root(lab, old);
    a = uf_root(lab, a);
  }
}

// The exchanged sites of one multi-cluster move of the pair whose overlap
// words are Q (bit set: q = -1) as colour words C (2 NW), by the team's
// threads t < T.  scr: the team's scratch after Q and C (row masks, coins,
// labels; 8-byte aligned).  `sync` orders the team's LDS accesses.
template <int D, typename Sync>
__device__ __forceinline__ void multi_cluster_words(const Geo& g, const uint32_t* Q, uint32_t* C,
                                                    uint32_t* scr, int s, int k, uint32_t v,
                                                    int t, int T, Sync sync) {
  const int L = g.L, NR = g.NR, N = g.N, NW = g.NW;
  const int nblk = (N + 127) / 128;
  uint64_t* qr = reinterpret_cast<uint64_t*>(scr);
  uint32_t* coin = scr + 2 * NR;
  uint32_t* lab = coin + 4 * nblk;
  const uint64_t full = L == 64 ? ~0ull : ((1ull << L) - 1ull);

  // 1. row masks and run roots; coins
  for (int R = t; R < NR; R += T) {
    const uint64_t m = row_q_mask(g, Q, R);
    qr[R] = m;
    if (!m) continue;
    uint32_t* row = lab + R * L;
    const uint32_t base = (uint32_t)(R * L);
    if (m == full) {
      for (int x0 = 0; x0 < L; ++x0) row[x0] = base;
      continue;
    }
    // the run through x0 = L - 1 continues at x0 = 0 when both are q = -1;
    // its lowest site is then x0 = 0
    const bool wrap = (m & 1ull) && ((m >> (L - 1)) & 1ull);
    const int last = L - (int)__clzll((long long)~(m << (64 - L)));  // start of the run ending at L-1
    int start = 0;
    for (int x0 = 0; x0 < L; ++x0) {
      if (!((m >> x0) & 1ull)) continue;
      if (x0 == 0 || !((m >> (x0 - 1)) & 1ull)) start = x0;
      row[x0] = base + (uint32_t)((wrap && x0 >= last) ? 0 : start);
    }
  }
  for (int blk = t; blk < nblk; blk += T) {
    const Ctr4 r = philox10(Ctr4{(uint32_t)blk, v, (uint32_t)k, (kTagHouMulti << 28) | (uint32_t)s},
                            g.key0, g.key1);
    coin[4 * blk + 0] = r.x;
    coin[4 * blk + 1] = r.y;
    coin[4 * blk + 2] = r.z;
    coin[4 * blk + 3] = r.w;
  }
  sync();

  // 2. unite the runs that overlap along x1 (and x2), once per overlap segment
  for (int R = t; R < NR; R += T) {
    const uint64_t m = qr[R];
    if (!m) continue;
    int up[D - 1];
    rows_up(g, R, up);
#pragma unroll
    for (int j = 0; j < D - 1; ++j) {
      const uint64_t e = m & qr[up[j]];
      if (!e) continue;
      // first site of each segment (cyclically); a full overlap is one segment
      uint64_t first = e & ~(((e << 1) | (e >> (L - 1))) & full);
      if (e == full) first = 1ull;
      for (; first; first &= first - 1ull) {
        const int x0 = (int)__ffsll((long long)first) - 1;
        uf_unite(lab, (uint32_t)(R * L + x0), (uint32_t)(up[j] * L + x0));
      }
    }
  }
  sync();

  // 3. every q = -1 site takes its root (once per run, written to its sites)
  for (int R = t; R < NR; R += T) {
    const uint64_t m = qr[R];
    if (!m) continue;
    uint32_t* row = lab + R * L;
    uint32_t last_root = 0, root = 0;
    for (int x0 = 0; x0 < L; ++x0) {
      if (!((m >> x0) & 1ull)) continue;
      const uint32_t r0 = row[x0];
      if (x0 == 0 || r0 != last_root) {
        last_root = r0;
        root = uf_root(lab, (uint32_t)(R * L + x0));
      }
      row[x0] = root;
    }
  }
  sync();

  // 4. exchanged sites: the q = -1 sites whose root's coin is set
  for (int i = t; i < 2 * NW; i += T) {
    const int c = i >= NW ? 1 : 0, w = i - c * NW;
    const uint32_t qw = Q[i];
    uint32_t out = 0;
    if (qw) {
      const WordNb q = word_nb(g, w);
      const int p = (c + q.par) & 1;  // x0 parity of colour c in this word's rows
      for (int f = 0; f < g.P; ++f) {
        const uint32_t bits = (qw >> (f * g.H)) & g.maskH;
        if (!bits) continue;
        const int R = word_row(g, q, f);
        for (uint32_t rest = bits; rest; rest &= rest - 1u) {
          const int b = __ffs(rest) - 1;
          const uint32_t m = lab[R * L + 2 * b + p];
          if ((coin[m >> 5] >> (m & 31)) & 1u) out |= 1u << (f * g.H + b);
        }
      }
    }
    C[i] = out;
  }
  sync();
}

}  // namespace ptsg
