// multicluster.h -- the multi-cluster variant of the Houdayer move (Sec. 3 and
// Sec. 5 propose it to remove the load imbalance of single clusters): every
// nearest-neighbour cluster of q = -1 sites of a pair is exchanged,
// independently, with probability 1/2.  A cluster is named by its lowest
// site m (site i = x0 + L x1 + L^2 x2) and is exchanged iff bit m mod 128 of
// the Philox output for counter (m / 128, v, k, 6 << 28 | sample) is set (bit
// j = bit j mod 32 of word j / 32).
//
// Connected components by union-find over the runs of q = -1 sites along x0,
// by a team of threads (one wavefront in the fused step, one workgroup in the
// per-pair kernel), with a 32-bit parent label per run in LDS, kept at the
// run's lowest site (natural site order):
//   1. each row's q = -1 sites form runs along x0 (periodically), found with
//      bit operations on the row's 64-bit mask; a run is named by its lowest
//      site (its start, or x0 = 0 for the run that wraps through x0 = L - 1)
//      and starts as its own root;
//   2. every pair of runs overlapping along x1 (or x2) is united once, at the
//      first site of each overlap segment: the two roots are found (following
//      parents, each step also pointing the run passed at its grandparent)
//      and the larger is hooked under the smaller with an LDS atomic minimum;
//      if it had been hooked meanwhile, its new parent's root is united next;
//   3. every run takes its root, which is then its component's lowest site
//      (parents only ever point to lower runs of the same component, and
//      nothing hooks a component's lowest run);
//   4. the coins of all sites (one Philox call per 128 sites) and, for each
//      run, the coin of its root give the exchanged runs, whose bit masks
//      make the exchanged colour words.
// Concurrent finds and hooks only ever replace a parent by a lower ancestor
// in the same component, so every value read is valid and every find ends.
// All work is per run, not per site: a row of L sites holds at most L/2 runs.
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

// Bits 2b of x (b < 32) moved to bit b (the inverse of spread_bits).
__device__ __forceinline__ uint32_t compress_even_bits(uint64_t x) {
  x &= 0x5555555555555555ull;
  x = (x | (x >> 1)) & 0x3333333333333333ull;
  x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
  x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
  x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
  return (uint32_t)x;
}

// The runs of q = -1 sites of one row (L-bit mask m in x0 order, taken
// periodically).  starts: bit x0 set iff x0 is q = -1 and x0 - 1 is not;
// wrap: the start of the run through x0 = L - 1 when that run continues at
// x0 = 0 (-1 if none).  A row that is q = -1 everywhere has no start and is
// one run.
struct RowRuns {
  uint64_t m, starts;
  int wrap;
};

__device__ __forceinline__ RowRuns row_runs(uint64_t m, int L, uint64_t full) {
  RowRuns r;
  r.m = m;
  r.starts = m & ~(((m << 1) | (m >> (L - 1))) & full);
  r.wrap = (m != full && (m & 1ull) && ((m >> (L - 1)) & 1ull)) ? 63 - __clzll((long long)r.starts)
                                                                 : -1;
  return r;
}

// Name (lowest x0) of the run holding q = -1 site x0.
__device__ __forceinline__ int run_name(const RowRuns& r, int x0) {
  const uint64_t le = r.starts & ((2ull << x0) - 1ull);  // x0 = 63: every bit
  if (!le) return 0;  // no start at or below x0: the wrapping (or whole-row) run
  const int st = 63 - __clzll((long long)le);
  return st == r.wrap ? 0 : st;
}

// Sites of the run starting at `st` (st = r.wrap: the wrapping run).
__device__ __forceinline__ uint64_t run_mask(const RowRuns& r, int st, int L, uint64_t full) {
  const uint64_t above = full & ~((1ull << st) - 1ull);  // x0 >= st
  const uint64_t zeros = ~r.m & above;
  if (zeros) return above & ((1ull << (__ffsll((long long)zeros) - 1)) - 1ull);
  uint64_t mask = above;  // runs to x0 = L - 1
  if (st == r.wrap) {
    const uint64_t z = ~r.m & full;  // not empty: the row is not all q = -1
    mask |= (1ull << (__ffsll((long long)z) - 1)) - 1ull;
  }
  return mask;
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

  // 1. row masks; every run its own root, kept at its lowest site; coins
  for (int R = t; R < NR; R += T) {
    const uint64_t m = row_q_mask(g, Q, R);
    qr[R] = m;
    if (!m) continue;
    const RowRuns rr = row_runs(m, L, full);
    const uint32_t base = (uint32_t)(R * L);
    if (!rr.starts) {
      lab[base] = base;  // the whole row is one run
      continue;
    }
    for (uint64_t rest = rr.starts; rest; rest &= rest - 1ull) {
      const int st = __ffsll((long long)rest) - 1;
      const uint32_t name = base + (uint32_t)(st == rr.wrap ? 0 : st);
      lab[name] = name;
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
    const RowRuns rr = row_runs(m, L, full);
    int up[D - 1];
    rows_up(g, R, up);
#pragma unroll
    for (int j = 0; j < D - 1; ++j) {
      const uint64_t mu = qr[up[j]];
      const uint64_t e = m & mu;
      if (!e) continue;
      const RowRuns ru = row_runs(mu, L, full);
      // first site of each segment (cyclically); a full overlap is one segment
      uint64_t first = e & ~(((e << 1) | (e >> (L - 1))) & full);
      if (e == full) first = 1ull;
      for (; first; first &= first - 1ull) {
        const int x0 = (int)__ffsll((long long)first) - 1;
        uf_unite(lab, (uint32_t)(R * L + run_name(rr, x0)), (uint32_t)(up[j] * L + run_name(ru, x0)));
      }
    }
  }
  sync();

  // 3. every run takes its root
  for (int R = t; R < NR; R += T) {
    const uint64_t m = qr[R];
    if (!m) continue;
    const RowRuns rr = row_runs(m, L, full);
    const uint32_t base = (uint32_t)(R * L);
    if (!rr.starts) {
      lab[base] = uf_root(lab, base);
      continue;
    }
    for (uint64_t rest = rr.starts; rest; rest &= rest - 1ull) {
      const int st = __ffsll((long long)rest) - 1;
      const uint32_t name = base + (uint32_t)(st == rr.wrap ? 0 : st);
      lab[name] = uf_root(lab, name);
    }
  }
  sync();

  // 4. exchanged sites: the runs whose root's coin is set, as colour words
  for (int w = t; w < NW; w += T) {
    const WordNb q = word_nb(g, w);
    uint32_t out[2] = {0u, 0u};
    for (int f = 0; f < g.P; ++f) {
      const int R = word_row(g, q, f);
      const uint64_t m = qr[R];
      if (!m) continue;
      const RowRuns rr = row_runs(m, L, full);
      const uint32_t base = (uint32_t)(R * L);
      uint64_t X = 0;
      if (!rr.starts) {
        const uint32_t root = lab[base];
        if ((coin[root >> 5] >> (root & 31)) & 1u) X = full;
      } else {
        for (uint64_t rest = rr.starts; rest; rest &= rest - 1ull) {
          const int st = __ffsll((long long)rest) - 1;
          const uint32_t root = lab[base + (uint32_t)(st == rr.wrap ? 0 : st)];
          if ((coin[root >> 5] >> (root & 31)) & 1u) X |= run_mask(rr, st, L, full);
        }
      }
      if (!X) continue;
      const int p0 = row_parity(g, R);  // colour of the even-x0 sites
      out[p0] |= compress_even_bits(X) << (f * g.H);
      out[1 - p0] |= compress_even_bits(X >> 1) << (f * g.H);
    }
    C[w] = out[0];
    C[NW + w] = out[1];
  }
  sync();
}

}  // namespace ptsg
