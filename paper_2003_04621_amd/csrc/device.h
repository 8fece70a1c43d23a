// device.h -- device-side building blocks shared by the gfx950 kernels:
// Philox4x32-10, lattice geometry, the colour-split bit layout held in LDS,
// and the job's device counters.
//
// Bit layout ("row words").  A row is the set of L sites with fixed (x1, x2);
// R = x1 + L*x2 is its index, NR = L^(dim-1) rows per lattice.  For colour
// c in {0,1} of the checkerboard, the row word W[c][R] holds in bit b the spin
// of the site x0 = 2b + p(c,R), p(c,R) = (c + x1 + x2) & 1; bit set <=> s = -1.
// H = L/2 bits are used.  Because the checkerboard is bipartite for even L,
// every neighbour of a colour-c site is a colour-(1-c) site, and the six
// neighbour words of W[c][R] are:
//   +x0: rotr(W[1-c][R], p)        -x0: rotr(W[1-c][R], H-1+p)
//   +-x1: W[1-c][R +- e_x1]        +-x2: W[1-c][R +- e_x2]
// (rotations within H bits), so one word operation serves H sites.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptsg {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the S-box
// (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)) with the key
// advanced by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

struct Ctr4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ Ctr4 philox10(Ctr4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
    Ctr4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return c;
}

// Counter tags (top four bits of the fourth counter word).
constexpr uint32_t kTagInit = 2u, kTagMetro = 3u, kTagPT = 4u, kTagHou = 5u;

// ---------------------------------------------------------------------------
// Job description passed by value to every kernel.
// ---------------------------------------------------------------------------
enum : int { kLayoutInt8 = 0, kLayoutPacked = 1 };

struct Geo {
  int L, d, N, NR, H, G;  // G = ceil(L/8): Philox calls per row word
  uint32_t magicL;        // ceil(2^32 / L): x / L == umulhi(x, magicL) for x < 2^20
  uint32_t maskH;         // low H bits
  int S, NT, nslot;
  int layout;
  uint32_t key0, key1;
};

// Counters advanced on the device so that replays of captured work move on.
struct DevCounters {
  uint32_t t;       // sweeps done
  uint32_t u;       // exchange passes done
  uint32_t v;       // Houdayer passes done
  uint32_t n_meas;  // measurements done
  uint32_t pad[4];
};

__device__ __forceinline__ uint32_t divL(const Geo& g, uint32_t x) {
  return __umulhi(x, g.magicL);
}

__device__ __forceinline__ uint32_t load_counter(const uint32_t* p) {
  return __atomic_load_n(p, __ATOMIC_RELAXED);
}

// Counters are read by the kernels at their start and advanced afterwards by
// k_advance, a one-thread kernel enqueued behind them on the same stream (a
// per-block atomic on one address serialises tens of thousands of blocks).
struct CounterStep {
  uint32_t dt, du, dv, dm;
};

// Row geometry: coordinates and the four neighbour rows.
struct RowNb {
  int x1, x2, p0;        // p0 = (x1 + x2) & 1: colour of even x0
  int r1p, r1m, r2p, r2m;
};

__device__ __forceinline__ RowNb row_nb(const Geo& g, int R) {
  RowNb q;
  if (g.d == 3) {
    q.x2 = (int)divL(g, (uint32_t)R);
    q.x1 = R - q.x2 * g.L;
  } else {
    q.x2 = 0;
    q.x1 = R;
  }
  q.p0 = (q.x1 + q.x2) & 1;
  q.r1p = (q.x1 == g.L - 1) ? R - (g.L - 1) : R + 1;
  q.r1m = (q.x1 == 0) ? R + (g.L - 1) : R - 1;
  q.r2p = (q.x2 == g.L - 1) ? R - (g.L - 1) * g.L : R + g.L;
  q.r2m = (q.x2 == 0) ? R + (g.L - 1) * g.L : R - g.L;
  return q;
}

// +x0 / -x0 neighbour words of a colour-c word whose opposite-colour word in
// the same row is O; p = p(c, R).
__device__ __forceinline__ void x0_neighbours(const Geo& g, uint32_t O, int p,
                                              uint32_t& nplus, uint32_t& nminus) {
  const uint64_t OO = (uint64_t)O | ((uint64_t)O << g.H);
  nplus = (uint32_t)(OO >> p) & g.maskH;
  nminus = (uint32_t)(OO >> (g.H - 1 + p)) & g.maskH;
}

// ---------------------------------------------------------------------------
// Lattice <-> LDS row words.  W points at 2*NR words: W[c*NR + R].
// int8 layout: spins8[lat*N + i], +1 / -1.  Packed layout: spins32[lat*2*NR +
// c*NR + R] exactly as in LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void row_from_int8(const Geo& g, const int8_t* lat, int R,
                                              int p0, uint32_t& Weven, uint32_t& Wodd) {
  uint32_t e = 0, o = 0;
  const int8_t* row = lat + (size_t)R * g.L;
  if ((g.L & 3) == 0) {
    const uint32_t* r32 = reinterpret_cast<const uint32_t*>(row);
    for (int a = 0; a < g.L / 4; ++a) {
      const uint32_t v = r32[a];
      e |= (((v >> 7) & 1u) | ((v >> 22) & 2u)) << (2 * a);
      o |= (((v >> 15) & 1u) | ((v >> 30) & 2u)) << (2 * a);
    }
  } else {
    for (int x0 = 0; x0 < g.L; ++x0) {
      const uint32_t bit = row[x0] < 0 ? 1u : 0u;
      if (x0 & 1)
        o |= bit << (x0 >> 1);
      else
        e |= bit << (x0 >> 1);
    }
  }
  (void)p0;
  Weven = e;
  Wodd = o;
}

__device__ __forceinline__ void row_to_int8(const Geo& g, int8_t* lat, int R, uint32_t e,
                                            uint32_t o) {
  int8_t* row = lat + (size_t)R * g.L;
  if ((g.L & 3) == 0) {
    uint32_t* r32 = reinterpret_cast<uint32_t*>(row);
    for (int a = 0; a < g.L / 4; ++a) {
      const uint32_t ee = (e >> (2 * a)) & 3u, oo = (o >> (2 * a)) & 3u;
      const uint32_t bits = (ee & 1u) | ((oo & 1u) << 1) | ((ee & 2u) << 1) | ((oo & 2u) << 2);
      const uint32_t spread =
          (bits & 1u) | ((bits & 2u) << 7) | ((bits & 4u) << 14) | ((bits & 8u) << 21);
      r32[a] = 0x01010101u + spread * 0xFEu;
    }
  } else {
    for (int x0 = 0; x0 < g.L; ++x0) {
      const uint32_t w = (x0 & 1) ? o : e;
      row[x0] = ((w >> (x0 >> 1)) & 1u) ? (int8_t)-1 : (int8_t)1;
    }
  }
}

// Cooperative load of lattice `lat` into W by threads t = 0..T-1.
__device__ __forceinline__ void load_lattice(const Geo& g, const void* spins, size_t lat,
                                             uint32_t* W, int t, int T) {
  if (g.layout == kLayoutPacked) {
    const uint32_t* src = static_cast<const uint32_t*>(spins) + lat * 2 * (size_t)g.NR;
    for (int w = t; w < 2 * g.NR; w += T) W[w] = src[w];
  } else {
    const int8_t* src = static_cast<const int8_t*>(spins) + lat * (size_t)g.N;
    for (int R = t; R < g.NR; R += T) {
      const RowNb q = row_nb(g, R);
      uint32_t e, o;
      row_from_int8(g, src, R, q.p0, e, o);
      // even x0 has colour p0
      W[q.p0 * g.NR + R] = e;
      W[(1 - q.p0) * g.NR + R] = o;
    }
  }
}

// Cooperative store of rows R (all rows if `only_changed` is null; otherwise
// rows whose flag word only_changed[R] or only_changed[NR + R] is non-zero).
__device__ __forceinline__ void store_lattice(const Geo& g, void* spins, size_t lat,
                                              const uint32_t* W, int t, int T,
                                              const uint32_t* only_changed = nullptr) {
  if (g.layout == kLayoutPacked) {
    uint32_t* dst = static_cast<uint32_t*>(spins) + lat * 2 * (size_t)g.NR;
    for (int w = t; w < 2 * g.NR; w += T)
      if (!only_changed || only_changed[w]) dst[w] = W[w];
  } else {
    int8_t* dst = static_cast<int8_t*>(spins) + lat * (size_t)g.N;
    for (int R = t; R < g.NR; R += T) {
      if (only_changed && !(only_changed[R] | only_changed[g.NR + R])) continue;
      const RowNb q = row_nb(g, R);
      row_to_int8(g, dst, R, W[q.p0 * g.NR + R], W[(1 - q.p0) * g.NR + R]);
    }
  }
}

}  // namespace ptsg
