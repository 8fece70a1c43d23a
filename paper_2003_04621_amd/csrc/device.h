// device.h -- device-side building blocks shared by the gfx950 kernels:
// Philox4x32-10, lattice geometry, the colour-split bit layout held in LDS,
// and the job's device counters.
//
// Bit layout.  A row is the set of L sites with fixed (x1, x2); R = x1 + L*x2
// is its index, NR = L^(dim-1) rows per lattice.  For colour c of the
// checkerboard, the H = L/2 sites of colour c in row R (x0 = 2b + p(c,R),
// b < H, p(c,R) = (c + x1 + x2) & 1) form an H-bit "row field"; bit set <=>
// s = -1.  P row fields of the same lattice and colour share one 32-bit word:
// the slowest coordinate xs (x2 in 3D, x1 in 2D) is cut into P blocks of
// B = L/P values, xs = f*B + xs', and field f (bits f*H .. f*H+H-1) of word
// w = x1 + L*xs' (3D) or w = xs' (2D) holds the row with that xs.  B is even,
// so p(c,R) is the same for every field of a word.  NW = NR/P words per
// lattice and colour.
//
// Because the checkerboard is bipartite for even L, every neighbour of a
// colour-c site is a colour-(1-c) site, and the 2d neighbour words of a
// colour-c word w, with O = W[1-c]:
//   +x0: per field rotr(O[w], p)       -x0: per field rotr(O[w], H-1+p)
//   +-x1 (3D): O[w +- e_x1]
//   +-xs: O[w +- e_xs'] inside a block; across a block boundary the word at
//         the other end of the block with its fields rotated by one field.
// One word operation therefore serves P*H sites.
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

// Three-input bitwise function with truth table TT (gfx950 v_bitop3_b32):
// result bit = TT bit number (a_bit * 4 + b_bit * 2 + c_bit).  Through the
// compiler builtin rather than inline assembly, so that the scheduler sees the
// instruction: it can then fill the wait a 64-bit multiply needs after a VALU
// write of its operand with independent work instead of an s_nop.
template <unsigned TT>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}
// The same, for a wave-uniform third operand.
template <unsigned TT>
__device__ __forceinline__ uint32_t bop3s(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}
constexpr unsigned kXor3 = 0x96;   // a ^ b ^ c
constexpr unsigned kMaj3 = 0xE8;   // majority(a, b, c)
constexpr unsigned kAndOr = 0xEA;  // (a & b) | c

__device__ __forceinline__ Ctr4 philox10(Ctr4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
    Ctr4 n;
    n.x = bop3s<kXor3>((uint32_t)(p1 >> 32), c.y, k0);
    n.y = (uint32_t)p1;
    n.z = bop3s<kXor3>((uint32_t)(p0 >> 32), c.w, k1);
    n.w = (uint32_t)p0;
    c = n;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return c;
}

// The same function with round 1's key words folded into the counter words
// c1 and c3 first: for the Metropolis counters those are the same for every
// lane of a wavefront in the fused kernels (sweep number, colour, tag and
// sample), so c3 ^ k1 is one scalar operand and round 1 takes a two-input
// XOR where the three-input one would first copy one of its two scalar
// operands to a vector register (an instruction reads at most one scalar
// register).  Elsewhere the folded words are loop-invariant per lattice.  XOR
// is associative: the output words are identical.
__device__ __forceinline__ Ctr4 philox10_u(Ctr4 c, uint32_t k0, uint32_t k1) {
  const uint32_t y0 = c.y ^ k0;
  const uint32_t w1 = c.w ^ k1;
  const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
  const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
  c = Ctr4{(uint32_t)(p1 >> 32) ^ y0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ w1, (uint32_t)p0};
  k0 += kWeyl0;
  k1 += kWeyl1;
#pragma unroll
  for (int r = 1; r < 10; ++r) {
    const uint64_t q0 = (uint64_t)kPhiloxM0 * c.x;
    const uint64_t q1 = (uint64_t)kPhiloxM1 * c.z;
    Ctr4 n;
    n.x = bop3s<kXor3>((uint32_t)(q1 >> 32), c.y, k0);
    n.y = (uint32_t)q1;
    n.z = bop3s<kXor3>((uint32_t)(q0 >> 32), c.w, k1);
    n.w = (uint32_t)q0;
    c = n;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return c;
}

// (mask << 1) | (r < t): the borrow of r - t shifted into the mask, two VALU
// instructions.  t is a per-lane value (lanes of one wavefront may serve
// lattices at different temperatures).
__device__ __forceinline__ uint32_t shift_in_less(uint32_t mask, uint32_t r, uint32_t t) {
  uint32_t out, tmp;
  asm("v_sub_co_u32_e32 %1, vcc, %2, %3\n\t"
      "v_addc_co_u32_e32 %0, vcc, %4, %4, vcc"
      : "=v"(out), "=&v"(tmp)
      : "v"(r), "v"(t), "v"(mask)
      : "vcc");
  return out;
}

// 3D acceptance planes from two compares per site: with th6 <= th4 <= th2 the
// number of thresholds above r is k = 2 [r < th4] + [r < (r < th4 ? th6 : th2)],
// shifted in as bit planes K1 (the first term) and K0.  Two sites per block,
// r1 shifted in before r2, so that each select reads its compare's lane mask
// two instructions after it was written; carries out of the adds go to vcc.
__device__ __forceinline__ void shift_in_k_pair(uint32_t& K1, uint32_t& K0, uint32_t r1, uint32_t r2,
                                                uint32_t th2, uint32_t th4, uint32_t th6) {
  uint32_t t, ta, tb;
  uint64_t sa, sb;
  asm("v_sub_co_u32_e64 %[t], %[sa], %[r1], %[th4]\n\t"
      "v_addc_co_u32_e64 %[k1], vcc, %[k1], %[k1], %[sa]\n\t"
      "v_sub_co_u32_e64 %[t], %[sb], %[r2], %[th4]\n\t"
      "v_addc_co_u32_e64 %[k1], vcc, %[k1], %[k1], %[sb]\n\t"
      "v_cndmask_b32_e64 %[ta], %[th2], %[th6], %[sa]\n\t"
      "v_cndmask_b32_e64 %[tb], %[th2], %[th6], %[sb]\n\t"
      "v_sub_co_u32_e32 %[t], vcc, %[r1], %[ta]\n\t"
      "v_addc_co_u32_e32 %[k0], vcc, %[k0], %[k0], vcc\n\t"
      "v_sub_co_u32_e32 %[t], vcc, %[r2], %[tb]\n\t"
      "v_addc_co_u32_e32 %[k0], vcc, %[k0], %[k0], vcc"
      : [k1] "+v"(K1), [k0] "+v"(K0), [t] "=&v"(t), [ta] "=&v"(ta), [tb] "=&v"(tb),
        [sa] "=&s"(sa), [sb] "=&s"(sb)
      : [r1] "v"(r1), [r2] "v"(r2), [th2] "v"(th2), [th4] "v"(th4), [th6] "v"(th6)
      : "vcc");
}

// The same for one site.
__device__ __forceinline__ void shift_in_k_one(uint32_t& K1, uint32_t& K0, uint32_t r, uint32_t th2,
                                               uint32_t th4, uint32_t th6) {
  uint32_t t, ta;
  uint64_t sa;
  asm("v_sub_co_u32_e64 %[t], %[sa], %[r], %[th4]\n\t"
      "v_addc_co_u32_e64 %[k1], vcc, %[k1], %[k1], %[sa]\n\t"
      "s_nop 1\n\t"
      "v_cndmask_b32_e64 %[ta], %[th2], %[th6], %[sa]\n\t"
      "v_sub_co_u32_e32 %[t], vcc, %[r], %[ta]\n\t"
      "v_addc_co_u32_e32 %[k0], vcc, %[k0], %[k0], vcc"
      : [k1] "+v"(K1), [k0] "+v"(K0), [t] "=&v"(t), [ta] "=&v"(ta), [sa] "=&s"(sa)
      : [r] "v"(r), [th2] "v"(th2), [th4] "v"(th4), [th6] "v"(th6)
      : "vcc");
}

// Counter tags (top four bits of the fourth counter word).
constexpr uint32_t kTagInit = 2u, kTagMetro = 3u, kTagPT = 4u, kTagHou = 5u;

// ---------------------------------------------------------------------------
// Job description passed by value to every kernel.
// ---------------------------------------------------------------------------
enum : int { kLayoutInt8 = 0, kLayoutPacked = 1 };

struct Geo {
  int L, d, N, NR, H, G;  // G = ceil(L/8): Philox calls per row field
  int P, B, NW;           // fields per word, block length, words per colour
  uint32_t magicL;        // ceil(2^32 / L): x / L == umulhi(x, magicL) for x < 2^20
  uint32_t maskH;         // low H bits
  uint32_t maskW;         // low P*H bits
  uint32_t LB, HB;        // lowest / highest bit of every field
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

// Counters are read by the kernels at their start and advanced afterwards by
// k_advance, a one-thread kernel enqueued behind them on the same stream (a
// per-block atomic on one address serialises tens of thousands of blocks).
struct CounterStep {
  uint32_t dt, du, dv, dm;
  // measurement interval (0 or 1: dm as given); with every > 1 the dt sweeps
  // from t count dm * (number of their 1-based sweep numbers divisible by it)
  uint32_t every;
};

// Whether the step with 1-based sweep number t1 measures at interval `every`.
__host__ __device__ constexpr bool measures_at(uint32_t t1, uint32_t every) {
  return every <= 1u || t1 % every == 0u;
}

// The geometry fields of Geo, a function of L and d alone.  Fields per word:
// the most row fields of H = L/2 bits that fit 32 bits with a block length
// L/P that keeps every field of a word at the same checkerboard offset.
__host__ __device__ constexpr int fields_per_word(int L) {
  for (int p = 32 / (L / 2); p >= 1; --p)
    if (L % p == 0 && (L / p) % 2 == 0) return p;
  return 1;
}

__host__ __device__ constexpr Geo geo_shape(int L, int d) {
  Geo g{};
  g.L = L;
  g.d = d;
  g.N = d == 3 ? L * L * L : L * L;
  g.NR = g.N / L;
  g.H = L / 2;
  g.G = (L + 7) / 8;
  g.magicL = (uint32_t)((0x100000000ull + (uint64_t)L - 1) / (uint64_t)L);
  g.maskH = (g.H == 32) ? 0xFFFFFFFFu : ((1u << g.H) - 1u);
  g.P = fields_per_word(L);
  g.B = L / g.P;
  g.NW = g.NR / g.P;
  g.maskW = (g.P * g.H == 32) ? 0xFFFFFFFFu : ((1u << (g.P * g.H)) - 1u);
  g.LB = 0;
  for (int f = 0; f < g.P; ++f) g.LB |= 1u << (f * g.H);
  g.HB = g.LB << (g.H - 1);
  return g;
}

// g with its geometry fields replaced by compile-time constants for the
// shape (L, D) (LS = L; LS = 0 leaves g as it is), so that the compiler folds
// them; the caller has checked that g has this shape.
template <int D, int LS>
__device__ __forceinline__ Geo fixed_shape(const Geo& g) {
  if constexpr (LS == 0) {
    return g;
  } else {
    constexpr Geo k = geo_shape(LS, D);
    Geo c = g;
    c.L = k.L;
    c.d = k.d;
    c.N = k.N;
    c.NR = k.NR;
    c.H = k.H;
    c.G = k.G;
    c.P = k.P;
    c.B = k.B;
    c.NW = k.NW;
    c.magicL = k.magicL;
    c.maskH = k.maskH;
    c.maskW = k.maskW;
    c.LB = k.LB;
    c.HB = k.HB;
    return c;
  }
}

__device__ __forceinline__ uint32_t divL(const Geo& g, uint32_t x) {
  return __umulhi(x, g.magicL);
}

__device__ __forceinline__ uint32_t load_counter(const uint32_t* p) {
  return __atomic_load_n(p, __ATOMIC_RELAXED);
}

// ---------------------------------------------------------------------------
// Replica walk in temperature space and its round-trip (tunnelling) time,
// Sec. 2.3: the number of steps a configuration takes from the lowest
// temperature to the highest and back.  Called by one thread per replica set
// after exchange pass m (counted from 1; modulo 2^32) with the set's slots
// `cold` and `hot` now at the lowest and highest temperature.  wk holds the
// set's [NT][2] walk words: a label (0 = not yet at the lowest temperature,
// 1 = going up, 2 = going down: reached the highest while going up) and the
// pass at which the slot's current round trip began.  A slot labelled 2 that
// is back at the lowest temperature ends a round trip of m - begin passes,
// added to bin floor(log2 m) of the [32][3] sums `bins` (count, sum of
// lengths, sum of squared lengths; atomically, as the two replica sets of a
// sample may be walked at once), and begins the next one.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Two-replica modes (the spin-glass susceptibility and correlation-length modes
// that Sec. 3 names; usual definitions).  From the plane counts cnt[mu][x]
// (mu < d, x < L) of the sites where the two replicas differ, the overlap's
// plane sums are P_mu(x) = L^(d-1) - 2 cnt[mu][x]; returns
// A(delta) = sum_mu sum_x P_mu(x) P_mu((x + delta) mod L), an exact integer
// from which |sum_i q_i exp(i k x_mu)|^2 = sum_delta cos(k delta) A(delta).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t mode_autocorr(const Geo& g, const int32_t* cnt, int delta) {
  const int L = g.L, plane = g.N / L;
  int64_t A = 0;
  for (int mu = 0; mu < g.d; ++mu) {
    const int32_t* c = cnt + mu * L;
    int y = delta;
    for (int x = 0; x < L; ++x) {
      A += (int64_t)(plane - 2 * c[x]) * (int64_t)(plane - 2 * c[y]);
      if (++y == L) y = 0;
    }
  }
  return A;
}

// wk is 8-byte aligned; cold != hot (N_T >= 2), so both slots' words are read
// before either is written.
__device__ __forceinline__ void walk_observe(int32_t* wk, uint64_t* bins, int cold, int hot,
                                             uint32_t m) {
  int2* wc = reinterpret_cast<int2*>(wk) + cold;
  int32_t* wh = wk + 2 * hot;
  const int2 c = *wc;
  const int lab_hot = *wh;
  if (c.x == 2) {
    const uint64_t len = (uint32_t)(m - (uint32_t)c.y);
    unsigned long long* b = reinterpret_cast<unsigned long long*>(bins) + 3 * (31 - __clz(m | 1u));
    atomicAdd(b, 1ull);
    atomicAdd(b + 1, (unsigned long long)len);
    atomicAdd(b + 2, (unsigned long long)(len * len));
  }
  if (c.x != 1) *wc = make_int2(1, (int32_t)m);
  if (lab_hot == 1) *wh = 2;
}

// ---------------------------------------------------------------------------
// Word geometry.
// ---------------------------------------------------------------------------
struct WordNb {
  int x1, xs;     // 3D: x1 and x2' (block-local x2); 2D: xs = x1' (x1 unused)
  int par;        // p(c, word) = (c + par) & 1
  int w1p, w1m;   // 3D: words at x1 +- 1
  int wsp, wsm;   // words at xs +- 1 (other end of the block when crossing)
  bool crp, crm;  // the xs neighbour crosses a block boundary (rotate fields)
};

__device__ __forceinline__ WordNb word_nb(const Geo& g, int w) {
  WordNb q;
  if (g.d == 3) {
    q.xs = (int)divL(g, (uint32_t)w);
    q.x1 = w - q.xs * g.L;
    q.par = (q.x1 + q.xs) & 1;
    q.w1p = (q.x1 == g.L - 1) ? w - (g.L - 1) : w + 1;
    q.w1m = (q.x1 == 0) ? w + (g.L - 1) : w - 1;
    q.crp = q.xs == g.B - 1;
    q.crm = q.xs == 0;
    q.wsp = q.crp ? w - (g.B - 1) * g.L : w + g.L;
    q.wsm = q.crm ? w + (g.B - 1) * g.L : w - g.L;
  } else {
    q.xs = w;
    q.x1 = 0;
    q.par = w & 1;
    q.w1p = q.w1m = w;
    q.crp = q.xs == g.B - 1;
    q.crm = q.xs == 0;
    q.wsp = q.crp ? w - (g.B - 1) : w + 1;
    q.wsm = q.crm ? w + (g.B - 1) : w - 1;
  }
  return q;
}

// Row index of field f of word w.
__device__ __forceinline__ int word_row(const Geo& g, const WordNb& q, int f) {
  const int xs = f * g.B + q.xs;
  return g.d == 3 ? q.x1 + g.L * xs : xs;
}

// Word and field holding row R (the inverse of word_row).
__device__ __forceinline__ void row_word(const Geo& g, int R, int& w, int& f) {
  if (g.d == 3) {
    const int x2 = (int)divL(g, (uint32_t)R), x1 = R - x2 * g.L;
    f = x2 / g.B;
    w = x1 + g.L * (x2 - f * g.B);
  } else {
    f = R / g.B;
    w = R - f * g.B;
  }
}

// Colour of the even-x0 sites of row R: (x1 + x2) & 1.
__device__ __forceinline__ int row_parity(const Geo& g, int R) {
  if (g.d == 3) {
    const int x2 = (int)divL(g, (uint32_t)R);
    return (R - x2 * g.L + x2) & 1;
  }
  return R & 1;
}

// The q = -1 site with rank m (counted in increasing site order) inside row
// R, given the two colour words of R's word w and its field f.  Returns the
// colour c and the bit b = x0 >> 1 of that site within field f.
__device__ __forceinline__ void select_in_row(const Geo& g, int R, uint32_t Q0, uint32_t Q1, int f,
                                              uint32_t m, int& c_out, int& b_out) {
  const int p0 = row_parity(g, R);
  const uint32_t q0 = (Q0 >> (f * g.H)) & g.maskH, q1 = (Q1 >> (f * g.H)) & g.maskH;
  c_out = -1;
  b_out = 0;
  for (int x0 = 0; x0 < g.L; ++x0) {
    const int c = (x0 & 1) ^ p0;
    if ((((c ? q1 : q0) >> (x0 >> 1)) & 1u) == 0) continue;
    if (m == 0) {
      c_out = c;
      b_out = x0 >> 1;
      return;
    }
    --m;
  }
}

// Field rotations of a P*H-bit word: result field f = source field f+1
// (rot_fields_down) or f-1 (rot_fields_up), cyclically.
__device__ __forceinline__ uint32_t rot_fields_down(const Geo& g, uint32_t X) {
  if (g.P * g.H == 32) return __builtin_amdgcn_alignbit(X, X, (uint32_t)g.H);  // rotate right
  const uint64_t XX = (uint64_t)X | ((uint64_t)X << (g.P * g.H));
  return (uint32_t)(XX >> g.H) & g.maskW;
}
__device__ __forceinline__ uint32_t rot_fields_up(const Geo& g, uint32_t X) {
  if (g.P * g.H == 32) return __builtin_amdgcn_alignbit(X, X, (uint32_t)(32 - g.H));
  const uint64_t XX = (uint64_t)X | ((uint64_t)X << (g.P * g.H));
  return (uint32_t)(XX >> ((g.P - 1) * g.H)) & g.maskW;
}

// a if take else b, without a branch.
__device__ __forceinline__ uint32_t pick(bool take, uint32_t a, uint32_t b) {
  const uint32_t m = 0u - (uint32_t)take;
  return (a & m) | (b & ~m);
}

// +x0 / -x0 neighbour words of a colour-c word whose opposite-colour word is
// O; p = p(c, word).  Each field rotates by one bit within itself.
__device__ __forceinline__ void x0_neighbours(const Geo& g, uint32_t O, int p,
                                              uint32_t& nplus, uint32_t& nminus) {
  const uint32_t rr = ((O >> 1) & ~g.HB) | ((O & g.LB) << (g.H - 1));  // bit b <- b+1
  const uint32_t rl = ((O << 1) & ~g.LB & g.maskW) | ((O & g.HB) >> (g.H - 1));  // bit b <- b-1
  nplus = p ? rr : O;
  nminus = p ? O : rl;
}

// All 2d neighbour words of the colour-c word w; Wo = the colour-(1-c) words.
template <int D>
__device__ __forceinline__ void neighbour_words(const Geo& g, const uint32_t* Wo, int w,
                                                const WordNb& q, int p, uint32_t* n) {
  x0_neighbours(g, Wo[w], p, n[0], n[1]);
  if (D == 3) {
    n[2] = Wo[q.w1p];
    n[3] = Wo[q.w1m];
    const uint32_t sp = Wo[q.wsp], sm = Wo[q.wsm];
    n[4] = pick(q.crp, rot_fields_down(g, sp), sp);
    n[5] = pick(q.crm, rot_fields_up(g, sm), sm);
  } else {
    const uint32_t sp = Wo[q.wsp], sm = Wo[q.wsm];
    n[2] = pick(q.crp, rot_fields_down(g, sp), sp);
    n[3] = pick(q.crm, rot_fields_up(g, sm), sm);
  }
}

// ---------------------------------------------------------------------------
// Lattice <-> LDS words.  W points at 2*NW words: W[c*NW + w].
// int8 layout: spins8[lat*N + i], +1 / -1.  Packed layout: spins32[lat*2*NW +
// c*NW + w] exactly as in LDS.
// ---------------------------------------------------------------------------
// Row R as two H-bit fields: bits of the even-x0 sites and of the odd-x0 sites.
// Even- and odd-x0 sign bits of four int8 spins packed in v (sites 4a .. 4a+3),
// placed at bits 2a, 2a+1 of e and o.
__device__ __forceinline__ void gather4(uint32_t v, int a, uint32_t& e, uint32_t& o) {
  e |= (((v >> 7) & 1u) | ((v >> 22) & 2u)) << (2 * a);
  o |= (((v >> 15) & 1u) | ((v >> 30) & 2u)) << (2 * a);
}

__device__ __forceinline__ void row_from_int8(const Geo& g, const int8_t* lat, int R,
                                              uint32_t& Weven, uint32_t& Wodd) {
  uint32_t e = 0, o = 0;
  const int8_t* row = lat + (size_t)R * g.L;
  if ((g.L & 15) == 0) {
    // 16-byte loads (rows of a lattice start 16-byte aligned when 16 | L)
    const uint4* r128 = reinterpret_cast<const uint4*>(row);
    for (int a = 0; a < g.L / 16; ++a) {
      const uint4 v = r128[a];
      gather4(v.x, 4 * a + 0, e, o);
      gather4(v.y, 4 * a + 1, e, o);
      gather4(v.z, 4 * a + 2, e, o);
      gather4(v.w, 4 * a + 3, e, o);
    }
  } else if ((g.L & 3) == 0) {
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
  Weven = e;
  Wodd = o;
}

// Four int8 spins (sites 4a .. 4a+3) from bits 2a, 2a+1 of the even- and
// odd-x0 words e and o (bit set: -1).
__device__ __forceinline__ uint32_t spread4(uint32_t e, uint32_t o, int a) {
  const uint32_t ee = (e >> (2 * a)) & 3u, oo = (o >> (2 * a)) & 3u;
  const uint32_t bits = (ee & 1u) | ((oo & 1u) << 1) | ((ee & 2u) << 1) | ((oo & 2u) << 2);
  const uint32_t spread = (bits & 1u) | ((bits & 2u) << 7) | ((bits & 4u) << 14) | ((bits & 8u) << 21);
  return 0x01010101u + spread * 0xFEu;
}

__device__ __forceinline__ void row_to_int8(const Geo& g, int8_t* lat, int R, uint32_t e,
                                            uint32_t o) {
  int8_t* row = lat + (size_t)R * g.L;
  if ((g.L & 15) == 0) {
    uint4* r128 = reinterpret_cast<uint4*>(row);
    for (int a = 0; a < g.L / 16; ++a)
      r128[a] = make_uint4(spread4(e, o, 4 * a), spread4(e, o, 4 * a + 1), spread4(e, o, 4 * a + 2),
                           spread4(e, o, 4 * a + 3));
  } else if ((g.L & 3) == 0) {
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

// Both colour words of word w of an int8 lattice.  The even-x0 sites of a
// row have colour (x1 + x2) & 1 = par.
__device__ __forceinline__ void word_from_int8(const Geo& g, const int8_t* lat, int w,
                                               uint32_t& W0, uint32_t& W1) {
  const WordNb q = word_nb(g, w);
  uint32_t e = 0, o = 0;
  for (int f = 0; f < g.P; ++f) {
    uint32_t fe, fo;
    row_from_int8(g, lat, word_row(g, q, f), fe, fo);
    e |= fe << (f * g.H);
    o |= fo << (f * g.H);
  }
  W0 = q.par ? o : e;
  W1 = q.par ? e : o;
}

__device__ __forceinline__ void word_to_int8(const Geo& g, int8_t* lat, int w, uint32_t W0,
                                             uint32_t W1) {
  const WordNb q = word_nb(g, w);
  const uint32_t e = q.par ? W1 : W0, o = q.par ? W0 : W1;
  for (int f = 0; f < g.P; ++f)
    row_to_int8(g, lat, word_row(g, q, f), (e >> (f * g.H)) & g.maskH, (o >> (f * g.H)) & g.maskH);
}

// Cooperative load of lattice `lat` into W by threads t = 0..T-1.
__device__ __forceinline__ void load_lattice(const Geo& g, const void* spins, size_t lat,
                                             uint32_t* W, int t, int T) {
  if (g.layout == kLayoutPacked) {
    const uint32_t* src = static_cast<const uint32_t*>(spins) + lat * 2 * (size_t)g.NW;
    for (int i = t; i < 2 * g.NW; i += T) W[i] = src[i];
  } else {
    const int8_t* src = static_cast<const int8_t*>(spins) + lat * (size_t)g.N;
    for (int w = t; w < g.NW; w += T) word_from_int8(g, src, w, W[w], W[g.NW + w]);
  }
}

// Cooperative store (all words if `only_changed` is null; otherwise words w
// whose flag only_changed[w] or only_changed[NW + w] is non-zero).
__device__ __forceinline__ void store_lattice(const Geo& g, void* spins, size_t lat,
                                              const uint32_t* W, int t, int T,
                                              const uint32_t* only_changed = nullptr) {
  if (g.layout == kLayoutPacked) {
    uint32_t* dst = static_cast<uint32_t*>(spins) + lat * 2 * (size_t)g.NW;
    for (int i = t; i < 2 * g.NW; i += T)
      if (!only_changed || only_changed[i]) dst[i] = W[i];
  } else {
    int8_t* dst = static_cast<int8_t*>(spins) + lat * (size_t)g.N;
    for (int w = t; w < g.NW; w += T) {
      if (only_changed && !(only_changed[w] | only_changed[g.NW + w])) continue;
      word_to_int8(g, dst, w, W[w], W[g.NW + w]);
    }
  }
}

// ---------------------------------------------------------------------------
// Cross-lane moves within a wavefront (DPP).
// ---------------------------------------------------------------------------
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp_ones(uint32_t x) {  // lanes without a source: ~0
  return (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp_zero(uint32_t x) {  // lanes without a source: 0
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xF, ROWS == 0xF);
}
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShl4 = 0x104, kRowShl8 = 0x108;
constexpr int kBcast15 = 0x142, kBcast31 = 0x143;  // to rows 1, 3 / rows 2, 3
constexpr int kWaveRol1 = 0x134, kWaveRor1 = 0x13C;  // lane i takes lane i + 1 / i - 1 (mod 64)

// Sum over the wavefront as a wavefront constant, by DPP: row prefix sums,
// then the broadcasts of lanes 15 and 31 carry them on, so that lane 63 ends
// with the total (no LDS round trips).
__device__ __forceinline__ int wave_total(int v) {
  v += (int)dpp_zero<kRowShr1>((uint32_t)v);
  v += (int)dpp_zero<kRowShr2>((uint32_t)v);
  v += (int)dpp_zero<kRowShr4>((uint32_t)v);
  v += (int)dpp_zero<kRowShr8>((uint32_t)v);
  v += (int)dpp_zero<kBcast15, 0xA>((uint32_t)v);
  v += (int)dpp_zero<kBcast31, 0xC>((uint32_t)v);
  return __builtin_amdgcn_readlane(v, 63);
}

}  // namespace ptsg
