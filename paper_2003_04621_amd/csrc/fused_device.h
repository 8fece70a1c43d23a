// fused_device.h -- whole Monte Carlo steps (Sec. 2.4: Metropolis sweep, Houdayer
// move per same-temperature pair, replica-exchange pass, measurement) in one
// persistent kernel.  A workgroup holds one disorder sample (or one replica
// set of it, or one part of a sample too large for a workgroup) resident in
// LDS as colour-split row words for all steps of the launch; HBM is touched
// only to load the configurations at the start and store them at the end.
//
// Results are bit-identical to the per-step kernels: the same row update
// (rowops.h), the same Philox counters, exchange decisions taken in ascending
// k with the updated map, Houdayer seeds chosen in increasing site order.
#pragma once
#include <utility>

#include "device.h"
#include "kernels.h"
#include "houdayer_ops.h"
#include "multicluster.h"
#include "rowops.h"

namespace ptsg {


// 2D samples of 64 rows with one row per word get the in-register Houdayer
// move (one row per lane).
__host__ __device__ inline bool rows64_houdayer(const Geo& g) {
  return g.d == 2 && g.NW == 64 && g.P == 1;
}

// ---------------------------------------------------------------------------
// Wave-level helpers.  Lanes of one wavefront exchange data through LDS; the
// wavefront issues its LDS instructions in order, so a compiler fence plus a
// wait for outstanding LDS operations orders one lane's writes before
// another lane's later reads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Replica exchange for both sets of the resident sample.  The pass is
// sequential in k, but every decision depends only on which configuration is
// carried up from below: with the pre-pass map m0, the configuration at
// position k before step k is m0[j] for some j <= k, and b = m0[k+1].  All
// candidate decisions (c, k, j) are evaluated in parallel and kept as bits
// (one wavefront ballot per 64 of them), then one lane per set walks the
// chain.
// ---------------------------------------------------------------------------
// The inputs of pass u that the step's sweep and Houdayer move do not change:
// the map before the pass and one Philox word per (set, k).  Written before
// the sweep, so that the sweep's closing barrier orders them before the
// decisions.
__device__ __forceinline__ void exchange_prepare(const FusedArgs& A, uint32_t* lds, int s,
                                                 uint32_t u, int c_lo, int nsets) {
  const Geo& g = A.g;
  const int NT = g.NT, tid = threadIdx.x, T = blockDim.x;
  const int32_t* sotl = reinterpret_cast<const int32_t*>(lds + A.lay.sot);
  int32_t* sot0 = reinterpret_cast<int32_t*>(lds + A.lay.sot0);
  uint32_t* rpt = lds + A.lay.rpt;
  for (int i = tid; i < 2 * NT; i += T) sot0[i] = sotl[i];
  for (int i = tid; i < nsets * (NT - 1); i += T) {
    const int c = c_lo + i / (NT - 1), k = i - (c - c_lo) * (NT - 1);
    rpt[c * NT + k] =
        philox10(Ctr4{(uint32_t)k, u, (uint32_t)c, (kTagPT << 28) | (uint32_t)s}, g.key0, g.key1).x;
  }
}

// The pass itself, after exchange_prepare and a workgroup barrier; with WALK
// and `walk`, pass m (counted from 1) of the replica walk, with round trips
// summed in LDS (`walk` is false where the job does not track the walk or
// another workgroup of the sample keeps it).
template <bool WALK>
__device__ __forceinline__ void exchange_resident(const FusedArgs& A, uint32_t* lds, int c_lo,
                                                  int nsets, uint32_t m, bool walk) {
  const Geo& g = A.g;
  const int NT = g.NT, tid = threadIdx.x, T = blockDim.x;
  const int32_t* El = reinterpret_cast<const int32_t*>(lds + A.lay.E);
  int32_t* sotl = reinterpret_cast<int32_t*>(lds + A.lay.sot);
  int32_t* tosl = reinterpret_cast<int32_t*>(lds + A.lay.tos);
  const int32_t* sot0 = reinterpret_cast<const int32_t*>(lds + A.lay.sot0);
  const uint32_t* rpt = lds + A.lay.rpt;
  uint32_t* acc = lds + A.lay.acc;  // bit j of row (c, k): rows of NB bits, c-major
  const int NB = (NT + 31) & ~31;
  {
    const int lane = tid & 63, total = nsets * (NT - 1) * NB;  // a multiple of 32
    uint32_t* accs = acc + (size_t)c_lo * (NT - 1) * (NB >> 5);
    for (int base = tid - lane; base < total; base += T) {  // uniform per wavefront
      const int i = base + lane;
      bool ok = false;
      if (i < total) {
        const int row = i / NB, j = i - row * NB;
        const int cl = row / (NT - 1), k = row - cl * (NT - 1), c = c_lo + cl;
        if (j <= k) {
          const int a = sot0[c * NT + j], b = sot0[c * NT + k + 1];
          const int32_t D = El[c * NT + b] - El[c * NT + a];
          ok = D <= 0;
          if (!ok) {
            const int m = D >> 1;
            ok = m < A.M && rpt[c * NT + k] < A.thrpt[(size_t)k * A.M + m];
          }
        }
      }
      const uint64_t bits = __ballot(ok);
      if (lane == 0) accs[base >> 5] = (uint32_t)bits;
      if (lane == 32 && base + 32 < total) accs[(base >> 5) + 1] = (uint32_t)(bits >> 32);
    }
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, nwave = T >> 6;
  if (NT <= 64) {
    // One wavefront per set; lane k holds decision row k.  From the carried
    // position cur the next rejection is the first step k >= cur whose
    // decision for cur is a rejection, found by one ballot; the configuration
    // carried up from cur stops there and the one at k + 1 is carried on.
    // The walking wavefronts hold up the rest of the workgroup at the next
    // barrier, so they issue ahead of the CU's other wavefronts meanwhile.
    if (wave < nsets) __builtin_amdgcn_s_setprio(2);
    for (int cs = wave; cs < nsets; cs += nwave) {
      const int c = c_lo + cs;
      const int32_t* m0 = sot0 + c * NT;
      int32_t* so = sotl + c * NT;
      int32_t* to = tosl + c * NT;
      const uint32_t* arow = acc + (size_t)c * (NT - 1) * (NB >> 5);
      uint64_t row = 0;
      if (lane < NT - 1) {
        row = arow[lane * (NB >> 5)];
        if (NB > 32) row |= (uint64_t)arow[lane * (NB >> 5) + 1] << 32;
      }
      uint64_t rej = 0;  // steps that rejected
      int cur = 0;
      for (;;) {
        const uint64_t r = __ballot(lane >= cur && lane < NT - 1 && !((row >> cur) & 1u));
        if (r == 0) break;
        const int k = __ffsll((unsigned long long)r) - 1;
        rej |= 1ull << k;
        cur = k + 1;
      }
      // a rejecting step keeps the configuration carried from just after the
      // previous rejection (or from 0); an accepting one takes the one above
      if (lane < NT - 1) {
        int fin;
        if ((rej >> lane) & 1u) {
          const uint64_t below = rej & ((1ull << lane) - 1u);
          fin = m0[below ? 64 - __clzll((long long)below) : 0];
        } else {
          fin = m0[lane + 1];
        }
        so[lane] = fin;
        to[fin] = lane;
      }
      if (lane == 0) {
        const int hot = m0[cur];
        so[NT - 1] = hot;
        to[hot] = NT - 1;
        if (WALK && walk)
          walk_observe(reinterpret_cast<int32_t*>(lds + A.lay.walk) + 2 * c * NT,
                       reinterpret_cast<uint64_t*>(lds + A.lay.trip), so[0], hot, m);
      }
    }
    if (wave < nsets) __builtin_amdgcn_s_setprio(0);
  } else if (tid < nsets) {
    const int c = c_lo + tid;
    const int32_t* m0 = sot0 + c * NT;
    int32_t* so = sotl + c * NT;
    int32_t* to = tosl + c * NT;
    const uint32_t* arow = acc + (size_t)c * (NT - 1) * (NB >> 5);
    int cur = 0;
    for (int k = 0; k + 1 < NT; ++k) {
      int fin;
      if ((arow[k * (NB >> 5) + (cur >> 5)] >> (cur & 31)) & 1u) {
        fin = m0[k + 1];
      } else {
        fin = m0[cur];
        cur = k + 1;
      }
      so[k] = fin;
      to[fin] = k;
    }
    so[NT - 1] = m0[cur];
    to[m0[cur]] = NT - 1;
    if (WALK && walk)
      walk_observe(reinterpret_cast<int32_t*>(lds + A.lay.walk) + 2 * c * NT,
                   reinterpret_cast<uint64_t*>(lds + A.lay.trip), so[0], m0[cur], m);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Moments of one temperature from the energies of its two replicas and the
// number of sites where they differ: sum E (both replicas), sum E^2, q, |q|,
// q^2 and q^4 as a 128-bit (lo, hi) pair, with Q = N q = N - 2 neg.  Each
// word is added in place with a 64-bit LDS atomic (one thread per
// temperature, so the atomics only keep the compiler from holding all eight
// words in registers at once); the carry out of the low q^4 word comes from
// the value it replaced.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void add_moments(const Geo& g, int64_t* m, int32_t ea, int32_t eb, int neg) {
  const int64_t Q = (int64_t)g.N - 2 * (int64_t)neg;
  const int64_t Ea = ea, Eb = eb;
  unsigned long long* u = reinterpret_cast<unsigned long long*>(m);
  atomicAdd(u + 0, (unsigned long long)(Ea + Eb));
  atomicAdd(u + 1, (unsigned long long)(Ea * Ea + Eb * Eb));
  atomicAdd(u + 2, (unsigned long long)Q);
  atomicAdd(u + 3, (unsigned long long)(Q < 0 ? -Q : Q));
  const uint64_t q2 = (uint64_t)(Q * Q);
  atomicAdd(u + 4, (unsigned long long)q2);
  const uint64_t q4lo = q2 * q2, q4hi = __umul64hi(q2, q2);
  const uint64_t old = atomicAdd(u + 5, (unsigned long long)q4lo);
  atomicAdd(u + 6, (unsigned long long)(q4hi + (old + q4lo < old ? 1u : 0u)));
}

// ---------------------------------------------------------------------------
// Measurement of every temperature of the resident sample: one wavefront per
// temperature counts the sites where its two replicas differ and adds the
// moments.
// ---------------------------------------------------------------------------
typedef short __attribute__((ext_vector_type(2))) Short2;

// The two-replica modes of temperature k (mode_autocorr) by one wavefront,
// from the resident words of its two replicas: plane counts of the differing
// sites in the wavefront's LDS counters (slow axes by LDS atomics per word
// field; the fast axis x0, whose sites interleave inside a field, by one
// ballot per bit position: bit j of a colour-c word is the site
// x0 = 2 (j mod H) + ((c + par) & 1) of its field's row), then A(delta) for
// delta <= L/2 added to the item's LDS sums.
__device__ __forceinline__ void modes_resident(const Geo& g, const FusedLayout& lay, uint32_t* lds,
                                               const uint32_t* Wa, const uint32_t* Wb, int k,
                                               int wave, int lane) {
  const int L = g.L, NW = g.NW, MH = L / 2 + 1;
  int32_t* cnt = reinterpret_cast<int32_t*>(lds + lay.mcnt) + wave * 3 * L;
  int64_t* acc = reinterpret_cast<int64_t*>(lds + lay.modes) + (size_t)k * MH;
  for (int i = lane; i < 3 * L; i += 64) cnt[i] = 0;
  wave_lds_sync();
  int col = 0;  // lane x < L: differing sites at x0 = x
  for (int base = 0; base < NW; base += 64) {
    const int w = base + lane;
    uint32_t X0 = 0, X1 = 0;
    int par = 0;
    if (w < NW) {
      X0 = (Wa[w] ^ Wb[w]) & g.maskW;
      X1 = (Wa[NW + w] ^ Wb[NW + w]) & g.maskW;
      const WordNb q = word_nb(g, w);
      par = q.par;
      if (g.d == 3) {
        const int n = __popc(X0) + __popc(X1);
        if (n) atomicAdd(&cnt[L + q.x1], n);
      }
      for (int f = 0; f < g.P; ++f) {
        const uint32_t m = g.maskH << (f * g.H);
        const int n = __popc(X0 & m) + __popc(X1 & m);
        if (n) atomicAdd(&cnt[(g.d - 1) * L + f * g.B + q.xs], n);
      }
    }
    // colour-0 words hold the sites of x0 parity par, colour-1 words the other
    const uint32_t XE = par ? X1 : X0, XO = par ? X0 : X1;
    for (int bb = 0; bb < g.H; ++bb) {
      int even = 0, odd = 0;
      for (int f = 0; f < g.P; ++f) {
        const int j = f * g.H + bb;
        even += __popcll(__ballot((XE >> j) & 1u));
        odd += __popcll(__ballot((XO >> j) & 1u));
      }
      if (lane == 2 * bb) col += even;
      if (lane == 2 * bb + 1) col += odd;
    }
  }
  if (lane < L) cnt[lane] = col;
  wave_lds_sync();
  // Plane sums P = L^(d-1) - 2 cnt (|P| <= 2^12) packed in 16-bit pairs, in
  // place: per axis the L/2 even-aligned pairs (P(2i), P(2i+1)), then the L/2
  // odd-aligned ones (P(2i+1), P(2i+2 mod L)).  sum_x P(x) P(x + delta) is then
  // L/2 two-way dot products of pair i with the pair starting at 2i + delta,
  // an even- or odd-aligned one as delta is even or odd.
  const int half = L / 2, plane = g.N / L;
  uint32_t pe[3] = {0, 0, 0}, po[3] = {0, 0, 0};
  if (lane < half)
    for (int mu = 0; mu < g.d; ++mu) {
      const int32_t* c = cnt + mu * L;
      const int a = plane - 2 * c[2 * lane], b = plane - 2 * c[2 * lane + 1];
      const int e = plane - 2 * c[(2 * lane + 2) % L];
      pe[mu] = ((uint32_t)a & 0xFFFFu) | ((uint32_t)b << 16);
      po[mu] = ((uint32_t)b & 0xFFFFu) | ((uint32_t)e << 16);
    }
  wave_lds_sync();
  if (lane < half)
    for (int mu = 0; mu < g.d; ++mu) {
      cnt[mu * L + lane] = (int32_t)pe[mu];
      cnt[mu * L + half + lane] = (int32_t)po[mu];
    }
  wave_lds_sync();
  if (lane < MH) {
    int64_t A = 0;
    for (int mu = 0; mu < g.d; ++mu) {
      const Short2* E = reinterpret_cast<const Short2*>(cnt + mu * L);
      const Short2* Y = E + ((lane & 1) ? half : 0);
      int32_t sum = 0;  // <= L 2^24 <= 2^30
      int j = lane >> 1;
      for (int i = 0; i < half; ++i) {
        sum = __builtin_amdgcn_sdot2(E[i], Y[j], sum, false);
        if (++j == half) j = 0;
      }
      A += sum;
    }
    acc[lane] += A;
  }
  wave_lds_sync();
}

template <bool MODES>
__device__ __forceinline__ void measure_resident(const FusedArgs& A, uint32_t* lds) {
  const Geo& g = A.g;
  const int NT = g.NT, NW = g.NW, tid = threadIdx.x, T = blockDim.x;
  const uint32_t* W = lds + A.lay.W;
  const int32_t* El = reinterpret_cast<const int32_t*>(lds + A.lay.E);
  const int32_t* sotl = reinterpret_cast<const int32_t*>(lds + A.lay.sot);
  int64_t* mom = reinterpret_cast<int64_t*>(lds + A.lay.mom);
  const int wave = tid >> 6, lane = tid & 63, nwave = T >> 6;
  for (int k = wave; k < NT; k += nwave) {
    const int a = sotl[k], b = NT + sotl[NT + k];
    const uint32_t* Wa = W + (size_t)a * 2 * NW;
    const uint32_t* Wb = W + (size_t)b * 2 * NW;
    int neg = 0;
    for (int w = lane; w < 2 * NW; w += 64) neg += __popc(Wa[w] ^ Wb[w]);
    neg = wave_total(neg);
    if (lane == 0) add_moments(g, mom + (size_t)k * 8, El[a], El[b], neg);
    if (MODES && A.modes) modes_resident(g, A.lay, lds, Wa, Wb, k, wave, lane);
  }
  __syncthreads();
}


// Upward fill along the chain F_0, G_0, F_1, G_1, ... of every row field,
// where F_b -> G_b and G_b -> F_(b+1) (no link across a field boundary; nLB
// clears the lowest bit of each field): from seeds SF <= MF, SG <= MG, the
// sites of the masks MF, MG reachable by increasing steps.  F sites that can
// be entered from below form runs of R; adding the entry points Z to R
// carries through each run up to its first gap, so (R + Z) ^ R marks the
// reached bits of the run (an entry point already inside a carry is lost
// from the sum, hence the | Z).
__device__ __forceinline__ void chain_fill_up(uint32_t SF, uint32_t SG, uint32_t MF, uint32_t MG,
                                              uint32_t nLB, uint32_t& UF, uint32_t& UG) {
  const uint32_t Sp = SF | ((SG << 1) & nLB & MF);
  const uint32_t R = (MG << 1) & MF & nLB;
  const uint32_t Z = (Sp << 1) & R;
  const uint32_t V = (R & ((R + Z) ^ R)) | Z;
  UF = Sp | V;
  UG = SG | (UF & MG);
}

// Closure along x0 of the cluster words of one word index in row form: E and
// O hold the even and odd sites of each row field (E_0 O_0 E_1 O_1 ...), ME
// and MO the q sites, rME and rMO their bit reversals.  Every site of q
// linked to the cluster through a run of q sites of its row is added,
// periodic in x0: an upward fill and a bit-reversed (downward) fill cover
// each run from its lowest to its highest seed, and a run through the row's
// end is continued from its other end in one more pass.
__device__ __forceinline__ void row_closure(const Geo& g, uint32_t& E_io, uint32_t& O_io,
                                            uint32_t ME, uint32_t MO, uint32_t rME, uint32_t rMO) {
  const uint32_t nLB = ~g.LB, nLBr = ~__builtin_bitreverse32(g.HB);
  uint32_t SE = E_io, SO = O_io;
  for (;;) {
    uint32_t UE, UO, DO, DE;
    chain_fill_up(SE, SO, ME, MO, nLB, UE, UO);
    chain_fill_up(__builtin_bitreverse32(SO), __builtin_bitreverse32(SE), rMO, rME, nLBr, DO, DE);
    const uint32_t E = UE | __builtin_bitreverse32(DE), O = UO | __builtin_bitreverse32(DO);
    const uint32_t nE = E | (((O & g.HB) >> (g.H - 1)) & ME);  // O_(H-1) -> E_0
    const uint32_t nO = O | (((E & g.LB) << (g.H - 1)) & MO);  // E_0 -> O_(H-1)
    if (nE == E && nO == O) {
      E_io = E;
      O_io = O;
      return;
    }
    SE = nE;
    SO = nO;
  }
}

// The same closure for the colour words c0, c1 of a word whose rows have
// parity p0 (the even sites of a row have colour p0).
__device__ __forceinline__ void x0_closure(const Geo& g, uint32_t& c0, uint32_t& c1, uint32_t q0,
                                           uint32_t q1, int p0) {
  uint32_t E = p0 ? c1 : c0, O = p0 ? c0 : c1;
  const uint32_t ME = p0 ? q1 : q0, MO = p0 ? q0 : q1;
  row_closure(g, E, O, ME, MO, __builtin_bitreverse32(ME), __builtin_bitreverse32(MO));
  c0 = p0 ? O : E;
  c1 = p0 ? E : O;
}

// Grows both colour words w of a cluster: neighbours through other words,
// then the closure along x0, where the two colour words of index w are each
// other's only neighbours.  True if anything changed.  Stored cluster words
// are closed along x0, so without new bits from other words there is nothing
// to do, except on the first pass (`first`), which closes the seed.
template <int D>
__device__ __forceinline__ bool grow_pair(const Geo& g, uint32_t* C, const uint32_t* Q, int w,
                                          bool first) {
  const int NW = g.NW;
  const uint32_t q0 = Q[w], q1 = Q[NW + w];
  if (!(q0 | q1)) return false;
  const WordNb q = word_nb(g, w);
  const int p0 = q.par, p1 = 1 - q.par;  // p(0, w), p(1, w)
  uint32_t n0[2 * D], n1[2 * D];
  neighbour_words<D>(g, C + NW, w, q, p0, n0);  // colour-1 neighbours of colour-0 word
  neighbour_words<D>(g, C, w, q, p1, n1);       // colour-0 neighbours of colour-1 word
  uint32_t e0 = n0[2] | n0[3], e1 = n1[2] | n1[3];
  if (D == 3) {
    e0 |= n0[4] | n0[5];
    e1 |= n1[4] | n1[5];
  }
  const uint32_t c0_old = C[w], c1_old = C[NW + w];
  uint32_t c0 = c0_old | (q0 & e0);
  uint32_t c1 = c1_old | (q1 & e1);
  if (!(c0 | c1) || (!first && c0 == c0_old && c1 == c1_old)) return false;
  x0_closure(g, c0, c1, q0, q1, p0);
  if (c0 == c0_old && c1 == c1_old) return false;
  C[w] = c0;
  C[NW + w] = c1;
  return true;
}

// ---------------------------------------------------------------------------
// Column fills for a square lattice of 64 rows held one row per lane (2D,
// L = 64: one field per word, word = row).  The even sites of row r have
// colour r & 1, and the site above bit b of row r's even-site word is bit b
// of row r + 1's even-site word (likewise for the odd sites), so the chain
// X_r = even-site word of row r (and Y, the odd-site words) links equal bits
// of consecutive lanes, periodically (lane 63 to lane 0).  Filling a chain
// from its cluster bits through its q bits is a scan with the associative
// operator (q1, c1) then (q2, c2) -> (q1 & q2, c2 | (q2 & c1)).  Upward it
// runs over rows of 16 lanes by DPP row shifts and then across rows by the
// DPP broadcasts of lanes 15 and 31; downward by row shifts and then across
// rows through the four row totals read back as wavefront constants.  The
// AND-of-q half of every step depends on q alone and is computed once per
// pair; each fill then costs one DPP move and one AND-OR per step.
// ---------------------------------------------------------------------------
struct ColumnChain {
  uint32_t q;
  uint32_t p1, p2, p3, p4, p5, p6;  // upward: AND of q over the lanes each step has joined
  uint32_t d1, d2, d3;              // downward, within the row
  uint32_t m0, m1, m2, m3;          // AND of q from the lane to the top of its row, row r only
  uint32_t t0, t1, t2, t3;          // AND of q over all of row r (wavefront constants)
};

__device__ __forceinline__ ColumnChain column_chain(uint32_t q, int lane) {
  ColumnChain h;
  h.q = q;
  uint32_t p = q;
  h.p1 = p = p & dpp_ones<kRowShr1>(p);
  h.p2 = p = p & dpp_ones<kRowShr2>(p);
  h.p3 = p = p & dpp_ones<kRowShr4>(p);
  h.p4 = p = p & dpp_ones<kRowShr8>(p);
  h.p5 = p = p & dpp_ones<kBcast15, 0xA>(p);
  h.p6 = p & dpp_ones<kBcast31, 0xC>(p);
  uint32_t d = q;
  h.d1 = d = d & dpp_ones<kRowShl1>(d);
  h.d2 = d = d & dpp_ones<kRowShl2>(d);
  h.d3 = d = d & dpp_ones<kRowShl4>(d);
  d &= dpp_ones<kRowShl8>(d);
  const int row = lane >> 4;
  h.m0 = row == 0 ? d : 0u;
  h.m1 = row == 1 ? d : 0u;
  h.m2 = row == 2 ? d : 0u;
  h.m3 = row == 3 ? d : 0u;
  h.t0 = (uint32_t)__builtin_amdgcn_readlane((int)d, 0);
  h.t1 = (uint32_t)__builtin_amdgcn_readlane((int)d, 16);
  h.t2 = (uint32_t)__builtin_amdgcn_readlane((int)d, 32);
  h.t3 = (uint32_t)__builtin_amdgcn_readlane((int)d, 48);
  return h;
}

// Every q bit of the chain connected along it (periodically) to a bit of c,
// for c a subset of q.
__device__ __forceinline__ uint32_t column_fill(const ColumnChain& h, uint32_t c) {
  // upward; then what reaches lane 63 continues from lane 0
  uint32_t u = c;
  u |= dpp_zero<kRowShr1>(u) & h.q;
  u |= dpp_zero<kRowShr2>(u) & h.p1;
  u |= dpp_zero<kRowShr4>(u) & h.p2;
  u |= dpp_zero<kRowShr8>(u) & h.p3;
  u |= dpp_zero<kBcast15, 0xA>(u) & h.p4;
  u |= dpp_zero<kBcast31, 0xC>(u) & h.p5;
  u |= h.p6 & (uint32_t)__builtin_amdgcn_readlane((int)u, 63);
  // downward within rows, then across rows from the reach at each row's
  // lowest lane: r0 (lane 0, without the wrap) goes on from lane 63
  uint32_t d = c;
  d |= dpp_zero<kRowShl1>(d) & h.q;
  d |= dpp_zero<kRowShl2>(d) & h.d1;
  d |= dpp_zero<kRowShl4>(d) & h.d2;
  d |= dpp_zero<kRowShl8>(d) & h.d3;
  const uint32_t c0 = (uint32_t)__builtin_amdgcn_readlane((int)d, 0);
  const uint32_t c1 = (uint32_t)__builtin_amdgcn_readlane((int)d, 16);
  const uint32_t c2 = (uint32_t)__builtin_amdgcn_readlane((int)d, 32);
  const uint32_t c3 = (uint32_t)__builtin_amdgcn_readlane((int)d, 48);
  const uint32_t r0 = c0 | (h.t0 & (c1 | (h.t1 & (c2 | (h.t2 & c3)))));
  const uint32_t r48 = c3 | (h.t3 & r0);
  const uint32_t r32 = c2 | (h.t2 & r48);
  const uint32_t r16 = c1 | (h.t1 & r32);
  d |= (h.m0 & r16) | (h.m1 & r32) | (h.m2 & r48) | (h.m3 & r0);
  return u | d;
}

// The q site of rank m (counted in increasing x0) of a 64-site row held as
// its even-site word E and odd-site word O (site x0 = 2b + e is bit b of E
// for e = 0, of O for e = 1): sets that bit in SE or SO.  f(b), the number of
// q sites with x0 < 2b, is nondecreasing; a binary search finds the largest
// b with f(b) <= m, whose pair of sites holds the one sought.
__device__ __forceinline__ void rank_in_row64(uint32_t E, uint32_t O, uint32_t m, uint32_t& SE,
                                              uint32_t& SO) {
  int b = 0;
#pragma unroll
  for (int st = 16; st >= 1; st >>= 1) {
    const uint32_t lm = (1u << (b + st)) - 1u;
    if ((uint32_t)(__popc(E & lm) + __popc(O & lm)) <= m) b += st;
  }
  const uint32_t lm = (1u << b) - 1u;
  const bool even = ((E >> b) & 1u) && (uint32_t)(__popc(E & lm) + __popc(O & lm)) == m;
  SE = even ? 1u << b : 0u;
  SO = even ? 0u : 1u << b;
}

// The Houdayer cluster of pair k of a 2D sample with 64 rows (L = 64), one
// row per lane, everything in registers: overlap, seed (the m-th q = -1 site
// in site order, by a scan over lanes), flood fill alternating column fills
// and row closures until one of them adds nothing.  False (for the whole
// wavefront) if the pair has no q = -1 site; else c0, c1 are the cluster's
// colour-0 and colour-1 words of this lane's row.
__device__ __forceinline__ bool rows64_cluster(const Geo& g, const uint32_t* Wa, const uint32_t* Wb,
                                               int s, int k, uint32_t v, int lane, uint32_t& c0,
                                               uint32_t& c1) {
  const bool odd = lane & 1;  // parity of the row = colour of its even sites
  const uint32_t q0 = Wa[lane] ^ Wb[lane], q1 = Wa[64 + lane] ^ Wb[64 + lane];
  const uint32_t qx = odd ? q1 : q0, qy = odd ? q0 : q1;
  // q = -1 sites up to and including this row (a DPP scan over the rows)
  const uint32_t lc = __popc(q0) + __popc(q1);
  uint32_t incl = lc;
  incl += dpp_zero<kRowShr1>(incl);
  incl += dpp_zero<kRowShr2>(incl);
  incl += dpp_zero<kRowShr4>(incl);
  incl += dpp_zero<kRowShr8>(incl);
  incl += dpp_zero<kBcast15, 0xA>(incl);
  incl += dpp_zero<kBcast31, 0xC>(incl);
  const uint32_t n = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  if (n == 0) return false;
  // seed: the m-th q = -1 site in increasing site order (row by row)
  const Ctr4 r = philox10(Ctr4{(uint32_t)k, v, 0u, (kTagHou << 28) | (uint32_t)s}, g.key0, g.key1);
  const uint64_t r64 = (uint64_t)r.x | ((uint64_t)r.y << 32);
  const uint32_t m = (uint32_t)__umul64hi(r64, (uint64_t)n);
  uint32_t X = 0, Y = 0;  // cluster: even-site and odd-site words of the row
  if (m >= incl - lc && m < incl) rank_in_row64(qx, qy, m - (incl - lc), X, Y);
  const uint32_t rqx = __builtin_bitreverse32(qx), rqy = __builtin_bitreverse32(qy);
  row_closure(g, X, Y, qx, qy, rqx, rqy);
  const ColumnChain hx = column_chain(qx, lane), hy = column_chain(qy, lane);
  for (;;) {
    uint32_t nx = column_fill(hx, X), ny = column_fill(hy, Y);
    if (!__any(nx != X || ny != Y)) break;
    X = nx;
    Y = ny;
    row_closure(g, nx, ny, qx, qy, rqx, rqy);
    if (!__any(nx != X || ny != Y)) break;
    X = nx;
    Y = ny;
  }
  c0 = odd ? Y : X;
  c1 = odd ? X : Y;
  return true;
}

// The next pair of the Houdayer phase for this wavefront, from the hottest
// down (clusters grow larger and take more passes at high temperature), each
// to the next free wavefront; -1 when none is left.  Every lane adds 1 (one
// 64-count LDS atomic per take) and all read lane 0's result: a take under a
// lane-0 branch would let the compiler run the other lanes on into the next
// pair without it.  The counter is cleared after each Houdayer phase.
__device__ __forceinline__ int take_pair_hottest(uint32_t* hctr, int NT) {
  const uint32_t i = (uint32_t)__builtin_amdgcn_readfirstlane((int)atomicAdd(hctr, 1u)) >> 6;
  return i >= (uint32_t)NT ? -1 : NT - 1 - (int)i;
}

// Houdayer moves of a 2D sample with 64 rows (L = 64), one wavefront per
// pair at a time and one row per lane (rows64_cluster), then the energy
// change from the bonds leaving the cluster (vertical neighbours taken from
// the adjacent lanes) and the exchange on the cluster.
__device__ __forceinline__ void houdayer_rows64(const Geo& g, uint32_t* W, const uint32_t* Jl,
                                                int32_t* El, const int32_t* sotl, int s, uint32_t v,
                                                uint32_t* hctr, int lane) {
  const int NT = g.NT;
  const bool odd = lane & 1;
  for (;;) {
    const int k = take_pair_hottest(hctr, NT);
    if (k < 0) break;
    const int a = sotl[k], b = NT + sotl[NT + k];
    uint32_t* Wa = W + (size_t)a * 128;
    uint32_t* Wb = W + (size_t)b * 128;
    uint32_t c0, c1;
    if (!rows64_cluster(g, Wa, Wb, s, k, v, lane, c0, c1)) continue;
    const uint32_t a0 = Wa[lane], a1 = Wa[64 + lane], b0 = Wb[lane], b1 = Wb[64 + lane];
    // energy change of replica a over the bonds of the colour-0 sites (each
    // bond has one): +x0, -x0 in the row, +x1, -x1 in the next/previous row
    uint32_t nc[4], na[4];
    x0_neighbours(g, c1, odd, nc[0], nc[1]);
    x0_neighbours(g, a1, odd, na[0], na[1]);
    nc[2] = dpp_ones<kWaveRol1>(c1);  // row + 1 (lane 63 takes lane 0)
    nc[3] = dpp_ones<kWaveRor1>(c1);  // row - 1
    na[2] = dpp_ones<kWaveRol1>(a1);
    na[3] = dpp_ones<kWaveRor1>(a1);
    int cross = 0, cross_u = 0;
#pragma unroll
    for (int dir = 0; dir < 4; ++dir) {
      const uint32_t X = c0 ^ nc[dir];
      const uint32_t U = a0 ^ na[dir] ^ Jl[dir * 64 + lane];
      cross += __popc(X);
      cross_u += __popc(X & U);
    }
    uint32_t dsum = (uint32_t)(2 * (cross - 2 * cross_u));
    dsum += dpp_zero<kRowShr1>(dsum);
    dsum += dpp_zero<kRowShr2>(dsum);
    dsum += dpp_zero<kRowShr4>(dsum);
    dsum += dpp_zero<kRowShr8>(dsum);
    dsum += dpp_zero<kBcast15, 0xA>(dsum);
    dsum += dpp_zero<kBcast31, 0xC>(dsum);
    const int delta = __builtin_amdgcn_readlane((int)dsum, 63);
    Wa[lane] = a0 ^ c0;
    Wa[64 + lane] = a1 ^ c1;
    Wb[lane] = b0 ^ c0;
    Wb[64 + lane] = b1 ^ c1;
    if (lane == 0) {
      El[a] += delta;
      El[b] -= delta;
    }
  }
}

// ---------------------------------------------------------------------------
// Houdayer moves for all NT pairs of the resident sample: each wavefront
// takes one pair at a time and grows its cluster alone, so clusters of very
// different size (cold versus hot pairs) do not wait for one another.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void houdayer_resident(const FusedArgs& A, uint32_t* lds, int s,
                                                  uint32_t v) {
  const Geo& g = A.g;
  const int NT = g.NT, NW = g.NW, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, nwave = blockDim.x >> 6;
  uint32_t* W = lds + A.lay.W;
  const uint32_t* Jl = lds + A.lay.J;  // colour-0 direction words first
  int32_t* El = reinterpret_cast<int32_t*>(lds + A.lay.E);
  const int32_t* sotl = reinterpret_cast<const int32_t*>(lds + A.lay.sot);
  const int W2 = 2 * NW;
  uint32_t* Qw = lds + A.lay.Qs + (size_t)wave * 2 * W2;
  uint32_t* Cw = Qw + W2;
  const int rpl = (g.NR + 63) / 64;  // rows per lane for the seed search
  if (D == 2 && rows64_houdayer(g)) {
    houdayer_rows64(fixed_shape<2, 64>(g), W, Jl, El, sotl, s, v, lds + A.lay.hq, lane);
    __syncthreads();
    if (tid == 0) lds[A.lay.hq] = 0u;  // the next use is behind the step's barriers
    return;
  }
  for (int k = wave; k < NT; k += nwave) {
    const int a = sotl[k], b = NT + sotl[NT + k];
    uint32_t* Wa = W + (size_t)a * W2;
    uint32_t* Wb = W + (size_t)b * W2;
    int cnt = 0;
    for (int i = lane; i < W2; i += 64) {
      const uint32_t q = Wa[i] ^ Wb[i];
      Qw[i] = q;
      Cw[i] = 0;
      cnt += __popc(q);
    }
    const uint32_t n = (uint32_t)wave_sum(cnt);
    if (n == 0) continue;
    wave_lds_sync();
    // seed: the m-th q = -1 site in increasing i; lanes own contiguous rows
    const Ctr4 r = philox10(Ctr4{(uint32_t)k, v, 0u, (kTagHou << 28) | (uint32_t)s}, g.key0, g.key1);
    const uint64_t r64 = (uint64_t)r.x | ((uint64_t)r.y << 32);
    const uint32_t m = (uint32_t)__umul64hi(r64, (uint64_t)n);
    const int r0 = min(g.NR, lane * rpl), r1 = min(g.NR, r0 + rpl);
    uint32_t lc = 0;
    for (int R = r0; R < r1; ++R) lc += row_minus_count(g, Qw, R);
    const uint32_t incl = wave_inclusive_scan(lc, lane);
    if (m >= incl - lc && m < incl) seed_in_rows(g, Qw, Cw, r0, r1, m - (incl - lc));
    wave_lds_sync();
    // flood fill until no word of the pair changes
    for (bool first = true;; first = false) {
      int changed = 0;
      for (int w = lane; w < NW; w += 64)
        if (grow_pair<D>(g, Cw, Qw, w, first)) changed = 1;
      wave_lds_sync();
      if (!__any(changed)) break;
    }
    // energy change of replica a, then exchange the replicas on the cluster
    int dl = 0;
    for (int w = lane; w < NW; w += 64) dl += cluster_delta_word<D>(g, Cw, Wa, Jl, w);
    const int delta = wave_sum(dl);
    for (int i = lane; i < W2; i += 64) {
      const uint32_t cw = Cw[i];
      if (cw) {
        Wa[i] ^= cw;
        Wb[i] ^= cw;
      }
    }
    if (lane == 0) {
      El[a] += delta;
      El[b] -= delta;
    }
    wave_lds_sync();
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Multi-cluster Houdayer moves for all NT pairs of the resident sample: the
// first PC wavefronts (those with a scratch area) take the pairs in turn,
// each finding the exchanged clusters of its pair (multi_cluster_words),
// then applying them as the single-cluster move applies its cluster.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void houdayer_multi_resident(const FusedArgs& A, uint32_t* lds, int s,
                                                        uint32_t v) {
  const Geo& g = A.g;
  const int NT = g.NT, NW = g.NW, W2 = 2 * NW, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, PC = A.lay.PC;
  uint32_t* W = lds + A.lay.W;
  const uint32_t* Jl = lds + A.lay.J;
  int32_t* El = reinterpret_cast<int32_t*>(lds + A.lay.E);
  const int32_t* sotl = reinterpret_cast<const int32_t*>(lds + A.lay.sot);
  if (wave < PC) {
    const int stride = (multi_scratch_words(g.N, g.NR, NW) + 1) & ~1;
    uint32_t* Qw = lds + A.lay.Qs + (size_t)wave * stride;
    uint32_t* Cw = Qw + W2;
    for (int k = wave; k < NT; k += PC) {
      const int a = sotl[k], b = NT + sotl[NT + k];
      uint32_t* Wa = W + (size_t)a * W2;
      uint32_t* Wb = W + (size_t)b * W2;
      for (int i = lane; i < W2; i += 64) Qw[i] = Wa[i] ^ Wb[i];
      wave_lds_sync();
      multi_cluster_words<D>(g, Qw, Cw, Cw + W2, s, k, v, lane, 64, [] { wave_lds_sync(); });
      int dl = 0;
      for (int w = lane; w < NW; w += 64) dl += cluster_delta_word<D>(g, Cw, Wa, Jl, w);
      const int delta = wave_sum(dl);
      for (int i = lane; i < W2; i += 64) {
        const uint32_t cw = Cw[i];
        if (cw) {
          Wa[i] ^= cw;
          Wb[i] ^= cw;
        }
      }
      if (lane == 0) {
        El[a] += delta;
        El[b] -= delta;
      }
      wave_lds_sync();
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// One Metropolis sweep (colour 0, then colour 1) of the resident
// configurations ls in [0, nres): configuration ls is slot slot0 + ls, its
// words at W + ls * 2 NW, its couplings J (colour-c direction words at
// J + c * 2 D NW).  A configuration's colour-1 update reads only its own
// colour-0 words, so when each configuration's words fall to one wavefront
// (NW a multiple or a divisor of 64: the 64-item units of a configuration,
// or the whole configurations of a unit, all go to the same wavefront) every
// wavefront runs both half-sweeps of its configurations back to back,
// ordered by a wavefront-level LDS fence, as long as that spreads the words
// over the wavefronts as evenly as the flat loop; otherwise the workgroup
// meets between the colours.  Ends with a workgroup barrier.
// ---------------------------------------------------------------------------
template <int D, int LS>
__device__ __forceinline__ void sweep_resident_shape(const Geo& g, const FusedArgs& A,
                                                     const uint32_t* J, uint32_t* W, int32_t* El,
                                                     const int32_t* tosl, const uint32_t* thrl,
                                                     int slot0, int nres, int s, uint32_t t) {
  const int NW = g.NW, W2 = 2 * NW, items = nres * NW, tid = threadIdx.x, T = blockDim.x;
  auto update = [&](int it, int c) {
    const int ls = LS ? it / NW : (int)__umulhi((uint32_t)it, A.magicNW), w = it - ls * NW;
    const int slot = slot0 + ls;
    const int k = tosl[slot];
    int dE = 0;
    sweep_word<D>(g, W + ls * W2, J + c * 2 * D * NW, c, w, slot, s, t, thrl[k * 4 + 0],
                  thrl[k * 4 + 1], thrl[k * 4 + 2], dE);
    if (dE) atomicAdd(&El[slot], dE);
  };
  // whole configurations per wavefront only where that loads the wavefronts
  // as evenly as the flat loop (a split part can hold fewer configurations
  // than there are wavefronts)
  const int nwave = T >> 6;
  const bool owned =
      64 % NW == 0 ||
      (NW % 64 == 0 && (nres + nwave - 1) / nwave * nwave * NW <= (items + T - 1) / T * T);
  constexpr bool kWordPerLane = LS != 0 && geo_shape(LS, D).NW == 64;
  if constexpr (kWordPerLane) {
    // every unit is one configuration and lane w always updates word w: the
    // word's coupling words are loaded once per colour
    const int nunits = nres, lane = tid & 63, step = T >> 6;
    for (int c = 0; c < 2; ++c) {
      uint32_t jv[2 * D];
#pragma unroll
      for (int dir = 0; dir < 2 * D; ++dir) jv[dir] = J[(c * 2 * D + dir) * NW + lane];
      for (int u = tid >> 6; u < nunits; u += step) {
        const int slot = slot0 + u;
        const int k = tosl[slot];
        int dE = 0;
        sweep_word_j<D>(g, W + u * W2, jv, c, lane, slot, s, t, thrl[k * 4 + 0], thrl[k * 4 + 1],
                        thrl[k * 4 + 2], dE);
        if (dE) atomicAdd(&El[slot], dE);
      }
      if (c == 0) wave_lds_sync();
    }
  } else if (owned) {
    const int m = NW >= 64 ? NW >> 6 : 1;  // units per configuration (or 1)
    const int nunits = (items + 63) >> 6, lane = tid & 63, step = (T >> 6) * m;
    for (int c = 0; c < 2; ++c) {
      for (int u0 = (tid >> 6) * m; u0 < nunits; u0 += step)
        for (int u = u0; u < u0 + m; ++u) {
          const int it = (u << 6) + lane;
          if (it < items) update(it, c);
        }
      if (c == 0) wave_lds_sync();
    }
  } else {
    for (int it = tid; it < items; it += T) update(it, 0);
    __syncthreads();
    for (int it = tid; it < items; it += T) update(it, 1);
  }
  __syncthreads();
}

// The sweep with the geometry of the shapes the workloads run most folded to
// compile-time constants (3D L = 16, 2D L = 64; for split samples, which run
// one workgroup per CU whatever their registers, also 3D L = 24, 32 and 48),
// else from g.
template <int D, bool kSplitShapes = false>
__device__ __forceinline__ void sweep_resident(const FusedArgs& A, const uint32_t* J, uint32_t* W,
                                               int32_t* El, const int32_t* tosl,
                                               const uint32_t* thrl, int slot0, int nres, int s,
                                               uint32_t t) {
  constexpr int kFixedL = D == 3 ? 16 : 64;
  if (A.g.L == kFixedL) {
    sweep_resident_shape<D, kFixedL>(fixed_shape<D, kFixedL>(A.g), A, J, W, El, tosl, thrl, slot0,
                                     nres, s, t);
    return;
  }
  if constexpr (kSplitShapes && D == 3) {
    if (A.g.L == 32) {
      sweep_resident_shape<3, 32>(fixed_shape<3, 32>(A.g), A, J, W, El, tosl, thrl, slot0, nres,
                                  s, t);
      return;
    }
    if (A.g.L == 48) {
      sweep_resident_shape<3, 48>(fixed_shape<3, 48>(A.g), A, J, W, El, tosl, thrl, slot0, nres,
                                  s, t);
      return;
    }
    if (A.g.L == 24) {
      sweep_resident_shape<3, 24>(fixed_shape<3, 24>(A.g), A, J, W, El, tosl, thrl, slot0, nres,
                                  s, t);
      return;
    }
  }
  sweep_resident_shape<D, 0>(A.g, A, J, W, El, tosl, thrl, slot0, nres, s, t);
}

// ---------------------------------------------------------------------------
// nmcs Monte Carlo steps of sample s with replica sets [c_lo, c_lo + nsets)
// resident in LDS.  With one set only the sweep and the exchange run (the
// Houdayer move and the overlap need both sets).  Only the resident sets'
// state is written back, so the two sets of a sample may run in different
// workgroups at the same time.
// ---------------------------------------------------------------------------
// Adds the round trips a workgroup summed in LDS during the launch to the
// sample's totals (atomically: the sample's two replica sets may have run in
// two workgroups).
__device__ __forceinline__ void flush_trips(const FusedArgs& A, const uint32_t* lds, int s) {
  const uint64_t* bl = reinterpret_cast<const uint64_t*>(lds + A.lay.trip);
  unsigned long long* dst = reinterpret_cast<unsigned long long*>(A.trips) + (size_t)s * 32 * 3;
  for (int i = threadIdx.x; i < 32 * 3; i += blockDim.x)
    if (bl[i]) atomicAdd(dst + i, (unsigned long long)bl[i]);
}

template <int D, bool HOU, bool MEAS, bool WALK, bool MODES>
__device__ __forceinline__ void run_sample(const FusedArgs& A, uint32_t* lds, int s, int c_lo, int nsets) {
  const Geo& g = A.g;
  const int T = blockDim.x, tid = threadIdx.x;
  const int NW = g.NW, NT = g.NT, nslot = g.nslot, W2 = 2 * NW;
  const int slot0 = c_lo * NT, nres = nsets * NT;  // resident slots [slot0, slot0 + nres)
  uint32_t* W = lds + A.lay.W;                     // W[(slot - slot0) * W2 + ...]
  uint32_t* Jl = lds + A.lay.J;
  int32_t* El = reinterpret_cast<int32_t*>(lds + A.lay.E);
  int32_t* sotl = reinterpret_cast<int32_t*>(lds + A.lay.sot);
  int32_t* tosl = reinterpret_cast<int32_t*>(lds + A.lay.tos);
  uint32_t* thrl = lds + A.lay.thr;
  int64_t* mom = reinterpret_cast<int64_t*>(lds + A.lay.mom);
  const size_t lat0 = (size_t)s * nslot + slot0;
  const bool hou = HOU && A.hou && nsets == 2, meas = MEAS && A.meas && nsets == 2;

  // ---- load
  const int items = nres * NW;
  if (g.layout == kLayoutPacked) {
    const uint32_t* src = static_cast<const uint32_t*>(A.spins) + lat0 * W2;
    for (int i = tid; i < nres * W2; i += T) W[i] = src[i];
  } else {
    const int8_t* src = static_cast<const int8_t*>(A.spins) + lat0 * g.N;
#pragma unroll 2
    for (int it = tid; it < items; it += T) {
      const int ls = (int)__umulhi((uint32_t)it, A.magicNW), w = it - ls * NW;
      word_from_int8(g, src + (size_t)ls * g.N, w, W[ls * W2 + w], W[ls * W2 + NW + w]);
    }
  }
  const uint32_t* jws = A.jw + (size_t)s * 2 * 2 * D * NW;
  for (int i = tid; i < 2 * 2 * D * NW; i += T) Jl[i] = jws[i];
  for (int i = tid; i < nslot; i += T) El[i] = A.E[(size_t)s * nslot + i];
  for (int i = tid; i < 2 * NT; i += T) {
    sotl[i] = A.sot[(size_t)s * 2 * NT + i];
    tosl[i] = A.tos[(size_t)s * 2 * NT + i];
  }
  for (int i = tid; i < 4 * NT; i += T) thrl[i] = A.thr[i];
  if (meas)
    for (int i = tid; i < 8 * NT; i += T) mom[i] = A.mom[(size_t)s * NT * 8 + i];
  const bool modes = MODES && meas && A.modes != nullptr;
  const int MH = g.L / 2 + 1;
  int64_t* modl = reinterpret_cast<int64_t*>(lds + A.lay.modes);
  if (modes)
    for (int i = tid; i < NT * MH; i += T) modl[i] = A.modes[(size_t)s * NT * MH + i];
  const bool walk = WALK && A.walk != nullptr;
  int32_t* wkl = reinterpret_cast<int32_t*>(lds + A.lay.walk);
  if (walk) {
    for (int i = tid; i < 2 * nres; i += T) wkl[2 * slot0 + i] = A.walk[2 * lat0 + i];
    for (int i = tid; i < 2 * 32 * 3; i += T) lds[A.lay.trip + i] = 0u;
  }
  if (hou && tid == 0) lds[A.lay.hq] = 0u;
  const uint32_t t0 = A.ctr->t, u0 = A.ctr->u, v0 = A.ctr->v;
  __syncthreads();

  for (int step = 0; step < A.nmcs; ++step) {
    const uint32_t t = t0 + (uint32_t)step, u = u0 + (uint32_t)step;
    exchange_prepare(A, lds, s, u, c_lo, nsets);
    sweep_resident<D>(A, Jl, W, El, tosl, thrl, slot0, nres, s, t);
    if (hou) {
      if (A.hou == 2)
        houdayer_multi_resident<D>(A, lds, s, v0 + (uint32_t)step);
      else
        houdayer_resident<D>(A, lds, s, v0 + (uint32_t)step);
    }
    exchange_resident<WALK>(A, lds, c_lo, nsets, u + 1u, walk);
    if (meas && measures_at(t + 1u, (uint32_t)A.every)) measure_resident<MODES>(A, lds);
  }

  // ---- store the resident sets
  if (g.layout == kLayoutPacked) {
    uint32_t* dst = static_cast<uint32_t*>(A.spins) + lat0 * W2;
    for (int i = tid; i < nres * W2; i += T) dst[i] = W[i];
  } else {
    int8_t* dst = static_cast<int8_t*>(A.spins) + lat0 * g.N;
#pragma unroll 2
    for (int it = tid; it < items; it += T) {
      const int ls = (int)__umulhi((uint32_t)it, A.magicNW), w = it - ls * NW;
      word_to_int8(g, dst + (size_t)ls * g.N, w, W[ls * W2 + w], W[ls * W2 + NW + w]);
    }
  }
  for (int i = tid; i < nres; i += T) A.E[lat0 + i] = El[slot0 + i];
  for (int i = tid; i < nres; i += T) {
    A.sot[(size_t)s * 2 * NT + slot0 + i] = sotl[slot0 + i];
    A.tos[(size_t)s * 2 * NT + slot0 + i] = tosl[slot0 + i];
  }
  if (walk) {
    for (int i = tid; i < 2 * nres; i += T) A.walk[2 * lat0 + i] = wkl[2 * slot0 + i];
    flush_trips(A, lds, s);
  }
  if (modes)
    for (int i = tid; i < NT * MH; i += T) A.modes[(size_t)s * NT * MH + i] = modl[i];
  if (meas)
    for (int i = tid; i < 8 * NT; i += T) A.mom[(size_t)s * NT * 8 + i] = mom[i];
}

// ---------------------------------------------------------------------------
// Samples too large for one workgroup.  The 2 N_T configurations of a sample
// are split into `parts` groups of R slots, one workgroup each, for all steps
// of the launch: a replica exchange only relabels temperatures, so a
// configuration never changes workgroup.  Each step every part publishes the
// energies of its slots (and, when measuring, their configurations) to
// parity-double-buffered global scratch and meets the other parts at a
// per-sample counter barrier; then every part takes the same exchange
// decisions from the same energies and Philox words, so the maps agree
// without further communication, and temperature k is measured by the part
// holding its replica-set-0 configuration, which reads the set-1 partner from
// LDS or from the published configurations (only set-1 slots are published).
// A part overwrites a parity buffer two steps later, after a barrier that
// every reader of it has passed.
// ---------------------------------------------------------------------------

// About 60 s of the 100 MHz constant clock: far beyond any legitimate wait
// (all parts of a sample are taken from the queue together), so reaching it
// means the job's state can no longer be trusted.
constexpr uint64_t kBarrierTicks = 6000000000ull;

// Arrives at a sample's barrier and waits for `target` arrivals in all.
// Returns false if the wait gave up; the job's fault word is then set, and
// every later wait of the job gives up at once.  Only thread 0 synchronises
// with the other parts: every wavefront first waits until its own stores have
// completed (they are then in this XCD's L2, whose dirty lines thread 0's
// release writes back), and the workgroup barrier after thread 0's acquire fence
// (which invalidates the caches) orders every later load after it.
__device__ __forceinline__ bool part_barrier(uint32_t* bar, uint32_t target, uint32_t* fault,
                                             int* flag) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    const uint64_t t0 = wall_clock64();
    // poll with relaxed loads and acquire once, after the count is reached:
    // an acquire load invalidates caches on every poll, which would also
    // evict the data other workgroups on the same L2 are computing with
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 > kBarrierTicks) {
        __hip_atomic_store(fault, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    // the relaxed load read the value of the other parts' release increments:
    // this fence makes their published energies and words visible
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag = good;
  }
  __syncthreads();
  return *flag != 0;
}

// Overlaps and moment increments of the temperatures whose replica-set-0
// configuration this part holds (its slots below N_T, at temperature tos[r]),
// each against its set-1 partner: from LDS when this part holds the partner
// too, else from the words published this step (`pub`: [nslot][2NW], set-1
// slots).  The increments go to this part's LDS sums, which start each launch
// at zero and are combined across parts at its end (combine_split_moments).
// With the modes kept, the parts publish every slot and temperature k's modes
// are taken by part k mod parts from the published words.
template <bool MODES>
__device__ __forceinline__ void measure_split(const FusedArgs& A, uint32_t* lds, int part, int slot0,
                                              int nres, const uint32_t* W, const uint32_t* pub) {
  const Geo& g = A.g;
  const int NT = g.NT, W2 = 2 * g.NW, tid = threadIdx.x, T = blockDim.x;
  const int32_t* El = reinterpret_cast<const int32_t*>(lds + A.lay.E);
  const int32_t* sotl = reinterpret_cast<const int32_t*>(lds + A.lay.sot);
  const int32_t* tosl = reinterpret_cast<const int32_t*>(lds + A.lay.tos);
  int32_t* qneg = reinterpret_cast<int32_t*>(lds + A.lay.qneg);
  int64_t* mom = reinterpret_cast<int64_t*>(lds + A.lay.mom);
  const int n0 = max(0, min(slot0 + nres, NT) - slot0);  // this part's set-0 slots
  const int wave = tid >> 6, lane = tid & 63, nwave = T >> 6;
  for (int i = tid; i < n0; i += T) qneg[i] = 0;
  __syncthreads();
  // the (pair, 64-word chunk) space is cut into one contiguous range per
  // wavefront, so that every wavefront has many independent loads in flight
  // whatever the number of pairs; a wavefront adds its lanes' counts of the
  // differing sites once per pair in its range
  const int C64 = (W2 + 63) >> 6, items = n0 * C64, per = (items + nwave - 1) / nwave;
  const int hi = min(items, (wave + 1) * per);
  for (int it = wave * per; it < hi;) {
    const int i = it / C64, c1 = min(hi - i * C64, C64);
    const int r = slot0 + i, b = NT + sotl[NT + tosl[r]];
    const uint32_t* pa = W + (size_t)i * W2;
    const uint32_t* pb = (b < slot0 + nres) ? W + (size_t)(b - slot0) * W2 : pub + (size_t)b * W2;
    int neg = 0;
#pragma unroll 8
    for (int c = it - i * C64; c < c1; ++c) {
      const int w = c * 64 + lane;
      if (w < W2) neg += __popc(pa[w] ^ pb[w]);
    }
    neg = wave_total(neg);
    if (lane == 0 && neg) atomicAdd(&qneg[i], neg);
    it = i * C64 + c1;
  }
  __syncthreads();
  for (int i = tid; i < n0; i += T) {
    const int r = slot0 + i, k = tosl[r];
    add_moments(g, mom + (size_t)k * 8, El[r], El[NT + sotl[NT + k]], qneg[i]);
  }
  if (MODES && A.modes) {
    // the owned temperatures' modes, one wavefront each, from the published words
    const int nk = (NT - part + A.parts - 1) / A.parts;
    for (int kl = wave; kl < nk; kl += nwave) {
      const int k = part + kl * A.parts;
      modes_resident(g, A.lay, lds, pub + (size_t)sotl[k] * W2, pub + (size_t)(NT + sotl[NT + k]) * W2,
                     k, wave, lane);
    }
  }
  __syncthreads();
}

// The end of a measuring launch of a split sample: every part writes its
// moment increments to `scr` ([parts][N_T][8] 64-bit words; free once every
// part has passed the last step's barrier), meets the other parts once more,
// and part k mod parts adds the increments of temperature k (the Q^4 sum as a
// 128-bit pair) to the sums in global memory.  False if the wait gave up.
__device__ __forceinline__ bool combine_split_moments(const FusedArgs& A, const int64_t* mom, int s,
                                                      int part, uint64_t* scr, uint32_t* bar,
                                                      uint32_t target, uint32_t* fault, int* flag) {
  const int NT = A.g.NT, tid = threadIdx.x, T = blockDim.x;
  for (int i = tid; i < 8 * NT; i += T) scr[(size_t)part * 8 * NT + i] = (uint64_t)mom[i];
  if (!part_barrier(bar, target, fault, flag)) return false;
  for (int k = part + tid * A.parts; k < NT; k += T * A.parts) {
    uint64_t* dst = reinterpret_cast<uint64_t*>(A.mom) + ((size_t)s * NT + k) * 8;
    uint64_t m[8];
    for (int j = 0; j < 8; ++j) m[j] = dst[j];
    for (int p = 0; p < A.parts; ++p) {
      const uint64_t* q = scr + ((size_t)p * NT + k) * 8;
      for (int j = 0; j < 5; ++j) m[j] += q[j];
      const uint64_t lo = m[5] + q[5];
      m[6] += q[6] + (lo < m[5] ? 1u : 0u);
      m[5] = lo;
      m[7] += q[7];
    }
    for (int j = 0; j < 8; ++j) dst[j] = m[j];
  }
  return true;
}

// nmcs Monte Carlo steps (sweep, exchange, measurement) of part `part` of
// split sample s.
template <int D, bool MEAS, bool WALK, bool MODES>
__device__ __forceinline__ void run_split(const FusedArgs& A, uint32_t* lds, int s, int part,
                                          int* flag) {
  const Geo& g = A.g;
  const int T = blockDim.x, tid = threadIdx.x;
  const int NW = g.NW, NT = g.NT, nslot = g.nslot, W2 = 2 * NW;
  const int slot0 = part * A.R, nres = min(A.R, nslot - slot0);
  uint32_t* W = lds + A.lay.W;
  int32_t* El = reinterpret_cast<int32_t*>(lds + A.lay.E);
  int32_t* sotl = reinterpret_cast<int32_t*>(lds + A.lay.sot);
  int32_t* tosl = reinterpret_cast<int32_t*>(lds + A.lay.tos);
  uint32_t* thrl = lds + A.lay.thr;
  int64_t* mom = reinterpret_cast<int64_t*>(lds + A.lay.mom);
  const size_t lat0 = (size_t)s * nslot + slot0;
  const bool meas = MEAS && A.meas != 0;

  // ---- load this part's slots and the sample's shared state
  const int items = nres * NW;
  if (g.layout == kLayoutPacked) {
    const uint32_t* src = static_cast<const uint32_t*>(A.spins) + lat0 * W2;
    for (int i = tid; i < nres * W2; i += T) W[i] = src[i];
  } else {
    const int8_t* src = static_cast<const int8_t*>(A.spins) + lat0 * g.N;
#pragma unroll 2
    for (int it = tid; it < items; it += T) {
      const int ls = (int)__umulhi((uint32_t)it, A.magicNW), w = it - ls * NW;
      word_from_int8(g, src + (size_t)ls * g.N, w, W[ls * W2 + w], W[ls * W2 + NW + w]);
    }
  }
  const uint32_t* Jsrc = A.jw + (size_t)s * 2 * 2 * D * NW;
  if (A.jlds) {
    uint32_t* Jl = lds + A.lay.J;
    for (int i = tid; i < 2 * 2 * D * NW; i += T) Jl[i] = Jsrc[i];
    Jsrc = Jl;
  }
  for (int i = tid; i < nslot; i += T) El[i] = A.E[(size_t)s * nslot + i];
  for (int i = tid; i < 2 * NT; i += T) {
    sotl[i] = A.sot[(size_t)s * 2 * NT + i];
    tosl[i] = A.tos[(size_t)s * 2 * NT + i];
  }
  for (int i = tid; i < 4 * NT; i += T) thrl[i] = A.thr[i];
  // this launch's moment increments (combined across parts at its end)
  if (meas)
    for (int i = tid; i < 8 * NT; i += T) mom[i] = 0;
  // mode sums of the temperatures this part measures (k = part mod parts)
  const bool modes = MODES && meas && A.modes != nullptr;
  const int MH = g.L / 2 + 1;
  int64_t* modl = reinterpret_cast<int64_t*>(lds + A.lay.modes);
  if (modes)
    for (int k = part; k < NT; k += A.parts)
      for (int i = tid; i < MH; i += T) modl[k * MH + i] = A.modes[((size_t)s * NT + k) * MH + i];
  // part 0 keeps the sample's replica walk
  const bool walk = WALK && A.walk != nullptr && part == 0;
  int32_t* wkl = reinterpret_cast<int32_t*>(lds + A.lay.walk);
  if (walk) {
    for (int i = tid; i < 2 * nslot; i += T) wkl[i] = A.walk[(size_t)s * 2 * nslot + i];
    for (int i = tid; i < 2 * 32 * 3; i += T) lds[A.lay.trip + i] = 0u;
  }
  const uint32_t t0 = A.ctr->t, u0 = A.ctr->u;
  uint32_t* bar = A.bar + s;
  uint32_t* fault = A.bar + g.S;
  int32_t* Ex = A.Ex + (size_t)s * 2 * nslot;
  uint32_t* snap = A.snap + (size_t)s * 2 * nslot * W2;
  bool good = true;
  __syncthreads();

  for (int step = 0; step < A.nmcs; ++step) {
    const uint32_t t = t0 + (uint32_t)step, u = u0 + (uint32_t)step;
    exchange_prepare(A, lds, s, u, 0, 2);
    sweep_resident<D, true>(A, Jsrc, W, El, tosl, thrl, slot0, nres, s, t);
    // publish, meet, and take the sample-wide steps
    const int par = step & 1;
    const bool mstep = meas && measures_at(t + 1u, (uint32_t)A.every);
    for (int i = tid; i < nres; i += T) Ex[par * nslot + slot0 + i] = El[slot0 + i];
    if (mstep) {
      // the set-1 slots (every slot when the modes are kept)
      const int first = modes ? 0 : min(nres, max(0, NT - slot0));
      uint32_t* dst = snap + ((size_t)par * nslot + slot0) * W2;
      for (int i = first * W2 + tid; i < nres * W2; i += T) dst[i] = W[i];
    }
    if (!part_barrier(bar, (uint32_t)(A.parts * (step + 1)), fault, flag)) {
      good = false;
      break;
    }
    for (int i = tid; i < nslot; i += T) El[i] = Ex[par * nslot + i];
    __syncthreads();
    exchange_resident<WALK>(A, lds, 0, 2, u + 1u, walk);
    if (mstep) measure_split<MODES>(A, lds, part, slot0, nres, W, snap + (size_t)par * nslot * W2);
  }
  if (meas && good)
    combine_split_moments(A, mom, s, part,
                          reinterpret_cast<uint64_t*>(snap + (size_t)(A.nmcs & 1) * nslot * W2), bar,
                          (uint32_t)(A.parts * (A.nmcs + 1)), fault, flag);

  // ---- store this part's slots; part 0 stores the maps, owners the modes
  if (g.layout == kLayoutPacked) {
    uint32_t* dst = static_cast<uint32_t*>(A.spins) + lat0 * W2;
    for (int i = tid; i < nres * W2; i += T) dst[i] = W[i];
  } else {
    int8_t* dst = static_cast<int8_t*>(A.spins) + lat0 * g.N;
#pragma unroll 2
    for (int it = tid; it < items; it += T) {
      const int ls = (int)__umulhi((uint32_t)it, A.magicNW), w = it - ls * NW;
      word_to_int8(g, dst + (size_t)ls * g.N, w, W[ls * W2 + w], W[ls * W2 + NW + w]);
    }
  }
  for (int i = tid; i < nres; i += T) A.E[lat0 + i] = El[slot0 + i];
  if (part == 0)
    for (int i = tid; i < 2 * NT; i += T) {
      A.sot[(size_t)s * 2 * NT + i] = sotl[i];
      A.tos[(size_t)s * 2 * NT + i] = tosl[i];
    }
  if (walk) {
    for (int i = tid; i < 2 * nslot; i += T) A.walk[(size_t)s * 2 * nslot + i] = wkl[i];
    flush_trips(A, lds, s);
  }
  if (modes)
    for (int k = part; k < NT; k += A.parts)
      for (int i = tid; i < MH; i += T) A.modes[((size_t)s * NT + k) * MH + i] = modl[k * MH + i];
}

// ---------------------------------------------------------------------------
// Persistent batch kernel: workgroups take (job, sample, sets) items from a
// shared queue until it is empty.  Each job brings its own geometry,
// tables, state and LDS plan.  F says which kinds of work the launch holds
// (kFeatHou, kFeatMeas, kFeatSplit): code for the others is left out, which
// keeps the register count, and so the number of resident wavefronts, of a
// launch as low as its work allows.
// ---------------------------------------------------------------------------
// Wavefronts per SIMD the register allocation must allow.  The sweep +
// exchange (+ measurement, + replica walk) kernels are held to the 80 VGPRs
// that two 768-thread workgroups per CU need: left alone the scheduler takes
// a few more (for values used once per item, which then go to scratch
// instead, outside the step loop).  Every other variant gets what a
// 1024-thread workgroup needs.
template <int F>
constexpr int kWavesPerSimd = !(F & (kFeatHou | kFeatSplit)) ? 6 : 4;

template <int D, int F>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd<F>)))
k_batch(const FusedArgs* __restrict__ jobs, const BatchItem* __restrict__ items, int nitems,
        uint32_t* queue) {
  constexpr bool kHou = (F & kFeatHou) != 0, kMeas = (F & kFeatMeas) != 0;
  constexpr bool kSplit = (F & kFeatSplit) != 0, kWalk = (F & kFeatWalk) != 0;
  constexpr bool kModes = (F & kFeatModes) != 0;
  // 16-byte aligned: the moment words are updated with 64-bit LDS atomics,
  // which need naturally aligned addresses (the plan offsets are 8-byte
  // aligned relative to this base)
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ int cur, flag;
  for (;;) {
    if (threadIdx.x == 0) cur = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int i = __builtin_amdgcn_readfirstlane(cur);
    __syncthreads();
    if (i >= nitems) break;
    const BatchItem it = items[i];
    const FusedArgs A = jobs[it.job];
    if (A.nmcs > 0) {
      if (kSplit && it.nsets == 0)
        run_split<D, kMeas, kWalk, kModes>(A, lds, it.sample, it.c_lo, &flag);
      else
        run_sample<D, kHou, kMeas, kWalk, kModes>(A, lds, it.sample, it.c_lo, it.nsets);
    }
    __syncthreads();
  }
}

// Pointer to one variant of the batch kernel.
using BatchKernel = void (*)(const FusedArgs*, const BatchItem*, int, uint32_t*);

// The variant k_batch<D, BASE + feat> for feat in [0, sizeof...(F)).
template <int D, int BASE, int... F>
BatchKernel pick_kernel(int feat, std::integer_sequence<int, F...>, std::integral_constant<int, BASE>) {
  BatchKernel k = nullptr;
  ((k = (feat == F ? &k_batch<D, BASE + F> : k)), ...);
  return k;
}

// Defined in fused_k2a/k2b/k3a/k3b.hip: dimension 2 or 3, feature sets in
// [0, 16) (a) or [16, 32) (b).
BatchKernel batch_kernel_2a(int feat);
BatchKernel batch_kernel_2b(int feat);
BatchKernel batch_kernel_3a(int feat);
BatchKernel batch_kernel_3b(int feat);

}  // namespace ptsg
