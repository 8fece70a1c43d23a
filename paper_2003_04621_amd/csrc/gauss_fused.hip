// gauss_fused.hip -- whole Monte Carlo steps of Gaussian-coupling jobs in one
// launch (Sec. 2.4 with the Gaussian couplings of Sec. 2.1): Metropolis
// sweep, single-cluster Houdayer move per same-temperature pair, replica
// exchange pass and measurement, n steps per launch.  One workgroup holds
// one disorder sample, all 2 N_T configurations resident in LDS as
// colour-split row words, their 64-bit energies, the maps, the inverse
// temperatures and the moment sums; the coupling groups are read from global
// memory (each workgroup's sample stays in its XCD's L2).  HBM is touched to
// load the state at the start and store it at the end.
//
// Results are bit-identical to the per-step Gaussian kernels (gauss.hip):
// the same site groups and Philox counters, the same acceptance tiers, the
// exchange pass in ascending k with the updated map, the Houdayer seed as the
// m-th q = -1 site in increasing site order and the cluster as its connected
// component (found here by one wavefront per pair).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fused_device.h"
#include "gauss.h"
#include "gauss_kernels.h"

namespace ptsg {

namespace {

// Threads of the fused Gaussian workgroup: one per site group of a colour,
// at least 256 (four wavefronts for the Houdayer pairs), at most 512.
int gauss_fused_threads(const Geo& g) {
  const int groups = gauss_groups(g);
  return std::min(512, std::max(256, (groups + 63) / 64 * 64));
}

// LDS word offsets (64-bit arrays first, so that they stay 8-byte aligned).
struct GaussLayout {
  int E, beta, mom, cz, sot, tos, hq, W, Qs, words;
};

GaussLayout gauss_layout(const Geo& g, int nwave) {
  GaussLayout l;
  int o = 0;
  l.E = o;     o += 2 * 2 * g.NT;           // int64 [2 N_T] energies (2^-16 units)
  l.beta = o;  o += 2 * g.NT;               // double [N_T]
  l.mom = o;   o += 2 * 8 * g.NT;           // int64 [N_T][8] moment sums
  l.cz = o;    o += g.NT;                   // float [N_T] the float32 tier's constants
  l.sot = o;   o += 2 * g.NT;               // int32 [2][N_T]
  l.tos = o;   o += 2 * g.NT;               // int32 [2][N_T]
  l.hq = o;    o += 1;                      // the in-register Houdayer move's pair counter
  l.W = o;     o += 2 * g.NT * 2 * g.NW;    // [2 N_T][2 NW] configuration words
  // per wavefront: overlap and cluster words of the word-hop flood fill
  l.Qs = o;    o += rows64_houdayer(g) ? 0 : nwave * 4 * g.NW;
  l.words = o;
  return l;
}

// Wavefront sum of a 64-bit value.
__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Single-cluster Houdayer moves of all N_T pairs, one wavefront per pair at a
// time: overlap words, the seed (the m-th q = -1 site), the flood fill to the
// seed's connected q = -1 component, the energy change of replica a from the
// Gaussian couplings, then the exchange of the two configurations on the
// cluster.  Ends with a workgroup barrier.
template <int D>
__device__ void gauss_houdayer_resident(const Geo& g, uint32_t* W, int64_t* El, const int32_t* sotl,
                                        uint32_t* Qs, const int4* __restrict__ J0, int s,
                                        uint32_t v) {
  const int NT = g.NT, NW = g.NW, W2 = 2 * NW;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));  // as in gauss_houdayer_rows64
  const int wave = tid >> 6, lane = tid & 63, nwave = blockDim.x >> 6;
  uint32_t* Qw = Qs + (size_t)wave * 2 * W2;
  uint32_t* Cw = Qw + W2;
  const int rpl = (g.NR + 63) / 64;  // rows per lane for the seed search
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
    const uint32_t n = (uint32_t)wave_total(cnt);
    if (n == 0) continue;
    wave_lds_sync();
    const Ctr4 r = philox10(Ctr4{(uint32_t)k, v, 0u, (kTagHou << 28) | (uint32_t)s}, g.key0, g.key1);
    const uint64_t r64 = (uint64_t)r.x | ((uint64_t)r.y << 32);
    const uint32_t m = (uint32_t)__umul64hi(r64, (uint64_t)n);
    const int r0 = min(g.NR, lane * rpl), r1 = min(g.NR, r0 + rpl);
    uint32_t lc = 0;
    for (int R = r0; R < r1; ++R) lc += row_minus_count(g, Qw, R);
    const uint32_t incl = wave_inclusive_scan(lc, lane);
    if (m >= incl - lc && m < incl) seed_in_rows(g, Qw, Cw, r0, r1, m - (incl - lc));
    wave_lds_sync();
    for (bool first = true;; first = false) {
      int changed = 0;
      for (int w = lane; w < NW; w += 64)
        if (grow_pair<D>(g, Cw, Qw, w, first)) changed = 1;
      wave_lds_sync();
      if (!__any(changed)) break;
    }
    const int64_t delta = wave_sum64(gauss_cluster_delta<D>(g, Cw, Wa, J0, lane, 64));
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

// The same for a 2D sample with 64 rows (L = 64, one row per word): the
// cluster is found in registers, one row per lane (rows64_cluster), pairs from
// the hottest down; the energy change sums, over the cluster's boundary bonds
// from this row's colour-0 sites (a few per row), the bond's -2n from its
// coupling group with the sign of replica a across it.  Ends with a workgroup
// barrier, after which the pair counter is cleared.
__device__ void gauss_houdayer_rows64(const Geo& g, uint32_t* W, int64_t* El, const int32_t* sotl,
                                      const int4* __restrict__ J0, int s, uint32_t v, uint32_t* hctr) {
  const int NT = g.NT, NGc = gauss_groups(g);
  // recomputed at every call: what derives from the lane index (masks,
  // addresses) would otherwise be hoisted out of the step loop and stay live
  // through the sweep
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
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
    // the colour-0 sites' bonds: +x0, -x0 in the row, +x1, -x1 to the
    // next/previous row, the order of the coupling groups' directions
    uint32_t nc[4], na[4];
    x0_neighbours(g, c1, odd, nc[0], nc[1]);
    x0_neighbours(g, a1, odd, na[0], na[1]);
    nc[2] = dpp_ones<kWaveRol1>(c1);
    nc[3] = dpp_ones<kWaveRor1>(c1);
    na[2] = dpp_ones<kWaveRol1>(a1);
    na[3] = dpp_ones<kWaveRor1>(a1);
    int64_t dl = 0;
#pragma unroll
    for (int dir = 0; dir < 4; ++dir) {
      const uint32_t X = c0 ^ nc[dir];  // bonds leaving the cluster
      const uint32_t U = a0 ^ na[dir];  // replica a antiparallel across them
      for (uint32_t grp = X; grp;) {
        const int q = __builtin_ctz(grp) >> 2;  // group of four sites of the row
        const uint32_t xb = (X >> (4 * q)) & 0xFu, ub = (U >> (4 * q)) & 0xFu;
        grp &= ~(0xFu << (4 * q));
        const int4 m = J0[(size_t)dir * NGc + lane + 64 * q];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if ((xb >> j) & 1u) dl += ((ub >> j) & 1u) ? lane_of(m, j) : -lane_of(m, j);
      }
    }
    const int64_t delta = wave_sum64(dl);
    Wa[lane] = a0 ^ c0;
    Wa[64 + lane] = a1 ^ c1;
    Wb[lane] = b0 ^ c0;
    Wb[64 + lane] = b1 ^ c1;
    if (lane == 0) {
      El[a] += delta;
      El[b] -= delta;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *hctr = 0u;  // the next use is behind the step's barriers
}

// One workgroup per sample, `n` steps of sweep (+ Houdayer) + exchange
// (+ measurement at the job's interval).  The counters are read at the start;
// the caller advances them by n steps afterwards.
template <int D, bool HOU, bool MEAS>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_gfused(Geo g, void* spins, const int4* __restrict__ Jg,
                                                int64_t* __restrict__ E64, int32_t* __restrict__ sot,
                                                int32_t* __restrict__ tos,
                                                const double* __restrict__ beta,
                                                const float* __restrict__ cz, int64_t* __restrict__ mom,
                                                const DevCounters* __restrict__ ctr, int n, int every,
                                                GaussLayout lay) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int T = blockDim.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = T >> 6;
  const int NT = g.NT, NW = g.NW, W2 = 2 * NW, NS = 2 * NT, NGc = gauss_groups(g);
  const int s = blockIdx.x;
  int64_t* El = reinterpret_cast<int64_t*>(lds + lay.E);
  double* bl = reinterpret_cast<double*>(lds + lay.beta);
  int64_t* ml = reinterpret_cast<int64_t*>(lds + lay.mom);
  float* czl = reinterpret_cast<float*>(lds + lay.cz);
  int32_t* sotl = reinterpret_cast<int32_t*>(lds + lay.sot);
  int32_t* tosl = reinterpret_cast<int32_t*>(lds + lay.tos);
  uint32_t* W = lds + lay.W;
  const size_t lat0 = (size_t)s * g.nslot;

  // ---- load the sample's state
  for (int l = 0; l < NS; ++l) load_lattice(g, spins, lat0 + l, W + (size_t)l * W2, tid, T);
  for (int i = tid; i < NS; i += T) {
    El[i] = E64[lat0 + i];
    sotl[i] = sot[(size_t)s * NS + i];
    tosl[i] = tos[(size_t)s * NS + i];
  }
  for (int i = tid; i < NT; i += T) {
    bl[i] = beta[i];
    czl[i] = cz[i];
  }
  if (MEAS)
    for (int i = tid; i < 8 * NT; i += T) ml[i] = mom[(size_t)s * NT * 8 + i];
  if (tid == 0) lds[lay.hq] = 0u;
  const uint32_t t0 = load_counter(&ctr->t), u0 = load_counter(&ctr->u), v0 = load_counter(&ctr->v);
  __syncthreads();

  const int4* Js = Jg + (size_t)s * 2 * (2 * D + 1) * NGc;
  const uint32_t c3 = (kTagMetro << 28) | (uint32_t)s;
  for (int step = 0; step < n; ++step) {
    const uint32_t t = t0 + (uint32_t)step;
    // ---- Metropolis sweep: colour 0 of every configuration, then colour 1.
    // A thread takes a group of four same-colour sites (one Philox call, its
    // coupling data in registers) and updates it in every configuration.
    for (int c = 0; c < 2; ++c) {
      const int4* Jc = Js + (size_t)c * (2 * D + 1) * NGc;
      const uint32_t c1 = 2u * t + (uint32_t)c;
      for (int gi0 = 0; gi0 < NGc; gi0 += T) {
        // the group's position is recomputed every step: hoisted out of the
        // step loop it would stay live through the Houdayer move, whose
        // in-register cluster then no longer fits the register budget
        int gi = gi0 + tid;
        asm volatile("" : "+v"(gi));
        const bool valid = gi < NGc;
        int4 m[2 * D];
        int4 hs = make_int4(0, 0, 0, 0);
        GroupPos gp{};
        WordNb nb{};
        int p = 0;
        uint32_t c0 = 0;
        if (valid) {
#pragma unroll
          for (int k = 0; k < 2 * D; ++k) m[k] = Jc[(size_t)k * NGc + gi];
          hs = Jc[(size_t)2 * D * NGc + gi];
          gp = group_pos(g, gi);
          nb = word_nb(g, gp.w);
          p = (c + nb.par) & 1;
          c0 = (uint32_t)word_row(g, nb, gp.f) * (uint32_t)g.G + (uint32_t)gp.q;
        }
        if constexpr (D == 2) {
          // two configurations per round (2 N_T is even): two independent
          // chains of loads, Philox rounds and compares for the scheduler
          for (int l = 0; l < NS; l += 2) {
            int dE0 = 0, dE1 = 0;
            if (valid) {
              uint32_t* W0 = W + (size_t)l * W2;
              uint32_t* W1 = W0 + W2;
              const uint32_t Wc0 = W0[c * NW + gp.w], Wc1 = W1[c * NW + gp.w];
              uint32_t n0[2 * D], n1[2 * D], a0[2 * D], a1[2 * D];
              neighbour_words<D>(g, W0 + (1 - c) * NW, gp.w, nb, p, n0);
              neighbour_words<D>(g, W1 + (1 - c) * NW, gp.w, nb, p, n1);
#pragma unroll
              for (int k = 0; k < 2 * D; ++k) {
                a0[k] = (Wc0 ^ n0[k]) >> gp.shift;
                a1[k] = (Wc1 ^ n1[k]) >> gp.shift;
              }
              const Ctr4 r0 = philox10(Ctr4{c0, c1, (uint32_t)l, c3}, g.key0, g.key1);
              const Ctr4 r1 = philox10(Ctr4{c0, c1, (uint32_t)l + 1u, c3}, g.key0, g.key1);
              const int k0 = tosl[l], k1 = tosl[l + 1];
              int x0[4], x1[4];
              uint32_t F0, F1, u0, u1;
              gauss_group_fast<D>(a0, m, hs, gp.nv, r0, czl[k0], x0, F0, u0);
              gauss_group_fast<D>(a1, m, hs, gp.nv, r1, czl[k1], x1, F1, u1);
              F0 = gauss_group_finish(x0, r0, bl[k0], F0, u0, dE0);
              F1 = gauss_group_finish(x1, r1, bl[k1], F1, u1, dE1);
              if (F0) atomicXor(&W0[c * NW + gp.w], F0 << gp.shift);
              if (F1) atomicXor(&W1[c * NW + gp.w], F1 << gp.shift);
            }
            // every lane of the workgroup runs every round: DPP wavefront sums
            // (|sum| < 64 x 4 x 2 x 6 x 2^19 < 2^31), one LDS atomic each
            dE0 = wave_total(dE0);
            dE1 = wave_total(dE1);
            if (lane == 0) {
              if (dE0)
                atomicAdd(reinterpret_cast<unsigned long long*>(&El[l]), (unsigned long long)(int64_t)dE0);
              if (dE1)
                atomicAdd(reinterpret_cast<unsigned long long*>(&El[l + 1]), (unsigned long long)(int64_t)dE1);
            }
          }
        } else {
          // 3D: one configuration per round (two would not fit the register
          // budget of four wavefronts per SIMD)
          for (int l = 0; l < NS; ++l) {
            int dE = 0;
            if (valid) {
              uint32_t* Wl = W + (size_t)l * W2;
              const uint32_t Wc = Wl[c * NW + gp.w];
              uint32_t nw[2 * D], a[2 * D];
              neighbour_words<D>(g, Wl + (1 - c) * NW, gp.w, nb, p, nw);
#pragma unroll
              for (int k = 0; k < 2 * D; ++k) a[k] = (Wc ^ nw[k]) >> gp.shift;
              const Ctr4 r = philox10(Ctr4{c0, c1, (uint32_t)l, c3}, g.key0, g.key1);
              const int kt = tosl[l];
              const uint32_t F = gauss_group_flips<D>(a, m, hs, gp.nv, r, czl[kt], bl[kt], dE);
              if (F) atomicXor(&Wl[c * NW + gp.w], F << gp.shift);
            }
            dE = wave_total(dE);
            if (lane == 0 && dE)
              atomicAdd(reinterpret_cast<unsigned long long*>(&El[l]), (unsigned long long)(int64_t)dE);
          }
        }
      }
      __syncthreads();
    }
    // ---- Houdayer move per pair
    if (HOU) {
      if (D == 2 && rows64_houdayer(g))
        gauss_houdayer_rows64(fixed_shape<2, 64>(g), W, El, sotl, Js, s, v0 + (uint32_t)step,
                              lds + lay.hq);
      else
        gauss_houdayer_resident<D>(g, W, El, sotl, lds + lay.Qs, Js, s, v0 + (uint32_t)step);
    }
    // ---- replica exchange, one thread per set, k ascending with the updated map
    if (lane == 0 && wave < 2) {
      const int c = wave;
      const uint32_t u = u0 + (uint32_t)step;
      int32_t* so = sotl + c * NT;
      int32_t* to = tosl + c * NT;
      const int64_t* Es = El + c * NT;
      for (int k = 0; k + 1 < NT; ++k) {
        const int a = so[k], b = so[k + 1];
        const int64_t Dl = Es[b] - Es[a];
        bool acc = Dl <= 0;
        if (!acc) {
          const Ctr4 r = philox10(Ctr4{(uint32_t)k, u, (uint32_t)c, (kTagPT << 28) | (uint32_t)s},
                                  g.key0, g.key1);
          acc = gauss_accept_d(r.x, bl[k] - bl[k + 1], Dl);
        }
        if (acc) {
          so[k] = b;
          so[k + 1] = a;
          to[b] = k;
          to[a] = k + 1;
        }
      }
    }
    __syncthreads();
    // ---- measurement (Eqs. (3), (4)), one wavefront per temperature
    if (MEAS && measures_at(t + 1u, (uint32_t)every)) {
      for (int k = wave; k < NT; k += nwave) {
        const int a = sotl[k], b = NT + sotl[NT + k];
        const uint32_t* Wa = W + (size_t)a * W2;
        const uint32_t* Wb = W + (size_t)b * W2;
        int neg = 0;
        for (int i = lane; i < W2; i += 64) neg += __popc(Wa[i] ^ Wb[i]);
        neg = wave_total(neg);
        if (lane == 0) {
          const int64_t Q = (int64_t)g.N - 2 * (int64_t)neg;
          const int64_t Ea = El[a], Eb = El[b];
          int64_t* mk = ml + (size_t)k * 8;
          mk[0] += Ea + Eb;
          const uint64_t ua = (uint64_t)(Ea < 0 ? -Ea : Ea), ub = (uint64_t)(Eb < 0 ? -Eb : Eb);
          add128(&mk[1], &mk[7], ua * ua, __umul64hi(ua, ua));
          add128(&mk[1], &mk[7], ub * ub, __umul64hi(ub, ub));
          mk[2] += Q;
          mk[3] += Q < 0 ? -Q : Q;
          const uint64_t q2 = (uint64_t)(Q * Q);
          mk[4] += (int64_t)q2;
          add128(&mk[5], &mk[6], q2 * q2, __umul64hi(q2, q2));
        }
      }
      __syncthreads();
    }
  }

  // ---- store the sample's state
  for (int l = 0; l < NS; ++l) store_lattice(g, spins, lat0 + l, W + (size_t)l * W2, tid, T);
  for (int i = tid; i < NS; i += T) {
    E64[lat0 + i] = El[i];
    sot[(size_t)s * NS + i] = sotl[i];
    tos[(size_t)s * NS + i] = tosl[i];
  }
  if (MEAS)
    for (int i = tid; i < 8 * NT; i += T) mom[(size_t)s * NT * 8 + i] = ml[i];
}

template <int D, bool HOU, bool MEAS>
hipError_t launch_gfused(const Geo& g, void* spins, const int4* Jg, int64_t* E64, int32_t* sot,
                         int32_t* tos, const double* beta, const float* cz, int64_t* mom,
                         const DevCounters* ctr, int n, int every, hipStream_t st) {
  const int threads = gauss_fused_threads(g);
  const GaussLayout lay = gauss_layout(g, threads / 64);
  const size_t lds = sizeof(uint32_t) * (size_t)lay.words;
  auto k = k_gfused<D, HOU, MEAS>;
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)g.S), dim3(threads), lds, st, g, spins, Jg, E64, sot, tos, beta, cz,
                     mom, ctr, n, every, lay);
  return hipGetLastError();
}

}  // namespace

size_t gauss_fused_lds(const Geo& g) {
  return sizeof(uint32_t) * (size_t)gauss_layout(g, gauss_fused_threads(g) / 64).words;
}

hipError_t launch_gauss_fused(const Geo& g, void* spins, const int4* Jg, int64_t* E64, int32_t* sot,
                              int32_t* tos, const double* beta, const float* cz, int64_t* mom,
                              const DevCounters* ctr, int n, bool hou, bool meas, int every,
                              hipStream_t st) {
  if (gauss_fused_lds(g) > kGaussFusedMaxLds) return hipErrorInvalidValue;
#define PTSG_GF(DD, HH, MM) \
  return launch_gfused<DD, HH, MM>(g, spins, Jg, E64, sot, tos, beta, cz, mom, ctr, n, every, st)
  if (g.d == 3) {
    if (hou) {
      if (meas) PTSG_GF(3, true, true);
      PTSG_GF(3, true, false);
    }
    if (meas) PTSG_GF(3, false, true);
    PTSG_GF(3, false, false);
  }
  if (hou) {
    if (meas) PTSG_GF(2, true, true);
    PTSG_GF(2, true, false);
  }
  if (meas) PTSG_GF(2, false, true);
  PTSG_GF(2, false, false);
#undef PTSG_GF
}

}  // namespace ptsg
