// gauss.hip -- kernels of the Edwards-Anderson model with Gaussian couplings
// (Sec. 2.1; the 2D Gaussian workload of Sec. 4.2): coupling preparation,
// energies (Eq. (1)), the checkerboard Metropolis sweep (Sec. 2.2), the
// replica exchange (Eq. (5)), both Houdayer moves (Sec. 2.4, Eq. (10)) and the
// measurement (Eqs. (3)-(4)).  Spins use the same layouts and LDS words as the
// +-J kernels; the couplings and energies are integers of 2^-16 units
// (gauss.h), the energies 64-bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "gauss.h"
#include "gauss_kernels.h"
#include "houdayer_ops.h"
#include "multicluster.h"

namespace ptsg {

namespace {

// Block order that keeps consecutive logical blocks on one XCD (blocks are
// dealt to the eight XCDs in turn): the blocks of a sample then share that
// XCD's L2 copy of the sample's couplings.
__device__ __forceinline__ int xcd_block(int bx, int nb) {
  const int per = nb / 8, rem = nb % 8, x = bx % 8, i = bx / 8;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

}  // namespace

// ---------------------------------------------------------------------------
// Coupling units [S][d][N] -> group data Jg [S][2][2d+1][NGc] (gauss.h).
// ---------------------------------------------------------------------------
__global__ void k_gprepare(Geo g, const int32_t* __restrict__ Jn, int4* __restrict__ Jg) {
  const int NGc = gauss_groups(g);
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)g.S * 2 * NGc;
  if (idx >= total) return;
  const int gi = (int)(idx % NGc);
  const int sc = (int)(idx / NGc), s = sc >> 1, c = sc & 1;
  const GroupPos gp = group_pos(g, gi);
  const WordNb nb = word_nb(g, gp.w);
  const int R = word_row(g, nb, gp.f);
  const int L = g.L, x1 = g.d == 3 ? R % L : R, x2 = g.d == 3 ? R / L : 0;
  const int p = (c + x1 + x2) & 1;
  const int32_t* J = Jn + (size_t)s * g.d * g.N;
  int val[7][4];
  for (int j = 0; j < 4; ++j) {
    for (int k = 0; k < 7; ++k) val[k][j] = 0;
    const int b = 4 * gp.q + j;
    if (b >= g.H) continue;
    const int x0 = 2 * b + p;
    const int i = x0 + L * R;
    const int xm0 = (x0 + L - 1) % L, xm1 = (x1 + L - 1) % L, xm2 = (x2 + L - 1) % L;
    int n[6];
    n[0] = J[i];                                    // +x0
    n[1] = J[xm0 + L * R];                          // -x0
    n[2] = J[g.N + i];                              // +x1
    n[3] = J[g.N + x0 + L * (xm1 + L * x2)];        // -x1
    if (g.d == 3) {
      n[4] = J[2 * g.N + i];                        // +x2
      n[5] = J[2 * g.N + x0 + L * (x1 + L * xm2)];  // -x2
    }
    int hs = 0;
    for (int k = 0; k < 2 * g.d; ++k) {
      val[k][j] = -2 * n[k];
      hs += n[k];
    }
    val[2 * g.d][j] = hs;
  }
  int4* out = Jg + (size_t)sc * (2 * g.d + 1) * NGc + gi;
  for (int k = 0; k <= 2 * g.d; ++k)
    out[(size_t)k * NGc] = make_int4(val[k][0], val[k][1], val[k][2], val[k][3]);
}

// ---------------------------------------------------------------------------
// Energy (Eq. (1)) of every lattice: each bond has exactly one colour-0 end,
// so E = -(sum of x = s_i h_i over the colour-0 sites).  One block per lattice.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_genergy(Geo g, const void* spins, const int4* __restrict__ Jg,
                                                 int64_t* __restrict__ E64) {
  extern __shared__ __align__(16) uint32_t lds_e[];
  __shared__ unsigned long long acc;
  const int T = blockDim.x, t = threadIdx.x;
  const size_t lat = blockIdx.x;
  const int s = (int)(lat / g.nslot);
  const int NGc = gauss_groups(g);
  uint32_t* W = lds_e;
  if (t == 0) acc = 0ull;
  load_lattice(g, spins, lat, W, t, T);
  __syncthreads();
  const int4* J0 = Jg + (size_t)s * 2 * (2 * D + 1) * NGc;
  int64_t sum = 0;
  for (int gi = t; gi < NGc; gi += T) {
    const GroupPos gp = group_pos(g, gi);
    const WordNb nb = word_nb(g, gp.w);
    uint32_t n[2 * D], a[2 * D];
    neighbour_words<D>(g, W + g.NW, gp.w, nb, nb.par, n);
    const uint32_t Wc = W[gp.w];
    int4 m[2 * D];
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
      a[k] = (Wc ^ n[k]) >> gp.shift;
      m[k] = J0[(size_t)k * NGc + gi];
    }
    const int4 hs = J0[(size_t)2 * D * NGc + gi];
    int x[4];
    group_fields<D>(a, m, hs, x);
    for (int j = 0; j < gp.nv; ++j) sum += x[j];
  }
  if (sum) atomicAdd(&acc, (unsigned long long)(-sum));
  __syncthreads();
  if (t == 0) E64[lat] = (int64_t)acc;
}

// ---------------------------------------------------------------------------
// Metropolis sweeps (Sec. 2.2), checkerboard: block = (sample, set, chunk of
// CH temperatures' slots), the chunk's lattices in LDS for all n sweeps.  A
// thread takes a group of four same-colour sites (one Philox call, its
// coupling data in registers) and updates it in every lattice of the chunk;
// colour 0 of all the chunk's lattices, then colour 1 (lattices are
// independent, so this is each lattice's own colour-0-then-1 order).  Flips
// go into the word by an LDS atomic xor (the group's bits only), energy
// changes into 64-bit LDS sums.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(512) k_gsweep(Geo g, void* spins, const int4* __restrict__ Jg,
                                                int64_t* __restrict__ E64,
                                                const int32_t* __restrict__ tos,
                                                const double* __restrict__ beta,
                                                const float* __restrict__ cz,
                                                const DevCounters* __restrict__ ctr, int nsweeps,
                                                int CH, int nchunk) {
  extern __shared__ __align__(16) uint32_t lds_s[];
  const int T = blockDim.x, t = threadIdx.x;
  const int NW = g.NW, NGc = gauss_groups(g);
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int s = lb / (2 * nchunk), rest = lb - s * 2 * nchunk;
  const int set = rest / nchunk, j0 = (rest - set * nchunk) * CH;
  const int nl = min(CH, g.NT - j0);
  unsigned long long* El = reinterpret_cast<unsigned long long*>(lds_s);  // [CH]
  double* bl = reinterpret_cast<double*>(El + CH);                       // [CH]
  float* czl = reinterpret_cast<float*>(bl + CH);                        // [CH]
  uint32_t* W = reinterpret_cast<uint32_t*>(czl + CH);                   // [CH][2NW]
  const size_t lat0 = (size_t)s * g.nslot + (size_t)set * g.NT + j0;
  for (int l = t; l < nl; l += T) {
    const int k = tos[((size_t)s * 2 + set) * g.NT + j0 + l];
    El[l] = 0ull;
    bl[l] = beta[k];
    czl[l] = cz[k];
  }
  for (int l = 0; l < nl; ++l) load_lattice(g, spins, lat0 + l, W + (size_t)l * 2 * NW, t, T);
  __syncthreads();
  const uint32_t t0 = load_counter(&ctr->t);
  const uint32_t c3 = (kTagMetro << 28) | (uint32_t)s;
  const int4* Js = Jg + (size_t)s * 2 * (2 * D + 1) * NGc;
  for (int rep = 0; rep < nsweeps; ++rep) {
    for (int c = 0; c < 2; ++c) {
      const int4* Jc = Js + (size_t)c * (2 * D + 1) * NGc;
      const uint32_t c1 = 2u * (t0 + (uint32_t)rep) + (uint32_t)c;
      // every lane runs every round of the group loop (lanes past the last
      // group idle), so that the wavefront can add its lanes' energy changes
      // before one 64-bit LDS atomic (|sum| < 64 x 4 x 2 x 6 x 2^19 < 2^31)
      for (int gi0 = 0; gi0 < NGc; gi0 += T) {
        const int gi = gi0 + t;
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
        for (int l = 0; l < nl; ++l) {
          int dE = 0;
          if (valid) {
            uint32_t* Wl = W + (size_t)l * 2 * NW;
            const uint32_t Wc = Wl[c * NW + gp.w];
            uint32_t n[2 * D], a[2 * D];
            neighbour_words<D>(g, Wl + (1 - c) * NW, gp.w, nb, p, n);
#pragma unroll
            for (int k = 0; k < 2 * D; ++k) a[k] = (Wc ^ n[k]) >> gp.shift;
            const uint32_t slot = (uint32_t)(set * g.NT + j0 + l);
            const Ctr4 r = philox10(Ctr4{c0, c1, slot, c3}, g.key0, g.key1);
            const uint32_t F = gauss_group_flips<D>(a, m, hs, gp.nv, r, czl[l], bl[l], dE);
            if (F) atomicXor(&Wl[c * NW + gp.w], F << gp.shift);
          }
          // every lane of the wavefront is here (see above): a DPP sum
          dE = wave_total(dE);
          if ((t & 63) == 0 && dE) atomicAdd(&El[l], (unsigned long long)(int64_t)dE);
        }
      }
      __syncthreads();
    }
  }
  for (int l = 0; l < nl; ++l) store_lattice(g, spins, lat0 + l, W + (size_t)l * 2 * NW, t, T);
  for (int l = t; l < nl; l += T) E64[lat0 + l] += (int64_t)El[l];
}

// ---------------------------------------------------------------------------
// Replica exchange (Eq. (5)), one thread per (sample, set): k = 0 .. NT-2
// ascending with the updated map; D = E_b - E_a accepts iff D <= 0 or the
// pair's Philox word r < 2^32 exp(-(beta_k - beta_{k+1}) D 2^-16).
// ---------------------------------------------------------------------------
__global__ void k_gexchange(Geo g, const int64_t* __restrict__ E64, int32_t* __restrict__ sot,
                            int32_t* __restrict__ tos, const double* __restrict__ beta,
                            const DevCounters* __restrict__ ctr) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * g.S) return;
  const int s = idx >> 1, c = idx & 1;
  const uint32_t u = load_counter(&ctr->u);
  int32_t* so = sot + ((size_t)s * 2 + c) * g.NT;
  int32_t* to = tos + ((size_t)s * 2 + c) * g.NT;
  const int64_t* Es = E64 + (size_t)s * g.nslot + (size_t)c * g.NT;
  for (int k = 0; k + 1 < g.NT; ++k) {
    const int a = so[k], b = so[k + 1];
    const int64_t D = Es[b] - Es[a];
    bool acc = D <= 0;
    if (!acc) {
      const Ctr4 r = philox10(Ctr4{(uint32_t)k, u, (uint32_t)c, (kTagPT << 28) | (uint32_t)s}, g.key0,
                              g.key1);
      acc = gauss_accept_d(r.x, beta[k] - beta[k + 1], D);
    }
    if (acc) {
      so[k] = b;
      so[k + 1] = a;
      to[b] = k;
      to[a] = k + 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Houdayer moves (Sec. 2.4, Eq. (10)), one workgroup per (sample, temperature)
// pair: the cluster words are found exactly as for +-J couplings (the
// clusters ignore the couplings); the energy change of replica a is
// delta = sum over bonds leaving the exchanged set of 2 n s_i^a s_j^a, taken
// from the colour-0 end of every bond: with m = -2n, m (2 a - 1) where a = 1
// if the bond's two spins of replica a are antiparallel.
// ---------------------------------------------------------------------------
template <int D, bool MULTI>
__global__ void __launch_bounds__(256) k_ghoudayer(Geo g, void* spins, const int4* __restrict__ Jg,
                                                   int64_t* __restrict__ E64,
                                                   const int32_t* __restrict__ sot,
                                                   const DevCounters* __restrict__ ctr) {
  extern __shared__ __align__(16) uint32_t lds_h[];
  const int T = blockDim.x, t = threadIdx.x;
  const int NW = g.NW;
  uint32_t* A = lds_h;         // replica a, both colours
  uint32_t* Q = A + 2 * NW;    // overlap words (later replica b)
  uint32_t* Cl = Q + 2 * NW;   // exchanged sites
  uint32_t* scr = Cl + 2 * NW; // single: chunk prefix sums [T]; multi: the team's scratch
  __shared__ uint32_t n_minus;
  __shared__ unsigned long long delta_acc;

  const uint32_t v = load_counter(&ctr->v);
  const int pair = blockIdx.x;  // s*NT + k
  const int s = pair / g.NT, k = pair - s * g.NT;
  const int a = sot[((size_t)s * 2 + 0) * g.NT + k];
  const int b = g.NT + sot[((size_t)s * 2 + 1) * g.NT + k];
  const size_t lat_a = (size_t)s * g.nslot + a, lat_b = (size_t)s * g.nslot + b;

  load_lattice(g, spins, lat_a, A, t, T);
  load_lattice(g, spins, lat_b, Q, t, T);
  if (t == 0) delta_acc = 0ull;
  __syncthreads();
  for (int i = t; i < 2 * NW; i += T) {
    Q[i] ^= A[i];
    Cl[i] = 0;
  }
  __syncthreads();
  if constexpr (MULTI) {
    multi_cluster_words<D>(g, Q, Cl, scr, s, k, v, t, T, [] { __syncthreads(); });
  } else {
    const int chunk = (g.NR + T - 1) / T;
    const int r_begin = t * chunk, r_end = min(g.NR, r_begin + chunk);
    uint32_t cnt = 0;
    for (int R = r_begin; R < r_end; ++R) cnt += row_minus_count(g, Q, R);
    scr[t] = cnt;
    __syncthreads();
    if (t == 0) {
      uint32_t run = 0;
      for (int i = 0; i < T; ++i) {
        const uint32_t c = scr[i];
        scr[i] = run;
        run += c;
      }
      n_minus = run;
    }
    __syncthreads();
    const uint32_t n = n_minus;
    if (n == 0) return;  // uniform: nothing to exchange
    const Ctr4 r = philox10(Ctr4{(uint32_t)k, v, 0u, (kTagHou << 28) | (uint32_t)s}, g.key0, g.key1);
    const uint64_t r64 = (uint64_t)r.x | ((uint64_t)r.y << 32);
    const uint32_t m = (uint32_t)__umul64hi(r64, (uint64_t)n);
    if (m >= scr[t] && m < scr[t] + cnt) seed_in_rows(g, Q, Cl, r_begin, r_end, m - scr[t]);
    __syncthreads();
    int any;
    do {
      int changed = 0;
      for (int c = 0; c < 2; ++c) {
        for (int w = t; w < NW; w += T)
          if (grow_word<D>(g, Cl, Q, c, w)) changed = 1;
        if (c == 0) __syncthreads();
      }
      any = __syncthreads_or(changed);
    } while (any);
  }
  const int4* J0 = Jg + (size_t)s * 2 * (2 * D + 1) * gauss_groups(g);
  const int64_t dl = gauss_cluster_delta<D>(g, Cl, A, J0, t, T);
  if (dl) atomicAdd(&delta_acc, (unsigned long long)dl);
  __syncthreads();
  for (int i = t; i < 2 * NW; i += T) {
    const uint32_t an = A[i] ^ Cl[i];
    A[i] = an;
    Q[i] ^= an;
  }
  __syncthreads();
  store_lattice(g, spins, lat_a, A, t, T, Cl);
  store_lattice(g, spins, lat_b, Q, t, T, Cl);
  if (t == 0 && delta_acc != 0ull) {
    E64[lat_a] += (int64_t)delta_acc;
    E64[lat_b] -= (int64_t)delta_acc;
  }
}

// ---------------------------------------------------------------------------
// Measurement (Eqs. (3), (4)): per (sample, temperature) the sums of E, E^2
// over both replicas and of Q, |Q|, Q^2, Q^4.  mom [S][NT][8]: 0 sum E,
// 1 sum E^2 (low 64 bits), 2 sum Q, 3 sum |Q|, 4 sum Q^2, 5-6 sum Q^4 (low,
// high), 7 sum E^2 (high 64 bits).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_gmeasure(Geo g, const void* spins, const int64_t* __restrict__ E64,
                                                  const int32_t* __restrict__ sot, int64_t* mom,
                                                  const DevCounters* __restrict__ ctr, int every) {
  if (!measures_at(load_counter(&ctr->t) + 1u, (uint32_t)every)) return;  // uniform
  __shared__ int red;
  const int pair = blockIdx.x;  // s*NT + k
  const int s = pair / g.NT, k = pair - s * g.NT;
  const int a = sot[((size_t)s * 2 + 0) * g.NT + k];
  const int b = g.NT + sot[((size_t)s * 2 + 1) * g.NT + k];
  if (threadIdx.x == 0) red = 0;
  __syncthreads();
  int neg = 0;
  if (g.layout == kLayoutPacked) {
    const uint32_t* sa = static_cast<const uint32_t*>(spins) + ((size_t)s * g.nslot + a) * 2 * g.NW;
    const uint32_t* sb = static_cast<const uint32_t*>(spins) + ((size_t)s * g.nslot + b) * 2 * g.NW;
    for (int w = threadIdx.x; w < 2 * g.NW; w += blockDim.x) neg += __popc(sa[w] ^ sb[w]);
  } else {
    const uint32_t* sa = reinterpret_cast<const uint32_t*>(static_cast<const int8_t*>(spins) +
                                                           ((size_t)s * g.nslot + a) * g.N);
    const uint32_t* sb = reinterpret_cast<const uint32_t*>(static_cast<const int8_t*>(spins) +
                                                           ((size_t)s * g.nslot + b) * g.N);
    for (int w = threadIdx.x; w < g.N / 4; w += blockDim.x) neg += __popc((sa[w] ^ sb[w]) & 0x80808080u);
  }
  atomicAdd(&red, neg);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t Q = (int64_t)g.N - 2 * (int64_t)red;
    const int64_t Ea = E64[(size_t)s * g.nslot + a], Eb = E64[(size_t)s * g.nslot + b];
    int64_t* m = mom + (size_t)pair * 8;
    m[0] += Ea + Eb;
    const uint64_t ua = (uint64_t)(Ea < 0 ? -Ea : Ea), ub = (uint64_t)(Eb < 0 ? -Eb : Eb);
    add128(&m[1], &m[7], ua * ua, __umul64hi(ua, ua));
    add128(&m[1], &m[7], ub * ub, __umul64hi(ub, ub));
    m[2] += Q;
    m[3] += Q < 0 ? -Q : Q;
    const uint64_t q2 = (uint64_t)(Q * Q);
    m[4] += (int64_t)q2;
    add128(&m[5], &m[6], q2 * q2, __umul64hi(q2, q2));
  }
}

// ---------------------------------------------------------------------------
// Acceptance decisions for the tests: mode 0 the Metropolis tiers (u < 2^24),
// 1 the exchange tiers (double, then double-double), 2 double-double alone.
// ---------------------------------------------------------------------------
__global__ void k_gaccept(const uint32_t* __restrict__ r, const double* __restrict__ b,
                          const int64_t* __restrict__ u, int32_t* __restrict__ out, int n, int mode) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool acc;
  if (mode == 0)
    acc = gauss_accept_metro(r[i], gauss_cz(b[i]), b[i], (uint32_t)u[i]);
  else if (mode == 1)
    acc = gauss_accept_d(r[i], b[i], u[i]);
  else
    acc = gauss_accept_dd(r[i], b[i], u[i]);
  out[i] = acc ? 1 : 0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}
}  // namespace

hipError_t launch_gauss_prepare(const Geo& g, const int32_t* Jn, int4* Jg, hipStream_t st) {
  const long total = (long)g.S * 2 * gauss_groups(g);
  hipLaunchKernelGGL(k_gprepare, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g, Jn, Jg);
  return hipGetLastError();
}

hipError_t launch_gauss_energy(const Geo& g, const void* spins, const int4* Jg, int64_t* E64,
                               hipStream_t st) {
  const size_t lds = sizeof(uint32_t) * 2 * (size_t)g.NW;
  const unsigned blocks = (unsigned)((size_t)g.S * g.nslot);
  if (g.d == 3) {
    if (hipError_t e = allow_lds(k_genergy<3>, lds)) return e;
    hipLaunchKernelGGL(k_genergy<3>, dim3(blocks), dim3(256), lds, st, g, spins, Jg, E64);
  } else {
    if (hipError_t e = allow_lds(k_genergy<2>, lds)) return e;
    hipLaunchKernelGGL(k_genergy<2>, dim3(blocks), dim3(256), lds, st, g, spins, Jg, E64);
  }
  return hipGetLastError();
}

void gauss_sweep_shape(const Geo& g, int& threads, int& CH, int& nchunk, size_t& lds) {
  const int NGc = gauss_groups(g);
  threads = ((NGc + 63) / 64) * 64;
  if (threads > 512) threads = 512;
  const size_t per = 8 * (size_t)g.NW;  // one lattice's words
  const size_t budget = 40 * 1024;      // four 512-thread blocks per CU
  size_t ch = budget / (per + 20);
  if (ch < 1) ch = 1;
  if (ch > (size_t)g.NT) ch = (size_t)g.NT;
  CH = (int)ch;
  nchunk = (g.NT + CH - 1) / CH;
  lds = (size_t)CH * (20 + per);
}

hipError_t launch_gauss_sweep(const Geo& g, void* spins, const int4* Jg, int64_t* E64,
                              const int32_t* tos, const double* beta, const float* cz,
                              const DevCounters* ctr, int n, hipStream_t st) {
  int threads, CH, nchunk;
  size_t lds;
  gauss_sweep_shape(g, threads, CH, nchunk, lds);
  const unsigned blocks = (unsigned)((size_t)g.S * 2 * nchunk);
  if (g.d == 3) {
    if (hipError_t e = allow_lds(k_gsweep<3>, lds)) return e;
    hipLaunchKernelGGL(k_gsweep<3>, dim3(blocks), dim3(threads), lds, st, g, spins, Jg, E64, tos, beta,
                       cz, ctr, n, CH, nchunk);
  } else {
    if (hipError_t e = allow_lds(k_gsweep<2>, lds)) return e;
    hipLaunchKernelGGL(k_gsweep<2>, dim3(blocks), dim3(threads), lds, st, g, spins, Jg, E64, tos, beta,
                       cz, ctr, n, CH, nchunk);
  }
  return hipGetLastError();
}

hipError_t launch_gauss_exchange(const Geo& g, const int64_t* E64, int32_t* sot, int32_t* tos,
                                 const double* beta, const DevCounters* ctr, hipStream_t st) {
  const int n = 2 * g.S;
  hipLaunchKernelGGL(k_gexchange, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, g, E64, sot, tos,
                     beta, ctr);
  return hipGetLastError();
}

hipError_t launch_gauss_houdayer(const Geo& g, void* spins, const int4* Jg, int64_t* E64,
                                 const int32_t* sot, const DevCounters* ctr, bool multi,
                                 hipStream_t st) {
  // single cluster: one thread per colour word of the flood fill (at most
  // 256), so that a lattice with few words grows its cluster in one
  // wavefront; the multi-cluster teams take 256 threads
  const int threads = multi ? 256 : std::min(256, (g.NW + 63) / 64 * 64);
  if (multi && g.N > kMultiMaxSites) return hipErrorInvalidValue;
  // A, Q and the cluster words (6 NW), then the chunk sums [threads], or for
  // the multi-cluster move A and the team scratch (which begins with Q and C)
  const size_t words = multi ? 2 * (size_t)g.NW + (size_t)multi_scratch_words(g.N, g.NR, g.NW)
                             : 6 * (size_t)g.NW + (size_t)threads;
  const size_t lds = sizeof(uint32_t) * words;
  const unsigned blocks = (unsigned)(g.S * g.NT);
#define PTSG_GH(DD, MM)                                                                          \
  do {                                                                                           \
    if (hipError_t e = allow_lds(k_ghoudayer<DD, MM>, lds)) return e;                             \
    hipLaunchKernelGGL((k_ghoudayer<DD, MM>), dim3(blocks), dim3(threads), lds, st, g, spins, Jg, \
                       E64, sot, ctr);                                                           \
  } while (0)
  if (g.d == 3) {
    if (multi)
      PTSG_GH(3, true);
    else
      PTSG_GH(3, false);
  } else {
    if (multi)
      PTSG_GH(2, true);
    else
      PTSG_GH(2, false);
  }
#undef PTSG_GH
  return hipGetLastError();
}

hipError_t launch_gauss_measure(const Geo& g, const void* spins, const int64_t* E64, const int32_t* sot,
                                int64_t* mom, const DevCounters* ctr, int every, hipStream_t st) {
  hipLaunchKernelGGL(k_gmeasure, dim3((unsigned)(g.S * g.NT)), dim3(256), 0, st, g, spins, E64, sot, mom,
                     ctr, every);
  return hipGetLastError();
}

hipError_t launch_gauss_accept(const uint32_t* r, const double* b, const int64_t* u, int32_t* out, int n,
                               int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_gaccept, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, r, b, u, out, n,
                     mode);
  return hipGetLastError();
}

}  // namespace ptsg
