// steps.hip -- the smaller steps of the path: initial spins, coupling
// packing, energy recompute (Eq. (1)), replica exchange (Eq. (5)) and the
// measurement of Eqs. (3)-(4).
#include "device.h"
#include "kernels.h"
#include "rowops.h"

namespace ptsg {

// ---------------------------------------------------------------------------
// initial spins
// ---------------------------------------------------------------------------
__global__ void k_init_int8(Geo g, int8_t* spins) {
  const long groups = (long)g.N / 4;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)g.S * g.nslot * groups;
  if (idx >= total) return;
  const long lat = idx / groups;
  const uint32_t m = (uint32_t)(idx - lat * groups);
  const int s = (int)(lat / g.nslot), slot = (int)(lat - (long)s * g.nslot);
  const Ctr4 r = philox10(Ctr4{m, 0u, (uint32_t)slot, (kTagInit << 28) | (uint32_t)s}, g.key0, g.key1);
  const uint32_t v = (r.x >> 31 ? 0xFFu : 0x01u) | ((r.y >> 31 ? 0xFFu : 0x01u) << 8) |
                     ((r.z >> 31 ? 0xFFu : 0x01u) << 16) | ((r.w >> 31 ? 0xFFu : 0x01u) << 24);
  reinterpret_cast<uint32_t*>(spins)[idx] = v;
}

__global__ void k_init_packed(Geo g, uint32_t* spins) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)g.S * g.nslot * g.NW;
  if (idx >= total) return;
  const long lat = idx / g.NW;
  const int w = (int)(idx - lat * g.NW);
  const int s = (int)(lat / g.nslot), slot = (int)(lat - (long)s * g.nslot);
  const WordNb q = word_nb(g, w);
  uint32_t e = 0, o = 0;
  for (int f = 0; f < g.P; ++f) {
    const int R = word_row(g, q, f);
    uint32_t lastm = 0xFFFFFFFFu;
    Ctr4 r{0, 0, 0, 0};
    for (int x0 = 0; x0 < g.L; ++x0) {
      const uint32_t i = (uint32_t)(x0 + g.L * R);
      if ((i >> 2) != lastm) {
        lastm = i >> 2;
        r = philox10(Ctr4{lastm, 0u, (uint32_t)slot, (kTagInit << 28) | (uint32_t)s}, g.key0,
                     g.key1);
      }
      const uint32_t v = (i & 3) == 0 ? r.x : (i & 3) == 1 ? r.y : (i & 3) == 2 ? r.z : r.w;
      const uint32_t bit = (v >> 31) << (f * g.H + (x0 >> 1));
      if (x0 & 1)
        o |= bit;
      else
        e |= bit;
    }
  }
  uint32_t* dst = spins + lat * 2 * (size_t)g.NW;
  dst[w] = q.par ? o : e;
  dst[g.NW + w] = q.par ? e : o;
}

hipError_t launch_init_spins(const Geo& g, void* spins, hipStream_t st) {
  if (g.layout == kLayoutPacked) {
    const long total = (long)g.S * g.nslot * g.NW;
    hipLaunchKernelGGL(k_init_packed, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g,
                       static_cast<uint32_t*>(spins));
  } else {
    const long total = (long)g.S * g.nslot * (g.N / 4);
    hipLaunchKernelGGL(k_init_int8, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g,
                       static_cast<int8_t*>(spins));
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// spin layout conversion (int8 <-> packed colour words), one thread per
// colour-word index of a lattice
// ---------------------------------------------------------------------------
__global__ void k_convert_layout(Geo g, const void* __restrict__ src, void* __restrict__ dst,
                                 int to_packed) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)g.S * g.nslot * g.NW;
  if (idx >= total) return;
  const long lat = idx / g.NW;
  const int w = (int)(idx - lat * g.NW);
  if (to_packed) {
    uint32_t w0, w1;
    word_from_int8(g, static_cast<const int8_t*>(src) + lat * g.N, w, w0, w1);
    uint32_t* out = static_cast<uint32_t*>(dst) + lat * 2 * (size_t)g.NW;
    out[w] = w0;
    out[g.NW + w] = w1;
  } else {
    const uint32_t* in = static_cast<const uint32_t*>(src) + lat * 2 * (size_t)g.NW;
    word_to_int8(g, static_cast<int8_t*>(dst) + lat * g.N, w, in[w], in[g.NW + w]);
  }
}

hipError_t launch_convert_layout(const Geo& g, const void* src, void* dst, bool to_packed,
                                 hipStream_t st) {
  const long total = (long)g.S * g.nslot * g.NW;
  hipLaunchKernelGGL(k_convert_layout, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g,
                     src, dst, to_packed ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// couplings -> direction words
// ---------------------------------------------------------------------------
__global__ void k_pack_couplings(Geo g, const int8_t* __restrict__ J8, uint32_t* __restrict__ jw) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)g.S * 2 * g.NW;
  if (idx >= total) return;
  const int w = (int)(idx % g.NW);
  const long sc = idx / g.NW;
  const int c = (int)(sc & 1), s = (int)(sc >> 1);
  const WordNb q = word_nb(g, w);
  const int p = (c + q.par) & 1;
  const int8_t* Js = J8 + (size_t)s * g.d * g.N;
  uint32_t out[6] = {0, 0, 0, 0, 0, 0};
  for (int f = 0; f < g.P; ++f) {
    const int R = word_row(g, q, f);
    const int x1 = (g.d == 3) ? R % g.L : R;
    const int x2 = (g.d == 3) ? R / g.L : 0;
    const int R1m = (g.d == 3) ? ((x1 + g.L - 1) % g.L) + g.L * x2 : (x1 + g.L - 1) % g.L;
    const int R2m = (g.d == 3) ? x1 + g.L * ((x2 + g.L - 1) % g.L) : 0;
    for (int b = 0; b < g.H; ++b) {
      const int x0 = 2 * b + p;
      const int i = x0 + g.L * R;
      const int x0m = (x0 == 0) ? g.L - 1 : x0 - 1;
      const uint32_t bit = 1u << (f * g.H + b);
      if (Js[0 * g.N + i] < 0) out[0] |= bit;
      if (Js[0 * g.N + x0m + g.L * R] < 0) out[1] |= bit;
      if (Js[1 * g.N + i] < 0) out[2] |= bit;
      if (Js[1 * g.N + x0 + g.L * R1m] < 0) out[3] |= bit;
      if (g.d == 3) {
        if (Js[2 * g.N + i] < 0) out[4] |= bit;
        if (Js[2 * g.N + x0 + g.L * R2m] < 0) out[5] |= bit;
      }
    }
  }
  uint32_t* dst = jw + (((size_t)s * 2 + c) * 2 * g.d) * g.NW + w;
  for (int dir = 0; dir < 2 * g.d; ++dir) dst[(size_t)dir * g.NW] = out[dir];
}

hipError_t launch_pack_couplings(const Geo& g, const int8_t* J8, uint32_t* jw, hipStream_t st) {
  const long total = (long)g.S * 2 * g.NW;
  hipLaunchKernelGGL(k_pack_couplings, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g, J8,
                     jw);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// energy recompute: every bond has exactly one colour-0 end (L even), so
// #unsatisfied = sum over colour-0 words and the 2d directions of popc(U).
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_energy(Geo g, const void* spins, const uint32_t* __restrict__ jw,
                                                int32_t* E, int T, int LPB) {
  extern __shared__ uint32_t lds[];
  int* red = reinterpret_cast<int*>(lds);
  uint32_t* W = lds + LPB + (size_t)(threadIdx.x / T) * 2 * g.NW;
  const int li = threadIdx.x / T, t = threadIdx.x - li * T;
  const long lat = (long)blockIdx.x * LPB + li;
  const bool active = lat < (long)g.S * g.nslot;
  if (threadIdx.x < LPB) red[threadIdx.x] = 0;
  if (active) load_lattice(g, spins, (size_t)lat, W, t, T);
  __syncthreads();
  if (active) {
    const int s = (int)(lat / g.nslot);
    const uint32_t* jw0 = jw + (size_t)s * 2 * 2 * D * g.NW;  // colour 0
    int unsat = 0;
    for (int w = t; w < g.NW; w += T) unsat += unsatisfied_word<D>(g, W, jw0, w);
    atomicAdd(&red[li], unsat);
  }
  __syncthreads();
  if (active && t == 0) E[lat] = 2 * red[li] - g.d * g.N;
}

hipError_t launch_energy(const Geo& g, const void* spins, const uint32_t* jw, int32_t* E,
                         hipStream_t st) {
  int T, LPB, threads;
  size_t lds;
  sweep_shape(g, T, LPB, threads, lds);
  const long nlat = (long)g.S * g.nslot;
  const dim3 grid((unsigned)((nlat + LPB - 1) / LPB));
  if (g.d == 3) {
    if (lds > 65536) {
      const hipError_t ea = hipFuncSetAttribute((const void*)k_energy<3>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (ea != hipSuccess) return ea;
    }
    hipLaunchKernelGGL(k_energy<3>, grid, dim3(threads), lds, st, g, spins, jw, E, T, LPB);
  } else {
    if (lds > 65536) {
      const hipError_t ea = hipFuncSetAttribute((const void*)k_energy<2>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (ea != hipSuccess) return ea;
    }
    hipLaunchKernelGGL(k_energy<2>, grid, dim3(threads), lds, st, g, spins, jw, E, T, LPB);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// replica exchange, one lane per (sample, replica set); ascending k; then
// the set's replica-walk bookkeeping if the job keeps it (walk not null)
// ---------------------------------------------------------------------------
__global__ void k_exchange(Geo g, const int32_t* __restrict__ E, int32_t* __restrict__ sot,
                           int32_t* __restrict__ tos, const uint32_t* __restrict__ thrpt, int M,
                           int32_t* __restrict__ walk, uint64_t* __restrict__ trips,
                           DevCounters* ctr, int64_t* __restrict__ stats) {
  const uint32_t u = load_counter(&ctr->u);
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (long)g.S * 2) {
    const int s = (int)(idx >> 1), c = (int)(idx & 1);
    int32_t* so = sot + ((size_t)s * 2 + c) * g.NT;
    int32_t* to = tos + ((size_t)s * 2 + c) * g.NT;
    const int32_t* Es = E + (size_t)s * g.nslot + (size_t)c * g.NT;
    int a = so[0];
    for (int k = 0; k + 1 < g.NT; ++k) {
      const int b = so[k + 1];
      const int32_t D = Es[b] - Es[a];
      bool acc = D <= 0;
      if (!acc) {
        const int m = D >> 1;
        const uint32_t th = (m < M) ? thrpt[(size_t)k * M + m] : 0u;
        const Ctr4 r = philox10(Ctr4{(uint32_t)k, u, (uint32_t)c, (kTagPT << 28) | (uint32_t)s},
                                g.key0, g.key1);
        acc = r.x < th;
      }
      if (acc) {
        so[k] = b;
        so[k + 1] = a;
        to[b] = k;
        to[a] = k + 1;
        if (stats)  // both replica sets of the sample count here
          atomicAdd(reinterpret_cast<unsigned long long*>(stats + ((size_t)s * g.NT + k) * kNStat + 1),
                    1ull);
        // the configuration now at k+1 is a; keep carrying it upward
      } else {
        a = b;
      }
    }
    if (walk)
      walk_observe(walk + ((size_t)s * g.nslot + (size_t)c * g.NT) * 2, trips + (size_t)s * 32 * 3,
                   so[0], a, u + 1u);
  }
}

hipError_t launch_exchange(const Geo& g, const int32_t* E, int32_t* sot, int32_t* tos,
                           const uint32_t* thrpt, int M, int32_t* walk, uint64_t* trips,
                           DevCounters* ctr, int64_t* stats, hipStream_t st) {
  const long lanes = (long)g.S * 2;
  hipLaunchKernelGGL(k_exchange, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st, g, E, sot,
                     tos, thrpt, M, walk, trips, ctr, stats);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// measurement: one block per (sample, temperature)
// ---------------------------------------------------------------------------
// Plane counts cnt[mu][x] of the sites where the two replicas differ (the
// per-site form of the two-replica modes), by LDS atomics.
__device__ __forceinline__ void plane_counts_int8(const Geo& g, const int8_t* sa, const int8_t* sb,
                                                  int32_t* cnt) {
  const int L = g.L;
  for (int i = threadIdx.x; i < g.N; i += blockDim.x) {
    if (sa[i] == sb[i]) continue;
    const int r = i / L, x0 = i - r * L, x2 = r / L, x1 = r - x2 * L;
    atomicAdd(&cnt[x0], 1);
    atomicAdd(&cnt[L + x1], 1);
    if (g.d == 3) atomicAdd(&cnt[2 * L + x2], 1);
  }
}

__device__ __forceinline__ void plane_counts_packed(const Geo& g, const uint32_t* sa,
                                                    const uint32_t* sb, int32_t* cnt) {
  const int L = g.L;
  for (int w = threadIdx.x; w < g.NW; w += blockDim.x) {
    const WordNb q = word_nb(g, w);
    for (int c = 0; c < 2; ++c) {
      uint32_t X = (sa[c * g.NW + w] ^ sb[c * g.NW + w]) & g.maskW;
      while (X) {
        const int j = __ffs(X) - 1;
        X &= X - 1;
        const int f = j / g.H, bb = j - f * g.H;
        const int x0 = 2 * bb + ((c + q.par) & 1), xs = f * g.B + q.xs;
        atomicAdd(&cnt[x0], 1);
        if (g.d == 3) {
          atomicAdd(&cnt[L + q.x1], 1);
          atomicAdd(&cnt[2 * L + xs], 1);
        } else {
          atomicAdd(&cnt[L + xs], 1);
        }
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_measure(Geo g, const void* spins, const int32_t* __restrict__ E,
                                                 const int32_t* __restrict__ sot, int64_t* mom,
                                                 int64_t* modes, DevCounters* ctr, int every) {
  if (!measures_at(load_counter(&ctr->t) + 1u, (uint32_t)every)) return;  // uniform
  __shared__ int red;
  __shared__ int32_t cnt[3 * 64];
  const int pair = blockIdx.x;  // s*NT + k
  const int s = pair / g.NT, k = pair - s * g.NT;
  const int a = sot[((size_t)s * 2 + 0) * g.NT + k];
  const int b = g.NT + sot[((size_t)s * 2 + 1) * g.NT + k];
  if (threadIdx.x == 0) red = 0;
  if (modes)
    for (int i = threadIdx.x; i < 3 * g.L; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  if (modes) {
    if (g.layout == kLayoutPacked) {
      const uint32_t* base = static_cast<const uint32_t*>(spins) + (size_t)s * g.nslot * 2 * g.NW;
      plane_counts_packed(g, base + (size_t)a * 2 * g.NW, base + (size_t)b * 2 * g.NW, cnt);
    } else {
      const int8_t* base = static_cast<const int8_t*>(spins) + (size_t)s * g.nslot * g.N;
      plane_counts_int8(g, base + (size_t)a * g.N, base + (size_t)b * g.N, cnt);
    }
    __syncthreads();
    const int MH = g.L / 2 + 1;
    if ((int)threadIdx.x < MH) modes[(size_t)pair * MH + threadIdx.x] += mode_autocorr(g, cnt, threadIdx.x);
  }
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
    for (int w = threadIdx.x; w < g.N / 4; w += blockDim.x)
      neg += __popc((sa[w] ^ sb[w]) & 0x80808080u);
  }
  atomicAdd(&red, neg);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t Q = (int64_t)g.N - 2 * (int64_t)red;
    const int64_t Ea = E[(size_t)s * g.nslot + a], Eb = E[(size_t)s * g.nslot + b];
    int64_t* m = mom + (size_t)pair * 8;
    m[0] += Ea + Eb;
    m[1] += Ea * Ea + Eb * Eb;
    m[2] += Q;
    m[3] += Q < 0 ? -Q : Q;
    const uint64_t q2 = (uint64_t)(Q * Q);
    m[4] += (int64_t)q2;
    const uint64_t q4lo = q2 * q2, q4hi = __umul64hi(q2, q2);
    const uint64_t lo = (uint64_t)m[5] + q4lo;
    const uint64_t carry = lo < q4lo ? 1u : 0u;
    m[5] = (int64_t)lo;
    m[6] = (int64_t)((uint64_t)m[6] + q4hi + carry);
  }
}

hipError_t launch_measure(const Geo& g, const void* spins, const int32_t* E, const int32_t* sot,
                          int64_t* mom, int64_t* modes, DevCounters* ctr, int every,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_measure, dim3((unsigned)(g.S * g.NT)), dim3(256), 0, st, g, spins, E, sot, mom,
                     modes, ctr, every);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// counters
// ---------------------------------------------------------------------------
__global__ void k_advance(DevCounters* ctr, CounterStep step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const uint32_t t0 = ctr->t;
    ctr->t += step.dt;
    ctr->u += step.du;
    ctr->v += step.dv;
    ctr->n_meas += step.every > 1u
                       ? step.dm * ((t0 + step.dt) / step.every - t0 / step.every)
                       : step.dm;
  }
}

hipError_t launch_advance(DevCounters* ctr, CounterStep step, hipStream_t st) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, ctr, step);
  return hipGetLastError();
}

}  // namespace ptsg
