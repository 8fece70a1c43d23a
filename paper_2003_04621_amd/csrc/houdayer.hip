// houdayer.hip -- Houdayer cluster move in overlap space (Sec. 2.4, Eq. (10)),
// one workgroup per (sample, temperature) pair.
//
// The pair's two replicas a, b are read into LDS as colour words; the
// overlap word Q = W_a ^ W_b has a bit set where q_i = s_i^a s_i^b = -1.  The
// seed is the m-th set bit in increasing site order (per-thread chunks of
// rows, a prefix sum over chunks, then a walk along x0 inside the row).  The
// cluster grows by bit-parallel flood fill: C_c |= Q_c & (union of the
// neighbour words of C_{1-c}), alternating colours until no word changes --
// label propagation of the seed's single label, one word (P*H sites) per
// operation.  The energy change of replica a is delta = 2 (#boundary bonds -
// 2 #unsatisfied boundary bonds), counted on colour-0 words where every bond
// has one end.
#include "device.h"
#include "houdayer_ops.h"
#include "kernels.h"
#include "multicluster.h"

namespace ptsg {

// Diagnostics of one pass at temperature k of sample s that exchanged
// `size` > 0 sites (one thread per pair: no atomics needed).
__device__ __forceinline__ void count_exchanged(const Geo& g, int64_t* stats, int s, int k,
                                                uint32_t size) {
  int64_t* st = stats + ((size_t)s * g.NT + k) * kNStat;
  st[2] += 1;
  st[3] += size;
  st[4 + (31 - __clz(size))] += 1;
}

template <int D>
__global__ void __launch_bounds__(256) k_houdayer(Geo g, void* spins, const uint32_t* __restrict__ jw,
                                                  int32_t* __restrict__ E,
                                                  const int32_t* __restrict__ sot, DevCounters* ctr,
                                                  int64_t* __restrict__ stats) {
  extern __shared__ uint32_t lds[];
  const int T = blockDim.x, t = threadIdx.x;
  const int NW = g.NW;
  uint32_t* A = lds;               // replica a, both colours
  uint32_t* Q = A + 2 * NW;        // overlap words (later replica b)
  uint32_t* Cl = Q + 2 * NW;       // cluster words
  uint32_t* pre = Cl + 2 * NW;     // [T] chunk counts -> prefix sums
  __shared__ uint32_t n_minus, size_acc;
  __shared__ int delta_acc;

  const uint32_t v = load_counter(&ctr->v);
  const int pair = blockIdx.x;  // s*NT + k
  const int s = pair / g.NT, k = pair - s * g.NT;
  const int a = sot[((size_t)s * 2 + 0) * g.NT + k];
  const int b = g.NT + sot[((size_t)s * 2 + 1) * g.NT + k];
  const size_t lat_a = (size_t)s * g.nslot + a, lat_b = (size_t)s * g.nslot + b;

  load_lattice(g, spins, lat_a, A, t, T);
  load_lattice(g, spins, lat_b, Q, t, T);
  if (t == 0) {
    delta_acc = 0;
    size_acc = 0;
  }
  __syncthreads();
  for (int i = t; i < 2 * NW; i += T) {
    Q[i] ^= A[i];
    Cl[i] = 0;
  }
  __syncthreads();

  // q = -1 counts per contiguous chunk of rows (site order is row-major)
  const int chunk = (g.NR + T - 1) / T;
  const int r_begin = t * chunk, r_end = min(g.NR, r_begin + chunk);
  uint32_t cnt = 0;
  for (int R = r_begin; R < r_end; ++R) cnt += row_minus_count(g, Q, R);
  pre[t] = cnt;
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (int i = 0; i < T; ++i) {
      const uint32_t c = pre[i];
      pre[i] = run;
      run += c;
    }
    n_minus = run;
  }
  __syncthreads();
  const uint32_t n = n_minus;
  if (n > 0) {
    const Ctr4 r = philox10(Ctr4{(uint32_t)k, v, 0u, (kTagHou << 28) | (uint32_t)s}, g.key0, g.key1);
    const uint64_t r64 = (uint64_t)r.x | ((uint64_t)r.y << 32);
    const uint32_t m = (uint32_t)__umul64hi(r64, (uint64_t)n);
    if (m >= pre[t] && m < pre[t] + cnt) seed_in_rows(g, Q, Cl, r_begin, r_end, m - pre[t]);
    __syncthreads();

    // flood fill
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

    // energy change of replica a on the colour-0 words
    const uint32_t* jw0 = jw + (size_t)s * 2 * 2 * D * NW;
    int dl = 0;
    for (int w = t; w < NW; w += T) dl += cluster_delta_word<D>(g, Cl, A, jw0, w);
    if (dl) atomicAdd(&delta_acc, dl);
    if (stats) {
      uint32_t sz = 0;
      for (int i = t; i < 2 * NW; i += T) sz += __popc(Cl[i]);
      if (sz) atomicAdd(&size_acc, sz);
    }
    __syncthreads();

    // exchange the replicas on the cluster: a' = a ^ C, b' = Q ^ a'
    for (int i = t; i < 2 * NW; i += T) {
      const uint32_t an = A[i] ^ Cl[i];
      A[i] = an;
      Q[i] ^= an;
    }
    __syncthreads();
    store_lattice(g, spins, lat_a, A, t, T, Cl);
    store_lattice(g, spins, lat_b, Q, t, T, Cl);
    if (t == 0) {
      E[lat_a] += delta_acc;
      E[lat_b] -= delta_acc;
      if (stats) count_exchanged(g, stats, s, k, size_acc);
    }
  }
}

// The multi-cluster variant (multicluster.h), one workgroup per pair: the
// workgroup finds the exchanged clusters together, then computes the energy
// change and applies the exchange as the single-cluster kernel does.
template <int D>
__global__ void __launch_bounds__(256) k_houdayer_multi(Geo g, void* spins,
                                                        const uint32_t* __restrict__ jw,
                                                        int32_t* __restrict__ E,
                                                        const int32_t* __restrict__ sot,
                                                        DevCounters* ctr, int64_t* __restrict__ stats) {
  extern __shared__ __align__(16) uint32_t lds_m[];
  const int T = blockDim.x, t = threadIdx.x;
  const int NW = g.NW;
  uint32_t* A = lds_m;            // replica a, both colours
  uint32_t* Q = A + 2 * NW;       // overlap words (later replica b)
  uint32_t* Cl = Q + 2 * NW;      // exchanged sites
  uint32_t* scr = Cl + 2 * NW;    // row masks, coins, labels (2 NW is even: 8-byte aligned)
  __shared__ int delta_acc;
  __shared__ uint32_t size_acc;

  const uint32_t v = load_counter(&ctr->v);
  const int pair = blockIdx.x;  // s*NT + k
  const int s = pair / g.NT, k = pair - s * g.NT;
  const int a = sot[((size_t)s * 2 + 0) * g.NT + k];
  const int b = g.NT + sot[((size_t)s * 2 + 1) * g.NT + k];
  const size_t lat_a = (size_t)s * g.nslot + a, lat_b = (size_t)s * g.nslot + b;

  load_lattice(g, spins, lat_a, A, t, T);
  load_lattice(g, spins, lat_b, Q, t, T);
  if (t == 0) {
    delta_acc = 0;
    size_acc = 0;
  }
  __syncthreads();
  for (int i = t; i < 2 * NW; i += T) Q[i] ^= A[i];
  __syncthreads();
  multi_cluster_words<D>(g, Q, Cl, scr, s, k, v, t, T, [] { __syncthreads(); });

  const uint32_t* jw0 = jw + (size_t)s * 2 * 2 * D * NW;
  int dl = 0;
  for (int w = t; w < NW; w += T) dl += cluster_delta_word<D>(g, Cl, A, jw0, w);
  if (dl) atomicAdd(&delta_acc, dl);
  if (stats) {
    uint32_t sz = 0;
    for (int i = t; i < 2 * NW; i += T) sz += __popc(Cl[i]);
    if (sz) atomicAdd(&size_acc, sz);
  }
  __syncthreads();
  for (int i = t; i < 2 * NW; i += T) {
    const uint32_t an = A[i] ^ Cl[i];
    A[i] = an;
    Q[i] ^= an;
  }
  __syncthreads();
  store_lattice(g, spins, lat_a, A, t, T, Cl);
  store_lattice(g, spins, lat_b, Q, t, T, Cl);
  if (t == 0 && delta_acc != 0) {
    E[lat_a] += delta_acc;
    E[lat_b] -= delta_acc;
  }
  if (t == 0 && stats && size_acc) count_exchanged(g, stats, s, k, size_acc);
}

hipError_t launch_houdayer_multi(const Geo& g, void* spins, const uint32_t* jw, int32_t* E,
                                 const int32_t* sot, DevCounters* ctr, int64_t* stats,
                                 hipStream_t st) {
  if (g.N > kMultiMaxSites) return hipErrorInvalidValue;
  const int threads = 256;
  const size_t lds = sizeof(uint32_t) * (2 * (size_t)g.NW + multi_scratch_words(g.N, g.NR, g.NW));
  const unsigned blocks = (unsigned)(g.S * g.NT);
  const void* k = g.d == 3 ? (const void*)k_houdayer_multi<3> : (const void*)k_houdayer_multi<2>;
  if (lds > 65536) {
    const hipError_t ea = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  if (g.d == 3)
    hipLaunchKernelGGL(k_houdayer_multi<3>, dim3(blocks), dim3(threads), lds, st, g, spins, jw, E, sot,
                       ctr, stats);
  else
    hipLaunchKernelGGL(k_houdayer_multi<2>, dim3(blocks), dim3(threads), lds, st, g, spins, jw, E, sot,
                       ctr, stats);
  return hipGetLastError();
}

hipError_t launch_houdayer(const Geo& g, void* spins, const uint32_t* jw, int32_t* E,
                           const int32_t* sot, DevCounters* ctr, int64_t* stats, hipStream_t st) {
  int threads = ((g.NW + 63) / 64) * 64;
  if (threads > 256) threads = 256;
  const size_t lds = sizeof(uint32_t) * (6 * (size_t)g.NW + threads);
  const unsigned blocks = (unsigned)(g.S * g.NT);
  if (g.d == 3) {
    if (lds > 65536) {
      const hipError_t ea = hipFuncSetAttribute((const void*)k_houdayer<3>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (ea != hipSuccess) return ea;
    }
    hipLaunchKernelGGL(k_houdayer<3>, dim3(blocks), dim3(threads), lds, st, g, spins, jw, E, sot, ctr,
                       stats);
  } else {
    if (lds > 65536) {
      const hipError_t ea = hipFuncSetAttribute((const void*)k_houdayer<2>,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (ea != hipSuccess) return ea;
    }
    hipLaunchKernelGGL(k_houdayer<2>, dim3(blocks), dim3(threads), lds, st, g, spins, jw, E, sot, ctr,
                       stats);
  }
  return hipGetLastError();
}

}  // namespace ptsg
