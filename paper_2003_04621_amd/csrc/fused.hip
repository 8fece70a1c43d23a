// fused.hip -- whole Monte Carlo steps (Sec. 2.4: Metropolis sweep, Houdayer
// move per same-temperature pair, replica-exchange pass, measurement) for one
// disorder sample per workgroup, every configuration of the sample resident
// in LDS as colour-split row words for all steps of the launch.  HBM is
// touched only to load the sample at the start and store it at the end.
//
// Results are bit-identical to the per-step kernels: the same row update
// (rowops.h), the same Philox counters, exchange decisions taken in ascending
// k with the updated map, Houdayer seeds chosen in increasing site order.
#include "device.h"
#include "kernels.h"
#include "houdayer_ops.h"
#include "rowops.h"

namespace ptsg {

struct FusedArgs {
  Geo g;
  void* spins;
  const uint32_t* jw;
  int32_t* E;
  int32_t* sot;
  int32_t* tos;
  const uint32_t* thr;
  const uint32_t* thrpt;
  int M;
  int64_t* mom;
  const DevCounters* ctr;
  int nmcs, hou, meas;
  uint32_t magicNW;  // item / NW
  FusedLayout lay;
};

// ---------------------------------------------------------------------------
// Replica exchange for both sets of the resident sample.  The pass is
// sequential in k, but every decision depends only on which configuration is
// carried up from below: with the pre-pass map m0, the configuration at
// position k before step k is m0[j] for some j <= k, and b = m0[k+1].  All
// candidate decisions acc[c][k][j] are evaluated in parallel, then one lane
// per set walks the chain.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void exchange_resident(const FusedArgs& A, uint32_t* lds, int s,
                                                  uint32_t u) {
  const Geo& g = A.g;
  const int NT = g.NT, tid = threadIdx.x, T = blockDim.x;
  const int32_t* El = reinterpret_cast<const int32_t*>(lds + A.lay.E);
  int32_t* sotl = reinterpret_cast<int32_t*>(lds + A.lay.sot);
  int32_t* tosl = reinterpret_cast<int32_t*>(lds + A.lay.tos);
  int32_t* sot0 = reinterpret_cast<int32_t*>(lds + A.lay.sot0);
  uint32_t* rpt = lds + A.lay.rpt;
  uint8_t* acc = reinterpret_cast<uint8_t*>(lds + A.lay.acc);
  for (int i = tid; i < 2 * NT; i += T) sot0[i] = sotl[i];
  for (int i = tid; i < 2 * (NT - 1); i += T) {
    const int c = i / (NT - 1), k = i - c * (NT - 1);
    rpt[c * NT + k] =
        philox10(Ctr4{(uint32_t)k, u, (uint32_t)c, (kTagPT << 28) | (uint32_t)s}, g.key0, g.key1).x;
  }
  __syncthreads();
  const int per_set = (NT - 1) * NT;
  for (int i = tid; i < 2 * per_set; i += T) {
    const int c = i / per_set, rem = i - c * per_set, k = rem / NT, j = rem - k * NT;
    if (j > k) continue;
    const int a = sot0[c * NT + j], b = sot0[c * NT + k + 1];
    const int32_t D = El[c * NT + b] - El[c * NT + a];
    bool ok = D <= 0;
    if (!ok) {
      const int m = D >> 1;
      ok = m < A.M && rpt[c * NT + k] < A.thrpt[(size_t)k * A.M + m];
    }
    acc[(c * NT + k) * NT + j] = ok ? 1 : 0;
  }
  __syncthreads();
  if (tid < 2) {
    const int c = tid;
    const int32_t* m0 = sot0 + c * NT;
    int32_t* so = sotl + c * NT;
    int32_t* to = tosl + c * NT;
    int cur = 0;
    for (int k = 0; k + 1 < NT; ++k) {
      int fin;
      if (acc[(c * NT + k) * NT + cur]) {
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
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Measurement of every temperature of the resident sample.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void measure_resident(const FusedArgs& A, uint32_t* lds) {
  const Geo& g = A.g;
  const int NT = g.NT, NW = g.NW, tid = threadIdx.x, T = blockDim.x;
  const uint32_t* W = lds + A.lay.W;
  const int32_t* El = reinterpret_cast<const int32_t*>(lds + A.lay.E);
  const int32_t* sotl = reinterpret_cast<const int32_t*>(lds + A.lay.sot);
  int32_t* qneg = reinterpret_cast<int32_t*>(lds + A.lay.qneg);
  int64_t* mom = reinterpret_cast<int64_t*>(lds + A.lay.mom);
  if (tid < NT) qneg[tid] = 0;
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, nwave = T >> 6;
  for (int k = wave; k < NT; k += nwave) {
    const uint32_t* Wa = W + (size_t)sotl[k] * 2 * NW;
    const uint32_t* Wb = W + (size_t)(NT + sotl[NT + k]) * 2 * NW;
    int neg = 0;
    for (int w = lane; w < 2 * NW; w += 64) neg += __popc(Wa[w] ^ Wb[w]);
    if (neg) atomicAdd(&qneg[k], neg);
  }
  __syncthreads();
  if (tid < NT) {
    const int k = tid;
    const int a = sotl[k], b = NT + sotl[NT + k];
    const int64_t Q = (int64_t)g.N - 2 * (int64_t)qneg[k];
    const int64_t Ea = El[a], Eb = El[b];
    int64_t* m = mom + (size_t)k * 8;
    m[0] += Ea + Eb;
    m[1] += Ea * Ea + Eb * Eb;
    m[2] += Q;
    m[3] += Q < 0 ? -Q : Q;
    const uint64_t q2 = (uint64_t)(Q * Q);
    m[4] += (int64_t)q2;
    const uint64_t q4lo = q2 * q2, q4hi = __umul64hi(q2, q2);
    const uint64_t lo = (uint64_t)m[5] + q4lo;
    m[5] = (int64_t)lo;
    m[6] = (int64_t)((uint64_t)m[6] + q4hi + (lo < q4lo ? 1u : 0u));
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Houdayer moves for all NT pairs of the resident sample, PC pairs at a time,
// the pairs of a chunk growing their clusters together.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void houdayer_resident(const FusedArgs& A, uint32_t* lds, int s,
                                                  uint32_t v) {
  const Geo& g = A.g;
  const int NT = g.NT, NW = g.NW, tid = threadIdx.x, T = blockDim.x, PC = A.lay.PC;
  uint32_t* W = lds + A.lay.W;
  const uint32_t* Jl = lds + A.lay.J;  // colour 0 block first
  int32_t* El = reinterpret_cast<int32_t*>(lds + A.lay.E);
  const int32_t* sotl = reinterpret_cast<const int32_t*>(lds + A.lay.sot);
  uint32_t* Qs = lds + A.lay.Qs;
  uint32_t* Cs = lds + A.lay.Cs;
  uint32_t* hcnt = lds + A.lay.hcnt;
  int32_t* hdel = reinterpret_cast<int32_t*>(lds + A.lay.hdelta);
  const int W2 = 2 * NW;
  for (int p0 = 0; p0 < NT; p0 += PC) {
    const int np = min(PC, NT - p0);
    if (tid < np) {
      hcnt[tid] = 0;
      hdel[tid] = 0;
    }
    __syncthreads();
    for (int pl = 0; pl < np; ++pl) {
      const int k = p0 + pl;
      const uint32_t* Wa = W + (size_t)sotl[k] * W2;
      const uint32_t* Wb = W + (size_t)(NT + sotl[NT + k]) * W2;
      int cnt = 0;
      for (int i = tid; i < W2; i += T) {
        const uint32_t q = Wa[i] ^ Wb[i];
        Qs[pl * W2 + i] = q;
        Cs[pl * W2 + i] = 0;
        cnt += __popc(q);
      }
      if (cnt) atomicAdd(&hcnt[pl], (uint32_t)cnt);
    }
    __syncthreads();
    // seed of each pair: the m-th q = -1 site in increasing i
    if (tid < np) {
      const int pl = tid, k = p0 + pl;
      const uint32_t n = hcnt[pl];
      if (n > 0) {
        const Ctr4 r = philox10(Ctr4{(uint32_t)k, v, 0u, (kTagHou << 28) | (uint32_t)s}, g.key0, g.key1);
        const uint64_t r64 = (uint64_t)r.x | ((uint64_t)r.y << 32);
        seed_in_rows(g, Qs + pl * W2, Cs + pl * W2, 0, g.NR, (uint32_t)__umul64hi(r64, (uint64_t)n));
      }
    }
    __syncthreads();
    // flood fill, all pairs of the chunk together
    const int items = np * NW;
    int any;
    do {
      int changed = 0;
      for (int c = 0; c < 2; ++c) {
        for (int it = tid; it < items; it += T) {
          const int pl = (int)__umulhi((uint32_t)it, A.magicNW), w = it - pl * NW;
          if (hcnt[pl] == 0) continue;
          if (grow_word<D>(g, Cs + pl * W2, Qs + pl * W2, c, w)) changed = 1;
        }
        if (c == 0) __syncthreads();
      }
      any = __syncthreads_or(changed);
    } while (any);
    // energy change of replica a: bonds leaving the cluster, on colour-0 words
    for (int it = tid; it < items; it += T) {
      const int pl = (int)__umulhi((uint32_t)it, A.magicNW), w = it - pl * NW;
      if (hcnt[pl] == 0) continue;
      const int k = p0 + pl;
      const int dl = cluster_delta_word<D>(g, Cs + pl * W2, W + (size_t)sotl[k] * W2, Jl, w);
      if (dl) atomicAdd(&hdel[pl], dl);
    }
    __syncthreads();
    // exchange the two replicas on the clusters
    for (int pl = 0; pl < np; ++pl) {
      if (hcnt[pl] == 0) continue;
      const int k = p0 + pl;
      uint32_t* Wa = W + (size_t)sotl[k] * W2;
      uint32_t* Wb = W + (size_t)(NT + sotl[NT + k]) * W2;
      for (int i = tid; i < W2; i += T) {
        const uint32_t cw = Cs[pl * W2 + i];
        if (cw) {
          Wa[i] ^= cw;
          Wb[i] ^= cw;
        }
      }
    }
    if (tid < np && hcnt[tid] != 0) {
      const int k = p0 + tid;
      El[sotl[k]] += hdel[tid];
      El[NT + sotl[NT + k]] -= hdel[tid];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(1024) k_mcs(FusedArgs A) {
  extern __shared__ uint32_t lds[];
  const Geo& g = A.g;
  const int T = blockDim.x, tid = threadIdx.x, s = blockIdx.x;
  const int NW = g.NW, NT = g.NT, nslot = g.nslot, W2 = 2 * NW;
  uint32_t* W = lds + A.lay.W;
  uint32_t* Jl = lds + A.lay.J;
  int32_t* El = reinterpret_cast<int32_t*>(lds + A.lay.E);
  int32_t* sotl = reinterpret_cast<int32_t*>(lds + A.lay.sot);
  int32_t* tosl = reinterpret_cast<int32_t*>(lds + A.lay.tos);
  uint32_t* thrl = lds + A.lay.thr;
  int64_t* mom = reinterpret_cast<int64_t*>(lds + A.lay.mom);
  const size_t lat0 = (size_t)s * nslot;

  // ---- load the sample
  const int items = nslot * NW;
  if (g.layout == kLayoutPacked) {
    const uint32_t* src = static_cast<const uint32_t*>(A.spins) + lat0 * W2;
    for (int i = tid; i < nslot * W2; i += T) W[i] = src[i];
  } else {
    const int8_t* src = static_cast<const int8_t*>(A.spins) + lat0 * g.N;
    for (int it = tid; it < items; it += T) {
      const int slot = (int)__umulhi((uint32_t)it, A.magicNW), w = it - slot * NW;
      word_from_int8(g, src + (size_t)slot * g.N, w, W[slot * W2 + w], W[slot * W2 + NW + w]);
    }
  }
  const uint32_t* jws = A.jw + (size_t)s * 2 * 2 * D * NW;
  for (int i = tid; i < 2 * 2 * D * NW; i += T) Jl[i] = jws[i];
  for (int i = tid; i < nslot; i += T) El[i] = A.E[lat0 + i];
  for (int i = tid; i < 2 * NT; i += T) {
    sotl[i] = A.sot[(size_t)s * 2 * NT + i];
    tosl[i] = A.tos[(size_t)s * 2 * NT + i];
  }
  for (int i = tid; i < 4 * NT; i += T) thrl[i] = A.thr[i];
  if (A.meas)
    for (int i = tid; i < 8 * NT; i += T) mom[i] = A.mom[(size_t)s * NT * 8 + i];
  const uint32_t t0 = A.ctr->t, u0 = A.ctr->u, v0 = A.ctr->v;
  __syncthreads();

  for (int step = 0; step < A.nmcs; ++step) {
    const uint32_t t = t0 + (uint32_t)step;
    for (int c = 0; c < 2; ++c) {
      const uint32_t* Jc = Jl + c * 2 * D * NW;
      for (int it = tid; it < items; it += T) {
        const int slot = (int)__umulhi((uint32_t)it, A.magicNW), w = it - slot * NW;
        const int k = tosl[slot];
        int dE = 0;
        sweep_word<D>(g, W + slot * W2, Jc, c, w, slot, s, t, thrl[k * 4 + 0], thrl[k * 4 + 1],
                      thrl[k * 4 + 2], dE);
        if (dE) atomicAdd(&El[slot], dE);
      }
      __syncthreads();
    }
    if (A.hou) houdayer_resident<D>(A, lds, s, v0 + (uint32_t)step);
    exchange_resident(A, lds, s, u0 + (uint32_t)step);
    if (A.meas) measure_resident(A, lds);
  }

  // ---- store the sample
  if (g.layout == kLayoutPacked) {
    uint32_t* dst = static_cast<uint32_t*>(A.spins) + lat0 * W2;
    for (int i = tid; i < nslot * W2; i += T) dst[i] = W[i];
  } else {
    int8_t* dst = static_cast<int8_t*>(A.spins) + lat0 * g.N;
    for (int it = tid; it < items; it += T) {
      const int slot = (int)__umulhi((uint32_t)it, A.magicNW), w = it - slot * NW;
      word_to_int8(g, dst + (size_t)slot * g.N, w, W[slot * W2 + w], W[slot * W2 + NW + w]);
    }
  }
  for (int i = tid; i < nslot; i += T) A.E[lat0 + i] = El[i];
  for (int i = tid; i < 2 * NT; i += T) {
    A.sot[(size_t)s * 2 * NT + i] = sotl[i];
    A.tos[(size_t)s * 2 * NT + i] = tosl[i];
  }
  if (A.meas)
    for (int i = tid; i < 8 * NT; i += T) A.mom[(size_t)s * NT * 8 + i] = mom[i];
}

// ---------------------------------------------------------------------------
bool fused_plan(const Geo& g, bool hou, FusedLayout& lay) {
  const size_t budget = 160 * 1024 / 4;  // LDS words per workgroup on gfx950
  size_t off = 0;
  auto take = [&](size_t words, size_t align) {
    off = (off + align - 1) / align * align;
    const size_t at = off;
    off += words;
    return (int)at;
  };
  const size_t W2 = 2 * (size_t)g.NW;
  lay.W = take((size_t)g.nslot * W2, 1);
  lay.J = take(2 * 2 * (size_t)g.d * g.NW, 1);
  lay.E = take(g.nslot, 1);
  lay.sot = take(2 * g.NT, 1);
  lay.tos = take(2 * g.NT, 1);
  lay.sot0 = take(2 * g.NT, 1);
  lay.thr = take(4 * g.NT, 1);
  lay.mom = take(16 * (size_t)g.NT, 2);
  lay.qneg = take(g.NT, 1);
  lay.rpt = take(2 * g.NT, 1);
  lay.acc = take((2 * (size_t)g.NT * g.NT + 3) / 4, 1);
  lay.PC = 0;
  lay.Qs = lay.Cs = lay.hcnt = lay.hdelta = (int)off;
  if (hou) {
    if (off + 2 * W2 + 2 > budget) return false;
    const size_t per = 2 * W2 + 2;
    size_t pc = (budget - off) / per;
    if (pc > (size_t)g.NT) pc = g.NT;
    lay.PC = (int)pc;
    lay.Qs = take(pc * W2, 1);
    lay.Cs = take(pc * W2, 1);
    lay.hcnt = take(pc, 1);
    lay.hdelta = take(pc, 1);
  }
  lay.words = (int)off;
  return off <= budget;
}

hipError_t launch_mcs_fused(const Geo& g, const FusedLayout& lay, void* spins, const uint32_t* jw,
                            int32_t* E, int32_t* sot, int32_t* tos, const uint32_t* thr,
                            const uint32_t* thrpt, int M, int64_t* mom, const DevCounters* ctr,
                            int nmcs, bool hou, bool meas, hipStream_t st) {
  FusedArgs A;
  A.g = g;
  A.spins = spins;
  A.jw = jw;
  A.E = E;
  A.sot = sot;
  A.tos = tos;
  A.thr = thr;
  A.thrpt = thrpt;
  A.M = M;
  A.mom = mom;
  A.ctr = ctr;
  A.nmcs = nmcs;
  A.hou = hou ? 1 : 0;
  A.meas = meas ? 1 : 0;
  A.magicNW = (uint32_t)((0x100000000ull + (uint64_t)g.NW - 1) / (uint64_t)g.NW);
  A.lay = lay;
  const size_t bytes = (size_t)lay.words * 4;
  const dim3 grid((unsigned)g.S), block(1024);
  if (g.d == 3) {
    hipError_t e = hipFuncSetAttribute((const void*)k_mcs<3>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mcs<3>, grid, block, bytes, st, A);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)k_mcs<2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mcs<2>, grid, block, bytes, st, A);
  }
  return hipGetLastError();
}

}  // namespace ptsg
