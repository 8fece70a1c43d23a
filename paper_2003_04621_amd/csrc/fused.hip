// fused.hip -- host side of the fused Monte Carlo step kernels: the queue
// reset and counter advance kernels, LDS plans of resident and split samples,
// launch arguments, and the launch of the persistent batch kernel whose
// device code is in fused_device.h.
#include <map>
#include <mutex>
#include <utility>

#include "fused_device.h"

namespace ptsg {

// Clears the queue and the barrier counters of every split job (block j
// serves job j - 1).
__global__ void k_batch_reset(const FusedArgs* __restrict__ jobs, uint32_t* queue) {
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) *queue = 0u;
    return;
  }
  const FusedArgs& A = jobs[blockIdx.x - 1];
  if (A.parts == 0) return;
  for (int i = threadIdx.x; i < A.g.S; i += blockDim.x) A.bar[i] = 0u;
}

// Advances every job's counters by its own number of steps in this launch.
__global__ void k_batch_advance(const FusedArgs* __restrict__ jobs, int njobs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  const FusedArgs& A = jobs[j];
  DevCounters* c = const_cast<DevCounters*>(A.ctr);
  const uint32_t n = (uint32_t)A.nmcs, t0 = c->t, e = (uint32_t)A.every;
  c->t += n;
  c->u += n;
  if (A.hou) c->v += n;
  if (A.meas) c->n_meas += e > 1u ? (t0 + n) / e - t0 / e : n;
}

// ---------------------------------------------------------------------------
bool fused_plan(const Geo& g, bool hou, int nsets, int waves, FusedLayout& lay, bool walk,
                bool modes, bool multi) {
  // LDS words per workgroup on gfx950 (160 KiB), less room for static LDS
  const size_t budget = (160 * 1024 - 512) / 4;
  size_t off = 0;
  auto take = [&](size_t words, size_t align) {
    off = (off + align - 1) / align * align;
    const size_t at = off;
    off += words;
    return (int)at;
  };
  const size_t W2 = 2 * (size_t)g.NW;
  lay.W = take((size_t)nsets * g.NT * W2, 1);
  lay.J = take(2 * 2 * (size_t)g.d * g.NW, 1);
  lay.E = take(g.nslot, 1);
  lay.sot = take(2 * g.NT, 1);
  lay.tos = take(2 * g.NT, 1);
  lay.sot0 = take(2 * g.NT, 1);
  lay.thr = take(4 * g.NT, 1);
  lay.mom = take(16 * (size_t)g.NT, 2);
  lay.qneg = take(g.NT, 1);
  lay.rpt = take(2 * g.NT, 1);
  lay.acc = take(2 * (size_t)(g.NT - 1) * ((g.NT + 31) / 32), 1);
  lay.walk = take(walk ? 2 * (size_t)g.nslot : 0, walk ? 2 : 1);
  lay.trip = take(walk ? 2 * 32 * 3 : 0, walk ? 2 : 1);
  const bool md = modes && nsets == 2;
  lay.mcnt = take(md ? (size_t)waves * 3 * g.L : 0, 1);
  lay.modes = take(md ? 2 * (size_t)g.NT * (g.L / 2 + 1) : 0, md ? 2 : 1);
  lay.PC = 0;
  lay.Qs = (int)off;
  lay.hq = (int)off;
  if (hou && nsets == 2 && multi) {
    // multi-cluster moves: a scratch area for each of the first PC
    // wavefronts (8-byte aligned: the row masks are 64-bit), as many as fit
    if (g.N > kMultiMaxSites) return false;
    const size_t per = (size_t)((multi_scratch_words(g.N, g.NR, g.NW) + 1) & ~1);
    const size_t base = (off + 1) / 2 * 2;
    int pc = waves < 8 ? waves : 8;
    while (pc > 1 && base + pc * per > budget) --pc;
    lay.PC = pc;
    lay.Qs = take(pc * per, 2);
  } else if (hou && nsets == 2) {
    lay.hq = take(1, 1);  // Houdayer pair counter
    if (!rows64_houdayer(g)) {
      // overlap and cluster words for each wavefront
      lay.PC = waves;
      lay.Qs = take((size_t)waves * 2 * W2, 1);
    }
  }
  lay.words = (int)off;
  return off <= budget;
}

bool split_plan(const Geo& g, FusedLayout& lay, int& parts, int& R, int& jlds, bool walk,
                bool modes) {
  const int waves = 16;  // plane counters for up to 16 wavefronts
  const size_t mcnt = modes ? (size_t)waves * 3 * g.L : 0;
  const size_t mwords = modes ? 2 * (size_t)g.NT * (g.L / 2 + 1) : 0;
  const size_t budget = (160 * 1024 - 512) / 4;
  const size_t W2 = 2 * (size_t)g.NW, Jw = 2 * 2 * (size_t)g.d * g.NW;
  for (int jl = 1; jl >= 0; --jl) {
    // everything but the slots' words
    size_t fixed = jl ? Jw : 0;
    fixed += g.nslot + 3 * 2 * (size_t)g.NT + 4 * (size_t)g.NT;
    fixed = (fixed + 1) / 2 * 2 + 16 * (size_t)g.NT;
    fixed += g.NT + 2 * (size_t)g.NT + 2 * (size_t)(g.NT - 1) * ((g.NT + 31) / 32);
    if (walk) fixed = (fixed + 1) / 2 * 2 + 2 * (size_t)g.nslot + 2 * 32 * 3;
    if (modes) fixed = (fixed + mcnt + 1) / 2 * 2 + mwords;
    if (fixed >= budget) continue;
    const size_t rmax = std::min<size_t>((budget - fixed) / W2, (size_t)g.nslot);
    if (rmax < 1 || (jl && rmax < std::min(g.nslot, 8))) continue;
    const int p = (int)((g.nslot + rmax - 1) / rmax);
    // the parts' moment increments ([p][N_T][8] 64-bit words) are combined
    // through one parity half of the published-configuration scratch
    if (p > kMaxParts || (size_t)p * 8 > W2) continue;
    R = (g.nslot + p - 1) / p;
    parts = (g.nslot + R - 1) / R;
    jlds = jl;
    size_t off = 0;
    auto take = [&](size_t words, size_t align) {
      off = (off + align - 1) / align * align;
      const size_t at = off;
      off += words;
      return (int)at;
    };
    lay.W = take((size_t)R * W2, 1);
    lay.J = take(jl ? Jw : 0, 1);
    lay.E = take(g.nslot, 1);
    lay.sot = take(2 * g.NT, 1);
    lay.tos = take(2 * g.NT, 1);
    lay.sot0 = take(2 * g.NT, 1);
    lay.thr = take(4 * g.NT, 1);
    lay.mom = take(16 * (size_t)g.NT, 2);
    lay.qneg = take(g.NT, 1);
    lay.rpt = take(2 * g.NT, 1);
    lay.acc = take(2 * (size_t)(g.NT - 1) * ((g.NT + 31) / 32), 1);
    lay.walk = take(walk ? 2 * (size_t)g.nslot : 0, walk ? 2 : 1);
    lay.trip = take(walk ? 2 * 32 * 3 : 0, walk ? 2 : 1);
    lay.mcnt = take(mcnt, 1);
    lay.modes = take(mwords, modes ? 2 : 1);
    lay.PC = 0;
    lay.Qs = (int)off;
    lay.hq = (int)off;
    lay.words = (int)off;
    return off <= budget;
  }
  return false;
}

FusedArgs make_fused_args(const Geo& g, const FusedLayout& lay, void* spins, const uint32_t* jw,
                          int32_t* E, int32_t* sot, int32_t* tos, const uint32_t* thr,
                          const uint32_t* thrpt, int M, int64_t* mom, int32_t* walk,
                          uint64_t* trips, int64_t* modes, const DevCounters* ctr, int nmcs,
                          bool hou, bool meas) {
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
  A.walk = walk;
  A.trips = trips;
  A.modes = modes;
  A.ctr = ctr;
  A.nmcs = nmcs;
  A.hou = hou ? 1 : 0;
  A.meas = meas ? 1 : 0;
  A.every = 1;
  A.magicNW = (uint32_t)((0x100000000ull + (uint64_t)g.NW - 1) / (uint64_t)g.NW);
  A.lay = lay;
  A.parts = A.R = A.jlds = 0;
  A.Ex = nullptr;
  A.snap = nullptr;
  A.bar = nullptr;
  return A;
}

template <typename K>
static hipError_t lds_attr(K kernel, size_t bytes) {
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

namespace {
// The batch kernel variants are instantiated in four translation units
// (fused_k2a/k2b/k3a/k3b.hip: dimension, low or high half of the feature
// sets), so that they compile in parallel.
BatchKernel batch_kernel(int d, int feat) {
  feat &= 31;
  if (d == 3) return feat < 16 ? batch_kernel_3a(feat) : batch_kernel_3b(feat);
  return feat < 16 ? batch_kernel_2a(feat) : batch_kernel_2b(feat);
}
}  // namespace

hipError_t prepare_batch(int d, int feat, size_t lds_bytes, int* vgprs) {
  const BatchKernel k = batch_kernel(d, feat);
  // the dynamic-LDS limit of each variant is raised only when a launch needs
  // more than any before it on this device (kernel attributes are per device)
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> set_to;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  bool raise = false;
  {
    std::lock_guard<std::mutex> lk(mu);
    size_t& cur = set_to[{dev, (const void*)k}];
    raise = lds_bytes > cur;
  }
  if (raise) {
    e = lds_attr(k, lds_bytes);
    if (e == hipSuccess) {
      std::lock_guard<std::mutex> lk(mu);
      size_t& cur = set_to[{dev, (const void*)k}];
      if (lds_bytes > cur) cur = lds_bytes;
    }
  }
  if (e == hipSuccess && vgprs) {
    hipFuncAttributes at{};
    e = hipFuncGetAttributes(&at, (const void*)k);
    *vgprs = at.numRegs;
  }
  return e;
}

// Workgroups of `threads` threads with lds_bytes of LDS each that can be
// resident on one CU at once, as the runtime computes it for this kernel.
hipError_t batch_residency(int d, int feat, int threads, size_t lds_bytes, int* per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, batch_kernel(d, feat), threads,
                                                      lds_bytes);
}

hipError_t launch_batch(int d, int feat, const FusedArgs* jobs, int njobs, const BatchItem* items,
                        int nitems, uint32_t* queue, int blocks, int threads, size_t lds_bytes,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3((unsigned)njobs + 1), dim3(256), 0, st, jobs, queue);
  hipLaunchKernelGGL(batch_kernel(d, feat), dim3(blocks), dim3(threads), lds_bytes, st, jobs, items,
                     nitems, queue);
  hipLaunchKernelGGL(k_batch_advance, dim3((unsigned)((njobs + 255) / 256)), dim3(256), 0, st, jobs,
                     njobs);
  return hipGetLastError();
}

}  // namespace ptsg
