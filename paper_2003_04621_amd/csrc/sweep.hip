// sweep.hip -- checkerboard Metropolis sweeps (Sec. 2.2 of the paper; the
// update list of Sec. 2.4), one workgroup slice per lattice, the lattice held
// in LDS as colour-split row words for all n sweeps of a launch.
#include "device.h"
#include "kernels.h"
#include "rowops.h"

namespace ptsg {

// Grid: one block holds LPB lattices, T threads each (block = LPB*T threads).
template <int D>
__global__ void __launch_bounds__(256) k_sweep(Geo g, void* spins, const uint32_t* __restrict__ jw,
                                               int32_t* __restrict__ E,
                                               const int32_t* __restrict__ tos,
                                               const uint32_t* __restrict__ thr,
                                               DevCounters* ctr, int nsweeps, int T, int LPB,
                                               int64_t* stats) {
  extern __shared__ uint32_t lds[];
  int* red = reinterpret_cast<int*>(lds);  // [LPB] energy changes, then [LPB] flip counts
  uint32_t* W0 = lds + 2 * LPB;
  const int li = threadIdx.x / T, t = threadIdx.x - li * T;
  const long nlat = (long)g.S * g.nslot;
  const long lat = (long)blockIdx.x * LPB + li;
  const bool active = li < LPB && lat < nlat;
  uint32_t* W = W0 + (size_t)li * 2 * g.NW;
  if (threadIdx.x < 2 * LPB) red[threadIdx.x] = 0;

  int s = 0, slot = 0, k = 0;
  uint32_t th2 = 0, th4 = 0, th6 = 0;
  const uint32_t t0 = load_counter(&ctr->t);
  if (active) {
    s = (int)(lat / g.nslot);
    slot = (int)(lat - (long)s * g.nslot);
    const int set = slot / g.NT, j = slot - set * g.NT;
    k = tos[((size_t)s * 2 + set) * g.NT + j];
    th2 = thr[k * 4 + 0];
    th4 = thr[k * 4 + 1];
    th6 = thr[k * 4 + 2];
    load_lattice(g, spins, (size_t)lat, W, t, T);
  }
  __syncthreads();
  const uint32_t* jws = jw + (size_t)s * 2 * 2 * D * g.NW;
  int dE = 0, nf = 0;
  int* nfp = stats ? &nf : nullptr;
  for (int rep = 0; rep < nsweeps; ++rep) {
    for (int c = 0; c < 2; ++c) {
      if (active) {
        const uint32_t* jwc = jws + (size_t)c * 2 * D * g.NW;
        for (int w = t; w < g.NW; w += T)
          sweep_word<D>(g, W, jwc, c, w, slot, s, t0 + (uint32_t)rep, th2, th4, th6, dE, nfp);
      }
      __syncthreads();
    }
  }
  if (active) {
    store_lattice(g, spins, (size_t)lat, W, t, T);
    atomicAdd(&red[li], dE);
    if (stats && nf) atomicAdd(&red[LPB + li], nf);
  }
  __syncthreads();
  if (active && t == 0) {
    E[lat] += red[li];
    // a launch's sweeps all run at the slot's temperature (no exchange between them)
    if (stats && red[LPB + li])
      atomicAdd(reinterpret_cast<unsigned long long*>(stats + ((size_t)s * g.NT + k) * kNStat),
                (unsigned long long)red[LPB + li]);
  }
}

void sweep_shape(const Geo& g, int& T, int& LPB, int& threads, size_t& lds) {
  T = g.NW < 256 ? g.NW : 256;
  LPB = 256 / T;
  if (LPB < 1) LPB = 1;
  threads = T * LPB;
  lds = sizeof(uint32_t) * (2 * (size_t)LPB + (size_t)LPB * 2 * g.NW);
}

hipError_t launch_sweep(const Geo& g, void* spins, const uint32_t* jw, int32_t* E,
                        const int32_t* tos, const uint32_t* thr, DevCounters* ctr, int n,
                        int64_t* stats, hipStream_t st) {
  int T, LPB, threads;
  size_t lds;
  sweep_shape(g, T, LPB, threads, lds);
  const long nlat = (long)g.S * g.nslot;
  const unsigned blocks = (unsigned)((nlat + LPB - 1) / LPB);
  if (g.d == 3) {
    if (lds > 65536)
      { const hipError_t ea = hipFuncSetAttribute((const void*)k_sweep<3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); if (ea != hipSuccess) return ea; }
    hipLaunchKernelGGL(k_sweep<3>, dim3(blocks), dim3(threads), lds, st, g, spins, jw, E, tos, thr,
                       ctr, n, T, LPB, stats);
  } else {
    if (lds > 65536)
      { const hipError_t ea = hipFuncSetAttribute((const void*)k_sweep<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); if (ea != hipSuccess) return ea; }
    hipLaunchKernelGGL(k_sweep<2>, dim3(blocks), dim3(threads), lds, st, g, spins, jw, E, tos, thr,
                       ctr, n, T, LPB, stats);
  }
  return hipGetLastError();
}

}  // namespace ptsg
