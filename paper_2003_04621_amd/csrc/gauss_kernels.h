// gauss_kernels.h -- host-side launchers of the Gaussian-coupling kernels
// (gauss.hip).  All launchers enqueue on `st` and return hipGetLastError().
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace ptsg {

// Coupling units Jn int32 [S][d][N] (J = n 2^-16) -> group data Jg (gauss.h).
hipError_t launch_gauss_prepare(const Geo& g, const int32_t* Jn, int4* Jg, hipStream_t st);
// Energies of every slot from scratch, int64 units [S][2NT].
hipError_t launch_gauss_energy(const Geo& g, const void* spins, const int4* Jg, int64_t* E64,
                               hipStream_t st);
// n checkerboard Metropolis sweeps starting at sweep number ctr->t; beta
// double [NT], cz float [NT] = gauss_cz(beta).
hipError_t launch_gauss_sweep(const Geo& g, void* spins, const int4* Jg, int64_t* E64,
                              const int32_t* tos, const double* beta, const float* cz,
                              const DevCounters* ctr, int n, hipStream_t st);
// Launch shape of the sweep: threads per block, temperatures per block, blocks
// per (sample, set), dynamic LDS bytes.
void gauss_sweep_shape(const Geo& g, int& threads, int& CH, int& nchunk, size_t& lds);
// One exchange pass numbered ctr->u.
hipError_t launch_gauss_exchange(const Geo& g, const int64_t* E64, int32_t* sot, int32_t* tos,
                                 const double* beta, const DevCounters* ctr, hipStream_t st);
// One Houdayer pass numbered ctr->v, single-cluster or multi-cluster
// (multi needs g.N <= kMultiMaxSites).
hipError_t launch_gauss_houdayer(const Geo& g, void* spins, const int4* Jg, int64_t* E64,
                                 const int32_t* sot, const DevCounters* ctr, bool multi,
                                 hipStream_t st);
// One measurement into mom int64 [S][NT][8] (gauss.hip); with every > 1
// nothing happens unless measures_at(ctr->t + 1, every).
hipError_t launch_gauss_measure(const Geo& g, const void* spins, const int64_t* E64, const int32_t* sot,
                                int64_t* mom, const DevCounters* ctr, int every, hipStream_t st);
// Fused steps (gauss_fused.hip): n steps of sweep (+ single-cluster Houdayer)
// + exchange (+ measurement at interval `every`), one workgroup per sample
// holding all its configurations in LDS; the counters are read, not advanced.
// hipErrorInvalidValue if the sample does not fit (gauss_fused_lds above
// kGaussFusedMaxLds).
constexpr size_t kGaussFusedMaxLds = 160 * 1024;
size_t gauss_fused_lds(const Geo& g);
hipError_t launch_gauss_fused(const Geo& g, void* spins, const int4* Jg, int64_t* E64, int32_t* sot,
                              int32_t* tos, const double* beta, const float* cz, int64_t* mom,
                              const DevCounters* ctr, int n, bool hou, bool meas, int every,
                              hipStream_t st);
// Acceptance decisions of device arrays (tests): mode 0 Metropolis tiers,
// 1 exchange tiers, 2 double-double alone.
hipError_t launch_gauss_accept(const uint32_t* r, const double* b, const int64_t* u, int32_t* out, int n,
                               int mode, hipStream_t st);

}  // namespace ptsg
