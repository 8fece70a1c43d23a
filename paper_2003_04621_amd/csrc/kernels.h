// kernels.h -- host-side launchers of the gfx950 kernels (one per step of
// the path).  All launchers enqueue on `st` and return hipGetLastError().
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace ptsg {

// Initial spins: site i of slot r, sample s takes word i&3 of Philox counter
// (i>>2, 0, r, 2<<28 | s); s_i = -1 iff the word's top bit is set.
hipError_t launch_init_spins(const Geo& g, void* spins, hipStream_t st);

// The spins of every lattice from the int8 layout to the packed colour words
// (to_packed) or back; src and dst are distinct buffers.
hipError_t launch_convert_layout(const Geo& g, const void* src, void* dst, bool to_packed,
                                 hipStream_t st);

// int8 couplings [S][d][N] -> direction words jw [S][2][2d][NR]: bit b of
// jw[s][c][dir][R] is set iff the bond between the colour-c site b of row R and
// its neighbour in direction dir (+x0, -x0, +x1, -x1, +x2, -x2) is -1.
hipError_t launch_pack_couplings(const Geo& g, const int8_t* J8, uint32_t* jw, hipStream_t st);

// Energy of every slot from scratch: E = 2 * #unsatisfied bonds - d*N.
hipError_t launch_energy(const Geo& g, const void* spins, const uint32_t* jw, int32_t* E,
                         hipStream_t st);

// Run diagnostics per sample and temperature (jobs created with
// PT_TRACK_STATS): int64 [S][NT][kNStat] -- [0] accepted Metropolis flips of
// the configurations at that temperature, [1] accepted exchanges of the pair
// (k, k+1), [2] Houdayer passes that exchanged sites, [3] the sites they
// exchanged, [4 + b] passes that exchanged between 2^b and 2^(b+1) - 1 sites.
constexpr int kNStat = 24;

// n checkerboard Metropolis sweeps starting at sweep number ctr->t (stats:
// null, or the diagnostics above).
hipError_t launch_sweep(const Geo& g, void* spins, const uint32_t* jw, int32_t* E,
                        const int32_t* tos, const uint32_t* thr, DevCounters* ctr, int n,
                        int64_t* stats, hipStream_t st);

// One replica-exchange pass numbered ctr->u, followed by the replica-walk
// bookkeeping of walk_observe (walk [S][2NT][2], trips [S][32][3]; both null
// for a job that does not keep it).
hipError_t launch_exchange(const Geo& g, const int32_t* E, int32_t* sot, int32_t* tos,
                           const uint32_t* thrpt, int M, int32_t* walk, uint64_t* trips,
                           DevCounters* ctr, int64_t* stats, hipStream_t st);

// One Houdayer pass numbered ctr->v.
hipError_t launch_houdayer(const Geo& g, void* spins, const uint32_t* jw, int32_t* E,
                           const int32_t* sot, DevCounters* ctr, int64_t* stats, hipStream_t st);
// One multi-cluster Houdayer pass numbered ctr->v (g.N <= kMultiMaxSites).
hipError_t launch_houdayer_multi(const Geo& g, void* spins, const uint32_t* jw, int32_t* E,
                                 const int32_t* sot, DevCounters* ctr, int64_t* stats,
                                 hipStream_t st);

// One measurement; mom is int64 [S][NT][8]; modes (null: not kept) int64
// [S][NT][L/2+1] receives each temperature's mode_autocorr sums.  With
// every > 1 nothing happens unless measures_at(ctr->t + 1, every).
hipError_t launch_measure(const Geo& g, const void* spins, const int32_t* E,
                          const int32_t* sot, int64_t* mom, int64_t* modes, DevCounters* ctr,
                          int every, hipStream_t st);

// Advances the device counters by `step` (one thread; enqueued after the
// kernels that read them).
hipError_t launch_advance(DevCounters* ctr, CounterStep step, hipStream_t st);

// LDS word offsets of the fused Monte Carlo step kernel: configurations W,
// couplings J, energies E, maps sot/tos (and the pre-pass copy sot0),
// threshold rows, moments, overlap counts, exchange randoms and decision
// matrix, replica-walk words and the launch's round-trip sums (64-bit
// aligned), per-wavefront plane counters and the item's two-replica mode sums
// (64-bit), and the Houdayer words Qs of PC wavefronts; `words` in all.
struct FusedLayout {
  int W, J, E, sot, tos, sot0, thr, mom, qneg, rpt, acc, walk, trip, mcnt, modes, Qs, PC, hq, words;
};

// Everything one fused workgroup needs about a job, for nmcs steps.
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
  // replica walk (null unless the job tracks it): [S][2NT][2] label and pass
  // the current round trip began; [S][32][3] round trips per log2 bin
  int32_t* walk;
  uint64_t* trips;
  // two-replica modes (null unless the job keeps them): [S][NT][L/2+1]
  int64_t* modes;
  const DevCounters* ctr;
  int nmcs, hou, meas;
  int every;  // a measured step is one whose 1-based sweep number is a multiple
  uint32_t magicNW;  // item / NW
  FusedLayout lay;
  // Split samples (parts > 0): part p of a sample holds slots [p R, p R + R),
  // couplings in LDS iff jlds.  Ex [S][2][nslot] and snap [S][2][nslot][2NW]
  // are the parity-buffered published energies and configurations, bar [S+1]
  // the per-sample barrier counters followed by the job's fault word.
  int parts, R, jlds;
  int32_t* Ex;
  uint32_t* snap;
  uint32_t* bar;
};

// One work item of the persistent batch kernel: replica sets
// [c_lo, c_lo + nsets) of sample `sample` of job `job`, or with nsets == 0
// part c_lo of a split sample (the parts of a sample are consecutive items).
struct BatchItem {
  int job, sample, c_lo, nsets;
};

// Most workgroups one split sample may use (all of them must be running at
// the same time).
constexpr int kMaxParts = 64;

// Plans the LDS of a fused workgroup holding `nsets` replica sets of one
// sample (`waves` wavefronts); false if it does not fit in 160 KiB.  With
// houdayer and multi, the Houdayer moves are the multi-cluster variant, done
// by the first lay.PC wavefronts, each with a scratch area at lay.Qs.
bool fused_plan(const Geo& g, bool houdayer, int nsets, int waves, FusedLayout& lay,
                bool walk = false, bool modes = false, bool multi = false);

// Plans a split sample: the fewest parts (<= kMaxParts) whose R slots fit one
// workgroup's LDS, with the couplings in LDS when that still leaves room for
// min(2 N_T, 8) slots.  False if even one slot does not fit.
bool split_plan(const Geo& g, FusedLayout& lay, int& parts, int& R, int& jlds, bool walk = false,
                bool modes = false);

FusedArgs make_fused_args(const Geo& g, const FusedLayout& lay, void* spins, const uint32_t* jw,
                          int32_t* E, int32_t* sot, int32_t* tos, const uint32_t* thr,
                          const uint32_t* thrpt, int M, int64_t* mom, int32_t* walk,
                          uint64_t* trips, int64_t* modes, const DevCounters* ctr, int nmcs,
                          bool houdayer, bool measure);

// Kinds of work a batch launch holds (Houdayer moves, measurements, split
// samples, jobs that track the replica walk, jobs that measure the two-replica
// modes); the launch runs the kernel compiled for exactly that set.
constexpr int kFeatHou = 1, kFeatMeas = 2, kFeatSplit = 4, kFeatWalk = 8, kFeatModes = 16;

// Persistent batch: resets the queue, runs every item to its job's nmcs, then
// advances each job's counters.  `jobs` and `items` are device arrays.
// prepare_batch sets the kernel's dynamic LDS limit and reports its VGPRs
// per lane.
hipError_t prepare_batch(int d, int feat, size_t lds_bytes, int* vgprs);
// Workgroups of `threads` threads, lds_bytes of dynamic LDS each, that the
// runtime can keep resident on one CU at once for this kernel.
hipError_t batch_residency(int d, int feat, int threads, size_t lds_bytes, int* per_cu);
hipError_t launch_batch(int d, int feat, const FusedArgs* jobs, int njobs, const BatchItem* items,
                        int nitems, uint32_t* queue, int blocks, int threads, size_t lds_bytes,
                        hipStream_t st);

// Launch shape of the sweep kernel (threads per lattice T, lattices per block).
void sweep_shape(const Geo& g, int& T, int& LPB, int& threads, size_t& lds);

}  // namespace ptsg
