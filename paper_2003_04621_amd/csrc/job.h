// job.h -- host-side job state shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "kernels.h"

#define PT_API extern "C" __attribute__((visibility("default")))

// Records a thread-local error message and returns `code`.
int pt_fail(int code, const std::string& msg);
const char* pt_error_text();

// One job: S samples x 2 replica sets x N_T temperatures.  Pointers are device
// memory allocated through the hooks captured at creation.
struct pt_job {
  ptsg::Geo g{};
  hipStream_t stream = nullptr;
  void* spins = nullptr;     // int8 [S][2NT][N] or u32 [S][2NT][2][NW]
  uint32_t* jw = nullptr;    // [S][2][2d][NW]
  int32_t* E = nullptr;      // [S][2NT]
  int32_t* sot = nullptr;    // [S][2][NT]
  int32_t* tos = nullptr;    // [S][2][NT]
  uint32_t* thr = nullptr;   // [NT][4]
  uint32_t* thrpt = nullptr; // [NT-1][M]
  int M = 0;
  ptsg::DevCounters* ctr = nullptr;
  int64_t* mom = nullptr;    // [S][NT][8]
  // measured steps of pt_mcs / batches: 1-based sweep number a multiple of this
  int meas_every = 1;
  // two-replica modes, allocated only for jobs created with PT_TRACK_MODES
  bool track_modes = false;
  int64_t* modes = nullptr;  // [S][NT][L/2+1]
  // replica walk, allocated only for jobs created with PT_TRACK_WALK
  bool track_walk = false;
  int32_t* walk = nullptr;   // [S][2NT][2]: replica-walk label, pass its round trip began
  uint64_t* trips = nullptr; // [S][32][3]: round trips per log2 bin of the ending pass
  // run diagnostics, allocated only for jobs created with PT_TRACK_STATS
  // (such jobs always run the per-step kernels)
  bool track_stats = false;
  int64_t* stats = nullptr;  // [S][NT][kNStat]
  // fused-step LDS plans: both sets without / with Houdayer, one set, (3
  // unused: split samples have split_lay), both sets with multi-cluster
  // Houdayer moves
  ptsg::FusedLayout plan[5];
  bool fused_ok[5] = {false, false, false, false, false};
  // split-sample plan (samples whose sets do not fit one workgroup) and its
  // scratch: published energies / configurations and barrier counters
  ptsg::FusedLayout split_lay{};
  bool split_ok = false;
  int split_parts = 0, split_R = 0, split_jlds = 0;
  int32_t* Ex = nullptr;     // [S][2][2NT]
  uint32_t* snap = nullptr;  // [S][2][2NT][2NW]
  uint32_t* bar = nullptr;   // [S] barrier counters + fault word
  // Gaussian couplings (pt_init_gauss): integer units, 64-bit energies, the
  // per-group coupling data of gauss.h and the inverse temperatures; thr,
  // thrpt, jw and E stay null for such a job
  bool gauss = false;
  int32_t* gJn = nullptr;    // [S][d][N] coupling units
  int4* gJ = nullptr;        // [S][2][2d+1][NGc]
  int64_t* E64 = nullptr;    // [S][2NT]
  double* gbeta = nullptr;   // [NT]
  float* gcz = nullptr;      // [NT]
  bool poisoned = false;
  // bumped when device buffers held by launch arguments change (pt_set_layout)
  uint32_t epoch = 0;
  struct pt_batch* self_batch = nullptr;  // one-job batch behind pt_mcs
  std::vector<void*> allocs;
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_ctx = nullptr;

  size_t spin_bytes() const {
    const size_t lat = (size_t)g.S * g.nslot;
    return g.layout == ptsg::kLayoutPacked ? lat * 2 * g.NW * sizeof(uint32_t) : lat * g.N;
  }

  void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 4;
    if (alloc_fn) {
      p = alloc_fn(bytes, alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (p) allocs.push_back(p);
    return p;
  }
  // Frees one buffer from dalloc (after the work using it has completed).
  void dfree(void* p) {
    for (size_t i = 0; i < allocs.size(); ++i) {
      if (allocs[i] != p) continue;
      if (free_fn)
        free_fn(p, alloc_ctx);
      else
        (void)hipFree(p);
      allocs.erase(allocs.begin() + (long)i);
      return;
    }
  }
  void release() {
    for (void* p : allocs) {
      if (free_fn)
        free_fn(p, alloc_ctx);
      else
        (void)hipFree(p);
    }
    allocs.clear();
  }
};

// Batch internals used by the request server (batch.hip).
struct pt_batch;
pt_batch* batch_new(hipStream_t st);
int batch_round(pt_batch* b, const std::vector<pt_job*>& jobs, const std::vector<int>& steps,
                const std::vector<uint32_t>& flags);
void batch_free(pt_batch* b);
// mcs fused steps of one job through its own one-job batch (work list cached
// while mcs and flags repeat).
int batch_run_job(pt_batch* b, pt_job* job, int mcs, uint32_t flags);
// The same launch with its work list and queue counter in the library's
// static per-device scratch instead of batch-owned device memory (no device
// allocation); *nitems receives the work items of the launch.  PT_EINVAL when
// they exceed PT_NOALLOC_MAX_ITEMS.
int batch_run_job_noalloc(pt_job* job, int mcs, uint32_t flags, int* nitems);
// The launch arguments of job j for `mcs` fused steps in plan `mode` (as
// job_plan_mode returns it) with pt_mcs flags `flags`.
ptsg::FusedArgs job_fused_args(const pt_job* j, int mode, int mcs, uint32_t flags);
// Threads per workgroup and workgroups per CU of a persistent launch of the
// batch kernel (d, feat) with lds_bytes of LDS per workgroup over nitems items
// on ncu CUs; cfg_threads > 0 fixes the workgroup size.  PT_EINVAL if no
// workgroup fits.
int launch_shape(int d, int feat, size_t lds_bytes, int nitems, int ncu, int cfg_threads,
                 int* threads, int* per_cu);
// Enqueues launch(ctx) on st ordered after every earlier launch holding split
// samples on this device (see pt_batch_run), and creates the device's ordering
// event ahead of time.
hipError_t split_ordered(hipStream_t st, hipError_t (*launch)(void*), void* ctx);
hipError_t split_order_prepare();
// Whether job j can run `flags` fused (some workgroup plan fits).
bool job_is_resident(const pt_job* j, uint32_t flags);
// The fused plan a job alone takes for `flags` (as pt_get_plan), -1 if none.
int job_plan_mode(const pt_job* j, uint32_t flags);
// Work items one step of the job makes for `flags`, and attempted flips per
// step of its largest item.
void job_items(const pt_job* j, uint32_t flags, int& items, double& item_flips);
// Compute units of the batch's device (workgroup slots of a one-per-CU plan).
int batch_slots(const pt_batch* b);
// Whether a job of this shape needs the split-sample scratch (its two
// replica sets do not fit one workgroup together, but a split plan exists),
// and how many bytes that scratch takes.
size_t split_scratch_bytes(const ptsg::Geo& g, bool walk = false, bool modes = false);
// Device bytes a job of this shape allocates (an upper bound); `flags` as
// pt_init_ex's (a layout, optionally with PT_TRACK_WALK / PT_TRACK_MODES).
size_t job_device_bytes(int S, int NT, int L, int d, int flags, const double* betas);
// Length of a row of the exchange threshold table.
int pt_table_len(const double* betas, int NT, int d, long N);
// pt_init_ex with explicit allocation hooks (NULL: hipMalloc / hipFree).
// With `stage` set, the host data of the set-up (couplings, tables, maps) is
// first copied to host memory from stage(bytes, ctx), which must be pinned and
// stay unchanged until the work queued on `stream` is done, and the function
// returns once that work is queued: the caller orders every later use of the
// job after it (an event on `stream`).  Without it, it returns after the
// set-up has completed.
int job_create(pt_job** out, int32_t samples, int32_t replicas, int32_t L, int32_t dim,
               const int8_t* couplings, const double* betas, uint64_t seed, uint32_t flags,
               void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx,
               hipStream_t stream, void* (*stage)(size_t, void*) = nullptr);
