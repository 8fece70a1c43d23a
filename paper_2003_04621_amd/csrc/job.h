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
  // fused-step LDS plans: both sets without / with Houdayer, one set
  ptsg::FusedLayout plan[3];
  bool fused_ok[3] = {false, false, false};
  bool poisoned = false;
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
// Whether job j can run `flags` fused with at least one replica set resident.
bool job_is_resident(const pt_job* j, uint32_t flags);
// Device bytes a job of this shape allocates (an upper bound).
size_t job_device_bytes(int S, int NT, int L, int d, int layout, const double* betas);
// Length of a row of the exchange threshold table.
int pt_table_len(const double* betas, int NT, int d, long N);
// pt_init_ex with explicit allocation hooks (NULL: hipMalloc / hipFree).
int job_create(pt_job** out, int32_t samples, int32_t replicas, int32_t L, int32_t dim,
               const int8_t* couplings, const double* betas, uint64_t seed, uint32_t flags,
               void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx,
               hipStream_t stream);
