// runtime.hip -- the C ABI declared in include/pt.h: job state, argument
// validation, host-built acceptance tables, device memory and the
// sequencing of the kernels on the job's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gauss.h"
#include "gauss_kernels.h"
#include "job.h"
#include "kernels.h"
#include "multicluster.h"
#include "pt.h"

using namespace ptsg;

namespace {
thread_local std::string g_err;
}  // namespace

int pt_fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
const char* pt_error_text() { return g_err.c_str(); }

namespace {

void* (*g_alloc)(size_t, void*) = nullptr;
void (*g_free)(void*, void*) = nullptr;
void* g_ctx = nullptr;

// Acceptance probability p -> 32-bit threshold floor(2^32 p), clamped to
// [0, 2^32 - 1]; a uniform 32-bit word r accepts iff r < threshold.
uint32_t threshold_u32(double p) {
  const double v = std::floor(std::ldexp(p, 32));
  if (v >= 4294967295.0) return 0xFFFFFFFFu;
  if (v <= 0.0) return 0u;
  return (uint32_t)v;
}


// Lattice and word geometry of a job (Sec. 2.2 layout).
Geo make_geo(int S, int NT, int L, int dim, int layout, uint64_t seed) {
  Geo g = geo_shape(L, dim);
  g.S = S;
  g.NT = NT;
  g.nslot = 2 * NT;
  g.layout = layout;
  g.key0 = (uint32_t)seed;
  g.key1 = (uint32_t)(seed >> 32);
  return g;
}

}  // namespace


namespace {

// The LDS plans of a job of geometry job->g (host only).
void plan_job(pt_job* job) {
  const Geo& g = job->g;
  const bool w = job->track_walk, md = job->track_modes;
  job->fused_ok[0] = fused_plan(g, false, 2, 16, job->plan[0], w, md);
  job->fused_ok[1] = fused_plan(g, true, 2, 16, job->plan[1], w, md);
  job->fused_ok[2] = fused_plan(g, false, 1, 16, job->plan[2], w, md);
  job->fused_ok[4] = fused_plan(g, true, 2, 16, job->plan[4], w, md, true);
  job->split_ok = !job->fused_ok[0] && split_plan(g, job->split_lay, job->split_parts,
                                                   job->split_R, job->split_jlds, w, md);
}

// pt_get_plan's report for a planned job.
void plan_report(const pt_job* job, uint32_t flags, int32_t* out4) {
  const Geo& g = job->g;
  if (job->gauss) {
    // fused: one workgroup per sample (gauss_fused.hip); else per-step kernels
    const bool fused = !(flags & (PT_MCS_PLAIN | PT_MCS_MULTICLUSTER)) &&
                       gauss_fused_lds(g) <= kGaussFusedMaxLds;
    out4[0] = fused ? 0 : -1;
    out4[1] = fused ? 1 : 0;
    out4[2] = fused ? g.nslot : 0;
    out4[3] = fused ? (int32_t)gauss_fused_lds(g) : 0;
    return;
  }
  const int mode = (flags & PT_MCS_PLAIN) ? -1 : job_plan_mode(job, flags);
  out4[0] = mode == 4 ? 1 : mode;  // the multi-cluster plan is reported as mode 1
  if (mode < 0) {
    out4[1] = out4[2] = out4[3] = 0;
  } else if (mode == 3) {
    out4[1] = job->split_parts;
    out4[2] = job->split_R;
    out4[3] = 4 * job->split_lay.words;
  } else {
    out4[1] = mode == 2 ? 2 : 1;
    out4[2] = mode == 2 ? g.NT : g.nslot;
    out4[3] = 4 * job->plan[mode].words;
  }
}

int device_error(pt_job* job, hipError_t e, const char* where) {
  if (job) job->poisoned = true;
  return pt_fail(PT_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define PT_HIP(job, expr)                                      \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return device_error(job, e_, #expr); \
  } while (0)

int check_job(pt_job* job) {
  if (!job) return pt_fail(PT_EINVAL, "null job handle");
  if (job->poisoned) return pt_fail(PT_ESTATE, "job is poisoned by an earlier device error");
  return PT_OK;
}

// Waits for the job's stream and fails if a split sample's barrier gave up
// (the job's state is then unusable).
int check_fault(pt_job* job) {
  if (!job->bar) return PT_OK;
  uint32_t fault = 0;
  hipError_t e = hipMemcpyAsync(&fault, job->bar + job->g.S, sizeof(fault), hipMemcpyDeviceToHost,
                                job->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(job->stream);
  if (e != hipSuccess) return device_error(job, e, "pt_get_*");
  if (fault) {
    job->poisoned = true;
    return pt_fail(PT_EDEVICE, "a split sample's workgroups lost contact (barrier timed out)");
  }
  return PT_OK;
}

// Row of field f of word w (host copy of the device word geometry).
int host_word_row(const Geo& g, int w, int f) {
  if (g.d == 3) {
    const int xs = w / g.L, x1 = w % g.L;
    return x1 + g.L * (f * g.B + xs);
  }
  return f * g.B + w;
}

// int8 lattices <-> colour words (pt_get_spins / pt_set_spins, packed layout)
void pack_host(const Geo& g, const int8_t* in, uint32_t* out) {
  const size_t nlat = (size_t)g.S * g.nslot;
  for (size_t lat = 0; lat < nlat; ++lat) {
    const int8_t* s = in + lat * g.N;
    uint32_t* W = out + lat * 2 * g.NW;
    for (int w = 0; w < g.NW; ++w) {
      uint32_t c01[2] = {0, 0};
      for (int f = 0; f < g.P; ++f) {
        const int R = host_word_row(g, w, f);
        const int x1 = R % g.L, x2 = R / g.L;
        for (int x0 = 0; x0 < g.L; ++x0) {
          const int c = (x0 + x1 + x2) & 1;
          if (s[(size_t)R * g.L + x0] < 0) c01[c] |= 1u << (f * g.H + (x0 >> 1));
        }
      }
      W[w] = c01[0];
      W[g.NW + w] = c01[1];
    }
  }
}

void unpack_host(const Geo& g, const uint32_t* in, int8_t* out) {
  const size_t nlat = (size_t)g.S * g.nslot;
  for (size_t lat = 0; lat < nlat; ++lat) {
    int8_t* s = out + lat * g.N;
    const uint32_t* W = in + lat * 2 * g.NW;
    for (int w = 0; w < g.NW; ++w)
      for (int f = 0; f < g.P; ++f) {
        const int R = host_word_row(g, w, f);
        const int x1 = R % g.L, x2 = R / g.L;
        for (int x0 = 0; x0 < g.L; ++x0) {
          const int c = (x0 + x1 + x2) & 1;
          const uint32_t bit = (W[c * g.NW + w] >> (f * g.H + (x0 >> 1))) & 1u;
          s[(size_t)R * g.L + x0] = bit ? (int8_t)-1 : (int8_t)1;
        }
      }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
PT_API const char* pt_last_error(void) { return pt_error_text(); }
PT_API const char* pt_version(void) { return "ptsg-gfx950 0.1"; }

PT_API int pt_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx) {
  if ((alloc == nullptr) != (free_ == nullptr))
    return pt_fail(PT_EINVAL, "allocator and free hooks must both be set or both be NULL");
  g_alloc = alloc;
  g_free = free_;
  g_ctx = ctx;
  return PT_OK;
}

int job_create(pt_job** out, int32_t samples, int32_t replicas, int32_t L, int32_t dim,
               const int8_t* couplings, const double* betas, uint64_t seed, uint32_t flags,
               void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx,
               hipStream_t stream, void* (*stage)(size_t, void*)) {
  g_err.clear();
  if (!out || !couplings || !betas) return pt_fail(PT_EINVAL, "null pointer argument");
  if (dim != 2 && dim != 3) return pt_fail(PT_EINVAL, "dim must be 2 or 3");
  if (L < 4 || L > 64 || (L & 1)) return pt_fail(PT_EINVAL, "L must be even and in [4, 64]");
  if (samples < 1 || samples >= (1 << 28)) return pt_fail(PT_EINVAL, "samples must be in [1, 2^28)");
  if (replicas < 2 || replicas > 4096) return pt_fail(PT_EINVAL, "replicas must be in [2, 4096]");
  const uint32_t layout = flags & ~(uint32_t)(PT_TRACK_WALK | PT_TRACK_MODES | PT_TRACK_STATS);
  if (layout != PT_LAYOUT_INT8 && layout != PT_LAYOUT_PACKED) return pt_fail(PT_EINVAL, "unknown flags");
  for (int k = 0; k < replicas; ++k) {
    if (!std::isfinite(betas[k]) || !(betas[k] > 0.0))
      return pt_fail(PT_EINVAL, "betas must be finite and > 0");
    if (k > 0 && !(betas[k] < betas[k - 1]))
      return pt_fail(PT_EINVAL, "betas must be strictly decreasing (index 0 = coldest)");
  }
  const long N = (dim == 3) ? (long)L * L * L : (long)L * L;
  const long ncoup = (long)samples * dim * N;
  for (long i = 0; i < ncoup; ++i)
    if (couplings[i] != 1 && couplings[i] != -1) return pt_fail(PT_EINVAL, "couplings must be +1 or -1");
  const long nlat = (long)samples * 2 * replicas;
  if (nlat > 0x7FFFFFFFL || (long)samples * replicas > 0x7FFFFFFFL)
    return pt_fail(PT_EINVAL, "too many lattices for one job");

  pt_job* job = new (std::nothrow) pt_job();
  if (!job) return pt_fail(PT_ENOMEM, "host allocation failed");
  job->alloc_fn = alloc;
  job->free_fn = free_;
  job->alloc_ctx = ctx;
  job->stream = stream;
  job->track_walk = (flags & PT_TRACK_WALK) != 0;
  job->track_modes = (flags & PT_TRACK_MODES) != 0;
  job->track_stats = (flags & PT_TRACK_STATS) != 0;
  job->g = make_geo(samples, replicas, L, dim, (int)layout, seed);
  const Geo& g = job->g;

  // Metropolis thresholds: x = 2m (m = 1..d), energy change 4m.
  std::vector<uint32_t> thr((size_t)replicas * 4, 0u);
  for (int k = 0; k < replicas; ++k)
    for (int m = 1; m <= dim; ++m) {
      const double dE = (double)(4 * m);
      thr[(size_t)k * 4 + (m - 1)] = threshold_u32(std::exp(-(betas[k] * dE)));
    }
  // Exchange thresholds: D = 2m, row length M = first m where every row is 0.
  const int M = pt_table_len(betas, replicas, dim, N);
  std::vector<uint32_t> thrpt((size_t)(replicas - 1) * M, 0u);
  for (int k = 0; k + 1 < replicas; ++k) {
    const double db = betas[k] - betas[k + 1];
    thrpt[(size_t)k * M] = 0xFFFFFFFFu;
    for (int m = 1; m < M; ++m)
      thrpt[(size_t)k * M + m] = threshold_u32(std::exp(-(db * (double)(2 * m))));
  }
  job->M = M;
  plan_job(job);

  const size_t maps = sizeof(int32_t) * (size_t)samples * 2 * replicas;
  job->spins = job->dalloc(job->spin_bytes());
  job->jw = (uint32_t*)job->dalloc(sizeof(uint32_t) * (size_t)samples * 2 * 2 * dim * g.NW);
  job->E = (int32_t*)job->dalloc(sizeof(int32_t) * (size_t)nlat);
  job->sot = (int32_t*)job->dalloc(maps);
  job->tos = (int32_t*)job->dalloc(maps);
  job->thr = (uint32_t*)job->dalloc(sizeof(uint32_t) * thr.size());
  job->thrpt = (uint32_t*)job->dalloc(sizeof(uint32_t) * thrpt.size());
  job->ctr = (DevCounters*)job->dalloc(sizeof(DevCounters));
  job->mom = (int64_t*)job->dalloc(sizeof(int64_t) * 8 * (size_t)samples * replicas);
  if (job->track_walk) {
    job->walk = (int32_t*)job->dalloc(sizeof(int32_t) * 2 * (size_t)nlat);
    job->trips = (uint64_t*)job->dalloc(sizeof(uint64_t) * 32 * 3 * (size_t)samples);
  }
  const size_t mode_words = (size_t)samples * replicas * (L / 2 + 1);
  if (job->track_modes) job->modes = (int64_t*)job->dalloc(sizeof(int64_t) * mode_words);
  const size_t stat_words = (size_t)samples * replicas * kNStat;
  if (job->track_stats) job->stats = (int64_t*)job->dalloc(sizeof(int64_t) * stat_words);
  int8_t* J8 = (int8_t*)job->dalloc((size_t)ncoup);
  bool split_mem = true;
  if (job->split_ok) {
    const size_t W2 = 2 * (size_t)g.NW, per = (size_t)samples * 2 * g.nslot;
    job->Ex = (int32_t*)job->dalloc(sizeof(int32_t) * per);
    job->snap = (uint32_t*)job->dalloc(sizeof(uint32_t) * per * W2);
    job->bar = (uint32_t*)job->dalloc(sizeof(uint32_t) * ((size_t)samples + 1));
    split_mem = job->Ex && job->snap && job->bar;
  }
  if (!job->spins || !job->jw || !job->E || !job->sot || !job->tos || !job->thr || !job->thrpt ||
      !job->ctr || !job->mom || !J8 || !split_mem ||
      (job->track_walk && (!job->walk || !job->trips)) || (job->track_modes && !job->modes) ||
      (job->track_stats && !job->stats)) {
    job->release();
    delete job;
    return pt_fail(PT_ENOMEM, "device allocation failed");
  }
  std::vector<int32_t> ident((size_t)samples * 2 * replicas);
  for (size_t i = 0; i < ident.size(); ++i) ident[i] = (int32_t)(i % replicas);

  hipStream_t st = job->stream;
  hipError_t e = hipSuccess;
  auto step = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
  };
  // the copies' sources: the caller's and these vectors (the call then waits
  // for the set-up below), or pinned staging copies of them
  const void* src_J = couplings;
  const void* src_thr = thr.data();
  const void* src_thrpt = thrpt.data();
  const void* src_ident = ident.data();
  if (stage) {
    auto put = [&](const void* from, size_t bytes) -> const void* {
      void* to = stage(bytes, ctx);
      if (to) std::memcpy(to, from, bytes);
      return to;
    };
    src_J = put(couplings, (size_t)ncoup);
    src_thr = put(thr.data(), sizeof(uint32_t) * thr.size());
    src_thrpt = put(thrpt.data(), sizeof(uint32_t) * thrpt.size());
    src_ident = put(ident.data(), maps);
    if (!src_J || !src_thr || !src_thrpt || !src_ident) {
      job->release();
      delete job;
      return pt_fail(PT_ENOMEM, "pinned staging allocation failed");
    }
  }
  step(hipMemcpyAsync(J8, src_J, (size_t)ncoup, hipMemcpyHostToDevice, st));
  step(hipMemcpyAsync(job->thr, src_thr, sizeof(uint32_t) * thr.size(), hipMemcpyHostToDevice, st));
  step(hipMemcpyAsync(job->thrpt, src_thrpt, sizeof(uint32_t) * thrpt.size(), hipMemcpyHostToDevice,
                      st));
  step(hipMemcpyAsync(job->sot, src_ident, maps, hipMemcpyHostToDevice, st));
  step(hipMemcpyAsync(job->tos, src_ident, maps, hipMemcpyHostToDevice, st));
  step(hipMemsetAsync(job->ctr, 0, sizeof(DevCounters), st));
  step(hipMemsetAsync(job->mom, 0, sizeof(int64_t) * 8 * (size_t)samples * replicas, st));
  if (job->track_modes) step(hipMemsetAsync(job->modes, 0, sizeof(int64_t) * mode_words, st));
  if (job->track_stats) step(hipMemsetAsync(job->stats, 0, sizeof(int64_t) * stat_words, st));
  if (job->track_walk) {
    step(hipMemsetAsync(job->walk, 0, sizeof(int32_t) * 2 * (size_t)nlat, st));
    step(hipMemsetAsync(job->trips, 0, sizeof(uint64_t) * 32 * 3 * (size_t)samples, st));
  }
  if (job->bar) step(hipMemsetAsync(job->bar, 0, sizeof(uint32_t) * ((size_t)samples + 1), st));
  step(launch_pack_couplings(g, J8, job->jw, st));
  step(launch_init_spins(g, job->spins, st));
  step(launch_energy(g, job->spins, job->jw, job->E, st));
  if (!stage) step(hipStreamSynchronize(st));
  if (e != hipSuccess) {
    std::string msg = std::string("pt_init: ") + hipGetErrorString(e);
    job->release();
    delete job;
    return pt_fail(PT_EDEVICE, msg);
  }
  *out = job;
  return PT_OK;
}

PT_API int pt_init_ex(pt_job** out, int32_t samples, int32_t replicas, int32_t L, int32_t dim,
                      const int8_t* couplings, const double* betas, uint64_t seed, uint32_t flags) {
  return job_create(out, samples, replicas, L, dim, couplings, betas, seed, flags, g_alloc, g_free,
                    g_ctx, nullptr);
}

// A job with Gaussian couplings: float32 couplings on the 2^-16 grid (|J| <= 8)
// held as integer units; spins as pt_init_ex's layouts; no replica walk or
// modes.  The steps run as separate kernels on the job's stream.
PT_API int pt_init_gauss(pt_job** out, int32_t samples, int32_t replicas, int32_t L, int32_t dim,
                         const float* couplings, const double* betas, uint64_t seed, uint32_t flags) {
  g_err.clear();
  if (!out || !couplings || !betas) return pt_fail(PT_EINVAL, "null pointer argument");
  if (dim != 2 && dim != 3) return pt_fail(PT_EINVAL, "dim must be 2 or 3");
  if (L < 4 || L > 64 || (L & 1)) return pt_fail(PT_EINVAL, "L must be even and in [4, 64]");
  if (samples < 1 || samples >= (1 << 28)) return pt_fail(PT_EINVAL, "samples must be in [1, 2^28)");
  if (replicas < 2 || replicas > 4096) return pt_fail(PT_EINVAL, "replicas must be in [2, 4096]");
  if (flags != PT_LAYOUT_INT8 && flags != PT_LAYOUT_PACKED)
    return pt_fail(PT_EINVAL, "flags: a layout only (Gaussian jobs keep no replica walk or modes)");
  for (int k = 0; k < replicas; ++k) {
    if (!std::isfinite(betas[k]) || !(betas[k] > 0.0))
      return pt_fail(PT_EINVAL, "betas must be finite and > 0");
    if (k > 0 && !(betas[k] < betas[k - 1]))
      return pt_fail(PT_EINVAL, "betas must be strictly decreasing (index 0 = coldest)");
  }
  const long N = (dim == 3) ? (long)L * L * L : (long)L * L;
  const long ncoup = (long)samples * dim * N;
  const long nlat = (long)samples * 2 * replicas;
  if (nlat > 0x7FFFFFFFL || (long)samples * replicas > 0x7FFFFFFFL)
    return pt_fail(PT_EINVAL, "too many lattices for one job");
  std::vector<int32_t> units((size_t)ncoup);
  for (long i = 0; i < ncoup; ++i) {
    const float J = couplings[i];
    const double n = (double)J * 65536.0;  // exact: a power-of-two scale of a float
    if (!std::isfinite(J) || n != std::floor(n) || n > (double)kGaussMaxUnits ||
        n < -(double)kGaussMaxUnits)
      return pt_fail(PT_EINVAL, "Gaussian couplings must be multiples of 2^-16 in [-8, 8]");
    units[(size_t)i] = (int32_t)n;
  }

  pt_job* job = new (std::nothrow) pt_job();
  if (!job) return pt_fail(PT_ENOMEM, "host allocation failed");
  job->alloc_fn = g_alloc;
  job->free_fn = g_free;
  job->alloc_ctx = g_ctx;
  job->gauss = true;
  job->g = make_geo(samples, replicas, L, dim, (int)flags, seed);
  const Geo& g = job->g;
  const size_t maps = sizeof(int32_t) * (size_t)samples * 2 * replicas;
  const size_t ngrp = (size_t)samples * 2 * (2 * dim + 1) * gauss_groups(g);
  job->spins = job->dalloc(job->spin_bytes());
  job->gJn = (int32_t*)job->dalloc(sizeof(int32_t) * (size_t)ncoup);
  job->gJ = (int4*)job->dalloc(sizeof(int4) * ngrp);
  job->E64 = (int64_t*)job->dalloc(sizeof(int64_t) * (size_t)nlat);
  job->sot = (int32_t*)job->dalloc(maps);
  job->tos = (int32_t*)job->dalloc(maps);
  job->gbeta = (double*)job->dalloc(sizeof(double) * replicas);
  job->gcz = (float*)job->dalloc(sizeof(float) * replicas);
  job->ctr = (DevCounters*)job->dalloc(sizeof(DevCounters));
  job->mom = (int64_t*)job->dalloc(sizeof(int64_t) * 8 * (size_t)samples * replicas);
  if (!job->spins || !job->gJn || !job->gJ || !job->E64 || !job->sot || !job->tos || !job->gbeta ||
      !job->gcz || !job->ctr || !job->mom) {
    job->release();
    delete job;
    return pt_fail(PT_ENOMEM, "device allocation failed");
  }
  std::vector<int32_t> ident((size_t)samples * 2 * replicas);
  for (size_t i = 0; i < ident.size(); ++i) ident[i] = (int32_t)(i % replicas);
  std::vector<float> cz((size_t)replicas);
  for (int k = 0; k < replicas; ++k) cz[(size_t)k] = gauss_cz(betas[k]);
  hipStream_t st = job->stream;
  hipError_t e = hipSuccess;
  auto step = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
  };
  step(hipMemcpyAsync(job->gJn, units.data(), sizeof(int32_t) * units.size(), hipMemcpyHostToDevice, st));
  step(hipMemcpyAsync(job->gbeta, betas, sizeof(double) * replicas, hipMemcpyHostToDevice, st));
  step(hipMemcpyAsync(job->gcz, cz.data(), sizeof(float) * replicas, hipMemcpyHostToDevice, st));
  step(hipMemcpyAsync(job->sot, ident.data(), maps, hipMemcpyHostToDevice, st));
  step(hipMemcpyAsync(job->tos, ident.data(), maps, hipMemcpyHostToDevice, st));
  step(hipMemsetAsync(job->ctr, 0, sizeof(DevCounters), st));
  step(hipMemsetAsync(job->mom, 0, sizeof(int64_t) * 8 * (size_t)samples * replicas, st));
  step(launch_gauss_prepare(g, job->gJn, job->gJ, st));
  step(launch_init_spins(g, job->spins, st));
  step(launch_gauss_energy(g, job->spins, job->gJ, job->E64, st));
  step(hipStreamSynchronize(st));
  if (e != hipSuccess) {
    std::string msg = std::string("pt_init_gauss: ") + hipGetErrorString(e);
    job->release();
    delete job;
    return pt_fail(PT_EDEVICE, msg);
  }
  *out = job;
  return PT_OK;
}

bool job_is_resident(const pt_job* j, uint32_t flags) {
  return !j->track_stats && job_plan_mode(j, flags) >= 0;
}

int pt_table_len(const double* betas, int NT, int d, long N) {
  int M = 1;
  const long mmax = (long)d * N;
  for (int k = 0; k + 1 < NT; ++k) {
    const double db = betas[k] - betas[k + 1];
    long m = 1;
    while (m <= mmax && threshold_u32(std::exp(-(db * (double)(2 * m)))) != 0u) ++m;
    if (m > M) M = (int)m;
  }
  return M;
}

size_t split_scratch_bytes(const Geo& g, bool walk, bool modes) {
  FusedLayout lay;
  int parts, R, jlds;
  if (fused_plan(g, false, 2, 16, lay, walk, modes) || !split_plan(g, lay, parts, R, jlds, walk, modes))
    return 0;
  const size_t per = (size_t)g.S * 2 * g.nslot;
  return sizeof(int32_t) * per + sizeof(uint32_t) * per * 2 * g.NW + sizeof(uint32_t) * (g.S + 1);
}

size_t job_device_bytes(int S, int NT, int L, int d, int flags, const double* betas) {
  const int layout = flags & ~(int)(PT_TRACK_WALK | PT_TRACK_MODES | PT_TRACK_STATS);
  const bool walk = (flags & PT_TRACK_WALK) != 0, modes = (flags & PT_TRACK_MODES) != 0;
  const bool stats = (flags & PT_TRACK_STATS) != 0;
  const size_t N = (d == 3) ? (size_t)L * L * L : (size_t)L * L;
  const size_t NW = N / L / fields_per_word(L);
  const size_t lat = (size_t)S * 2 * NT;
  const size_t spins = layout == PT_LAYOUT_PACKED ? lat * 2 * NW * 4 : lat * N;
  const size_t jw = (size_t)S * 2 * 2 * d * NW * 4;
  const size_t small = sizeof(int32_t) * (lat + 4 * (size_t)S * NT) + sizeof(int64_t) * 8 * S * NT +
                       (walk ? sizeof(int32_t) * 2 * lat + sizeof(uint64_t) * 32 * 3 * (size_t)S : 0) +
                       (modes ? sizeof(int64_t) * (size_t)S * NT * (L / 2 + 1) : 0) +
                       (stats ? sizeof(int64_t) * (size_t)S * NT * kNStat : 0) +
                       sizeof(uint32_t) * (size_t)NT * (4 + pt_table_len(betas, NT, d, (long)N)) + 4096;
  return spins + jw + (size_t)S * d * N + small + split_scratch_bytes(make_geo(S, NT, L, d, layout, 0), walk, modes);
}

PT_API int pt_init(pt_job** out, int32_t samples, int32_t replicas, int32_t L, int32_t dim,
                   const int8_t* couplings, const double* betas, uint64_t seed) {
  return pt_init_ex(out, samples, replicas, L, dim, couplings, betas, seed, PT_LAYOUT_INT8);
}

PT_API int pt_destroy(pt_job* job) {
  if (!job) return pt_fail(PT_EINVAL, "null job handle");
  (void)hipStreamSynchronize(job->stream);
  (void)hipGetLastError();
  if (job->self_batch) batch_free(job->self_batch);
  job->release();
  delete job;
  return PT_OK;
}

PT_API int pt_set_measure_interval(pt_job* job, int32_t every) {
  if (int rc = check_job(job)) return rc;
  if (every < 1) return pt_fail(PT_EINVAL, "the measurement interval must be >= 1");
  job->meas_every = every;  // batches rebuild their work lists when it changes
  return PT_OK;
}

PT_API int pt_set_stream(pt_job* job, void* hip_stream) {
  if (int rc = check_job(job)) return rc;
  job->stream = (hipStream_t)hip_stream;
  return PT_OK;
}

// ---------------------------------------------------------------------------
// asynchronous steps
// ---------------------------------------------------------------------------
PT_API int pt_sweep(pt_job* job, int32_t n) {
  if (int rc = check_job(job)) return rc;
  if (n < 0) return pt_fail(PT_EINVAL, "n must be >= 0");
  const int chunk = 1000;
  for (int done = 0; done < n; done += chunk) {
    const int m = (n - done) < chunk ? (n - done) : chunk;
    if (job->gauss)
      PT_HIP(job, launch_gauss_sweep(job->g, job->spins, job->gJ, job->E64, job->tos, job->gbeta,
                                     job->gcz, job->ctr, m, job->stream));
    else
      PT_HIP(job, launch_sweep(job->g, job->spins, job->jw, job->E, job->tos, job->thr, job->ctr, m,
                               job->stats, job->stream));
    PT_HIP(job, launch_advance(job->ctr, CounterStep{(uint32_t)m, 0, 0, 0}, job->stream));
  }
  return PT_OK;
}

PT_API int pt_exchange(pt_job* job) {
  if (int rc = check_job(job)) return rc;
  if (job->gauss)
    PT_HIP(job, launch_gauss_exchange(job->g, job->E64, job->sot, job->tos, job->gbeta, job->ctr,
                                      job->stream));
  else
    PT_HIP(job, launch_exchange(job->g, job->E, job->sot, job->tos, job->thrpt, job->M, job->walk,
                                job->trips, job->ctr, job->stats, job->stream));
  PT_HIP(job, launch_advance(job->ctr, CounterStep{0, 1, 0, 0}, job->stream));
  return PT_OK;
}

PT_API int pt_houdayer(pt_job* job) {
  if (int rc = check_job(job)) return rc;
  if (job->gauss)
    PT_HIP(job, launch_gauss_houdayer(job->g, job->spins, job->gJ, job->E64, job->sot, job->ctr, false,
                                      job->stream));
  else
    PT_HIP(job, launch_houdayer(job->g, job->spins, job->jw, job->E, job->sot, job->ctr, job->stats,
                                job->stream));
  PT_HIP(job, launch_advance(job->ctr, CounterStep{0, 0, 1, 0}, job->stream));
  return PT_OK;
}

PT_API int pt_houdayer_multi(pt_job* job) {
  if (int rc = check_job(job)) return rc;
  if (job->g.N > kMultiMaxSites)
    return pt_fail(PT_EINVAL, "multi-cluster moves need L^dim <= " + std::to_string(kMultiMaxSites));
  if (job->gauss)
    PT_HIP(job, launch_gauss_houdayer(job->g, job->spins, job->gJ, job->E64, job->sot, job->ctr, true,
                                      job->stream));
  else
    PT_HIP(job, launch_houdayer_multi(job->g, job->spins, job->jw, job->E, job->sot, job->ctr,
                                      job->stats, job->stream));
  PT_HIP(job, launch_advance(job->ctr, CounterStep{0, 0, 1, 0}, job->stream));
  return PT_OK;
}

PT_API int pt_measure(pt_job* job) {
  if (int rc = check_job(job)) return rc;
  if (job->gauss)
    PT_HIP(job, launch_gauss_measure(job->g, job->spins, job->E64, job->sot, job->mom, job->ctr, 1,
                                     job->stream));
  else
    PT_HIP(job, launch_measure(job->g, job->spins, job->E, job->sot, job->mom, job->modes, job->ctr, 1,
                             job->stream));
  PT_HIP(job, launch_advance(job->ctr, CounterStep{0, 0, 0, 1}, job->stream));
  return PT_OK;
}

namespace {
// Argument checks of pt_mcs.
int check_mcs(pt_job* job, int32_t n, uint32_t flags) {
  if (int rc = check_job(job)) return rc;
  if (n < 0) return pt_fail(PT_EINVAL, "n must be >= 0");
  if (flags & ~(uint32_t)(PT_MCS_HOUDAYER | PT_MCS_MEASURE | PT_MCS_PLAIN | PT_MCS_MULTICLUSTER))
    return pt_fail(PT_EINVAL, "unknown flags");
  if ((flags & PT_MCS_MULTICLUSTER) && !(flags & PT_MCS_HOUDAYER))
    return pt_fail(PT_EINVAL, "PT_MCS_MULTICLUSTER needs PT_MCS_HOUDAYER");
  if ((flags & PT_MCS_MULTICLUSTER) && job->g.N > kMultiMaxSites)
    return pt_fail(PT_EINVAL, "multi-cluster moves need L^dim <= " + std::to_string(kMultiMaxSites));
  return PT_OK;
}

// n Monte Carlo steps as separate kernels, one launch per step and kernel
// (no scratch, no allocation).  Within one step every counter is read by
// exactly one kernel, so a single advance per step keeps the numbering of
// the separate entry points.
int mcs_per_step(pt_job* job, int32_t n, uint32_t flags) {
  const Geo& g = job->g;
  hipStream_t st = job->stream;
  const bool hou = flags & PT_MCS_HOUDAYER, meas = flags & PT_MCS_MEASURE;
  const bool multi = flags & PT_MCS_MULTICLUSTER;
  const CounterStep adv{1, 1, hou ? 1u : 0u, meas ? 1u : 0u, (uint32_t)job->meas_every};
  for (int i = 0; i < n; ++i) {
    if (job->gauss) {
      PT_HIP(job, launch_gauss_sweep(g, job->spins, job->gJ, job->E64, job->tos, job->gbeta, job->gcz,
                                     job->ctr, 1, st));
      if (hou)
        PT_HIP(job, launch_gauss_houdayer(g, job->spins, job->gJ, job->E64, job->sot, job->ctr, multi, st));
      PT_HIP(job, launch_gauss_exchange(g, job->E64, job->sot, job->tos, job->gbeta, job->ctr, st));
      if (meas)
        PT_HIP(job, launch_gauss_measure(g, job->spins, job->E64, job->sot, job->mom, job->ctr,
                                         job->meas_every, st));
    } else {
      PT_HIP(job, launch_sweep(g, job->spins, job->jw, job->E, job->tos, job->thr, job->ctr, 1, job->stats, st));
      if (hou && multi)
        PT_HIP(job, launch_houdayer_multi(g, job->spins, job->jw, job->E, job->sot, job->ctr, job->stats, st));
      else if (hou)
        PT_HIP(job, launch_houdayer(g, job->spins, job->jw, job->E, job->sot, job->ctr, job->stats, st));
      PT_HIP(job, launch_exchange(g, job->E, job->sot, job->tos, job->thrpt, job->M, job->walk,
                                  job->trips, job->ctr, job->stats, st));
      if (meas)
        PT_HIP(job, launch_measure(g, job->spins, job->E, job->sot, job->mom, job->modes, job->ctr,
                                   job->meas_every, st));
    }
    PT_HIP(job, launch_advance(job->ctr, adv, st));
  }
  return PT_OK;
}
// Whether a Gaussian job's steps with these flags run fused (gauss_fused.hip):
// single-cluster Houdayer moves or none, and the sample's configurations fit
// one workgroup's LDS.
bool gauss_fused_ok(const pt_job* job, uint32_t flags) {
  return job->gauss && !(flags & (PT_MCS_PLAIN | PT_MCS_MULTICLUSTER)) &&
         gauss_fused_lds(job->g) <= kGaussFusedMaxLds;
}

// n fused steps of a Gaussian job, in launches of at most 500 steps, each
// followed by the counters' advance (allocates nothing).
int mcs_gauss_fused(pt_job* job, int32_t n, uint32_t flags) {
  const bool hou = flags & PT_MCS_HOUDAYER, meas = flags & PT_MCS_MEASURE;
  const int chunk = 500;
  for (int done = 0; done < n; done += chunk) {
    const uint32_t m = (uint32_t)((n - done) < chunk ? (n - done) : chunk);
    PT_HIP(job, launch_gauss_fused(job->g, job->spins, job->gJ, job->E64, job->sot, job->tos,
                                   job->gbeta, job->gcz, job->mom, job->ctr, (int)m, hou, meas,
                                   job->meas_every, job->stream));
    // n_meas: m measurements at interval 1, else one per multiple of the
    // interval among the m sweep numbers (CounterStep's rule)
    const uint32_t every = (uint32_t)job->meas_every;
    const CounterStep adv{m, m, hou ? m : 0u, meas ? (every > 1u ? 1u : m) : 0u, every};
    PT_HIP(job, launch_advance(job->ctr, adv, job->stream));
  }
  return PT_OK;
}
}  // namespace

PT_API int pt_mcs(pt_job* job, int32_t n, uint32_t flags) {
  if (int rc = check_mcs(job, n, flags)) return rc;
  if (gauss_fused_ok(job, flags)) return mcs_gauss_fused(job, n, flags);
  // fused through the job's one-job batch whenever a workgroup plan exists:
  // both sets per workgroup, one set per workgroup (no overlap needed), or
  // the sample split over several workgroups (no Houdayer move)
  if (!job->gauss && !(flags & PT_MCS_PLAIN) && job_is_resident(job, flags)) {
    if (!job->self_batch) job->self_batch = batch_new(job->stream);
    if (!job->self_batch) return pt_fail(PT_ENOMEM, "pt_mcs: host allocation failed");
    const int chunk = 500;
    for (int done = 0; done < n; done += chunk) {
      const int m = (n - done) < chunk ? (n - done) : chunk;
      const int rc = batch_run_job(job->self_batch, job, m,
                                   flags & (PT_MCS_HOUDAYER | PT_MCS_MEASURE | PT_MCS_MULTICLUSTER));
      if (rc != PT_OK) {
        job->poisoned = rc == PT_EDEVICE;
        return rc;
      }
    }
    return PT_OK;
  }
  return mcs_per_step(job, n, flags);
}

PT_API int pt_mcs_noalloc(pt_job* job, int32_t n, uint32_t flags) {
  if (int rc = check_mcs(job, n, flags)) return rc;
  if (gauss_fused_ok(job, flags)) return mcs_gauss_fused(job, n, flags);
  if (job->gauss || (flags & PT_MCS_PLAIN) || !job_is_resident(job, flags))
    return mcs_per_step(job, n, flags);  // per-step kernels use no scratch
  const int chunk = 500;
  for (int done = 0; done < n; done += chunk) {
    const int m = (n - done) < chunk ? (n - done) : chunk;
    const int rc = batch_run_job_noalloc(job, m, flags & (PT_MCS_HOUDAYER | PT_MCS_MEASURE | PT_MCS_MULTICLUSTER),
                                         nullptr);
    if (rc != PT_OK) {
      job->poisoned = rc == PT_EDEVICE;
      return rc;
    }
  }
  return PT_OK;
}

PT_API int pt_get_plan(pt_job* job, uint32_t flags, int32_t* out4) {
  if (int rc = check_job(job)) return rc;
  if (!out4) return pt_fail(PT_EINVAL, "null output");
  if (flags & ~(uint32_t)(PT_MCS_HOUDAYER | PT_MCS_MEASURE | PT_MCS_PLAIN | PT_MCS_MULTICLUSTER))
    return pt_fail(PT_EINVAL, "unknown flags");
  if ((flags & PT_MCS_MULTICLUSTER) && !(flags & PT_MCS_HOUDAYER))
    return pt_fail(PT_EINVAL, "PT_MCS_MULTICLUSTER needs PT_MCS_HOUDAYER");
  plan_report(job, flags, out4);
  return PT_OK;
}

PT_API int pt_plan_query(int32_t dim, int32_t L, int32_t replicas, uint32_t flags, int32_t* out4) {
  if (!out4) return pt_fail(PT_EINVAL, "null output");
  if (dim != 2 && dim != 3) return pt_fail(PT_EINVAL, "dim must be 2 or 3");
  if (L < 4 || L > 64 || (L & 1)) return pt_fail(PT_EINVAL, "L must be even and in [4, 64]");
  if (replicas < 2) return pt_fail(PT_EINVAL, "replicas must be >= 2");
  const uint32_t track = PT_TRACK_WALK | PT_TRACK_MODES;
  if (flags & ~(uint32_t)(PT_MCS_HOUDAYER | PT_MCS_MEASURE | PT_MCS_PLAIN | PT_MCS_MULTICLUSTER | track))
    return pt_fail(PT_EINVAL, "unknown flags");
  if ((flags & PT_MCS_MULTICLUSTER) && !(flags & PT_MCS_HOUDAYER))
    return pt_fail(PT_EINVAL, "PT_MCS_MULTICLUSTER needs PT_MCS_HOUDAYER");
  pt_job job;
  job.g = make_geo(1, replicas, L, dim, PT_LAYOUT_INT8, 0);
  job.track_walk = (flags & PT_TRACK_WALK) != 0;
  job.track_modes = (flags & PT_TRACK_MODES) != 0;
  plan_job(&job);
  plan_report(&job, flags & ~track, out4);
  return PT_OK;
}

PT_API int pt_job_bytes(int32_t samples, int32_t replicas, int32_t L, int32_t dim, uint32_t layout,
                        const double* betas, uint64_t* out) {
  if (!out || !betas) return pt_fail(PT_EINVAL, "null argument");
  if (dim != 2 && dim != 3) return pt_fail(PT_EINVAL, "dim must be 2 or 3");
  if (L < 4 || L > 64 || (L & 1)) return pt_fail(PT_EINVAL, "L must be even and in [4, 64]");
  if (samples < 1 || replicas < 2) return pt_fail(PT_EINVAL, "need samples >= 1 and replicas >= 2");
  const uint32_t lay = layout & ~(uint32_t)(PT_TRACK_WALK | PT_TRACK_MODES | PT_TRACK_STATS);
  if (lay != PT_LAYOUT_INT8 && lay != PT_LAYOUT_PACKED) return pt_fail(PT_EINVAL, "unknown layout");
  for (int k = 0; k < replicas; ++k)
    if (!(betas[k] > 0.0) || (k > 0 && !(betas[k] < betas[k - 1])))
      return pt_fail(PT_EINVAL, "betas must be > 0 and strictly decreasing");
  *out = (uint64_t)job_device_bytes(samples, replicas, L, dim, (int)layout, betas);
  return PT_OK;
}

// ---------------------------------------------------------------------------
// synchronous state access
// ---------------------------------------------------------------------------
PT_API int pt_get_counters(pt_job* job, uint64_t* out) {
  if (int rc = check_job(job)) return rc;
  if (int rc = check_fault(job)) return rc;
  if (!out) return pt_fail(PT_EINVAL, "null output");
  DevCounters c;
  PT_HIP(job, hipMemcpyAsync(&c, job->ctr, sizeof(c), hipMemcpyDeviceToHost, job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  out[0] = c.t;
  out[1] = c.u;
  out[2] = c.v;
  out[3] = c.n_meas;
  return PT_OK;
}

PT_API int pt_get_spins(pt_job* job, int8_t* out) {
  if (int rc = check_job(job)) return rc;
  if (int rc = check_fault(job)) return rc;
  if (!out) return pt_fail(PT_EINVAL, "null output");
  const Geo& g = job->g;
  if (g.layout == kLayoutPacked) {
    std::vector<uint32_t> tmp(job->spin_bytes() / sizeof(uint32_t));
    PT_HIP(job, hipMemcpyAsync(tmp.data(), job->spins, job->spin_bytes(), hipMemcpyDeviceToHost,
                               job->stream));
    PT_HIP(job, hipStreamSynchronize(job->stream));
    unpack_host(g, tmp.data(), out);
  } else {
    PT_HIP(job, hipMemcpyAsync(out, job->spins, job->spin_bytes(), hipMemcpyDeviceToHost, job->stream));
    PT_HIP(job, hipStreamSynchronize(job->stream));
  }
  return PT_OK;
}

PT_API int pt_set_spins(pt_job* job, const int8_t* in) {
  if (int rc = check_job(job)) return rc;
  if (!in) return pt_fail(PT_EINVAL, "null input");
  const Geo& g = job->g;
  const size_t n = (size_t)g.S * g.nslot * g.N;
  for (size_t i = 0; i < n; ++i)
    if (in[i] != 1 && in[i] != -1) return pt_fail(PT_EINVAL, "spins must be +1 or -1");
  if (g.layout == kLayoutPacked) {
    std::vector<uint32_t> tmp(job->spin_bytes() / sizeof(uint32_t));
    pack_host(g, in, tmp.data());
    PT_HIP(job, hipMemcpyAsync(job->spins, tmp.data(), job->spin_bytes(), hipMemcpyHostToDevice,
                               job->stream));
    if (job->gauss)
      PT_HIP(job, launch_gauss_energy(g, job->spins, job->gJ, job->E64, job->stream));
    else
      PT_HIP(job, launch_energy(g, job->spins, job->jw, job->E, job->stream));
    PT_HIP(job, hipStreamSynchronize(job->stream));
  } else {
    PT_HIP(job, hipMemcpyAsync(job->spins, in, n, hipMemcpyHostToDevice, job->stream));
    if (job->gauss)
      PT_HIP(job, launch_gauss_energy(g, job->spins, job->gJ, job->E64, job->stream));
    else
      PT_HIP(job, launch_energy(g, job->spins, job->jw, job->E, job->stream));
    PT_HIP(job, hipStreamSynchronize(job->stream));
  }
  return PT_OK;
}

PT_API int pt_get_layout(pt_job* job, uint32_t* out) {
  if (int rc = check_job(job)) return rc;
  if (!out) return pt_fail(PT_EINVAL, "null output");
  *out = (uint32_t)job->g.layout;
  return PT_OK;
}

PT_API int pt_set_layout(pt_job* job, uint32_t layout) {
  if (int rc = check_job(job)) return rc;
  if (layout != PT_LAYOUT_INT8 && layout != PT_LAYOUT_PACKED) return pt_fail(PT_EINVAL, "unknown layout");
  if (int rc = check_fault(job)) return rc;
  if ((int)layout == job->g.layout) return PT_OK;
  // work on any stream may still read the spins (a batch launch runs on the
  // batch's stream): wait for the device before converting and freeing
  PT_HIP(job, hipDeviceSynchronize());
  Geo to = job->g;
  to.layout = (int)layout;
  const size_t lat = (size_t)to.S * to.nslot;
  void* dst = job->dalloc(to.layout == kLayoutPacked ? lat * 2 * to.NW * sizeof(uint32_t) : lat * to.N);
  if (!dst) return pt_fail(PT_ENOMEM, "pt_set_layout: device allocation failed");
  const hipError_t e = launch_convert_layout(job->g, job->spins, dst, to.layout == kLayoutPacked,
                                             job->stream);
  const hipError_t es = e == hipSuccess ? hipStreamSynchronize(job->stream) : e;
  if (es != hipSuccess) {
    job->dfree(dst);
    return pt_fail(PT_EDEVICE, std::string("pt_set_layout: ") + hipGetErrorString(es));
  }
  job->dfree(job->spins);
  job->spins = dst;
  job->g.layout = to.layout;
  ++job->epoch;
  return PT_OK;
}

PT_API int pt_get_energies(pt_job* job, int32_t* out) {
  if (int rc = check_job(job)) return rc;
  if (job->gauss) return pt_fail(PT_EINVAL, "Gaussian energies are 64-bit: use pt_get_energies64");
  if (int rc = check_fault(job)) return rc;
  if (!out) return pt_fail(PT_EINVAL, "null output");
  const size_t n = (size_t)job->g.S * job->g.nslot;
  PT_HIP(job, hipMemcpyAsync(out, job->E, sizeof(int32_t) * n, hipMemcpyDeviceToHost, job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  return PT_OK;
}

PT_API int pt_get_maps(pt_job* job, int32_t* slot_of_temp, int32_t* temp_of_slot) {
  if (int rc = check_job(job)) return rc;
  if (int rc = check_fault(job)) return rc;
  const size_t n = sizeof(int32_t) * (size_t)job->g.S * 2 * job->g.NT;
  if (slot_of_temp)
    PT_HIP(job, hipMemcpyAsync(slot_of_temp, job->sot, n, hipMemcpyDeviceToHost, job->stream));
  if (temp_of_slot)
    PT_HIP(job, hipMemcpyAsync(temp_of_slot, job->tos, n, hipMemcpyDeviceToHost, job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  return PT_OK;
}

PT_API int pt_get_moments(pt_job* job, int64_t* out) {
  if (int rc = check_job(job)) return rc;
  if (job->gauss) return pt_fail(PT_EINVAL, "Gaussian jobs keep 128-bit E^2 sums: use pt_get_moments8");
  if (int rc = check_fault(job)) return rc;
  if (!out) return pt_fail(PT_EINVAL, "null output");
  const size_t n = (size_t)job->g.S * job->g.NT;
  std::vector<int64_t> m(8 * n);
  PT_HIP(job, hipMemcpyAsync(m.data(), job->mom, sizeof(int64_t) * m.size(), hipMemcpyDeviceToHost,
                             job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  for (size_t i = 0; i < n; ++i)
    for (int c = 0; c < 7; ++c) out[i * 7 + c] = m[i * 8 + c];
  return PT_OK;
}

PT_API int pt_get_energies64(pt_job* job, int64_t* out) {
  if (int rc = check_job(job)) return rc;
  if (int rc = check_fault(job)) return rc;
  if (!out) return pt_fail(PT_EINVAL, "null output");
  const size_t n = (size_t)job->g.S * job->g.nslot;
  if (job->gauss) {
    PT_HIP(job, hipMemcpyAsync(out, job->E64, sizeof(int64_t) * n, hipMemcpyDeviceToHost, job->stream));
    PT_HIP(job, hipStreamSynchronize(job->stream));
    return PT_OK;
  }
  std::vector<int32_t> e32(n);
  PT_HIP(job, hipMemcpyAsync(e32.data(), job->E, sizeof(int32_t) * n, hipMemcpyDeviceToHost, job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  for (size_t i = 0; i < n; ++i) out[i] = e32[i];
  return PT_OK;
}

PT_API int pt_get_moments8(pt_job* job, int64_t* out) {
  if (int rc = check_job(job)) return rc;
  if (int rc = check_fault(job)) return rc;
  if (!out) return pt_fail(PT_EINVAL, "null output");
  const size_t n = (size_t)job->g.S * job->g.NT;
  PT_HIP(job, hipMemcpyAsync(out, job->mom, sizeof(int64_t) * 8 * n, hipMemcpyDeviceToHost, job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  if (!job->gauss)
    for (size_t i = 0; i < n; ++i) out[i * 8 + 7] = 0;  // +-J: E^2 sums fit 64 bits
  return PT_OK;
}

PT_API int pt_gauss_accept_test(const uint32_t* r, const double* b, const int64_t* u, int32_t* out,
                                int32_t n, int32_t mode) {
  if (!r || !b || !u || !out || n < 0) return pt_fail(PT_EINVAL, "null pointer or n < 0");
  if (mode < 0 || mode > 2) return pt_fail(PT_EINVAL, "mode must be 0, 1 or 2");
  for (int32_t i = 0; i < n; ++i) {
    if (!(b[i] > 0.0) || !std::isfinite(b[i]) || u[i] <= 0 || u[i] > (int64_t)1 << 52)
      return pt_fail(PT_EINVAL, "need b > 0 finite and 0 < u <= 2^52");
    if (mode == 0 && u[i] >= ((int64_t)1 << 24)) return pt_fail(PT_EINVAL, "mode 0 needs u < 2^24");
  }
  if (n == 0) return PT_OK;
  uint32_t* dr = nullptr;
  double* db = nullptr;
  int64_t* du = nullptr;
  int32_t* dout = nullptr;
  hipError_t e = hipMalloc((void**)&dr, sizeof(uint32_t) * n);
  if (e == hipSuccess) e = hipMalloc((void**)&db, sizeof(double) * n);
  if (e == hipSuccess) e = hipMalloc((void**)&du, sizeof(int64_t) * n);
  if (e == hipSuccess) e = hipMalloc((void**)&dout, sizeof(int32_t) * n);
  if (e == hipSuccess) e = hipMemcpy(dr, r, sizeof(uint32_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(db, b, sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(du, u, sizeof(int64_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_gauss_accept(dr, db, du, dout, n, mode, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, dout, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
  (void)hipFree(dr);
  (void)hipFree(db);
  (void)hipFree(du);
  (void)hipFree(dout);
  if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_gauss_accept_test: ") + hipGetErrorString(e));
  return PT_OK;
}

PT_API int pt_gauss_accept_host(uint32_t r, double b, int64_t u) {
  if (!(b > 0.0) || !std::isfinite(b) || u <= 0 || u > (int64_t)1 << 52)
    return pt_fail(PT_EINVAL, "need b > 0 finite and 0 < u <= 2^52");
  return gauss_accept_dd(r, b, u) ? 1 : 0;
}

PT_API int pt_get_walk(pt_job* job, int32_t* label, uint32_t* begin, uint64_t* trips) {
  if (int rc = check_job(job)) return rc;
  if (!job->track_walk) return pt_fail(PT_EINVAL, "the job was created without PT_TRACK_WALK");
  if (int rc = check_fault(job)) return rc;
  const Geo& g = job->g;
  const size_t lat = (size_t)g.S * g.nslot;
  if (label || begin) {
    std::vector<int32_t> w(2 * lat);
    PT_HIP(job, hipMemcpyAsync(w.data(), job->walk, sizeof(int32_t) * w.size(), hipMemcpyDeviceToHost,
                               job->stream));
    PT_HIP(job, hipStreamSynchronize(job->stream));
    for (size_t i = 0; i < lat; ++i) {
      if (label) label[i] = w[2 * i];
      if (begin) begin[i] = (uint32_t)w[2 * i + 1];
    }
  }
  if (trips) {
    PT_HIP(job, hipMemcpyAsync(trips, job->trips, sizeof(uint64_t) * 32 * 3 * (size_t)g.S,
                               hipMemcpyDeviceToHost, job->stream));
    PT_HIP(job, hipStreamSynchronize(job->stream));
  }
  return PT_OK;
}

PT_API int pt_tunnel_summary(const uint64_t* trips, int32_t rows, uint64_t passes, double* tau_b,
                             double* err_b, double* tau, int32_t* equilibrated) {
  if (!trips || rows < 1) return pt_fail(PT_EINVAL, "need one or more rows of round-trip bins");
  // exact pooled sums per bin: count, sum of lengths, sum of squared lengths
  unsigned __int128 C[32] = {}, D[32] = {}, Q[32] = {};
  for (int32_t r = 0; r < rows; ++r)
    for (int b = 0; b < 32; ++b) {
      const uint64_t* t = trips + ((size_t)r * 32 + b) * 3;
      C[b] += t[0];
      D[b] += t[1];
      Q[b] += t[2];
    }
  const double nan = std::numeric_limits<double>::quiet_NaN();
  double mean[32], se[32];
  unsigned __int128 Ct = 0, Dt = 0;
  for (int b = 0; b < 32; ++b) {
    Ct += C[b];
    Dt += D[b];
    mean[b] = C[b] ? (double)D[b] / (double)C[b] : nan;
    se[b] = nan;
    if (C[b] > 1) {
      // C Q - D^2 >= 0 (Cauchy-Schwarz), exact in 128 bits while C Q < 2^128
      const unsigned __int128 num = C[b] * Q[b] - D[b] * D[b];
      const double c = (double)C[b];
      se[b] = std::sqrt((double)num / (c * c * (double)(C[b] - 1)));
    }
    if (tau_b) tau_b[b] = mean[b];
    if (err_b) err_b[b] = se[b];
  }
  if (tau) *tau = Ct ? (double)Dt / (double)Ct : nan;
  if (equilibrated) {
    // the last bin b complete after `passes` passes: 2^(b+1) - 1 <= passes
    int top = -1;
    while (top < 31 && ((uint64_t)2 << (top + 1)) - 1 <= passes) ++top;
    int ok = top >= 2;
    for (int b = top - 2; ok && b <= top; ++b) ok = C[b] > 1;
    for (int i = top - 2; ok && i <= top; ++i)
      for (int j = i + 1; ok && j <= top; ++j)
        ok = std::fabs(mean[i] - mean[j]) <= 2.0 * std::sqrt(se[i] * se[i] + se[j] * se[j]);
    *equilibrated = ok;
  }
  return PT_OK;
}

PT_API int pt_get_stats(pt_job* job, int64_t* out) {
  if (int rc = check_job(job)) return rc;
  if (int rc = check_fault(job)) return rc;
  if (!out) return pt_fail(PT_EINVAL, "null output");
  if (!job->track_stats) return pt_fail(PT_EINVAL, "the job was not created with PT_TRACK_STATS");
  PT_HIP(job, hipMemcpyAsync(out, job->stats, sizeof(int64_t) * (size_t)job->g.S * job->g.NT * kNStat,
                             hipMemcpyDeviceToHost, job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  return PT_OK;
}

PT_API int pt_get_modes(pt_job* job, int64_t* out) {
  if (int rc = check_job(job)) return rc;
  if (!job->track_modes) return pt_fail(PT_EINVAL, "the job was created without PT_TRACK_MODES");
  if (int rc = check_fault(job)) return rc;
  if (!out) return pt_fail(PT_EINVAL, "null output");
  const Geo& g = job->g;
  PT_HIP(job, hipMemcpyAsync(out, job->modes, sizeof(int64_t) * (size_t)g.S * g.NT * (g.L / 2 + 1),
                             hipMemcpyDeviceToHost, job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  return PT_OK;
}

namespace {
// cos(2 pi m / L), exact where it is 0 or +-1.
double cos_frac(long m, int L) {
  m %= L;
  if (m == 0) return 1.0;
  if (2 * m == L) return -1.0;
  if (4 * m == L || 4 * m == 3 * (long)L) return 0.0;
  return std::cos(2.0 * M_PI * (double)m / (double)L);
}
}  // namespace

PT_API int pt_correlation_length(pt_job* job, double* chi0, double* chik, double* xi) {
  if (int rc = check_job(job)) return rc;
  if (!job->track_modes) return pt_fail(PT_EINVAL, "the job was created without PT_TRACK_MODES");
  if (int rc = check_fault(job)) return rc;
  const Geo& g = job->g;
  const int L = g.L, MH = L / 2 + 1;
  const size_t n = (size_t)g.S * g.NT;
  std::vector<int64_t> md(n * MH), m(8 * n);
  DevCounters c;
  PT_HIP(job, hipMemcpyAsync(md.data(), job->modes, sizeof(int64_t) * md.size(), hipMemcpyDeviceToHost,
                             job->stream));
  PT_HIP(job, hipMemcpyAsync(m.data(), job->mom, sizeof(int64_t) * m.size(), hipMemcpyDeviceToHost,
                             job->stream));
  PT_HIP(job, hipMemcpyAsync(&c, job->ctr, sizeof(c), hipMemcpyDeviceToHost, job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  const double nm = (double)c.n_meas, N = (double)g.N, S = (double)g.S;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  for (int k = 0; k < g.NT; ++k) {
    // integer sums over samples first
    std::vector<int64_t> A(MH, 0);
    int64_t q2 = 0;
    for (int s = 0; s < g.S; ++s) {
      const size_t i = (size_t)s * g.NT + k;
      for (int j = 0; j < MH; ++j) A[j] += md[i * MH + j];
      q2 += m[i * 8 + 4];
    }
    double p1 = 0.0;  // sum over delta in [0, L) of cos(2 pi delta / L) A(delta)
    for (int delta = 0; delta < L; ++delta)
      p1 += cos_frac(delta, L) * (double)A[delta <= L / 2 ? delta : L - delta];
    const double c0 = (double)q2 / (S * nm * N), ck = p1 / ((double)g.d * S * nm * N);
    double x = nan;
    if (ck > 0.0 && c0 / ck >= 1.0) x = std::sqrt(c0 / ck - 1.0) / (2.0 * std::sin(M_PI / L));
    if (chi0) chi0[k] = c0;
    if (chik) chik[k] = ck;
    if (xi) xi[k] = x;
  }
  return PT_OK;
}

PT_API int pt_observables(pt_job* job, double* per_sample, double* disorder, int64_t* n_meas) {
  if (int rc = check_job(job)) return rc;
  if (int rc = check_fault(job)) return rc;
  const Geo& g = job->g;
  const size_t n = (size_t)g.S * g.NT;
  std::vector<int64_t> m(8 * n);
  DevCounters c;
  PT_HIP(job, hipMemcpyAsync(m.data(), job->mom, sizeof(int64_t) * m.size(), hipMemcpyDeviceToHost,
                             job->stream));
  PT_HIP(job, hipMemcpyAsync(&c, job->ctr, sizeof(c), hipMemcpyDeviceToHost, job->stream));
  PT_HIP(job, hipStreamSynchronize(job->stream));
  if (n_meas) *n_meas = (int64_t)c.n_meas;
  const double nm = (double)c.n_meas, Nd = (double)g.N;
  const double N2 = Nd * Nd, N4 = N2 * N2;
  // energies per spin in coupling units: Gaussian sums are in 2^-16 units
  const double unit = job->gauss ? 1.0 / 65536.0 : 1.0;
  auto q4_of = [&](size_t i) {
    const unsigned __int128 v =
        ((unsigned __int128)(uint64_t)m[i * 8 + 6] << 64) | (unsigned __int128)(uint64_t)m[i * 8 + 5];
    return v;
  };
  if (per_sample) {
    for (size_t i = 0; i < n; ++i) {
      double* o = per_sample + i * 5;
      o[0] = (double)m[i * 8 + 0] * unit / (2.0 * nm * Nd);
      o[1] = (double)m[i * 8 + 2] / (nm * Nd);
      o[2] = (double)m[i * 8 + 3] / (nm * Nd);
      o[3] = (double)m[i * 8 + 4] / (nm * N2);
      o[4] = (double)q4_of(i) / (nm * N4);
    }
  }
  if (disorder) {
    const double S = (double)g.S;
    for (int k = 0; k < g.NT; ++k) {
      int64_t sE = 0, sQ = 0, sAQ = 0, sQ2 = 0;
      unsigned __int128 sQ4 = 0;
      for (int s = 0; s < g.S; ++s) {
        const size_t i = (size_t)s * g.NT + k;
        sE += m[i * 8 + 0];
        sQ += m[i * 8 + 2];
        sAQ += m[i * 8 + 3];
        sQ2 += m[i * 8 + 4];
        sQ4 += q4_of(i);
      }
      double* o = disorder + (size_t)k * 6;
      o[0] = (double)sE * unit / (S * 2.0 * nm * Nd);
      o[1] = (double)sQ / (S * nm * Nd);
      o[2] = (double)sAQ / (S * nm * Nd);
      o[3] = (double)sQ2 / (S * nm * N2);
      o[4] = (double)sQ4 / (S * nm * N4);
      o[5] = 0.5 * (3.0 - o[4] / (o[3] * o[3]));
    }
  }
  return PT_OK;
}

// ---------------------------------------------------------------------------
// checkpoint / restore
// ---------------------------------------------------------------------------
namespace {
struct StateHeader {
  uint64_t magic;
  int32_t S, NT, L, d, layout, pad;
  uint64_t spin_bytes;
};
constexpr uint64_t kStateMagic = 0x50545347'53544154ull;  // "PTSGSTAT"

size_t state_size(const pt_job* job) {
  const Geo& g = job->g;
  const size_t lat = (size_t)g.S * g.nslot;
  // energies: int32 for +-J jobs, int64 (2^-16 units) for Gaussian ones
  const size_t ebytes = (job->gauss ? sizeof(int64_t) : sizeof(int32_t)) * lat;
  return sizeof(StateHeader) + job->spin_bytes() + ebytes +
         2 * sizeof(int32_t) * (size_t)g.S * 2 * g.NT + sizeof(DevCounters) +
         sizeof(int64_t) * 8 * (size_t)g.S * g.NT +
         (job->track_walk ? sizeof(int32_t) * 2 * lat + sizeof(uint64_t) * 32 * 3 * (size_t)g.S : 0) +
         (job->track_modes ? sizeof(int64_t) * (size_t)g.S * g.NT * (g.L / 2 + 1) : 0) +
         (job->track_stats ? sizeof(int64_t) * (size_t)g.S * g.NT * kNStat : 0);
}

int32_t state_flags(const pt_job* job) {
  return (job->track_walk ? 1 : 0) | (job->track_modes ? 2 : 0) | (job->track_stats ? 4 : 0) |
         (job->gauss ? 8 : 0);
}
}  // namespace

PT_API int pt_get_state(pt_job* job, void* buf, size_t* len) {
  if (int rc = check_job(job)) return rc;
  if (int rc = check_fault(job)) return rc;
  if (!len) return pt_fail(PT_EINVAL, "null length");
  const size_t need = state_size(job);
  if (!buf) {
    *len = need;
    return PT_OK;
  }
  if (*len < need) return pt_fail(PT_EINVAL, "state buffer too small");
  const Geo& g = job->g;
  char* p = static_cast<char*>(buf);
  StateHeader h{kStateMagic, g.S, g.NT, g.L, g.d, g.layout, state_flags(job),
                (uint64_t)job->spin_bytes()};
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  const size_t lat = (size_t)g.S * g.nslot, maps = sizeof(int32_t) * (size_t)g.S * 2 * g.NT;
  hipStream_t st = job->stream;
  PT_HIP(job, hipMemcpyAsync(p, job->spins, job->spin_bytes(), hipMemcpyDeviceToHost, st));
  p += job->spin_bytes();
  const size_t ebytes = (job->gauss ? sizeof(int64_t) : sizeof(int32_t)) * lat;
  const void* Esrc = job->gauss ? (const void*)job->E64 : (const void*)job->E;
  PT_HIP(job, hipMemcpyAsync(p, Esrc, ebytes, hipMemcpyDeviceToHost, st));
  p += ebytes;
  PT_HIP(job, hipMemcpyAsync(p, job->sot, maps, hipMemcpyDeviceToHost, st));
  p += maps;
  PT_HIP(job, hipMemcpyAsync(p, job->tos, maps, hipMemcpyDeviceToHost, st));
  p += maps;
  PT_HIP(job, hipMemcpyAsync(p, job->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, st));
  p += sizeof(DevCounters);
  PT_HIP(job, hipMemcpyAsync(p, job->mom, sizeof(int64_t) * 8 * (size_t)g.S * g.NT,
                             hipMemcpyDeviceToHost, st));
  p += sizeof(int64_t) * 8 * (size_t)g.S * g.NT;
  if (job->track_walk) {
    PT_HIP(job, hipMemcpyAsync(p, job->walk, sizeof(int32_t) * 2 * lat, hipMemcpyDeviceToHost, st));
    p += sizeof(int32_t) * 2 * lat;
    PT_HIP(job, hipMemcpyAsync(p, job->trips, sizeof(uint64_t) * 32 * 3 * (size_t)g.S,
                               hipMemcpyDeviceToHost, st));
    p += sizeof(uint64_t) * 32 * 3 * (size_t)g.S;
  }
  if (job->track_modes) {
    PT_HIP(job, hipMemcpyAsync(p, job->modes, sizeof(int64_t) * (size_t)g.S * g.NT * (g.L / 2 + 1),
                               hipMemcpyDeviceToHost, st));
    p += sizeof(int64_t) * (size_t)g.S * g.NT * (g.L / 2 + 1);
  }
  if (job->track_stats)
    PT_HIP(job, hipMemcpyAsync(p, job->stats, sizeof(int64_t) * (size_t)g.S * g.NT * kNStat,
                               hipMemcpyDeviceToHost, st));
  PT_HIP(job, hipStreamSynchronize(st));
  *len = need;
  return PT_OK;
}

PT_API int pt_set_state(pt_job* job, const void* buf, size_t len) {
  if (int rc = check_job(job)) return rc;
  if (!buf) return pt_fail(PT_EINVAL, "null state buffer");
  if (len != state_size(job)) return pt_fail(PT_EINVAL, "state size does not match this job");
  const Geo& g = job->g;
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kStateMagic || h.S != g.S || h.NT != g.NT || h.L != g.L || h.d != g.d ||
      h.layout != g.layout || h.pad != state_flags(job) ||
      h.spin_bytes != job->spin_bytes())
    return pt_fail(PT_EINVAL, "state was taken from a job of another shape or layout");
  const char* p = static_cast<const char*>(buf) + sizeof(h);
  const size_t lat = (size_t)g.S * g.nslot, maps = sizeof(int32_t) * (size_t)g.S * 2 * g.NT;
  hipStream_t st = job->stream;
  PT_HIP(job, hipMemcpyAsync(job->spins, p, job->spin_bytes(), hipMemcpyHostToDevice, st));
  p += job->spin_bytes();
  const size_t ebytes = (job->gauss ? sizeof(int64_t) : sizeof(int32_t)) * lat;
  void* Edst = job->gauss ? (void*)job->E64 : (void*)job->E;
  PT_HIP(job, hipMemcpyAsync(Edst, p, ebytes, hipMemcpyHostToDevice, st));
  p += ebytes;
  PT_HIP(job, hipMemcpyAsync(job->sot, p, maps, hipMemcpyHostToDevice, st));
  p += maps;
  PT_HIP(job, hipMemcpyAsync(job->tos, p, maps, hipMemcpyHostToDevice, st));
  p += maps;
  PT_HIP(job, hipMemcpyAsync(job->ctr, p, sizeof(DevCounters), hipMemcpyHostToDevice, st));
  p += sizeof(DevCounters);
  PT_HIP(job, hipMemcpyAsync(job->mom, p, sizeof(int64_t) * 8 * (size_t)g.S * g.NT,
                             hipMemcpyHostToDevice, st));
  p += sizeof(int64_t) * 8 * (size_t)g.S * g.NT;
  if (job->track_walk) {
    PT_HIP(job, hipMemcpyAsync(job->walk, p, sizeof(int32_t) * 2 * lat, hipMemcpyHostToDevice, st));
    p += sizeof(int32_t) * 2 * lat;
    PT_HIP(job, hipMemcpyAsync(job->trips, p, sizeof(uint64_t) * 32 * 3 * (size_t)g.S,
                               hipMemcpyHostToDevice, st));
    p += sizeof(uint64_t) * 32 * 3 * (size_t)g.S;
  }
  if (job->track_modes) {
    PT_HIP(job, hipMemcpyAsync(job->modes, p, sizeof(int64_t) * (size_t)g.S * g.NT * (g.L / 2 + 1),
                               hipMemcpyHostToDevice, st));
    p += sizeof(int64_t) * (size_t)g.S * g.NT * (g.L / 2 + 1);
  }
  if (job->track_stats)
    PT_HIP(job, hipMemcpyAsync(job->stats, p, sizeof(int64_t) * (size_t)g.S * g.NT * kNStat,
                               hipMemcpyHostToDevice, st));
  PT_HIP(job, hipStreamSynchronize(st));
  return PT_OK;
}
