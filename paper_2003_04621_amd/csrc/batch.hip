// batch.hip -- many independent jobs (any L, N_T, samples, spin layout) in
// one persistent launch per call: a work list of (job, sample, replica sets)
// items consumed from a device queue, the launch optionally captured once as
// a hipGraph and replayed, and an autotuner that picks the launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "job.h"
#include "kernels.h"
#include "pt.h"

using namespace ptsg;

struct BatchConfig {
  int threads = 0;     // threads per workgroup: 256, 512 or 1024; 0 = chosen per launch
  int sets = 2;        // replica sets per item when both fit (2) or always one (1)
  int order = 0;       // 0: largest items first, 1: job order
};

struct pt_batch {
  std::vector<pt_job*> jobs;
  int d = 3;
  int ncu = 256;
  hipStream_t stream = nullptr;
  BatchConfig cfg;
  // device work list for the last (mcs, flags, cfg)
  FusedArgs* d_jobs = nullptr;
  BatchItem* d_items = nullptr;
  uint32_t* d_queue = nullptr;
  int cap_jobs = 0, cap_items = 0;
  int nitems = 0;
  size_t lds_bytes = 0;
  int blocks = 0;
  bool built = false;
  int built_mcs = -1;
  uint32_t built_flags = 0;
  BatchConfig built_cfg;
  std::vector<int> built_every;
  std::vector<uint32_t> built_epoch;  // the jobs' epochs when the list was built
  // captured launch (captured on a private stream, replayed on `stream`)
  hipStream_t cap_stream = nullptr;
  hipEvent_t side_ev = nullptr;  // orders per-step jobs against the batch stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graph_ok = false;
  bool has_split = false;  // the work list holds split samples
  int feat = 0;            // kinds of work in the work list (kFeat*)
  int threads = 0;         // threads per workgroup of the built launch
  int per_cu = 0;          // workgroups of that size resident per CU
  // pinned staging of the work list (the upload is then truly asynchronous)
  // and the events ordering its reuse: stage_ev after the last upload from
  // it, last_ev after the last launch reading the device work list
  void* h_stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t stage_ev = nullptr, last_ev = nullptr;
  std::vector<FusedArgs> args;  // host copy of the uploaded launch arguments
};

namespace {

// Launches holding split samples are ordered one after another across all
// streams of the process (per device): two of them running side by side
// could each hold part of the machine while waiting for workgroups that only
// the other one's exit would make room for.
std::mutex g_split_mu;
hipEvent_t g_split_ev[64] = {};

template <typename F>
hipError_t ordered_split_launch(hipStream_t st, F&& launch) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_split_mu);
  if (!g_split_ev[dev]) e = hipEventCreateWithFlags(&g_split_ev[dev], hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, g_split_ev[dev], 0);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(g_split_ev[dev], st);
  return e;
}

bool same_cfg(const BatchConfig& a, const BatchConfig& b) {
  return a.threads == b.threads && a.sets == b.sets && a.order == b.order;
}

void drop_graph(pt_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_ok = false;
}

// Plan of a job for the given flags and config: 0 both sets per workgroup,
// 1 the same with Houdayer room, 2 one set per workgroup, 3 split sample, 4
// both sets with multi-cluster Houdayer room; -1 if none exists.
int job_mode(const pt_job* j, uint32_t flags, const BatchConfig& cfg) {
  const bool hou = flags & PT_MCS_HOUDAYER, meas = flags & PT_MCS_MEASURE;
  if (hou && (flags & PT_MCS_MULTICLUSTER)) return j->fused_ok[4] ? 4 : -1;
  if (hou) return j->fused_ok[1] ? 1 : -1;
  if (cfg.sets == 2 && j->fused_ok[0]) return 0;
  if (meas) return j->fused_ok[0] ? 0 : (j->split_ok ? 3 : -1);
  if (j->fused_ok[2]) return 2;
  if (j->fused_ok[0]) return 0;
  return j->split_ok ? 3 : -1;
}

}  // namespace

// The launch arguments of job j for `mcs` fused steps in plan `mode`.
FusedArgs job_fused_args(const pt_job* j, int mode, int mcs, uint32_t flags) {
  const bool hou = flags & PT_MCS_HOUDAYER, meas = flags & PT_MCS_MEASURE;
  const FusedLayout& lay = mode == 3 ? j->split_lay : j->plan[mode];
  FusedArgs A = make_fused_args(j->g, lay, j->spins, j->jw, j->E, j->sot, j->tos, j->thr, j->thrpt,
                                j->M, j->mom, j->walk, j->trips, j->modes, j->ctr, mcs,
                                mode == 3 ? false : hou, meas);
  A.every = j->meas_every;
  if (A.hou && (flags & PT_MCS_MULTICLUSTER)) A.hou = 2;
  if (mode == 3) {
    A.parts = j->split_parts;
    A.R = j->split_R;
    A.jlds = j->split_jlds;
    A.Ex = j->Ex;
    A.snap = j->snap;
    A.bar = j->bar;
  }
  return A;
}

// Persistent grid: as many workgroups as can be resident at once (the
// runtime's occupancy for this kernel, LDS plan and workgroup size).  Unless
// configured (cfg_threads > 0), the workgroup size is a multiple of four
// wavefronts, so that every SIMD of a CU holds the same number of them (a CU
// places a workgroup's wavefronts on its four SIMDs in turn; with 6 or 10 per
// workgroup two SIMDs carry more than the others and set the pace).  With no
// more items than CUs each item runs alone, on the largest workgroup;
// otherwise the size with the most wavefronts per CU, then at least two
// workgroups per CU (they fill each other's barriers and serial exchange
// passes), then the larger workgroup (fewer items in flight leave fewer CUs
// idle at the end).
int launch_shape(int d, int feat, size_t lds_bytes, int nitems, int ncu, int cfg_threads,
                 int* threads_out, int* per_cu_out) {
  // the runtime's answer for a (device, kernel variant, workgroup size, LDS)
  // never changes, so each is asked once
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int, size_t>, int> known;
  int dev = 0;
  (void)hipGetDevice(&dev);
  auto resident = [&](int threads) {
    const auto key = std::make_tuple(dev, d, feat, threads, lds_bytes);
    {
      std::lock_guard<std::mutex> lk(mu);
      const auto it = known.find(key);
      if (it != known.end()) return it->second;
    }
    int n = 0;
    if (batch_residency(d, feat, threads, lds_bytes, &n) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    std::lock_guard<std::mutex> lk(mu);
    known[key] = n;
    return n;
  };
  int threads = cfg_threads;
  if (threads == 0) {
    int best_n = 0, best_waves = 0;
    for (int t : {1024, 768, 512, 256}) {
      const int n = resident(t), waves = n * t / 64;
      if (n < 1) continue;
      bool better;
      if (best_n == 0) {
        better = true;
      } else if (nitems <= ncu) {
        better = false;  // sizes are tried largest first
      } else {
        better = waves > best_waves || (waves == best_waves && n >= 2 && best_n < 2);
      }
      if (better) {
        best_n = n;
        best_waves = waves;
        threads = t;
      }
    }
    if (threads == 0) threads = 256;
  }
  const int per_cu = resident(threads);
  if (per_cu < 1)
    return pt_fail(PT_EINVAL, "no workgroup of " + std::to_string(threads) +
                                  " threads fits a CU with this launch's LDS and registers");
  *threads_out = threads;
  *per_cu_out = per_cu;
  return PT_OK;
}

// ordered_split_launch for callers outside this file.
hipError_t split_ordered(hipStream_t st, hipError_t (*launch)(void*), void* ctx) {
  return ordered_split_launch(st, [&] { return launch(ctx); });
}

// Creates the current device's ordering event for split launches now (it is
// otherwise created by the first such launch).
hipError_t split_order_prepare() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_split_mu);
  if (!g_split_ev[dev]) e = hipEventCreateWithFlags(&g_split_ev[dev], hipEventDisableTiming);
  return e;
}

namespace {

// A launch's work list as built on the host: the jobs' launch arguments,
// the items (split samples first), the LDS words of the largest plan and the
// kinds of work present.
struct HostWorklist {
  std::vector<FusedArgs> jobs;
  std::vector<BatchItem> items;
  size_t lds_words = 0;
  int feat = 0;
  bool has_split = false;
};

// Work list for per-job step counts and flags (jobs with 0 steps get no item).
int plan_worklist(const std::vector<pt_job*>& jobs, const BatchConfig& cfg, const std::vector<int>& steps,
                  const std::vector<uint32_t>& jflags, HostWorklist& out) {
  std::vector<FusedArgs>& hj = out.jobs;
  std::vector<BatchItem>& hi = out.items;
  std::vector<BatchItem> split;
  std::vector<std::pair<double, size_t>> split_groups;  // (cost of a part, first item)
  std::vector<double> cost;
  size_t lds_words = 0;
  int feat = 0;
  hj.clear();
  hi.clear();
  for (size_t jx = 0; jx < jobs.size(); ++jx) {
    pt_job* j = jobs[jx];
    const uint32_t flags = jflags[jx];
    const bool hou = flags & PT_MCS_HOUDAYER, meas = flags & PT_MCS_MEASURE;
    const int mcs = steps[jx];
    const int mode = job_mode(j, flags, cfg);
    if (mode < 0) {
      // no fused plan for these flags: the job's steps run through the
      // per-step kernels beside the launch (pt_batch_run); here it only keeps
      // its index, with no steps and no items
      hj.push_back(job_fused_args(j, 0, 0, 0u));
      continue;
    }
    if (mcs > 0 && meas) feat |= kFeatMeas;
    if (mcs > 0 && hou) feat |= kFeatHou;
    if (mcs > 0 && mode == 3) feat |= kFeatSplit;
    if (mcs > 0 && j->track_walk) feat |= kFeatWalk;
    if (mcs > 0 && meas && j->track_modes) feat |= kFeatModes;
    if (mode == 3) {
      hj.push_back(job_fused_args(j, mode, mcs, flags));
      lds_words = std::max(lds_words, (size_t)j->split_lay.words);
      if (mcs <= 0) continue;
      // the parts of a sample are consecutive, and split samples go first so
      // that all parts are taken while every workgroup is still free
      for (int s = 0; s < j->g.S; ++s) {
        split_groups.push_back({(double)j->split_R * j->g.N * mcs, split.size()});
        for (int p = 0; p < j->split_parts; ++p) split.push_back(BatchItem{(int)jx, s, p, 0});
      }
      continue;
    }
    const int nsets = mode == 2 ? 1 : 2;
    hj.push_back(job_fused_args(j, mode, mcs, flags));
    lds_words = std::max(lds_words, (size_t)j->plan[mode].words);
    if (mcs <= 0) continue;
    const double c = (double)nsets * j->g.NT * j->g.N * mcs;
    for (int s = 0; s < j->g.S; ++s)
      for (int c_lo = 0; c_lo < 2; c_lo += nsets) {
        hi.push_back(BatchItem{(int)jx, s, c_lo, nsets});
        cost.push_back(c);
      }
  }
  if (cfg.order == 0) {
    std::vector<size_t> idx(hi.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<BatchItem> sorted(hi.size());
    for (size_t i = 0; i < idx.size(); ++i) sorted[i] = hi[idx[i]];
    hi.swap(sorted);
  }
  if (cfg.order == 0 && split_groups.size() > 1) {
    // split samples longest parts first, each sample's parts kept together
    std::stable_sort(split_groups.begin(), split_groups.end(),
                     [](const std::pair<double, size_t>& x, const std::pair<double, size_t>& y) {
                       return x.first > y.first;
                     });
    std::vector<BatchItem> sorted;
    sorted.reserve(split.size());
    for (const auto& gr : split_groups) {
      const size_t end = gr.second + (size_t)jobs[split[gr.second].job]->split_parts;
      for (size_t i = gr.second; i < end; ++i) sorted.push_back(split[i]);
    }
    split.swap(sorted);
  }
  hi.insert(hi.begin(), split.begin(), split.end());
  out.has_split = !split.empty();
  out.lds_words = lds_words;
  out.feat = feat;
  return PT_OK;
}

// Uploads launch arguments (and, if ni > 0, work items) to the batch's
// device buffers.  The upload goes through pinned staging memory, so it is
// asynchronous and ordered on the stream before the launch that reads it: the
// host does not wait for the GPU.  The staging area is rewritten only after
// the previous upload from it has been done (stage_ev), and the device list
// only after the last launch that read it, whatever stream that ran on
// (last_ev).
int upload_worklist(pt_batch* b, const FusedArgs* args, size_t nj, const BatchItem* items, size_t ni) {
  hipError_t e = hipSuccess;
  const size_t jbytes = sizeof(FusedArgs) * nj, ibytes = sizeof(BatchItem) * ni;
  if (!b->stage_ev) e = hipEventCreateWithFlags(&b->stage_ev, hipEventDisableTiming);
  if (e == hipSuccess && !b->last_ev) e = hipEventCreateWithFlags(&b->last_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventSynchronize(b->stage_ev);
  if (e == hipSuccess && jbytes + ibytes > b->stage_cap) {
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    b->h_stage = nullptr;
    b->stage_cap = 0;
    e = hipHostMalloc(&b->h_stage, jbytes + ibytes, hipHostMallocDefault);
    if (e != hipSuccess) return pt_fail(PT_ENOMEM, "pt_batch_run: pinned staging allocation failed");
    b->stage_cap = jbytes + ibytes;
  }
  if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_batch_run: ") + hipGetErrorString(e));
  unsigned char* stage = static_cast<unsigned char*>(b->h_stage);
  std::memcpy(stage, args, jbytes);
  if (ibytes) std::memcpy(stage + jbytes, items, ibytes);
  e = hipStreamWaitEvent(b->stream, b->last_ev, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_jobs, stage, jbytes, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && ibytes)
    e = hipMemcpyAsync(b->d_items, stage + jbytes, ibytes, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->stage_ev, b->stream);
  if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_batch_run: ") + hipGetErrorString(e));
  return PT_OK;
}

// Work list for per-job step counts and flags, uploaded to the batch's own
// device buffers (grown as needed).
int build_worklist_ex(pt_batch* b, const std::vector<int>& steps, const std::vector<uint32_t>& jflags) {
  HostWorklist wl;
  if (int rc = plan_worklist(b->jobs, b->cfg, steps, jflags, wl)) return rc;
  const std::vector<FusedArgs>& hj = wl.jobs;
  const std::vector<BatchItem>& hi = wl.items;
  const size_t lds_words = wl.lds_words;
  const int feat = wl.feat;
  b->has_split = wl.has_split;
  hipError_t e = hipSuccess;
  if ((int)hj.size() > b->cap_jobs) {
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    b->d_jobs = nullptr;
    e = hipMalloc((void**)&b->d_jobs, sizeof(FusedArgs) * hj.size());
    if (e != hipSuccess) return pt_fail(PT_ENOMEM, "pt_batch_run: device allocation failed");
    b->cap_jobs = (int)hj.size();
  }
  if ((int)hi.size() > b->cap_items) {
    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    e = hipMalloc((void**)&b->d_items, sizeof(BatchItem) * hi.size());
    if (e != hipSuccess) return pt_fail(PT_ENOMEM, "pt_batch_run: device allocation failed");
    b->cap_items = (int)hi.size();
  }
  if (!b->d_queue) {
    e = hipMalloc((void**)&b->d_queue, 256);
    if (e != hipSuccess) return pt_fail(PT_ENOMEM, "pt_batch_run: device allocation failed");
  }
  if (int rc = upload_worklist(b, hj.data(), hj.size(), hi.data(), hi.size())) return rc;
  b->args = hj;
  b->nitems = (int)hi.size();
  b->lds_bytes = lds_words * 4;
  b->feat = feat;
  e = prepare_batch(b->d, feat, b->lds_bytes, nullptr);
  if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_batch_run: ") + hipGetErrorString(e));
  int threads = 0, per_cu = 0;
  if (int rc = launch_shape(b->d, feat, b->lds_bytes, b->nitems, b->ncu, b->cfg.threads, &threads,
                            &per_cu))
    return rc;
  b->threads = threads;
  b->per_cu = per_cu;
  b->blocks = std::max(1, std::min(b->ncu * per_cu, b->nitems));
  b->built = false;
  drop_graph(b);
  return PT_OK;
}

int build_worklist(pt_batch* b, int mcs, uint32_t flags) {
  std::vector<int> every(b->jobs.size());  // the work list carries each job's interval
  std::vector<uint32_t> epoch(b->jobs.size());  // and its buffers and layout
  for (size_t i = 0; i < b->jobs.size(); ++i) {
    every[i] = b->jobs[i]->meas_every;
    epoch[i] = b->jobs[i]->epoch;
  }
  const bool same = b->built && b->built_flags == flags && same_cfg(b->built_cfg, b->cfg) &&
                    b->built_every == every && b->built_epoch == epoch;
  if (same && b->built_mcs == mcs) return PT_OK;
  if (same && b->built_mcs > 0 && mcs > 0) {
    // only the step count differs: the items, their order and the launch
    // shape stay, and the kernels read the count from the launch arguments
    // in device memory (a captured graph stays valid too)
    for (FusedArgs& a : b->args) a.nmcs = mcs;
    if (int rc = upload_worklist(b, b->args.data(), b->args.size(), nullptr, 0)) return rc;
    b->built_mcs = mcs;
    return PT_OK;
  }
  b->built_every = every;
  b->built_epoch = epoch;
  const std::vector<int> steps(b->jobs.size(), mcs);
  const std::vector<uint32_t> fl(b->jobs.size(), flags);
  if (int rc = build_worklist_ex(b, steps, fl)) return rc;
  b->built = true;
  b->built_mcs = mcs;
  b->built_flags = flags;
  b->built_cfg = b->cfg;
  return PT_OK;
}

int run_once(pt_batch* b, bool use_graph) {
  if (b->nitems == 0) return PT_OK;
  if (!use_graph) {
    auto launch = [&] {
      return launch_batch(b->d, b->feat, b->d_jobs, (int)b->jobs.size(), b->d_items, b->nitems,
                          b->d_queue, b->blocks, b->threads, b->lds_bytes, b->stream);
    };
    hipError_t e = b->has_split ? ordered_split_launch(b->stream, launch) : launch();
    if (e == hipSuccess && b->last_ev) e = hipEventRecord(b->last_ev, b->stream);
    if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_batch_run: ") + hipGetErrorString(e));
    return PT_OK;
  }
  if (!b->graph_ok) {
    hipError_t e = hipSuccess;
    if (!b->cap_stream) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t el = launch_batch(b->d, b->feat, b->d_jobs, (int)b->jobs.size(), b->d_items,
                                         b->nitems, b->d_queue, b->blocks, b->threads,
                                         b->lds_bytes, b->cap_stream);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(b->cap_stream, &g);
      if (e == hipSuccess && el != hipSuccess) e = el;
      if (e == hipSuccess) {
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
      } else if (g) {
        (void)hipGraphDestroy(g);
      }
    }
    if (e != hipSuccess) {
      drop_graph(b);
      return pt_fail(PT_EDEVICE, std::string("pt_batch_run graph capture: ") + hipGetErrorString(e));
    }
    b->graph_ok = true;
  }
  auto replay = [&] { return hipGraphLaunch(b->exec, b->stream); };
  hipError_t e = b->has_split ? ordered_split_launch(b->stream, replay) : replay();
  if (e == hipSuccess && b->last_ev) e = hipEventRecord(b->last_ev, b->stream);
  if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_batch_run: ") + hipGetErrorString(e));
  return PT_OK;
}

// ---- state snapshot for tuning trials --------------------------------------
struct Snap {
  std::vector<void*> bufs;
};

int snapshot(pt_batch* b, Snap& sn, bool restore) {
  size_t k = 0;
  for (pt_job* j : b->jobs) {
    const size_t lat = (size_t)j->g.S * j->g.nslot, maps = sizeof(int32_t) * (size_t)j->g.S * 2 * j->g.NT;
    void* src[9] = {j->spins, j->E, j->sot, j->tos, j->ctr, j->mom, j->walk, j->trips, j->modes};
    const size_t len[9] = {j->spin_bytes(),
                           sizeof(int32_t) * lat,
                           maps,
                           maps,
                           sizeof(DevCounters),
                           sizeof(int64_t) * 8 * (size_t)j->g.S * j->g.NT,
                           sizeof(int32_t) * 2 * lat,
                           sizeof(uint64_t) * 32 * 3 * (size_t)j->g.S,
                           sizeof(int64_t) * (size_t)j->g.S * j->g.NT * (j->g.L / 2 + 1)};
    for (int i = 0; i < 9; ++i) {
      if (!src[i]) continue;  // no replica walk or modes kept
      const size_t at = k++;
      if (!restore) {
        void* p = nullptr;
        if (hipMalloc(&p, len[i]) != hipSuccess) return pt_fail(PT_ENOMEM, "pt_batch_tune: snapshot allocation failed");
        sn.bufs.push_back(p);
        if (hipMemcpyAsync(p, src[i], len[i], hipMemcpyDeviceToDevice, b->stream) != hipSuccess)
          return pt_fail(PT_EDEVICE, "pt_batch_tune: snapshot copy failed");
      } else if (hipMemcpyAsync(src[i], sn.bufs[at], len[i], hipMemcpyDeviceToDevice, b->stream) !=
                 hipSuccess) {
        return pt_fail(PT_EDEVICE, "pt_batch_tune: restore copy failed");
      }
    }
  }
  return hipStreamSynchronize(b->stream) == hipSuccess ? PT_OK
                                                        : pt_fail(PT_EDEVICE, "pt_batch_tune: sync failed");
}

std::string cache_key(const pt_batch* b, uint32_t flags) {
  // dimension, flags and the sorted multiset of (L, N_T, samples, layout)
  std::vector<std::string> parts;
  for (const pt_job* j : b->jobs)
    parts.push_back(std::to_string(j->g.L) + "x" + std::to_string(j->g.NT) + "x" +
                    std::to_string(j->g.S) + "x" + std::to_string(j->g.layout) +
                    (j->track_walk ? "w" : "") + (j->track_modes ? "m" : ""));
  std::sort(parts.begin(), parts.end());
  std::string key = "gfx950/d" + std::to_string(b->d) + "/f" + std::to_string(flags) + "/";
  size_t i = 0;
  while (i < parts.size()) {
    size_t n = 1;
    while (i + n < parts.size() && parts[i + n] == parts[i]) ++n;
    key += parts[i] + "*" + std::to_string(n) + ";";
    i += n;
  }
  return key;
}

bool cache_lookup(const char* path, const std::string& key, BatchConfig& cfg, int* layout) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    // {"key": "<key>", "threads": T, "sets": S, "order": O}
    const std::string l(line);
    const std::string want = "\"key\": \"" + key + "\"";
    if (l.find(want) == std::string::npos) continue;
    int t = 0, s = 0, o = 0, ly = -1;
    const char* p = std::strstr(line, "\"threads\":");
    const char* q = std::strstr(line, "\"sets\":");
    const char* r = std::strstr(line, "\"order\":");
    const char* y = std::strstr(line, "\"layout\":");
    if (p && q && r && std::sscanf(p, "\"threads\": %d", &t) == 1 && std::sscanf(q, "\"sets\": %d", &s) == 1 &&
        std::sscanf(r, "\"order\": %d", &o) == 1) {
      if (!y || std::sscanf(y, "\"layout\": %d", &ly) != 1 ||
          (ly != (int)PT_LAYOUT_INT8 && ly != (int)PT_LAYOUT_PACKED))
        ly = -1;
      cfg.threads = t;
      cfg.sets = s;
      cfg.order = o;
      *layout = ly;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

// layout < 0: the trials kept every job's layout
void cache_store(const char* path, const std::string& key, const BatchConfig& cfg, int layout, double ms) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  if (layout < 0)
    std::fprintf(f, "{\"key\": \"%s\", \"threads\": %d, \"sets\": %d, \"order\": %d, \"trial_ms\": %.4f}\n",
                 key.c_str(), cfg.threads, cfg.sets, cfg.order, ms);
  else
    std::fprintf(f,
                 "{\"key\": \"%s\", \"threads\": %d, \"sets\": %d, \"order\": %d, \"layout\": %d, "
                 "\"trial_ms\": %.4f}\n",
                 key.c_str(), cfg.threads, cfg.sets, cfg.order, layout, ms);
  std::fclose(f);
}

// Every job of the batch to one spin layout.
int set_layout_all(pt_batch* b, int layout) {
  for (pt_job* j : b->jobs)
    if (int rc = pt_set_layout(j, (uint32_t)layout)) return rc;
  return PT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Internal entry points for the request server: one launch over a changing
// set of resident jobs with per-job step counts and flags.
pt_batch* batch_new(hipStream_t st) {
  pt_batch* b = new (std::nothrow) pt_batch();
  if (!b) return nullptr;
  b->stream = st;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    b->ncu = ncu;
  (void)hipGetLastError();
  return b;
}

int batch_round(pt_batch* b, const std::vector<pt_job*>& jobs, const std::vector<int>& steps,
                const std::vector<uint32_t>& flags) {
  if (jobs.empty()) return PT_OK;
  b->jobs = jobs;
  b->d = jobs[0]->g.d;
  if (int rc = build_worklist_ex(b, steps, flags)) return rc;
  return run_once(b, false);
}

int batch_run_job(pt_batch* b, pt_job* job, int mcs, uint32_t flags) {
  if (b->jobs.size() != 1 || b->jobs[0] != job) {
    b->jobs.assign(1, job);
    b->d = job->g.d;
    b->built = false;
  }
  b->stream = job->stream;
  if (int rc = build_worklist(b, mcs, flags)) return rc;
  return run_once(b, false);
}

// ---- the work list in library-held device memory (pt_mcs_noalloc) ---------
namespace {
// Library-held scratch of pt_mcs_noalloc, one copy per GPU for the life of
// the process: the work-queue counter (first 256 bytes), then the job's
// launch arguments, then the work items.  In host code `scratch` only names
// the symbol; the device address comes from hipGetSymbolAddress.
constexpr size_t kScratchArgsAt = 256;
constexpr size_t kScratchItemsAt = (kScratchArgsAt + sizeof(FusedArgs) + 255) / 256 * 256;
constexpr size_t kScratchMaxItems = PT_NOALLOC_MAX_ITEMS;
constexpr size_t kScratchBytes = kScratchItemsAt + kScratchMaxItems * sizeof(BatchItem);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[64] = {};
int g_scratch_ncu[64] = {};

// The current device's address of `scratch` (and its CU count), looked up
// once per device with that device current; the split-launch ordering event
// is created at the same time, so later calls create nothing.
int scratch_for_device(unsigned char** ptr, int* ncu) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return pt_fail(PT_EDEVICE, "pt_mcs_noalloc: no current device");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return pt_fail(PT_EDEVICE, std::string("pt_mcs_noalloc: scratch address: ") + hipGetErrorString(e));
    int n = 0;
    e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = split_order_prepare();
    if (e != hipSuccess)
      return pt_fail(PT_EDEVICE, std::string("pt_mcs_noalloc: set-up: ") + hipGetErrorString(e));
    g_scratch_ncu[dev] = n > 0 ? n : 256;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *ptr = g_scratch_ptr[dev];
  *ncu = g_scratch_ncu[dev];
  return PT_OK;
}
}  // namespace

int batch_run_job_noalloc(pt_job* job, int mcs, uint32_t flags, int* nitems_out) {
  HostWorklist wl;
  if (int rc = plan_worklist({job}, BatchConfig{}, {mcs}, {flags}, wl)) return rc;
  if (nitems_out) *nitems_out = (int)wl.items.size();
  if (wl.items.size() > kScratchMaxItems)
    return pt_fail(PT_EINVAL, "pt_mcs_noalloc: " + std::to_string(wl.items.size()) +
                                  " work items exceed the library scratch (at most " +
                                  std::to_string(kScratchMaxItems) + ")");
  if (wl.items.empty()) return PT_OK;
  unsigned char* base = nullptr;
  int ncu = 0;
  if (int rc = scratch_for_device(&base, &ncu)) return rc;
  FusedArgs* d_jobs = reinterpret_cast<FusedArgs*>(base + kScratchArgsAt);
  BatchItem* d_items = reinterpret_cast<BatchItem*>(base + kScratchItemsAt);
  uint32_t* d_queue = reinterpret_cast<uint32_t*>(base);
  const int d = job->g.d;
  const size_t lds_bytes = wl.lds_words * 4;
  hipError_t e = prepare_batch(d, wl.feat, lds_bytes, nullptr);
  if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_mcs_noalloc: ") + hipGetErrorString(e));
  const int nitems = (int)wl.items.size();
  int threads = 0, per_cu = 0;
  if (int rc = launch_shape(d, wl.feat, lds_bytes, nitems, ncu, 0, &threads, &per_cu)) return rc;
  const int blocks = std::max(1, std::min(ncu * per_cu, nitems));
  // pageable host sources: each copy has read its source when it returns,
  // and it is ordered on the stream before the launch that reads it
  e = hipMemcpyAsync(d_jobs, wl.jobs.data(), sizeof(FusedArgs), hipMemcpyHostToDevice, job->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_items, wl.items.data(), sizeof(BatchItem) * wl.items.size(),
                       hipMemcpyHostToDevice, job->stream);
  if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_mcs_noalloc: ") + hipGetErrorString(e));
  auto launch = [&] {
    return launch_batch(d, wl.feat, d_jobs, 1, d_items, nitems, d_queue, blocks, threads, lds_bytes,
                        job->stream);
  };
  e = wl.has_split ? ordered_split_launch(job->stream, launch) : launch();
  if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_mcs_noalloc: ") + hipGetErrorString(e));
  return PT_OK;
}

int job_plan_mode(const pt_job* j, uint32_t flags) { return job_mode(j, flags, BatchConfig{}); }

void job_items(const pt_job* j, uint32_t flags, int& items, double& item_flips) {
  const int mode = job_mode(j, flags, BatchConfig{});
  const double lat = (double)j->g.N;
  if (mode == 3) {
    items = j->g.S * j->split_parts;
    item_flips = lat * j->split_R;
  } else if (mode == 2) {
    items = j->g.S * 2;
    item_flips = lat * j->g.NT;
  } else {
    items = j->g.S;
    item_flips = lat * (mode < 0 ? j->g.NT : j->g.nslot);
  }
}

int batch_slots(const pt_batch* b) { return b->ncu; }

void batch_free(pt_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_queue) (void)hipFree(b->d_queue);
  if (b->stage_ev) (void)hipEventSynchronize(b->stage_ev);
  if (b->h_stage) (void)hipHostFree(b->h_stage);
  if (b->stage_ev) (void)hipEventDestroy(b->stage_ev);
  if (b->last_ev) (void)hipEventDestroy(b->last_ev);
  if (b->side_ev) (void)hipEventDestroy(b->side_ev);
  (void)hipGetLastError();
  delete b;
}

// ---------------------------------------------------------------------------
PT_API int pt_batch_create(pt_job* const* jobs, int32_t n, pt_batch** out) {
  if (!jobs || !out || n < 1) return pt_fail(PT_EINVAL, "pt_batch_create: need n >= 1 jobs and an output");
  const int d = jobs[0] ? jobs[0]->g.d : 0;
  for (int i = 0; i < n; ++i) {
    if (!jobs[i]) return pt_fail(PT_EINVAL, "pt_batch_create: null job");
    if (jobs[i]->poisoned) return pt_fail(PT_ESTATE, "pt_batch_create: a job is poisoned");
    if (jobs[i]->g.d != d) return pt_fail(PT_EINVAL, "pt_batch_create: all jobs must have the same dim");
    if (jobs[i]->gauss)
      return pt_fail(PT_EINVAL, "pt_batch_create: jobs with Gaussian couplings run alone (pt_mcs)");
    if (jobs[i]->track_stats)
      return pt_fail(PT_EINVAL, "pt_batch_create: jobs keeping run diagnostics run alone (pt_mcs)");
    for (int k = 0; k < i; ++k)
      if (jobs[k] == jobs[i]) return pt_fail(PT_EINVAL, "pt_batch_create: a job appears twice");
  }
  pt_batch* b = new (std::nothrow) pt_batch();
  if (!b) return pt_fail(PT_ENOMEM, "pt_batch_create: host allocation failed");
  b->jobs.assign(jobs, jobs + n);
  b->d = d;
  b->stream = jobs[0]->stream;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    b->ncu = ncu;
  (void)hipGetLastError();
  *out = b;
  return PT_OK;
}

PT_API int pt_batch_set_stream(pt_batch* b, void* hip_stream) {
  if (!b) return pt_fail(PT_EINVAL, "null batch");
  b->stream = (hipStream_t)hip_stream;
  drop_graph(b);
  return PT_OK;
}

namespace {
// The steps of the jobs that have no fused plan for these flags, through the
// per-step kernels on each job's own stream: after the batch stream's earlier
// work (the job's earlier fused steps), and before its later work.
int run_unplanned(pt_batch* b, int mcs, uint32_t work_flags) {
  std::vector<pt_job*> side;
  for (pt_job* j : b->jobs)
    if (job_mode(j, work_flags, b->cfg) < 0) side.push_back(j);
  if (side.empty()) return PT_OK;
  hipError_t e = hipSuccess;
  if (!b->side_ev) e = hipEventCreateWithFlags(&b->side_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(b->side_ev, b->stream);
  for (pt_job* j : side)
    if (e == hipSuccess) e = hipStreamWaitEvent(j->stream, b->side_ev, 0);
  if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_batch_run: ") + hipGetErrorString(e));
  for (pt_job* j : side) {
    if (int rc = pt_mcs(j, mcs, work_flags | PT_MCS_PLAIN)) return rc;
    e = hipEventRecord(b->side_ev, j->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->side_ev, 0);
    if (e != hipSuccess) return pt_fail(PT_EDEVICE, std::string("pt_batch_run: ") + hipGetErrorString(e));
  }
  return PT_OK;
}
}  // namespace

PT_API int pt_batch_run(pt_batch* b, int32_t mcs, uint32_t flags) {
  if (!b) return pt_fail(PT_EINVAL, "null batch");
  if (mcs < 0) return pt_fail(PT_EINVAL, "pt_batch_run: mcs must be >= 0");
  if (flags & ~(uint32_t)(PT_MCS_HOUDAYER | PT_MCS_MEASURE | PT_MCS_MULTICLUSTER | PT_BATCH_GRAPH))
    return pt_fail(PT_EINVAL, "pt_batch_run: unknown flags");
  if ((flags & PT_MCS_MULTICLUSTER) && !(flags & PT_MCS_HOUDAYER))
    return pt_fail(PT_EINVAL, "pt_batch_run: PT_MCS_MULTICLUSTER needs PT_MCS_HOUDAYER");
  for (pt_job* j : b->jobs)
    if (j->poisoned) return pt_fail(PT_ESTATE, "pt_batch_run: a job is poisoned");
  if (mcs == 0) return PT_OK;
  const uint32_t work_flags = flags & (PT_MCS_HOUDAYER | PT_MCS_MEASURE | PT_MCS_MULTICLUSTER);
  if (int rc = build_worklist(b, mcs, work_flags)) return rc;
  const int rc = run_once(b, (flags & PT_BATCH_GRAPH) != 0);
  if (rc != PT_OK) {
    for (pt_job* j : b->jobs) j->poisoned = true;
    return rc;
  }
  return run_unplanned(b, mcs, work_flags);
}

PT_API int pt_batch_get_config(pt_batch* b, int32_t* cfg3) {
  if (!b || !cfg3) return pt_fail(PT_EINVAL, "null argument");
  cfg3[0] = b->cfg.threads == 0 && b->built ? b->threads : b->cfg.threads;
  cfg3[1] = b->cfg.sets;
  cfg3[2] = b->cfg.order;
  return PT_OK;
}

PT_API int pt_batch_launch_shape(pt_batch* b, int32_t* out3) {
  if (!b || !out3) return pt_fail(PT_EINVAL, "null argument");
  out3[0] = b->blocks;
  out3[1] = b->threads;
  out3[2] = b->per_cu;
  return PT_OK;
}

PT_API int pt_batch_set_config(pt_batch* b, int32_t threads, int32_t sets, int32_t order) {
  if (!b) return pt_fail(PT_EINVAL, "null batch");
  if (threads < 0 || threads > 1024 || threads % 64 != 0 || (sets != 1 && sets != 2) ||
      (order != 0 && order != 1))
    return pt_fail(PT_EINVAL,
                   "pt_batch_set_config: threads 0 (auto) or a multiple of 64 up to 1024, sets in "
                   "{1,2}, order in {0,1}");
  b->cfg = BatchConfig{threads, sets, order};
  return PT_OK;
}

PT_API int pt_batch_tune(pt_batch* b, int32_t trial_mcs, uint32_t flags, const char* cache_path) {
  if (!b) return pt_fail(PT_EINVAL, "null batch");
  if (trial_mcs < 1) return pt_fail(PT_EINVAL, "pt_batch_tune: trial_mcs must be >= 1");
  const uint32_t work_flags = flags & (PT_MCS_HOUDAYER | PT_MCS_MEASURE | PT_MCS_MULTICLUSTER);
  const bool try_layouts = (flags & PT_TUNE_LAYOUT) != 0;
  const std::string key = cache_key(b, work_flags | (try_layouts ? PT_TUNE_LAYOUT : 0u));
  BatchConfig cached;
  int cached_layout = -1;
  if (cache_lookup(cache_path, key, cached, &cached_layout)) {
    if (try_layouts && cached_layout >= 0)
      if (int rc = set_layout_all(b, cached_layout)) return rc;
    b->cfg = cached;
    return PT_OK;
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const BatchConfig start = b->cfg;
  BatchConfig best = start;
  int best_layout = -1;
  double best_ms = 1e300;
  int rc = PT_OK;
  // with PT_TUNE_LAYOUT every configuration is timed with all jobs in the
  // int8 layout, then in the packed one (the conversion is exact, so both
  // start from the same state); otherwise in the jobs' own layouts
  const std::vector<int> layouts = try_layouts ? std::vector<int>{(int)PT_LAYOUT_INT8, (int)PT_LAYOUT_PACKED}
                                               : std::vector<int>{-1};
  bool warmed = false;
  for (int layout : layouts) {
    if (rc != PT_OK) break;
    if (layout >= 0 && (rc = set_layout_all(b, layout))) break;
    Snap sn;
    rc = snapshot(b, sn, false);
    if (rc == PT_OK && !warmed) {
      // one untimed trial first (the GPU clock and the caches settle), then
      // each configuration timed twice from the same state, keeping its
      // faster run
      b->cfg = start;
      rc = build_worklist(b, trial_mcs, work_flags);
      if (rc == PT_OK) rc = run_once(b, false);
      if (rc == PT_OK) rc = snapshot(b, sn, true);
      warmed = true;
    }
    for (int threads : {1024, 768, 512, 256}) {
      for (int sets : {2, 1}) {
        for (int order : {0, 1}) {
          if (rc != PT_OK) break;
          b->cfg = BatchConfig{threads, sets, order};
          if ((rc = build_worklist(b, trial_mcs, work_flags))) break;
          double cfg_ms = 1e300;
          for (int rep = 0; rep < 2 && rc == PT_OK; ++rep) {
            (void)hipEventRecord(e0, b->stream);
            if ((rc = run_once(b, false))) break;
            (void)hipEventRecord(e1, b->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < cfg_ms) cfg_ms = ms;
            rc = snapshot(b, sn, true);
          }
          if (rc == PT_OK && cfg_ms < best_ms) {
            best_ms = cfg_ms;
            best = b->cfg;
            best_layout = layout;
          }
        }
      }
    }
    for (void* p : sn.bufs) (void)hipFree(p);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PT_OK) {
    b->cfg = start;
    return rc;
  }
  // the jobs hold their starting state, in the last layout tried
  if (best_layout >= 0 && (rc = set_layout_all(b, best_layout))) return rc;
  b->cfg = best;
  cache_store(cache_path, key, best, best_layout, best_ms);
  return PT_OK;
}

PT_API int pt_batch_destroy(pt_batch* b) {
  if (!b) return pt_fail(PT_EINVAL, "null batch");
  (void)hipStreamSynchronize(b->stream);
  batch_free(b);
  return PT_OK;
}
