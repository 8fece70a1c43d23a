// server.hip -- continuous-batching request server for parallel-tempering jobs.
//
// Requests are admitted in arrival order while their device memory fits the
// HBM budget, stay resident on the device, and advance together: every round
// runs up to `steps_per_round` Monte Carlo steps of every active job in one
// persistent batch launch (jobs with no workgroup plan run their per-step
// kernels on a second stream at the same time).  A job measures only after
// its burn-in.  While a round runs on the GPU, the worker thread reads out
// and releases the jobs that finished in the previous round and creates the
// newly admitted ones on a third stream, from a stream-ordered memory pool,
// so that job set-up and tear-down overlap the rounds.  Admitted requests get
// their jobs created only while the round in flight still runs (the rest
// wait, their memory reserved, for the next round), so that a large admission
// never holds the GPU idle between rounds.  Results depend only on
// the request, never on what else ran beside it.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <limits>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "job.h"
#include "pt.h"

namespace {

struct Request {
  uint64_t ticket = 0;
  int dim = 3, L = 0, NT = 0, S = 0, sweeps = 0, burn_in = 0, every = 1;
  uint32_t flags = 0, layout = 0;
  uint64_t seed = 0;
  std::vector<double> betas;
  std::vector<int8_t> J;
  double t_submit = 0;
};

struct Active {
  Request req;
  pt_job* job = nullptr;
  int done = 0;
  size_t bytes = 0;
  double t_admit = 0;
};

struct Finished {
  int status = 0;
  int64_t n_meas = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::vector<double> disorder;  // [NT][6]
  double tau = 0;                // round-trip time (walk kept), else NaN
  int equilibrated = -1;         // its logarithmic-binning check, else -1
  std::vector<double> corr;      // [NT][3] chi_SG(0), chi_SG(k_min), xi (modes kept), else NaN
};

// Round-trip summary of a job keeping the replica walk (Sec. 2.3): mean trip
// length and the logarithmic-binning check after the job's exchange passes.
int walk_summary(pt_job* job, double& tau, int& eq) {
  std::vector<uint64_t> trips((size_t)job->g.S * 32 * 3);
  uint64_t ctr[4];
  if (int rc = pt_get_walk(job, nullptr, nullptr, trips.data())) return rc;
  if (int rc = pt_get_counters(job, ctr)) return rc;
  int32_t e = 0;
  if (int rc = pt_tunnel_summary(trips.data(), job->g.S, ctr[1], nullptr, nullptr, &tau, &e)) return rc;
  eq = e;
  return PT_OK;
}

}  // namespace

struct pt_server {
  size_t budget = 0, used = 0;
  int steps_per_round = 100;
  int device = 0;
  // st_main: the 3D batch launch of a round; st_two: the 2D one (the two
  // run side by side); st_side: per-step jobs; st_admit: job set-up and
  // tear-down
  hipStream_t st_main = nullptr, st_two = nullptr, st_side = nullptr, st_admit = nullptr;
  hipMemPool_t pool = nullptr;  // device memory of the jobs
  // Pinned host blocks the set-up copies of the jobs created during one round
  // read from (bump-allocated; reused once that set-up has completed, which
  // admit_ev marks), and the event every stream of the next round waits for.
  std::vector<std::pair<char*, size_t>> stage_blocks;
  size_t stage_block = 0, stage_used = 0;
  hipEvent_t admit_ev = nullptr;
  pt_batch* batch[2] = {nullptr, nullptr};  // 2D and 3D jobs
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Request> pending;
  std::vector<Active> active;
  std::unordered_map<uint64_t, Finished> finished;
  std::unordered_set<uint64_t> live;    // admitted requests not finished yet
  std::unordered_set<uint64_t> cancel;  // live requests to end between rounds
  size_t n_active = 0;                  // jobs of the current round
  size_t n_staged = 0;                  // admitted, memory reserved, job not created yet
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::thread worker;
  std::chrono::steady_clock::time_point t0;
  // statistics
  double flips = 0, busy = 0;
  uint64_t rounds = 0, admitted = 0, completed = 0, cancelled = 0;
  size_t peak_used = 0;
  int max_active = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// Job memory from the server's stream-ordered pool: allocated and released
// on st_admit, never while a round that uses it can still run.
void* pool_alloc(size_t bytes, void* ctx) {
  pt_server* sv = static_cast<pt_server*>(ctx);
  void* p = nullptr;
  if (hipMallocFromPoolAsync(&p, bytes, sv->pool, sv->st_admit) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void pool_free(void* p, void* ctx) {
  pt_server* sv = static_cast<pt_server*>(ctx);
  (void)hipFreeAsync(p, sv->st_admit);
}

// Pinned host memory for one job's set-up copies (see stage_blocks).
void* stage_take(size_t bytes, void* ctx) {
  pt_server* sv = static_cast<pt_server*>(ctx);
  bytes = (bytes + 255) & ~(size_t)255;
  while (sv->stage_block < sv->stage_blocks.size() &&
         sv->stage_used + bytes > sv->stage_blocks[sv->stage_block].second) {
    ++sv->stage_block;
    sv->stage_used = 0;
  }
  if (sv->stage_block == sv->stage_blocks.size()) {
    const size_t cap = bytes > ((size_t)8 << 20) ? bytes : ((size_t)8 << 20);
    void* p = nullptr;
    if (hipHostMalloc(&p, cap, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    sv->stage_blocks.push_back({static_cast<char*>(p), cap});
    sv->stage_used = 0;
  }
  char* p = sv->stage_blocks[sv->stage_block].first + sv->stage_used;
  sv->stage_used += bytes;
  return p;
}

void finish(pt_server* sv, Active& a, int status) {
  if (a.job) a.job->stream = sv->st_admit;  // the next round may already run on st_main
  Finished f;
  f.status = status;
  f.t_submit = a.req.t_submit;
  f.t_admit = a.t_admit;
  f.disorder.assign((size_t)a.req.NT * 6, 0.0);
  f.tau = std::numeric_limits<double>::quiet_NaN();
  f.corr.assign((size_t)a.req.NT * 3, std::numeric_limits<double>::quiet_NaN());
  if (status == PT_OK && a.job) {
    int64_t n = 0;
    int rc = pt_observables(a.job, nullptr, f.disorder.data(), &n);
    if (rc == PT_OK && a.job->track_walk) rc = walk_summary(a.job, f.tau, f.equilibrated);
    if (rc == PT_OK && a.job->track_modes) {
      std::vector<double> c0(a.req.NT), ck(a.req.NT), xi(a.req.NT);
      rc = pt_correlation_length(a.job, c0.data(), ck.data(), xi.data());
      for (int k = 0; k < a.req.NT; ++k) {
        f.corr[(size_t)k * 3 + 0] = c0[k];
        f.corr[(size_t)k * 3 + 1] = ck[k];
        f.corr[(size_t)k * 3 + 2] = xi[k];
      }
    }
    if (rc != PT_OK) f.status = rc;
    f.n_meas = n;
  }
  if (a.job) pt_destroy(a.job);
  a.job = nullptr;
  f.t_done = sv->now();
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->used -= a.bytes;
  if (status == PT_ECANCELED)
    sv->cancelled += 1;
  else
    sv->completed += 1;
  sv->cancel.erase(a.req.ticket);
  sv->live.erase(a.req.ticket);
  sv->finished[a.req.ticket] = std::move(f);
  sv->cv_done.notify_all();
}

void fail_request(pt_server* sv, const Request& r, int status) {
  Finished f;
  f.status = status;
  f.t_submit = r.t_submit;
  f.t_admit = f.t_done = sv->now();
  f.disorder.assign((size_t)r.NT * 6, 0.0);
  f.tau = std::numeric_limits<double>::quiet_NaN();
  f.corr.assign((size_t)r.NT * 3, std::numeric_limits<double>::quiet_NaN());
  sv->finished[r.ticket] = std::move(f);
  sv->cv_done.notify_all();
}

// Moves queued requests to `staged` in arrival order while the budget holds
// (their memory is reserved from then on).
void take_admissions(pt_server* sv, std::deque<Request>& staged) {
  std::lock_guard<std::mutex> lk(sv->mu);
  size_t used = sv->used;
  while (!sv->pending.empty()) {
    Request& r = sv->pending.front();
    const size_t need = job_device_bytes(r.S, r.NT, r.L, r.dim, (int)r.layout, r.betas.data());
    if (need > sv->budget) {
      fail_request(sv, r, PT_ENOMEM);
      sv->pending.pop_front();
      continue;
    }
    if (used + need > sv->budget) break;
    used += need;
    sv->live.insert(r.ticket);
    staged.push_back(std::move(r));
    sv->pending.pop_front();
  }
  sv->used = used;
  sv->n_staged = staged.size();
  if (used > sv->peak_used) sv->peak_used = used;
}

// Creates admitted jobs on st_admit (they join the next round), oldest
// first, while `staged` is not empty and more() holds; at least one job is
// created per call.  A staged request cancelled meanwhile ends here without a
// job.
template <class More>
void create_jobs(pt_server* sv, std::deque<Request>& staged, std::vector<Active>& ready, More more) {
  if (staged.empty()) return;
  // the set-up queued by the last call has completed before the round that
  // is now running started (it waited for admit_ev): its staging is free
  (void)hipEventSynchronize(sv->admit_ev);
  sv->stage_block = 0;
  sv->stage_used = 0;
  bool first = true;
  while (!staged.empty() && (first || more())) {
    first = false;
    Request r = std::move(staged.front());
    staged.pop_front();
    Active a;
    a.bytes = job_device_bytes(r.S, r.NT, r.L, r.dim, (int)r.layout, r.betas.data());
    a.t_admit = sv->now();
    bool gone;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->n_staged = staged.size();
      gone = sv->cancel.erase(r.ticket) > 0;
    }
    if (gone) {
      a.req = std::move(r);
      finish(sv, a, PT_ECANCELED);
      continue;
    }
    const int rc = job_create(&a.job, r.S, r.NT, r.L, r.dim, r.J.data(), r.betas.data(), r.seed,
                              r.layout, pool_alloc, pool_free, sv, sv->st_admit, stage_take);
    a.req = std::move(r);
    a.req.J.clear();
    a.req.J.shrink_to_fit();
    if (rc != PT_OK) {
      a.job = nullptr;
      finish(sv, a, rc);
      continue;
    }
    a.job->stream = sv->st_main;
    a.job->meas_every = a.req.every;
    ready.push_back(std::move(a));
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->admitted += 1;
  }
  (void)hipEventRecord(sv->admit_ev, sv->st_admit);
}

// Orders the next round's streams after the set-up of the jobs created so far.
hipError_t wait_admitted(pt_server* sv) {
  hipError_t e = hipSuccess;
  for (hipStream_t st : {sv->st_main, sv->st_two, sv->st_side})
    if (e == hipSuccess) e = hipStreamWaitEvent(st, sv->admit_ev, 0);
  return e;
}

// Job creation time allowed before the first round of an idle server.
constexpr double kFirstFill = 0.005;

// Whether work of the round in flight is still queued or running.
bool round_running(const pt_server* sv) {
  for (hipStream_t st : {sv->st_main, sv->st_two, sv->st_side})
    if (hipStreamQuery(st) == hipErrorNotReady) return true;
  return false;
}

void serve(pt_server* sv) {
  (void)hipSetDevice(sv->device);
  std::vector<Active> done;    // finished in the last round, not yet read out
  std::deque<Request> staged;  // admitted, memory reserved, job not created yet
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait(lk, [&] {
        return sv->stopping || !sv->pending.empty() || !sv->active.empty() || !done.empty() ||
               !staged.empty();
      });
      if (sv->stopping && sv->pending.empty() && sv->active.empty() && done.empty() && staged.empty())
        break;
    }
    {
      // cancelled running jobs end here, between rounds (nothing of theirs is
      // on the GPU); the other jobs are not touched
      std::vector<Active> keep, gone;
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (Active& a : sv->active) {
          if (sv->cancel.erase(a.req.ticket))
            gone.push_back(std::move(a));
          else
            keep.push_back(std::move(a));
        }
        // admitted requests whose jobs were not created yet end without one
        for (auto it = staged.begin(); it != staged.end();) {
          if (sv->cancel.erase(it->ticket)) {
            Active a;
            a.bytes = job_device_bytes(it->S, it->NT, it->L, it->dim, (int)it->layout, it->betas.data());
            a.t_admit = sv->now();
            a.req = std::move(*it);
            gone.push_back(std::move(a));
            it = staged.erase(it);
          } else {
            ++it;
          }
        }
        sv->n_staged = staged.size();
      }
      sv->active.swap(keep);
      for (Active& a : gone) finish(sv, a, PT_ECANCELED);
    }
    if (sv->active.empty()) {
      // nothing on the GPU: read out, then admit, and start a round with the
      // jobs created within a few milliseconds; the other admitted requests
      // are created while it runs
      for (Active& a : done) finish(sv, a, PT_OK);
      done.clear();
      take_admissions(sv, staged);
      const double until = sv->now() + kFirstFill;
      create_jobs(sv, staged, sv->active, [&] { return sv->now() < until; });
      if (sv->active.empty()) continue;
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->n_active = sv->active.size();
      if ((int)sv->n_active > sv->max_active) sv->max_active = (int)sv->n_active;
    }

    // one round: every active job advances, measuring after its burn-in
    const double t_round = sv->now();
    std::vector<pt_job*> res_jobs[2];
    std::vector<int> res_steps[2];
    std::vector<uint32_t> res_flags[2];
    std::vector<size_t> side;
    double round_flips = 0;
    std::vector<int> steps(sv->active.size());
    std::vector<uint32_t> flags(sv->active.size());
    // Round length: steps_per_round steps of the job with the largest work
    // item.  When every item gets a workgroup of its own, jobs with smaller
    // items take proportionally more steps, so that all items of the round
    // last about as long and no workgroup idles until the round ends.
    std::vector<double> item_flips(sv->active.size());
    int total_items = 0;
    double f_max = 0;
    for (size_t i = 0; i < sv->active.size(); ++i) {
      Active& a = sv->active[i];
      const uint32_t f = (a.req.flags & (PT_MCS_HOUDAYER | PT_MCS_MULTICLUSTER)) |
                         (a.done < a.req.burn_in ? 0u : (uint32_t)PT_MCS_MEASURE);
      int items = 0;
      job_items(a.job, f, items, item_flips[i]);
      total_items += items;
      if (item_flips[i] > f_max) f_max = item_flips[i];
    }
    const bool stretch = total_items <= batch_slots(sv->batch[1]);
    for (size_t i = 0; i < sv->active.size(); ++i) {
      Active& a = sv->active[i];
      const int left = a.req.sweeps - a.done;
      int quota = sv->steps_per_round;
      if (stretch && item_flips[i] > 0) {
        const double q = (double)sv->steps_per_round * f_max / item_flips[i];
        quota = q > 1e9 ? 1000000000 : (int)q;
      }
      int n = left < quota ? left : quota;
      uint32_t f = a.req.flags & (PT_MCS_HOUDAYER | PT_MCS_MULTICLUSTER);
      if (a.done < a.req.burn_in) {
        const int to_burn = a.req.burn_in - a.done;
        if (n > to_burn) n = to_burn;
      } else {
        f |= PT_MCS_MEASURE;
      }
      steps[i] = n;
      flags[i] = f;
      round_flips += (double)n * a.job->g.S * a.job->g.nslot * a.job->g.N;
      if (job_is_resident(a.job, f)) {
        const int b = a.job->g.d == 3 ? 1 : 0;
        res_jobs[b].push_back(a.job);
        res_steps[b].push_back(n);
        res_flags[b].push_back(f);
      } else {
        side.push_back(i);
      }
    }
    int rc = wait_admitted(sv) == hipSuccess ? PT_OK : PT_EDEVICE;
    for (int b = 0; b < 2 && rc == PT_OK; ++b)
      rc = batch_round(sv->batch[b], res_jobs[b], res_steps[b], res_flags[b]);
    for (size_t i : side) {
      if (rc != PT_OK) break;
      Active& a = sv->active[i];
      a.job->stream = sv->st_side;
      rc = pt_mcs(a.job, steps[i], flags[i]);
      a.job->stream = sv->st_main;
    }

    // while the round runs: read out and release the last round's finished
    // jobs, then create the newly admitted ones
    for (Active& a : done) finish(sv, a, PT_OK);
    done.clear();
    std::vector<Active> ready;
    if (rc == PT_OK) {
      take_admissions(sv, staged);
      create_jobs(sv, staged, ready, [&] { return round_running(sv); });
    }

    if (rc == PT_OK && hipStreamSynchronize(sv->st_main) != hipSuccess) rc = PT_EDEVICE;
    if (rc == PT_OK && hipStreamSynchronize(sv->st_two) != hipSuccess) rc = PT_EDEVICE;
    if (rc == PT_OK && hipStreamSynchronize(sv->st_side) != hipSuccess) rc = PT_EDEVICE;
    // the set-up queued during this round runs once the round has freed the
    // CUs; a failure of it shows here or at the next round's sync
    const hipError_t qa = hipStreamQuery(sv->st_admit);
    if (rc == PT_OK && qa != hipSuccess && qa != hipErrorNotReady) rc = PT_EDEVICE;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->busy += sv->now() - t_round;
      sv->rounds += 1;
      if (rc == PT_OK) sv->flips += round_flips;
    }
    // completions
    std::vector<Active> still;
    for (size_t i = 0; i < sv->active.size(); ++i) {
      Active& a = sv->active[i];
      if (rc != PT_OK) {
        finish(sv, a, rc);
        continue;
      }
      a.done += steps[i];
      bool end = a.done >= a.req.sweeps;
      if (!end && (a.req.flags & PT_SERVE_UNTIL_EQUILIBRATED) && a.done > a.req.burn_in) {
        // ends early once its round trips pass the logarithmic-binning check
        double tau = 0;
        int eq = 0;
        if (walk_summary(a.job, tau, eq) == PT_OK && eq == 1) end = true;
      }
      if (end)
        done.push_back(std::move(a));
      else
        still.push_back(std::move(a));
    }
    for (Active& a : ready) still.push_back(std::move(a));
    sv->active.swap(still);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->n_active = sv->active.size();
  }
}

}  // namespace

// ---------------------------------------------------------------------------
PT_API int pt_server_start(size_t hbm_budget, int32_t steps_per_round, pt_server** out) {
  if (!out || hbm_budget == 0 || steps_per_round < 1)
    return pt_fail(PT_EINVAL, "pt_server_start: need a budget > 0, steps_per_round >= 1, an output");
  pt_server* sv = new (std::nothrow) pt_server();
  if (!sv) return pt_fail(PT_ENOMEM, "pt_server_start: host allocation failed");
  sv->budget = hbm_budget;
  sv->steps_per_round = steps_per_round;
  sv->t0 = std::chrono::steady_clock::now();
  (void)hipGetDevice(&sv->device);
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = sv->device;
  uint64_t keep = UINT64_MAX;  // freed blocks stay in the pool for reuse
  if (hipStreamCreateWithFlags(&sv->st_main, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->st_two, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->st_side, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->st_admit, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&sv->admit_ev, hipEventDisableTiming) != hipSuccess ||
      hipMemPoolCreate(&sv->pool, &props) != hipSuccess ||
      hipMemPoolSetAttribute(sv->pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
    (void)hipGetLastError();
    if (sv->st_main) (void)hipStreamDestroy(sv->st_main);
    if (sv->st_two) (void)hipStreamDestroy(sv->st_two);
    if (sv->st_side) (void)hipStreamDestroy(sv->st_side);
    if (sv->st_admit) (void)hipStreamDestroy(sv->st_admit);
    if (sv->admit_ev) (void)hipEventDestroy(sv->admit_ev);
    if (sv->pool) (void)hipMemPoolDestroy(sv->pool);
    delete sv;
    return pt_fail(PT_EDEVICE, "pt_server_start: stream or memory pool creation failed");
  }
  sv->batch[0] = batch_new(sv->st_two);
  sv->batch[1] = batch_new(sv->st_main);
  if (!sv->batch[0] || !sv->batch[1]) {
    batch_free(sv->batch[0]);
    batch_free(sv->batch[1]);
    delete sv;
    return pt_fail(PT_ENOMEM, "pt_server_start: host allocation failed");
  }
  sv->worker = std::thread(serve, sv);
  *out = sv;
  return PT_OK;
}

PT_API int pt_server_submit(pt_server* sv, const pt_request* req, uint64_t* ticket) {
  if (!sv || !req || !ticket) return pt_fail(PT_EINVAL, "pt_server_submit: null argument");
  if (!req->betas || !req->couplings) return pt_fail(PT_EINVAL, "pt_server_submit: null arrays");
  if (req->dim != 2 && req->dim != 3) return pt_fail(PT_EINVAL, "pt_server_submit: dim must be 2 or 3");
  if (req->L < 4 || req->L > 64 || (req->L & 1))
    return pt_fail(PT_EINVAL, "pt_server_submit: L must be even and in [4, 64]");
  if (req->samples < 1 || req->replicas < 2 || req->sweeps < 0 || req->burn_in < 0 ||
      req->burn_in > req->sweeps)
    return pt_fail(PT_EINVAL, "pt_server_submit: need samples >= 1, replicas >= 2, 0 <= burn_in <= sweeps");
  if (req->measure_every < 0) return pt_fail(PT_EINVAL, "pt_server_submit: measure_every must be >= 0");
  if (req->flags & ~(uint32_t)(PT_MCS_HOUDAYER | PT_MCS_MULTICLUSTER | PT_SERVE_UNTIL_EQUILIBRATED))
    return pt_fail(PT_EINVAL, "pt_server_submit: unknown flags");
  if ((req->flags & PT_MCS_MULTICLUSTER) &&
      (!(req->flags & PT_MCS_HOUDAYER) ||
       (req->dim == 3 ? (long)req->L * req->L * req->L : (long)req->L * req->L) > 32768))
    return pt_fail(PT_EINVAL, "pt_server_submit: PT_MCS_MULTICLUSTER needs PT_MCS_HOUDAYER and "
                              "L^dim <= 32768");
  const uint32_t layout = req->layout & ~(uint32_t)(PT_TRACK_WALK | PT_TRACK_MODES);
  if (layout != PT_LAYOUT_INT8 && layout != PT_LAYOUT_PACKED)
    return pt_fail(PT_EINVAL, "pt_server_submit: unknown layout");
  if ((req->flags & PT_SERVE_UNTIL_EQUILIBRATED) && !(req->layout & PT_TRACK_WALK))
    return pt_fail(PT_EINVAL, "pt_server_submit: stopping at equilibrium needs PT_TRACK_WALK");
  for (int k = 0; k < req->replicas; ++k)
    if (!(req->betas[k] > 0.0) || (k > 0 && !(req->betas[k] < req->betas[k - 1])))
      return pt_fail(PT_EINVAL, "pt_server_submit: betas must be > 0 and strictly decreasing");
  const size_t N = req->dim == 3 ? (size_t)req->L * req->L * req->L : (size_t)req->L * req->L;
  const size_t nJ = (size_t)req->samples * req->dim * N;
  for (size_t i = 0; i < nJ; ++i)
    if (req->couplings[i] != 1 && req->couplings[i] != -1)
      return pt_fail(PT_EINVAL, "pt_server_submit: couplings must be +1 or -1");
  Request r;
  r.dim = req->dim;
  r.L = req->L;
  r.NT = req->replicas;
  r.S = req->samples;
  r.sweeps = req->sweeps;
  r.burn_in = req->burn_in;
  r.every = req->measure_every < 1 ? 1 : req->measure_every;
  r.flags = req->flags;
  r.layout = req->layout;
  r.seed = req->seed;
  r.betas.assign(req->betas, req->betas + req->replicas);
  r.J.assign(req->couplings, req->couplings + nJ);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stopping) return pt_fail(PT_ESTATE, "pt_server_submit: server is stopping");
  r.ticket = sv->next_ticket++;
  r.t_submit = sv->now();
  *ticket = r.ticket;
  sv->pending.push_back(std::move(r));
  sv->cv.notify_all();
  return PT_OK;
}

PT_API int pt_server_poll(pt_server* sv, uint64_t ticket, pt_result* out, double* disorder) {
  return pt_server_poll_ex(sv, ticket, out, disorder, nullptr);
}

PT_API int pt_server_poll_ex(pt_server* sv, uint64_t ticket, pt_result* out, double* disorder,
                             double* correlation) {
  if (!sv || !out) return pt_fail(PT_EINVAL, "pt_server_poll: null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->finished.find(ticket);
  if (it == sv->finished.end()) {
    if (ticket == 0 || ticket >= sv->next_ticket) return pt_fail(PT_EINVAL, "pt_server_poll: unknown ticket");
    return 1;  // queued or running
  }
  const Finished& f = it->second;
  out->status = f.status;
  out->n_meas = f.n_meas;
  out->t_submit = f.t_submit;
  out->t_admit = f.t_admit;
  out->t_done = f.t_done;
  out->equilibrated = f.equilibrated;
  out->tau_tunnel = f.tau;
  if (disorder) std::copy(f.disorder.begin(), f.disorder.end(), disorder);
  if (correlation) std::copy(f.corr.begin(), f.corr.end(), correlation);
  sv->finished.erase(it);
  return PT_OK;
}

PT_API int pt_server_cancel(pt_server* sv, uint64_t ticket) {
  if (!sv) return pt_fail(PT_EINVAL, "pt_server_cancel: null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticket == 0 || ticket >= sv->next_ticket) return pt_fail(PT_EINVAL, "pt_server_cancel: unknown ticket");
  if (sv->finished.count(ticket)) return 1;  // its result is waiting to be polled
  for (auto it = sv->pending.begin(); it != sv->pending.end(); ++it) {
    if (it->ticket != ticket) continue;
    Finished f;
    f.status = PT_ECANCELED;
    f.t_submit = it->t_submit;
    f.t_admit = f.t_done = sv->now();
    f.disorder.assign((size_t)it->NT * 6, 0.0);
    f.tau = std::numeric_limits<double>::quiet_NaN();
    f.corr.assign((size_t)it->NT * 3, std::numeric_limits<double>::quiet_NaN());
    sv->finished[ticket] = std::move(f);
    sv->pending.erase(it);
    sv->cancelled += 1;
    sv->cv_done.notify_all();
    return PT_OK;
  }
  if (!sv->live.count(ticket)) return pt_fail(PT_EINVAL, "pt_server_cancel: result already collected");
  // admitted: the worker ends it at the next round boundary unless it has
  // completed its steps by then
  sv->cancel.insert(ticket);
  sv->cv.notify_all();
  return PT_OK;
}

PT_API int pt_server_stats(pt_server* sv, double* out) {
  if (!sv || !out) return pt_fail(PT_EINVAL, "pt_server_stats: null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  out[0] = sv->flips;
  out[1] = sv->busy;
  out[2] = (double)sv->rounds;
  out[3] = (double)sv->admitted;
  out[4] = (double)sv->completed;
  out[5] = (double)sv->peak_used;
  out[6] = (double)sv->max_active;
  out[7] = sv->now();
  out[8] = (double)(sv->pending.size() + sv->n_staged);
  out[9] = (double)sv->n_active;
  out[10] = (double)sv->cancelled;
  return PT_OK;
}

PT_API int pt_server_stop(pt_server* sv) {
  if (!sv) return pt_fail(PT_EINVAL, "null server");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
    sv->cv.notify_all();
  }
  if (sv->worker.joinable()) sv->worker.join();
  batch_free(sv->batch[0]);
  batch_free(sv->batch[1]);
  (void)hipStreamSynchronize(sv->st_admit);
  for (auto& blk : sv->stage_blocks) (void)hipHostFree(blk.first);
  (void)hipEventDestroy(sv->admit_ev);
  (void)hipStreamDestroy(sv->st_main);
  (void)hipStreamDestroy(sv->st_two);
  (void)hipStreamDestroy(sv->st_side);
  (void)hipStreamDestroy(sv->st_admit);
  (void)hipMemPoolDestroy(sv->pool);
  (void)hipGetLastError();
  delete sv;
  return PT_OK;
}
