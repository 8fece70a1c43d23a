// sanitize_runtime.cpp -- test driver, not part of the library.
//
// Exercises the host side of libptsg's C ABI on a machine without a GPU: the
// argument checks of every entry point (each refusal must leave the handle
// untouched and set a message), the host-only planners (pt_plan_query,
// pt_job_bytes over every lattice shape), the round-trip summary, the
// Gaussian acceptance decision on the host, and the failure paths of job,
// batch and server creation when no device is present.  Built from
// host-only objects with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py; any report ends the run with a non-zero status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "pt.h"

namespace {
int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (%s)\n", what, pt_last_error());
    ++failures;
  }
}

void refusal(int rc, const char* what) {
  expect(rc == PT_EINVAL, what);
  expect(std::strlen(pt_last_error()) > 0, what);
}
}  // namespace

int main() {
  expect(std::strncmp(pt_version(), "ptsg", 4) == 0, "version");

  // host-only planners over every accepted shape and flag combination
  const uint32_t flag_sets[] = {0u, PT_MCS_MEASURE, PT_MCS_HOUDAYER | PT_MCS_MEASURE,
                                PT_MCS_HOUDAYER | PT_MCS_MULTICLUSTER | PT_MCS_MEASURE,
                                PT_MCS_MEASURE | PT_TRACK_WALK, PT_MCS_MEASURE | PT_TRACK_MODES};
  const int ladders[] = {2, 3, 16, 24, 32, 48, 64, 65, 160};
  for (int d = 2; d <= 3; ++d)
    for (int L = 4; L <= 64; L += 2)
      for (int NT : ladders) {
        std::vector<double> betas(NT);
        for (int k = 0; k < NT; ++k) betas[k] = 1.0 / (0.5 + 1.5 * k / (NT - 1));
        for (uint32_t f : flag_sets) {
          int32_t plan[4] = {-9, -9, -9, -9};
          const int rc = pt_plan_query(d, L, NT, f, plan);
          expect(rc == PT_OK && plan[0] >= -1 && plan[0] <= 4, "plan query");
        }
        uint64_t bytes = 0;
        for (uint32_t lay : {PT_LAYOUT_INT8, PT_LAYOUT_PACKED, PT_LAYOUT_INT8 | PT_TRACK_WALK,
                             PT_LAYOUT_PACKED | PT_TRACK_MODES})
          expect(pt_job_bytes(3, NT, L, d, lay, betas.data(), &bytes) == PT_OK && bytes > 0,
                 "job bytes");
      }
  int32_t plan[4];
  refusal(pt_plan_query(4, 16, 8, 0, plan), "plan query dim 4");
  refusal(pt_plan_query(3, 15, 8, 0, plan), "plan query odd L");
  refusal(pt_plan_query(3, 16, 8, 0, nullptr), "plan query null output");

  // round-trip summary: sparse and dense bins, one and several rows
  std::vector<uint64_t> trips(3 * 32 * 3, 0);
  for (int r = 0; r < 3; ++r)
    for (int b = 3; b < 12; ++b) {
      uint64_t* t = &trips[(r * 32 + b) * 3];
      const uint64_t n = 2 + b + r, len = 40 + 3 * b;
      t[0] = n;
      t[1] = n * len + (uint64_t)r;
      t[2] = n * len * len + 7 * (uint64_t)b;
    }
  double tau_b[32], err_b[32], tau = 0;
  int32_t eq = -1;
  expect(pt_tunnel_summary(trips.data(), 3, 4000, tau_b, err_b, &tau, &eq) == PT_OK, "summary");
  expect(pt_tunnel_summary(trips.data(), 1, 1, nullptr, nullptr, nullptr, nullptr) == PT_OK,
         "summary, no outputs");
  refusal(pt_tunnel_summary(nullptr, 1, 10, tau_b, err_b, &tau, &eq), "summary null trips");
  refusal(pt_tunnel_summary(trips.data(), 0, 10, tau_b, err_b, &tau, &eq), "summary no rows");

  // the Gaussian acceptance decision on the host across its range
  uint32_t r = 12345u;
  for (int i = 0; i < 20000; ++i) {
    r = r * 1664525u + 1013904223u;
    const double b = 0.05 + 0.001 * (i % 3000);
    const int64_t u = 1 + (int64_t)((uint64_t)r * 2654435761u % (1ull << 24));
    const int a = pt_gauss_accept_host(r, b, u);
    expect(a == 0 || a == 1, "gauss accept");
  }

  // argument checks of job creation: nothing is created
  std::vector<int8_t> J(2 * 3 * 512, 1);
  const double betas3[3] = {1.0, 0.7, 0.4};
  pt_job* job = nullptr;
  refusal(pt_init(&job, 2, 3, 8, 4, J.data(), betas3, 1), "init dim");
  refusal(pt_init(&job, 2, 3, 7, 3, J.data(), betas3, 1), "init odd L");
  refusal(pt_init(&job, 0, 3, 8, 3, J.data(), betas3, 1), "init samples");
  refusal(pt_init(&job, 2, 1, 8, 3, J.data(), betas3, 1), "init replicas");
  refusal(pt_init(&job, 2, 3, 8, 3, nullptr, betas3, 1), "init null couplings");
  refusal(pt_init(&job, 2, 3, 8, 3, J.data(), nullptr, 1), "init null betas");
  const double bad_betas[3] = {1.0, 1.0, 0.4};
  refusal(pt_init(&job, 2, 3, 8, 3, J.data(), bad_betas, 1), "init betas order");
  J[17] = 0;
  refusal(pt_init(&job, 2, 3, 8, 3, J.data(), betas3, 1), "init coupling value");
  J[17] = 1;
  refusal(pt_init_ex(&job, 2, 3, 8, 3, J.data(), betas3, 1, 0x7u), "init flags");
  std::vector<float> G(2 * 3 * 512, 0.5f);
  G[5] = 0.1f;  // off the 2^-16 grid
  refusal(pt_init_gauss(&job, 2, 3, 8, 3, G.data(), betas3, 1, 0), "gauss off grid");
  expect(job == nullptr, "no job after refusals");

  // no GPU here: creation fails cleanly, leaving no handle behind
  const int rc = pt_init(&job, 2, 3, 8, 3, J.data(), betas3, 1);
  expect(rc != PT_OK && job == nullptr, "init without a device");
  G[5] = 0.5f;
  const int rcg = pt_init_gauss(&job, 2, 3, 8, 3, G.data(), betas3, 1, 0);
  expect(rcg != PT_OK && job == nullptr, "gauss init without a device");

  // every job entry point refuses a null handle
  refusal(pt_sweep(nullptr, 1), "sweep null");
  refusal(pt_exchange(nullptr), "exchange null");
  refusal(pt_houdayer(nullptr), "houdayer null");
  refusal(pt_houdayer_multi(nullptr), "houdayer multi null");
  refusal(pt_measure(nullptr), "measure null");
  refusal(pt_mcs(nullptr, 1, 0), "mcs null");
  refusal(pt_mcs_noalloc(nullptr, 1, 0), "mcs noalloc null");
  refusal(pt_set_measure_interval(nullptr, 2), "interval null");
  refusal(pt_observables(nullptr, nullptr, nullptr, nullptr), "observables null");
  refusal(pt_get_spins(nullptr, nullptr), "get spins null");
  refusal(pt_get_state(nullptr, nullptr, nullptr), "get state null");
  refusal(pt_destroy(nullptr), "destroy null");
  pt_batch* batch = nullptr;
  refusal(pt_batch_create(nullptr, 0, &batch), "batch of nothing");
  refusal(pt_batch_run(nullptr, 1, 0), "batch run null");
  refusal(pt_server_submit(nullptr, nullptr, nullptr), "submit null");
  refusal(pt_server_stop(nullptr), "stop null");
  pt_server* srv = nullptr;
  const int rcs = pt_server_start(1u << 20, 0, &srv);
  expect(rcs != PT_OK && srv == nullptr, "server start refused");

  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("sanitized runtime host checks complete\n");
  return 0;
}
