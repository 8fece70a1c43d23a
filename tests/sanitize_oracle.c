/*
 * sanitize_oracle.c -- test driver, not part of the library.
 *
 * Calls every routine the CPU oracle exports (oracle/ea_oracle.c,
 * oracle/gauss_oracle.c, oracle/enum.c) on small lattices of both dimensions,
 * even and odd L, with every step kind (sweeps, exchanges, both Houdayer
 * variants, measurements with the two-replica modes and an interval), and
 * every getter into a buffer of exactly the documented size.  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer (no recovery) by
 * tests/test_sanitizers.py: an out-of-bounds access, a leak, a use after free
 * or undefined arithmetic in the oracle ends the run with a report and a
 * non-zero status.  Exit 0 when everything ran.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct or_job or_job;
typedef struct org_job org_job;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_philox_stream(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, const uint32_t key[2],
                      int64_t n, uint32_t *out);
int64_t or_energy(int L, int d, const int8_t *J, const int8_t *s);
int or_local_x(int L, int d, const int8_t *J, const int8_t *s, int i);
void or_metro_thresholds(const double *betas, int NT, int d, uint32_t *thr);
int or_pt_thresholds(const double *betas, int NT, int d, int N, uint32_t *thr, int M_alloc);
void or_recompute_energies(or_job *jb);
or_job *or_create(int S, int NT, int L, int d, const int8_t *J, const double *betas, uint64_t seed,
                  const uint32_t *sample_key);
void or_destroy(or_job *jb);
void or_sweep(or_job *jb, int n);
void or_exchange(or_job *jb);
int64_t or_houdayer_move(int L, int d, const int8_t *J, int8_t *sa, int8_t *sb, uint64_t r64,
                         int8_t *cluster_out, int32_t *cluster_size);
void or_houdayer(or_job *jb);
int64_t or_houdayer_multi_move(int L, int d, const int8_t *J, int8_t *sa, int8_t *sb,
                               const uint8_t *coin, int8_t *flip_out, int32_t *nclusters);
void or_multi_coins(uint64_t seed, uint32_t sample, uint32_t k, uint32_t v, int N, uint8_t *coin);
void or_houdayer_multi(or_job *jb);
void or_overlap_modes(int L, int d, const int8_t *sa, const int8_t *sb, int64_t *out);
void or_enable_modes(or_job *jb);
void or_measure(or_job *jb);
void or_set_measure_every(or_job *jb, int every);
void or_mcs(or_job *jb, int n, int houdayer, int measure);
void or_observables(const or_job *jb, double *per_sample, double *disorder, int64_t *n_meas);
void or_get_spins(const or_job *jb, int8_t *out);
void or_set_spins(or_job *jb, const int8_t *in);
void or_get_energies(const or_job *jb, int64_t *out);
void or_get_maps(const or_job *jb, int32_t *sot, int32_t *tos);
void or_get_counters(const or_job *jb, uint64_t out[4]);
void or_get_moments(const or_job *jb, int64_t *mE, int64_t *mE2, int64_t *mQ, int64_t *mAQ,
                    int64_t *mQ2, uint64_t *mQ4_lohi);
void or_get_walk(const or_job *jb, int32_t *label, uint32_t *begin, uint64_t *trips);
void or_get_stats(const or_job *jb, int64_t *out);
void or_get_modes(const or_job *jb, int64_t *out);
int or_pt_table_len(const or_job *jb);
void or_get_pt_table(const or_job *jb, uint32_t *out);
void or_sweep_order(int L, int d, int32_t *order);
int or_metro_rule(int x, uint32_t r, const uint32_t *thr_row);

int64_t org_energy(int L, int d, const int32_t *J, const int8_t *s);
int64_t org_local_x(int L, int d, const int32_t *J, const int8_t *s, int i);
int org_accept(uint32_t r, double b, int64_t u);
void org_recompute_energies(org_job *jb);
org_job *org_create(int S, int NT, int L, int d, const int32_t *J, const double *betas,
                    uint64_t seed, const uint32_t *sample_key);
void org_destroy(org_job *jb);
void org_set_measure_every(org_job *jb, int every);
void org_mcs(org_job *jb, int n, int houdayer, int measure);
void org_observables(const org_job *jb, double *per_sample, double *disorder, int64_t *n_meas);
void org_get_spins(const org_job *jb, int8_t *out);
void org_set_spins(org_job *jb, const int8_t *in);
void org_get_energies(const org_job *jb, int64_t *out);
void org_get_maps(const org_job *jb, int32_t *sot, int32_t *tos);
void org_get_counters(const org_job *jb, uint64_t *out);
void org_get_moments(const org_job *jb, int64_t *E, uint64_t *E2, int64_t *Q, int64_t *AQ,
                     int64_t *Q2, uint64_t *Q4);

int en_density_of_states(int L, int d, const int8_t *J, uint64_t *counts);
int en_state_energies(int L, int d, const int8_t *J, int32_t *E_out);

static uint64_t g_rng = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void) {
  g_rng = g_rng * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(g_rng >> 32);
}

/* malloc of exactly n bytes (n > 0), aborting on failure */
static void *xmalloc(size_t n) {
  void *p = malloc(n ? n : 1);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return p;
}

static int sites(int L, int d) { return d == 3 ? L * L * L : L * L; }

static void run_pm_j(int L, int d, int S, int NT, int with_keys) {
  const int N = sites(L, d), nslot = 2 * NT;
  int8_t *J = xmalloc((size_t)S * d * N);
  for (size_t i = 0; i < (size_t)S * d * N; ++i) J[i] = (next_u32() >> 31) ? 1 : -1;
  double *betas = xmalloc(sizeof(double) * NT);
  for (int k = 0; k < NT; ++k) betas[k] = 1.5 - k * (1.2 / NT);
  uint32_t *keys = NULL;
  if (with_keys) {
    keys = xmalloc(sizeof(uint32_t) * S);
    for (int s = 0; s < S; ++s) keys[s] = 17u + 3u * (uint32_t)s;
  }
  or_job *jb = or_create(S, NT, L, d, J, betas, 0x1234567890ull + (uint64_t)L, keys);
  if (!jb) {
    fprintf(stderr, "or_create failed L=%d d=%d\n", L, d);
    exit(3);
  }
  or_enable_modes(jb);
  or_mcs(jb, 6, 1, 1);
  or_set_measure_every(jb, 2);
  or_mcs(jb, 5, 2, 1);
  or_mcs(jb, 3, 0, 1);
  or_sweep(jb, 2);
  or_houdayer(jb);
  or_houdayer_multi(jb);
  or_exchange(jb);
  or_measure(jb);
  or_recompute_energies(jb);

  const size_t ST = (size_t)S * NT, lat = (size_t)S * nslot;
  int8_t *sp = xmalloc(lat * N);
  or_get_spins(jb, sp);
  or_set_spins(jb, sp);
  int64_t *E = xmalloc(sizeof(int64_t) * lat);
  or_get_energies(jb, E);
  int32_t *sot = xmalloc(sizeof(int32_t) * S * 2 * NT), *tos = xmalloc(sizeof(int32_t) * S * 2 * NT);
  or_get_maps(jb, sot, tos);
  or_get_maps(jb, NULL, tos);
  uint64_t ctr[4];
  or_get_counters(jb, ctr);
  int64_t *m[5];
  for (int i = 0; i < 5; ++i) m[i] = xmalloc(sizeof(int64_t) * ST);
  uint64_t *q4 = xmalloc(sizeof(uint64_t) * 2 * ST);
  or_get_moments(jb, m[0], m[1], m[2], m[3], m[4], q4);
  int32_t *lab = xmalloc(sizeof(int32_t) * lat);
  uint32_t *beg = xmalloc(sizeof(uint32_t) * lat);
  uint64_t *trips = xmalloc(sizeof(uint64_t) * S * 32 * 3);
  or_get_walk(jb, lab, beg, trips);
  int64_t *st = xmalloc(sizeof(int64_t) * ST * 24);
  or_get_stats(jb, st);
  int64_t *modes = xmalloc(sizeof(int64_t) * ST * (L / 2 + 1));
  or_get_modes(jb, modes);
  const int M = or_pt_table_len(jb);
  uint32_t *tab = xmalloc(sizeof(uint32_t) * (NT - 1) * M);
  or_get_pt_table(jb, tab);
  double *ps = xmalloc(sizeof(double) * ST * 5), *dis = xmalloc(sizeof(double) * NT * 6);
  int64_t nm = 0;
  or_observables(jb, ps, dis, &nm);

  /* the stand-alone routines on the first sample's first pair */
  int8_t *sa = xmalloc(N), *sb = xmalloc(N), *cl = xmalloc(N);
  memcpy(sa, sp, N);
  memcpy(sb, sp + (size_t)NT * N, N);
  int32_t csize = 0;
  (void)or_houdayer_move(L, d, J, sa, sb, ((uint64_t)next_u32() << 32) | next_u32(), cl, &csize);
  uint8_t *coin = xmalloc(N);
  or_multi_coins(77, 1, 2, 3, N, coin);
  int32_t ncl = 0;
  (void)or_houdayer_multi_move(L, d, J, sa, sb, coin, cl, &ncl);
  int64_t *am = xmalloc(sizeof(int64_t) * (L / 2 + 1));
  or_overlap_modes(L, d, sa, sb, am);
  (void)or_energy(L, d, J, sa);
  for (int i = 0; i < N; ++i) (void)or_local_x(L, d, J, sa, i);
  int32_t *order = xmalloc(sizeof(int32_t) * N);
  or_sweep_order(L, d, order);
  uint32_t *thr = xmalloc(sizeof(uint32_t) * NT * d);
  or_metro_thresholds(betas, NT, d, thr);
  for (int x = -2 * d; x <= 2 * d; x += 2) (void)or_metro_rule(x, next_u32(), thr);
  const int M2 = or_pt_thresholds(betas, NT, d, N, NULL, 0);
  uint32_t *thr2 = xmalloc(sizeof(uint32_t) * (NT - 1) * (M2 + 3));
  (void)or_pt_thresholds(betas, NT, d, N, thr2, M2 + 3);

  or_destroy(jb);
  free(J); free(betas); free(keys); free(sp); free(E); free(sot); free(tos);
  for (int i = 0; i < 5; ++i) free(m[i]);
  free(q4); free(lab); free(beg); free(trips); free(st); free(modes); free(tab); free(ps);
  free(dis); free(sa); free(sb); free(cl); free(coin); free(am); free(order); free(thr); free(thr2);
}

static void run_gauss(int L, int d, int S, int NT) {
  const int N = sites(L, d), nslot = 2 * NT;
  int32_t *J = xmalloc(sizeof(int32_t) * S * d * N);
  for (size_t i = 0; i < (size_t)S * d * N; ++i)
    J[i] = (int32_t)(next_u32() % (2u * 8u * 65536u + 1u)) - 8 * 65536;
  double *betas = xmalloc(sizeof(double) * NT);
  for (int k = 0; k < NT; ++k) betas[k] = 2.0 - k * (1.5 / NT);
  org_job *jb = org_create(S, NT, L, d, J, betas, 99 + (uint64_t)L, NULL);
  if (!jb) {
    fprintf(stderr, "org_create failed L=%d d=%d\n", L, d);
    exit(3);
  }
  org_mcs(jb, 4, 1, 1);
  org_set_measure_every(jb, 3);
  org_mcs(jb, 4, 2, 1);
  org_mcs(jb, 2, 0, 0);
  org_recompute_energies(jb);
  const size_t ST = (size_t)S * NT, lat = (size_t)S * nslot;
  int8_t *sp = xmalloc(lat * N);
  org_get_spins(jb, sp);
  org_set_spins(jb, sp);
  int64_t *E = xmalloc(sizeof(int64_t) * lat);
  org_get_energies(jb, E);
  int32_t *sot = xmalloc(sizeof(int32_t) * S * 2 * NT), *tos = xmalloc(sizeof(int32_t) * S * 2 * NT);
  org_get_maps(jb, sot, tos);
  uint64_t ctr[4];
  org_get_counters(jb, ctr);
  int64_t *mE = xmalloc(sizeof(int64_t) * ST), *mQ = xmalloc(sizeof(int64_t) * ST);
  int64_t *mAQ = xmalloc(sizeof(int64_t) * ST), *mQ2 = xmalloc(sizeof(int64_t) * ST);
  uint64_t *mE2 = xmalloc(sizeof(uint64_t) * 2 * ST), *mQ4 = xmalloc(sizeof(uint64_t) * 2 * ST);
  org_get_moments(jb, mE, mE2, mQ, mAQ, mQ2, mQ4);
  double *ps = xmalloc(sizeof(double) * ST * 5), *dis = xmalloc(sizeof(double) * NT * 6);
  int64_t nm = 0;
  org_observables(jb, ps, dis, &nm);
  (void)org_energy(L, d, J, sp);
  for (int i = 0; i < N; ++i) (void)org_local_x(L, d, J, sp, i);
  for (int i = 0; i < 64; ++i) (void)org_accept(next_u32(), 0.1 + 0.05 * i, (int64_t)(next_u32() % 4000000u) + 1);
  org_destroy(jb);
  free(J); free(betas); free(sp); free(E); free(sot); free(tos); free(mE); free(mQ); free(mAQ);
  free(mQ2); free(mE2); free(mQ4); free(ps); free(dis);
}

int main(void) {
  uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
  or_philox4x32_10(ctr, key, out);
  uint32_t *stream = xmalloc(sizeof(uint32_t) * 4 * 100);
  or_philox_stream(7, 8, 9, 10, key, 100, stream);
  free(stream);

  static const int shapes[][2] = {{3, 2}, {4, 2}, {5, 2}, {6, 2}, {10, 2}, {16, 2},
                                  {3, 3}, {4, 3}, {5, 3}, {6, 3}};
  for (size_t i = 0; i < sizeof shapes / sizeof shapes[0]; ++i) {
    run_pm_j(shapes[i][0], shapes[i][1], 2, 3, (int)(i & 1));
    run_gauss(shapes[i][0], shapes[i][1], 2, 3);
  }
  run_pm_j(4, 2, 1, 2, 0);  /* smallest ladder */
  run_gauss(4, 3, 3, 5);

  int8_t J[2 * 9];
  for (int i = 0; i < 18; ++i) J[i] = (next_u32() >> 31) ? 1 : -1;
  uint64_t counts[2 * 2 * 9 + 1];
  memset(counts, 0, sizeof counts);
  if (en_density_of_states(3, 2, J, counts) != 0) return 4;
  int32_t *Es = xmalloc(sizeof(int32_t) * 512);
  if (en_state_energies(3, 2, J, Es) != 0) return 5;
  free(Es);
  printf("sanitized oracle run complete\n");
  return 0;
}
