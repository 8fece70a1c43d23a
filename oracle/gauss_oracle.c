/*
 * gauss_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain CPU reference for the Edwards-Anderson spin glass with Gaussian
 * couplings (Sec. 2.1: the couplings are drawn from a standard normal or from
 * the bimodal distribution; Sec. 4.2 benchmarks the 2D Gaussian model), as
 * the GPU library simulates it.  Like ea_oracle.c it shares nothing with the
 * GPU code; it uses ea_oracle.c's Philox generator.
 *
 * Readings (the paper stores Gaussian couplings as 32-bit floats and says no
 * more about the arithmetic):
 *   - couplings lie on a fixed-point grid, J = n 2^-16 with |J| <= 8 (the
 *     harness rounds its normal draws to the grid); they are held here as the
 *     integers n.  Every local field and every energy is then an exact integer
 *     number of 2^-16 units whatever the order of summation, so results do not
 *     depend on how a parallel code groups its sums;
 *   - a Metropolis flip with energy change dE > 0 is accepted iff the site's
 *     32-bit Philox word r satisfies r < 2^32 exp(-beta dE), and a replica
 *     exchange with D = E_b - E_a > 0 iff r < 2^32 exp(-(beta_k - beta_{k+1})
 *     D), the difference of inverse temperatures taken in double precision:
 *     exact comparisons of the integer r with real numbers, decided here in
 *     113-bit floating point (libquadmath), which settles every case except
 *     those where the two sides differ by less than about 2^-80 of 2^32;
 *   - everything else (checkerboard order, random-number counters, exchange
 *     order, Houdayer moves, both variants, measurement cadence) is as for
 *     the bimodal couplings in ea_oracle.c.
 * Energies are int64 numbers of 2^-16 units; the measured sums of E^2 are
 * kept in 128 bits.
 */
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* ea_oracle.c */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_multi_coins(uint64_t seed, uint32_t sample, uint32_t k, uint32_t v, int N,
                    uint8_t *coin);

enum { G_TAG_INIT = 2, G_TAG_METRO = 3, G_TAG_PT = 4, G_TAG_HOU = 5 };

static uint32_t g_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                       uint32_t sample, int word) {
  uint32_t ctr[4] = {c0, c1, c2, (tag << 28) | sample};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  or_philox4x32_10(ctr, key, out);
  return out[word];
}

/* Geometry (Sec. 2.1: square or simple cubic, periodic): site i = x0 + L x1
   (+ L^2 x2); the bond (i, i + e_mu) is stored at J[mu][i]. */
static int g_neighbour(int L, int d, int i, int mu, int dir) {
  int x[3] = {i % L, (i / L) % L, d == 3 ? i / (L * L) : 0};
  x[mu] = (x[mu] + dir + L) % L;
  return x[0] + L * x[1] + (d == 3 ? L * L * x[2] : 0);
}

static int g_colour(int L, int d, int i) {
  return (i % L + (i / L) % L + (d == 3 ? i / (L * L) : 0)) & 1;
}

static int32_t g_bond(const int32_t *J, int L, int d, int N, int i, int mu, int dir) {
  if (dir > 0) return J[(size_t)mu * N + i];
  return J[(size_t)mu * N + g_neighbour(L, d, i, mu, -1)];
}

/* Eq. (1) at H = 0 in 2^-16 units: E = -sum_<ij> n_ij s_i s_j. */
OR_EXPORT int64_t org_energy(int L, int d, const int32_t *J, const int8_t *s) {
  int N = d == 3 ? L * L * L : L * L;
  int64_t E = 0;
  for (int i = 0; i < N; ++i)
    for (int mu = 0; mu < d; ++mu)
      E -= (int64_t)J[(size_t)mu * N + i] * s[i] * s[g_neighbour(L, d, i, mu, +1)];
  return E;
}

/* x = s_i h_i in 2^-16 units; flipping s_i changes the energy by 2x. */
OR_EXPORT int64_t org_local_x(int L, int d, const int32_t *J, const int8_t *s, int i) {
  int N = d == 3 ? L * L * L : L * L;
  int64_t h = 0;
  for (int mu = 0; mu < d; ++mu)
    for (int dir = -1; dir <= 1; dir += 2)
      h += (int64_t)g_bond(J, L, d, N, i, mu, dir) * s[g_neighbour(L, d, i, mu, dir)];
  return s[i] * h;
}

/* r < 2^32 exp(-b u 2^-16) for b > 0 (a double) and u > 0 (an integer number
   of 2^-16 units): the product b u is exact in 113 bits; an exponential that
   underflows even there is positive, so only r = 0 lies below it. */
OR_EXPORT int org_accept(uint32_t r, double b, int64_t u) {
  __float128 y = (__float128)b * (__float128)u;
  y = ldexpq(y, -16);
  __float128 t = ldexpq(expq(-y), 32);
  if (t == 0) return r == 0;
  return (__float128)r < t;
}

typedef struct {
  int S, NT, L, d, N, nslot;
  uint64_t seed;
  uint32_t *key;          /* [S] sample index used in the counters */
  int32_t *J;             /* [S][d][N] coupling units */
  int8_t *s;              /* [S][2NT][N] */
  int64_t *E;             /* [S][2NT] */
  int32_t *sot, *tos;     /* [S][2][NT] */
  double *beta;           /* [NT] */
  uint64_t t, u, v, n_meas;
  int every;
  int64_t *mE, *mQ, *mAQ, *mQ2;           /* [S][NT] */
  unsigned __int128 *mE2, *mQ4;           /* [S][NT] */
} org_job;

static int8_t *g_lat(org_job *jb, int s, int slot) {
  return jb->s + ((size_t)s * jb->nslot + slot) * jb->N;
}
static const int32_t *g_cpl(const org_job *jb, int s) {
  return jb->J + (size_t)s * jb->d * jb->N;
}

OR_EXPORT void org_recompute_energies(org_job *jb) {
  for (int s = 0; s < jb->S; ++s)
    for (int r = 0; r < jb->nslot; ++r)
      jb->E[(size_t)s * jb->nslot + r] = org_energy(jb->L, jb->d, g_cpl(jb, s), g_lat(jb, s, r));
}

/* A job as ea_oracle.c's or_create, with coupling units J. */
OR_EXPORT org_job *org_create(int S, int NT, int L, int d, const int32_t *J, const double *betas,
                              uint64_t seed, const uint32_t *sample_key) {
  if (S < 1 || NT < 2 || L < 3 || (d != 2 && d != 3)) return NULL;
  org_job *jb = (org_job *)calloc(1, sizeof(org_job));
  jb->S = S;
  jb->NT = NT;
  jb->L = L;
  jb->d = d;
  jb->N = d == 3 ? L * L * L : L * L;
  jb->nslot = 2 * NT;
  jb->seed = seed;
  jb->every = 1;
  size_t N = jb->N, ST = (size_t)S * NT;
  jb->key = (uint32_t *)malloc(sizeof(uint32_t) * S);
  for (int s = 0; s < S; ++s) jb->key[s] = sample_key ? sample_key[s] : (uint32_t)s;
  jb->J = (int32_t *)malloc(sizeof(int32_t) * (size_t)S * d * N);
  memcpy(jb->J, J, sizeof(int32_t) * (size_t)S * d * N);
  jb->s = (int8_t *)malloc((size_t)S * jb->nslot * N);
  jb->E = (int64_t *)calloc((size_t)S * jb->nslot, sizeof(int64_t));
  jb->sot = (int32_t *)malloc(sizeof(int32_t) * S * 2 * NT);
  jb->tos = (int32_t *)malloc(sizeof(int32_t) * S * 2 * NT);
  jb->beta = (double *)malloc(sizeof(double) * NT);
  memcpy(jb->beta, betas, sizeof(double) * NT);
  jb->mE = (int64_t *)calloc(ST, sizeof(int64_t));
  jb->mQ = (int64_t *)calloc(ST, sizeof(int64_t));
  jb->mAQ = (int64_t *)calloc(ST, sizeof(int64_t));
  jb->mQ2 = (int64_t *)calloc(ST, sizeof(int64_t));
  jb->mE2 = (unsigned __int128 *)calloc(ST, sizeof(unsigned __int128));
  jb->mQ4 = (unsigned __int128 *)calloc(ST, sizeof(unsigned __int128));
  for (int s = 0; s < S; ++s)
    for (int r = 0; r < jb->nslot; ++r) {
      int8_t *lat = g_lat(jb, s, r);
      for (int i = 0; i < (int)N; ++i) {
        uint32_t w = g_word(seed, (uint32_t)(i >> 2), 0u, (uint32_t)r, G_TAG_INIT, jb->key[s], i & 3);
        lat[i] = (w >> 31) ? (int8_t)-1 : (int8_t)1;
      }
    }
  for (int s = 0; s < S; ++s)
    for (int c = 0; c < 2; ++c)
      for (int k = 0; k < NT; ++k) {
        jb->sot[((size_t)s * 2 + c) * NT + k] = k;
        jb->tos[((size_t)s * 2 + c) * NT + k] = k;
      }
  org_recompute_energies(jb);
  return jb;
}

OR_EXPORT void org_destroy(org_job *jb) {
  if (!jb) return;
  free(jb->key); free(jb->J); free(jb->s); free(jb->E); free(jb->sot); free(jb->tos);
  free(jb->beta); free(jb->mE); free(jb->mQ); free(jb->mAQ); free(jb->mQ2); free(jb->mE2);
  free(jb->mQ4);
  free(jb);
}

/* Metropolis sweep (Sec. 2.2), checkerboard, the same site order and Philox
   counters as the bimodal model: site i of colour c in sweep t draws word
   b & 3 of counter (R G + (b >> 2), 2t + c, slot, 3<<28 | sample), R = i / L,
   b = (i mod L) >> 1, G = ceil(L/8). */
OR_EXPORT void org_sweep(org_job *jb, int n) {
  const int L = jb->L, d = jb->d, N = jb->N, NT = jb->NT;
  const uint32_t G = (uint32_t)((L + 7) / 8);
  for (int rep = 0; rep < n; ++rep) {
    for (int s = 0; s < jb->S; ++s) {
      const int32_t *Js = g_cpl(jb, s);
      for (int slot = 0; slot < jb->nslot; ++slot) {
        int k = jb->tos[((size_t)s * 2 + slot / NT) * NT + slot % NT];
        int8_t *lat = g_lat(jb, s, slot);
        int64_t *Es = &jb->E[(size_t)s * jb->nslot + slot];
        for (int colour = 0; colour < 2; ++colour)
          for (int i = 0; i < N; ++i) {
            if (g_colour(L, d, i) != colour) continue;
            int64_t x = org_local_x(L, d, Js, lat, i);
            int flip = x <= 0;
            if (!flip) {
              uint32_t R = (uint32_t)(i / L), b = (uint32_t)((i % L) >> 1);
              uint32_t r = g_word(jb->seed, R * G + (b >> 2), (uint32_t)(2 * jb->t + colour),
                                  (uint32_t)slot, G_TAG_METRO, jb->key[s], (int)(b & 3));
              flip = org_accept(r, jb->beta[k], 2 * x);
            }
            if (flip) {
              lat[i] = (int8_t)-lat[i];
              *Es += 2 * x;
            }
          }
      }
    }
    jb->t += 1;
  }
}

/* Replica exchange (Eq. (5)): per sample and set, k = 0 .. NT-2 ascending,
   word 0 of counter (k, u, set, 4<<28 | sample). */
OR_EXPORT void org_exchange(org_job *jb) {
  const int NT = jb->NT;
  for (int s = 0; s < jb->S; ++s)
    for (int c = 0; c < 2; ++c) {
      int32_t *sot = &jb->sot[((size_t)s * 2 + c) * NT];
      int32_t *tos = &jb->tos[((size_t)s * 2 + c) * NT];
      for (int k = 0; k + 1 < NT; ++k) {
        int a = sot[k], b = sot[k + 1];
        int64_t D = jb->E[(size_t)s * jb->nslot + c * NT + b] - jb->E[(size_t)s * jb->nslot + c * NT + a];
        int acc = D <= 0;
        if (!acc) {
          uint32_t r = g_word(jb->seed, (uint32_t)k, (uint32_t)jb->u, (uint32_t)c, G_TAG_PT, jb->key[s], 0);
          acc = org_accept(r, jb->beta[k] - jb->beta[k + 1], D);
        }
        if (acc) {
          sot[k] = b;
          sot[k + 1] = a;
          tos[b] = k;
          tos[a] = k + 1;
        }
      }
    }
  jb->u += 1;
}

/* Energy change of replica a when both replicas are negated on the sites
   marked in `in`: 2 n_ij s_i s_j over the bonds leaving that set. */
static int64_t g_boundary(const org_job *jb, const int32_t *Js, const int8_t *sa, const int8_t *in) {
  const int L = jb->L, d = jb->d, N = jb->N;
  int64_t delta = 0;
  for (int i = 0; i < N; ++i) {
    if (!in[i]) continue;
    for (int mu = 0; mu < d; ++mu)
      for (int dir = -1; dir <= 1; dir += 2) {
        int j = g_neighbour(L, d, i, mu, dir);
        if (!in[j]) delta += 2 * (int64_t)g_bond(Js, L, d, N, i, mu, dir) * sa[i] * sa[j];
      }
  }
  return delta;
}

/* Houdayer pass (Sec. 2.4, Eq. (10)), single-cluster (multi = 0: seed the
   m-th q = -1 site in increasing i, m = floor(r64 n / 2^64), r64 from
   counter (k, v, 0, 5<<28 | sample)) or multi-cluster (multi = 1: every
   cluster exchanged iff the coin of its lowest site is set, as ea_oracle.c's
   or_houdayer_multi).  The clusters ignore the couplings. */
OR_EXPORT void org_houdayer(org_job *jb, int multi) {
  const int L = jb->L, d = jb->d, N = jb->N, NT = jb->NT;
  int8_t *in = (int8_t *)malloc((size_t)N);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * N);
  uint8_t *coin = (uint8_t *)malloc((size_t)N);
  uint32_t key[2] = {(uint32_t)jb->seed, (uint32_t)(jb->seed >> 32)};
  for (int s = 0; s < jb->S; ++s)
    for (int k = 0; k < NT; ++k) {
      int a = jb->sot[((size_t)s * 2 + 0) * NT + k];
      int b = NT + jb->sot[((size_t)s * 2 + 1) * NT + k];
      int8_t *sa = g_lat(jb, s, a), *sb = g_lat(jb, s, b);
      memset(in, 0, (size_t)N);
      if (multi) {
        or_multi_coins(jb->seed, jb->key[s], (uint32_t)k, (uint32_t)jb->v, N, coin);
        int8_t *seen = (int8_t *)calloc((size_t)N, 1);
        for (int m = 0; m < N; ++m) {
          if (seen[m] || sa[m] == sb[m]) continue;
          int head = 0, tail = 0;
          seen[m] = 1;
          queue[tail++] = m;
          while (head < tail) {
            int i = queue[head++];
            for (int mu = 0; mu < d; ++mu)
              for (int dir = -1; dir <= 1; dir += 2) {
                int j = g_neighbour(L, d, i, mu, dir);
                if (!seen[j] && sa[j] != sb[j]) {
                  seen[j] = 1;
                  queue[tail++] = j;
                }
              }
          }
          if (coin[m])
            for (int q = 0; q < tail; ++q) in[queue[q]] = 1;
        }
        free(seen);
      } else {
        int nm = 0;
        for (int i = 0; i < N; ++i) nm += sa[i] != sb[i];
        if (nm == 0) continue;
        uint32_t ctr[4] = {(uint32_t)k, (uint32_t)jb->v, 0u, ((uint32_t)G_TAG_HOU << 28) | jb->key[s]};
        uint32_t w[4];
        or_philox4x32_10(ctr, key, w);
        uint64_t r64 = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
        uint64_t idx = (uint64_t)(((unsigned __int128)r64 * (uint64_t)nm) >> 64);
        int i0 = -1;
        for (int i = 0, c = 0; i < N; ++i)
          if (sa[i] != sb[i] && c++ == (int)idx) {
            i0 = i;
            break;
          }
        int head = 0, tail = 0;
        in[i0] = 1;
        queue[tail++] = i0;
        while (head < tail) {
          int i = queue[head++];
          for (int mu = 0; mu < d; ++mu)
            for (int dir = -1; dir <= 1; dir += 2) {
              int j = g_neighbour(L, d, i, mu, dir);
              if (!in[j] && sa[j] != sb[j]) {
                in[j] = 1;
                queue[tail++] = j;
              }
            }
        }
      }
      int64_t delta = g_boundary(jb, g_cpl(jb, s), sa, in);
      for (int i = 0; i < N; ++i)
        if (in[i]) {
          sa[i] = (int8_t)-sa[i];
          sb[i] = (int8_t)-sb[i];
        }
      jb->E[(size_t)s * jb->nslot + a] += delta;
      jb->E[(size_t)s * jb->nslot + b] -= delta;
    }
  free(in);
  free(queue);
  free(coin);
  jb->v += 1;
}

/* Measurement (Eqs. (3), (4)): exact sums of E, E^2 (both replicas of the
   pair), Q, |Q|, Q^2, Q^4 per sample and temperature. */
OR_EXPORT void org_measure(org_job *jb) {
  const int NT = jb->NT, N = jb->N;
  for (int s = 0; s < jb->S; ++s)
    for (int k = 0; k < NT; ++k) {
      int a = jb->sot[((size_t)s * 2 + 0) * NT + k];
      int b = NT + jb->sot[((size_t)s * 2 + 1) * NT + k];
      const int8_t *la = g_lat(jb, s, a), *lb = g_lat(jb, s, b);
      int64_t Q = 0;
      for (int i = 0; i < N; ++i) Q += (int64_t)la[i] * lb[i];
      int64_t Ea = jb->E[(size_t)s * jb->nslot + a], Eb = jb->E[(size_t)s * jb->nslot + b];
      size_t o = (size_t)s * NT + k;
      jb->mE[o] += Ea + Eb;
      jb->mE2[o] += (unsigned __int128)((__int128)Ea * Ea) + (unsigned __int128)((__int128)Eb * Eb);
      jb->mQ[o] += Q;
      jb->mAQ[o] += Q < 0 ? -Q : Q;
      jb->mQ2[o] += Q * Q;
      unsigned __int128 q2 = (unsigned __int128)(Q * Q);
      jb->mQ4[o] += q2 * q2;
    }
  jb->n_meas += 1;
}

OR_EXPORT void org_set_measure_every(org_job *jb, int every) { jb->every = every < 1 ? 1 : every; }

/* Monte Carlo steps in the order of Sec. 2.4; houdayer = 0 none, 1 single-
   cluster, 2 multi-cluster moves. */
OR_EXPORT void org_mcs(org_job *jb, int n, int houdayer, int measure) {
  for (int i = 0; i < n; ++i) {
    org_sweep(jb, 1);
    if (houdayer) org_houdayer(jb, houdayer == 2);
    org_exchange(jb);
    if (measure && jb->t % (uint64_t)jb->every == 0) org_measure(jb);
  }
}

/* per_sample [S][NT][5] = e, q, |q|, q^2, q^4; disorder [NT][6] = the same
   averaged over samples (integer numerators summed first) and the Binder
   parameter; energies per spin in coupling units (E 2^-16 / N). */
OR_EXPORT void org_observables(const org_job *jb, double *per_sample, double *disorder,
                               int64_t *n_meas) {
  const int NT = jb->NT;
  const double n = (double)jb->n_meas, N = (double)jb->N, unit = 1.0 / 65536.0;
  if (n_meas) *n_meas = (int64_t)jb->n_meas;
  if (per_sample)
    for (int s = 0; s < jb->S; ++s)
      for (int k = 0; k < NT; ++k) {
        size_t o = (size_t)s * NT + k;
        double *out = per_sample + o * 5;
        out[0] = (double)jb->mE[o] * unit / (2.0 * n * N);
        out[1] = (double)jb->mQ[o] / (n * N);
        out[2] = (double)jb->mAQ[o] / (n * N);
        out[3] = (double)jb->mQ2[o] / (n * (N * N));
        out[4] = (double)jb->mQ4[o] / (n * ((N * N) * (N * N)));
      }
  if (disorder) {
    const double S = (double)jb->S;
    for (int k = 0; k < NT; ++k) {
      int64_t sE = 0, sQ = 0, sAQ = 0, sQ2 = 0;
      unsigned __int128 sQ4 = 0;
      for (int s = 0; s < jb->S; ++s) {
        size_t o = (size_t)s * NT + k;
        sE += jb->mE[o];
        sQ += jb->mQ[o];
        sAQ += jb->mAQ[o];
        sQ2 += jb->mQ2[o];
        sQ4 += jb->mQ4[o];
      }
      double *out = disorder + (size_t)k * 6;
      out[0] = (double)sE * unit / (S * 2.0 * n * N);
      out[1] = (double)sQ / (S * n * N);
      out[2] = (double)sAQ / (S * n * N);
      out[3] = (double)sQ2 / (S * n * (N * N));
      out[4] = (double)sQ4 / (S * n * ((N * N) * (N * N)));
      out[5] = 0.5 * (3.0 - out[4] / (out[3] * out[3]));
    }
  }
}

/* State access for the tests. */
OR_EXPORT void org_get_spins(const org_job *jb, int8_t *out) {
  memcpy(out, jb->s, (size_t)jb->S * jb->nslot * jb->N);
}
OR_EXPORT void org_set_spins(org_job *jb, const int8_t *in) {
  memcpy(jb->s, in, (size_t)jb->S * jb->nslot * jb->N);
  org_recompute_energies(jb);
}
OR_EXPORT void org_get_energies(const org_job *jb, int64_t *out) {
  memcpy(out, jb->E, sizeof(int64_t) * (size_t)jb->S * jb->nslot);
}
OR_EXPORT void org_get_maps(const org_job *jb, int32_t *sot, int32_t *tos) {
  memcpy(sot, jb->sot, sizeof(int32_t) * (size_t)jb->S * 2 * jb->NT);
  memcpy(tos, jb->tos, sizeof(int32_t) * (size_t)jb->S * 2 * jb->NT);
}
OR_EXPORT void org_get_counters(const org_job *jb, uint64_t *out) {
  out[0] = jb->t;
  out[1] = jb->u;
  out[2] = jb->v;
  out[3] = jb->n_meas;
}
/* [S][NT] each: sum E, sum Q, sum |Q|, sum Q^2; E^2 and Q^4 as (lo, hi) 64-bit halves. */
OR_EXPORT void org_get_moments(const org_job *jb, int64_t *E, uint64_t *E2, int64_t *Q, int64_t *AQ,
                               int64_t *Q2, uint64_t *Q4) {
  size_t ST = (size_t)jb->S * jb->NT;
  for (size_t o = 0; o < ST; ++o) {
    E[o] = jb->mE[o];
    E2[2 * o] = (uint64_t)jb->mE2[o];
    E2[2 * o + 1] = (uint64_t)(jb->mE2[o] >> 64);
    Q[o] = jb->mQ[o];
    AQ[o] = jb->mAQ[o];
    Q2[o] = jb->mQ2[o];
    Q4[2 * o] = (uint64_t)jb->mQ4[o];
    Q4[2 * o + 1] = (uint64_t)(jb->mQ4[o] >> 64);
  }
}
