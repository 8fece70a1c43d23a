/*
 * ea_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU reference of the parallel-tempering
 * simulation of the Edwards-Anderson (EA) Ising spin glass described in
 * Kumar, Gross, Janke, Weigel, "Massively parallel simulations for disordered
 * systems" (arXiv:2003.04621).  It exists so that the GPU library can be
 * checked against something obviously correct; nothing in the product path
 * may call it.  It shares no code, header, table builder or constant with the
 * GPU library.  Only the test-suite, the smoke check and the benchmark's CPU
 * baseline load it.
 *
 * What it follows:
 *   - Hamiltonian, zero field: Sec. 2.1, Eq. (1); bimodal couplings Eq. (2).
 *   - Energy per spin and overlap: Sec. 2.1, Eqs. (3) and (4).
 *   - Single-spin-flip Metropolis: Sec. 2.2 (Metropolis transition rates).
 *   - Replica exchange acceptance: Sec. 2.2, Eq. (5); exchange of temperatures
 *     rather than configurations with two index arrays: Sec. 2.2 and Sec. 3.
 *   - Houdayer cluster move in overlap space: Sec. 2.4, Eq. (10); its
 *     multi-cluster variant, which Sec. 3 and Sec. 5 propose.
 *   - One Monte Carlo step = Metropolis sweep, Houdayer move per same-T pair,
 *     PT update over neighbouring-T pairs: Sec. 2.4 (enumerated update scheme).
 *   - Counter-based Philox random numbers: Sec. 3 (Salmon et al. 2011).
 *   - Round-trip (tunnelling) time of the replica walk in temperature space
 *     and its logarithmically binned time series: Sec. 2.3.
 *   - Two-replica modes for the spin-glass susceptibility and correlation
 *     length (named in Sec. 3, not defined there; the usual definitions).
 *
 * Readings where the paper is silent (all documented in the design notes):
 *   checkerboard order (colour 0 then colour 1, increasing site index inside a
 *   colour); acceptance thresholds as floor(2^32 p) compared with a 32-bit
 *   random word; the Philox counter layout; initial spins from Philox; PT pairs
 *   visited in ascending temperature order with an independent ladder per
 *   replica set; the Houdayer seed chosen uniformly by a 64-bit multiply-shift;
 *   a Houdayer pass with no q=-1 site is a no-op.
 *
 * Geometry: site i = x0 + L*x1 (+ L^2*x2), x0 fastest, periodic boundaries.
 * The bond (i, i+e_mu) is stored at J[mu][i].  A "row" is the set of L sites
 * sharing (x1, x2); row index R = i / L.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, written from Salmon, Moraes, Dror, Shaw, "Parallel random   */
/* numbers: as easy as 1, 2, 3" (SC'11): ten rounds of the Philox S-box with  */
/* multipliers 0xD2511F53, 0xCD9E8D57 and a Weyl key schedule with           */
/* increments 0x9E3779B9 (golden ratio) and 0xBB67AE85 (sqrt(3)-1).           */
/* ------------------------------------------------------------------------ */
OR_EXPORT void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                                uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* n consecutive Philox calls with counters (c0 + i, c1, c2, c3), i < n;
   out receives 4n words.  Used by the statistical tests of the generator. */
OR_EXPORT void or_philox_stream(uint32_t c0, uint32_t c1, uint32_t c2,
                                uint32_t c3, const uint32_t key[2], int64_t n,
                                uint32_t *out) {
  for (int64_t i = 0; i < n; ++i) {
    uint32_t ctr[4] = {c0 + (uint32_t)i, c1, c2, c3};
    or_philox4x32_10(ctr, key, out + 4 * i);
  }
}

/* Counter tags: the top four bits of the fourth counter word. */
enum { OR_TAG_INIT = 2, OR_TAG_METRO = 3, OR_TAG_PT = 4, OR_TAG_HOU = 5, OR_TAG_HOU_MULTI = 6 };

static uint32_t or_rand_word(uint64_t seed, uint32_t c0, uint32_t c1,
                             uint32_t c2, uint32_t tag, uint32_t sample,
                             int word) {
  uint32_t ctr[4] = {c0, c1, c2, (tag << 28) | sample};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  or_philox4x32_10(ctr, key, out);
  return out[word];
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry (Sec. 2.1: square or simple cubic, periodic).             */
/* ------------------------------------------------------------------------ */
static void or_coords(int L, int d, int i, int x[3]) {
  x[0] = i % L;
  x[1] = (i / L) % L;
  x[2] = (d == 3) ? i / (L * L) : 0;
}

static int or_site(int L, int d, const int x[3]) {
  return x[0] + L * x[1] + (d == 3 ? L * L * x[2] : 0);
}

/* neighbour of i one step along +e_mu (dir=+1) or -e_mu (dir=-1) */
static int or_neighbour(int L, int d, int i, int mu, int dir) {
  int x[3];
  or_coords(L, d, i, x);
  x[mu] = (x[mu] + dir + L) % L;
  return or_site(L, d, x);
}

static int or_colour(int L, int d, int i) {
  int x[3];
  or_coords(L, d, i, x);
  return (x[0] + x[1] + x[2]) & 1;
}

/* Bond value J_ij between i and its neighbour along (mu, dir). */
static int or_bond(const int8_t *Jsample, int L, int d, int N, int i, int mu,
                   int dir) {
  if (dir > 0) return Jsample[(size_t)mu * N + i];
  return Jsample[(size_t)mu * N + or_neighbour(L, d, i, mu, -1)];
}

/* Eq. (1) at H = 0: E = -sum_<ij> J_ij s_i s_j, each bond counted once. */
OR_EXPORT int64_t or_energy(int L, int d, const int8_t *Jsample,
                            const int8_t *spins) {
  int N = (d == 3) ? L * L * L : L * L;
  int64_t E = 0;
  for (int i = 0; i < N; ++i)
    for (int mu = 0; mu < d; ++mu) {
      int j = or_neighbour(L, d, i, mu, +1);
      E -= (int64_t)Jsample[(size_t)mu * N + i] * spins[i] * spins[j];
    }
  return E;
}

/* x = s_i * h_i with h_i = sum over the 2d neighbours of J_ij s_j.  Flipping
   s_i changes the energy by 2x. */
OR_EXPORT int or_local_x(int L, int d, const int8_t *Jsample,
                         const int8_t *spins, int i) {
  int N = (d == 3) ? L * L * L : L * L;
  int h = 0;
  for (int mu = 0; mu < d; ++mu)
    for (int dir = -1; dir <= 1; dir += 2) {
      int j = or_neighbour(L, d, i, mu, dir);
      h += or_bond(Jsample, L, d, N, i, mu, dir) * spins[j];
    }
  return spins[i] * h;
}

/* ------------------------------------------------------------------------ */
/* Acceptance thresholds.                                                      */
/* Metropolis (Sec. 2.2): an uphill move with energy change dE = 2x > 0 is     */
/* accepted with probability exp(-beta dE).  The probability enters as the     */
/* integer floor(2^32 p), clamped to 2^32-1, and a 32-bit uniform word r        */
/* accepts iff r < threshold.  thr[k*d + (x/2 - 1)] for x = 2, 4, ..., 2d.      */
/* ------------------------------------------------------------------------ */
static uint32_t or_prob_to_u32(double p) {
  double v = floor(ldexp(p, 32));
  if (v >= 4294967295.0) return 0xFFFFFFFFu;
  if (v <= 0.0) return 0u;
  return (uint32_t)v;
}

OR_EXPORT void or_metro_thresholds(const double *betas, int NT, int d,
                                   uint32_t *thr) {
  for (int k = 0; k < NT; ++k)
    for (int m = 1; m <= d; ++m) {
      int x = 2 * m;
      double dE = (double)(2 * x);
      thr[k * d + (m - 1)] = or_prob_to_u32(exp(-(betas[k] * dE)));
    }
}

/* Replica exchange, Eq. (5): for the pair (k, k+1), with k the colder
   temperature, the swap is accepted with min[1, exp((beta_k - beta_{k+1})
   (E_k - E_{k+1}))].  With D = E_{k+1} - E_k > 0 even, D = 2m, this is
   exp(-(beta_k - beta_{k+1}) * 2m), tabulated for m = 1 .. M-1.  Entry m = 0
   is unused.  Returns the row length M (the smallest M such that every entry
   from M on would be 0, capped at d*N + 1); if thr is NULL only M is
   computed. */
OR_EXPORT int or_pt_thresholds(const double *betas, int NT, int d, int N,
                               uint32_t *thr, int M_alloc) {
  int M = 1;
  for (int k = 0; k + 1 < NT; ++k) {
    double db = betas[k] - betas[k + 1];
    int m = 1;
    while (m <= d * N) {
      if (or_prob_to_u32(exp(-(db * (double)(2 * m)))) == 0u) break;
      ++m;
    }
    if (m > M) M = m;
  }
  if (thr) {
    for (int k = 0; k + 1 < NT; ++k) {
      double db = betas[k] - betas[k + 1];
      thr[(size_t)k * M_alloc + 0] = 0xFFFFFFFFu;
      for (int m = 1; m < M_alloc; ++m)
        thr[(size_t)k * M_alloc + m] =
            (m <= d * N) ? or_prob_to_u32(exp(-(db * (double)(2 * m)))) : 0u;
    }
  }
  return M;
}

/* ------------------------------------------------------------------------ */
/* Job state.                                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  int S, NT, L, d, N, nslot;
  uint64_t seed;
  uint32_t *sample_key;   /* [S] per-sample index used in every RNG counter */
  int8_t *J;              /* [S][d][N] */
  int8_t *s;              /* [S][2NT][N] */
  int64_t *E;             /* [S][2NT] */
  int32_t *sot;           /* [S][2][NT]: slot within set c at temperature k */
  int32_t *tos;           /* [S][2][NT]: temperature of slot j of set c */
  double *beta;           /* [NT] */
  uint32_t *thr;          /* [NT][d] */
  uint32_t *thrpt;        /* [NT-1][M] */
  int M;
  uint64_t t, u, v, n_meas;
  int64_t *mE, *mE2, *mQ, *mAQ, *mQ2; /* [S][NT] */
  unsigned __int128 *mQ4;             /* [S][NT] */
  int32_t *wlab;          /* [S][2NT]: walk label of slot (0 none, 1 up, 2 down) */
  uint32_t *wbeg;         /* [S][2NT]: pass at which its current round trip began */
  uint64_t *trip;         /* [S][32][3]: per log2 bin: trips, sum len, sum len^2 */
  int modes_on;
  int64_t *modes;         /* [S][NT][L/2+1]: plane-sum autocorrelations A(delta) */
  int every;              /* or_mcs measures when the sweep count is a multiple */
  int64_t *stats;         /* [S][NT][OR_NSTAT] run diagnostics (always kept here) */
} or_job;

/* Run diagnostics per sample and temperature k (Sec. 2.3 discusses acceptance
   rates, Sec. 3 the spread of cluster sizes): [0] accepted Metropolis flips of
   the configurations at k during a sweep (both sets), [1] accepted exchanges
   of the pair (k, k+1) (both sets), [2] Houdayer passes at k that exchanged at
   least one site, [3] sites they exchanged, [4 + b] passes that exchanged
   between 2^b and 2^(b+1) - 1 sites. */
#define OR_NSTAT 24

static int8_t *or_lat(or_job *jb, int s, int slot) {
  return jb->s + ((size_t)s * jb->nslot + slot) * jb->N;
}
static const int8_t *or_cpl(const or_job *jb, int s) {
  return jb->J + (size_t)s * jb->d * jb->N;
}

OR_EXPORT void or_recompute_energies(or_job *jb) {
  for (int s = 0; s < jb->S; ++s)
    for (int r = 0; r < jb->nslot; ++r)
      jb->E[(size_t)s * jb->nslot + r] =
          or_energy(jb->L, jb->d, or_cpl(jb, s), or_lat(jb, s, r));
}

/* Create a job.  sample_key may be NULL (samples keyed 0..S-1); otherwise it
   gives the index each sample uses in its random-number counters, so that a
   subset of a larger job can be reproduced exactly. */
OR_EXPORT or_job *or_create(int S, int NT, int L, int d, const int8_t *J,
                            const double *betas, uint64_t seed,
                            const uint32_t *sample_key) {
  if (S < 1 || NT < 2 || L < 3 || (d != 2 && d != 3)) return NULL;
  or_job *jb = (or_job *)calloc(1, sizeof(or_job));
  jb->S = S; jb->NT = NT; jb->L = L; jb->d = d;
  jb->N = (d == 3) ? L * L * L : L * L;
  jb->nslot = 2 * NT;
  jb->seed = seed;
  size_t N = jb->N;
  jb->sample_key = (uint32_t *)malloc(sizeof(uint32_t) * S);
  for (int s = 0; s < S; ++s) jb->sample_key[s] = sample_key ? sample_key[s] : (uint32_t)s;
  jb->J = (int8_t *)malloc((size_t)S * d * N);
  memcpy(jb->J, J, (size_t)S * d * N);
  jb->s = (int8_t *)malloc((size_t)S * jb->nslot * N);
  jb->E = (int64_t *)calloc((size_t)S * jb->nslot, sizeof(int64_t));
  jb->sot = (int32_t *)malloc(sizeof(int32_t) * S * 2 * NT);
  jb->tos = (int32_t *)malloc(sizeof(int32_t) * S * 2 * NT);
  jb->beta = (double *)malloc(sizeof(double) * NT);
  memcpy(jb->beta, betas, sizeof(double) * NT);
  jb->thr = (uint32_t *)malloc(sizeof(uint32_t) * NT * d);
  or_metro_thresholds(betas, NT, d, jb->thr);
  jb->M = or_pt_thresholds(betas, NT, d, (int)N, NULL, 0);
  jb->thrpt = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(NT - 1) * jb->M);
  or_pt_thresholds(betas, NT, d, (int)N, jb->thrpt, jb->M);
  size_t ST = (size_t)S * NT;
  jb->mE = (int64_t *)calloc(ST, sizeof(int64_t));
  jb->mE2 = (int64_t *)calloc(ST, sizeof(int64_t));
  jb->mQ = (int64_t *)calloc(ST, sizeof(int64_t));
  jb->mAQ = (int64_t *)calloc(ST, sizeof(int64_t));
  jb->mQ2 = (int64_t *)calloc(ST, sizeof(int64_t));
  jb->mQ4 = (unsigned __int128 *)calloc(ST, sizeof(unsigned __int128));
  jb->wlab = (int32_t *)calloc((size_t)S * jb->nslot, sizeof(int32_t));
  jb->wbeg = (uint32_t *)calloc((size_t)S * jb->nslot, sizeof(uint32_t));
  jb->trip = (uint64_t *)calloc((size_t)S * 32 * 3, sizeof(uint64_t));
  jb->every = 1;
  jb->stats = (int64_t *)calloc((size_t)S * NT * OR_NSTAT, sizeof(int64_t));
  /* initial spins: one Philox word per site, s = -1 iff its top bit is set */
  for (int s = 0; s < S; ++s)
    for (int r = 0; r < jb->nslot; ++r) {
      int8_t *lat = or_lat(jb, s, r);
      for (int i = 0; i < (int)N; ++i) {
        uint32_t w = or_rand_word(seed, (uint32_t)(i >> 2), 0u, (uint32_t)r,
                                  OR_TAG_INIT, jb->sample_key[s], i & 3);
        lat[i] = (w >> 31) ? (int8_t)-1 : (int8_t)1;
      }
    }
  /* identity temperature maps: slot j of each set starts at temperature j */
  for (int s = 0; s < S; ++s)
    for (int c = 0; c < 2; ++c)
      for (int k = 0; k < NT; ++k) {
        jb->sot[((size_t)s * 2 + c) * NT + k] = k;
        jb->tos[((size_t)s * 2 + c) * NT + k] = k;
      }
  or_recompute_energies(jb);
  return jb;
}

OR_EXPORT void or_destroy(or_job *jb) {
  if (!jb) return;
  free(jb->sample_key); free(jb->J); free(jb->s); free(jb->E);
  free(jb->sot); free(jb->tos); free(jb->beta); free(jb->thr); free(jb->thrpt);
  free(jb->mE); free(jb->mE2); free(jb->mQ); free(jb->mAQ); free(jb->mQ2);
  free(jb->mQ4); free(jb->wlab); free(jb->wbeg); free(jb->trip); free(jb->modes);
  free(jb->stats);
  free(jb);
}

/* ------------------------------------------------------------------------ */
/* Metropolis sweep (Sec. 2.2 and the update list of Sec. 2.4).               */
/* Checkerboard order: all colour-0 sites in increasing i, then colour 1.     */
/* The random word of site i in sweep t comes from the Philox counter         */
/*   (R*G + (b>>2), 2t + colour, slot, TAG_METRO<<28 | sample)                */
/* with R = i / L the row, b = x0 >> 1 the rank of the site among the sites  */
/* of its colour in that row, G = ceil(L/8) Philox blocks per row, and the     */
/* word b & 3 of the four the call returns.                                   */
/* ------------------------------------------------------------------------ */
OR_EXPORT void or_sweep(or_job *jb, int n) {
  const int L = jb->L, d = jb->d, N = jb->N, NT = jb->NT;
  const uint32_t G = (uint32_t)((L + 7) / 8);
  for (int rep = 0; rep < n; ++rep) {
    for (int s = 0; s < jb->S; ++s) {
      const int8_t *Js = or_cpl(jb, s);
      for (int slot = 0; slot < jb->nslot; ++slot) {
        int set = slot / NT, j = slot % NT;
        int k = jb->tos[((size_t)s * 2 + set) * NT + j];
        int8_t *lat = or_lat(jb, s, slot);
        int64_t *Eslot = &jb->E[(size_t)s * jb->nslot + slot];
        for (int colour = 0; colour < 2; ++colour) {
          for (int i = 0; i < N; ++i) {
            if (or_colour(L, d, i) != colour) continue;
            int x = or_local_x(L, d, Js, lat, i);
            int flip;
            if (x <= 0) {
              flip = 1;
            } else {
              uint32_t R = (uint32_t)(i / L), b = (uint32_t)((i % L) >> 1);
              uint32_t r = or_rand_word(jb->seed, R * G + (b >> 2),
                                        (uint32_t)(2 * jb->t + colour),
                                        (uint32_t)slot, OR_TAG_METRO,
                                        jb->sample_key[s], (int)(b & 3));
              flip = r < jb->thr[k * d + (x / 2 - 1)];
            }
            if (flip) {
              lat[i] = (int8_t)-lat[i];
              *Eslot += 2 * x;
              jb->stats[((size_t)s * NT + k) * OR_NSTAT + 0] += 1;
            }
          }
        }
      }
    }
    jb->t += 1;
  }
}

/* ------------------------------------------------------------------------ */
/* Replica walk and round-trip time (Sec. 2.3).  The round-trip or tunnelling */
/* time is the expected number of Monte Carlo steps a configuration needs to   */
/* travel from the lowest temperature to the highest and back.  Reading:       */
/* every stored configuration (slot) is looked at after each exchange pass,    */
/* numbered m = 1, 2, ... (the pass counter after the pass).  A slot carries a */
/* label: 0 until it first sits at the lowest temperature; 1 ("going up") from */
/* then on; 2 ("going down") once it reaches the highest temperature while     */
/* labelled 1.  When a slot labelled 2 is back at the lowest temperature, one  */
/* round trip ends; its length is m minus the pass at which the label last    */
/* became 1, and the label becomes 1 again with the new trip beginning at m.   */
/* Slots revisiting the lowest temperature while labelled 1 change nothing.   */
/* A trip ending at pass m is filed in the logarithmic bin floor(log2 m) of    */
/* its sample (both replica sets together): count, sum of lengths, sum of      */
/* squared lengths.  Houdayer moves exchange spins, not slots, and do not     */
/* enter.  Called once per set and pass, after the pass.                       */
/* ------------------------------------------------------------------------ */
static void or_walk_observe(or_job *jb, int s, int c, uint64_t m) {
  const int NT = jb->NT;
  for (int j = 0; j < NT; ++j) {
    const size_t o = (size_t)s * jb->nslot + (size_t)c * NT + j;
    const int k = jb->tos[((size_t)s * 2 + c) * NT + j];
    if (k == 0) {
      if (jb->wlab[o] == 2) {
        uint64_t len = m - (uint64_t)jb->wbeg[o];
        int bin = 0;
        while ((m >> (bin + 1)) != 0) ++bin;
        uint64_t *t = &jb->trip[((size_t)s * 32 + bin) * 3];
        t[0] += 1;
        t[1] += len;
        t[2] += len * len;
      }
      if (jb->wlab[o] != 1) {
        jb->wlab[o] = 1;
        jb->wbeg[o] = (uint32_t)m;
      }
    } else if (k == NT - 1 && jb->wlab[o] == 1) {
      jb->wlab[o] = 2;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Parallel-tempering pass (Sec. 2.2, Eq. (5); temperatures are exchanged,    */
/* not configurations, via two index arrays, Sec. 3).  For each sample and     */
/* each replica set c separately, k = 0 .. NT-2 in ascending order.            */
/* Random word: Philox counter (k, u, c, TAG_PT<<28 | sample), word 0.         */
/* ------------------------------------------------------------------------ */
OR_EXPORT void or_exchange(or_job *jb) {
  const int NT = jb->NT;
  for (int s = 0; s < jb->S; ++s)
    for (int c = 0; c < 2; ++c) {
      int32_t *sot = &jb->sot[((size_t)s * 2 + c) * NT];
      int32_t *tos = &jb->tos[((size_t)s * 2 + c) * NT];
      for (int k = 0; k + 1 < NT; ++k) {
        int a = sot[k], b = sot[k + 1];
        int64_t Ea = jb->E[(size_t)s * jb->nslot + c * NT + a];
        int64_t Eb = jb->E[(size_t)s * jb->nslot + c * NT + b];
        int64_t D = Eb - Ea;
        int acc;
        if (D <= 0) {
          acc = 1;
        } else {
          int64_t m = D / 2;
          uint32_t th = (m < jb->M) ? jb->thrpt[(size_t)k * jb->M + m] : 0u;
          uint32_t r = or_rand_word(jb->seed, (uint32_t)k, (uint32_t)jb->u,
                                    (uint32_t)c, OR_TAG_PT, jb->sample_key[s], 0);
          acc = r < th;
        }
        if (acc) {
          sot[k] = b; sot[k + 1] = a;
          tos[b] = k; tos[a] = k + 1;
          jb->stats[((size_t)s * NT + k) * OR_NSTAT + 1] += 1;
        }
      }
      or_walk_observe(jb, s, c, jb->u + 1);
    }
  jb->u += 1;
}

/* ------------------------------------------------------------------------ */
/* Houdayer cluster move (Sec. 2.4, Eq. (10)) on one pair of replicas a, b     */
/* sharing disorder and temperature.  q_i = s_i^a s_i^b.  The seed i0 is the   */
/* idx-th q=-1 site in increasing i, idx = floor(r64 * n_minus / 2^64).  The   */
/* cluster is every q=-1 site reachable from i0 through nearest neighbours     */
/* with q=-1 (breadth-first search, couplings ignored).  Both replicas are     */
/* negated on the cluster, which is the same as exchanging them there.         */
/* Returns delta with E_a += delta, E_b -= delta.  cluster_out (may be NULL)   */
/* receives 1 on cluster sites.  Returns 0 and leaves everything untouched     */
/* when no site has q=-1.                                                     */
/* ------------------------------------------------------------------------ */
OR_EXPORT int64_t or_houdayer_move(int L, int d, const int8_t *Jsample,
                                   int8_t *sa, int8_t *sb, uint64_t r64,
                                   int8_t *cluster_out, int32_t *cluster_size) {
  int N = (d == 3) ? L * L * L : L * L;
  int32_t *minus = (int32_t *)malloc(sizeof(int32_t) * N);
  int nm = 0;
  for (int i = 0; i < N; ++i)
    if (sa[i] != sb[i]) minus[nm++] = i;
  if (cluster_size) *cluster_size = 0;
  if (nm == 0) {
    if (cluster_out) memset(cluster_out, 0, (size_t)N);
    free(minus);
    return 0;
  }
  uint64_t idx = (uint64_t)(((unsigned __int128)r64 * (uint64_t)nm) >> 64);
  int i0 = minus[idx];
  free(minus);

  int8_t *in = (int8_t *)calloc((size_t)N, 1);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * N);
  int head = 0, tail = 0;
  in[i0] = 1;
  queue[tail++] = i0;
  while (head < tail) {
    int i = queue[head++];
    for (int mu = 0; mu < d; ++mu)
      for (int dir = -1; dir <= 1; dir += 2) {
        int j = or_neighbour(L, d, i, mu, dir);
        if (!in[j] && sa[j] != sb[j]) {
          in[j] = 1;
          queue[tail++] = j;
        }
      }
  }
  /* energy change of replica a: every bond leaving the cluster changes sign */
  int64_t delta = 0;
  for (int q = 0; q < tail; ++q) {
    int i = queue[q];
    for (int mu = 0; mu < d; ++mu)
      for (int dir = -1; dir <= 1; dir += 2) {
        int j = or_neighbour(L, d, i, mu, dir);
        if (!in[j])
          delta += 2 * (int64_t)or_bond(Jsample, L, d, N, i, mu, dir) * sa[i] * sa[j];
      }
  }
  for (int q = 0; q < tail; ++q) {
    int i = queue[q];
    sa[i] = (int8_t)-sa[i];
    sb[i] = (int8_t)-sb[i];
  }
  if (cluster_out) memcpy(cluster_out, in, (size_t)N);
  if (cluster_size) *cluster_size = tail;
  free(in);
  free(queue);
  return delta;
}

/* Diagnostics of one Houdayer move at temperature k that exchanged `size`
   sites. */
static void or_count_exchanged(or_job *jb, int s, int k, int32_t size) {
  if (size <= 0) return;
  int64_t *st = &jb->stats[((size_t)s * jb->NT + k) * OR_NSTAT];
  int b = 0;
  while ((size >> (b + 1)) != 0) ++b;
  st[2] += 1;
  st[3] += size;
  st[4 + b] += 1;
}

/* One Houdayer pass: every sample, every temperature k, pair (set 0, set 1)
   at k after the temperature relabelling.  Random word: Philox counter
   (k, v, 0, TAG_HOU<<28 | sample), r64 = w0 | w1 << 32. */
OR_EXPORT void or_houdayer(or_job *jb) {
  const int NT = jb->NT;
  uint32_t key[2] = {(uint32_t)jb->seed, (uint32_t)(jb->seed >> 32)};
  for (int s = 0; s < jb->S; ++s)
    for (int k = 0; k < NT; ++k) {
      int a = 0 * NT + jb->sot[((size_t)s * 2 + 0) * NT + k];
      int b = 1 * NT + jb->sot[((size_t)s * 2 + 1) * NT + k];
      uint32_t ctr[4] = {(uint32_t)k, (uint32_t)jb->v, 0u,
                         ((uint32_t)OR_TAG_HOU << 28) | jb->sample_key[s]};
      uint32_t w[4];
      or_philox4x32_10(ctr, key, w);
      uint64_t r64 = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
      int32_t size = 0;
      int64_t delta = or_houdayer_move(jb->L, jb->d, or_cpl(jb, s),
                                       or_lat(jb, s, a), or_lat(jb, s, b), r64,
                                       NULL, &size);
      jb->E[(size_t)s * jb->nslot + a] += delta;
      jb->E[(size_t)s * jb->nslot + b] -= delta;
      or_count_exchanged(jb, s, k, size);
    }
  jb->v += 1;
}

/* ------------------------------------------------------------------------ */
/* Multi-cluster variant of the Houdayer move.  Sec. 3 proposes turning the    */
/* single-cluster update into a multi-cluster one, and Sec. 5 names this as    */
/* the way to remove the idling that clusters of uneven size cause.  On the    */
/* pair (a, b), every nearest-neighbour cluster of q = -1 sites is exchanged,  */
/* independently of the others, with probability 1/2.  A cluster is named by   */
/* its lowest site m and is exchanged iff coin[m] != 0 (coin has N entries;    */
/* only those of the clusters' lowest sites are read).  Clusters are found in  */
/* increasing order of m: a breadth-first search from each q = -1 site not     */
/* yet in a cluster, taken in increasing i, starts at the cluster's lowest     */
/* site.  Two clusters are never adjacent (adjacent q = -1 sites belong to one */
/* cluster), so the neighbours outside a cluster have q = +1 and no exchange   */
/* moves them: each cluster's energy change is computed from the state before */
/* the move, and the order of the exchanges does not matter.  Returns delta    */
/* with E_a += delta, E_b -= delta.  flip_out (may be NULL) receives 1 on      */
/* exchanged sites, *nclusters (may be NULL) the number of clusters.           */
/* ------------------------------------------------------------------------ */
OR_EXPORT int64_t or_houdayer_multi_move(int L, int d, const int8_t *Jsample,
                                         int8_t *sa, int8_t *sb, const uint8_t *coin,
                                         int8_t *flip_out, int32_t *nclusters) {
  int N = (d == 3) ? L * L * L : L * L;
  int8_t *seen = (int8_t *)calloc((size_t)N, 1);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * N);
  int64_t delta = 0;
  int32_t count = 0;
  if (flip_out) memset(flip_out, 0, (size_t)N);
  for (int m = 0; m < N; ++m) {
    if (seen[m] || sa[m] == sb[m]) continue;
    /* the cluster whose lowest site is m */
    int head = 0, tail = 0;
    seen[m] = 1;
    queue[tail++] = m;
    while (head < tail) {
      int i = queue[head++];
      for (int mu = 0; mu < d; ++mu)
        for (int dir = -1; dir <= 1; dir += 2) {
          int j = or_neighbour(L, d, i, mu, dir);
          if (!seen[j] && sa[j] != sb[j]) {
            seen[j] = 1;
            queue[tail++] = j;
          }
        }
    }
    count += 1;
    if (!coin[m]) continue;
    /* every bond leaving the cluster changes sign in replica a */
    for (int q = 0; q < tail; ++q) {
      int i = queue[q];
      for (int mu = 0; mu < d; ++mu)
        for (int dir = -1; dir <= 1; dir += 2) {
          int j = or_neighbour(L, d, i, mu, dir);
          if (sa[j] == sb[j])
            delta += 2 * (int64_t)or_bond(Jsample, L, d, N, i, mu, dir) * sa[i] * sa[j];
        }
    }
    for (int q = 0; q < tail; ++q) {
      int i = queue[q];
      sa[i] = (int8_t)-sa[i];
      sb[i] = (int8_t)-sb[i];
      if (flip_out) flip_out[i] = 1;
    }
  }
  if (nclusters) *nclusters = count;
  free(seen);
  free(queue);
  return delta;
}

/* Coins of one multi-cluster move: coin[m] = bit (m mod 128) of the 128-bit
   output of the Philox counter (m / 128, v, k, TAG_HOU_MULTI<<28 | sample),
   bit j of the output being bit j mod 32 of word j / 32. */
OR_EXPORT void or_multi_coins(uint64_t seed, uint32_t sample, uint32_t k, uint32_t v, int N,
                              uint8_t *coin) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int m = 0; m < N; m += 128) {
    uint32_t ctr[4] = {(uint32_t)(m / 128), v, k, ((uint32_t)OR_TAG_HOU_MULTI << 28) | sample};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    for (int j = 0; j < 128 && m + j < N; ++j) coin[m + j] = (uint8_t)((w[j / 32] >> (j % 32)) & 1u);
  }
}

/* One multi-cluster Houdayer pass: every sample, every temperature k, pair
   (set 0, set 1) at k after the temperature relabelling, coins from
   or_multi_coins with the Houdayer pass counter v (shared with the
   single-cluster move). */
OR_EXPORT void or_houdayer_multi(or_job *jb) {
  const int NT = jb->NT;
  uint8_t *coin = (uint8_t *)malloc((size_t)jb->N);
  for (int s = 0; s < jb->S; ++s)
    for (int k = 0; k < NT; ++k) {
      int a = 0 * NT + jb->sot[((size_t)s * 2 + 0) * NT + k];
      int b = 1 * NT + jb->sot[((size_t)s * 2 + 1) * NT + k];
      or_multi_coins(jb->seed, jb->sample_key[s], (uint32_t)k, (uint32_t)jb->v, jb->N, coin);
      int8_t *fl = (int8_t *)malloc((size_t)jb->N);
      int64_t delta = or_houdayer_multi_move(jb->L, jb->d, or_cpl(jb, s), or_lat(jb, s, a),
                                             or_lat(jb, s, b), coin, fl, NULL);
      jb->E[(size_t)s * jb->nslot + a] += delta;
      jb->E[(size_t)s * jb->nslot + b] -= delta;
      int32_t size = 0;
      for (int i = 0; i < jb->N; ++i) size += fl[i];
      free(fl);
      or_count_exchanged(jb, s, k, size);
    }
  free(coin);
  jb->v += 1;
}

/* ------------------------------------------------------------------------ */
/* Two-replica modes (usual definitions; the paper names the quantities but   */
/* does not define them).  With the overlap field q_i = s_i^a s_i^b and the    */
/* plane sums P_mu(x) = sum of q_i over the sites with coordinate x_mu = x,     */
/* the Fourier mode of q along axis mu at k = 2 pi n / L has                   */
/*   |sum_i q_i e^{i k x_mu}|^2 = sum_{delta=0}^{L-1} cos(k delta) C_mu(delta), */
/* C_mu(delta) = sum_x P_mu(x) P_mu((x + delta) mod L).  A(delta) is the sum    */
/* of C_mu(delta) over the d axes, an exact integer; C_mu(L - delta) =          */
/* C_mu(delta), so delta = 0 .. floor(L/2) carries everything.  Writes          */
/* A(0 .. floor(L/2)) to out.                                                   */
/* ------------------------------------------------------------------------ */
OR_EXPORT void or_overlap_modes(int L, int d, const int8_t *sa, const int8_t *sb,
                                int64_t *out) {
  int N = (d == 3) ? L * L * L : L * L;
  int64_t *P = (int64_t *)calloc((size_t)3 * L, sizeof(int64_t));
  for (int i = 0; i < N; ++i) {
    int x[3];
    or_coords(L, d, i, x);
    int q = sa[i] * sb[i];
    for (int mu = 0; mu < d; ++mu) P[mu * L + x[mu]] += q;
  }
  for (int delta = 0; delta <= L / 2; ++delta) {
    int64_t A = 0;
    for (int mu = 0; mu < d; ++mu)
      for (int x = 0; x < L; ++x)
        A += P[mu * L + x] * P[mu * L + (x + delta) % L];
    out[delta] = A;
  }
  free(P);
}

/* Accumulate the modes at every measurement from now on. */
OR_EXPORT void or_enable_modes(or_job *jb) {
  if (jb->modes_on) return;
  jb->modes_on = 1;
  jb->modes = (int64_t *)calloc((size_t)jb->S * jb->NT * (jb->L / 2 + 1), sizeof(int64_t));
}

/* ------------------------------------------------------------------------ */
/* Measurement (Sec. 2.1, Eqs. (3), (4); measurement step of Sec. 3).          */
/* Per sample and temperature k: the two replicas at k (one per set) give      */
/* E_a, E_b and the overlap Q = sum_i s_i^a s_i^b.  Exact integer sums of E,    */
/* E^2 (both replicas), Q, |Q|, Q^2, Q^4 are accumulated.                      */
/* ------------------------------------------------------------------------ */
OR_EXPORT void or_measure(or_job *jb) {
  const int NT = jb->NT, N = jb->N;
  for (int s = 0; s < jb->S; ++s)
    for (int k = 0; k < NT; ++k) {
      int a = 0 * NT + jb->sot[((size_t)s * 2 + 0) * NT + k];
      int b = 1 * NT + jb->sot[((size_t)s * 2 + 1) * NT + k];
      const int8_t *la = or_lat(jb, s, a), *lb = or_lat(jb, s, b);
      int64_t Q = 0;
      for (int i = 0; i < N; ++i) Q += (int64_t)la[i] * lb[i];
      int64_t Ea = jb->E[(size_t)s * jb->nslot + a];
      int64_t Eb = jb->E[(size_t)s * jb->nslot + b];
      size_t o = (size_t)s * NT + k;
      jb->mE[o] += Ea + Eb;
      jb->mE2[o] += Ea * Ea + Eb * Eb;
      jb->mQ[o] += Q;
      jb->mAQ[o] += Q < 0 ? -Q : Q;
      jb->mQ2[o] += Q * Q;
      unsigned __int128 q2 = (unsigned __int128)(Q * Q);
      jb->mQ4[o] += q2 * q2;
      if (jb->modes_on) {
        const int nm = jb->L / 2 + 1;
        int64_t *A = (int64_t *)malloc(sizeof(int64_t) * nm);
        or_overlap_modes(jb->L, jb->d, la, lb, A);
        for (int m = 0; m < nm; ++m) jb->modes[o * nm + m] += A[m];
        free(A);
      }
    }
  jb->n_meas += 1;
}

/* Measurements at intervals (Sec. 3): or_mcs then measures only after the
   sweeps whose count (from 1) is a multiple of every. */
OR_EXPORT void or_set_measure_every(or_job *jb, int every) {
  jb->every = every < 1 ? 1 : every;
}

/* One Monte Carlo step in the order of Sec. 2.4: one Metropolis sweep, then
   (optionally) one Houdayer move per same-temperature pair -- houdayer = 1
   the single-cluster move, 2 the multi-cluster one -- then one
   replica-exchange pass, then (optionally) one measurement. */
OR_EXPORT void or_mcs(or_job *jb, int n, int houdayer, int measure) {
  for (int i = 0; i < n; ++i) {
    or_sweep(jb, 1);
    if (houdayer == 2) or_houdayer_multi(jb);
    else if (houdayer) or_houdayer(jb);
    or_exchange(jb);
    if (measure && jb->t % (uint64_t)jb->every == 0) or_measure(jb);
  }
}

/* Observables.  per_sample [S][NT][5] = e, q, |q|, q^2, q^4 (Eqs. (3), (4)
   without the disorder average); disorder [NT][6] = the same disorder-averaged
   (integer numerators summed over samples first) plus the Binder parameter
   g = (3 - [<q^4>] / [<q^2>]^2) / 2.  Either output may be NULL. */
OR_EXPORT void or_observables(const or_job *jb, double *per_sample,
                              double *disorder, int64_t *n_meas) {
  const int NT = jb->NT;
  const double n = (double)jb->n_meas, N = (double)jb->N;
  if (n_meas) *n_meas = (int64_t)jb->n_meas;
  if (per_sample) {
    for (int s = 0; s < jb->S; ++s)
      for (int k = 0; k < NT; ++k) {
        size_t o = (size_t)s * NT + k;
        double *out = per_sample + o * 5;
        out[0] = (double)jb->mE[o] / (2.0 * n * N);
        out[1] = (double)jb->mQ[o] / (n * N);
        out[2] = (double)jb->mAQ[o] / (n * N);
        out[3] = (double)jb->mQ2[o] / (n * (N * N));
        out[4] = (double)jb->mQ4[o] / (n * ((N * N) * (N * N)));
      }
  }
  if (disorder) {
    const double S = (double)jb->S;
    for (int k = 0; k < NT; ++k) {
      int64_t sE = 0, sQ = 0, sAQ = 0, sQ2 = 0;
      unsigned __int128 sQ4 = 0;
      for (int s = 0; s < jb->S; ++s) {
        size_t o = (size_t)s * NT + k;
        sE += jb->mE[o]; sQ += jb->mQ[o]; sAQ += jb->mAQ[o];
        sQ2 += jb->mQ2[o]; sQ4 += jb->mQ4[o];
      }
      double *out = disorder + (size_t)k * 6;
      out[0] = (double)sE / (S * 2.0 * n * N);
      out[1] = (double)sQ / (S * n * N);
      out[2] = (double)sAQ / (S * n * N);
      out[3] = (double)sQ2 / (S * n * (N * N));
      out[4] = (double)sQ4 / (S * n * ((N * N) * (N * N)));
      out[5] = 0.5 * (3.0 - out[4] / (out[3] * out[3]));
    }
  }
}

/* ------------------------------------------------------------------------ */
/* State access for the tests.                                                */
/* ------------------------------------------------------------------------ */
OR_EXPORT void or_get_spins(const or_job *jb, int8_t *out) {
  memcpy(out, jb->s, (size_t)jb->S * jb->nslot * jb->N);
}
/* Replaces every spin and recomputes every energy from scratch. */
OR_EXPORT void or_set_spins(or_job *jb, const int8_t *in) {
  memcpy(jb->s, in, (size_t)jb->S * jb->nslot * jb->N);
  or_recompute_energies(jb);
}
OR_EXPORT void or_get_energies(const or_job *jb, int64_t *out) {
  memcpy(out, jb->E, sizeof(int64_t) * jb->S * jb->nslot);
}
OR_EXPORT void or_get_maps(const or_job *jb, int32_t *sot, int32_t *tos) {
  if (sot) memcpy(sot, jb->sot, sizeof(int32_t) * jb->S * 2 * jb->NT);
  if (tos) memcpy(tos, jb->tos, sizeof(int32_t) * jb->S * 2 * jb->NT);
}
OR_EXPORT void or_get_counters(const or_job *jb, uint64_t out[4]) {
  out[0] = jb->t; out[1] = jb->u; out[2] = jb->v; out[3] = jb->n_meas;
}
/* Raw moment numerators, [S][NT] each; Q^4 as (lo, hi) 64-bit halves. */
OR_EXPORT void or_get_moments(const or_job *jb, int64_t *mE, int64_t *mE2,
                              int64_t *mQ, int64_t *mAQ, int64_t *mQ2,
                              uint64_t *mQ4_lohi) {
  size_t ST = (size_t)jb->S * jb->NT;
  memcpy(mE, jb->mE, sizeof(int64_t) * ST);
  memcpy(mE2, jb->mE2, sizeof(int64_t) * ST);
  memcpy(mQ, jb->mQ, sizeof(int64_t) * ST);
  memcpy(mAQ, jb->mAQ, sizeof(int64_t) * ST);
  memcpy(mQ2, jb->mQ2, sizeof(int64_t) * ST);
  for (size_t o = 0; o < ST; ++o) {
    mQ4_lohi[2 * o] = (uint64_t)jb->mQ4[o];
    mQ4_lohi[2 * o + 1] = (uint64_t)(jb->mQ4[o] >> 64);
  }
}
/* Walk labels and trip beginnings [S][2NT]; round-trip bins [S][32][3]. */
OR_EXPORT void or_get_walk(const or_job *jb, int32_t *label, uint32_t *begin,
                           uint64_t *trips) {
  size_t n = (size_t)jb->S * jb->nslot;
  if (label) memcpy(label, jb->wlab, sizeof(int32_t) * n);
  if (begin) memcpy(begin, jb->wbeg, sizeof(uint32_t) * n);
  if (trips) memcpy(trips, jb->trip, sizeof(uint64_t) * (size_t)jb->S * 32 * 3);
}
/* Run diagnostics [S][NT][OR_NSTAT]. */
OR_EXPORT void or_get_stats(const or_job *jb, int64_t *out) {
  memcpy(out, jb->stats, sizeof(int64_t) * (size_t)jb->S * jb->NT * OR_NSTAT);
}

/* Accumulated modes [S][NT][L/2+1] (zeros if never enabled). */
OR_EXPORT void or_get_modes(const or_job *jb, int64_t *out) {
  size_t n = (size_t)jb->S * jb->NT * (jb->L / 2 + 1);
  if (jb->modes_on) memcpy(out, jb->modes, sizeof(int64_t) * n);
  else memset(out, 0, sizeof(int64_t) * n);
}
OR_EXPORT int or_pt_table_len(const or_job *jb) { return jb->M; }
OR_EXPORT void or_get_pt_table(const or_job *jb, uint32_t *out) {
  memcpy(out, jb->thrpt, sizeof(uint32_t) * (size_t)(jb->NT - 1) * jb->M);
}

/* The order in which one sweep visits sites: colour 0 in increasing i, then
   colour 1.  Writes N site indices. */
OR_EXPORT void or_sweep_order(int L, int d, int32_t *order) {
  int N = (d == 3) ? L * L * L : L * L, n = 0;
  for (int colour = 0; colour < 2; ++colour)
    for (int i = 0; i < N; ++i)
      if (or_colour(L, d, i) == colour) order[n++] = i;
}

/* The single-site Metropolis rule: flip iff x <= 0 or r < thr_row[x/2 - 1]. */
OR_EXPORT int or_metro_rule(int x, uint32_t r, const uint32_t *thr_row) {
  if (x <= 0) return 1;
  return r < thr_row[x / 2 - 1];
}
