/*
 * enum.c -- TEST INFRASTRUCTURE ONLY: exact enumeration of tiny lattices.
 *
 * Independent of ea_oracle.c (its own geometry and energy loop) so that it can
 * pin the simulation oracle: equilibrium averages of the EA Hamiltonian,
 * Sec. 2.1 Eq. (1) at zero field, follow exactly from the density of states.
 * A state z in [0, 2^N) has s_i = -1 iff bit i of z is set; sites are
 * numbered x0 + L*x1 (+ L^2*x2) and the bond (i, i+e_mu) is J[mu*N + i].
 */
#include <stdint.h>
#include <stdlib.h>

#define EN_EXPORT __attribute__((visibility("default")))

static int en_nsites(int L, int d) { return d == 3 ? L * L * L : L * L; }

/* nb[i*2d + 2mu] = i + e_mu, nb[i*2d + 2mu + 1] = i - e_mu (periodic);
   jb[...] the coupling of that bond. */
static void en_tables(int L, int d, const int8_t *J, int32_t *nb, int8_t *jb) {
  int N = en_nsites(L, d);
  for (int i = 0; i < N; ++i) {
    int c[3] = {i % L, (i / L) % L, d == 3 ? i / (L * L) : 0};
    for (int mu = 0; mu < d; ++mu) {
      int up[3] = {c[0], c[1], c[2]}, dn[3] = {c[0], c[1], c[2]};
      up[mu] = (c[mu] + 1) % L;
      dn[mu] = (c[mu] + L - 1) % L;
      int iu = up[0] + L * up[1] + L * L * up[2];
      int id = dn[0] + L * dn[1] + L * L * dn[2];
      nb[i * 2 * d + 2 * mu] = iu;
      nb[i * 2 * d + 2 * mu + 1] = id;
      jb[i * 2 * d + 2 * mu] = J[mu * N + i];
      jb[i * 2 * d + 2 * mu + 1] = J[mu * N + id];
    }
  }
}

/* Density of states: counts[E + d*N] = #states with energy E.  Gray-code walk,
   one spin flip per step.  N <= 30. */
EN_EXPORT int en_density_of_states(int L, int d, const int8_t *J,
                                   uint64_t *counts) {
  int N = en_nsites(L, d);
  if (N > 30) return -1;
  int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * N * 2 * d);
  int8_t *jb = (int8_t *)malloc((size_t)N * 2 * d);
  en_tables(L, d, J, nb, jb);
  int8_t *s = (int8_t *)malloc((size_t)N);
  for (int i = 0; i < N; ++i) s[i] = 1;
  int64_t E = 0;
  for (int i = 0; i < N; ++i)
    for (int mu = 0; mu < d; ++mu) E -= jb[i * 2 * d + 2 * mu];
  for (int e = 0; e <= 2 * d * N; ++e) counts[e] = 0;
  counts[E + (int64_t)d * N] += 1;
  uint64_t total = (uint64_t)1 << N;
  for (uint64_t g = 1; g < total; ++g) {
    int i = __builtin_ctzll(g);
    int h = 0;
    for (int q = 0; q < 2 * d; ++q) h += jb[i * 2 * d + q] * s[nb[i * 2 * d + q]];
    E += 2 * s[i] * h;
    s[i] = (int8_t)-s[i];
    counts[E + (int64_t)d * N] += 1;
  }
  free(nb); free(jb); free(s);
  return 0;
}

/* Energy of every state z (N <= 24).  E_out has 2^N entries. */
EN_EXPORT int en_state_energies(int L, int d, const int8_t *J, int32_t *E_out) {
  int N = en_nsites(L, d);
  if (N > 24) return -1;
  int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * N * 2 * d);
  int8_t *jb = (int8_t *)malloc((size_t)N * 2 * d);
  en_tables(L, d, J, nb, jb);
  uint64_t total = (uint64_t)1 << N;
  for (uint64_t z = 0; z < total; ++z) {
    int32_t E = 0;
    for (int i = 0; i < N; ++i) {
      int si = (z >> i) & 1 ? -1 : 1;
      for (int mu = 0; mu < d; ++mu) {
        int j = nb[i * 2 * d + 2 * mu];
        int sj = (z >> j) & 1 ? -1 : 1;
        E -= jb[i * 2 * d + 2 * mu] * si * sj;
      }
    }
    E_out[z] = E;
  }
  free(nb); free(jb);
  return 0;
}
