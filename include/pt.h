/*
 * pt.h -- C ABI of the MI355X (gfx950) parallel-tempering EA spin-glass library.
 *
 * The library simulates the +-J Edwards-Anderson Ising spin glass, Eq. (1) of
 * Kumar, Gross, Janke, Weigel (arXiv:2003.04621) at zero field, for many
 * disorder samples at once.  Every sample carries two replica sets (N_C = 2,
 * Sec. 3) of N_T temperatures each, i.e. 2*N_T configurations ("slots").
 * One Monte Carlo step (Sec. 2.4) is: pt_sweep(job, 1), then optionally
 * pt_houdayer(job), then pt_exchange(job), then optionally pt_measure(job).
 *
 * Conventions used by every entry point:
 *   - Lattice: L^dim sites, square (dim 2) or simple cubic (dim 3), periodic.
 *     Site i = x0 + L*x1 (+ L^2*x2).  L must be even, 4 <= L <= 64.
 *   - Couplings: int8 [samples][dim][L^dim], each +1 or -1; entry [s][mu][i]
 *     is the bond between site i and i + e_mu (Eq. (2) draws them).
 *   - Spins: int8 +1/-1 [samples][2*replicas][L^dim], indexed by slot
 *     r = c*replicas + j (replica set c in {0,1}, j < replicas).
 *   - Temperatures: betas[k] = 1/T_k, k = 0 the coldest; strictly decreasing.
 *   - Temperature maps (Sec. 3, two index arrays): slot_of_temp[s][c][k] = j
 *     means slot c*replicas + j currently runs at beta_k; temp_of_slot is its
 *     inverse.  Replica exchange swaps map entries, never spins.
 *   - Energies: int32 [samples][2*replicas], E = -sum_<ij> J_ij s_i s_j.
 *   - Randomness: Philox4x32-10 (Sec. 3, Salmon et al. 2011) keyed by the
 *     64-bit seed; the counter of every draw is a pure function of (sample,
 *     slot, site, sweep/pass), so results do not depend on launch shape.
 *
 * Ownership: input arrays are host memory owned by the caller and are copied
 * before the call returns.  Output arrays are host memory allocated by the
 * caller.  Device state belongs to the job until pt_destroy and is allocated
 * through the hooks of pt_set_allocator (hipMalloc/hipFree if none are set).
 *
 * Synchronisation: pt_sweep, pt_exchange, pt_houdayer, pt_measure and pt_mcs
 * only enqueue work on the job's stream.  pt_observables, pt_get_*, pt_set_*,
 * pt_get_state, pt_set_state and pt_destroy synchronise that stream.  A job
 * handle is not thread-safe; distinct handles may be used concurrently.
 *
 * Errors: every function returns PT_OK (0) or a negative code and never
 * throws.  pt_last_error() gives a thread-local message for the last failure.
 * Invalid arguments (PT_EINVAL) leave the job unchanged.  A HIP failure
 * (PT_EDEVICE) poisons the job; every later call on it returns PT_ESTATE
 * except pt_destroy.
 */
#ifndef PT_SPINGLASS_H
#define PT_SPINGLASS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PT_OK 0
#define PT_EINVAL (-1)
#define PT_ENOMEM (-2)
#define PT_EDEVICE (-3)
#define PT_ESTATE (-4)
#define PT_ECANCELED (-5) /* a served request ended by pt_server_cancel */

/* Device spin layouts (pt_init_ex flags). */
#define PT_LAYOUT_INT8 0u   /* one int8 per spin, lattice-contiguous */
#define PT_LAYOUT_PACKED 1u /* one bit per spin, split by checkerboard colour */
/* Also a pt_init_ex flag (ORed with the layout; accepted by pt_plan_query,
 * pt_job_bytes and in pt_request.layout): the job keeps the replica walk in
 * temperature space and its round trips (pt_get_walk).  Off by default: the
 * fused kernels then carry no walk code at all. */
#define PT_TRACK_WALK 0x10u
/* Also a pt_init_ex flag (same places as PT_TRACK_WALK): every measurement
 * also accumulates the two-replica modes of each temperature (pt_get_modes,
 * pt_correlation_length).  Off by default: the fused kernels then carry no
 * mode code. */
#define PT_TRACK_MODES 0x20u
/* Also a pt_init_ex flag (and accepted by pt_job_bytes): the job keeps run
 * diagnostics per sample and temperature (pt_get_stats).  Such a job always
 * runs the per-step kernels (pt_mcs and pt_mcs_noalloc take them; batches
 * and the server refuse it); results are bit-identical either way. */
#define PT_TRACK_STATS 0x80u

/* pt_mcs flags */
#define PT_MCS_HOUDAYER 1u
#define PT_MCS_MEASURE 2u
#define PT_MCS_PLAIN 4u /* force the separate per-step kernels */
#define PT_BATCH_GRAPH 8u /* pt_batch_run: replay a captured hipGraph of the launch */
/* With PT_MCS_HOUDAYER (pt_mcs, pt_batch_run, pt_request.flags):
 * the Houdayer moves are the multi-cluster variant (pt_houdayer_multi). */
#define PT_MCS_MULTICLUSTER 0x40u

typedef struct pt_job pt_job;
typedef struct pt_batch pt_batch;
typedef struct pt_server pt_server;

/* A request to the server: one job (arrays are copied at submission). */
typedef struct {
  int32_t dim, L, replicas, samples; /* as pt_init */
  const double *betas;               /* [replicas] */
  const int8_t *couplings;           /* [samples][dim][L^dim] */
  uint64_t seed;
  int32_t sweeps;                    /* Monte Carlo steps in total */
  int32_t burn_in;                   /* steps before the first measurement */
  uint32_t flags;                    /* PT_MCS_HOUDAYER (| PT_MCS_MULTICLUSTER) and/or
                                        PT_SERVE_UNTIL_EQUILIBRATED, or 0 */
  uint32_t layout;                   /* PT_LAYOUT_INT8 or PT_LAYOUT_PACKED, | PT_TRACK_WALK/_MODES */
  int32_t measure_every;             /* measurement interval (0 or 1: every step), as
                                        pt_set_measure_interval: a step after the burn-in
                                        measures iff its absolute 1-based sweep number is a
                                        multiple of it (so with burn_in 9 and interval 5 the
                                        first measurement is sweep 10) */
  int32_t reserved;
} pt_request;

/* pt_request flag: the job ends between rounds, once past its burn-in, as soon
 * as its round trips pass the logarithmic-binning check of pt_tunnel_summary
 * (Sec. 2.3); `sweeps` is then an upper bound.  Needs PT_TRACK_WALK. */
#define PT_SERVE_UNTIL_EQUILIBRATED 0x100u

/* pt_batch_tune flag: try both spin layouts as well as the launch shapes. */
#define PT_TUNE_LAYOUT 0x200u

/* The outcome of a request; times in seconds since pt_server_start. */
typedef struct {
  int32_t status;       /* PT_OK, or the error that ended the request */
  int32_t equilibrated; /* with PT_TRACK_WALK: the round-trip check, 1 or 0; else -1 */
  int64_t n_meas;       /* measurements taken: the steps after the burn-in whose sweep
                           number is a multiple of measure_every (all of them for 0 or 1) */
  double t_submit, t_admit, t_done;
  double tau_tunnel;    /* with PT_TRACK_WALK: mean round trip in passes (NaN if none) */
} pt_result;

/* Creates a job: copies the couplings in, draws the initial spins (one
 * Philox word per site), sets the maps to the identity, computes every
 * energy and zeroes the sweep/exchange/Houdayer counters and the moments.
 * Sec. 2.1 (model, Eqs. (1)-(2)), Sec. 3 (replica layout).
 *   out       receives the handle (unchanged on failure)
 *   samples   >= 1 and < 2^28
 *   replicas  N_T >= 2
 *   L, dim    even L in [4, 64]; dim 2 or 3
 *   couplings host int8 [samples][dim][L^dim], every entry +1 or -1
 *   betas     host double [replicas], finite, > 0, strictly decreasing
 *   seed      Philox key
 * Returns PT_EINVAL for any violated condition, PT_ENOMEM if allocation
 * fails, PT_EDEVICE on a HIP error. */
int pt_init(pt_job **out, int32_t samples, int32_t replicas, int32_t L,
            int32_t dim, const int8_t *couplings, const double *betas,
            uint64_t seed);

/* pt_init with a device spin layout: flags = PT_LAYOUT_INT8 or
 * PT_LAYOUT_PACKED, optionally | PT_TRACK_WALK and/or | PT_TRACK_MODES.
 * Results are bit-identical for both layouts, with or without either. */
int pt_init_ex(pt_job **out, int32_t samples, int32_t replicas, int32_t L,
               int32_t dim, const int8_t *couplings, const double *betas,
               uint64_t seed, uint32_t flags);

/* A job with Gaussian couplings (Sec. 2.1: couplings drawn from a standard
 * normal distribution; the 2D Gaussian workload of Sec. 4.2).  Couplings are
 * host float32 [samples][dim][L^dim], each a multiple of 2^-16 with |J| <= 8
 * (workloads.couplings_gauss draws them so), held internally as the integers
 * n = J 2^16, so every local field and energy is an exact integer number of
 * 2^-16 units.  Other arguments, the initial spins, maps, counters and
 * random-number counters are pt_init_ex's; flags is a layout
 * (PT_LAYOUT_INT8 or PT_LAYOUT_PACKED) with no tracking flags.
 * The steps of such a job differ from the +-J rule only in the acceptance: a
 * Metropolis flip with x = s_i h_i > 0 (energy change 2x units) is accepted
 * iff its Philox word r < 2^32 exp(-beta_k 2x 2^-16), and an exchange with
 * D > 0 units iff r < 2^32 exp(-(beta_k - beta_{k+1}) D 2^-16), both decided
 * exactly (real-number comparisons of the integer r; see pt_gauss_accept_test).
 * pt_sweep, pt_exchange, pt_houdayer, pt_houdayer_multi, pt_measure, pt_mcs
 * (fused, n steps per launch with one workgroup per sample holding all its
 * configurations, when pt_get_plan reports mode 0: single-cluster or no
 * Houdayer moves and a sample that fits one workgroup's LDS; otherwise, and
 * with PT_MCS_PLAIN, the per-step kernels; both bit-identical),
 * pt_mcs_noalloc (the same), pt_get_plan, pt_observables (energies per spin in
 * coupling units), pt_get/set_spins, pt_get_maps, pt_get_counters,
 * pt_set_measure_interval, pt_get_state / pt_set_state and pt_destroy take
 * such jobs; energies and moments are read with pt_get_energies64 and
 * pt_get_moments8; pt_get_energies, pt_get_moments, batches and the server
 * refuse them (PT_EINVAL).  PT_EINVAL also for a coupling off the grid or out of range. */
int pt_init_gauss(pt_job **out, int32_t samples, int32_t replicas, int32_t L,
                  int32_t dim, const float *couplings, const double *betas,
                  uint64_t seed, uint32_t flags);

/* The acceptance decisions of Gaussian jobs for test inputs (host arrays of
 * n words r, inverse-temperature factors b > 0 and energy changes u > 0 in
 * 2^-16 units, u <= 2^52): out[i] = 1 iff r[i] < 2^32 exp(-b[i] u[i] 2^-16),
 * computed on the device by mode 0 the Metropolis path (u < 2^24: float32,
 * then double, then double-double where a tier's error bound leaves the
 * answer open), 1 the exchange path (double, then double-double), 2 the
 * double-double evaluation alone.  Synchronous; allocates its own device
 * buffers.  PT_EINVAL for out-of-range inputs or mode. */
int pt_gauss_accept_test(const uint32_t *r, const double *b, const int64_t *u, int32_t *out,
                         int32_t n, int32_t mode);

/* The double-double decision of pt_gauss_accept_test's mode 2 run on the
 * host: 1 accept, 0 reject, PT_EINVAL for b <= 0 or u out of (0, 2^52]. */
int pt_gauss_accept_host(uint32_t r, double b, int64_t u);

/* n >= 0 Metropolis sweeps (Sec. 2.2) of every configuration: colour 0 of
 * the checkerboard, then colour 1.  A site with x = s_i * sum_j J_ij s_j <= 0
 * always flips; otherwise it flips iff its 32-bit Philox word r satisfies
 * r < floor(2^32 exp(-2 x beta_k)) (clamped to 2^32-1), beta_k being the
 * slot's current temperature.  Energies are updated by 2x per flip.  The word
 * of a site comes from counter (R*ceil(L/8) + (b>>2), 2t + colour, slot,
 * 3<<28 | sample), word b & 3, where R = i / L, b = (i % L) >> 1 and t the
 * job's sweep counter, which advances by n.  PT_EINVAL if n < 0. */
int pt_sweep(pt_job *job, int32_t n);

/* One replica-exchange pass (Sec. 2.2, Eq. (5)).  For each sample and each
 * replica set separately, k = 0 .. N_T-2 ascending: with a, b the slots at
 * beta_k, beta_{k+1} and D = E_b - E_a, the temperatures are swapped iff
 * D <= 0 or r < floor(2^32 exp(-(beta_k - beta_{k+1}) D)), r being word 0 of
 * the Philox counter (k, u, set, 4<<28 | sample), u the exchange counter.
 * In a job created with PT_TRACK_WALK every pass, fused or not, then updates
 * the replica walk (pt_get_walk). */
int pt_exchange(pt_job *job);

/* One Houdayer cluster move (Sec. 2.4, Eq. (10)) per sample and temperature
 * k, on the pair (set 0, set 1) currently at beta_k.  With q_i = s_i^a s_i^b
 * and n the number of q = -1 sites, nothing happens if n = 0; otherwise the
 * seed is the m-th q = -1 site in increasing i, m = floor(r64 n / 2^64) with
 * r64 = w0 | w1 << 32 from Philox counter (k, v, 0, 5<<28 | sample); the
 * cluster is its nearest-neighbour connected component of q = -1 sites, and
 * both replicas are negated on it (equivalently: exchanged there).  E_a
 * changes by delta and E_b by -delta. */
int pt_houdayer(pt_job *job);

/* One multi-cluster Houdayer move per sample and temperature k (the variant
 * Sec. 3 proposes and Sec. 5 names as the remedy for the load imbalance of
 * single clusters): on the pair (set 0, set 1) at beta_k, every
 * nearest-neighbour cluster of q = -1 sites is exchanged, independently of
 * the others, with probability 1/2.  A cluster is named by its lowest site m
 * and exchanged iff bit m mod 128 of Philox counter (m / 128, v, k,
 * 6<<28 | sample) is set, bit j of the 128-bit output being bit j mod 32 of
 * word j / 32; v is the Houdayer pass counter the single-cluster move also
 * advances.  E_a changes by delta, E_b by -delta (E_a + E_b is conserved).
 * PT_EINVAL if L^dim > 32768 (16-bit cluster labels). */
int pt_houdayer_multi(pt_job *job);

/* Accumulates one measurement (Eqs. (3), (4)): per sample and temperature,
 * exact integer sums of E (both replicas), E^2, Q, |Q|, Q^2 and Q^4 (128-bit)
 * with Q = sum_i s_i^a s_i^b over the pair at that temperature. */
int pt_measure(pt_job *job);

/* n Monte Carlo steps (Sec. 2.4): sweep, Houdayer if flags has
 * PT_MCS_HOUDAYER (the multi-cluster variant with PT_MCS_MULTICLUSTER too),
 * exchange, measure if flags has PT_MCS_MEASURE.  The steps
 * run fused, the configurations resident in LDS for the whole launch, with
 * the first plan that fits a workgroup (pt_get_plan): both replica sets of a
 * sample in one workgroup; one set per workgroup (no measurement, no
 * Houdayer); or, without Houdayer, the sample's configurations split over
 * several workgroups that meet once per step.  With no such plan, or with
 * PT_MCS_PLAIN, one launch per step and kernel.  All forms give
 * bit-identical results. */
int pt_mcs(pt_job *job, int32_t n, uint32_t flags);

/* Most work items (samples, or parts of split samples, of one launch) that
 * pt_mcs_noalloc takes. */
#define PT_NOALLOC_MAX_ITEMS 65536

/* pt_mcs that allocates no device memory, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, steps and results as pt_mcs, bit for bit.
 * pt_mcs keeps each job's work list, queue counter and launch state in device
 * memory it allocates on first use; this entry point instead writes them to
 * a static scratch array of the library (about 1 MiB per GPU, held from the
 * first call on that GPU until the process ends) and needs nothing else (the
 * per-step kernels it takes when no fused plan fits, and the fused steps of
 * Gaussian-coupling jobs, use no scratch).  Every
 * call on one GPU shares that GPU's scratch: calls that overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller.
 * PT_EINVAL if one launch would need more than PT_NOALLOC_MAX_ITEMS work
 * items (nothing runs); otherwise errors as pt_mcs. */
int pt_mcs_noalloc(pt_job *job, int32_t n, uint32_t flags);

/* Measurement interval (Sec. 3: measurements are taken at intervals): from
 * now on a step of pt_mcs or pt_batch_run with PT_MCS_MEASURE measures only if
 * its 1-based sweep number (the sweep counter after the step) is a multiple
 * of `every` (>= 1; 1, the default, measures every step).  The rule follows
 * the job's own counter, so results do not depend on how the steps are split
 * into calls.  pt_measure still measures when called.  A job setting, not
 * part of the checkpoint.  PT_EINVAL if every < 1. */
int pt_set_measure_interval(pt_job *job, int32_t every);

/* The plan pt_mcs takes for these flags, int32 [4]: mode (0 both sets per
 * workgroup, 1 the same with Houdayer, 2 one set per workgroup, 3 split
 * sample, -1 per-step kernels), workgroups per sample, configurations per
 * workgroup, and LDS bytes per workgroup (0 for mode -1).  A Gaussian job
 * reports mode 0 for its fused steps (with or without Houdayer moves) and -1
 * for the per-step kernels.  Host only. */
int pt_get_plan(pt_job *job, uint32_t flags, int32_t *out4);

/* The same report for a job of this shape before it exists (host only, no
 * device call): a plan depends on dim, L and replicas, not on samples, and on
 * whether PT_TRACK_WALK (also accepted in flags here) keeps the walk. */
int pt_plan_query(int32_t dim, int32_t L, int32_t replicas, uint32_t flags, int32_t *out4);

/* Upper bound of the device bytes pt_init_ex allocates for this shape
 * (including the split-sample scratch when the plan needs it); layout as
 * pt_init_ex's flags.  The request server admits by this figure.  Host
 * only; PT_EINVAL as pt_init_ex. */
int pt_job_bytes(int32_t samples, int32_t replicas, int32_t L, int32_t dim, uint32_t layout,
                 const double *betas, uint64_t *out);

/* Observables from the accumulated moments, in double precision: the energy
 * per spin of Eq. (3) and the overlap of Eq. (4) with its moments, thermal
 * averages over the measurements and disorder averages over the samples.
 *   per_sample [samples][replicas][5]: <e>, <q>, <|q|>, <q^2>, <q^4>
 *   disorder   [replicas][6]: the same averaged over samples (integer
 *              numerators summed first) and the Binder parameter
 *              g = (3 - [<q^4>]/[<q^2>]^2) / 2
 *   n_meas     number of measurements
 * Any output pointer may be NULL.  With no measurement the averages are NaN. */
int pt_observables(pt_job *job, double *per_sample, double *disorder,
                   int64_t *n_meas);

/* Releases the job and its device memory (synchronises its stream). */
int pt_destroy(pt_job *job);

/* ---- state access (synchronous) ---------------------------------------- */
/* int8 [samples][2*replicas][L^dim] */
int pt_get_spins(pt_job *job, int8_t *out);
/* Replaces every spin (entries must be +1/-1) and recomputes every energy. */
int pt_set_spins(pt_job *job, const int8_t *in);
/* Moves the job's spins to another layout (PT_LAYOUT_INT8 or
 * PT_LAYOUT_PACKED, Sec. 2.2): a new spin buffer is allocated through the
 * job's allocator, filled by a conversion kernel and the old one freed, so the
 * configuration, energies, counters and random-number streams are unchanged and
 * later steps give the same results as without the move.  Waits for all work
 * queued on the device first (a batch launch on another stream may still read
 * the spins); batches holding the job rebuild their work list and graph on
 * their next run.  A checkpoint from pt_get_state restores only into the
 * layout it was taken from.  PT_OK at once if the job already has the layout;
 * PT_EINVAL for another value, PT_ENOMEM if the allocation fails (the job
 * keeps its layout). */
int pt_set_layout(pt_job *job, uint32_t layout);
/* The job's spin layout now (PT_LAYOUT_INT8 or PT_LAYOUT_PACKED). */
int pt_get_layout(pt_job *job, uint32_t *out);
/* int32 [samples][2*replicas] */
int pt_get_energies(pt_job *job, int32_t *out);
/* int32 [samples][2][replicas] each; either may be NULL */
int pt_get_maps(pt_job *job, int32_t *slot_of_temp, int32_t *temp_of_slot);
/* uint64 [4]: sweeps t, exchange passes u, Houdayer passes v, measurements */
int pt_get_counters(pt_job *job, uint64_t *out);
/* int64 [samples][replicas][7]: sum E, sum E^2, sum Q, sum |Q|, sum Q^2,
 * sum Q^4 low 64 bits, sum Q^4 high 64 bits */
int pt_get_moments(pt_job *job, int64_t *out);
/* Energies as int64 [samples][2*replicas]: in 2^-16 units for a Gaussian
 * job, the +-J energies widened otherwise (Eq. (1)). */
int pt_get_energies64(pt_job *job, int64_t *out);
/* int64 [samples][replicas][8]: sum E, sum E^2 (low 64 bits), sum Q, sum |Q|,
 * sum Q^2, sum Q^4 (low, high 64 bits), sum E^2 (high 64 bits; 0 for +-J
 * jobs, whose E^2 sums fit 64 bits).  E in 2^-16 units for Gaussian jobs.
 * Eqs. (3)-(4). */
int pt_get_moments8(pt_job *job, int64_t *out);
/* Replica walk in temperature space and round-trip times (Sec. 2.3: the
 * round-trip or tunnelling time is the expected number of Monte Carlo steps a
 * configuration needs from the lowest temperature to the highest and back).
 * Each slot is looked at after every exchange pass m = u (the exchange
 * counter after the pass, from 1).  Its label is 0 until it first sits at the
 * lowest temperature, then 1 ("going up"), and 2 ("going down") once it
 * reaches the highest temperature while labelled 1.  A slot labelled 2 back
 * at the lowest temperature ends a round trip of m - begin passes and begins
 * the next (label 1, begin = m).  Houdayer moves leave slots where they are.
 *   label  int32  [samples][2*replicas]  (slot r of set c at index c*replicas+r)
 *   begin  uint32 [samples][2*replicas]  pass at which the current trip began
 *   trips  uint64 [samples][32][3]       trips ending in passes [2^b, 2^(b+1)),
 *          both replica sets: count, sum of lengths, sum of squared lengths
 * Any output may be NULL.  Synchronous.  The pass clock is the 32-bit
 * exchange counter.  PT_EINVAL for a job created without PT_TRACK_WALK. */
int pt_get_walk(pt_job *job, int32_t *label, uint32_t *begin, uint64_t *trips);

/* Round-trip time estimates from `rows` rows of round-trip bins
 * ([rows][32][3] as pt_get_walk writes them; every row is pooled), after
 * `passes` exchange passes.  Host-only, no job needed.  Outputs (any may be
 * NULL):
 *   tau_b [32]  mean trip length of bin b (NaN if empty)
 *   err_b [32]  its standard error sqrt((C Q - D^2) / (C^2 (C - 1))) from the
 *               bin's count C, sum D and sum of squares Q (NaN if C < 2)
 *   tau         mean length over every trip (NaN if none)
 *   equilibrated  1 iff the last three complete bins (bin b is complete once
 *               passes >= 2^(b+1) - 1) each hold two or more trips and every
 *               two of them differ by at most 2 sqrt(err_i^2 + err_j^2): the
 *               logarithmic-binning check of Sec. 2.3.
 * PT_EINVAL if trips is NULL or rows < 1. */
int pt_tunnel_summary(const uint64_t *trips, int32_t rows, uint64_t passes,
                      double *tau_b, double *err_b, double *tau,
                      int32_t *equilibrated);

/* Two-replica modes for the spin-glass susceptibility and correlation length
 * (Sec. 3 names them as two-replica measurements; the usual definitions).
 * Per measurement and temperature, with q_i = s_i^a s_i^b the overlap of the
 * set-0 and set-1 replicas at that temperature and P_mu(x) the sum of q_i
 * over the sites whose coordinate along axis mu is x, the job adds
 *   A(delta) = sum over axes mu of sum_x P_mu(x) P_mu((x + delta) mod L),
 * delta = 0 .. L/2 (A(L - delta) = A(delta)): exact integers, from which
 * sum_mu |sum_i q_i exp(2 pi i n x_mu / L)|^2 = sum_{delta<L} cos(2 pi n
 * delta / L) A(delta).
 *   out int64 [samples][replicas][L/2 + 1]
 * Synchronous.  PT_EINVAL for a job created without PT_TRACK_MODES. */
int pt_get_modes(pt_job *job, int64_t *out);

/* Run diagnostics of a job created with PT_TRACK_STATS (Sec. 2.3 discusses
 * the exchange acceptance rates, Sec. 3 the spread of cluster sizes that
 * unbalances the cluster kernel): int64 out [samples][replicas][24], counted
 * since creation (kept by pt_get_state / pt_set_state) --
 *   [0]      accepted Metropolis flips of the configurations at temperature
 *            k, both replica sets (divide by 2 N and the sweeps for a rate)
 *   [1]      accepted exchanges of the pair (k, k+1), both replica sets
 *   [2]      Houdayer passes at k that exchanged at least one site
 *   [3]      the sites those passes exchanged
 *   [4 + b]  passes that exchanged between 2^b and 2^(b+1) - 1 sites
 * Synchronises the stream.  PT_EINVAL for a job without diagnostics. */
int pt_get_stats(pt_job *job, int64_t *out);

/* Per temperature k (int32 index 0 = coldest), disorder-averaged from integer
 * sums over samples: chi0[k] = chi_SG(0) = [sum Q^2] / (S n_meas N) (the
 * overlap moment, Q = sum_i q_i), chik[k] = chi_SG(k_min) = [sum_delta
 * cos(2 pi delta / L) A(delta)] / (d S n_meas N) with k_min = 2 pi / L along
 * each axis (averaged over the d axes), and xi[k] = sqrt(chi0/chik - 1) /
 * (2 sin(pi / L)), the second-moment correlation length (NaN if chik <= 0 or
 * chi0 < chik).  Outputs double [replicas]; any may be NULL.  The cosine is
 * taken exactly where it is 0 or +-1.  PT_EINVAL as pt_get_modes. */
int pt_correlation_length(pt_job *job, double *chi0, double *chik, double *xi);

/* Checkpoint: the whole dynamic state (spins, energies -- 64-bit for
 * Gaussian jobs --, maps, counters, moments, and the replica walk, modes and
 * run diagnostics if kept).  With buf == NULL, *len receives the size.
 * Otherwise *len must hold at least that size.  pt_set_state restores a
 * state taken from a job of identical shape, layout, coupling kind and kept
 * extras; continuing is bit-identical to never stopping. */
int pt_get_state(pt_job *job, void *buf, size_t *len);
int pt_set_state(pt_job *job, const void *buf, size_t len);

/* ---- batched form ---------------------------------------------------------- */
/* Groups n >= 1 distinct jobs of the same dim (any L, replicas, samples,
 * layout) so that pt_batch_run advances all of them in one persistent launch.
 * The batch borrows the handles (they must outlive it) and uses the stream of
 * jobs[0] unless pt_batch_set_stream says otherwise.  Each job's results are
 * bit-identical to running it alone with pt_mcs: every random number is keyed
 * by the job's own seed and sample index. */
int pt_batch_create(pt_job *const *jobs, int32_t n, pt_batch **out);
int pt_batch_set_stream(pt_batch *b, void *hip_stream);

/* mcs Monte Carlo steps of every job (Sec. 2.4), flags as pt_mcs
 * (PT_MCS_HOUDAYER, PT_MCS_MEASURE) plus PT_BATCH_GRAPH: the launch
 * (queue reset, persistent kernel, counter advance) is captured once as a
 * hipGraph per (mcs, flags, configuration) and replayed; the device counters
 * make every replay continue the random-number streams.  Workgroups take
 * (job, sample, replica sets) items from a device queue, largest first by
 * default; each job runs the plan pt_get_plan reports for these flags.  The
 * parts of a split sample are queued first and consecutively, and launches
 * holding split samples are ordered across the process's streams (their
 * workgroups wait for one another once per step).  A job with no plan for
 * these flags (Houdayer moves on a sample whose two sets do not fit one
 * workgroup) runs its steps through the per-step kernels on its own stream
 * (pt_set_stream), ordered by events after the batch stream's earlier work and
 * before its later work, and outside any captured graph. */
int pt_batch_run(pt_batch *b, int32_t mcs, uint32_t flags);

/* Autotuner: after one untimed trial, times trial_mcs steps of each launch
 * configuration (threads per workgroup 1024/768/512/256, one or two replica
 * sets per item, largest-first or job order) twice on the batch itself,
 * restoring every job's state after each trial, and keeps the configuration
 * whose faster run was fastest.  With PT_TUNE_LAYOUT in flags the spin
 * layout is a further axis: every configuration is timed with all jobs in the
 * int8 layout and again in the packed one (pt_set_layout), and the jobs are
 * left in the winning layout.  cache_path (may be NULL) is a JSON-lines file
 * keyed by the batch shape, the flags and the jobs' layouts at the call; a hit
 * skips the trials (and applies the cached layout). */
int pt_batch_tune(pt_batch *b, int32_t trial_mcs, uint32_t flags, const char *cache_path);
/* cfg3 = {threads per workgroup, replica sets per item, order}.  threads 0
 * (the default) picks per launch one of 1024/768/512/256 threads (a multiple
 * of four wavefronts, so that a CU's four SIMDs carry equal shares): with no
 * more items than CUs the largest; otherwise the one with the most wavefronts
 * resident per CU (the runtime's occupancy for the launch's LDS plan and
 * kernel), then two or more workgroups per CU, then the larger size;
 * get_config then reports the size last used. */
int pt_batch_get_config(pt_batch *b, int32_t *cfg3);
/* threads: 0 (automatic) or a multiple of 64 up to 1024; sets: 1 or 2
 * replica sets per item when a sample's two sets may run apart; order: 0
 * largest items first, 1 job order.  PT_EINVAL otherwise. */
int pt_batch_set_config(pt_batch *b, int32_t threads, int32_t sets, int32_t order);
/* out3 = {workgroups, threads per workgroup, workgroups resident per CU} of
 * the grid the batch last built (the runtime's occupancy for the launch's
 * kernel, LDS plan and workgroup size); zeros before the first run. */
int pt_batch_launch_shape(pt_batch *b, int32_t *out3);
int pt_batch_destroy(pt_batch *b);

/* ---- served form ----------------------------------------------------------- */
/* Starts a request server on the current device with its own worker thread
 * and streams.  Requests are admitted in arrival order while the device bytes
 * of the admitted jobs stay within hbm_budget (a request that alone exceeds
 * it fails with PT_ENOMEM); admitted jobs stay resident and advance together,
 * steps_per_round Monte Carlo steps per round in one persistent batch launch
 * (continuous batching: admissions and completions happen between rounds).
 * Each job measures every step after its burn-in; on completion its
 * disorder-averaged observables are kept for pt_server_poll and its memory is
 * released.  Job set-up and read-out overlap the running round on a stream of
 * their own; device memory comes from a stream-ordered pool owned by the
 * server (not the allocator hooks) and returns to it when a job finishes.
 * Admitted requests (their bytes counted against the budget from then on)
 * get their jobs created oldest first while the round in flight still runs,
 * at least one per round (an idle server starts its first round after 5 ms of
 * set-up); the others join later rounds. */
int pt_server_start(size_t hbm_budget, int32_t steps_per_round, pt_server **out);
/* A round gives each job up to steps_per_round steps; when every work item of
 * the round has a workgroup of its own, jobs whose items are smaller than the
 * largest get proportionally more, so that all items take about as long. */
/* Copies the request and queues it; *ticket identifies it.  PT_EINVAL for
 * arguments pt_init would reject (or burn_in outside [0, sweeps]). */
int pt_server_submit(pt_server *s, const pt_request *req, uint64_t *ticket);
/* Returns 1 while the request is queued or running; PT_OK once it finished,
 * filling *out and (if not NULL) disorder [replicas][6] as pt_observables,
 * after which the ticket is forgotten; PT_EINVAL for an unknown ticket.  A
 * request's layout may carry PT_TRACK_WALK (results then include the
 * round-trip time) and PT_TRACK_MODES (see pt_server_poll_ex). */
int pt_server_poll(pt_server *s, uint64_t ticket, pt_result *out, double *disorder);
/* pt_server_poll that also fills (if not NULL) correlation [replicas][3]:
 * chi_SG(0), chi_SG(k_min) and xi as pt_correlation_length, for a request
 * whose layout carries PT_TRACK_MODES (NaN otherwise). */
int pt_server_poll_ex(pt_server *s, uint64_t ticket, pt_result *out, double *disorder,
                      double *correlation);
/* out[11] = {attempted flips completed, busy seconds, rounds, admitted,
 *            completed, peak admitted bytes, peak concurrent jobs, uptime s,
 *            queue depth (requests waiting for admission or for their
 *            job to be created), jobs in the current round, cancelled
 *            requests} */
int pt_server_stats(pt_server *s, double *out);
/* Cancels a request, leaving every other request's work and result as if it
 * had never been submitted (each job's result depends only on its own
 * request).  A queued request is dropped at once; an admitted one ends at
 * the next round boundary (unless it completes its steps first, in which case its
 * normal result stands) and its device memory returns to the budget.  The
 * cancelled request's pt_server_poll result has status PT_ECANCELED and no
 * observables.  Returns PT_OK when the cancellation is recorded, 1 if the
 * request has already finished (its result waits to be polled), PT_EINVAL
 * for an unknown ticket or one whose result was already collected.
 * Operational control of the served form: not a step of the method. */
int pt_server_cancel(pt_server *s, uint64_t ticket);
/* Finishes every queued and running request, then stops the server. */
int pt_server_stop(pt_server *s);

/* ---- plumbing ------------------------------------------------------------ */
/* Makes the job enqueue on a HIP stream (hipStream_t; NULL = null stream). */
int pt_set_stream(pt_job *job, void *hip_stream);
/* Process-wide device allocator hooks used by later pt_init calls; pass NULLs
 * to restore hipMalloc/hipFree.  alloc(bytes, ctx) returns device memory or
 * NULL; free_(ptr, ctx) releases it. */
int pt_set_allocator(void *(*alloc)(size_t, void *),
                     void (*free_)(void *, void *), void *ctx);
/* Thread-local message for the last failure on this thread ("" if none). */
const char *pt_last_error(void);
/* Library version string. */
const char *pt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PT_SPINGLASS_H */
