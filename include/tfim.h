/*
 * tfim.h - C ABI of libtfim: Metropolis + parallel tempering sampling of the
 * classical Trotter-Suzuki lattice of the 2D transverse-field Ising spin
 * glass, multispin-coded (64 disorder samples per uint64), on one MI355X.
 *
 * Paper: Bernaschi, Gonzalez-Adalid Pemartin, Martin-Mayor, Parisi,
 * "The Quantum Transition of the Two-Dimensional Ising Spin Glass"
 * (arXiv:2310.07486).  A problem is what the paper's Methods define it by:
 * an instance of +-1 couplings ("Model and simulations"), lattice sizes L and
 * Ltau and a coupling k or a ladder of k ("The Trotter-Suzuki formula":
 * p(S) = exp(-k E(S))/Z, periodic in tau), real replicas and tempering over
 * k ("Simulation details", Table I), and the one-time observables
 * ("One-time observables": M, M-hat, chi^(2), F^(2), xi^(2)).
 *
 * Conventions used by every call:
 *   - Site (x, y, tau), xy = x + L*y, lin = xy + L*L*tau.  Colour
 *     (x + y + tau) mod 2; L and Ltau must be even.
 *   - Spin bit 1 <=> S = -1; coupling bit 1 <=> J = -1.  Bit b of sample
 *     word j is sample 64*j + b of the shape.
 *   - Canonical host layouts: spins u64[r][w][j][tau][y][x] (replica r,
 *     walker w), couplings u64[j][d][y][x] (d = 0: bond (x,y)-(x+1,y);
 *     d = 1: bond (x,y)-(x,y+1)), k labels u8[r][s][w] (k-index of walker w
 *     of replica r, sample s), energies u32[r][s][w] = number of
 *     unsatisfied bonds U (E = 2U - 3N, N = L*L*Ltau).
 *   - Random numbers: Philox4x32-10, key = seed, counter layout fixed by
 *     the library (a shape's streams depend on seed, stream_id, the global
 *     word index word_offset + j, the sweep counter t and the tempering
 *     counter m), so a shape reproduces bit-for-bit whether it runs alone
 *     or batched, whole or split into word ranges.
 *
 * Ownership: the caller allocates ONE device arena of the size reported by
 * tfim_plan_sizes and keeps it alive while the plan is bound; the library
 * never allocates or frees device memory of its own (it creates HIP graph,
 * stream and event objects only).  The plan (an opaque host object) owns
 * its copies of the shapes, the threshold tables, the tuner choice and the
 * graph cache.
 *
 * Errors: every call returns a tfim_status and never throws.  Argument
 * errors return before anything is enqueued and leave the state unchanged.
 * A device error poisons the plan for the rest of its life: every later call
 * that uses it (tfim_bind included) returns TFIM_ESTATE; a saved state is
 * resumed on a new plan with tfim_set_state.  tfim_last_error_detail()
 * describes the last failure of this thread.
 *
 * Failure injection (for tests of the error path; nothing reaches the GPU):
 * when the environment variable TFIM_FAIL_AFTER = n >= 1 is set at
 * tfim_plan_create, the n-th call of that plan that would enqueue device work
 * (init, sweep, pt_swap, set_state and the measurement calls) enqueues
 * nothing and fails as a device error does: it returns TFIM_EDEVICE and
 * poisons the plan.
 *
 * Concurrency: calls that enqueue work (init, sweep, pt_swap) are
 * asynchronous on the bound stream; calls that return data to the host
 * (measure, export, get_state) synchronise that stream.  A plan is not
 * thread-safe; distinct plans are independent.
 */
#ifndef TFIM_H
#define TFIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tfim_status;
#define TFIM_OK 0
#define TFIM_EINVAL (-1)       /* bad argument or shape */
#define TFIM_EUNSUPPORTED (-2) /* valid request this build does not provide */
#define TFIM_EDEVICE (-3)      /* HIP runtime or kernel failure */
#define TFIM_ESTATE (-4)       /* wrong call order, unbound or poisoned plan */
#define TFIM_EOVERFLOW (-5)    /* sweep or tempering counter would pass 2^32 */

/* Boundary condition along tau (Methods, "The Trotter-Suzuki formula"). */
#define TFIM_BC_PERIODIC 0u
#define TFIM_BC_ANTIPERIODIC 1u /* the temporal bond tau = Ltau-1 -- 0 has the sign -1 */

/* One problem shape: n_words*64 disorder samples of an L x L x Ltau lattice,
 * n_replicas independent real replicas, each with n_k walkers that share the
 * ladder k[0] < k[1] < ... < k[n_k-1] through tempering. */
typedef struct {
    uint32_t L;           /* even, 2..24 (one thread per spatial column) */
    uint32_t Ltau;        /* even, 4..65536; multispin form: a multiple of 8
                             (else TFIM_EUNSUPPORTED) */
    uint32_t n_words;     /* >= 1; samples = 64*n_words (plain form: samples) */
    uint32_t word_offset; /* global index of word 0 (the words used end below 2^20) */
    uint32_t n_replicas;  /* 1..64 */
    uint32_t n_k;         /* 1..255 */
    const double *k;      /* n_k couplings, > 0, strictly increasing; copied */
    uint32_t bc_tau;      /* TFIM_BC_PERIODIC or TFIM_BC_ANTIPERIODIC (Methods,
                             "The Trotter-Suzuki formula": antiperiodic along tau only) */
    uint32_t pt_every;    /* tempering after every pt_every-th sweep; 0 = never */
    uint32_t stream_id;   /* 0..255, distinct within a plan */
} tfim_shape;

typedef struct tfim_plan tfim_plan;

/* Representation of a plan's spins (Methods, "The Trotter-Suzuki formula":
 * classical spins S = +-1; "Simulation details": multispin coding).
 * TFIM_FORM_MULTISPIN: 64 disorder samples per uint64 word, as above.
 * TFIM_FORM_PLAIN_I8: one signed byte (+1 / -1) per spin and coupling, one
 *   sample per configuration; tfim_shape.n_words then counts SAMPLES, and
 *   sample s draws every random number of word word_offset + s/64, lane
 *   s % 64, so its trajectory is exactly that lane's in a multispin run.
 *   Canonical layouts: spins int8 [r][w][s][tau][y][x], couplings int8
 *   [s][d][y][x]; k labels and energies as above.  Ltau needs only be even.
 *   Runs the per-shape schedule; tfim_measure (records in the plain
 *   per-sample mode, buckets, energies) and tfim_measure_range (mode 1);
 *   batched/concurrent schedules, the autotuner, three-replica and two-time
 *   records and the debug dump return TFIM_EUNSUPPORTED. */
#define TFIM_FORM_MULTISPIN 0u
#define TFIM_FORM_PLAIN_I8 1u

/* Device arena layout, in bytes (offsets are 256-byte aligned). */
typedef struct {
    size_t total;     /* size of the arena to pass to tfim_bind */
    size_t spins;     /* all shapes' spin words */
    size_t couplings; /* all shapes' coupling words */
    size_t labels;    /* k labels, walker-of-k maps, energies, lane masks */
    size_t tables;    /* threshold tables and counters */
    size_t measure;   /* measurement records */
} tfim_sizes;

/* Create a plan for n_shapes shapes sampled together with one seed, in the
 * given form (TFIM_FORM_MULTISPIN or TFIM_FORM_PLAIN_I8).
 * TFIM_EINVAL: unknown form, odd or out-of-range L/Ltau, n_words = 0, bad
 * ladder, repeated stream_id, unknown bc_tau. */
tfim_status tfim_plan_create(const tfim_shape *shapes, uint32_t n_shapes, uint64_t seed,
                             uint32_t form, tfim_plan **plan_out);
void tfim_plan_destroy(tfim_plan *plan);

/* Sizes of the device arena (host-only). */
tfim_status tfim_plan_sizes(const tfim_plan *plan, tfim_sizes *sizes_out);

/* Bind the caller's device arena (at least sizes.total bytes, 256-byte
 * aligned) and HIP stream (NULL = default stream) to the plan. */
tfim_status tfim_bind(tfim_plan *plan, void *device_arena, size_t arena_bytes,
                      void *hip_stream);

/* Instance (Methods, "Model and simulations": J = +-1 with probability 1/2).
 * J_host == NULL: draw the couplings on the device from the seed;
 * otherwise copy the canonical host array: n_words*2*L*L uint64 words
 * (multispin) or samples*2*L*L int8 values +-1 (plain; anything else is
 * TFIM_EINVAL). */
tfim_status tfim_init_couplings(tfim_plan *plan, uint32_t shape, const void *J_host);

/* Initial state: hot start (i.i.d. spins) when S_host == NULL, otherwise a
 * canonical host array of n_replicas*n_k*n_words*L*L*Ltau uint64 words
 * (multispin) or n_replicas*n_k*samples*L*L*Ltau int8 values +-1 (plain).
 * Resets k labels to the identity, recounts energies and sets t = m = 0 for
 * the whole plan.  Couplings must be initialised first (else TFIM_ESTATE). */
tfim_status tfim_init_spins(tfim_plan *plan, uint32_t shape, const void *S_host);

/* n sweeps of every shape (Methods, "Simulation details"; Table I): a
 * checkerboard Metropolis sweep (colour 0 then colour 1), the energy
 * recount, and a tempering step after sweep t when pt_every > 0 and
 * (t+1) % pt_every == 0.  Asynchronous.  TFIM_EOVERFLOW, before anything is
 * enqueued, if t + n would pass 2^32 - 1. */
tfim_status tfim_sweep(tfim_plan *plan, uint64_t n);

/* One explicit tempering step of every shape (uses and advances m;
 * TFIM_EOVERFLOW if m would pass 2^32 - 1). */
tfim_status tfim_pt_swap(tfim_plan *plan);

/* Measurement (Methods, "One-time observables"), synchronous.
 * what = TFIM_MEASURE_RECORDS: int64 records [n_k][samples][pairs][2L+3],
 *   pairs = replica pairs a<b in lexicographic order, each record
 *   [D_x[0..L-1], D_y[0..L-1], trQ, sum Q^2, sum Q^4] where, for the
 *   configurations S^a, S^b (L^2 x Ltau, +-1) at k-index i,
 *   G = S S^T, D_x[d] = sum_{(x1-y1) mod L = d} G^a_xy G^b_xy,
 *   Q = S^aT S^b.  Needs 2..6 replicas and L <= 32 (else TFIM_EUNSUPPORTED;
 *   the paper's runs use 6).
 * what = TFIM_MEASURE_BUCKETS: int64 A[n_k][2][L] = records' D_x and D_y
 *   summed over samples and pairs.
 * what = TFIM_MEASURE_ENERGY: u32 U[r][s][i] of the walker at k-index i.
 * host_bytes must be at least the size of the result. */
#define TFIM_MEASURE_RECORDS 1u
#define TFIM_MEASURE_BUCKETS 2u
#define TFIM_MEASURE_ENERGY 3u
tfim_status tfim_measure(tfim_plan *plan, uint32_t shape, uint32_t what, void *host_out,
                         size_t host_bytes);

/* Measurement of a range of configurations cfg = i*samples + s,
 * cfg0 .. cfg0+ncfg-1, into int64 records [ncfg][pairs][2L+3] (layout as
 * TFIM_MEASURE_RECORDS).  mode 0: batched int8-MFMA kernels (default);
 * mode 1: plain per-sample form (one launch per configuration, one matrix
 * element per thread, int32 multiply-accumulate, no MFMA).  flags:
 * TFIM_MEASURE_REUSE_LAYOUT skips the bit transposition (valid only if the
 * state did not change since the last measurement of this shape).
 * out == NULL: enqueue only (asynchronous, for timing); otherwise the call
 * synchronises and copies the records.  ncfg = 0 measures nothing (the bit
 * layout is still refreshed unless TFIM_MEASURE_REUSE_LAYOUT); a range
 * past the last configuration is TFIM_EINVAL. */
#define TFIM_MEASURE_REUSE_LAYOUT 1u
tfim_status tfim_measure_range(tfim_plan *plan, uint32_t shape, uint32_t mode, uint32_t cfg0,
                               uint32_t ncfg, uint32_t flags, int64_t *out, size_t out_bytes);

/* Measurement form used by tfim_measure (0 batched MFMA, 1 plain). */
tfim_status tfim_set_measure_mode(tfim_plan *plan, uint32_t mode);

/* Debug dump of the integer matrices of one configuration pair:
 * G^a (L^2 x L^2, int32), G^b, and Q^{ab} (Ltau x Ltau, int32) for sample s
 * at k-index i, replicas a < b.  Synchronous. */
tfim_status tfim_dump_gram(tfim_plan *plan, uint32_t shape, uint32_t i, uint32_t s,
                           uint32_t a, uint32_t b, int32_t *Ga, int32_t *Gb, int32_t *Q);

/* Second-moment correlation length (Methods, "One-time observables"):
 * for each k-index, chi = sum_d A[d], F = sum_d A[d] cos(2 pi d/L),
 * xi = sqrt(chi/F - 1) / (2 sin(pi/L)); +inf if F <= 0, NaN if chi/F < 1.
 * A is [n_k][L] int64 (e.g. the D_x half of the buckets).  Host-only. */
tfim_status tfim_xi2(const int64_t *A, uint32_t L, uint32_t n_k, double *xi_out);

/* Three-replica records (Methods, "One-time observables": chi^(r) and F^(r)
 * with r = 3; replica estimators of "Simulation details").  For
 * configuration cfg = i*samples + s and each replica triple a < b < c
 * (lexicographic; n_triples = R(R-1)(R-2)/6), with G^r = S^r S^rT:
 *   T_x[d] = sum over the carrier e in {a,b,c}, f < g the other two, of
 *            sum_{(x1-y1) mod L = d} G^e_xy (G^f G^g)_yx
 * and T_y[d] likewise with x2 - y2.  sum_d T_x[d] = 3 Tr[G^a G^b G^c] ~ Tr[M^3]
 * and sum_d T_x[d] cos(2 pi d/L) ~ Tr[M-hat M^2] (phase on the carrier,
 * averaged over the three choices).  Records are int64
 * [ncfg][n_triples][2L] = [T_x[0..L-1], T_y[0..L-1]], exact.
 * Needs 3 to 6 replicas, L <= 32, L^2 (Ltau/2)^2 < 2^31 and
 * 3 L^6 Ltau^3 < 2^63 (else TFIM_EUNSUPPORTED).
 * tfim_triples_workspace: bytes of device workspace for ncfg configurations
 *   (records, then int8 planes of G/2 for every replica; about
 *   2 R (64 ceil(L/8)^2)^2 bytes per configuration).  Host-only.
 * tfim_measure_triples: configurations cfg0 .. cfg0+ncfg-1; ws is caller-owned
 *   device memory (256-byte aligned, at least the workspace size), used as
 *   scratch and holding the records at its start afterwards.  flags as for
 *   tfim_measure_range.  out == NULL: enqueue only (asynchronous); otherwise
 *   the call synchronises and copies the records to out.  ncfg = 0 launches
 *   nothing and returns TFIM_OK (the range is still checked). */
tfim_status tfim_triples_workspace(const tfim_plan *plan, uint32_t shape, uint32_t ncfg,
                                   size_t *bytes_out);
tfim_status tfim_measure_triples(tfim_plan *plan, uint32_t shape, uint32_t cfg0, uint32_t ncfg,
                                 uint32_t flags, void *workspace, size_t workspace_bytes,
                                 int64_t *out, size_t out_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * records of tfim_measure_triples with no workspace argument.  The int8 G/2
 * digit planes live in a device array that the library holds on every GPU
 * it runs on until the process ends (64 MiB; about 2 R (64 ceil(L/8)^2)^2
 * bytes per configuration, so at L = 24 at most 16 configurations with six
 * replicas or 24 with four per call: more is TFIM_EINVAL, with the limit in
 * the detail).  rec_dev: caller-owned device memory (8-byte aligned) of at
 * least ncfg * n_triples * 2L int64, written with the records of
 * configurations cfg0 .. cfg0+ncfg-1 (layout as tfim_measure_triples).
 * flags as for tfim_measure_range.  Enqueues on the plan's stream and
 * returns (asynchronous); allocates nothing and records no memset.  Every
 * call on one GPU shares that GPU's array and leaves it holding its planes:
 * calls that overlap on one GPU (several streams or host threads) race.
 * ncfg = 0 launches nothing and returns TFIM_OK. */
tfim_status tfim_measure_triples_noalloc(tfim_plan *plan, uint32_t shape, uint32_t cfg0,
                                         uint32_t ncfg, uint32_t flags, int64_t *rec_dev,
                                         size_t rec_bytes);

/* Two-time records (Methods, "Two-times observables"): for configuration
 * cfg = i*samples + s, with the time Gram H^r = S^rT S^r of each replica
 * (Ltau x Ltau, H_t1t2 = sum_x S_x,t1 S_x,t2),
 *   c[d]  = sum_r sum_t1 H^r_t1,(t1+d) mod Ltau
 *   q2[d] = sum_r sum_t1 (H^r_t1,(t1+d) mod Ltau)^2,   d = 0..Ltau-1,
 * as int64 [ncfg][2][Ltau] = [c[0..Ltau-1], q2[0..Ltau-1]], exact.
 * C(tau) = c[tau] / (R L^2 Ltau) and Q2(tau) = q2[tau] / (R L^4 Ltau)
 * (C(0) = Q2(0) = 1).  With bc_tau = TFIM_BC_ANTIPERIODIC the configuration
 * continues past Ltau with the opposite sign, so the terms of c with
 * t1 + d >= Ltau enter with the sign -1 (c[Ltau - d] = -c[d]).  Needs 1..6 replicas, L <= 32, Ltau <= 4096 (else
 * TFIM_EUNSUPPORTED).  ws: caller-owned device memory, 256-byte aligned, at
 * least ncfg*2*Ltau*8 bytes, holding the records afterwards.  flags as for
 * tfim_measure_range.  out == NULL: enqueue only (asynchronous); otherwise
 * the call synchronises and copies the records to out.  ncfg = 0 launches
 * nothing and returns TFIM_OK (the range is still checked). */
tfim_status tfim_measure_time(tfim_plan *plan, uint32_t shape, uint32_t cfg0, uint32_t ncfg,
                              uint32_t flags, void *workspace, size_t workspace_bytes,
                              int64_t *out, size_t out_bytes);

/* xi^(3) per k-index (Methods, "One-time observables") from three-replica
 * records rec[n_k][n_per_k][2L] (n_per_k = samples x triples x measurements):
 * A[d] = sum of T_x[d] (direction 0), T_y[d] (1) or both (2), summed exactly;
 * chi = sum_d A[d], F = sum_d A[d] cos(2 pi d/L), xi = sqrt(chi/F - 1) /
 * (2 sin(pi/L)); +inf if F <= 0, NaN if chi/F < 1.  Host-only. */
tfim_status tfim_xi3(const int64_t *rec, uint32_t L, uint32_t n_k, uint32_t n_per_k,
                     uint32_t direction, double *xi_out);

/* Binder ratio B = Q_4 / Q_2^2 per k-index (Methods, "One-time
 * observables") from pair records rec[n_k][n_per_k][2L+3] (the layout of
 * TFIM_MEASURE_RECORDS; n_per_k = samples x pairs x measurements).  With the
 * tau average of each replica, Q_2 ~ sum Q^2 / Ltau^2 and Q_4 ~ sum Q^4 /
 * Ltau^2 for the overlap Q = S^aT S^b, so
 * B = Ltau^2 n_per_k (sum Q^4) / (sum Q^2)^2 over the k-index's records
 * (exact integer sums; NaN if sum Q^2 = 0).  Host-only. */
tfim_status tfim_binder(const int64_t *rec, uint32_t L, uint32_t Ltau, uint32_t n_k,
                        uint32_t n_per_k, double *B_out);

/* Transfer matrix of one plane (Methods, "The Trotter-Suzuki formula":
 * Z = Tr T^Ltau, the antiperiodic boundary as Tr P T^Ltau with the global
 * flip P; "Simulation details": exact diagonalisation in parity sectors).
 * For one sample's couplings Jx, Jy (host int8, +-1, L*L each, the canonical
 * coupling layout of a lane) and 2 <= L <= 5 (else TFIM_EUNSUPPORTED):
 *   T[s,s'] = exp(k/2 E0(s)) exp(k sum_x s_x s'_x) exp(k/2 E0(s')),
 *   E0(s) = sum over spatial bonds (each once) of J_b s_x s_y,
 * on 2^(L^2) states, bit x of the index set when s_x = -1.  T equals the
 * paper's exp(-k/2 H0) exp(-k H1) exp(-k/2 H0) up to a constant factor.
 * tfim_tm_apply: w = T v for device vectors of 2^(L^2) doubles (distinct),
 *   asynchronous on hip_stream.
 * tfim_tm_top: the n_eig (1 or 2) largest eigenvalues of the even (sector
 *   0, P = +1) or odd (sector 1) sector, e^(k E_0) and e^(k E_1) of that
 *   sector, by power iteration from fixed start vectors (the second with
 *   the first eigenvector removed from every product), each until two
 *   successive Rayleigh quotients differ by at most tol relative or max_iter
 *   products; the normalised eigenvectors are left at the start of ws
 *   (2^(L^2) doubles each).  ws: caller-owned device memory of at least
 *   tfim_tm_workspace bytes, 256-byte aligned.  Synchronous.  lambda_out
 *   and iters_out (may be NULL) take n_eig values. */
tfim_status tfim_tm_workspace(uint32_t L, size_t *bytes_out);
tfim_status tfim_tm_apply(uint32_t L, double k, const int8_t *Jx, const int8_t *Jy,
                          const double *v, double *w, void *hip_stream);
tfim_status tfim_tm_top(uint32_t L, double k, const int8_t *Jx, const int8_t *Jy, uint32_t sector,
                        uint32_t n_eig, double tol, uint32_t max_iter, void *workspace,
                        size_t workspace_bytes, void *hip_stream, double *lambda_out,
                        uint32_t *iters_out);

/* Threshold tables of a shape (host-only): Tm[n_k][3] with
 * Tm[i][u] = floor(2^32 exp(-k_i (12 - 4u))) for u = 0,1,2 unsatisfied
 * bonds of six; dmax[n_k-1]; Tpt[sum dmax] with, for pair i, entries
 * d = 1..dmax[i] equal to floor(2^32 exp(-(k_{i+1}-k_i) 2d)).
 * Any pointer may be NULL.  *n_tpt receives sum(dmax). */
tfim_status tfim_get_thresholds(const tfim_plan *plan, uint32_t shape, uint32_t *Tm,
                                uint32_t *dmax, uint32_t *Tpt, size_t tpt_capacity,
                                size_t *n_tpt);

/* Copy state back in the form's canonical layouts (synchronous): uint64
 * words (multispin) or int8 +-1 (plain). */
tfim_status tfim_export_spins(tfim_plan *plan, uint32_t shape, void *S_host);
tfim_status tfim_export_couplings(tfim_plan *plan, uint32_t shape, void *J_host);
tfim_status tfim_get_state(tfim_plan *plan, uint32_t shape, uint8_t *kidx_host,
                           uint32_t *U_host);
/* Sweep counter t and tempering counter m of a shape (they key its random
 * streams; every shape's t advances with each tfim_sweep). */
tfim_status tfim_get_counters(const tfim_plan *plan, uint32_t shape, uint64_t *t, uint64_t *m);

/* Restore a saved state: spins (canonical) and k labels of one shape, and
 * that shape's counters t, m; energies and lane masks are recomputed.  Resuming from
 * a saved state continues bit-for-bit. */
tfim_status tfim_set_state(tfim_plan *plan, uint32_t shape, const void *S_host,
                           const uint8_t *kidx_host, uint64_t t, uint64_t m);

/* Launch schedules of tfim_sweep (both give bit-identical spins, labels,
 * energies and counters).
 * TFIM_SCHED_PER_SHAPE (default): per sweep, one sweep-kernel launch per
 *   shape (one workgroup per configuration), then per shape a tempering
 *   launch when due and the counter advance: the plain form.
 * TFIM_SCHED_BATCHED: per sweep, ONE launch of a persistent kernel for all
 *   shapes.  Its workgroups take work items (shape, run of configurations)
 *   from a device queue in longest-first order, and pack several
 *   configurations of a small shape into one workgroup.  Then one tempering
 *   launch covers every shape; a shape whose tempering is not due skips
 *   itself.  One counter advance follows.  Runs of up to 16 sweeps are
 *   captured once in a HIP graph and replayed from it.  Needs a bound plan.
 *   Whether a sweep recounts U is decided on the device from the counters. */
#define TFIM_SCHED_BATCHED 0u
#define TFIM_SCHED_PER_SHAPE 1u
/* TFIM_SCHED_CONCURRENT: per sweep, the per-shape sweep launches run on
 *   parallel branches of one HIP graph (fork from the plan's stream, one
 *   branch per shape, join), then one tempering launch for all shapes and
 *   one counter advance, as in the batched schedule.  Each shape keeps its
 *   own workgroup size, and workgroups of different shapes may share a
 *   compute unit.  Runs of up to 16 sweeps are captured once and replayed.
 *   Needs a bound plan. */
#define TFIM_SCHED_CONCURRENT 2u
tfim_status tfim_set_schedule(tfim_plan *plan, uint32_t schedule);

/* Geometry of the batched launch.  threads: threads per workgroup, a
 * multiple of 64, at least the largest shape's L^2 rounded up to 64, at
 * most 768.  blocks_per_cu: resident workgroups per compute unit (0 = as
 * many as fit).  A configuration needs the shape's L^2 (rounded up to 64)
 * threads, and a workgroup sweeps as many configurations of one shape at
 * once as fit in its threads and LDS.  At 768 threads a shape with L^2 =
 * 576 runs one configuration per workgroup with helper waves, as sweep
 * variant 3 does.  Bound plan only; TFIM_EINVAL for a geometry that does not
 * fit. */
tfim_status tfim_set_batch(tfim_plan *plan, uint32_t threads, uint32_t blocks_per_cu);

typedef struct {
    uint32_t schedule;             /* TFIM_SCHED_* in use */
    uint32_t variant;              /* sweep-kernel variant of the per-shape schedule */
    uint32_t batch_threads;        /* batched geometry (0 if never set up) */
    uint32_t batch_blocks_per_cu;
    uint32_t batch_blocks;         /* workgroups of one batched launch */
    uint32_t batch_items;          /* work items of one batched sweep */
    double ms_per_sweep;           /* best trial of the last tfim_autotune, 0 if none */
} tfim_tuning;

/* Autotuner.  Under each candidate (per-shape and concurrent schedules with
 * sweep variants 3, 0 and 2; batched schedule with every workgroup size
 * from the largest team up to 768 threads that packs the shapes' teams
 * differently)
 * it runs one untimed sweep, then `sweeps_per_trial` sweeps timed with HIP
 * events, and keeps the fastest.  The trial sweeps are ordinary sweeps of
 * the chain and every candidate gives the same bits, so the state
 * afterwards equals that after the same number of tfim_sweep calls of one
 * sweep; *sweeps_done (may be NULL) returns that number.
 * cache_path (may be NULL): a choice stored there for the same device and
 * shapes is applied without trials (*sweeps_done = 0); a new choice is
 * written back (one line per key).  Synchronous.  Bound plan only. */
tfim_status tfim_autotune(tfim_plan *plan, uint32_t sweeps_per_trial, const char *cache_path,
                          uint64_t *sweeps_done);
tfim_status tfim_get_tuning(const tfim_plan *plan, tfim_tuning *out);

/* Sweep kernel variant of the per-shape schedule (all give bit-identical
 * chains): 0 = streaming (one barrier per two tau planes), 1 = chunked
 * (eight tau planes per step), 2 = streaming compiled for at least five
 * waves per SIMD, 3 (default) = streaming with three helper waves that
 * compute the uniforms and lane masks of the three column waves sharing a
 * SIMD (L = 24 only; other shapes run variant 0).  Host-only. */
tfim_status tfim_set_variant(tfim_plan *plan, uint32_t variant);

/* Kernel timing: while enabled, tfim_sweep records a pair of HIP events on
 * the bound stream around every sweep-kernel launch (per-shape schedule:
 * one launch per shape and sweep) or around every graph replay (batched
 * schedule: the span covers the sweeps, tempering and counter advances of
 * the replay, and counts as that many launches).  tfim_get_timing
 * synchronises the stream, returns the summed time in ms and the number of
 * timed launches since the last call, and resets them. */
tfim_status tfim_set_timing(tfim_plan *plan, uint32_t enable);
tfim_status tfim_get_timing(tfim_plan *plan, double *kernel_ms, uint64_t *launches);

/* Wait for the bound stream; asynchronous device faults surface here as
 * TFIM_EDEVICE. */
tfim_status tfim_sync(tfim_plan *plan);

const char *tfim_strerror(tfim_status status);
const char *tfim_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* TFIM_H */
