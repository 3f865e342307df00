/*
 * Oracle for the Trotter-Suzuki transverse-field Ising spin glass sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * CPU statement of what the GPU path computes.  Only the tests, the smoke
 * entry point and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it and shares no code with it.
 *
 * Paper: Bernaschi, Gonzalez-Adalid Pemartin, Martin-Mayor, Parisi,
 * "The Quantum Transition of the Two-Dimensional Ising Spin Glass"
 * (arXiv:2310.07486).  Passages followed:
 *   - Methods, "Model and simulations": L x L periodic square lattice,
 *     nearest-neighbour couplings J = +-1 with probability 1/2.
 *   - Methods, "The Trotter-Suzuki formula": classical spins S(x,tau) = +-1
 *     on an L x L x Ltau lattice, p(S) = exp(-k E(S)) / Z with the action
 *     E(S) = -sum_tau [ 1/2 sum_{x,y} J_xy S_x,tau S_y,tau
 *                       + sum_x S_x,tau S_x,tau+1 ],
 *     periodic along tau.  Each bond is counted once.  The same passage
 *     also uses antiperiodic conditions along tau only: the temporal bond
 *     between tau = Ltau-1 and tau = 0 then enters with the sign -1.
 *   - Methods, "Simulation details" and Table I: Metropolis full-lattice
 *     sweeps, parallel tempering (Hukushima-Nemoto) over k, independent
 *     real replicas.
 *
 * Representation: one signed byte per spin (+1 / -1), one signed byte per
 * coupling.  Samples are processed one by one (no multispin coding).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), written here from that
 * paper's definition.  The counter layout is the project's convention
 * (the paper does not name its generator): see oracle_metro_uniform,
 * oracle_pt_uniform and the init functions below.
 *
 * Thresholds: a Metropolis move with energy change dE > 0 is accepted iff
 * R < floor(2^32 exp(-k dE)) for a 32-bit uniform R; dE <= 0 is always
 * accepted.  A tempering swap between k_i and k_{i+1} is accepted iff
 * E_a <= E_b or R < floor(2^32 exp(-(k_{i+1}-k_i)(E_a-E_b))).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TAG_METRO 0u
#define TAG_PT 1u
#define TAG_SPIN 2u
#define TAG_COUPLING 3u

/* ------------------------------------------------------------------ */
/* Philox4x32-10, as defined in the SC'11 paper: ten rounds of the     */
/* two-multiplier S-box, key bumped by the Weyl constants each round.  */
/* ------------------------------------------------------------------ */
void oracle_philox(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t key0 = (uint32_t)(seed & 0xffffffffu);
    uint32_t key1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ key0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ key1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        key0 += W0;
        key1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Fourth counter word: global sample-word index, shape stream, purpose. */
static uint32_t word3(uint32_t j_global, uint32_t stream_id, uint32_t tag)
{
    return (j_global & 0xFFFFFu) | ((stream_id & 0xFFu) << 20) | (tag << 28);
}

/* The 64 bits that seed one (purpose, counter) pair: out0 | out1 << 32. */
static uint64_t philox_bits64(uint32_t c0, uint32_t c1, uint32_t c2,
                              uint32_t c3, uint64_t seed)
{
    uint32_t ctr[4] = {c0, c1, c2, c3}, o[4];
    oracle_philox(ctr, seed, o);
    return (uint64_t)o[0] | ((uint64_t)o[1] << 32);
}

/* Shape of one problem.  Samples are identified by their index s inside the
 * shape (0 .. 64*n_words-1); sample s lives in word j = word_offset + s/64,
 * bit s%64 of the multispin layout, and uses that word's random numbers. */
typedef struct {
    int32_t L, Ltau;
    int32_t n_replicas, n_k;
    uint32_t word_offset, stream_id;
    int32_t pt_every;
    int32_t bc_tau; /* 0: periodic along tau, 1: antiperiodic */
    uint64_t seed;
    const double *k; /* n_k couplings, strictly increasing */
} oracle_shape;

/* ------------------------------------------------------------------ */
/* Instance: J = +-1 with probability 1/2 on every spatial bond.       */
/* Jx[xy] couples (x,y) with (x+1,y); Jy[xy] couples (x,y) with (x,y+1) */
/* ------------------------------------------------------------------ */
void oracle_init_couplings(const oracle_shape *sh, const int32_t *samples,
                           int32_t n_samples, int8_t *Jx, int8_t *Jy)
{
    const int L = sh->L, L2 = L * L;
    for (int si = 0; si < n_samples; ++si) {
        uint32_t s = (uint32_t)samples[si];
        uint32_t j = sh->word_offset + s / 64u, b = s % 64u;
        for (int xy = 0; xy < L2; ++xy) {
            for (int d = 0; d < 2; ++d) {
                uint64_t w = philox_bits64((uint32_t)xy, (uint32_t)d, 0u,
                                           word3(j, sh->stream_id, TAG_COUPLING),
                                           sh->seed);
                int8_t J = ((w >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
                (d == 0 ? Jx : Jy)[(size_t)si * L2 + xy] = J;
            }
        }
    }
}

/* Hot start: every spin of every (replica, walker) i.i.d. +-1.
 * S index: (((r*n_k + w)*n_samples + si)*Ltau + tau)*L*L + xy. */
void oracle_init_spins(const oracle_shape *sh, const int32_t *samples,
                       int32_t n_samples, int8_t *S)
{
    const int L2 = sh->L * sh->L, N = L2 * sh->Ltau;
    for (int r = 0; r < sh->n_replicas; ++r)
        for (int w = 0; w < sh->n_k; ++w)
            for (int si = 0; si < n_samples; ++si) {
                uint32_t s = (uint32_t)samples[si];
                uint32_t j = sh->word_offset + s / 64u, b = s % 64u;
                int8_t *cfg = S + ((size_t)(r * sh->n_k + w) * n_samples + si) * N;
                for (int lin = 0; lin < N; ++lin) {
                    uint64_t word = philox_bits64((uint32_t)lin,
                                                  (uint32_t)(r * sh->n_k + w), 0u,
                                                  word3(j, sh->stream_id, TAG_SPIN),
                                                  sh->seed);
                    cfg[lin] = ((word >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
                }
            }
}

/* ------------------------------------------------------------------ */
/* The action E(S), each bond once; bc = 1 puts the sign -1 on the      */
/* temporal bonds between tau = Ltau-1 and tau = 0 (antiperiodic).      */
/* ------------------------------------------------------------------ */
int64_t oracle_action(int L, int Ltau, int bc, const int8_t *S, const int8_t *Jx,
                      const int8_t *Jy)
{
    const int L2 = L * L;
    int64_t E = 0;
    for (int tau = 0; tau < Ltau; ++tau) {
        const int8_t *P = S + (size_t)tau * L2;
        const int8_t *Pn = S + (size_t)(tau + 1 == Ltau ? 0 : tau + 1) * L2;
        const int64_t ct = (bc && tau == Ltau - 1) ? -1 : 1;
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int xy = x + L * y;
                int xp = (x + 1 == L ? 0 : x + 1) + L * y;
                int yp = x + L * (y + 1 == L ? 0 : y + 1);
                E -= (int64_t)Jx[xy] * P[xy] * P[xp];
                E -= (int64_t)Jy[xy] * P[xy] * P[yp];
                E -= ct * P[xy] * Pn[xy];
            }
    }
    return E;
}

/* Number of unsatisfied bonds, from E = 2U - 3N (N sites, 3N bonds). */
static uint32_t unsat_from_action(int64_t E, int64_t N)
{
    return (uint32_t)((E + 3 * N) / 2);
}

/* Metropolis thresholds: T[i][q] = floor(2^32 exp(-k_i dE)) for the three
 * positive energy changes dE = 4(q+1), q = 0,1,2. */
void oracle_metro_thresholds(const double *k, int n_k, uint32_t *T)
{
    for (int i = 0; i < n_k; ++i)
        for (int q = 0; q < 3; ++q) {
            double dE = 4.0 * (double)(q + 1);
            double p = exp(-(k[i] * dE));
            double v = floor(p * 4294967296.0);
            T[i * 3 + q] = v >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)v;
        }
}

/* Swap threshold for E_a - E_b = dE > 0 between k_i and k_{i+1}. */
uint32_t oracle_pt_threshold(double dk, int64_t dE)
{
    double p = exp(-(dk * (double)dE));
    double v = floor(p * 4294967296.0);
    if (v >= 4294967295.0) return 0xFFFFFFFFu;
    if (v <= 0.0) return 0u;
    return (uint32_t)v;
}

/* Uniform for the Metropolis move at site (xy, tau) of colour c.  The
 * same-colour sites of one column are numbered h = tau/2; four of them
 * share one Philox call (q = h/4), each taking output h%4. */
static uint32_t oracle_metro_uniform(const oracle_shape *sh, uint32_t t,
                                     int r, int w, int c, int xy, int tau,
                                     uint32_t j)
{
    const int L2 = sh->L * sh->L;
    int h = tau >> 1, q = h >> 2;
    uint32_t ctr[4] = {(uint32_t)(xy + L2 * q), t,
                       ((uint32_t)(r * sh->n_k + w) << 1) | (uint32_t)c,
                       word3(j, sh->stream_id, TAG_METRO)};
    uint32_t o[4];
    oracle_philox(ctr, sh->seed, o);
    return o[h & 3];
}

/* Uniform for the tempering decision of pair (i, i+1), step m, replica r,
 * sample bit b of word j: one Philox call serves four consecutive bits. */
static uint32_t oracle_pt_uniform(const oracle_shape *sh, uint32_t m, int r,
                                  int i, uint32_t j, uint32_t b)
{
    uint32_t ctr[4] = {(b >> 2) | ((uint32_t)i << 4), m, (uint32_t)r,
                       word3(j, sh->stream_id, TAG_PT)};
    uint32_t o[4];
    oracle_philox(ctr, sh->seed, o);
    return o[b & 3];
}

/* Recount U for every (r, si, w) from the action. */
void oracle_energy(const oracle_shape *sh, int32_t n_samples, const int8_t *S,
                   const int8_t *Jx, const int8_t *Jy, uint32_t *U)
{
    const int L2 = sh->L * sh->L, N = L2 * sh->Ltau;
    const int nk = sh->n_k;
#pragma omp parallel for collapse(2) schedule(static)
    for (int r = 0; r < sh->n_replicas; ++r)
        for (int w = 0; w < nk; ++w)
            for (int si = 0; si < n_samples; ++si) {
                const int8_t *cfg = S + ((size_t)(r * nk + w) * n_samples + si) * N;
                int64_t E = oracle_action(sh->L, sh->Ltau, sh->bc_tau, cfg, Jx + (size_t)si * L2,
                                          Jy + (size_t)si * L2);
                U[((size_t)r * n_samples + si) * nk + w] = unsat_from_action(E, N);
            }
}

/* Energy change of flipping site (x, y, tau): dE = 2 S h, with h the local
 * field of the four spatial and two temporal neighbours (the neighbour
 * across the tau wrap with the sign -1 when bc = 1). */
static int site_dE(int L, int Ltau, int bc, const int8_t *cfg, const int8_t *jx,
                   const int8_t *jy, int x, int y, int tau)
{
    const int L2 = L * L;
    int xy = x + L * y;
    int xm = (x == 0 ? L - 1 : x - 1) + L * y, xp = (x + 1 == L ? 0 : x + 1) + L * y;
    int ym = x + L * (y == 0 ? L - 1 : y - 1), yp = x + L * (y + 1 == L ? 0 : y + 1);
    int tm = tau == 0 ? Ltau - 1 : tau - 1, tp = tau + 1 == Ltau ? 0 : tau + 1;
    const int8_t *P = cfg + (size_t)tau * L2;
    const int cm = (bc && tau == 0) ? -1 : 1, cp = (bc && tau == Ltau - 1) ? -1 : 1;
    int h = jx[xy] * P[xp] + jx[xm] * P[xm] + jy[xy] * P[yp] + jy[ym] * P[ym] +
            cm * cfg[(size_t)tm * L2 + xy] + cp * cfg[(size_t)tp * L2 + xy];
    return 2 * P[xy] * h;
}

int oracle_local_dE(int L, int Ltau, int bc, const int8_t *cfg, const int8_t *jx,
                    const int8_t *jy, int xy, int tau)
{
    return site_dE(L, Ltau, bc, cfg, jx, jy, xy % L, xy / L, tau);
}

/* One Metropolis half-sweep over the sites of colour c = (x+y+tau) mod 2
 * for every (replica, walker, sample): flip iff dE <= 0 or
 * R < T[k-index][dE/4 - 1].  Sites of one colour only have neighbours of
 * the other colour, so the visiting order is irrelevant.  The uniforms
 * depend on the sample only through its word, so they are drawn once per
 * word into a table R[tau][xy] and then read by each sample of the word. */
static void half_sweep(const oracle_shape *sh, int32_t n_samples,
                       const int32_t *samples, int c, uint32_t t, int8_t *S,
                       const int8_t *Jx, const int8_t *Jy, const uint8_t *kidx,
                       const uint32_t *T)
{
    const int L = sh->L, Lt = sh->Ltau, L2 = L * L, N = L2 * Lt;
    const int nk = sh->n_k;
#pragma omp parallel
    {
        uint32_t *Rtab = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)N);
#pragma omp for collapse(2) schedule(dynamic)
        for (int r = 0; r < sh->n_replicas; ++r)
            for (int w = 0; w < nk; ++w) {
                uint32_t jR = 0xFFFFFFFFu;
                for (int si = 0; si < n_samples; ++si) {
                    uint32_t j = sh->word_offset + (uint32_t)samples[si] / 64u;
                    if (j != jR) {
                        for (int tau = 0; tau < Lt; ++tau)
                            for (int y = 0; y < L; ++y)
                                for (int x = 0; x < L; ++x)
                                    if (((x + y + tau) & 1) == c)
                                        Rtab[(size_t)tau * L2 + x + L * y] =
                                            oracle_metro_uniform(sh, t, r, w, c, x + L * y, tau, j);
                        jR = j;
                    }
                    int8_t *cfg = S + ((size_t)(r * nk + w) * n_samples + si) * N;
                    const int8_t *jx = Jx + (size_t)si * L2, *jy = Jy + (size_t)si * L2;
                    const int i = kidx[((size_t)r * n_samples + si) * nk + w];
                    for (int tau = 0; tau < Lt; ++tau)
                        for (int y = 0; y < L; ++y)
                            for (int x = ((c + y + tau) & 1); x < L; x += 2) {
                                int dE = site_dE(L, Lt, sh->bc_tau, cfg, jx, jy, x, y, tau);
                                size_t lin = (size_t)tau * L2 + x + L * y;
                                /* the table index is only used when dE > 0 */
                                int q = dE > 0 ? dE / 4 - 1 : 0;
                                int accept = (dE <= 0) | (Rtab[lin] < T[i * 3 + q]);
                                cfg[lin] = (int8_t)(accept ? -cfg[lin] : cfg[lin]);
                            }
                }
            }
        free(Rtab);
    }
}

/* One parallel-tempering step: pairs (i, i+1) with i = m mod 2, m mod 2 + 2,
 * ...; for each (replica, sample) independently.  kidx[r][si][w] is the
 * k-index of walker w; walkers keep their configuration, k labels move. */
void oracle_pt_step(const oracle_shape *sh, int32_t n_samples,
                    const int32_t *samples, uint32_t m, const uint32_t *U,
                    uint8_t *kidx)
{
    const int nk = sh->n_k;
    int *winv = (int *)malloc(sizeof(int) * (size_t)nk);
    for (int r = 0; r < sh->n_replicas; ++r)
        for (int si = 0; si < n_samples; ++si) {
            uint32_t s = (uint32_t)samples[si];
            uint32_t j = sh->word_offset + s / 64u, b = s % 64u;
            uint8_t *ki = kidx + ((size_t)r * n_samples + si) * nk;
            const uint32_t *Ur = U + ((size_t)r * n_samples + si) * nk;
            for (int w = 0; w < nk; ++w) winv[ki[w]] = w;
            for (int i = (int)(m & 1u); i + 1 < nk; i += 2) {
                int wa = winv[i], wb = winv[i + 1];
                /* E = 2U - 3N, so E_a - E_b = 2 (U_a - U_b). */
                int64_t dE = 2 * ((int64_t)Ur[wa] - (int64_t)Ur[wb]);
                uint32_t R = oracle_pt_uniform(sh, m, r, i, j, b);
                int accept = dE <= 0 ||
                             R < oracle_pt_threshold(sh->k[i + 1] - sh->k[i], dE);
                if (accept) {
                    ki[wa] = (uint8_t)(i + 1);
                    ki[wb] = (uint8_t)i;
                    winv[i] = wb;
                    winv[i + 1] = wa;
                }
            }
        }
    free(winv);
}

/* n sweeps: colour 0, colour 1, energy recount, and a tempering step after
 * sweep t when pt_every > 0 and (t+1) is a multiple of pt_every.
 * t and m are advanced in place. */
void oracle_run(const oracle_shape *sh, int32_t n_samples, const int32_t *samples,
                int64_t n_sweeps, int8_t *S, const int8_t *Jx, const int8_t *Jy,
                uint8_t *kidx, uint32_t *U, uint32_t *t, uint32_t *m)
{
    uint32_t *T = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)sh->n_k);
    oracle_metro_thresholds(sh->k, sh->n_k, T);
    for (int64_t it = 0; it < n_sweeps; ++it) {
        half_sweep(sh, n_samples, samples, 0, *t, S, Jx, Jy, kidx, T);
        half_sweep(sh, n_samples, samples, 1, *t, S, Jx, Jy, kidx, T);
        oracle_energy(sh, n_samples, S, Jx, Jy, U);
        if (sh->pt_every > 0 && ((*t + 1u) % (uint32_t)sh->pt_every) == 0u) {
            oracle_pt_step(sh, n_samples, samples, *m, U, kidx);
            *m += 1u;
        }
        *t += 1u;
    }
    free(T);
}

/* Identity k labels, as at a fresh start. */
void oracle_reset_kidx(const oracle_shape *sh, int32_t n_samples, uint8_t *kidx)
{
    for (int r = 0; r < sh->n_replicas; ++r)
        for (int si = 0; si < n_samples; ++si)
            for (int w = 0; w < sh->n_k; ++w)
                kidx[((size_t)r * n_samples + si) * sh->n_k + w] = (uint8_t)w;
}
