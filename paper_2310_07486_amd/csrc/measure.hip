// Measurement: replica Gram / overlap integers on int8 MFMA, fused int64
// reductions.
//
// Paper: arXiv:2310.07486, Methods, "One-time observables" (M_xy, M-hat, the
// susceptibilities chi^(2), F^(2) and the second-moment length) with the
// tau average of "The Trotter-Suzuki formula" and the replica estimators of
// "Simulation details".
//
// For configuration (k-index i, sample s) and replica r, S^r is the
// L^2 x Ltau matrix of +-1 spins of walker kidx^-1[i] (lane s).  With
// B = (1 - S)/2 in {0,1}:
//   G^r = S S^T = Ltau - 2 (n_x + n_y) + 4 (B B^T)_xy,  n_x = sum_tau B_x,tau
//   Q^ab = S^aT S^b = L^2 - 2 (m^a_tau + m^b_tau') + 4 (B^aT B^b)_tau,tau'
// so the GEMMs run on {0,1} int8 operands (cheap to unpack from bits) with
// int32 accumulation on v_mfma_i32_32x32x32_i8, exactly.  Per pair a < b the
// epilogues reduce, in int64,
//   D_x[d] = sum_{(x1-y1) mod L = d} G^a_xy G^b_xy (and D_y in x2 - y2),
//   trQ = sum_tau Q_tau,tau,  sum Q^2,  sum Q^4,
// without storing G or Q.
//
// 1. k_transpose turns the multispin words (64 samples per word) into one
//    bit row per sample, in two layouts: bits along tau (Pt, the K axis of G)
//    and bits along xy (Px, the K axis of Q), by 64x64 bit transposes across
//    a wavefront (six xor-shuffle butterfly stages).
// 2. k_gram_mfma: one workgroup per configuration at a time, 64x64 tiles of
//    G (upper triangle of tile pairs), all replicas at once, bucket sums in
//    LDS, flushed once per configuration; for Ltau <= 8192 on fp4 MFMAs
//    (v_mfma_scale_f32_32x32x64_f8f6f4: {0, 0.5} operands, exact in fp32).
// 3. k_overlap_mfma: every wave alone (no LDS, no barrier) on 64x64 tiles of
//    a group of 2 pairs at once that share a replica on one side (one launch
//    per group, two waves per SIMD), operands unpacked in registers, the rank-one corrections folded into one more
//    K step so the accumulator is Q; per-lane int64 sums flushed once per
//    configuration by each of the wave teams that share it.
// The plain per-sample form (k_*_plain) computes one matrix element per
// thread with an int32 multiply-accumulate loop over unpacked spins, one
// launch per configuration: the reference point for the batched form.
#include <algorithm>
#include <type_traits>

#include "tfim_internal.h"

namespace tfim {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));


constexpr int kMaxR = 6;       // replicas handled by the MFMA kernels
constexpr int kMaxP = kMaxR * (kMaxR - 1) / 2;

constexpr int kTP = 65;  // padded row pitch (words) of the transpose tiles
constexpr size_t kTransposeLds = (size_t)64 * kTP * 8 + 64 * 4;

__global__ void __launch_bounds__(256) k_transpose(ShapeDev sh, long long items) {
    extern __shared__ uint64_t tlds[];
    uint64_t(*tile)[kTP] = (uint64_t(*)[kTP])tlds;
    int* mrow = (int*)(tlds + 64 * kTP);
    const int L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, W = sh.W, R = sh.R;
    const int S = 64 * W;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (long long item = blockIdx.x; item < items; item += gridDim.x) {
        const int g = (int)(item % sh.nx);
        const long long rest = item / sh.nx;
        const int c = (int)(rest % sh.nc);
        const int cfg = (int)(rest / sh.nc);  // (r*nk + w)*W + j
        const int j = cfg % W, rw = cfg / W, w = rw % nk, r = rw / nk;
        __syncthreads();
        if (tid < 64) {
            const int s = 64 * j + tid;
            const int i = sh.kidx[((size_t)r * S + s) * nk + w];
            mrow[tid] = (i * S + s) * R + r;
        }
        // the 64 x 64 words of the tile: all 16 loads of a thread in flight
        // at once (the loops are unrolled so that they can be)
        uint64_t v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k;
            const int t = e >> 6, u = e & 63, tau = 64 * c + t, xy = 64 * g + u;
            v[k] = (tau < Lt && xy < L2) ? sh.S[((size_t)cfg * Lt + tau) * L2 + xy] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k;
            tile[e >> 6][e & 63] = v[k];
        }
        __syncthreads();
        // both transposes from the tile into registers, the sixteen of each
        // wave independent chains of lane exchanges; then the tile's LDS
        // serves as the staging buffer of each output in turn (one 33 KB
        // buffer per workgroup)
        uint64_t vt[16], vx[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            vt[k] = tile[lane][wv * 16 + k];  // column u: lanes = tau
            vx[k] = tile[wv * 16 + k][lane];  // row t: lanes = xy
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            vt[k] = wave_transpose64(vt[k]);  // lane = sample bit b, bits along tau
            vx[k] = wave_transpose64(vx[k]);  // lane = sample bit b, bits along xy
        }
        __syncthreads();  // every wave has read the tile
#pragma unroll
        for (int k = 0; k < 16; ++k) tile[lane][wv * 16 + k] = vt[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k;
            const int b = e >> 6, u = e & 63;
            sh.Pt[((size_t)mrow[b] * sh.nc + c) * sh.nxp + 64 * g + u] = tile[b][u];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) tile[lane][wv * 16 + k] = vx[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = tid + 256 * k;
            const int b = e >> 6, t = e & 63, tau = 64 * c + t;
            if (tau < Lt) sh.Px[((size_t)mrow[b] * sh.nx + g) * Lt + tau] = tile[b][t];
        }
    }
}

// ---------------------------------------------------------------------------
// G tiles and the D buckets.
//
// One workgroup takes one configuration at a time.  It first counts the
// down spins n^r_x of every site row (popcount along tau) into LDS; then its
// four waves share the tile pairs (X, Y), X <= Y, of the upper triangle,
// each wave alone (no barrier inside a configuration), one wave per SIMD:
// the 2 x 2 blocks of 32 x 32 of every replica's G^r = S S^T, accumulators
// in the AGPRs, K = tau in chunks of 64, the {0,1} operands built in
// registers from each lane's bit row.  With the int32 epilogue (NARROW), up
// to 4 replicas and more configurations than CUs, two workgroups share a
// CU, two waves a SIMD (one's MFMAs run while the other builds operands),
// each wave on half a tile pair (the 2 x 1 blocks of a column half) above 2
// replicas.  The epilogue forms
// G = Ltau - 2 (n_x + n_y) + 4 (B B^T)_xy and the products G^a G^b.
//
// An element (x, y) of an off-diagonal pair stands for (y, x) too, with the
// displacements negated; its products go to U, those of the diagonal
// blocks of diagonal pairs to F, and the flush folds D[d] = F[d] + U[d] +
// U[-d mod L].  In a diagonal pair the block (rows 32.., columns 0..31) is
// the mirror of (rows 0.., columns 32..): only the latter is computed, into
// U.
//
// BLK (L a multiple of 8): tile X holds the 8 x 8 block of sites
// (bx, by) = (X mod L/8, X div L/8), row r the site (8bx + r mod 8,
// 8by + r div 8).  The 16 elements of a lane then take 4 values of x1 - y1
// (one per q mod 4) and 4 of x2 - y2 (one per q div 4), so each lane sums
// them in registers and adds 8 bucket values per pair and block, not 32.
// Otherwise tile X holds the sites 64X .. 64X + 63 and every element adds
// its own two.
//
// NARROW (BLK and Ltau <= 8192): the products and the lane sums are int32
// (24-bit multiplies), and a lane's x1 - y1 sums, the same in every block
// of a tile pair, are flushed once per pair; otherwise they are int64.
// ---------------------------------------------------------------------------
constexpr int kGramWaves = 4;
constexpr int kNarrowLt = 8192;  // the int32 epilogue: |G| <= 2^13
// waves per SIMD: two where a wave's accumulators (RR x 2 x NV blocks of
// 16 per lane) fit in half the register file, with the int32 epilogue
constexpr int gram_wpe(int RR, int NV, bool narrow) { return narrow && RR * NV <= 4 ? 2 : 1; }

template <int RR, int NV, bool BLK, bool NARROW>
__global__ void __launch_bounds__(64 * kGramWaves)
    __attribute__((amdgpu_waves_per_eu(gram_wpe(RR, NV, NARROW), gram_wpe(RR, NV, NARROW))))
k_gram_mfma(ShapeDev sh, int cfg0, int ncfg) {
    static_assert(BLK || !NARROW, "the int32 epilogue takes the 8 x 8 site blocks");
    constexpr int PP = RR * (RR - 1) / 2;
    extern __shared__ __align__(16) uint8_t smem[];
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt, nc = sh.nc, nxp = sh.nxp;
    unsigned long long* Fb = (unsigned long long*)smem;  // [PP][2][L]
    unsigned long long* Ub = Fb + PP * 2 * L;             // [PP][2][L]
    int* nS = (int*)(Ub + PP * 2 * L);                    // [RR][nxp]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i = lane & 31, h = lane >> 5, sh4 = 4 * h;
    const int ntile = sh.nx;
    const int ntp = ntile * (ntile + 1) / 2;
    const int nbl = L >> 3;
    auto site = [&](int X, int r) {
        if constexpr (BLK) return (8 * (X / nbl) + (r >> 3)) * L + 8 * (X % nbl) + (r & 7);
        return 64 * X + r;
    };
    for (int e = tid; e < 2 * PP * 2 * L; e += 64 * kGramWaves) Fb[e] = 0;  // F and U
    for (int cfg = cfg0 + blockIdx.x; cfg < cfg0 + ncfg; cfg += gridDim.x) {
        const uint64_t* const pt = sh.Pt + (size_t)cfg * RR * nc * nxp;
        for (int e = tid; e < RR * nxp; e += 64 * kGramWaves) {
            const int r = e / nxp, xy = e - r * nxp;
            int n = 0;
            for (int c = 0; c < nc; ++c) n += __popcll(pt[((size_t)r * nc + c) * nxp + xy]);
            nS[e] = n;
        }
        __syncthreads();
        // work units: tile pairs, or (NV = 1) their two column halves
        for (int unit = wv; unit < ntp * (2 / NV); unit += kGramWaves) {
            const int tp = NV == 2 ? unit : unit >> 1;
            const int v0 = NV == 2 ? 0 : (unit & 1);  // first column block
            int X = 0, rem = tp;
            while (rem >= ntile - X) { rem -= ntile - X; ++X; }
            const int Y = X + rem;
            const int sa[2] = {site(X, i), site(X, 32 + i)};
            int sb[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) sb[v] = site(Y, 32 * (v0 + v) + i);
            // NARROW: fp32 accumulators of the fp4 form (below), else int32
            using Acc = std::conditional_t<NARROW, v16f, v16i>;
            Acc acc[RR][2][NV];
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < NV; ++v)
#pragma unroll
                        for (int q = 0; q < 16; ++q) acc[r][u][v][q] = 0;
            // The fp4 K loop: 64 values of tau per MFMA.  Lane (i, h) feeds
            // row i with the 32 bits of half h of its chunk word, element
            // 8m + j (register m, nibble j) being bit 4j + m, as the e2m1
            // values 0 and 0.5 (nibble 0 or 1: one mask per register).  The
            // row side's block scale 2^4 makes each coincidence add 4, so the
            // accumulator holds 4 (B B^T), exact in fp32 (at most 4 Ltau).
            auto kloop4 = [&](auto diagC) {
                constexpr bool kDiag = decltype(diagC)::value;
                constexpr int NB = kDiag ? 0 : NV;
                const uint32_t* const pt32 = (const uint32_t*)pt;
                auto fetch = [&](int c, uint32_t (&wa)[2][RR], uint32_t (&wb)[NV][RR]) {
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        const size_t o = ((size_t)r * nc + c) * nxp;
#pragma unroll
                        for (int u = 0; u < 2; ++u) wa[u][r] = pt32[2 * (o + sa[u]) + h];
#pragma unroll
                        for (int v = 0; v < NB; ++v) wb[v][r] = pt32[2 * (o + sb[v]) + h];
                    }
                };
                auto chunk = [&](const uint32_t (&wa)[2][RR], const uint32_t (&wb)[NV][RR]) {
                    i32x8 A[2][RR], B[NV][RR];
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
#pragma unroll
                        for (int u = 0; u < 2; ++u) A[u][r] = fp4_bits_operand(wa[u][r]);
#pragma unroll
                        for (int v = 0; v < NB; ++v) B[v][r] = fp4_bits_operand(wb[v][r]);
                    }
#pragma unroll
                    for (int r = 0; r < RR; ++r)
#pragma unroll
                        for (int u = 0; u < 2; ++u)
#pragma unroll
                            for (int v = 0; v < NV; ++v) {
                                if (kDiag && NV == 2 && u == 1 && v == 0) continue;
                                const i32x8 b = kDiag ? A[NV == 2 ? v : v0][r] : B[v][r];
                                acc[r][u][v] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                                    A[u][r], b, acc[r][u][v], kFp4, kFp4, 0, kScaleRow, 0, kScaleOne);
                            }
                };
                uint32_t w0a[2][RR], w0b[NV][RR], w1a[2][RR], w1b[NV][RR];
                fetch(0, w0a, w0b);
                for (int c = 0; c + 1 < nc; c += 2) {
                    fetch(c + 1, w1a, w1b);
                    chunk(w0a, w0b);
                    fetch(min(c + 2, nc - 1), w0a, w0b);
                    chunk(w1a, w1b);
                }
                if (nc & 1) chunk(w0a, w0b);
            };
            // the K loop; kDiag: Y = X, the column rows are row rows (no
            // loads of their own) and, with both column blocks, the block
            // (1, 0) is skipped
            auto kloop = [&](auto diagC) {
                constexpr bool kDiag = decltype(diagC)::value;
                constexpr int NB = kDiag ? 0 : NV;  // column-side words loaded
                auto fetch = [&](int c, uint64_t (&wa)[2][RR], uint64_t (&wb)[NV][RR]) {
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        const size_t o = ((size_t)r * nc + c) * nxp;
#pragma unroll
                        for (int u = 0; u < 2; ++u) wa[u][r] = pt[o + sa[u]];
#pragma unroll
                        for (int v = 0; v < NB; ++v) wb[v][r] = pt[o + sb[v]];
                    }
                };
                auto chunk = [&](const uint64_t (&wa)[2][RR], const uint64_t (&wb)[NV][RR]) {
#pragma unroll
                    for (int ks = 0; ks < 2; ++ks) {
                        i32x4 A[2][RR], B[NV][RR];
#pragma unroll
                        for (int r = 0; r < RR; ++r) {
#pragma unroll
                            for (int u = 0; u < 2; ++u)
                                A[u][r] = mfma_bits_operand<false>((uint32_t)(wa[u][r] >> (32 * ks)) >> sh4);
#pragma unroll
                            for (int v = 0; v < NB; ++v)
                                B[v][r] = mfma_bits_operand<false>((uint32_t)(wb[v][r] >> (32 * ks)) >> sh4);
                        }
#pragma unroll
                        for (int r = 0; r < RR; ++r)
#pragma unroll
                            for (int u = 0; u < 2; ++u)
#pragma unroll
                                for (int v = 0; v < NV; ++v) {
                                    if (kDiag && NV == 2 && u == 1 && v == 0) continue;
                                    const i32x4 b = kDiag ? A[NV == 2 ? v : v0][r] : B[v][r];
                                    acc[r][u][v] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[u][r], b, acc[r][u][v],
                                                                                         0, 0, 0);
                                }
                    }
                };
                // two word sets in turn, the next chunk in flight during this
                // one; one straight loop block (a fetch past the last chunk
                // reloads it) keeps the loads ahead and the waits exact
                uint64_t w0a[2][RR], w0b[NV][RR], w1a[2][RR], w1b[NV][RR];
                fetch(0, w0a, w0b);
                for (int c = 0; c + 1 < nc; c += 2) {
                    fetch(c + 1, w1a, w1b);
                    chunk(w0a, w0b);
                    fetch(min(c + 2, nc - 1), w0a, w0b);
                    chunk(w1a, w1b);
                }
                if (nc & 1) chunk(w0a, w0b);
            };
            // the K loop and the epilogue of a diagonal or an off-diagonal
            // pair, each its own straight code (the accumulators never meet
            // at a branch join)
            auto finish = [&](auto diagC) {
            constexpr bool diag = decltype(diagC)::value;
            if constexpr (NARROW)
                kloop4(diagC);
            else
                kloop(diagC);
            // epilogue, block by block
            if constexpr (NARROW) {
                // |G| <= Ltau <= 8192: a product is below 2^26 and a sum of
                // 16 of them below 2^30, so both are formed in int32 with
                // 24-bit multiplies.  The x1 - y1 buckets of a lane are the
                // same in every block of the tile, so an off-diagonal pair
                // sums them over its blocks and flushes them once.
                const int x1 = 8 * (X % nbl) + 4 * h, y1 = 8 * (Y % nbl) + (i & 7);
                int sxa[PP][4];
#pragma unroll
                for (int p = 0; p < PP; ++p)
#pragma unroll
                    for (int j = 0; j < 4; ++j) sxa[p][j] = 0;
                auto flush_x = [&](unsigned long long* Db) {
#pragma unroll
                    for (int p = 0; p < PP; ++p)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            atomicAdd(&Db[(p * 2 + 0) * L + (x1 + j - y1 + L) % L],
                                      (unsigned long long)(long long)sxa[p][j]);
                            sxa[p][j] = 0;
                        }
                };
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    int rn[RR][16];  // 2 n^r of the rows of this lane's elements
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int xs = site(X, 32 * u + 8 * (q >> 2) + 4 * h + (q & 3));
#pragma unroll
                        for (int r = 0; r < RR; ++r) rn[r][q] = 2 * nS[r * nxp + xs];
                    }
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const int V = v0 + v;
                        if (diag && NV == 2 && u == 1 && V == 0) continue;
                        unsigned long long* Db = (diag && (NV == 1 || u == V)) ? Fb : Ub;
                        const int x2 = 8 * (X / nbl) + 4 * u, y2 = 8 * (Y / nbl) + ((32 * V + i) >> 3);
                        int G[RR][16];
#pragma unroll
                        for (int r = 0; r < RR; ++r) {
                            const int nb = Lt - 2 * nS[r * nxp + sb[v]];
#pragma unroll
                            for (int q = 0; q < 16; ++q) G[r][q] = nb - rn[r][q] + (int)acc[r][u][v][q];
                        }
                        int p = 0;
#pragma unroll
                        for (int a = 0; a < RR; ++a)
#pragma unroll
                            for (int b = a + 1; b < RR; ++b, ++p) {
                                int sy[4] = {0, 0, 0, 0};
#pragma unroll
                                for (int q = 0; q < 16; ++q) {
                                    const int hv = __mul24(G[a][q], G[b][q]);
                                    sxa[p][q & 3] += hv;
                                    sy[q >> 2] += hv;
                                }
#pragma unroll
                                for (int j = 0; j < 4; ++j)
                                    atomicAdd(&Db[(p * 2 + 1) * L + (x2 + j - y2 + L) % L],
                                              (unsigned long long)(long long)sy[j]);
                            }
                        if (diag) flush_x(Db);
                    }
                }
                if (!diag) flush_x(Ub);
            } else
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const int V = v0 + v;  // column block in the tile
                    if (diag && NV == 2 && u == 1 && V == 0) continue;
                    unsigned long long* Db = (diag && (NV == 1 || u == V)) ? Fb : Ub;
                    const int ys = sb[v];  // this lane's column site
                    int nb[RR];
#pragma unroll
                    for (int r = 0; r < RR; ++r) nb[r] = Lt - 2 * nS[r * nxp + ys];
                    // G^r of element q (|G| <= Ltau <= 2^16)
                    auto gram = [&](int q, int (&G)[RR]) {
                        const int xs = site(X, 32 * u + 8 * (q >> 2) + 4 * h + (q & 3));
#pragma unroll
                        for (int r = 0; r < RR; ++r) G[r] = nb[r] - 2 * nS[r * nxp + xs] + 4 * acc[r][u][v][q];
                    };
                    if constexpr (BLK) {
                        // x1 - y1 by q mod 4 and x2 - y2 by q div 4, all sites valid
                        const int col = 32 * V + i;
                        const int y1 = 8 * (Y % nbl) + (col & 7), y2 = 8 * (Y / nbl) + (col >> 3);
                        const int x1 = 8 * (X % nbl) + 4 * h, x2 = 8 * (X / nbl) + 4 * u;
                        int Gq[RR][16];
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            int G[RR];
                            gram(q, G);
#pragma unroll
                            for (int r = 0; r < RR; ++r) Gq[r][q] = G[r];
                        }
                        int p = 0;
#pragma unroll
                        for (int a = 0; a < RR; ++a)
#pragma unroll
                            for (int b = a + 1; b < RR; ++b, ++p) {
                                long long sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
#pragma unroll
                                for (int q = 0; q < 16; ++q) {
                                    const long long hv = (long long)Gq[a][q] * Gq[b][q];
                                    sx[q & 3] += hv;
                                    sy[q >> 2] += hv;
                                }
#pragma unroll
                                for (int j = 0; j < 4; ++j) {
                                    atomicAdd(&Db[(p * 2 + 0) * L + (x1 + j - y1 + L) % L], (unsigned long long)sx[j]);
                                    atomicAdd(&Db[(p * 2 + 1) * L + (x2 + j - y2 + L) % L], (unsigned long long)sy[j]);
                                }
                            }
                    } else {
                        const int y = ys;
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            const int x = site(X, 32 * u + 8 * (q >> 2) + 4 * h + (q & 3));
                            if (x >= L2 || y >= L2) continue;
                            int G[RR];
                            gram(q, G);
                            const int dx = (x % L - y % L + L) % L, dy = (x / L - y / L + L) % L;
                            int p = 0;
#pragma unroll
                            for (int a = 0; a < RR; ++a)
#pragma unroll
                                for (int b = a + 1; b < RR; ++b, ++p) {
                                    const unsigned long long hv = (unsigned long long)((long long)G[a] * G[b]);
                                    atomicAdd(&Db[(p * 2 + 0) * L + dx], hv);
                                    atomicAdd(&Db[(p * 2 + 1) * L + dy], hv);
                                }
                        }
                    }
                }
            };
            if (X == Y)
                finish(std::true_type{});
            else
                finish(std::false_type{});
        }
        __syncthreads();
        // D[d] = F[d] + U[d] + U[-d]; sum Q^2 = sum_xy G^a_xy G^b_xy =
        // sum_d D_x[d] (one workgroup holds all of this configuration's
        // buckets)
        const int rl = 2 * L + 3;
        for (int e = tid; e < PP * 2 * L; e += 64 * kGramWaves) {
            const int d = e % L;
            Fb[e] += Ub[e] + Ub[e - d + (L - d) % L];
        }
        __syncthreads();
        if (tid < PP) {
            unsigned long long q2 = 0;
            for (int d = 0; d < L; ++d) q2 += Fb[(tid * 2 + 0) * L + d];
            sh.rec[((size_t)cfg * PP + tid) * rl + 2 * L + 1] = (int64_t)q2;
        }
        for (int e = tid; e < PP * 2 * L; e += 64 * kGramWaves) {
            const int p = e / (2 * L), d = e % (2 * L);
            sh.rec[((size_t)cfg * PP + p) * rl + d] = (int64_t)Fb[e];
        }
        __syncthreads();
        for (int e = tid; e < 2 * PP * 2 * L; e += 64 * kGramWaves) Fb[e] = 0;
    }
}

// ---------------------------------------------------------------------------
// Q tiles: trQ and sum Q^4 for the NP pairs of launch group GI (records of
// pairs a < b in lexicographic order; sum Q^2 comes from the Gram buckets).
//
// Every wave works alone, with no LDS and no barrier: a 64 x 64 tile
// (tau in 64T + [0, 64), tau' in 64T2 + [0, 64)) of each of its pairs as
// 2 x 2 blocks of 32 x 32, the accumulators 64 registers per pair, two pairs
// per launch, two waves per SIMD (one wave's MFMAs run while the other
// builds its operands).  The operands come straight from each lane's
// packed row words: in K step ks of chunk g, lane (i, h) of a block feeds
// row i with bits 8j + 4h + m (j, m < 4) of the 32-bit half ks of its word,
// one byte each, in the same order on both sides.  Row-side bytes are 4 B
// (0 or 4), column-side bytes B, so the K steps sum 4 B^aT B^b; one more K
// step adds X_tau + Y_tau' with X = h2 - 2 m^a_tau and
// Y = (L^2 - h2) - 2 m^b_tau' (h2 = floor(L^2 / 2)), held as sixteen int8
// pieces on one side against ones on the other.  The accumulator is then
// Q itself: the epilogue squares it twice and adds.
//
// Waves form teams of wc.  Team t takes configurations t, t + nteams, ...;
// its member j the tiles j, j + wc, ... of each, and it flushes its sums
// once per configuration.  Workgroup b runs on XCD b mod nxcd, so a team
// no larger than an XCD's share of waves reads its rows from one L2.
// ---------------------------------------------------------------------------
// The launch groups of the replica pairs (pair p = (a, b), a < b, in
// lexicographic order): two pairs (a, b), (a, c) with the same row-side
// replica per group, the pairs left over two at a time, the last alone.  A
// group then builds 3 operand sets for its 4 MFMA blocks per K step.
template <int RR>
struct PairGroups {
    static constexpr int PP = RR * (RR - 1) / 2;
    int pair[PP] = {};   // pair indices in launch order
    int first[PP] = {};  // first position of group k in pair[]
    int size[PP] = {};   // pairs of group k (1 or 2)
    int n = 0;           // groups
    constexpr PairGroups() {
        int left[PP] = {}, nl = 0, at = 0, p = 0;
        for (int a = 0; a < RR; ++a) {
            const int p0 = p, cnt = RR - 1 - a;
            p += cnt;
            int k = 0;
            for (; k + 1 < cnt; k += 2) {
                first[n] = at; size[n++] = 2;
                pair[at++] = p0 + k;
                pair[at++] = p0 + k + 1;
            }
            if (k < cnt) left[nl++] = p0 + k;
        }
        for (int k = 0; k < nl; k += 2) {
            first[n] = at; size[n++] = k + 1 < nl ? 2 : 1;
            pair[at++] = left[k];
            if (k + 1 < nl) pair[at++] = left[k + 1];
        }
    }
};
constexpr int pair_row(int R, int p) {
    int a = 0;
    while (p >= R - 1 - a) { p -= R - 1 - a; ++a; }
    return a;
}
constexpr int pair_col(int R, int p) {
    int a = 0;
    while (p >= R - 1 - a) { p -= R - 1 - a; ++a; }
    return a + 1 + p;
}

// Row-side and column-side replica slots of launch group GI (NP pairs).
template <int RR, int GI, int NP>
struct PairSides {
    int na = 0, nb = 0;
    int ra[RR] = {}, rb[RR] = {};  // replica of each row-side / column-side slot
    int pa[NP] = {}, pb[NP] = {};  // slots of the group's pair p
    int pi[NP] = {};               // record index of the group's pair p
    constexpr PairSides() {
        constexpr PairGroups<RR> grp{};
        int sa[RR] = {}, sb[RR] = {};
        for (int r = 0; r < RR; ++r) sa[r] = sb[r] = -1;
        for (int k = 0; k < NP; ++k) {
            const int p = grp.pair[grp.first[GI] + k];
            const int a = pair_row(RR, p), b = pair_col(RR, p);
            if (sa[a] < 0) { sa[a] = na; ra[na++] = a; }
            if (sb[b] < 0) { sb[b] = nb; rb[nb++] = b; }
            pa[k] = sa[a];
            pb[k] = sb[b];
            pi[k] = p;
        }
    }
};

constexpr int kTeamWaves = 4;  // waves per workgroup of the overlap kernel

template <int RR, int GI, int NP>
__global__ void __launch_bounds__(64 * kTeamWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_overlap_mfma(ShapeDev sh, int cfg0, int ncfg, int wc, int nxcd) {
    constexpr PairSides<RR, GI, NP> ps{};
    constexpr int NA = ps.na, NB = ps.nb;
    constexpr int PP = RR * (RR - 1) / 2;
    const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5, sh4 = 4 * h;
    const int G = gridDim.x * kTeamWaves, gx = G / nxcd;
    const int xcd = blockIdx.x % nxcd;
    const int s = (blockIdx.x / nxcd) * kTeamWaves + (threadIdx.x >> 6);
    int team, member;
    if (wc <= gx) {
        team = xcd * (gx / wc) + s / wc;
        member = s % wc;
    } else {
        const int k = wc / gx;
        team = xcd / k;
        member = (xcd % k) * gx + s;
    }
    const int nteams = G / wc;
    const int L2 = sh.L2, Lt = sh.Lt, nx = sh.nx, ntt = (Lt + 63) / 64, ntiles = ntt * ntt;
    const int h2 = L2 >> 1;
    const int rl = 2 * sh.L + 3;
    if (member >= ntiles) return;
    for (int cfg = cfg0 + team; cfg < cfg0 + ncfg; cfg += nteams) {
        unsigned long long s4[NP];
        int tr[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            s4[p] = 0;
            tr[p] = 0;
        }
        const uint64_t* const px = sh.Px + (size_t)cfg * RR * nx * Lt;
        for (int t = member; t < ntiles; t += wc) {
            const int T = t / ntt, T2 = t - T * ntt;
            // this lane's rows: tau = 64T + 32u + i (row side), 64T2 + 32v + i
            // (column side), clamped into [0, Lt): a row past Lt only feeds
            // elements of its own row or column, which the epilogue skips, and
            // loads without a branch let the wait counts stay exact
            const int ta0 = 64 * T + i, tb0 = 64 * T2 + i;
            const int rowa[2] = {min(ta0, Lt - 1), min(ta0 + 32, Lt - 1)};
            const int rowb[2] = {min(tb0, Lt - 1), min(tb0 + 32, Lt - 1)};
            auto fetch = [&](int g, uint64_t (&wa)[2][NA], uint64_t (&wb)[2][NB]) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
#pragma unroll
                    for (int a = 0; a < NA; ++a) wa[u][a] = px[((size_t)ps.ra[a] * nx + g) * Lt + rowa[u]];
#pragma unroll
                    for (int b = 0; b < NB; ++b) wb[u][b] = px[((size_t)ps.rb[b] * nx + g) * Lt + rowb[u]];
                }
            };
            v16i acc[NP][2][2];
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v)
#pragma unroll
                        for (int q = 0; q < 16; ++q) acc[p][u][v][q] = 0;
            int ma[2][NA], mb[2][NB];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
#pragma unroll
                for (int a = 0; a < NA; ++a) ma[u][a] = 0;
#pragma unroll
                for (int b = 0; b < NB; ++b) mb[u][b] = 0;
            }
            auto chunk = [&](const uint64_t (&wa)[2][NA], const uint64_t (&wb)[2][NB]) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
#pragma unroll
                    for (int a = 0; a < NA; ++a) ma[u][a] += __popcll(wa[u][a]);
#pragma unroll
                    for (int b = 0; b < NB; ++b) mb[u][b] += __popcll(wb[u][b]);
                }
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    v4i A[2][NA], B[2][NB];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
#pragma unroll
                        for (int a = 0; a < NA; ++a)
                            A[u][a] = mfma_bits_operand<true>((uint32_t)(wa[u][a] >> (32 * ks)) >> sh4);
#pragma unroll
                        for (int b = 0; b < NB; ++b)
                            B[u][b] = mfma_bits_operand<false>((uint32_t)(wb[u][b] >> (32 * ks)) >> sh4);
                    }
#pragma unroll
                    for (int p = 0; p < NP; ++p)
#pragma unroll
                        for (int u = 0; u < 2; ++u)
#pragma unroll
                            for (int v = 0; v < 2; ++v)
                                acc[p][u][v] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                    A[u][ps.pa[p]], B[v][ps.pb[p]], acc[p][u][v], 0, 0, 0);
                }
            };
            // two word sets in turn, the next chunk's loads in flight during
            // this chunk's MFMAs; the loop body is one straight block (past
            // the last chunk a fetch reloads it) so that the loads stay ahead
            // of their uses and the wait counts are fixed
            uint64_t w0a[2][NA], w0b[2][NB], w1a[2][NA], w1b[2][NB];
            fetch(0, w0a, w0b);
            for (int g = 0; g + 1 < nx; g += 2) {
                fetch(g + 1, w1a, w1b);
                chunk(w0a, w0b);
                fetch(min(g + 2, nx - 1), w0a, w0b);
                chunk(w1a, w1b);
            }
            if (nx & 1) chunk(w0a, w0b);
            // the correction step: X on the row side's first half-wave, Y on
            // the column side's second, ones against them
            {
                const v4i ones = {0x01010101, 0x01010101, 0x01010101, 0x01010101};
                v4i A[2][NA], B[2][NB];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
#pragma unroll
                    for (int a = 0; a < NA; ++a) A[u][a] = h ? ones : mfma_pieces16(h2 - 2 * ma[u][a]);
#pragma unroll
                    for (int b = 0; b < NB; ++b) B[u][b] = h ? mfma_pieces16(L2 - h2 - 2 * mb[u][b]) : ones;
                }
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int v = 0; v < 2; ++v)
                            acc[p][u][v] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                A[u][ps.pa[p]], B[v][ps.pb[p]], acc[p][u][v], 0, 0, 0);
            }
            // epilogue: |Q| <= L^2, Q^2 < 2^20, Q^4 < 2^40
            if (64 * (T + 1) <= Lt && 64 * (T2 + 1) <= Lt && T != T2) {
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int v = 0; v < 2; ++v)
#pragma unroll
                            for (int q = 0; q < 16; ++q) {
                                const int qv = acc[p][u][v][q];
                                const uint32_t q2 = (uint32_t)__mul24(qv, qv);
                                s4[p] += (unsigned long long)q2 * q2;
                            }
            } else {
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        const int col = 64 * T2 + 32 * v + i;
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            const int row = 64 * T + 32 * u + 8 * (q >> 2) + 4 * h + (q & 3);
                            if (row >= Lt || col >= Lt) continue;
#pragma unroll
                            for (int p = 0; p < NP; ++p) {
                                const int qv = acc[p][u][v][q];
                                const uint32_t q2 = (uint32_t)__mul24(qv, qv);
                                s4[p] += (unsigned long long)q2 * q2;
                                if (row == col) tr[p] += qv;
                            }
                        }
                    }
            }
        }
        // per-configuration flush: wave reduction, one atomic per value
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                s4[p] += (unsigned long long)__shfl_xor((long long)s4[p], off, 64);
                tr[p] += __shfl_xor(tr[p], off, 64);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                unsigned long long* rp = (unsigned long long*)(sh.rec + ((size_t)cfg * PP + ps.pi[p]) * rl);
                atomicAdd(rp + 2 * sh.L, (unsigned long long)(long long)tr[p]);
                atomicAdd(rp + 2 * sh.L + 2, s4[p]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Plain per-sample form: one configuration per launch, one matrix element
// per thread, int32 multiply-accumulate over unpacked +-1 spins.
// ---------------------------------------------------------------------------
// +-1 spins t = 0..63 of a 64-bit row word: 1 - 2 bit_t, 0 past n valid bits.
__device__ __forceinline__ int dot64(uint64_t a, uint64_t b, int n) {
    int acc = 0;
    for (int t = 0; t < n; ++t)
        acc += (1 - 2 * (int)((a >> t) & 1ull)) * (1 - 2 * (int)((b >> t) & 1ull));
    return acc;
}

__global__ void __launch_bounds__(256) k_gram_plain(ShapeDev sh, int cfg) {
    __shared__ unsigned long long Dblk[kMaxP * 2 * 32];
    const int L = sh.L, L2 = sh.L2, R = sh.R, P = sh.P;
    for (int e = threadIdx.x; e < P * 2 * L; e += blockDim.x) Dblk[e] = 0;
    __syncthreads();
    const long long el = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (el < (long long)L2 * L2) {
        const int x = (int)(el / L2), y = (int)(el % L2);
        int G[kMaxR];
        for (int r = 0; r < R; ++r) {
            const size_t m = (size_t)cfg * R + r;
            int acc = 0;
            for (int c = 0; c < sh.nc; ++c)
                acc += dot64(sh.Pt[(m * sh.nc + c) * sh.nxp + x], sh.Pt[(m * sh.nc + c) * sh.nxp + y],
                             min(64, sh.Lt - 64 * c));
            G[r] = acc;
        }
        const int dx = ((x % L) - (y % L) + L) % L, dy = ((x / L) - (y / L) + L) % L;
        int p = 0;
        for (int a = 0; a < R; ++a)
            for (int b = a + 1; b < R; ++b, ++p) {
                const unsigned long long h = (unsigned long long)((long long)G[a] * G[b]);
                atomicAdd(&Dblk[(p * 2 + 0) * L + dx], h);
                atomicAdd(&Dblk[(p * 2 + 1) * L + dy], h);
            }
    }
    __syncthreads();
    const int rl = 2 * L + 3;
    for (int e = threadIdx.x; e < P * 2 * L; e += blockDim.x)
        atomicAdd((unsigned long long*)&sh.rec[((size_t)cfg * P + e / (2 * L)) * rl + e % (2 * L)], Dblk[e]);
}

__global__ void __launch_bounds__(256) k_overlap_plain(ShapeDev sh, int cfg) {
    __shared__ unsigned long long red[kMaxP * 3];
    const int Lt = sh.Lt, L2 = sh.L2, R = sh.R, P = sh.P;
    for (int e = threadIdx.x; e < P * 3; e += blockDim.x) red[e] = 0;
    __syncthreads();
    const long long el = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (el < (long long)Lt * Lt) {
        const int tau = (int)(el / Lt), tau2 = (int)(el % Lt);
        int p = 0;
        for (int a = 0; a < R; ++a)
            for (int b = a + 1; b < R; ++b, ++p) {
                const size_t ma = (size_t)cfg * R + a, mb = (size_t)cfg * R + b;
                int q = 0;
                for (int g = 0; g < sh.nx; ++g)
                    q += dot64(sh.Px[(ma * sh.nx + g) * Lt + tau], sh.Px[(mb * sh.nx + g) * Lt + tau2],
                               min(64, L2 - 64 * g));
                const long long q2 = (long long)q * q;
                atomicAdd(&red[p * 3 + 1], (unsigned long long)q2);
                atomicAdd(&red[p * 3 + 2], (unsigned long long)(q2 * q2));
                if (tau == tau2) atomicAdd(&red[p * 3 + 0], (unsigned long long)(long long)q);
            }
    }
    __syncthreads();
    const int rl = 2 * sh.L + 3;
    for (int e = threadIdx.x; e < P * 3; e += blockDim.x)
        atomicAdd((unsigned long long*)&sh.rec[((size_t)cfg * P + e / 3) * rl + 2 * sh.L + e % 3], red[e]);
}

// Debug dump of G^a, G^b (L2 x L2) and Q^ab (Ltau x Ltau) of one configuration.
__global__ void k_dump(ShapeDev sh, int cfg, int a, int b) {
    const int L2 = sh.L2, Lt = sh.Lt, R = sh.R;
    const long long n1 = (long long)L2 * L2, n = 2 * n1 + (long long)Lt * Lt;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        int acc = 0;
        if (e < 2 * n1) {
            const int r = e < n1 ? a : b;
            const long long f = e % n1;
            const int x = (int)(f / L2), y = (int)(f % L2);
            const size_t m = (size_t)cfg * R + r;
            for (int c = 0; c < sh.nc; ++c)
                acc += dot64(sh.Pt[(m * sh.nc + c) * sh.nxp + x], sh.Pt[(m * sh.nc + c) * sh.nxp + y],
                             min(64, Lt - 64 * c));
        } else {
            const long long f = e - 2 * n1;
            const int tau = (int)(f / Lt), tau2 = (int)(f % Lt);
            const size_t ma = (size_t)cfg * R + a, mb = (size_t)cfg * R + b;
            for (int g = 0; g < sh.nx; ++g)
                acc += dot64(sh.Px[(ma * sh.nx + g) * Lt + tau], sh.Px[(mb * sh.nx + g) * Lt + tau2],
                             min(64, L2 - 64 * g));
        }
        sh.dump[e] = acc;
    }
}

// A[i][h][d] = sum over samples and pairs of the records' D_x (h=0), D_y (h=1).
__global__ void k_buckets(ShapeDev sh) {
    const int L = sh.L, S = 64 * sh.W, P = sh.P, rl = 2 * L + 3;
    const int n = sh.nk * 2 * L;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int i = e / (2 * L), hd = e % (2 * L);
        long long acc = 0;
        for (int s = 0; s < S; ++s)
            for (int p = 0; p < P; ++p) acc += sh.rec[((size_t)(i * S + s) * P + p) * rl + hd];
        sh.buckets[e] = acc;
    }
}

size_t gram_lds(int RR, int L) {
    const int PP = RR * (RR - 1) / 2;
    const int nxp = 64 * ((L * L + 63) / 64);
    return (size_t)2 * PP * 2 * L * 8 + (size_t)RR * nxp * 4;
}
// Launch groups GI .. of RR replicas, one launch each.
template <int RR, int GI>
hipError_t launch_overlap(const ShapeDev& sh, int cfg0, int ncfg, int grid, int wc, int nxcd, hipStream_t st) {
    constexpr PairGroups<RR> grp{};
    constexpr int n = grp.size[GI];
    hipLaunchKernelGGL((k_overlap_mfma<RR, GI, n>), dim3(grid), dim3(64 * kTeamWaves), 0, st, sh, cfg0, ncfg,
                       wc, nxcd);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (GI + 1 < grp.n) return launch_overlap<RR, GI + 1>(sh, cfg0, ncfg, grid, wc, nxcd, st);
    return hipSuccess;
}

template <int RR>
hipError_t launch_mfma(const ShapeDev& sh, int cfg0, int ncfg, hipStream_t st) {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    // a wave holds every replica's G of its unit: 64 x 64 up to 4 replicas,
    // 64 x 32 above; with the int32 epilogue and more configurations than
    // CUs two waves share a SIMD, each with at most 128 accumulators (64 x 64
    // for 2 replicas, else 64 x 32)
    constexpr int NV = RR <= 4 ? 2 : 1;
    constexpr int NVn = RR <= 2 ? 2 : 1;
    static bool lds_set = false;
    if (!lds_set) {
        for (const void* f : {(const void*)k_gram_mfma<RR, NVn, true, true>, (const void*)k_gram_mfma<RR, NV, true, true>,
                              (const void*)k_gram_mfma<RR, NV, true, false>, (const void*)k_gram_mfma<RR, NV, false, false>}) {
            const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)gram_lds(RR, 32));
            if (e != hipSuccess) return e;
        }
        lds_set = true;
    }
    const int ggrid = std::min(ncfg, ncu);
    auto narrow = [&](auto nvC) {
        constexpr int nv = decltype(nvC)::value;
        hipLaunchKernelGGL((k_gram_mfma<RR, nv, true, true>), dim3(std::min(ncfg, gram_wpe(RR, nv, true) * ncu)),
                           dim3(64 * kGramWaves), gram_lds(RR, sh.L), st, sh, cfg0, ncfg);
    };
    if (sh.L % 8 == 0 && sh.Lt <= kNarrowLt && ncfg > ncu)
        narrow(std::integral_constant<int, NVn>{});
    else if (sh.L % 8 == 0 && sh.Lt <= kNarrowLt)
        narrow(std::integral_constant<int, NV>{});
    else if (sh.L % 8 == 0)
        hipLaunchKernelGGL((k_gram_mfma<RR, NV, true, false>), dim3(ggrid), dim3(64 * kGramWaves), gram_lds(RR, sh.L),
                           st, sh, cfg0, ncfg);
    else
        hipLaunchKernelGGL((k_gram_mfma<RR, NV, false, false>), dim3(ggrid), dim3(64 * kGramWaves),
                           gram_lds(RR, sh.L), st, sh, cfg0, ncfg);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // overlap: two workgroups of kTeamWaves waves per CU; teams of wc waves,
    // an XCD's share (a power-of-two fraction of it while a configuration
    // has fewer tiles, a multiple while there are fewer configurations than
    // teams)
    const int nxcd = ncu % 8 == 0 ? 8 : 1;
    const int G = kTeamWaves * 2 * ncu, gx = G / nxcd;
    const int ntt = (sh.Lt + 63) / 64, ntiles = ntt * ntt;
    int wc = gx;
    while (wc % 2 == 0 && wc / 2 >= ntiles) wc /= 2;
    auto fits = [&](int w) { return w <= gx ? gx % w == 0 : (w % gx == 0 && nxcd % (w / gx) == 0); };
    while (wc < G && G / wc > ncfg && fits(2 * wc)) wc *= 2;
    return launch_overlap<RR, 0>(sh, cfg0, ncfg, 2 * ncu, wc, nxcd, st);
}

}  // namespace

bool measure_ok(const ShapeDev& sh) { return sh.R >= 2 && sh.R <= kMaxR && sh.L <= 32; }


hipError_t launch_transpose(const ShapeDev& sh, hipStream_t st) {
    const long long items = (long long)sh.R * sh.nk * sh.W * sh.nc * sh.nx;
    const int grid = (int)std::min<long long>(items, 8192);
    static bool lds_set = false;  // above 64 KiB of LDS per workgroup
    if (!lds_set) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_transpose,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)kTransposeLds);
        if (e != hipSuccess) return e;
        lds_set = true;
    }
    hipLaunchKernelGGL(k_transpose, dim3(grid), dim3(256), kTransposeLds, st, sh, items);
    return hipGetLastError();
}

hipError_t launch_measure(const ShapeDev& sh, int mode, int cfg0, int ncfg, hipStream_t st) {
    if (ncfg <= 0) return hipSuccess;
    if (mode == 0) {
        switch (sh.R) {
            case 2: return launch_mfma<2>(sh, cfg0, ncfg, st);
            case 3: return launch_mfma<3>(sh, cfg0, ncfg, st);
            case 4: return launch_mfma<4>(sh, cfg0, ncfg, st);
            case 5: return launch_mfma<5>(sh, cfg0, ncfg, st);
            case 6: return launch_mfma<6>(sh, cfg0, ncfg, st);
            default: return hipErrorInvalidValue;
        }
    }
    for (int cfg = cfg0; cfg < cfg0 + ncfg; ++cfg) {
        const long long ng = (long long)sh.L2 * sh.L2, nq = (long long)sh.Lt * sh.Lt;
        hipLaunchKernelGGL(k_gram_plain, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, sh, cfg);
        hipLaunchKernelGGL(k_overlap_plain, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, sh, cfg);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_buckets(const ShapeDev& sh, hipStream_t st) {
    hipLaunchKernelGGL(k_buckets, dim3(16), dim3(256), 0, st, sh);
    return hipGetLastError();
}

hipError_t launch_dump(const ShapeDev& sh, int cfg, int a, int b, hipStream_t st) {
    hipLaunchKernelGGL(k_dump, dim3(1024), dim3(256), 0, st, sh, cfg, a, b);
    return hipGetLastError();
}

}  // namespace tfim
