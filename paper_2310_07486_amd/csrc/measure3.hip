// Three-replica records for chi^(3) and F^(3) on int8 MFMA.
//
// Paper: arXiv:2310.07486, Methods, "One-time observables" (chi^(r), F^(r)
// and the second-moment length xi^(r), here r = 3) with the independent
// replicas of "Simulation details".
//
// For configuration (k-index i, sample s) and replicas r = 0..R-1 with
// G^r = S^r S^rT (L^2 x L^2), the record of a replica triple a < b < c is
//   T_x[d] = sum_{carrier e in {a,b,c}, f < g the other two}
//            sum_{(x1 - y1) mod L = d} G^e_xy (G^f G^g)_yx     (T_y: x2 - y2)
// so that Tr[M^3] ~ sum_d T_x[d] and Tr[M-hat M^2] ~ sum_d T_x[d] cos(2 pi d/L)
// (the phase on the carrier's factor, averaged over the three choices).
//
// 1. k_gram_store computes G of every replica from the bit rows along tau
//    (the {0,1} algebra of the pair measurement) and writes G' = G/2 (exact:
//    every entry has the parity of Ltau, which is even), |G'| <= Ltau/2,
//    as two int8 digits G' = 64 h + l, h in [-16, 16], l in [-32, 31], to
//    the caller's workspace.  Sites are stored in 8 x 8 blocks, one 64-row
//    tile per block (zero rows and columns where L is not a multiple of 8),
//    in a slot order chosen so that the 16 outputs a lane holds in the
//    32x32 MFMA layout cover four values of y1 and four of y2.
// 2. k_triple_mfma forms P = G'^f G'^g = 4096 h^f h^g + 64 (h^f l^g + l^f h^g)
//    + l^f l^g with three exact int8 GEMMs on v_mfma_i32_32x32x32_i8 (the
//    middle one with K doubled), |P| <= L^2 (Ltau/2)^2 < 2^31.  Its epilogue
//    multiplies P_yx by G'^e_xy of each carrier e outside {f, g} and sums
//    each lane's 16 products into four x-buckets and four y-buckets of the
//    triple {e, f, g}.  A work item is one output tile of one configuration
//    with every replica pair unrolled, so these sums stay in registers
//    across the pairs and reach the LDS buckets once per tile.  With 5 or 6
//    replicas (10 or 20 triples) one launch per replica pair forms that
//    pair's product once and serves the 3 or 4 triples that contain it, one
//    carrier each.  Records are
//    scaled by 8 at the flush (G = 2 G').  Work items are handed out so that
//    the workgroups with the same blockIdx.x mod 8 (one XCD under round-robin
//    dispatch) share one configuration at a time.
#include <algorithm>

#include "tfim_internal.h"

namespace tfim {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kPitch = 80;  // bytes per 64-byte staged row in LDS (16-byte aligned)
constexpr int kMaxL = 32;
constexpr int kStage = 4 * 64 * kPitch;  // bytes of one staged chunk of the pair-product operands

// Slot rho in [0, 64) of a tile <-> offsets (d1, d2) in [0, 8)^2 within the
// 8 x 8 site block: rho = 32 (d2 >> 2) + 8 (d2 & 3) + 4 (d1 >> 2) + (d1 & 3).
// Output row 32 wx + 8 g + 4 h + j of the MFMA layout is then d1 = 4 h + j,
// d2 = 4 wx + g.
__device__ __forceinline__ int slot_d1(int rho) { return 4 * ((rho >> 2) & 1) + (rho & 3); }
__device__ __forceinline__ int slot_d2(int rho) { return 4 * (rho >> 5) + ((rho >> 3) & 3); }

__device__ __forceinline__ v4i lds_v4(const uint8_t* base) { return *(const v4i*)base; }

__device__ __forceinline__ int mod_l(int v, int L) {
    v %= L;
    return v < 0 ? v + L : v;
}

// ---------------------------------------------------------------------------
// G' of every replica into the workspace, digit planes [cl][r][plane][Np][Np].
// One workgroup per configuration: it counts the down spins of every site
// row into LDS, then its four waves share the tile pairs (X, Y), X <= Y,
// each wave alone, one per SIMD, every replica's G of its 64 x 64 tile (64 x
// 32 above 4 replicas) in the AGPRs, the {0,1} operands built in registers
// from the bit rows along tau.  A block is written where it stands (one byte
// per element) and, transposed, where its mirror stands (G is symmetric; four
// consecutive row slots per 32-bit store).  In a diagonal pair with both
// column blocks the block (1, 0) is not computed: the block (0, 1) writes it.
// ---------------------------------------------------------------------------
constexpr int kStoreWaves = 4;

template <int RR, int NV>
__global__ void __launch_bounds__(64 * kStoreWaves) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_gram_store(ShapeDev sh, int cfg0, int ncfg, int nb, int8_t* __restrict__ ws) {
    extern __shared__ int nS[];  // [RR][nxp] popcounts along tau
    const int L = sh.L, Lt = sh.Lt, nc = sh.nc, nxp = sh.nxp;
    const int nt = nb * nb, Np = 64 * nt;
    const size_t plane = (size_t)Np * Np;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i = lane & 31, h5 = lane >> 5, sh4 = 4 * h5;
    const int ntp = nt * (nt + 1) / 2;
    // site of slot rho of tile T, -1 on padding
    auto site = [&](int T, int rho) {
        const int x1 = 8 * (T % nb) + slot_d1(rho), x2 = 8 * (T / nb) + slot_d2(rho);
        return (x1 < L && x2 < L) ? x1 + L * x2 : -1;
    };
    for (int cl = blockIdx.x; cl < ncfg; cl += gridDim.x) {
        const uint64_t* const pt = sh.Pt + (size_t)(cfg0 + cl) * RR * nc * nxp;
        __syncthreads();  // the previous configuration's epilogues have read nS
        for (int e = tid; e < RR * nxp; e += 64 * kStoreWaves) {
            const int r = e / nxp, xy = e - r * nxp;
            int n = 0;
            for (int c = 0; c < nc; ++c) n += __popcll(pt[((size_t)r * nc + c) * nxp + xy]);
            nS[e] = n;
        }
        __syncthreads();
        for (int unit = wv; unit < ntp * (2 / NV); unit += kStoreWaves) {
            const int tp = NV == 2 ? unit : unit >> 1;
            const int v0 = NV == 2 ? 0 : (unit & 1);
            int X = 0, rem = tp;
            while (rem >= nt - X) { rem -= nt - X; ++X; }
            const int Y = X + rem;
            const int xa[2] = {site(X, i), site(X, 32 + i)};
            int xb[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) xb[v] = site(Y, 32 * (v0 + v) + i);
            // padding rows read site 0 and are zeroed in the epilogue
            const int sa[2] = {max(xa[0], 0), max(xa[1], 0)};
            int sb[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) sb[v] = max(xb[v], 0);
            v16i acc[RR][2][NV];
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < NV; ++v)
#pragma unroll
                        for (int q = 0; q < 16; ++q) acc[r][u][v][q] = 0;
            auto kloop = [&](auto diagC) {
                constexpr bool kDiag = decltype(diagC)::value;
                constexpr int NB = kDiag ? 0 : NV;
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
            // pair, each its own straight code
            auto finish = [&](auto diagC) {
            constexpr bool diag = decltype(diagC)::value;
            kloop(diagC);
            // G = Ltau - 2 (n_row + n_col) + 4 (B B^T), G' = G / 2 as two
            // digits G' = 64 h + l, zero on padding
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const int V = v0 + v;
                    if (diag && NV == 2 && u == 1 && V == 0) continue;
                    const int col = 32 * V + i;
                    const bool col_ok = xb[v] >= 0;
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        const size_t m = (size_t)cl * RR + r;
                        int8_t* ph = ws + (2 * m) * plane;
                        int8_t* pl = ph + plane;
                        const int nb_ = Lt - 2 * nS[r * nxp + sb[v]];
                        uint32_t hw[4] = {0u, 0u, 0u, 0u}, lw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            const int row = 32 * u + 8 * (q >> 2) + 4 * h5 + (q & 3);
                            const int xs = site(X, row);
                            const int G = nb_ - 2 * nS[r * nxp + max(xs, 0)] + 4 * acc[r][u][v][q];
                            const int gp = (col_ok && xs >= 0) ? (G >> 1) : 0;
                            const int hd = (gp + 32) >> 6;
                            const int ld = gp - 64 * hd;
                            hw[q >> 2] |= ((uint32_t)hd & 0xFFu) << (8 * (q & 3));
                            lw[q >> 2] |= ((uint32_t)ld & 0xFFu) << (8 * (q & 3));
                            if (!diag || (NV == 2 && u != V)) {  // the block itself, one byte per element
                                const size_t o = (size_t)(64 * X + row) * Np + 64 * Y + col;
                                ph[o] = (int8_t)hd;
                                pl[o] = (int8_t)ld;
                            }
                        }
                        // the mirror: row 64 Y + col, four consecutive row slots
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const size_t o = (size_t)(64 * Y + col) * Np + 64 * X + 32 * u + 8 * g + 4 * h5;
                            *(uint32_t*)(ph + o) = hw[g];
                            *(uint32_t*)(pl + o) = lw[g];
                        }
                    }
                }
            };
            if (X == Y)
                finish(std::true_type{});
            else
                finish(std::false_type{});
        }
    }
}

// ---------------------------------------------------------------------------
// Pair products and the carrier epilogue; records [cl][NT][2][L].
// ---------------------------------------------------------------------------
constexpr int pair_f(int R, int p) {
    int f = 0;
    while (p >= R - 1 - f) { p -= R - 1 - f; ++f; }
    return f;
}
constexpr int pair_g(int R, int p) {
    int f = 0;
    while (p >= R - 1 - f) { p -= R - 1 - f; ++f; }
    return f + 1 + p;
}
constexpr int carrier_of(int R, int f, int g, int ci) {
    int n = 0;
    for (int e = 0; e < R; ++e)
        if (e != f && e != g) {
            if (n == ci) return e;
            ++n;
        }
    return 0;
}
constexpr int triple_of(int R, int e, int f, int g) {  // index of the sorted triple {e, f, g}
    const int a = e < f ? e : f, c = e > g ? e : g, b = e + f + g - a - c;
    int t = 0;
    for (int i = 0; i < R; ++i)
        for (int j = i + 1; j < R; ++j)
            for (int k = j + 1; k < R; ++k) {
                if (i == a && j == b && k == c) return t;
                ++t;
            }
    return 0;
}

// Whether pair P has a carrier whose triple lies in [T0, T0 + NTG).
constexpr bool pair_needed(int R, int P, int T0, int NTG) {
    const int f = pair_f(R, P), g = pair_g(R, P);
    for (int ci = 0; ci < R - 2; ++ci) {
        const int t = triple_of(R, carrier_of(R, f, g, ci), f, g);
        if (t >= T0 && t < T0 + NTG) return true;
    }
    return false;
}

// Accumulator slot of carrier C of pair P in one launch.  The triple-group
// form (PM < 0) keeps the triples T0 .. T0 + NTG - 1 and forms every pair
// product they need; the pair-major form (PM >= 0) forms only the product of
// pair PM, once, with one slot per carrier (the triples that contain the
// pair).  -1: not in this launch.
constexpr int acc_slot(int R, int T0, int NTG, int PM, int P, int C) {
    if (PM >= 0) return P == PM ? C : -1;
    const int f = pair_f(R, P), g = pair_g(R, P);
    const int t = triple_of(R, carrier_of(R, f, g, C), f, g);
    return t >= T0 && t < T0 + NTG ? t - T0 : -1;
}
// The record triple of every slot of a launch.
template <int RR, int T0, int NTG, int PM>
struct SlotTriples {
    int t[NTG] = {};
    constexpr SlotTriples() {
        for (int s = 0; s < NTG; ++s) {
            if (PM < 0) {
                t[s] = T0 + s;
            } else {
                const int f = pair_f(RR, PM), g = pair_g(RR, PM);
                t[s] = triple_of(RR, carrier_of(RR, f, g, s), f, g);
            }
        }
    }
};

// Accumulators of the slots of one launch over one output tile.
template <int RR, int NTG>
struct TriAcc {
    long long tx[NTG][4], ty[NTG][4];  // x-buckets by j, y-buckets by g4
    uint32_t cw[RR][2][4];             // G'^e digits at (x = column slot, y = row slots)
};

struct TriGeom {
    const int8_t* base;
    size_t plane;
    int Np, nt, X, Y, tid, lane, wx, wy, h5;
    uint8_t* stg;
};

template <int RR, int T0, int NTG, int PM, int C, int P>
struct CarrierStep {
    static __device__ __forceinline__ void run(TriAcc<RR, NTG>& a, int q, int Pv) {
        constexpr int f = pair_f(RR, P), g = pair_g(RR, P);
        constexpr int e = carrier_of(RR, f, g, C);
        constexpr int sl = acc_slot(RR, T0, NTG, PM, P, C);
        if constexpr (sl >= 0) {
            const int j = q & 3, g4 = q >> 2;
            const int hb = (int)(int8_t)(a.cw[e][0][g4] >> (8 * j));
            const int lb = (int)(int8_t)(a.cw[e][1][g4] >> (8 * j));
            const long long v = (long long)(64 * hb + lb) * (long long)Pv;
            a.tx[sl][j] += v;
            a.ty[sl][g4] += v;
        }
        CarrierStep<RR, T0, NTG, PM, C + 1, P>::run(a, q, Pv);
    }
};
template <int RR, int T0, int NTG, int PM, int P>
struct CarrierStep<RR, T0, NTG, PM, RR - 2, P> {
    static __device__ __forceinline__ void run(TriAcc<RR, NTG>&, int, int) {}
};

template <int RR, int T0, int NTG, int PM, int P>
struct PairStep {
    static __device__ __forceinline__ void run(TriAcc<RR, NTG>& a, const TriGeom& G) {
        if constexpr (PM >= 0 ? P == PM : pair_needed(RR, P, T0, NTG)) product(a, G);
        PairStep<RR, T0, NTG, PM, P + 1>::run(a, G);
    }
    static __device__ __forceinline__ void product(TriAcc<RR, NTG>& a, const TriGeom& G) {
        constexpr int f = pair_f(RR, P), g = pair_g(RR, P);
        const int8_t* pf = G.base + (size_t)(2 * f) * G.plane;  // rows of tile Y
        const int8_t* pg = G.base + (size_t)(2 * g) * G.plane;  // rows of tile X
        const int srow = G.tid >> 2, spart = 16 * (G.tid & 3);
        const int8_t* src[4] = {pf + (size_t)(64 * G.Y + srow) * G.Np + spart,
                                pf + G.plane + (size_t)(64 * G.Y + srow) * G.Np + spart,
                                pg + (size_t)(64 * G.X + srow) * G.Np + spart,
                                pg + G.plane + (size_t)(64 * G.X + srow) * G.Np + spart};
        v16i hh, xx, ll;
#pragma unroll
        for (int q = 0; q < 16; ++q) hh[q] = xx[q] = ll[q] = 0;
        const int lane = G.lane;
        auto fetch = [&](int kc, v4i (&vn)[4]) {
#pragma unroll
            for (int k = 0; k < 4; ++k) vn[k] = *(const v4i*)(src[k] + 64 * kc);
        };
        // chunk kc through staging buffer kc & 1, the data of chunk kc + 2 in
        // flight meanwhile: a buffer was last read two chunks earlier, before
        // the barrier of the chunk in between; the barrier before the first
        // chunk orders this product after the previous one's reads
        auto stage = [&](int kc, v4i (&vn)[4]) {
            uint8_t* const sb = G.stg + (kc & 1) * kStage;
#pragma unroll
            for (int k = 0; k < 4; ++k) *(v4i*)(sb + (k * 64 + srow) * kPitch + spart) = vn[k];
            __syncthreads();
            fetch(min(kc + 2, G.nt - 1), vn);  // past the end: a reload, never used
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const int ko = 32 * ks + 16 * G.h5;
                const v4i ah = lds_v4(sb + (0 * 64 + 32 * G.wx + (lane & 31)) * kPitch + ko);
                const v4i al = lds_v4(sb + (1 * 64 + 32 * G.wx + (lane & 31)) * kPitch + ko);
                const v4i bh = lds_v4(sb + (2 * 64 + 32 * G.wy + (lane & 31)) * kPitch + ko);
                const v4i bl = lds_v4(sb + (3 * 64 + 32 * G.wy + (lane & 31)) * kPitch + ko);
                hh = __builtin_amdgcn_mfma_i32_32x32x32_i8(ah, bh, hh, 0, 0, 0);
                ll = __builtin_amdgcn_mfma_i32_32x32x32_i8(al, bl, ll, 0, 0, 0);
                xx = __builtin_amdgcn_mfma_i32_32x32x32_i8(ah, bl, xx, 0, 0, 0);
                xx = __builtin_amdgcn_mfma_i32_32x32x32_i8(al, bh, xx, 0, 0, 0);
            }
        };
        v4i v0[4], v1[4];
        fetch(0, v0);
        fetch(min(1, G.nt - 1), v1);
        __syncthreads();
        for (int kc = 0; kc + 1 < G.nt; kc += 2) {
            stage(kc, v0);
            stage(kc + 1, v1);
        }
        if (G.nt & 1) stage(G.nt - 1, v0);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int Pv = 4096 * hh[q] + 64 * xx[q] + ll[q];
            CarrierStep<RR, T0, NTG, PM, 0, P>::run(a, q, Pv);
        }
    }
};
template <int RR, int T0, int NTG, int PM>
struct PairStep<RR, T0, NTG, PM, RR * (RR - 1) / 2> {
    static __device__ __forceinline__ void run(TriAcc<RR, NTG>&, const TriGeom&) {}
};

// Records of the slots of one launch (triples in lexicographic order
// a < b < c): up to 4 replicas one launch takes every triple and forms the 6
// pair products; with 5 or 6, one launch per replica pair forms that pair's
// product once and adds it, times each carrier's G, into the records of the
// 3 or 4 triples that contain the pair (every pair product formed once, the
// int64 sums of a tile in registers).
template <int RR, int T0, int NTG, int PM>
__global__ void __launch_bounds__(256) k_triple_mfma(int L, int ncfg, int nb,
                                                     const int8_t* __restrict__ ws,
                                                     int64_t* __restrict__ rec) {
    constexpr int NT = RR * (RR - 1) * (RR - 2) / 6;
    constexpr SlotTriples<RR, T0, NTG, PM> stab{};
    __shared__ __align__(16) uint8_t stg[2 * kStage];  // twice: f high, f low, g high, g low
    __shared__ unsigned long long Tb[NTG * 2 * kMaxL];
    const int nt = nb * nb, Np = 64 * nt;
    const size_t plane = (size_t)Np * Np;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wx = wv & 1, wy = wv >> 1, h5 = lane >> 5;
    const int ipc = nt * nt;  // output tiles per configuration, all pairs each
    const int grp = blockIdx.x & 7, ngrp_blocks = (int)(gridDim.x >> 3), kk = (int)(blockIdx.x >> 3);
    const int ncg = grp < ncfg ? (ncfg - grp + 7) / 8 : 0;  // configurations grp, grp + 8, ...
    const int rl = NT * 2 * L, nl = NTG * 2 * L;  // record, the launch's slots
    // element e of the slot buckets -> its place in a configuration's record
    auto rec_at = [&](int e) {
        const int sl = e / (2 * L);
        int t = 0;
#pragma unroll
        for (int k = 0; k < NTG; ++k)
            if (k == sl) t = stab.t[k];
        return (size_t)t * 2 * L + (e - sl * 2 * L);
    };
    for (int e = tid; e < nl; e += 256) Tb[e] = 0;
    int cur = -1;
    for (long long s = kk; s < (long long)ncg * ipc; s += ngrp_blocks) {
        const int cfg = grp + 8 * (int)(s / ipc);
        const int it = (int)(s % ipc);
        if (cfg != cur) {  // uniform over the workgroup
            __syncthreads();
            if (cur >= 0)
                for (int e = tid; e < nl; e += 256) {
                    atomicAdd((unsigned long long*)&rec[(size_t)cur * rl + rec_at(e)], Tb[e] * 8ull);
                    Tb[e] = 0;
                }
            __syncthreads();
            cur = cfg;
        }
        const int Y = it / nt, X = it % nt;
        const int8_t* base = ws + (size_t)cfg * RR * 2 * plane;
        const int col = 32 * wy + (lane & 31);
        TriAcc<RR, NTG> a;
#pragma unroll
        for (int t = 0; t < NTG; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) a.tx[t][j] = a.ty[t][j] = 0;
#pragma unroll
        for (int e = 0; e < RR; ++e)
#pragma unroll
            for (int pl = 0; pl < 2; ++pl)
#pragma unroll
                for (int g4 = 0; g4 < 4; ++g4)
                    a.cw[e][pl][g4] = *(const uint32_t*)(base + (size_t)(2 * e + pl) * plane +
                                                         (size_t)(64 * X + col) * Np + 64 * Y + 32 * wx +
                                                         8 * g4 + 4 * h5);
        const TriGeom G{base, plane, Np, nt, X, Y, tid, lane, wx, wy, h5, stg};
        PairStep<RR, T0, NTG, PM, 0>::run(a, G);
        const int x1 = 8 * (X % nb) + slot_d1(col), x2 = 8 * (X / nb) + slot_d2(col);
        const int y1b = 8 * (Y % nb) + 4 * h5, y2b = 8 * (Y / nb) + 4 * wx;
#pragma unroll
        for (int t = 0; t < NTG; ++t) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                atomicAdd(&Tb[(t * 2 + 0) * L + mod_l(x1 - y1b - j, L)], (unsigned long long)a.tx[t][j]);
#pragma unroll
            for (int g4 = 0; g4 < 4; ++g4)
                atomicAdd(&Tb[(t * 2 + 1) * L + mod_l(x2 - y2b - g4, L)], (unsigned long long)a.ty[t][g4]);
        }
    }
    __syncthreads();
    if (cur >= 0)
        for (int e = tid; e < nl; e += 256)
            atomicAdd((unsigned long long*)&rec[(size_t)cur * rl + rec_at(e)], Tb[e] * 8ull);
}

// Up to 4 replicas: the triples T0 .. NT - 1 in launches of at most 4.
template <int RR, int T0>
hipError_t launch_triple_groups(int L, int ncfg, int nb, const int8_t* gw, int64_t* rec, int grid,
                                hipStream_t st) {
    constexpr int NT = RR * (RR - 1) * (RR - 2) / 6;
    constexpr int n = NT - T0 < 4 ? NT - T0 : 4;
    hipLaunchKernelGGL((k_triple_mfma<RR, T0, n, -1>), dim3(grid), dim3(256), 0, st, L, ncfg, nb, gw, rec);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (T0 + n < NT) return launch_triple_groups<RR, T0 + n>(L, ncfg, nb, gw, rec, grid, st);
    return hipSuccess;
}

// 5 or 6 replicas: one launch per replica pair P, P .. pairs - 1.
template <int RR, int P>
hipError_t launch_triple_pairs(int L, int ncfg, int nb, const int8_t* gw, int64_t* rec, int grid,
                               hipStream_t st) {
    constexpr int PP = RR * (RR - 1) / 2;
    hipLaunchKernelGGL((k_triple_mfma<RR, 0, RR - 2, P>), dim3(grid), dim3(256), 0, st, L, ncfg, nb, gw, rec);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (P + 1 < PP) return launch_triple_pairs<RR, P + 1>(L, ncfg, nb, gw, rec, grid, st);
    return hipSuccess;
}

// The records are sums of atomic adds: cleared first by a kernel (no memset
// node, so the launch sequence may be captured in a graph).
__global__ void k_zero_records(int64_t* __restrict__ rec, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        rec[i] = 0;
}

template <int RR>
hipError_t launch_triples_rr(const ShapeDev& sh, int cfg0, int ncfg, const TripleLayout& lay,
                             int64_t* rec, int8_t* gw, hipStream_t st) {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e;
    const size_t nrec = (size_t)ncfg * (RR * (RR - 1) * (RR - 2) / 6) * 2 * sh.L;
    hipLaunchKernelGGL(k_zero_records, dim3((unsigned)std::min<size_t>((nrec + 255) / 256, 1024)), dim3(256), 0,
                       st, rec, nrec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    constexpr int NV = RR <= 4 ? 2 : 1;
    const size_t lds = (size_t)RR * sh.nxp * 4;
    hipLaunchKernelGGL((k_gram_store<RR, NV>), dim3(std::min(ncfg, ncu)), dim3(64 * kStoreWaves), lds, st, sh, cfg0,
                       ncfg, lay.nb, gw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const long long ipc = (long long)lay.nt * lay.nt;
    const long long per_grp = std::max<long long>(1, (long long)((ncfg + 7) / 8) * ipc);
    const int g2 = 8 * (int)std::min<long long>(per_grp, (long long)(4 * ncu) / 8);
    if constexpr (RR >= 5) return launch_triple_pairs<RR, 0>(sh.L, ncfg, lay.nb, (const int8_t*)gw, rec, g2, st);
    else return launch_triple_groups<RR, 0>(sh.L, ncfg, lay.nb, (const int8_t*)gw, rec, g2, st);
}

}  // namespace

TripleLayout triple_layout(const ShapeDev& sh, int ncfg) {
    TripleLayout t;
    t.nb = (sh.L + 7) / 8;
    t.nt = t.nb * t.nb;
    t.Np = 64 * t.nt;
    const int NT = sh.R * (sh.R - 1) * (sh.R - 2) / 6;
    t.rec_bytes = ((size_t)ncfg * NT * 2 * sh.L * 8 + 255) & ~(size_t)255;
    t.g_bytes = (size_t)ncfg * sh.R * 2 * (size_t)t.Np * t.Np;
    return t;
}

const char* triples_unsupported(const ShapeDev& sh) {
    if (sh.R < 3 || sh.R > 6) return "three-replica records need 3 to 6 replicas";
    if (sh.L > kMaxL) return "three-replica records need L <= 32";
    // |G'^f G'^g| <= L^2 (Ltau/2)^2 must fit the int32 accumulators
    const unsigned long long half = (unsigned long long)sh.Lt / 2;
    if ((unsigned long long)sh.L2 * half * half >= (1ull << 31))
        return "L^2 (Ltau/2)^2 exceeds the int32 range of the pair products";
    // a record of three carriers, 3 L^6 Ltau^3, must fit int64
    const unsigned __int128 n = (unsigned)sh.L2, t = (unsigned)sh.Lt;
    if (3 * n * n * n * t * t * t >= ((unsigned __int128)1 << 63))
        return "3 L^6 Ltau^3 exceeds the int64 range of a record";
    return nullptr;
}

hipError_t launch_triples(const ShapeDev& sh, int cfg0, int ncfg, int64_t* rec, int8_t* gw, hipStream_t st) {
    if (ncfg <= 0) return hipSuccess;
    const TripleLayout lay = triple_layout(sh, ncfg);
    switch (sh.R) {
        case 3: return launch_triples_rr<3>(sh, cfg0, ncfg, lay, rec, gw, st);
        case 4: return launch_triples_rr<4>(sh, cfg0, ncfg, lay, rec, gw, st);
        case 5: return launch_triples_rr<5>(sh, cfg0, ncfg, lay, rec, gw, st);
        case 6: return launch_triples_rr<6>(sh, cfg0, ncfg, lay, rec, gw, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tfim
