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
//    LDS, flushed once per configuration.
// 3. k_overlap_mfma: 64x64 tiles of every Q^ab, all pairs at once for up to
//    4 replicas (5 or 6: one launch per group of 5 pairs); per-lane int64
//    sums flushed once per configuration.
// The plain per-sample form (k_*_plain) computes one matrix element per
// thread with an int32 multiply-accumulate loop over unpacked spins, one
// launch per configuration: the reference point for the batched form.
#include <algorithm>

#include "tfim_internal.h"

namespace tfim {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kRowPitch = 80;  // bytes per unpacked 64-element row in LDS (16-byte aligned)
constexpr int kMaxR = 6;       // replicas handled by the MFMA kernels
constexpr int kMaxP = kMaxR * (kMaxR - 1) / 2;

constexpr int kTP = 65;  // padded row pitch (words) of the transpose tiles
constexpr size_t kTransposeLds = (size_t)2 * 64 * kTP * 8 + 64 * 4;

__global__ void __launch_bounds__(256) k_transpose(ShapeDev sh, long long items) {
    extern __shared__ uint64_t tlds[];
    uint64_t(*tile)[kTP] = (uint64_t(*)[kTP])tlds;
    uint64_t(*outw)[kTP] = (uint64_t(*)[kTP])(tlds + 64 * kTP);
    int* mrow = (int*)(tlds + 2 * 64 * kTP);
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
        for (int e = tid; e < 4096; e += 256) {
            const int t = e >> 6, u = e & 63, tau = 64 * c + t, xy = 64 * g + u;
            tile[t][u] = (tau < Lt && xy < L2) ? sh.S[((size_t)cfg * Lt + tau) * L2 + xy] : 0ull;
        }
        __syncthreads();
        // bits along tau: column u of the tile, lanes = tau
        for (int uu = 0; uu < 16; ++uu) {
            const int u = wv * 16 + uu;
            outw[lane][u] = wave_transpose64(tile[lane][u]);  // lane = sample bit b
        }
        __syncthreads();
        for (int e = tid; e < 4096; e += 256) {
            const int b = e >> 6, u = e & 63;
            sh.Pt[((size_t)mrow[b] * sh.nc + c) * sh.nxp + 64 * g + u] = outw[b][u];
        }
        __syncthreads();
        // bits along xy: row t of the tile, lanes = xy
        for (int tt = 0; tt < 16; ++tt) {
            const int t = wv * 16 + tt;
            outw[lane][t] = wave_transpose64(tile[t][lane]);
        }
        __syncthreads();
        for (int e = tid; e < 4096; e += 256) {
            const int b = e >> 6, t = e & 63, tau = 64 * c + t;
            if (tau < Lt) sh.Px[((size_t)mrow[b] * sh.nx + g) * Lt + tau] = outw[b][t];
        }
    }
}

// 64 bits -> 64 bytes in {0,1} (byte t = bit t), written as four 16-byte stores.
__device__ __forceinline__ void unpack64(uint64_t v, uint8_t* dst) {
    uint32_t out[16];
#pragma unroll
    for (int d = 0; d < 16; ++d) {
        const uint32_t nib = (uint32_t)(v >> (4 * d)) & 0xFu;
        out[d] = __umul24(nib, 0x00204081u) & 0x01010101u;
    }
    v4i* p = (v4i*)dst;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v4i x;
        x[0] = (int)out[4 * q]; x[1] = (int)out[4 * q + 1];
        x[2] = (int)out[4 * q + 2]; x[3] = (int)out[4 * q + 3];
        p[q] = x;
    }
}

__device__ __forceinline__ uint64_t low_bits(int n) {
    return n >= 64 ? ~0ull : (n <= 0 ? 0ull : ((1ull << n) - 1ull));
}

__device__ __forceinline__ v4i lds_v4(const uint8_t* base) { return *(const v4i*)base; }

// ---------------------------------------------------------------------------
// G tiles and the D buckets.
// ---------------------------------------------------------------------------
template <int RR>
__global__ void __launch_bounds__(256) k_gram_mfma(ShapeDev sh, int cfg0, int ncfg) {
    constexpr int PP = RR * (RR - 1) / 2;
    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t* Al = smem;                                   // [RR][64][kRowPitch]
    uint8_t* Bl = smem + RR * 64 * kRowPitch;             // [RR][64][kRowPitch]
    int* nA = (int*)(Bl + RR * 64 * kRowPitch);           // [RR][64]
    int* nB = nA + RR * 64;                               // [RR][64]
    unsigned long long* Dblk = (unsigned long long*)(nB + RR * 64);  // [PP][2][L]
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wx = wv & 1, wy = wv >> 1;
    const int ntile = sh.nx;
    const int ntp = ntile * (ntile + 1) / 2;
    for (int e = tid; e < PP * 2 * L; e += 256) Dblk[e] = 0;
    for (int cfg = cfg0 + blockIdx.x; cfg < cfg0 + ncfg; cfg += gridDim.x) {
        for (int tp = 0; tp < ntp; ++tp) {
            // tile pair (X, Y), X <= Y, in row-major order of the upper triangle
            int X = 0, rem = tp;
            while (rem >= ntile - X) { rem -= ntile - X; ++X; }
            const int Y = X + rem;
            const bool diag = X == Y;
            const uint8_t* Bsrc = diag ? Al : Bl;
            const int* nBsrc = diag ? nA : nB;
            v16i acc[RR];
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[r][q] = 0;
            __syncthreads();  // previous tile's epilogue has read nA, nB
            for (int e = tid; e < 2 * RR * 64; e += 256) nA[e] = 0;  // nA and nB
            for (int c = 0; c < sh.nc; ++c) {
                __syncthreads();
                const uint64_t vm = low_bits(Lt - 64 * c);
                for (int e = tid; e < (diag ? 1 : 2) * RR * 64; e += 256) {
                    const int side = e / (RR * 64), rr = (e / 64) % RR, row = e & 63;
                    const int xy0 = 64 * (side ? Y : X);
                    const size_t m = (size_t)cfg * RR + rr;
                    const uint64_t v = sh.Pt[(m * sh.nc + c) * sh.nxp + xy0 + row] & vm;
                    (side ? nB : nA)[rr * 64 + row] += __popcll(v);
                    unpack64(v, (side ? Bl : Al) + (rr * 64 + row) * kRowPitch);
                }
                __syncthreads();
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int ko = 32 * ks + 16 * (lane >> 5);
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        const v4i a = lds_v4(Al + (r * 64 + 32 * wx + (lane & 31)) * kRowPitch + ko);
                        const v4i b = lds_v4(Bsrc + (r * 64 + 32 * wy + (lane & 31)) * kRowPitch + ko);
                        acc[r] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[r], 0, 0, 0);
                    }
                }
            }
            __syncthreads();  // popcounts complete
            const int col = 32 * wy + (lane & 31);
            const int y = 64 * Y + col;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int row = 32 * wx + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                const int x = 64 * X + row;
                if (x >= L2 || y >= L2) continue;
                long long G[RR];
#pragma unroll
                for (int r = 0; r < RR; ++r)
                    G[r] = (long long)Lt - 2ll * (nA[r * 64 + row] + nBsrc[r * 64 + col]) +
                           4ll * acc[r][q];
                const int x1 = x % L, x2 = x / L, y1 = y % L, y2 = y / L;
                const int dx = (x1 - y1 + L) % L, dy = (x2 - y2 + L) % L;
                int p = 0;
#pragma unroll
                for (int a = 0; a < RR; ++a)
#pragma unroll
                    for (int b = a + 1; b < RR; ++b, ++p) {
                        const unsigned long long h = (unsigned long long)(G[a] * G[b]);
                        atomicAdd(&Dblk[(p * 2 + 0) * L + dx], h);
                        atomicAdd(&Dblk[(p * 2 + 1) * L + dy], h);
                        if (!diag) {  // the mirror element (y, x)
                            atomicAdd(&Dblk[(p * 2 + 0) * L + (L - dx) % L], h);
                            atomicAdd(&Dblk[(p * 2 + 1) * L + (L - dy) % L], h);
                        }
                    }
            }
        }
        __syncthreads();
        const int rl = 2 * L + 3;
        for (int e = tid; e < PP * 2 * L; e += 256) {
            const int p = e / (2 * L), d = e % (2 * L);
            atomicAdd((unsigned long long*)&sh.rec[((size_t)cfg * PP + p) * rl + d], Dblk[e]);
            Dblk[e] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Q tiles: trQ, sum Q^2, sum Q^4 for the pairs P0 .. P0 + NP - 1 (pairs a < b
// in lexicographic order).  Up to 4 replicas one launch takes every pair;
// with 5 or 6 one launch per group of 5 pairs keeps the accumulators of a
// tile (16 per pair and lane) within the register budget.
// ---------------------------------------------------------------------------
template <int RR, int P0, int NP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_overlap_mfma(ShapeDev sh, int cfg0, int ncfg) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t* Al = smem;
    uint8_t* Bl = smem + RR * 64 * kRowPitch;
    int* mA = (int*)(Bl + RR * 64 * kRowPitch);
    int* mB = mA + RR * 64;
    unsigned long long* red = (unsigned long long*)(mB + RR * 64);  // [NP][2]: trQ, sum Q^4
    const int L2 = sh.L2, Lt = sh.Lt;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wx = wv & 1, wy = wv >> 1;
    const int ntt = (Lt + 63) / 64;
    constexpr int kRows = 2 * RR * 64;        // operand rows of one K chunk (A and B)
    constexpr int kPer = (kRows + 255) / 256;  // rows per thread
    for (int e = tid; e < NP * 2; e += 256) red[e] = 0;
    for (int cfg = cfg0 + blockIdx.x; cfg < cfg0 + ncfg; cfg += gridDim.x) {
        unsigned long long s4u[NP];
        long long tr[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            s4u[p] = 0;
            tr[p] = 0;
        }
        for (int tt = 0; tt < ntt * ntt; ++tt) {
            const int T = tt / ntt, T2 = tt % ntt;
            const bool diag = T == T2;
            const uint8_t* Bsrc = diag ? Al : Bl;
            const int* mBsrc = diag ? mA : mB;
            const int nrows = (diag ? 1 : 2) * RR * 64;
            // operand rows of K chunk g: side (A: tile T, B: tile T2), replica, tau
            auto fetch = [&](int g, uint64_t (&v)[kPer]) {
                const uint64_t vm = low_bits(L2 - 64 * g);
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const int e = tid + 256 * k;
                    v[k] = 0;
                    if (e < nrows) {
                        const int side = e / (RR * 64), rr = (e / 64) % RR, row = e & 63;
                        const int tau = 64 * (side ? T2 : T) + row;
                        const size_t m = (size_t)cfg * RR + rr;
                        v[k] = tau < Lt ? (sh.Px[(m * sh.nx + g) * Lt + tau] & vm) : 0ull;
                    }
                }
            };
            v16i acc[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[p][q] = 0;
            uint64_t vn[kPer];
            fetch(0, vn);
            __syncthreads();  // previous tile's epilogue has read mA, mB
            for (int e = tid; e < 2 * RR * 64; e += 256) mA[e] = 0;
            for (int g = 0; g < sh.nx; ++g) {
                __syncthreads();
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const int e = tid + 256 * k;
                    if (e < nrows) {
                        const int side = e / (RR * 64), rr = (e / 64) % RR, row = e & 63;
                        (side ? mB : mA)[rr * 64 + row] += __popcll(vn[k]);
                        unpack64(vn[k], (side ? Bl : Al) + (rr * 64 + row) * kRowPitch);
                    }
                }
                __syncthreads();
                if (g + 1 < sh.nx) fetch(g + 1, vn);  // in flight during the MFMAs
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int ko = 32 * ks + 16 * (lane >> 5);
                    v4i a[RR - 1], b[RR - 1];
#pragma unroll
                    for (int r = 0; r < RR - 1; ++r) {
                        a[r] = lds_v4(Al + (r * 64 + 32 * wx + (lane & 31)) * kRowPitch + ko);
                        b[r] = lds_v4(Bsrc + ((r + 1) * 64 + 32 * wy + (lane & 31)) * kRowPitch + ko);
                    }
                    int p = 0;
#pragma unroll
                    for (int ra = 0; ra < RR; ++ra)
#pragma unroll
                        for (int rb = ra + 1; rb < RR; ++rb, ++p)
                            if (p >= P0 && p < P0 + NP)
                                acc[p - P0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[ra], b[rb - 1],
                                                                                    acc[p - P0], 0, 0, 0);
                }
            }
            __syncthreads();
            // epilogue: Q = L^2 - 2 (m_tau + m_tau') + 4 B^aT B^b; |Q| <= L^2,
            // Q^2 < 2^19, Q^4 < 2^38
            const int col = 32 * wy + (lane & 31);
            const int tau2 = 64 * T2 + col;
            int cc[RR];
#pragma unroll
            for (int rb = 0; rb < RR; ++rb) cc[rb] = -2 * mBsrc[rb * 64 + col];
            if (!diag && 64 * (T + 1) <= Lt && 64 * (T2 + 1) <= Lt) {
                // interior off-diagonal tile: no bounds, no trace; Q^4 summed
                // unsigned, one 32x32->64 multiply-add per element and pair
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int row = 32 * wx + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                    int cr[RR];
#pragma unroll
                    for (int ra = 0; ra < RR; ++ra) cr[ra] = L2 - 2 * mA[ra * 64 + row];
                    int p = 0;
#pragma unroll
                    for (int ra = 0; ra < RR; ++ra)
#pragma unroll
                        for (int rb = ra + 1; rb < RR; ++rb, ++p) {
                            if (p < P0 || p >= P0 + NP) continue;
                            const int qv = cr[ra] + cc[rb] + 4 * acc[p - P0][q];
                            const uint32_t q2 = (uint32_t)(qv * qv);
                            s4u[p - P0] += (unsigned long long)q2 * q2;
                        }
                }
            } else {
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int row = 32 * wx + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                    const int tau = 64 * T + row;
                    if (tau >= Lt || tau2 >= Lt) continue;
                    int cr[RR];
#pragma unroll
                    for (int ra = 0; ra < RR; ++ra) cr[ra] = L2 - 2 * mA[ra * 64 + row];
                    int p = 0;
#pragma unroll
                    for (int ra = 0; ra < RR; ++ra)
#pragma unroll
                        for (int rb = ra + 1; rb < RR; ++rb, ++p) {
                            if (p < P0 || p >= P0 + NP) continue;
                            const int qv = cr[ra] + cc[rb] + 4 * acc[p - P0][q];
                            const uint32_t q2 = (uint32_t)__mul24(qv, qv);
                            s4u[p - P0] += (unsigned long long)q2 * q2;
                            if (diag && tau == tau2) tr[p - P0] += qv;
                        }
                }
            }
        }
        // per-configuration flush: wave reduction, then one atomic per value
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                s4u[p] += (unsigned long long)__shfl_xor((long long)s4u[p], off, 64);
                tr[p] += __shfl_xor(tr[p], off, 64);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                atomicAdd(&red[p * 2 + 0], (unsigned long long)tr[p]);
                atomicAdd(&red[p * 2 + 1], s4u[p]);
            }
        }
        __syncthreads();
        // sum Q^2 = sum_xy G^a_xy G^b_xy = sum_d D_x[d]: the Gram kernel's
        // buckets of this configuration are complete (earlier launch)
        const int rl = 2 * sh.L + 3;
        constexpr int PP = RR * (RR - 1) / 2;
        for (int e = tid; e < NP * 3; e += 256) {
            const int p = e / 3, k = e % 3;
            int64_t* rp = sh.rec + ((size_t)cfg * PP + P0 + p) * rl;
            if (k == 1) {
                int64_t q2 = 0;
                for (int d = 0; d < sh.L; ++d) q2 += rp[d];
                rp[2 * sh.L + 1] = q2;
            } else {
                rp[2 * sh.L + k] = (int64_t)red[p * 2 + (k == 0 ? 0 : 1)];
            }
        }
        __syncthreads();
        for (int e = tid; e < NP * 2; e += 256) red[e] = 0;
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
    return (size_t)2 * RR * 64 * kRowPitch + (size_t)2 * RR * 64 * 4 + (size_t)PP * 2 * L * 8;
}
size_t overlap_lds(int RR, int NP) {
    return (size_t)2 * RR * 64 * kRowPitch + (size_t)2 * RR * 64 * 4 + (size_t)NP * 2 * 8;
}

// Pairs P0 .. PP - 1 of RR replicas in launches of at most NP pairs.
template <int RR, int P0, int NP>
hipError_t launch_overlap(const ShapeDev& sh, int cfg0, int ncfg, int grid, hipStream_t st) {
    constexpr int PP = RR * (RR - 1) / 2;
    constexpr int n = PP - P0 < NP ? PP - P0 : NP;
    hipLaunchKernelGGL((k_overlap_mfma<RR, P0, n>), dim3(grid), dim3(256), overlap_lds(RR, n), st, sh, cfg0,
                       ncfg);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (P0 + n < PP) return launch_overlap<RR, P0 + n, NP>(sh, cfg0, ncfg, grid, st);
    return hipSuccess;
}

template <int RR>
hipError_t launch_mfma(const ShapeDev& sh, int cfg0, int ncfg, hipStream_t st) {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int grid = std::min(ncfg, 4 * ncu);
    static bool lds_set = false;  // 6 replicas at L = 32 take above 64 KiB
    if (!lds_set) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_gram_mfma<RR>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)gram_lds(RR, 32));
        if (e != hipSuccess) return e;
        lds_set = true;
    }
    hipLaunchKernelGGL(k_gram_mfma<RR>, dim3(grid), dim3(256), gram_lds(RR, sh.L), st, sh, cfg0, ncfg);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_overlap<RR, 0, (RR <= 4 ? RR * (RR - 1) / 2 : 5)>(sh, cfg0, ncfg, grid, st);
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
