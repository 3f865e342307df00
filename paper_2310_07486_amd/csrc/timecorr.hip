// Two-time correlations on int8 MFMA.
//
// Paper: arXiv:2310.07486, Methods, "Two-times observables": C_A(tau) is the
// average over tau1 of A(S_tau1) A(S_tau1+tau) along the periodic time
// direction, for A = sigma^Z_x summed over sites (C(tau)) and for
// A = sigma^Z_x sigma^Z_y summed over site pairs (Q2(tau)).
//
// Both come from the time Gram of one replica, H = S^T S (Ltau x Ltau,
// H_t1t2 = sum_x S_x,t1 S_x,t2, |H| <= L^2):
//   c[d]  = sum_t1 H_t1,(t1+d) mod Ltau,   q2[d] = sum_t1 H_t1,(t1+d) mod Ltau ^ 2,
// summed over the replicas of the configuration.  With B = (1 - S)/2,
// H = L^2 - 2 (m_t1 + m_t2) + 4 (B^T B), so the contraction over sites runs on
// int8 operands (v_mfma_i32_32x32x32_i8) built in registers from the bit
// rows along xy, as in the replica overlap, with the rank-one corrections in
// one more K step so that the accumulator is H itself.
//
// One workgroup takes one configuration at a time; its four waves share the
// upper triangle of 64 x 64 tiles (each wave alone, no barrier inside a
// configuration) and take the replicas two at a time.  Each element with
// t1 <= t2 adds sum_r H^r and sum_r (H^r)^2 to the LDS buckets U of its
// diagonal d = t2 - t1: for element q of a 32 x 32 block all lanes of a
// half-wave sit at the same row offset r_q, so rotating the lanes by r_q
// (ds_bpermute) brings the elements of one diagonal into one lane, which
// sums them and adds two values per block (d >= 0 and d - 32) instead of
// one per element.  H is symmetric, so the record is
// c[d] = U[d] + U[Ltau - d] (c[0] = U[0]), stored once per configuration.
#include <algorithm>

#include "tfim_internal.h"

namespace tfim {
namespace {

typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kMaxLtTime = 4096;
constexpr int kTcWaves = 4;  // waves per workgroup

template <int RR>
__global__ void __launch_bounds__(64 * kTcWaves) __attribute__((amdgpu_waves_per_eu(2))) k_timecorr_mfma(ShapeDev sh, int cfg0, int ncfg,
                                                                int64_t* __restrict__ rec) {
    extern __shared__ unsigned long long Cb[];  // [2][Lt]: c, q2
    const int L2 = sh.L2, Lt = sh.Lt, nx = sh.nx;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i = lane & 31, h = lane >> 5, sh4 = 4 * h;
    const int ntt = (Lt + 63) / 64;
    const int ntp = ntt * (ntt + 1) / 2;
    const int h2 = L2 >> 1;
    for (int e = tid; e < 2 * Lt; e += 64 * kTcWaves) Cb[e] = 0;
    __syncthreads();
    for (int cl = blockIdx.x; cl < ncfg; cl += gridDim.x) {
        const uint64_t* const px = sh.Px + (size_t)(cfg0 + cl) * RR * nx * Lt;
        for (int tp = wv; tp < ntp; tp += kTcWaves) {
            int T = 0, rem = tp;
            while (rem >= ntt - T) { rem -= ntt - T; ++T; }
            const int T2 = T + rem;
            // rows clamped into [0, Lt): a row past Lt only feeds elements
            // the epilogue drops
            const int ta0 = 64 * T + i, tb0 = 64 * T2 + i;
            const int rowa[2] = {min(ta0, Lt - 1), min(ta0 + 32, Lt - 1)};
            const int rowb[2] = {min(tb0, Lt - 1), min(tb0 + 32, Lt - 1)};
            const bool edge = 64 * (T2 + 1) > Lt;  // T <= T2
#pragma unroll
            for (int r0 = 0; r0 < RR; r0 += 2) {
                constexpr int kG = 2;
                const int ng = min(kG, RR - r0);  // replicas of this group (uniform)
                auto fetch = [&](int g, uint64_t (&wa)[2][kG], uint64_t (&wb)[2][kG]) {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int a = 0; a < kG; ++a) {
                            const size_t m = (size_t)min(r0 + a, RR - 1) * nx + g;
                            wa[u][a] = px[m * Lt + rowa[u]];
                            wb[u][a] = px[m * Lt + rowb[u]];
                        }
                };
                v16i acc[kG][2][2];
#pragma unroll
                for (int a = 0; a < kG; ++a)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int v = 0; v < 2; ++v)
#pragma unroll
                            for (int q = 0; q < 16; ++q) acc[a][u][v][q] = 0;
                int ma[2][kG], mb[2][kG];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int a = 0; a < kG; ++a) ma[u][a] = mb[u][a] = 0;
                auto chunk = [&](const uint64_t (&wa)[2][kG], const uint64_t (&wb)[2][kG]) {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int a = 0; a < kG; ++a) {
                            ma[u][a] += __popcll(wa[u][a]);
                            mb[u][a] += __popcll(wb[u][a]);
                        }
#pragma unroll
                    for (int ks = 0; ks < 2; ++ks) {
                        i32x4 A[2][kG], B[2][kG];
#pragma unroll
                        for (int u = 0; u < 2; ++u)
#pragma unroll
                            for (int a = 0; a < kG; ++a) {
                                A[u][a] = mfma_bits_operand<true>((uint32_t)(wa[u][a] >> (32 * ks)) >> sh4);
                                B[u][a] = mfma_bits_operand<false>((uint32_t)(wb[u][a] >> (32 * ks)) >> sh4);
                            }
#pragma unroll
                        for (int a = 0; a < kG; ++a)
#pragma unroll
                            for (int u = 0; u < 2; ++u)
#pragma unroll
                                for (int v = 0; v < 2; ++v)
                                    acc[a][u][v] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[u][a], B[v][a],
                                                                                         acc[a][u][v], 0, 0, 0);
                    }
                };
                // two word sets in turn, the next chunk in flight during this
                // one; one straight loop block (a fetch past the last chunk
                // reloads it) keeps the loads ahead and the waits exact
                uint64_t w0a[2][kG], w0b[2][kG], w1a[2][kG], w1b[2][kG];
                fetch(0, w0a, w0b);
                for (int g = 0; g + 1 < nx; g += 2) {
                    fetch(g + 1, w1a, w1b);
                    chunk(w0a, w0b);
                    fetch(min(g + 2, nx - 1), w0a, w0b);
                    chunk(w1a, w1b);
                }
                if (nx & 1) chunk(w0a, w0b);
                {  // H = 4 B^T B + X_t1 + Y_t2, X = h2 - 2 m_t1, Y = L^2 - h2 - 2 m_t2
                    const i32x4 ones = {0x01010101, 0x01010101, 0x01010101, 0x01010101};
                    i32x4 A[2][kG], B[2][kG];
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int a = 0; a < kG; ++a) {
                            A[u][a] = h ? ones : mfma_pieces16(h2 - 2 * ma[u][a]);
                            B[u][a] = h ? mfma_pieces16(L2 - h2 - 2 * mb[u][a]) : ones;
                        }
#pragma unroll
                    for (int a = 0; a < kG; ++a)
#pragma unroll
                        for (int u = 0; u < 2; ++u)
#pragma unroll
                            for (int v = 0; v < 2; ++v)
                                acc[a][u][v] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[u][a], B[v][a],
                                                                                     acc[a][u][v], 0, 0, 0);
                }
                // epilogue: lane l gathers, for each q, the element of column
                // (l + r_q) mod 32, which lies on diagonal l (or l - 32).
                // kEdge: a tile that reaches past Ltau drops those elements
                // (compiled apart, so the other tiles test nothing per
                // element).
                auto epilogue = [&](auto edgeC) {
                    constexpr bool kEdge = decltype(edgeC)::value;
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int v = 0; v < 2; ++v) {
                            const int D0 = 64 * (T2 - T) + 32 * (v - u);
                            if (D0 + 31 < 0) continue;  // below the diagonal
                            const int tau2 = 64 * T2 + 32 * v + i;
                            // all of a lane's gathered values, and those of
                            // diagonal l - 32 (i + r_q >= 32) apart
                            int sA = 0, sN = 0, qA = 0, qN = 0;
#pragma unroll
                            for (int q = 0; q < 16; ++q) {
                                const int r = 8 * (q >> 2) + 4 * h + (q & 3);
                                int hs = 0, hq = 0;  // |H| <= L^2: a group's sums stay below 2^21
#pragma unroll
                                for (int a = 0; a < kG; ++a) {
                                    if (a >= ng) continue;
                                    const int Hv = acc[a][u][v][q];
                                    hs += Hv;
                                    hq += __mul24(Hv, Hv);
                                }
                                if constexpr (kEdge) {
                                    const bool out = 64 * T + 32 * u + r >= Lt || tau2 >= Lt;
                                    hs = out ? 0 : hs;
                                    hq = out ? 0 : hq;
                                }
                                const int src = ((lane & 32) | ((lane + r) & 31)) << 2;
                                const int gs = __builtin_amdgcn_ds_bpermute(src, hs);
                                const int gq = __builtin_amdgcn_ds_bpermute(src, hq);
                                const bool neg = i + r >= 32;
                                sA += gs;
                                qA += gq;
                                sN += neg ? gs : 0;
                                qN += neg ? gq : 0;
                            }
                            const int sP = sA - sN, qP = qA - qN;
                            const int dP = D0 + i, dN = D0 + i - 32;
                            if (dP >= 0 && dP < Lt) {
                                atomicAdd(&Cb[dP], (unsigned long long)(long long)sP);
                                atomicAdd(&Cb[Lt + dP], (unsigned long long)qP);
                            }
                            if (dN >= 0 && dN < Lt) {
                                atomicAdd(&Cb[dN], (unsigned long long)(long long)sN);
                                atomicAdd(&Cb[Lt + dN], (unsigned long long)qN);
                            }
                        }
                };
                if (edge)
                    epilogue(std::true_type{});
                else
                    epilogue(std::false_type{});
            }
        }
        __syncthreads();
        // c[d] = U[d] + U[Ltau - d] for d > 0, c[0] = U[0] (likewise q2).  The
        // terms of U[Ltau - d] cross the tau wrap: with an antiperiodic
        // boundary they enter c with the sign -1 (q2 squares the sign away).
        const bool anti = sh.apm != 0ull;
        for (int e = tid; e < 2 * Lt; e += 64 * kTcWaves) {
            const int hh = e / Lt, d = e % Lt;
            const unsigned long long w = d ? Cb[hh * Lt + Lt - d] : 0ull;
            const unsigned long long uu = (anti && hh == 0) ? Cb[e] - w : Cb[e] + w;
            rec[(size_t)cl * 2 * Lt + e] = (int64_t)uu;
        }
        __syncthreads();
        for (int e = tid; e < 2 * Lt; e += 64 * kTcWaves) Cb[e] = 0;
        __syncthreads();
    }
}

size_t timecorr_lds(int Lt) { return (size_t)2 * Lt * 8; }

template <int RR>
hipError_t launch_timecorr_rr(const ShapeDev& sh, int cfg0, int ncfg, int64_t* rec, hipStream_t st) {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t lds = timecorr_lds(sh.Lt);
    static bool lds_set = false;  // above 64 KiB of LDS per workgroup
    if (!lds_set) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_timecorr_mfma<RR>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)timecorr_lds(kMaxLtTime));
        if (e != hipSuccess) return e;
        lds_set = true;
    }
    const int grid = std::min(ncfg, 2 * ncu);
    hipLaunchKernelGGL(k_timecorr_mfma<RR>, dim3(grid), dim3(64 * kTcWaves), lds, st, sh, cfg0, ncfg, rec);
    return hipGetLastError();
}

}  // namespace

const char* timecorr_unsupported(const ShapeDev& sh) {
    if (sh.R < 1 || sh.R > 6) return "two-time records need 1 to 6 replicas";
    if (sh.L > 32) return "two-time records need L <= 32";
    if (sh.Lt > kMaxLtTime) return "two-time records need Ltau <= 4096";
    return nullptr;
}

size_t timecorr_record_bytes(const ShapeDev& sh, int ncfg) { return (size_t)ncfg * 2 * sh.Lt * 8; }

hipError_t launch_timecorr(const ShapeDev& sh, int cfg0, int ncfg, int64_t* rec, hipStream_t st) {
    if (ncfg <= 0) return hipSuccess;
    switch (sh.R) {
        case 1: return launch_timecorr_rr<1>(sh, cfg0, ncfg, rec, st);
        case 2: return launch_timecorr_rr<2>(sh, cfg0, ncfg, rec, st);
        case 3: return launch_timecorr_rr<3>(sh, cfg0, ncfg, rec, st);
        case 4: return launch_timecorr_rr<4>(sh, cfg0, ncfg, rec, st);
        case 5: return launch_timecorr_rr<5>(sh, cfg0, ncfg, rec, st);
        case 6: return launch_timecorr_rr<6>(sh, cfg0, ncfg, rec, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tfim
