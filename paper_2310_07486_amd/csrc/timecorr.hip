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
// {0,1} int8 operands (v_mfma_i32_32x32x32_i8) unpacked from the bit rows
// along xy, as in the replica overlap.  One workgroup takes one
// configuration at a time and walks the upper triangle of 64 x 64 tiles of
// every replica's H; each element with t1 <= t2 adds sum_r H^r and
// sum_r (H^r)^2 to LDS buckets U of its diagonal d = t2 - t1, and since H is
// symmetric the record is c[d] = U[d] + U[Ltau - d] (c[0] = U[0]), stored
// once per configuration.
#include <algorithm>

#include "tfim_internal.h"

namespace tfim {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kPitch = 80;  // bytes per unpacked 64-element row in LDS
constexpr int kMaxLtTime = 4096;

__device__ __forceinline__ uint64_t low_bits(int n) {
    return n >= 64 ? ~0ull : (n <= 0 ? 0ull : ((1ull << n) - 1ull));
}

// 64 bits -> 64 bytes in {0,1} (byte t = bit t), four 16-byte stores.
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

__device__ __forceinline__ v4i lds_v4(const uint8_t* base) { return *(const v4i*)base; }

template <int RR>
__global__ void __launch_bounds__(256) k_timecorr_mfma(ShapeDev sh, int cfg0, int ncfg,
                                                       int64_t* __restrict__ rec) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t* Al = smem;                                   // [RR][64][kPitch]
    uint8_t* Bl = smem + RR * 64 * kPitch;                // [RR][64][kPitch]
    int* mA = (int*)(Bl + RR * 64 * kPitch);              // [RR][64] popcounts along xy
    int* mB = mA + RR * 64;                               // [RR][64]
    unsigned long long* Cb = (unsigned long long*)(mB + RR * 64);  // [2][Lt]: c, q2
    const int L2 = sh.L2, Lt = sh.Lt;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wx = wv & 1, wy = wv >> 1;
    const int ntt = (Lt + 63) / 64;
    const int ntp = ntt * (ntt + 1) / 2;
    constexpr int kPer = (2 * RR * 64 + 255) / 256;  // bit rows per thread and K chunk
    for (int e = tid; e < 2 * Lt; e += 256) Cb[e] = 0;
    for (int cl = blockIdx.x; cl < ncfg; cl += gridDim.x) {
        const size_t mbase = (size_t)(cfg0 + cl) * RR;
        for (int tp = 0; tp < ntp; ++tp) {
            int T = 0, rem = tp;
            while (rem >= ntt - T) { rem -= ntt - T; ++T; }
            const int T2 = T + rem;
            const bool diag = T == T2;
            const uint8_t* Bsrc = diag ? Al : Bl;
            const int* mBsrc = diag ? mA : mB;
            const int nrows = (diag ? 1 : 2) * RR * 64;
            uint64_t vn[kPer];
            auto fetch = [&](int g) {
                const uint64_t vm = low_bits(L2 - 64 * g);
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const int e = tid + 256 * k;
                    vn[k] = 0;
                    if (e < nrows) {
                        const int side = e / (RR * 64), rr = (e / 64) % RR, row = e & 63;
                        const int tau = 64 * (side ? T2 : T) + row;
                        if (tau < Lt) vn[k] = sh.Px[((mbase + rr) * sh.nx + g) * Lt + tau] & vm;
                    }
                }
            };
            v16i acc[RR];
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[r][q] = 0;
            fetch(0);
            __syncthreads();  // the previous tile's epilogue has read mA, mB
            for (int e = tid; e < 2 * RR * 64; e += 256) mA[e] = 0;  // mA and mB
            for (int g = 0; g < sh.nx; ++g) {
                __syncthreads();
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const int e = tid + 256 * k;
                    if (e < nrows) {
                        const int side = e / (RR * 64), rr = (e / 64) % RR, row = e & 63;
                        (side ? mB : mA)[rr * 64 + row] += __popcll(vn[k]);
                        unpack64(vn[k], (side ? Bl : Al) + (rr * 64 + row) * kPitch);
                    }
                }
                __syncthreads();
                if (g + 1 < sh.nx) fetch(g + 1);  // in flight during the MFMAs
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int ko = 32 * ks + 16 * (lane >> 5);
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        const v4i a = lds_v4(Al + (r * 64 + 32 * wx + (lane & 31)) * kPitch + ko);
                        const v4i b = lds_v4(Bsrc + (r * 64 + 32 * wy + (lane & 31)) * kPitch + ko);
                        acc[r] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[r], 0, 0, 0);
                    }
                }
            }
            __syncthreads();  // popcounts complete
            const int col = 32 * wy + (lane & 31);
            const int tau2 = 64 * T2 + col;
            int cc[RR];
#pragma unroll
            for (int r = 0; r < RR; ++r) cc[r] = L2 - 2 * mBsrc[r * 64 + col];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int row = 32 * wx + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                const int tau = 64 * T + row;
                if (tau >= Lt || tau2 >= Lt) continue;
                int hs = 0, h2 = 0;  // |H| <= L^2 <= 1024: sum of RR squares < 2^23
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    const int h = cc[r] - 2 * mA[r * 64 + row] + 4 * acc[r][q];
                    hs += h;
                    h2 += h * h;
                }
                // upper triangle only (tau <= tau2): the mirror element lands on
                // Ltau - d, added when the record is stored
                if (tau2 < tau) continue;
                const int d = tau2 - tau;
                atomicAdd(&Cb[d], (unsigned long long)(long long)hs);
                atomicAdd(&Cb[Lt + d], (unsigned long long)h2);
            }
        }
        __syncthreads();
        // c[d] = U[d] + U[Ltau - d] for d > 0, c[0] = U[0] (likewise q2).  The
        // terms of U[Ltau - d] cross the tau wrap: with an antiperiodic
        // boundary they enter c with the sign -1 (q2 squares the sign away).
        const bool anti = sh.apm != 0ull;
        for (int e = tid; e < 2 * Lt; e += 256) {
            const int h = e / Lt, d = e % Lt;
            const unsigned long long w = d ? Cb[h * Lt + Lt - d] : 0ull;
            const unsigned long long u = (anti && h == 0) ? Cb[e] - w : Cb[e] + w;
            rec[(size_t)cl * 2 * Lt + e] = (int64_t)u;
        }
        __syncthreads();
        for (int e = tid; e < 2 * Lt; e += 256) Cb[e] = 0;
        __syncthreads();
    }
}

size_t timecorr_lds(int RR, int Lt) {
    return (size_t)2 * RR * 64 * kPitch + (size_t)2 * RR * 64 * 4 + (size_t)2 * Lt * 8;
}

template <int RR>
hipError_t launch_timecorr_rr(const ShapeDev& sh, int cfg0, int ncfg, int64_t* rec, hipStream_t st) {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t lds = timecorr_lds(RR, sh.Lt);
    static bool lds_set = false;  // above 64 KiB of LDS per workgroup
    if (!lds_set) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_timecorr_mfma<RR>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)timecorr_lds(RR, kMaxLtTime));
        if (e != hipSuccess) return e;
        lds_set = true;
    }
    const int grid = std::min(ncfg, 4 * ncu);
    hipLaunchKernelGGL(k_timecorr_mfma<RR>, dim3(grid), dim3(256), lds, st, sh, cfg0, ncfg, rec);
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
