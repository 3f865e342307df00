// Transfer matrix of one plane: matrix-free product and the largest
// eigenvalue of each parity sector.
//
// Paper: arXiv:2310.07486, Methods, "The Trotter-Suzuki formula" (the weight
// exp(-k E) of the L x L x Ltau lattice, Z = Tr T^Ltau with the transfer
// matrix T between consecutive planes, and the parity operator for the
// antiperiodic boundary) and "Simulation details" (exact diagonalisation of
// the transfer matrix, in parity sectors of half the size).
//
// With E0(s) = sum over spatial bonds (each once) of J_b s_x s_y,
//   T = D^1/2 K D^1/2,  D = diag(exp(k E0)),  K = (x)_x [[e^k, e^-k], [e^-k, e^k]],
// on 2^N states (N = L^2; bit x of the index is set when s_x = -1).  K is
// applied as N two-term butterflies, one per bit: w[s] <- e^k w[s] +
// e^-k w[s ^ 2^x].  The first pass takes bits 0..11 of contiguous chunks of
// 4096 states in LDS (and the D^1/2 scale on the way in); further passes take
// up to 8 bits each on tiles of 16 consecutive low indices (128-byte rows),
// in place, the last one scaling by D^1/2 on the way out.  E0(s) comes from
// popcounts of s xor its neighbour-permuted copies against the masks of the
// +1 and -1 couplings; exp(k E0 / 2) is a table of 4N + 1 entries.  The
// product is HBM-bound: each pass reads and writes the whole vector.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tfim_internal.h"

namespace tfim {
namespace {

constexpr int kLowBits = 12;   // bits of the first pass (4096 states per block)
constexpr int kMidBits = 8;    // bits per later pass
constexpr int kCols = 16;      // consecutive low indices per later-pass tile
constexpr int kMaxN = 25;      // L <= 5

struct TmParams {
    int N, L, S0;              // sites, edge, sum of all couplings
    uint32_t jxp, jxm, jyp, jym, lastcol, full;
    double a, b;               // e^k, e^-k
    double dtab[4 * kMaxN + 1];  // exp(k E0 / 2) at E0 + 2N
};

__device__ __forceinline__ double half_diag(const TmParams& P, uint32_t s, const double* dt) {
    // neighbour-permuted copies: bit i of rx is the bit of the +x neighbour of i
    const uint32_t rx = ((s >> 1) & ~P.lastcol) | ((s << (P.L - 1)) & P.lastcol);
    const uint32_t ry = ((s >> P.L) | (s << (P.N - P.L))) & P.full;
    const uint32_t dx = s ^ rx, dy = s ^ ry;
    const int e0 = P.S0 - 2 * (__popc(dx & P.jxp) - __popc(dx & P.jxm) + __popc(dy & P.jyp) -
                               __popc(dy & P.jym));
    return dt[e0 + 2 * P.N];
}

// in -> out: D^1/2 scale, butterflies of bits 0 .. nlow-1 on chunks of 2^nlow
// contiguous states, and the final D^1/2 scale when no pass follows.
__global__ void __launch_bounds__(256) k_tm_low(TmParams P, const double* __restrict__ in,
                                                double* __restrict__ out, int nlow, int last) {
    __shared__ double sh[1 << kLowBits];
    __shared__ double dt[4 * kMaxN + 1];
    const int tid = threadIdx.x;
    const int chunk = 1 << nlow;
    const uint32_t base = (uint32_t)blockIdx.x << nlow;
    for (int e = tid; e < 4 * P.N + 1; e += 256) dt[e] = P.dtab[e];
    __syncthreads();
    for (int e = tid; e < chunk; e += 256) sh[e] = in[base + e] * half_diag(P, base + e, dt);
    __syncthreads();
    for (int j = 0; j < nlow; ++j) {
        for (int p = tid; p < chunk / 2; p += 256) {
            const int i0 = ((p >> j) << (j + 1)) | (p & ((1 << j) - 1));
            const int i1 = i0 | (1 << j);
            const double x0 = sh[i0], x1 = sh[i1];
            sh[i0] = P.a * x0 + P.b * x1;
            sh[i1] = P.b * x0 + P.a * x1;
        }
        __syncthreads();
    }
    for (int e = tid; e < chunk; e += 256) out[base + e] = last ? sh[e] * half_diag(P, base + e, dt) : sh[e];
}

// In place: butterflies of bits bit0 .. bit0+nb-1.  A block takes kCols
// consecutive low indices (below bit0) and every value of the nb bits, for
// one value of the bits above.
__global__ void __launch_bounds__(256) k_tm_mid(TmParams P, double* __restrict__ v, int bit0, int nb,
                                                int last) {
    __shared__ double sh[(1 << kMidBits) * kCols];
    __shared__ double dt[4 * kMaxN + 1];
    const int tid = threadIdx.x;
    const int ng = 1 << nb;
    const uint32_t nlo = 1u << bit0;
    const uint32_t lo0 = (blockIdx.x % (nlo / kCols)) * kCols;
    const uint32_t hi = blockIdx.x / (nlo / kCols);
    const uint32_t base = lo0 + (hi << (bit0 + nb));
    for (int e = tid; e < 4 * P.N + 1; e += 256) dt[e] = P.dtab[e];
    for (int e = tid; e < ng * kCols; e += 256) {
        const int g = e / kCols, c = e % kCols;
        sh[e] = v[base + c + ((uint32_t)g << bit0)];
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        for (int p = tid; p < (ng / 2) * kCols; p += 256) {
            const int c = p % kCols, q = p / kCols;
            const int g0 = ((q >> j) << (j + 1)) | (q & ((1 << j) - 1));
            const int i0 = g0 * kCols + c, i1 = (g0 | (1 << j)) * kCols + c;
            const double x0 = sh[i0], x1 = sh[i1];
            sh[i0] = P.a * x0 + P.b * x1;
            sh[i1] = P.b * x0 + P.a * x1;
        }
        __syncthreads();
    }
    for (int e = tid; e < ng * kCols; e += 256) {
        const int g = e / kCols, c = e % kCols;
        const uint32_t s = base + c + ((uint32_t)g << bit0);
        v[s] = last ? sh[e] * half_diag(P, s, dt) : sh[e];
    }
}

// Projection on a parity sector: w[s], w[~s] <- (w[s] + sign w[~s]) / 2, sign w[s].
__global__ void k_tm_project(double* __restrict__ w, uint32_t n, double sign) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n / 2; s += gridDim.x * blockDim.x) {
        const uint32_t t = n - 1 - s;
        const double m = 0.5 * (w[s] + sign * w[t]);
        w[s] = m;
        w[t] = sign * m;
    }
}

// Per-block partial sums of <x, y> and <y, y> (summed on the host in block order).
constexpr int kDotBlocks = 256;
__global__ void __launch_bounds__(256) k_tm_dots(const double* __restrict__ x, const double* __restrict__ y,
                                                 uint32_t n, double* __restrict__ part) {
    __shared__ double r0[256], r1[256];
    double a = 0.0, c = 0.0;
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n; s += kDotBlocks * 256) {
        a += x[s] * y[s];
        c += y[s] * y[s];
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = r0[0];
        part[kDotBlocks + blockIdx.x] = r1[0];
    }
}

__global__ void k_tm_scale(const double* __restrict__ x, double* __restrict__ y, uint32_t n, double f) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) y[s] = x[s] * f;
}

__global__ void k_tm_start(double* __restrict__ v, uint32_t n, double sign) {
    // the even sector starts from all ones, the odd one from +1 / -1 halves
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x)
        v[s] = (sign > 0.0 || s < n / 2) ? 1.0 : -1.0;
}

}  // namespace

const char* tm_unsupported(int L) {
    if (L < 2 || L * L > kMaxN) return "transfer matrix needs 2 <= L <= 5";
    return nullptr;
}

size_t tm_workspace_bytes(int L) {
    const size_t n = (size_t)1 << (L * L);
    return 2 * n * 8 + 2 * kDotBlocks * 8 + 256;
}

static TmParams tm_params(int L, double k, const int8_t* Jx, const int8_t* Jy) {
    TmParams P{};
    P.L = L;
    P.N = L * L;
    P.full = P.N == 32 ? 0xFFFFFFFFu : ((1u << P.N) - 1u);
    int S0 = 0;
    for (int i = 0; i < P.N; ++i) {
        if (Jx[i] > 0) P.jxp |= 1u << i; else P.jxm |= 1u << i;
        if (Jy[i] > 0) P.jyp |= 1u << i; else P.jym |= 1u << i;
        S0 += Jx[i] + Jy[i];
        if (i % L == L - 1) P.lastcol |= 1u << i;
    }
    P.S0 = S0;
    P.a = std::exp(k);
    P.b = std::exp(-k);
    for (int e = -2 * P.N; e <= 2 * P.N; ++e) P.dtab[e + 2 * P.N] = std::exp(0.5 * k * (double)e);
    return P;
}

static hipError_t tm_apply_params(const TmParams& P, const double* v, double* w, hipStream_t st) {
    const int nlow = std::min(P.N, kLowBits);
    const uint32_t n = 1u << P.N;
    hipLaunchKernelGGL(k_tm_low, dim3(n >> nlow), dim3(256), 0, st, P, v, w, nlow, (int)(P.N == nlow));
    hipError_t e = hipGetLastError();
    for (int bit0 = nlow; e == hipSuccess && bit0 < P.N; bit0 += kMidBits) {
        const int nb = std::min(kMidBits, P.N - bit0);
        const uint32_t blocks = ((1u << bit0) / kCols) << (P.N - bit0 - nb);
        hipLaunchKernelGGL(k_tm_mid, dim3(blocks), dim3(256), 0, st, P, w, bit0, nb, (int)(bit0 + nb == P.N));
        e = hipGetLastError();
    }
    return e;
}

hipError_t tm_apply(int L, double k, const int8_t* Jx, const int8_t* Jy, const double* v, double* w,
                    hipStream_t st) {
    return tm_apply_params(tm_params(L, k, Jx, Jy), v, w, st);
}

hipError_t tm_top(int L, double k, const int8_t* Jx, const int8_t* Jy, int odd, double tol, int max_iter,
                  void* ws, double* lambda, int* iters, hipStream_t st) {
    const TmParams P = tm_params(L, k, Jx, Jy);
    const uint32_t n = 1u << P.N;
    double* v = (double*)ws;
    double* w = v + n;
    double* part = w + n;
    const double sign = odd ? -1.0 : 1.0;
    const int grid = (int)std::min<uint32_t>(1024, (n + 255) / 256);
    std::vector<double> hp(2 * kDotBlocks);
    hipLaunchKernelGGL(k_tm_start, dim3(grid), dim3(256), 0, st, v, n, sign);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {  // normalise the start vector
        hipLaunchKernelGGL(k_tm_dots, dim3(kDotBlocks), dim3(256), 0, st, v, v, n, part);
        e = hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        double nn = 0.0;
        for (int i = 0; i < kDotBlocks; ++i) nn += hp[kDotBlocks + i];
        if (e == hipSuccess) hipLaunchKernelGGL(k_tm_scale, dim3(grid), dim3(256), 0, st, v, v, n, 1.0 / std::sqrt(nn));
    }
    double lam = 0.0, prev = 0.0;
    int it = 0;
    for (; e == hipSuccess && it < max_iter; ++it) {
        e = tm_apply_params(P, v, w, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_tm_project, dim3(grid), dim3(256), 0, st, w, n, sign);
        hipLaunchKernelGGL(k_tm_dots, dim3(kDotBlocks), dim3(256), 0, st, v, w, n, part);
        e = hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        double vw = 0.0, ww = 0.0;
        for (int i = 0; i < kDotBlocks; ++i) {
            vw += hp[i];
            ww += hp[kDotBlocks + i];
        }
        prev = lam;
        lam = vw;  // Rayleigh quotient: v has unit norm
        hipLaunchKernelGGL(k_tm_scale, dim3(grid), dim3(256), 0, st, w, v, n, 1.0 / std::sqrt(ww));
        if (it >= 2 && std::fabs(lam - prev) <= tol * std::fabs(lam)) {
            ++it;
            break;
        }
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    *lambda = lam;
    *iters = it;
    return e;
}

}  // namespace tfim
