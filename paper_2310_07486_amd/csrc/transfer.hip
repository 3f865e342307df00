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
// e^-k w[s ^ 2^x].  For N >= 16 every pass works on tiles of 4096 states (32
// KB of LDS): the first on bits 0..11 of contiguous chunks (and the D^1/2
// scale on the way in), the others on up to 8 bits with 16 to 256 columns
// of consecutive lower indices (128-byte or longer rows), in place, the last
// one scaling by D^1/2 on the way out.  Each thread applies four butterflies
// at a time in registers between LDS exchanges.  N <= 12 (L = 2, 3) takes
// one block per 2^N states.  E0(s) comes from popcounts of s xor its
// neighbour-permuted copies against the masks of the +1 and -1 couplings;
// exp(k E0 / 2) is a table of 4N + 1 entries.  The product is HBM-bound:
// each pass reads and writes the whole vector (three passes at L = 5).
#include <algorithm>
#include <cmath>
#include <vector>

#include "tfim_internal.h"

namespace tfim {
namespace {

constexpr int kLowBits = 12;   // bits of the first pass (4096 states per block)
constexpr int kMidBits = 8;    // bits per later pass
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

// One pass over tiles of 4096 states: rows g = the nb bits bit0 .. bit0+nb-1
// of the index, columns c = C = 4096 / 2^nb consecutive indices below bit0
// (C = 1 in the first pass), one tile per value of the bits above.  Each
// thread holds 16 states whose row indices differ in four bits and applies
// those four butterflies in registers; LDS exchanges the states between
// groups of four bits (bits left over when nb is not a multiple of 4 take one
// LDS round trip each).  Optional D^1/2 scale on the way in and on the way
// out; in and out may be the same vector (each tile is read whole first).
__global__ void __launch_bounds__(256) k_tm_tile(TmParams P, const double* in, double* out, int bit0, int nb,
                                                 int first, int last) {
    __shared__ double sh[4096 + 4096 / 32];
    __shared__ double dt[4 * kMaxN + 1];
    const int tid = threadIdx.x;
    const int C = 4096 >> nb;
    const int nlo = 1 << bit0;                 // indices below bit0
    const uint32_t tiles_lo = (uint32_t)(nlo / C);
    const uint32_t lo0 = (blockIdx.x % tiles_lo) * (uint32_t)C;
    const uint32_t hi = blockIdx.x / tiles_lo;
    const uint32_t base = lo0 + (hi << (bit0 + nb));
    auto pad = [](int e) { return e + (e >> 5); };  // one spare slot per 32 doubles
    auto gidx = [&](int e) -> uint32_t { return base + (uint32_t)(e % C) + ((uint32_t)(e / C) << bit0); };
    for (int e = tid; e < 4 * P.N + 1; e += 256) dt[e] = P.dtab[e];
    if (first) __syncthreads();
    double r[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = tid + 256 * i;
        const uint32_t s = gidx(e);
        r[i] = first ? in[s] * half_diag(P, s, dt) : in[s];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) sh[pad(tid + 256 * i)] = r[i];
    __syncthreads();
    int b0 = nb;
    while (b0 >= 4) {  // groups of four row bits, from the top
        b0 -= 4;
        const int o = tid / C, c = tid % C;
        const int g0 = ((o >> b0) << (b0 + 4)) | (o & ((1 << b0) - 1));
#pragma unroll
        for (int i = 0; i < 16; ++i) r[i] = sh[pad((g0 | (i << b0)) * C + c)];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (!(i & (1 << j))) {
                    const double x0 = r[i], x1 = r[i | (1 << j)];
                    r[i] = P.a * x0 + P.b * x1;
                    r[i | (1 << j)] = P.b * x0 + P.a * x1;
                }
#pragma unroll
        for (int i = 0; i < 16; ++i) sh[pad((g0 | (i << b0)) * C + c)] = r[i];
        __syncthreads();
    }
    for (int j = 0; j < b0; ++j) {  // leftover row bits 0 .. b0-1
        for (int q = tid; q < 2048; q += 256) {
            const int c = q % C, gq = q / C;
            const int g = ((gq >> j) << (j + 1)) | (gq & ((1 << j) - 1));
            const int i0 = pad(g * C + c), i1 = pad((g | (1 << j)) * C + c);
            const double x0 = sh[i0], x1 = sh[i1];
            sh[i0] = P.a * x0 + P.b * x1;
            sh[i1] = P.b * x0 + P.a * x1;
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = tid + 256 * i;
        const uint32_t s = gidx(e);
        const double x = sh[pad(e)];
        out[s] = last ? x * half_diag(P, s, dt) : x;
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

// Per-block partial sums of <x, y>, <y, y> and, when z is given, <z, y>
// (summed on the host in block order).
constexpr int kDotBlocks = 1024;
__global__ void __launch_bounds__(256) k_tm_dots(const double* __restrict__ x, const double* __restrict__ y,
                                                 const double* __restrict__ z, uint32_t n,
                                                 double* __restrict__ part) {
    __shared__ double r0[256], r1[256], r2[256];
    double a = 0.0, c = 0.0, d = 0.0;
    for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n; s += kDotBlocks * 256) {
        const double ys = y[s];
        a += x[s] * ys;
        c += ys * ys;
        if (z) d += z[s] * ys;
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = c;
    r2[threadIdx.x] = d;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = r0[0];
        part[kDotBlocks + blockIdx.x] = r1[0];
        part[2 * kDotBlocks + blockIdx.x] = r2[0];
    }
}

// v = (w - c z) f  (z may be null: v = w f); v may be w
__global__ void k_tm_next(const double* w, const double* __restrict__ z, double c, double f, uint32_t n,
                          double* v) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x)
        v[s] = (z ? w[s] - c * z[s] : w[s]) * f;
}

__global__ void k_tm_start(double* __restrict__ v, uint32_t n, double sign, int second) {
    // the top: all ones (even sector) or +1 / -1 halves (odd sector); the
    // second: a fixed pseudo-random vector, projected on the sector below
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        if (second) {
            uint32_t h = s * 0x9E3779B1u;
            h ^= h >> 15;
            h *= 0x85EBCA77u;
            h ^= h >> 13;
            v[s] = (double)(h & 0xFFFFu) / 32768.0 - 1.0;
        } else {
            v[s] = (sign > 0.0 || s < n / 2) ? 1.0 : -1.0;
        }
    }
}

}  // namespace

const char* tm_unsupported(int L) {
    if (L < 2 || L * L > kMaxN) return "transfer matrix needs 2 <= L <= 5";
    return nullptr;
}

size_t tm_workspace_bytes(int L) {
    const size_t n = (size_t)1 << (L * L);
    return 3 * n * 8 + 3 * kDotBlocks * 8 + 256;
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
    const uint32_t n = 1u << P.N;
    if (P.N >= kLowBits + 4) {
        // tiles of 4096 states: 12 bits, then passes of 8 bits (rows) x 16
        // columns, the last pass taking what is left (at least 4 bits)
        hipError_t e = hipSuccess;
        int bit0 = 0;
        while (e == hipSuccess && bit0 < P.N) {
            int nb = bit0 == 0 ? kLowBits : std::min(kMidBits, P.N - bit0);
            if (bit0 > 0 && P.N - bit0 - nb > 0 && P.N - bit0 - nb < 4) nb = P.N - bit0 - 4;  // keep >= 4 for the last
            const uint32_t blocks = n / 4096;
            hipLaunchKernelGGL(k_tm_tile, dim3(blocks), dim3(256), 0, st, P, bit0 == 0 ? v : (const double*)w, w,
                               bit0, nb, (int)(bit0 == 0), (int)(bit0 + nb == P.N));
            e = hipGetLastError();
            bit0 += nb;
        }
        return e;
    }
    if (P.N > kLowBits) return hipErrorInvalidValue;  // N = L^2 is 4, 9, 16 or 25
    hipLaunchKernelGGL(k_tm_low, dim3(n >> P.N), dim3(256), 0, st, P, v, w, P.N, 1);
    return hipGetLastError();
}

hipError_t tm_apply(int L, double k, const int8_t* Jx, const int8_t* Jy, const double* v, double* w,
                    hipStream_t st) {
    return tm_apply_params(tm_params(L, k, Jx, Jy), v, w, st);
}

// Power iteration in one parity sector; with defl, every product has the
// component along the unit vector defl removed (the second eigenvalue).
static hipError_t tm_power(const TmParams& P, double sign, double tol, int max_iter, double* v, double* w,
                           const double* defl, double* part, std::vector<double>& hp, double* lambda,
                           int* iters, hipStream_t st) {
    const uint32_t n = 1u << P.N;
    const int grid = (int)std::min<uint32_t>(8192, (n + 255) / 256);
    auto sums = [&](const double* x, const double* y, const double* z, double out[3]) -> hipError_t {
        hipLaunchKernelGGL(k_tm_dots, dim3(kDotBlocks), dim3(256), 0, st, x, y, z, n, part);
        hipError_t e = hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        out[0] = out[1] = out[2] = 0.0;
        for (int q = 0; q < 3; ++q)
            for (int i = 0; i < kDotBlocks; ++i) out[q] += hp[q * kDotBlocks + i];
        return e;
    };
    hipLaunchKernelGGL(k_tm_start, dim3(grid), dim3(256), 0, st, v, n, sign, defl ? 1 : 0);
    hipLaunchKernelGGL(k_tm_project, dim3(grid), dim3(256), 0, st, v, n, sign);
    double d[3];
    hipError_t e = sums(v, v, defl, d);  // |v|^2 and <defl, v>
    if (e != hipSuccess) return e;
    {
        const double c = defl ? d[2] : 0.0;
        const double nn = d[1] - c * c;
        hipLaunchKernelGGL(k_tm_next, dim3(grid), dim3(256), 0, st, v, defl, c, 1.0 / std::sqrt(nn), n, v);
    }
    double lam = 0.0, prev = 0.0;
    int it = 0;
    for (; it < max_iter; ++it) {
        e = tm_apply_params(P, v, w, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_tm_project, dim3(grid), dim3(256), 0, st, w, n, sign);
        if ((e = sums(v, w, defl, d)) != hipSuccess) break;
        prev = lam;
        lam = d[0];  // Rayleigh quotient: v is a unit vector orthogonal to defl
        const double c = defl ? d[2] : 0.0;
        hipLaunchKernelGGL(k_tm_next, dim3(grid), dim3(256), 0, st, w, defl, c,
                           1.0 / std::sqrt(d[1] - c * c), n, v);
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

hipError_t tm_top(int L, double k, const int8_t* Jx, const int8_t* Jy, int odd, int nev, double tol,
                  int max_iter, void* ws, double* lambda, int* iters, hipStream_t st) {
    const TmParams P = tm_params(L, k, Jx, Jy);
    const uint32_t n = 1u << P.N;
    double* v0 = (double*)ws;   // the sector's top eigenvector
    double* v1 = v0 + n;        // the second
    double* w = v1 + n;
    double* part = w + n;
    const double sign = odd ? -1.0 : 1.0;
    std::vector<double> hp(3 * kDotBlocks);
    hipError_t e = tm_power(P, sign, tol, max_iter, v0, w, nullptr, part, hp, &lambda[0], &iters[0], st);
    if (e == hipSuccess && nev > 1)
        e = tm_power(P, sign, tol, max_iter, v1, w, v0, part, hp, &lambda[1], &iters[1], st);
    return e;
}

}  // namespace tfim
