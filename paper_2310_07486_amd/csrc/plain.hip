// Plain form of the sampler: one signed byte per spin, one sample per
// configuration, no multispin coding.  It is the reference point for the
// multispin path and the form in which a single disorder sample is run.
//
// Paper: arXiv:2310.07486, Methods, "The Trotter-Suzuki formula" (classical
// spins S = +-1 on the L x L x Ltau lattice, p(S) ~ exp(-k E(S)), the action
// with J on spatial and +1 on temporal bonds, periodic or antiperiodic along
// tau) and "Simulation details" (Metropolis sweeps, parallel tempering over
// k, real replicas); "Model and simulations" for J = +-1 with probability 1/2.
//
// Layouts (canonical, also on the device; ns = number of samples):
//   spins      int8 [R][nk][ns][Ltau][L*L]   +1 / -1
//   couplings  int8 [ns][2][L*L]             +1 / -1 (d = 0: +x bond, 1: +y bond)
//   k labels, walker maps, energies as in the multispin form, [R][ns][nk].
// Sample s draws every random number from word j = word_offset + s/64 and
// lane s%64 of the multispin counter layout, so it follows exactly the
// trajectory of lane s%64 of that word in a multispin run.
//
// Kernels reuse ShapeDev: W holds the number of samples ns, S and J point at
// the int8 arrays.
#include "tfim_internal.h"

namespace tfim {
namespace {

__device__ __forceinline__ uint32_t plain_word(const ShapeDev& sh, int s) {
    return sh.word_offset + (uint32_t)s / 64u;
}

// J = -1 where bit s%64 of the coupling word (xy, d) of word j is set.
__global__ void k_plain_init_couplings(ShapeDev sh, uint32_t key0, uint32_t key1) {
    int8_t* J = (int8_t*)sh.J;
    const size_t total = (size_t)sh.W * 2 * sh.L2;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t xy = (uint32_t)(i % sh.L2);
        const uint32_t d = (uint32_t)((i / sh.L2) % 2);
        const int s = (int)(i / (2 * (size_t)sh.L2));
        const U4 o = philox10(xy, d, 0u, ctr_word3(plain_word(sh, s), sh.sid, kTagCoupling), key0, key1);
        const uint64_t word = (uint64_t)o.v[0] | ((uint64_t)o.v[1] << 32);
        J[i] = ((word >> (s & 63)) & 1ull) ? (int8_t)-1 : (int8_t)1;
    }
}

// Hot start: spin (r, w, s, lin) = -1 where bit s%64 of the spin word is set.
__global__ void k_plain_init_spins(ShapeDev sh, uint32_t key0, uint32_t key1) {
    int8_t* S8 = (int8_t*)sh.S;
    const size_t N = (size_t)sh.L2 * sh.Lt;
    const size_t total = (size_t)sh.R * sh.nk * sh.W * N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t lin = (uint32_t)(i % N);
        const size_t cfg = i / N;  // (r*nk + w)*ns + s
        const int s = (int)(cfg % sh.W);
        const uint32_t rw = (uint32_t)(cfg / sh.W);
        const U4 o = philox10(lin, rw, 0u, ctr_word3(plain_word(sh, s), sh.sid, kTagSpin), key0, key1);
        const uint64_t word = (uint64_t)o.v[0] | ((uint64_t)o.v[1] << 32);
        S8[i] = ((word >> (s & 63)) & 1ull) ? (int8_t)-1 : (int8_t)1;
    }
}

// Metropolis half-sweep of colour c.  One thread takes the four sites of
// colour c at tau = 8q + 2hh + p (hh = 0..3, p = (c + x + y) mod 2) of one
// column: they share one Philox call, output hh.  A site's energy change is
// dE = 2 S h with h its local field (the wrap neighbour along tau with the
// sign -1 when antiperiodic); the move is taken iff dE <= 0 or
// R < Tu[k-index][u] with u = (12 - dE)/4 unsatisfied bonds.  Sites of one
// colour only neighbour the other colour, so threads never race.
__global__ void __launch_bounds__(256) k_plain_half(ShapeDev sh, uint32_t key0, uint32_t key1,
                                                    const Counters* __restrict__ ctr, int c) {
    int8_t* S8 = (int8_t*)sh.S;
    const int8_t* J = (const int8_t*)sh.J;
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, ns = sh.W;
    const int nq = (Lt + 7) / 8;
    const uint32_t t = ctr->t;
    const int sgn = sh.apm ? -1 : 1;
    const size_t total = (size_t)sh.R * nk * ns * L2 * nq;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const int q = (int)(i % nq);
        const size_t rest = i / nq;
        const int xy = (int)(rest % L2);
        const size_t cfg = rest / L2;  // (r*nk + w)*ns + s
        const int s = (int)(cfg % ns);
        const int rw = (int)(cfg / ns);
        const int r = rw / nk, w = rw % nk;
        const int x = xy % L, y = xy / L;
        const int xm = (x + L - 1) % L + L * y, xp = (x + 1) % L + L * y;
        const int ym = x + L * ((y + L - 1) % L), yp = x + L * ((y + 1) % L);
        const int8_t* jb = J + (size_t)s * 2 * L2;
        const int jxp = jb[xy], jxm = jb[xm], jyp = jb[L2 + xy], jym = jb[L2 + ym];
        const U4 o = philox10((uint32_t)(xy + L2 * q), t, ((uint32_t)rw << 1) | (uint32_t)c,
                              ctr_word3(plain_word(sh, s), sh.sid, kTagMetro), key0, key1);
        const int kix = sh.kidx[((size_t)r * ns + s) * nk + w];
        int8_t* cf = S8 + cfg * (size_t)L2 * Lt;
        const int p = (c + x + y) & 1;
#pragma unroll
        for (int hh = 0; hh < 4; ++hh) {
            const int tau = 8 * q + 2 * hh + p;
            if (tau >= Lt) break;
            const int8_t* P = cf + (size_t)tau * L2;
            const int tm = tau == 0 ? Lt - 1 : tau - 1, tp = tau == Lt - 1 ? 0 : tau + 1;
            const int cm = tau == 0 ? sgn : 1, cp = tau == Lt - 1 ? sgn : 1;
            const int h = jxp * P[xp] + jxm * P[xm] + jyp * P[yp] + jym * P[ym] +
                          cm * cf[(size_t)tm * L2 + xy] + cp * cf[(size_t)tp * L2 + xy];
            const int sv = P[xy];
            const int dE = 2 * sv * h;
            bool flip = dE <= 0;
            if (!flip) flip = o.v[hh] < sh.Tu[kix * 3 + (12 - dE) / 4];
            if (flip) cf[(size_t)tau * L2 + xy] = (int8_t)(-sv);
        }
    }
}

// Unsatisfied bonds U of every configuration from the action: each site
// counts its +x, +y and +tau bonds (E = 2U - 3N).  One workgroup per
// configuration.
__global__ void __launch_bounds__(256) k_plain_energy(ShapeDev sh) {
    __shared__ uint32_t tot;
    const int8_t* S8 = (const int8_t*)sh.S;
    const int8_t* J = (const int8_t*)sh.J;
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, ns = sh.W;
    const int cfg = blockIdx.x;  // (r*nk + w)*ns + s
    const int s = cfg % ns, rw = cfg / ns, r = rw / nk, w = rw % nk;
    const int8_t* cf = S8 + (size_t)cfg * L2 * Lt;
    const int8_t* jb = J + (size_t)s * 2 * L2;
    const int sgn = sh.apm ? -1 : 1;
    if (threadIdx.x == 0) tot = 0;
    __syncthreads();
    uint32_t u = 0;
    for (int lin = threadIdx.x; lin < L2 * Lt; lin += blockDim.x) {
        const int xy = lin % L2, tau = lin / L2;
        const int x = xy % L, y = xy / L;
        const int xp = (x + 1) % L + L * y, yp = x + L * ((y + 1) % L);
        const int8_t* P = cf + (size_t)tau * L2;
        const int tn = tau == Lt - 1 ? 0 : tau + 1;
        const int ct = tau == Lt - 1 ? sgn : 1;
        const int sv = P[xy];
        u += (jb[xy] * sv * P[xp] < 0) + (jb[L2 + xy] * sv * P[yp] < 0) +
             (ct * sv * cf[(size_t)tn * L2 + xy] < 0);
    }
    atomicAdd(&tot, u);
    __syncthreads();
    if (threadIdx.x == 0) sh.U[((size_t)r * ns + s) * nk + w] = tot;
}

// One tempering step for every (r, s): pairs (i, i+1), i = m mod 2, m mod 2 + 2,
// ...; d = U_a - U_b of the walkers at k_i, k_{i+1}; accept iff d <= 0 or
// R < Tpt[i][d] (the exchange ratio with E = 2U - 3N); R = output s%4 of the
// Philox call ((s%64)/4 | i << 4, m, r, word j), one uniform per sample.
__global__ void k_plain_temper(ShapeDev sh, uint32_t key0, uint32_t key1, const Counters* __restrict__ ctr) {
    const int nk = sh.nk, ns = sh.W;
    const uint32_t m = ctr->m;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= sh.R * ns) return;
    const int r = g / ns, s = g % ns;
    const uint32_t b = (uint32_t)(s & 63);
    uint8_t* ki = sh.kidx + (size_t)g * nk;
    uint8_t* wi = sh.winv + (size_t)g * nk;
    const uint32_t* U = sh.U + (size_t)g * nk;
    const uint32_t c3 = ctr_word3(plain_word(sh, s), sh.sid, kTagTemper);
    for (int i = (int)(m & 1u); i + 1 < nk; i += 2) {
        const int wa = wi[i], wb = wi[i + 1];
        const int64_t d = (int64_t)U[wa] - (int64_t)U[wb];
        const U4 o = philox10((b >> 2) | ((uint32_t)i << 4), m, (uint32_t)r, c3, key0, key1);
        const uint32_t R = o.v[b & 3];
        bool acc = d <= 0;
        if (!acc && d <= (int64_t)sh.dmax[i]) acc = R < sh.Tpt[sh.tpt_off[i] + (uint32_t)(d - 1)];
        if (acc) {
            ki[wa] = (uint8_t)(i + 1);
            ki[wb] = (uint8_t)i;
            wi[i] = (uint8_t)wb;
            wi[i + 1] = (uint8_t)wa;
        }
    }
}

// Identity k labels: walker w of every (r, s) at k-index w.  The plain
// label arrays hold R * ns * nk entries (ns samples, not 64 per word).
__global__ void k_plain_labels(ShapeDev sh) {
    const size_t total = (size_t)sh.R * sh.W * sh.nk;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint8_t v = (uint8_t)(i % sh.nk);
        sh.kidx[i] = v;
        sh.winv[i] = v;
    }
}

__global__ void k_plain_zero(int64_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

constexpr int kPlainMaxP = 15;  // six replicas

// Pair records of configuration cfg = cfg0 + blockIdx.y (k-index i, sample s):
// G^r_xy = sum_tau S^r_x,tau S^r_y,tau of the walker at k-index i of every
// replica, one element (x, y) per thread, int32; D_x[d] += G^a_xy G^b_xy at
// d = (x1 - y1) mod L (D_y in x2 - y2), in int64.
__global__ void __launch_bounds__(256) k_plain_gram(ShapeDev sh, int cfg0) {
    __shared__ unsigned long long D[kPlainMaxP * 2 * 24];
    const int8_t* S8 = (const int8_t*)sh.S;
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, ns = sh.W, R = sh.R, P = sh.P;
    const int cfg = cfg0 + blockIdx.y;
    const int i = cfg / ns, s = cfg % ns;
    for (int e = threadIdx.x; e < P * 2 * L; e += blockDim.x) D[e] = 0;
    __syncthreads();
    const long long nel = (long long)L2 * L2;
    for (long long el = (long long)blockIdx.x * blockDim.x + threadIdx.x; el < nel;
         el += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(el / L2), y = (int)(el % L2);
        int G[6];
        for (int r = 0; r < R; ++r) {
            const int w = sh.winv[((size_t)r * ns + s) * nk + i];
            const int8_t* cf = S8 + ((size_t)(r * nk + w) * ns + s) * L2 * Lt;
            int acc = 0;
            for (int tau = 0; tau < Lt; ++tau) acc += cf[(size_t)tau * L2 + x] * cf[(size_t)tau * L2 + y];
            G[r] = acc;
        }
        const int dx = ((x % L) - (y % L) + L) % L, dy = ((x / L) - (y / L) + L) % L;
        int p = 0;
        for (int a = 0; a < R; ++a)
            for (int b = a + 1; b < R; ++b, ++p) {
                const unsigned long long h = (unsigned long long)((long long)G[a] * G[b]);
                atomicAdd(&D[(p * 2 + 0) * L + dx], h);
                atomicAdd(&D[(p * 2 + 1) * L + dy], h);
            }
    }
    __syncthreads();
    const int rl = 2 * L + 3;
    for (int e = threadIdx.x; e < P * 2 * L; e += blockDim.x)
        if (D[e]) atomicAdd((unsigned long long*)&sh.rec[((size_t)cfg * P + e / (2 * L)) * rl + e % (2 * L)], D[e]);
}

// Overlap part of the pair records: Q^ab_t1,t2 = sum_x S^a_x,t1 S^b_x,t2, one
// element per thread; trQ, sum Q^2, sum Q^4 in int64 (|Q| <= L^2).
__global__ void __launch_bounds__(256) k_plain_overlap(ShapeDev sh, int cfg0) {
    __shared__ unsigned long long red[kPlainMaxP * 3];
    const int8_t* S8 = (const int8_t*)sh.S;
    const int L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, ns = sh.W, R = sh.R, P = sh.P;
    const int cfg = cfg0 + blockIdx.y;
    const int i = cfg / ns, s = cfg % ns;
    for (int e = threadIdx.x; e < P * 3; e += blockDim.x) red[e] = 0;
    __syncthreads();
    const long long nel = (long long)Lt * Lt;
    for (long long el = (long long)blockIdx.x * blockDim.x + threadIdx.x; el < nel;
         el += (long long)gridDim.x * blockDim.x) {
        const int t1 = (int)(el / Lt), t2 = (int)(el % Lt);
        int p = 0;
        for (int a = 0; a < R; ++a)
            for (int b = a + 1; b < R; ++b, ++p) {
                const int wa = sh.winv[((size_t)a * ns + s) * nk + i];
                const int wb = sh.winv[((size_t)b * ns + s) * nk + i];
                const int8_t* pa = S8 + (((size_t)(a * nk + wa) * ns + s) * Lt + t1) * L2;
                const int8_t* pb = S8 + (((size_t)(b * nk + wb) * ns + s) * Lt + t2) * L2;
                int q = 0;
                for (int x = 0; x < L2; ++x) q += pa[x] * pb[x];
                const long long q2 = (long long)q * q;
                atomicAdd(&red[p * 3 + 1], (unsigned long long)q2);
                atomicAdd(&red[p * 3 + 2], (unsigned long long)(q2 * q2));
                if (t1 == t2) atomicAdd(&red[p * 3 + 0], (unsigned long long)(long long)q);
            }
    }
    __syncthreads();
    const int rl = 2 * sh.L + 3;
    for (int e = threadIdx.x; e < P * 3; e += blockDim.x)
        if (red[e]) atomicAdd((unsigned long long*)&sh.rec[((size_t)cfg * P + e / 3) * rl + 2 * sh.L + e % 3], red[e]);
}

// A[i][h][d] = sum over samples and pairs of the records' D_x (h = 0), D_y (h = 1).
__global__ void k_plain_buckets(ShapeDev sh) {
    const int L = sh.L, ns = sh.W, P = sh.P, rl = 2 * L + 3;
    const int n = sh.nk * 2 * L;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int i = e / (2 * L), hd = e % (2 * L);
        long long acc = 0;
        for (int s = 0; s < ns; ++s)
            for (int p = 0; p < P; ++p) acc += sh.rec[((size_t)(i * ns + s) * P + p) * rl + hd];
        sh.buckets[e] = acc;
    }
}

unsigned grid_of(size_t total, size_t cap = 65536) {
    size_t b = (total + 255) / 256;
    if (b > cap) b = cap;
    if (b == 0) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t plain_init_couplings(const ShapeDev& sh, uint64_t seed, hipStream_t st) {
    const size_t total = (size_t)sh.W * 2 * sh.L2;
    hipLaunchKernelGGL(k_plain_init_couplings, dim3(grid_of(total)), dim3(256), 0, st, sh, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t plain_init_spins(const ShapeDev& sh, uint64_t seed, hipStream_t st) {
    const size_t total = (size_t)sh.R * sh.nk * sh.W * sh.L2 * sh.Lt;
    hipLaunchKernelGGL(k_plain_init_spins, dim3(grid_of(total)), dim3(256), 0, st, sh, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t plain_labels_identity(const ShapeDev& sh, hipStream_t st) {
    const size_t total = (size_t)sh.R * sh.W * sh.nk;
    hipLaunchKernelGGL(k_plain_labels, dim3(grid_of(total)), dim3(256), 0, st, sh);
    return hipGetLastError();
}

hipError_t plain_energy(const ShapeDev& sh, hipStream_t st) {
    hipLaunchKernelGGL(k_plain_energy, dim3(sh.R * sh.nk * sh.W), dim3(256), 0, st, sh);
    return hipGetLastError();
}

hipError_t plain_sweep(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st) {
    const size_t total = (size_t)sh.R * sh.nk * sh.W * sh.L2 * ((sh.Lt + 7) / 8);
    for (int c = 0; c < 2; ++c) {
        hipLaunchKernelGGL(k_plain_half, dim3(grid_of(total)), dim3(256), 0, st, sh, (uint32_t)seed,
                           (uint32_t)(seed >> 32), ctr, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return plain_energy(sh, st);
}

hipError_t plain_temper(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st) {
    const int n = sh.R * sh.W;
    hipLaunchKernelGGL(k_plain_temper, dim3((n + 63) / 64), dim3(64), 0, st, sh, (uint32_t)seed,
                       (uint32_t)(seed >> 32), ctr);
    return hipGetLastError();
}

bool plain_measure_ok(const ShapeDev& sh) { return sh.R >= 2 && sh.R <= 6 && sh.L <= 24; }

hipError_t plain_measure(const ShapeDev& sh, int cfg0, int ncfg, hipStream_t st) {
    if (ncfg <= 0) return hipSuccess;
    const size_t rl = (size_t)(2 * sh.L + 3) * sh.P;
    hipLaunchKernelGGL(k_plain_zero, dim3(grid_of((size_t)ncfg * rl, 4096)), dim3(256), 0, st,
                       sh.rec + (size_t)cfg0 * rl, (size_t)ncfg * rl);
    hipError_t e = hipGetLastError();
    // at most 65535 configurations per launch along y
    for (int c = 0; c < ncfg && e == hipSuccess; c += 65535) {
        const int n = ncfg - c < 65535 ? ncfg - c : 65535;
        const unsigned gx = grid_of((size_t)sh.L2 * sh.L2, 64);
        const unsigned gq = grid_of((size_t)sh.Lt * sh.Lt, 256);
        hipLaunchKernelGGL(k_plain_gram, dim3(gx, n), dim3(256), 0, st, sh, cfg0 + c);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_plain_overlap, dim3(gq, n), dim3(256), 0, st, sh, cfg0 + c);
        e = hipGetLastError();
    }
    return e;
}

hipError_t plain_buckets(const ShapeDev& sh, hipStream_t st) {
    hipLaunchKernelGGL(k_plain_buckets, dim3(16), dim3(256), 0, st, sh);
    return hipGetLastError();
}

}  // namespace tfim
