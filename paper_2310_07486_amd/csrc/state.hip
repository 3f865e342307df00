// Instance and state initialisation, parallel tempering, lane masks.
//
// Paper: arXiv:2310.07486, Methods, "Model and simulations" (J = +-1 with
// probability 1/2 on nearest-neighbour bonds) and "Simulation details"
// (parallel tempering over k, Hukushima-Nemoto; independent real replicas).
#include "tfim_internal.h"

namespace tfim {
namespace {

// One coupling word per (j, d, xy): bit b set <=> J = -1 for sample b.
__global__ void k_init_couplings(ShapeDev sh, uint32_t key0, uint32_t key1) {
    const size_t total = (size_t)sh.W * 2 * sh.L2;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t xy = (uint32_t)(i % sh.L2);
        const uint32_t d = (uint32_t)((i / sh.L2) % 2);
        const uint32_t j = (uint32_t)(i / (2 * (size_t)sh.L2));
        const U4 o = philox10(xy, d, 0u, ctr_word3(sh.word_offset + j, sh.sid, kTagCoupling),
                              key0, key1);
        sh.J[i] = (uint64_t)o.v[0] | ((uint64_t)o.v[1] << 32);
    }
}

// Hot start: one spin word per (r, w, j, lin), i.i.d. bits.
__global__ void k_init_spins(ShapeDev sh, uint32_t key0, uint32_t key1) {
    const size_t N = (size_t)sh.L2 * sh.Lt;
    const size_t total = (size_t)sh.R * sh.nk * sh.W * N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t lin = (uint32_t)(i % N);
        const size_t cfg = i / N;  // (r*nk + w)*W + j
        const uint32_t j = (uint32_t)(cfg % sh.W);
        const uint32_t rw = (uint32_t)(cfg / sh.W);
        const U4 o = philox10(lin, rw, 0u, ctr_word3(sh.word_offset + j, sh.sid, kTagSpin), key0,
                              key1);
        sh.S[i] = (uint64_t)o.v[0] | ((uint64_t)o.v[1] << 32);
    }
}

__global__ void k_labels_identity(ShapeDev sh) {
    const size_t total = (size_t)sh.R * sh.W * 64 * sh.nk;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint8_t v = (uint8_t)(i % sh.nk);
        sh.kidx[i] = v;
        sh.winv[i] = v;
    }
}

// Lane masks of one (r, j) group from the k labels of its 64 lanes:
// mask[w][K] = lanes whose walker w has k-index < K.  Lane = sample; wave v
// of the workgroup builds walkers v, v + (waves), ...
__device__ void rebuild_masks(const ShapeDev& sh, int r, int j, const uint8_t* kl /*[64][nk]*/) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int nk = sh.nk;
    uint64_t* out = sh.mask + (size_t)(r * sh.W + j) * nk * (nk + 1);
    for (int w = wave; w < nk; w += nwaves) {
        const int mine = kl[lane * nk + w];
        for (int K0 = 0; K0 <= nk; K0 += 64) {
            uint64_t keep = 0;
            for (int K = K0; K < K0 + 64 && K <= nk; ++K) {
                const uint64_t bal = __ballot(mine < K);
                if (lane == K - K0) keep = bal;
            }
            if (K0 + lane <= nk) out[(size_t)w * (nk + 1) + K0 + lane] = keep;
        }
    }
}

__global__ void __launch_bounds__(64) k_mask_rebuild(ShapeDev sh) {
    extern __shared__ uint8_t kl[];
    const int r = blockIdx.x / sh.W, j = blockIdx.x % sh.W;
    const int lane = threadIdx.x, nk = sh.nk;
    const size_t base = ((size_t)r * sh.W * 64 + (size_t)j * 64 + lane) * nk;
    for (int w = 0; w < nk; ++w) kl[lane * nk + w] = sh.kidx[base + w];
    __syncthreads();
    rebuild_masks(sh, r, j, kl);
}

// One tempering step for every (r, sample) of word j: pairs (i, i+1) with
// i = m mod 2, m mod 2 + 2, ...; walker a holds k_i, walker b holds k_{i+1};
// with d = U_a - U_b the swap of labels is accepted iff d <= 0 or
// R < floor(2^32 exp(-(k_{i+1} - k_i) 2d)) (the exchange ratio of the two
// Boltzmann weights, E = 2U - 3N).  One uniform per lane.
constexpr int kTemperThreads = 1024;  // 64 lanes x 16 pair slots

__device__ void temper_group(const ShapeDev& sh, int r, int j, uint32_t key0, uint32_t key1,
                             uint32_t m, uint8_t* kl /*[2][64][nk]*/) {
    const int nk = sh.nk, tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, slot = tid >> 6, nslots = nthr >> 6;
    uint8_t* K = kl;             // [64][nk]: k-index of each walker
    uint8_t* Wv = kl + 64 * nk;  // [64][nk]: walker of each k-index
    // the group's labels are 64 nk contiguous bytes
    const size_t gbase = ((size_t)r * sh.W * 64 + (size_t)j * 64) * nk;
    for (int e = tid; e < 64 * nk; e += nthr) {
        K[e] = sh.kidx[gbase + e];
        Wv[e] = sh.winv[gbase + e];
    }
    __syncthreads();
    // the pairs of one step are disjoint (they touch different k-indices and
    // walkers), so the slots of a lane decide theirs in parallel
    uint8_t* ki = K + lane * nk;
    uint8_t* wi = Wv + lane * nk;
    const size_t base = gbase + (size_t)lane * nk;
    const uint32_t c3 = ctr_word3(sh.word_offset + (uint32_t)j, sh.sid, kTagTemper);
    for (int i = (int)(m & 1u) + 2 * slot; i + 1 < nk; i += 2 * nslots) {
        const int wa = wi[i], wb = wi[i + 1];
        const int64_t d = (int64_t)sh.U[base + wa] - (int64_t)sh.U[base + wb];
        const U4 o = philox10(((uint32_t)lane >> 2) | ((uint32_t)i << 4), m, (uint32_t)r, c3, key0,
                              key1);
        const uint32_t R = (lane & 2) ? ((lane & 1) ? o.v[3] : o.v[2]) : ((lane & 1) ? o.v[1] : o.v[0]);
        bool acc = d <= 0;
        if (!acc && d <= (int64_t)sh.dmax[i]) acc = R < sh.Tpt[sh.tpt_off[i] + (uint32_t)(d - 1)];
        if (acc) {
            ki[wa] = (uint8_t)(i + 1);
            ki[wb] = (uint8_t)i;
            wi[i] = (uint8_t)wb;
            wi[i + 1] = (uint8_t)wa;
        }
    }
    __syncthreads();
    for (int e = tid; e < 64 * nk; e += nthr) {
        sh.kidx[gbase + e] = K[e];
        sh.winv[gbase + e] = Wv[e];
    }
    rebuild_masks(sh, r, j, K);
}

__global__ void __launch_bounds__(kTemperThreads) k_temper(ShapeDev sh, uint32_t key0, uint32_t key1,
                                               const Counters* __restrict__ ctr) {
    extern __shared__ uint8_t kl[];  // [64][nk] labels, then [64][nk] inverse
    temper_group(sh, (int)blockIdx.x / sh.W, (int)blockIdx.x % sh.W, key0, key1, ctr->m, kl);
}

__device__ __forceinline__ bool pt_due(const ShapeDev& sh, uint32_t t) {
    return sh.pt_every != 0 && ((t + 1) % sh.pt_every) == 0;
}

// Every shape's (r, j) groups in one launch; a shape whose tempering is not
// due after this sweep is skipped.
__global__ void __launch_bounds__(kTemperThreads) k_temper_batch(TemperBatchArgs a) {
    extern __shared__ uint8_t kl[];
    const uint32_t b = blockIdx.x;
    uint32_t s = 0;
    while (s + 1 < a.n_shapes && b >= a.first[s + 1]) ++s;
    const ShapeDev sh = a.shapes[s];
    if (!pt_due(sh, a.ctr[s].t)) return;
    const int loc = (int)(b - a.first[s]);
    temper_group(sh, loc / sh.W, loc % sh.W, a.key0, a.key1, a.ctr[s].m, kl);
}

__global__ void k_advance_batch(TemperBatchArgs a) {
    const uint32_t s = threadIdx.x;
    if (blockIdx.x == 0 && s < a.n_shapes) {
        const uint32_t t = a.ctr[s].t;
        const bool due = pt_due(a.shapes[s], t);
        a.ctr[s].t = t + 1;
        a.ctr[s].m += due ? 1u : 0u;
    }
}

__global__ void k_advance(Counters* ctr, uint32_t dt, uint32_t dm) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctr->t += dt;
        ctr->m += dm;
    }
}

unsigned grid_for(size_t total) {
    size_t b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b == 0) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_init_couplings(const ShapeDev& sh, uint64_t seed, hipStream_t st) {
    const size_t total = (size_t)sh.W * 2 * sh.L2;
    hipLaunchKernelGGL(k_init_couplings, dim3(grid_for(total)), dim3(256), 0, st, sh,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_init_spins(const ShapeDev& sh, uint64_t seed, hipStream_t st) {
    const size_t total = (size_t)sh.R * sh.nk * sh.W * sh.L2 * sh.Lt;
    hipLaunchKernelGGL(k_init_spins, dim3(grid_for(total)), dim3(256), 0, st, sh, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_labels_identity(const ShapeDev& sh, hipStream_t st) {
    const size_t total = (size_t)sh.R * sh.W * 64 * sh.nk;
    hipLaunchKernelGGL(k_labels_identity, dim3(grid_for(total)), dim3(256), 0, st, sh);
    return hipGetLastError();
}

hipError_t launch_mask_rebuild(const ShapeDev& sh, hipStream_t st) {
    hipLaunchKernelGGL(k_mask_rebuild, dim3(sh.R * sh.W), dim3(64), (size_t)64 * sh.nk, st, sh);
    return hipGetLastError();
}

hipError_t launch_temper(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st) {
    hipLaunchKernelGGL(k_temper, dim3(sh.R * sh.W), dim3(kTemperThreads), (size_t)128 * sh.nk, st, sh,
                       (uint32_t)seed, (uint32_t)(seed >> 32), ctr);
    return hipGetLastError();
}

hipError_t launch_temper_batch(const TemperBatchArgs& a, int blocks, int max_nk, hipStream_t st) {
    hipLaunchKernelGGL(k_temper_batch, dim3(blocks), dim3(kTemperThreads), (size_t)128 * max_nk, st, a);
    return hipGetLastError();
}

hipError_t launch_advance_batch(const TemperBatchArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_advance_batch, dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_advance(Counters* ctr, uint32_t dt, uint32_t dm, hipStream_t st) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, ctr, dt, dm);
    return hipGetLastError();
}

}  // namespace tfim
