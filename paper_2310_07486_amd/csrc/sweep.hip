// Multispin checkerboard Metropolis sweep of the Trotter lattice.
//
// Paper: arXiv:2310.07486, Methods, "The Trotter-Suzuki formula" (the
// action and p(S) = exp(-k E)/Z) and "Simulation details" (full-lattice
// Metropolis sweeps, multispin coding).  64 disorder samples share each
// uint64 word; bit b of a word is sample b of that word (bit 1 = spin -1).
//
// One workgroup sweeps one configuration (replica r, walker w, word j); one
// thread owns one spatial column xy and walks the tau axis in chunks of 8
// planes.  Both colours are fused into a single pass (a tau wavefront):
//   chunk q, colour 0 -> chunk q-1, colour 1 -> store chunk q-1,
// so every spin word is read once and written once per sweep.  Spatial
// neighbours come from LDS half-planes (one colour of 8 planes), temporal
// neighbours from the thread's own registers.  On the periodic tau axis the
// colour-1 sites of plane 0 need colour 0 of plane Ltau-1, which is only
// known at the end, so they are updated last.
//
// Per site and lane: u = number of unsatisfied bonds among the six (bit
// sliced: two full adders over the bond parities); the move costs
// dE = 12 - 4u and is taken iff u >= 3 or R < Tu[k-index][u], where the
// uniform R is shared by the 64 lanes.  Lanes sit at different k-indices
// (tempering moves labels, not spins); Tu[i][u] falls with i, so the lanes
// that accept are those with k-index < K_u(R) = #{i : Tu[i][u] > R}, read
// from a per-(walker, word) table of lane masks.  The colour-1 pass also
// counts, per lane, the unsatisfied bonds of the final state (every bond
// joins a colour-0 and a colour-1 site), which gives U exactly.
#include "tfim_internal.h"

namespace tfim {
namespace {

constexpr int kChunk = 8;        // planes per chunk (4 same-colour sites)
constexpr int kMaxThreads = 576; // one thread per column, L <= 24
constexpr int kSmallBits = 5;    // per-chunk unsatisfied count <= 4*6 = 24
constexpr int kBigBits = 12;     // per-thread counter, flushed every 128 chunks
constexpr int kFlushChunks = 128;

struct Vcount {
    uint64_t big[kBigBits];
};

// Add a 3-bit per-lane value (b0 + 2 b1 + 4 b2) into a 5-bit counter.
__device__ inline void add3(uint64_t (&a)[kSmallBits], uint64_t b0, uint64_t b1, uint64_t b2) {
    uint64_t c = a[0] & b0;
    a[0] ^= b0;
    uint64_t t = a[1] ^ b1;
    uint64_t c2 = (a[1] & b1) | (t & c);
    a[1] = t ^ c;
    c = c2;
    t = a[2] ^ b2;
    c2 = (a[2] & b2) | (t & c);
    a[2] = t ^ c;
    c = c2;
    c2 = a[3] & c;
    a[3] ^= c;
    a[4] ^= c2;
}

// big += small (5-bit), ripple carry.
__device__ inline void add_small(Vcount& v, const uint64_t (&a)[kSmallBits]) {
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < kBigBits; ++i) {
        const uint64_t x = i < kSmallBits ? a[i] : 0;
        const uint64_t t = v.big[i] ^ x;
        const uint64_t c2 = (v.big[i] & x) | (t & c);
        v.big[i] = t ^ c;
        c = c2;
    }
}

// Per-lane integer counts of a wave's vertical counters, accumulated into the
// workgroup's 64 LDS counters (lane b of the wave owns sample bit b).
__device__ inline void flush_counts(Vcount& v, uint32_t* Ublk) {
    const int lane = threadIdx.x & 63;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kBigBits; ++k) {
        for (int b = 0; b < 64; ++b) {
            const uint64_t bal = __ballot((v.big[k] >> b) & 1ull);
            const uint32_t cnt = (uint32_t)__popcll(bal);
            if (lane == b) acc += cnt << k;
        }
        v.big[k] = 0;
    }
    atomicAdd(&Ublk[lane], acc);
}

// K_u(R) = #{i : Tu[i][u] > R}; Tu[.][u] is strictly decreasing in i.
__device__ inline int k_count(const uint32_t* Tu_lds, int nk, uint32_t R, int u) {
    int K = 0;
#pragma unroll
    for (int step = 128; step > 0; step >>= 1) {
        const int c = K + step;
        if (c <= nk && Tu_lds[(c - 1) * 3 + u] > R) K = c;
    }
    return K;
}

struct SiteOut {
    uint64_t s;       // new spin word
    uint64_t f0, f1, f2;  // u_final = f0 + 2 f1 + 4 f2 (unsatisfied bonds after the move)
};

// One Metropolis site update of 64 lanes.
__device__ inline SiteOut metro(uint64_t s, uint64_t nxp, uint64_t nxm, uint64_t nyp,
                                uint64_t nym, uint64_t jxp, uint64_t jxm, uint64_t jyp,
                                uint64_t jym, uint64_t up, uint64_t dn, uint32_t R,
                                const uint64_t* ml, const uint32_t* Tu_lds, int nk) {
    // bond parities: 1 = unsatisfied
    const uint64_t p1 = s ^ nxp ^ jxp;
    const uint64_t p2 = s ^ nxm ^ jxm;
    const uint64_t p3 = s ^ nyp ^ jyp;
    const uint64_t p4 = s ^ nym ^ jym;
    const uint64_t p5 = s ^ up;
    const uint64_t p6 = s ^ dn;
    // two full adders: u = s1 + s2 + 2 (c1 + c2)
    const uint64_t s1 = p1 ^ p2 ^ p3;
    const uint64_t c1 = (p1 & p2) | (p3 & (p1 ^ p2));
    const uint64_t s2 = p4 ^ p5 ^ p6;
    const uint64_t c2 = (p4 & p5) | (p6 & (p4 ^ p5));
    const uint64_t ge1 = s1 | s2 | c1 | c2;
    const uint64_t ge2 = c1 | c2 | (s1 & s2);
    const uint64_t ge3 = (c1 & c2) | ((c1 | c2) & (s1 | s2));
    const uint64_t m0 = ml[k_count(Tu_lds, nk, R, 0)];
    const uint64_t m1 = ml[k_count(Tu_lds, nk, R, 1)];
    const uint64_t m2 = ml[k_count(Tu_lds, nk, R, 2)];
    const uint64_t flip = ge3 | (ge2 & m2) | (ge1 & m1) | m0;
    SiteOut o;
    o.s = s ^ flip;
    // after the move every bond parity toggles where flipped (u -> 6 - u)
    const uint64_t a1 = s1 ^ flip, a2 = s2 ^ flip, b1 = c1 ^ flip, b2 = c2 ^ flip;
    // u_final = a1 + a2 + 2 (b1 + b2) in binary
    const uint64_t lo = a1 ^ a2, carry = a1 & a2;
    const uint64_t mid = b1 ^ b2 ^ carry;
    const uint64_t hi = (b1 & b2) | (carry & (b1 ^ b2));
    o.f0 = lo;
    o.f1 = mid;
    o.f2 = hi;
    return o;
}

struct Geo {
    int hx, hxp, hxm, hyp, hym, p;
};

__device__ inline Geo geo_of(int xy, int L) {
    Geo g;
    const int x = xy % L, y = xy / L;
    g.p = (x + y) & 1;
    g.hx = xy >> 1;
    g.hxp = (((x + 1) % L) + L * y) >> 1;
    g.hxm = (((x + L - 1) % L) + L * y) >> 1;
    g.hyp = (x + L * ((y + 1) % L)) >> 1;
    g.hym = (x + L * ((y + L - 1) % L)) >> 1;
    return g;
}

// A thread's words of one chunk, split by colour: A[m] is its colour-0 site
// at local plane p + 2m, B[m] its colour-1 site at local plane 1 - p + 2m
// (p = (x + y) mod 2).  In this order the temporal neighbours are fixed
// register slots selected by p, so no register array is indexed at run time.
struct Chunk {
    uint64_t A[4], B[4];
};

__device__ inline void load_chunk(Chunk& c, const uint64_t* col, int q, int p, int L2, bool active) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        c.A[m] = active ? col[(size_t)(kChunk * q + p + 2 * m) * L2] : 0;
        c.B[m] = active ? col[(size_t)(kChunk * q + 1 - p + 2 * m) * L2] : 0;
    }
}

__device__ inline void store_chunk(const Chunk& c, uint64_t* col, int q, int p, int L2) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        col[(size_t)(kChunk * q + p + 2 * m) * L2] = c.A[m];
        col[(size_t)(kChunk * q + 1 - p + 2 * m) * L2] = c.B[m];
    }
}

__global__ void __launch_bounds__(kMaxThreads) k_sweep_fused(ShapeDev sh, uint32_t key0, uint32_t key1,
                                                      const Counters* __restrict__ ctr) {
    extern __shared__ uint64_t lds[];
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, W = sh.W;
    const int H = L2 >> 1;  // half-plane words
    uint64_t* c1_old = lds;                      // [8][H]  colour-1 words of chunk q (old)
    uint64_t* c0_new = lds + kChunk * H;         // [8][H]  colour-0 words of chunk q-1 (new)
    uint64_t* ml = lds + 2 * kChunk * H;         // [nk+1] lane masks
    uint32_t* Tu_lds = (uint32_t*)(ml + nk + 1); // [nk][3]
    uint32_t* Ublk = Tu_lds + 3 * nk;            // [64]

    const int cfg = blockIdx.x;  // ((r*nk + w)*W + j)
    const int j = cfg % W;
    const int rw = cfg / W;
    const int w = rw % nk;
    const int r = rw / nk;
    const int tid = threadIdx.x;
    const bool active = tid < L2;

    for (int i = tid; i <= nk; i += blockDim.x)
        ml[i] = sh.mask[((size_t)(r * W + j) * nk + w) * (nk + 1) + i];
    for (int i = tid; i < 3 * nk; i += blockDim.x) Tu_lds[i] = sh.Tu[i];
    if (tid < 64) Ublk[tid] = 0;

    const uint32_t t = ctr->t;
    const uint32_t c3 = ctr_word3(sh.word_offset + (uint32_t)j, sh.sid, kTagMetro);
    const uint32_t c2base = (uint32_t)rw << 1;

    const int xy = active ? tid : 0;
    const Geo g = geo_of(xy, L);
    const int p = g.p;
    const int x = xy % L, y = xy / L;
    const uint64_t* Jb = sh.J + (size_t)j * 2 * L2;
    uint64_t jxp = 0, jxm = 0, jyp = 0, jym = 0;
    if (active) {
        jxp = Jb[xy];
        jxm = Jb[((x + L - 1) % L) + L * y];
        jyp = Jb[L2 + xy];
        jym = Jb[L2 + x + L * ((y + L - 1) % L)];
    }
    uint64_t* col = sh.S + (size_t)cfg * Lt * L2 + xy;
    const int hA = g.hx, hB = g.hx;
    const int planeA = p, planeB = 1 - p;  // local plane of A[0], B[0]

    const int nq = Lt / kChunk;
    Chunk cur, nxt, prv;
    // plane Ltau-1 (colour 1 when p = 0) before the sweep: the tau-wrap
    // neighbour of the first colour-0 site of column parity 0.  Words used
    // across the tau wrap are complemented when the boundary is
    // antiperiodic (apm = all ones): the wrap bond has the sign -1.
    const uint64_t apm = sh.apm;
    const uint64_t lastplane_old = active ? col[(size_t)(Lt - 1) * L2] ^ apm : 0;
    uint64_t A0_first_new = 0;   // chunk 0, A[0] after colour 0
    uint64_t B0_first_old = 0;   // chunk 0, B[0] before the sweep
    uint64_t App3 = 0;           // chunk q-2, A[3] (final)
    uint32_t Rdef = 0;
    Vcount vc;
#pragma unroll
    for (int i = 0; i < kBigBits; ++i) vc.big[i] = 0;
    uint64_t small[kSmallBits];
#pragma unroll
    for (int m = 0; m < 4; ++m) prv.A[m] = prv.B[m] = 0;

    load_chunk(nxt, col, 0, p, L2, active);
    B0_first_old = nxt.B[0];
    __syncthreads();  // ml, Tu_lds, Ublk ready

    for (int q = 0; q < nq; ++q) {
        cur = nxt;
        if (q + 1 < nq) load_chunk(nxt, col, q + 1, p, L2, active);
        if (active) {
#pragma unroll
            for (int m = 0; m < 4; ++m) c1_old[(planeB + 2 * m) * H + hB] = cur.B[m];
        }
        __syncthreads();
        if (active) {
            // colour 0 of chunk q: neighbours along tau are colour-1 words (old)
            const U4 R4 = philox10((uint32_t)(xy + L2 * q), t, c2base | 0u, c3, key0, key1);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const uint64_t dn_p0 = m > 0 ? cur.B[m > 0 ? m - 1 : 0]
                                             : (q > 0 ? prv.B[3] : lastplane_old);
                const uint64_t up_p1 = m < 3 ? cur.B[m < 3 ? m + 1 : 3]
                                             : (q + 1 < nq ? nxt.B[0] : B0_first_old ^ apm);
                const uint64_t dn = p ? cur.B[m] : dn_p0;
                const uint64_t up = p ? up_p1 : cur.B[m];
                const uint64_t* P = c1_old + (planeA + 2 * m) * H;
                const SiteOut o = metro(cur.A[m], P[g.hxp], P[g.hxm], P[g.hyp], P[g.hym], jxp,
                                        jxm, jyp, jym, up, dn, R4.v[m], ml, Tu_lds, nk);
                cur.A[m] = o.s;
            }
            if (q == 0) A0_first_new = cur.A[0];
            // colour 1 of chunk q-1: neighbours along tau are colour-0 words (new)
            if (q >= 1) {
                const int cq = q - 1;
                const U4 R4b = philox10((uint32_t)(xy + L2 * cq), t, c2base | 1u, c3, key0, key1);
#pragma unroll
                for (int i = 0; i < kSmallBits; ++i) small[i] = 0;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    if (m == 0 && cq == 0 && p == 1) {
                        Rdef = R4b.v[0];  // plane 0: deferred to the end
                        continue;
                    }
                    const uint64_t dn_p1 = m > 0 ? prv.A[m > 0 ? m - 1 : 0] : App3;
                    const uint64_t up_p0 = m < 3 ? prv.A[m < 3 ? m + 1 : 3] : cur.A[0];
                    const uint64_t dn = p ? dn_p1 : prv.A[m];
                    const uint64_t up = p ? prv.A[m] : up_p0;
                    const uint64_t* P = c0_new + (planeB + 2 * m) * H;
                    const SiteOut o = metro(prv.B[m], P[g.hxp], P[g.hxm], P[g.hyp], P[g.hym], jxp,
                                            jxm, jyp, jym, up, dn, R4b.v[m], ml, Tu_lds, nk);
                    prv.B[m] = o.s;
                    add3(small, o.f0, o.f1, o.f2);
                }
                add_small(vc, small);
                store_chunk(prv, col, cq, p, L2);
            }
        }
        if (q >= 1 && (q % kFlushChunks) == 0) flush_counts(vc, Ublk);
        __syncthreads();
        if (active) {
#pragma unroll
            for (int m = 0; m < 4; ++m) c0_new[(planeA + 2 * m) * H + hA] = cur.A[m];
        }
        App3 = prv.A[3];
        prv = cur;
    }
    __syncthreads();  // colour-0 words of the last chunk visible
    if (active) {
        const int cq = nq - 1;
        const U4 R4b = philox10((uint32_t)(xy + L2 * cq), t, c2base | 1u, c3, key0, key1);
#pragma unroll
        for (int i = 0; i < kSmallBits; ++i) small[i] = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (m == 0 && cq == 0 && p == 1) {
                Rdef = R4b.v[0];
                continue;
            }
            const uint64_t dn_p1 = m > 0 ? prv.A[m > 0 ? m - 1 : 0] : App3;
            const uint64_t up_p0 = m < 3 ? prv.A[m < 3 ? m + 1 : 3] : A0_first_new ^ apm;
            const uint64_t dn = p ? dn_p1 : prv.A[m];
            const uint64_t up = p ? prv.A[m] : up_p0;
            const uint64_t* P = c0_new + (planeB + 2 * m) * H;
            const SiteOut o = metro(prv.B[m], P[g.hxp], P[g.hxm], P[g.hyp], P[g.hym], jxp, jxm,
                                    jyp, jym, up, dn, R4b.v[m], ml, Tu_lds, nk);
            prv.B[m] = o.s;
            add3(small, o.f0, o.f1, o.f2);
        }
        add_small(vc, small);
        store_chunk(prv, col, cq, p, L2);
    }
    __syncthreads();
    // deferred colour-1 sites of plane 0 (columns with x + y odd): their
    // spatial neighbours are the final colour-0 words of plane 0
    if (active && p == 0) c0_new[hA] = A0_first_new;
    __syncthreads();
    if (active && p == 1) {
        const uint64_t* P = c0_new;
#pragma unroll
        for (int i = 0; i < kSmallBits; ++i) small[i] = 0;
        // tau-1 = Ltau-1 is the last chunk's A[3] (across the wrap); tau+1 = 1
        // is chunk 0's A[0]
        const SiteOut o = metro(B0_first_old, P[g.hxp], P[g.hxm], P[g.hyp], P[g.hym], jxp, jxm,
                                jyp, jym, A0_first_new, prv.A[3] ^ apm, Rdef, ml, Tu_lds, nk);
        col[0] = o.s;
        add3(small, o.f0, o.f1, o.f2);
        add_small(vc, small);
    }
    flush_counts(vc, Ublk);
    __syncthreads();
    if (tid < 64) sh.U[((size_t)r * W * 64 + (size_t)j * 64 + tid) * nk + w] = Ublk[tid];
}

// Energy recount of every configuration (used after initialisation and
// state import): each site counts its +x, +y and +tau bonds.
__global__ void __launch_bounds__(kMaxThreads) k_energy(ShapeDev sh) {
    extern __shared__ uint64_t lds[];
    uint32_t* Ublk = (uint32_t*)lds;
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, W = sh.W;
    const int cfg = blockIdx.x;
    const int j = cfg % W;
    const int rw = cfg / W;
    const int w = rw % nk;
    const int r = rw / nk;
    const int tid = threadIdx.x;
    const bool active = tid < L2;
    if (tid < 64) Ublk[tid] = 0;
    __syncthreads();
    Vcount vc;
#pragma unroll
    for (int i = 0; i < kBigBits; ++i) vc.big[i] = 0;
    uint64_t small[kSmallBits];
    const int xy = active ? tid : 0;
    const int x = xy % L, y = xy / L;
    const int xp = ((x + 1) % L) + L * y, yp = x + L * ((y + 1) % L);
    const uint64_t* Jb = sh.J + (size_t)j * 2 * L2;
    const uint64_t jx = active ? Jb[xy] : 0, jy = active ? Jb[L2 + xy] : 0;
    const uint64_t* base = sh.S + (size_t)cfg * Lt * L2;
    for (int q = 0; q * kChunk < Lt; ++q) {
#pragma unroll
        for (int i = 0; i < kSmallBits; ++i) small[i] = 0;
        if (active) {
            for (int l = 0; l < kChunk && kChunk * q + l < Lt; ++l) {
                const int tau = kChunk * q + l;
                const uint64_t* P = base + (size_t)tau * L2;
                const uint64_t s = P[xy];
                const uint64_t bx = s ^ P[xp] ^ jx;
                const uint64_t by = s ^ P[yp] ^ jy;
                const uint64_t bt = s ^ base[(size_t)((tau + 1) % Lt) * L2 + xy] ^
                                    (tau == Lt - 1 ? sh.apm : 0ull);  // the wrap bond
                add3(small, bx ^ by ^ bt, (bx & by) | (bt & (bx ^ by)), 0);
            }
        }
        add_small(vc, small);
        if (q >= 1 && (q % kFlushChunks) == 0) flush_counts(vc, Ublk);
    }
    flush_counts(vc, Ublk);
    __syncthreads();
    if (tid < 64) sh.U[((size_t)r * W * 64 + (size_t)j * 64 + tid) * nk + w] = Ublk[tid];
}

size_t sweep_lds_bytes(const ShapeDev& sh) {
    return (size_t)(2 * kChunk * (sh.L2 / 2) + sh.nk + 1) * 8 + (size_t)3 * sh.nk * 4 + 64 * 4;
}

int block_for(const ShapeDev& sh) { return ((sh.L2 + 63) / 64) * 64; }

}  // namespace

int sweep_variants() { return 4; }
const char* sweep_variant_name(int v) {
    switch (v) {
        case 0: return "stream";
        case 1: return "chunk8";
        case 2: return "stream-occ5";
        case 3: return "stream-helped";
        default: return "?";
    }
}

hipError_t launch_sweep(const ShapeDev& sh, uint64_t seed, const Counters* ctr, int variant,
                        bool energy, hipStream_t st) {
    if (variant == 3 && sweep_helped_ok(sh)) return launch_sweep_helped(sh, seed, ctr, energy, st);
    if ((variant == 0 || variant == 2 || variant == 3) && sweep_stream_ok(sh))
        return launch_sweep_stream(sh, seed, ctr, energy, variant == 2 ? 5 : 1, st);
    const int nblk = sh.R * sh.nk * sh.W;
    hipLaunchKernelGGL(k_sweep_fused, dim3(nblk), dim3(block_for(sh)), sweep_lds_bytes(sh), st, sh,
                       (uint32_t)seed, (uint32_t)(seed >> 32), ctr);
    return hipGetLastError();
}

hipError_t prepare_sweep(const ShapeDev& sh, int variant, bool energy) {
    if (variant == 3 && sweep_helped_ok(sh)) return prepare_sweep_helped(sh, energy);
    if ((variant == 0 || variant == 2 || variant == 3) && sweep_stream_ok(sh))
        return prepare_sweep_stream(sh, energy, variant == 2 ? 5 : 1);
    return hipSuccess;  // the chunked kernel stays within 64 KiB of LDS
}

hipError_t launch_energy(const ShapeDev& sh, hipStream_t st) {
    const int nblk = sh.R * sh.nk * sh.W;
    hipLaunchKernelGGL(k_energy, dim3(nblk), dim3(block_for(sh)), 64 * 4, st, sh);
    return hipGetLastError();
}

}  // namespace tfim
