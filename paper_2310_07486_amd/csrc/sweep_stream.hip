// Multispin checkerboard Metropolis sweep, streaming form (the default).
//
// Paper: arXiv:2310.07486, Methods, "The Trotter-Suzuki formula" (action,
// p(S) = exp(-k E)/Z, periodic tau) and "Simulation details" (full-lattice
// Metropolis sweeps, multispin coding, tempering over k).
//
// One workgroup sweeps one configuration (replica r, walker w, word j); one
// thread owns one spatial column xy (parity p = (x+y) mod 2).  Segment
// sigma updates the thread's colour-0 site at plane A = 2 sigma + p and, one
// segment behind, its colour-1 site of the previous step at plane A - 3, so
// both colours are fused into one pass over tau with ONE workgroup barrier
// per segment (two planes):
//   - colour 0 at A needs the old colour-1 words at A-1, A+1 (own column,
//     registers) and the old colour-1 words of the four spatial neighbours
//     at A (published in LDS buffer X before the barrier);
//   - colour 1 at A-3 needs the new colour-0 words at A-4, A-2 (registers)
//     and the new colour-0 words of the neighbours at A-3 (LDS buffer Y).
// X and Y are double-buffered by segment parity.  A thread keeps a window of
// planes A-4 .. A+5 in registers (two in flight), so every spin word is read
// once and written once per sweep.  The colour-1 site of step 0 needs colour
// 0 of plane Ltau-1, known only at the end: it is updated in one extra
// segment, where the periodic tau wrap brings exactly the right words back
// through the same pipeline.
//
// Per site and lane: u = number of unsatisfied bonds among six (bond parities
// and two full adders on v_bitop3); the move (dE = 12 - 4u) is taken iff
// u >= 3 or R < Tu[k-index][u].  The uniform R is shared by the 64 lanes; the
// lanes sit at different k-indices, and {lanes : R < Tu[kidx][u]} is a lane
// mask selected by K_u(R) = #{i : Tu[i][u] > R}, looked up in a bucket table
// over the top bits of R whose entries carry the two candidate masks.
// The colour-1 update also yields, per lane, the number of unsatisfied bonds
// of its site in the final state; summing it over the colour-1 sites gives U
// exactly (every bond joins a colour-0 and a colour-1 site).
#include <type_traits>

#include "tfim_internal.h"

namespace tfim {
namespace {

constexpr int kMaxCols = 576;  // one thread per column, L <= 24

// v_bitop3: bit i of the immediate is f(a_i, b_i, c_i) with the operands
// weighted 0xF0 (a), 0xCC (b), 0xAA (c).
constexpr uint32_t kA = 0xF0, kB = 0xCC, kC = 0xAA;
constexpr uint32_t kXor3 = (kA ^ kB ^ kC) & 0xFF;
constexpr uint32_t kMaj = ((kA & kB) | (kA & kC) | (kB & kC)) & 0xFF;
constexpr uint32_t kOr3 = (kA | kB | kC) & 0xFF;
constexpr uint32_t kAorBandC = (kA | (kB & kC)) & 0xFF;       // a | (b & c)
constexpr uint32_t kAandBorC = ((kA & kB) | kC) & 0xFF;       // (a & b) | c
constexpr uint32_t kAxorBorC = (kA ^ (kB | kC)) & 0xFF;       // a ^ (b | c)
constexpr uint32_t kBothIfC = ((~kA & ~kB & kC) | (kA & kB & ~kC)) & 0xFF;  // c ? ~a&~b : a&b

template <uint32_t IMM>
__device__ __forceinline__ uint64_t b3(uint64_t a, uint64_t b, uint64_t c) {
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, IMM);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32),
                                                    (uint32_t)(c >> 32), IMM);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t xor3_32(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, kXor3);
}

// Philox4x32-10 with three-input XORs (same function as philox10).
__device__ __forceinline__ U4 philox_dev(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t key0, uint32_t key1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_32((uint32_t)(pb >> 32), c1, key0);
        const uint32_t n2 = xor3_32((uint32_t)(pa >> 32), c3, key1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        key0 += 0x9E3779B9u;
        key1 += 0xBB67AE85u;
    }
    U4 r;
    r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
    return r;
}

struct Nb {
    uint64_t xp, xm, yp, ym;
};

struct Tables {
    const uint32_t* T[3];  // Tstar per bucket
    const uint64_t* M[3];  // (mask below, mask above) per bucket
    uint32_t sh[3], nb[3];
};

__device__ __forceinline__ uint64_t lane_mask(const Tables& tb, int u, uint32_t R) {
    const uint32_t a = min(R >> tb.sh[u], tb.nb[u]);
    const uint32_t T = tb.T[u][a];
    const uint64_t lo = tb.M[u][2 * a], hi = tb.M[u][2 * a + 1];
    return R < T ? hi : lo;
}

// One site of 64 lanes.  Returns the new word; if kE, also the three bits of
// the final unsatisfied-bond count (f0 + 2 f1 + 4 f2).
template <bool kE>
__device__ __forceinline__ uint64_t site(uint64_t s, const Nb& n, uint64_t jxp, uint64_t jxm,
                                         uint64_t jyp, uint64_t jym, uint64_t up, uint64_t dn,
                                         uint32_t R, const Tables& tb, uint64_t& f0, uint64_t& f1,
                                         uint64_t& f2) {
    const uint64_t p1 = b3<kXor3>(s, n.xp, jxp);
    const uint64_t p2 = b3<kXor3>(s, n.xm, jxm);
    const uint64_t p3 = b3<kXor3>(s, n.yp, jyp);
    const uint64_t p4 = b3<kXor3>(s, n.ym, jym);
    const uint64_t p5 = s ^ up;
    const uint64_t p6 = s ^ dn;
    const uint64_t s1 = b3<kXor3>(p1, p2, p3);
    const uint64_t c1 = b3<kMaj>(p1, p2, p3);
    const uint64_t s2 = b3<kXor3>(p4, p5, p6);
    const uint64_t c2 = b3<kMaj>(p4, p5, p6);
    const uint64_t so = s1 | s2;
    const uint64_t co = c1 | c2;
    const uint64_t ge1 = so | co;                     // u >= 1
    const uint64_t ge2 = b3<kAorBandC>(co, s1, s2);   // u >= 2
    const uint64_t ge3 = b3<kMaj>(c1, c2, so);        // u >= 3
    const uint64_t m0 = lane_mask(tb, 0, R);
    const uint64_t m1 = lane_mask(tb, 1, R);
    const uint64_t m2 = lane_mask(tb, 2, R);
    // masks are nested (m0 in m1 in m2): flip = ge3 | ge2&m2 | ge1&m1 | m0
    const uint64_t t1 = b3<kAandBorC>(ge2, m2, m0);
    const uint64_t t2 = b3<kAandBorC>(ge1, m1, t1);
    if constexpr (kE) {
        const uint64_t f = ge3 | t2;
        // after the move the six parities toggle where flipped: counts are
        // (s1^f) + (s2^f) + 2 (c1^f) + 2 (c2^f)
        const uint64_t y1 = b3<kBothIfC>(s1, s2, f);  // (s1^f) & (s2^f)
        const uint64_t y2 = b3<kBothIfC>(c1, c2, f);  // (c1^f) & (c2^f)
        const uint64_t x2 = c1 ^ c2;
        f0 = s1 ^ s2;
        f1 = x2 ^ y1;
        f2 = b3<kAorBandC>(y2, x2, y1);
    }
    return b3<kAxorBorC>(s, ge3, t2);  // s ^ flip
}

// 5-bit per-lane counter += 3-bit value.
__device__ __forceinline__ void add3v(uint64_t (&a)[5], uint64_t f0, uint64_t f1, uint64_t f2) {
    uint64_t k = a[0] & f0;
    a[0] ^= f0;
    const uint64_t k1 = b3<kMaj>(a[1], f1, k);
    a[1] = b3<kXor3>(a[1], f1, k);
    const uint64_t k2 = b3<kMaj>(a[2], f2, k1);
    a[2] = b3<kXor3>(a[2], f2, k1);
    const uint64_t k3 = a[3] & k2;
    a[3] ^= k2;
    a[4] ^= k3;
}

constexpr int kDeep = 12;          // per-thread counter bits (kept in LDS)
constexpr int kFlushMacros = 128;  // 128 * 24 < 2^12

// deep += small (5 bits), ripple carry; deep lives in LDS, plane k of
// thread t at d[k * stride + t].
__device__ __forceinline__ void add_deep(uint64_t* d, int stride, uint64_t (&a)[5]) {
    uint64_t k = 0;
#pragma unroll
    for (int i = 0; i < kDeep; ++i) {
        const uint64_t v = d[i * stride];
        if (i < 5) {
            const uint64_t nk = b3<kMaj>(v, a[i], k);
            d[i * stride] = b3<kXor3>(v, a[i], k);
            k = nk;
            a[i] = 0;
        } else {
            d[i * stride] = v ^ k;
            k = v & k;
        }
    }
}

// Per-lane sums of the workgroup's vertical counters into Ublk[64].
__device__ void flush_deep(uint64_t* d, int stride, uint32_t* Ublk) {
    const int lane = threadIdx.x & 63;
    uint32_t acc = 0;
    for (int k = 0; k < kDeep; ++k) {
        const uint64_t v = d[k * stride];
        for (int b = 0; b < 64; ++b) {
            const uint32_t cnt = (uint32_t)__popcll(__ballot((v >> b) & 1ull));
            acc += (lane == b) ? (cnt << k) : 0u;
        }
        d[k * stride] = 0;
    }
    atomicAdd(&Ublk[lane], acc);
}

// kOcc: minimum waves per SIMD the register allocation must allow (1 = no
// constraint); a tuning knob, the results do not depend on it.
template <bool kE, int kOcc>
__global__ void __launch_bounds__(kMaxCols) __attribute__((amdgpu_waves_per_eu(kOcc)))
k_sweep_stream(ShapeDev sh, uint32_t key0,
                                                           uint32_t key1,
                                                           const Counters* __restrict__ ctr) {
    extern __shared__ uint64_t lds[];
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, W = sh.W;
    // X, Y: one word per column (each column publishes the word at its own,
    // parity-dependent plane; its four neighbours have the other parity).
    const int H = L2;
    uint64_t* X = lds;           // [2][L2] colour-1 words (old) for the colour-0 step
    uint64_t* Y = lds + 2 * H;   // [2][L2] colour-0 words (new) for the colour-1 step
    uint64_t* ml = lds + 4 * H;  // [nk+1] lane masks of this walker and word
    uint64_t* MM = ml + nk + 1;  // bucket masks, all u
    const int nb0 = sh.bnb[0] + 1, nb1 = sh.bnb[1] + 1, nb2 = sh.bnb[2] + 1;
    uint64_t* DEEP = MM + 2 * (nb0 + nb1 + nb2);  // [kDeep][blockDim] energy counters
    uint32_t* TT = (uint32_t*)(DEEP + (kE ? kDeep * blockDim.x : 0));
    uint32_t* Ublk = TT + nb0 + nb1 + nb2;

    const int cfg = blockIdx.x;  // ((r*nk + w)*W + j)
    const int j = cfg % W;
    const int rw = cfg / W;
    const int w = rw % nk;
    const int r = rw / nk;
    const int tid = threadIdx.x;
    const bool active = tid < L2;

    for (int i = tid; i <= nk; i += blockDim.x)
        ml[i] = sh.mask[((size_t)(r * W + j) * nk + w) * (nk + 1) + i];
    if (kE && tid < 64) Ublk[tid] = 0;
    if (kE)
        for (int i = 0; i < kDeep; ++i) DEEP[i * blockDim.x + tid] = 0;
    __syncthreads();
    {
        const int nbs[3] = {nb0, nb1, nb2};
        int base = 0;
        for (int u = 0; u < 3; ++u) {
            for (int a = tid; a < nbs[u]; a += blockDim.x) {
                const uint64_t e = sh.btab[sh.boff[u] + a];
                const uint32_t kb = (uint32_t)(e >> 32) & 0xFFFFu, mu = (uint32_t)(e >> 48);
                TT[base + a] = (uint32_t)e;
                MM[2 * (base + a)] = ml[kb];
                MM[2 * (base + a) + 1] = ml[kb + mu];
            }
            base += nbs[u];
        }
    }
    Tables tb;
    tb.T[0] = TT; tb.T[1] = TT + nb0; tb.T[2] = TT + nb0 + nb1;
    tb.M[0] = MM; tb.M[1] = MM + 2 * nb0; tb.M[2] = MM + 2 * (nb0 + nb1);
    for (int u = 0; u < 3; ++u) {
        tb.sh[u] = (uint32_t)sh.bsh[u];
        tb.nb[u] = (uint32_t)sh.bnb[u];
    }

    const uint32_t t = ctr->t;
    const uint32_t c3 = ctr_word3(sh.word_offset + (uint32_t)j, sh.sid, kTagMetro);
    const uint32_t c2_0 = (uint32_t)rw << 1, c2_1 = c2_0 | 1u;

    const int xy = active ? tid : 0;
    const int x = xy % L, y = xy / L;
    const int p = (x + y) & 1;
    const int hx = xy;
    const int hxp = ((x + 1) % L) + L * y;
    const int hxm = ((x + L - 1) % L) + L * y;
    const int hyp = x + L * ((y + 1) % L);
    const int hym = x + L * ((y + L - 1) % L);
    const uint64_t* Jb = sh.J + (size_t)j * 2 * L2;
    uint64_t jxp = 0, jxm = 0, jyp = 0, jym = 0;
    if (active) {
        jxp = Jb[xy];
        jxm = Jb[((x + L - 1) % L) + L * y];
        jyp = Jb[L2 + xy];
        jym = Jb[L2 + x + L * ((y + L - 1) % L)];
    }
    uint64_t* col = sh.S + (size_t)cfg * Lt * L2 + xy;
    const int half = Lt >> 1;      // colour-0 steps
    const int nq = Lt >> 3;        // Philox groups per colour and column
    auto wrap = [Lt](int P) { return P >= Lt ? P - Lt : (P < 0 ? P + Lt : P); };
    auto ld = [&](int P) -> uint64_t {
        return (active && P <= Lt + 1) ? col[(size_t)wrap(P) * L2] : 0ull;
    };

    // window: w0..w5 = planes A-4 .. A+1, pf = A+2, A+3, nx = A+4, A+5
    uint64_t w0 = 0, w1 = 0, w2 = 0, w3, w4, w5, pf0, pf1, nx0, nx1;
    w3 = ld(p - 1);
    w4 = ld(p);
    w5 = ld(p + 1);
    pf0 = ld(p + 2);
    pf1 = ld(p + 3);
    U4 G0, G1;
    uint32_t prevlast = 0;
    uint64_t sm[5] = {0, 0, 0, 0, 0};
    uint64_t* deep = DEEP + tid;
    const int dstride = blockDim.x;
    uint64_t f0 = 0, f1 = 0, f2 = 0;

    if (active) X[hx] = p ? w3 : w5;  // X(0)
    __syncthreads();

    // one segment; IS = sigma & 3 is a compile-time constant
    auto segment = [&](const int sigma, const auto ISc, const bool do_c0, const bool do_c1) {
        constexpr int IS = decltype(ISc)::value;
        const int A = 2 * sigma + p;
        nx0 = ld(A + 4);
        nx1 = ld(A + 5);
        if (do_c0) {
            if (IS == 0) G0 = philox_dev((uint32_t)(xy + L2 * (sigma >> 2)), t, c2_0, c3, key0, key1);
            const uint64_t* Xb = X + (IS & 1) * H;
            const Nb n{Xb[hxp], Xb[hxm], Xb[hyp], Xb[hym]};
            uint64_t d0, d1, d2;
            w4 = site<false>(w4, n, jxp, jxm, jyp, jym, w5, w3, G0.v[IS], tb, d0, d1, d2);
            if (active) col[(size_t)A * L2] = w4;
        }
        if (IS == 1) {  // colour-1 Philox group of step s = sigma - 1 (s % 4 == 0)
            prevlast = G1.v[3];
            int q = (sigma - 1) >> 2;
            if (q >= nq) q -= nq;
            G1 = philox_dev((uint32_t)(xy + L2 * q), t, c2_1, c3, key0, key1);
        }
        if (do_c1) {
            constexpr int S3 = (IS + 3) & 3;  // (sigma - 1) & 3
            const uint32_t R1 = p ? G1.v[S3] : (S3 == 0 ? prevlast : G1.v[(S3 + 3) & 3]);
            const uint64_t* Yb = Y + ((IS + 1) & 1) * H;
            const Nb n{Yb[hxp], Yb[hxm], Yb[hyp], Yb[hym]};
            w1 = site<kE>(w1, n, jxp, jxm, jyp, jym, w2, w0, R1, tb, f0, f1, f2);
            if (kE && active) add3v(sm, f0, f1, f2);  // padding threads count nothing
            if (active) col[(size_t)wrap(A - 3) * L2] = w1;
        }
        if (active) {
            Y[(IS & 1) * H + hx] = p ? w2 : w4;
            X[((IS + 1) & 1) * H + hx] = p ? w5 : pf1;
        }
        __syncthreads();
        w0 = w2; w1 = w3; w2 = w4; w3 = w5; w4 = pf0; w5 = pf1; pf0 = nx0; pf1 = nx1;
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;

    for (int g = 0; g < nq; ++g) {
        const int s0 = 4 * g;
        segment(s0 + 0, I0{}, true, g > 0);
        segment(s0 + 1, I1{}, true, g > 0);
        segment(s0 + 2, I2{}, true, true);
        segment(s0 + 3, I3{}, true, true);
        if (kE) {
            add_deep(deep, dstride, sm);
            if ((g % kFlushMacros) == kFlushMacros - 1) flush_deep(deep, dstride, Ublk);
        }
    }
    segment(half, I0{}, false, true);      // colour 1, step half-1
    segment(half + 1, I1{}, false, true);  // colour 1, step half == step 0 (tau wrap)
    if (kE) {
        add_deep(deep, dstride, sm);
        flush_deep(deep, dstride, Ublk);
        __syncthreads();
        if (tid < 64) sh.U[((size_t)r * W * 64 + (size_t)j * 64 + tid) * nk + w] = Ublk[tid];
    }
}

}  // namespace

size_t sweep_stream_lds_bytes(const ShapeDev& sh) {
    const size_t nb = (size_t)(sh.bnb[0] + 1) + (sh.bnb[1] + 1) + (sh.bnb[2] + 1);
    const size_t threads = ((sh.L2 + 63) / 64) * 64;
    return (size_t)(4 * sh.L2 + sh.nk + 1) * 8 + nb * 16 + threads * kDeep * 8 + nb * 4 + 64 * 4;
}

bool sweep_stream_ok(const ShapeDev& sh) {
    return sh.bnb[0] >= 0 && sh.bnb[1] >= 0 && sh.bnb[2] >= 0 && sh.L2 <= kMaxCols &&
           (sh.Lt % 8) == 0 && sh.Lt >= 8;
}

template <bool kE, int kOcc>
static hipError_t launch_one(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st) {
    const int nblk = sh.R * sh.nk * sh.W;
    const int threads = ((sh.L2 + 63) / 64) * 64;
    const size_t lds = sweep_stream_lds_bytes(sh);
    static size_t lds_set = 0;  // dynamic LDS above 64 KiB must be allowed per kernel
    if (lds > lds_set) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_sweep_stream<kE, kOcc>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = lds;
    }
    hipLaunchKernelGGL((k_sweep_stream<kE, kOcc>), dim3(nblk), dim3(threads), lds, st, sh,
                       (uint32_t)seed, (uint32_t)(seed >> 32), ctr);
    return hipGetLastError();
}

hipError_t launch_sweep_stream(const ShapeDev& sh, uint64_t seed, const Counters* ctr,
                               bool energy, int occ, hipStream_t st) {
    if (occ >= 5)
        return energy ? launch_one<true, 5>(sh, seed, ctr, st) : launch_one<false, 5>(sh, seed, ctr, st);
    return energy ? launch_one<true, 1>(sh, seed, ctr, st) : launch_one<false, 1>(sh, seed, ctr, st);
}

}  // namespace tfim
