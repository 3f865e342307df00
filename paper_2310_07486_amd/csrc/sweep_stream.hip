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
constexpr int kMaxBatchThreads = 768;  // 12 waves: 3 per SIMD at up to 168 VGPRs

// Raw buffer access to one configuration's spin words: the descriptor covers
// exactly its bytes (0 for a team without a configuration: loads return 0
// and stores are dropped), the plane offset is a scalar.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ uint64_t buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return ((uint64_t)v.y << 32) | v.x;
}

__device__ __forceinline__ void buf_store(uint64_t x, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    u32x2 v;
    v.x = (unsigned)x;
    v.y = (unsigned)(x >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
}

// v_bitop3: bit i of the immediate is f(a_i, b_i, c_i) with the operands
// weighted 0xF0 (a), 0xCC (b), 0xAA (c).
constexpr uint32_t kA = 0xF0, kB = 0xCC, kC = 0xAA;
constexpr uint32_t kXor3 = (kA ^ kB ^ kC) & 0xFF;
constexpr uint32_t kMaj = ((kA & kB) | (kA & kC) | (kB & kC)) & 0xFF;
constexpr uint32_t kOr3 = (kA | kB | kC) & 0xFF;
constexpr uint32_t kAorBandC = (kA | (kB & kC)) & 0xFF;       // a | (b & c)
constexpr uint32_t kAandBorC = ((kA & kB) | kC) & 0xFF;       // (a & b) | c
constexpr uint32_t kAxorBorC = (kA ^ (kB | kC)) & 0xFF;       // a ^ (b | c)
constexpr uint32_t kAxorBandNotC = (kA ^ (kB & ~kC)) & 0xFF;      // a ^ (b & ~c)
constexpr uint32_t kAandNotBandNotC = (kA & ~kB & ~kC) & 0xFF;    // a & ~b & ~c

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

// Philox4x32-10 with three-input XORs (same function as philox10).  The
// four outputs are one vector value, so a parity select between two of them
// stays in registers.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 philox_dev(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
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
    u32x4 r;
    r.x = c0;
    r.y = c1;
    r.z = c2;
    r.w = c3;
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

// The threshold is read first, then only the mask it selects (12 bytes of
// LDS per lane instead of 20): entry 2a + (R < T) of M.  The index is the
// borrow of R - T carried into a + a, two ALU instructions.
__device__ __forceinline__ uint32_t mask_index(const Tables& tb, int u, uint32_t R) {
    const uint32_t a = min(R >> tb.sh[u], tb.nb[u]);
    const uint32_t T = tb.T[u][a];
    uint32_t diff, idx;
    asm("v_sub_co_u32 %0, vcc, %2, %3\n\tv_addc_co_u32 %1, vcc, %4, %4, vcc"
        : "=&v"(diff), "=v"(idx)
        : "v"(R), "v"(T), "v"(a)
        : "vcc");
    return idx;
}

__device__ __forceinline__ uint64_t lane_mask(const Tables& tb, int u, uint32_t R) {
    return tb.M[u][mask_index(tb, u, R)];
}

// One site of 64 lanes given the three lane masks m_u = {lanes : R <
// T[kidx][u]}.  Returns the new word; if kE, also the three bits of the
// final unsatisfied-bond count (f0 + 2 f1 + 4 f2).
template <bool kE>
__device__ __forceinline__ uint64_t site_m(uint64_t s, const Nb& n, uint64_t jxp, uint64_t jxm,
                                           uint64_t jyp, uint64_t jym, uint64_t up, uint64_t dn,
                                           uint64_t m0, uint64_t m1, uint64_t m2, uint64_t& f0,
                                           uint64_t& f1, uint64_t& f2) {
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
    // u = s1 + s2 + 2 (c1 + c2) = u0 + 2 u1 + 4 u2
    const uint64_t u0 = s1 ^ s2;
    const uint64_t h = s1 & s2;
    const uint64_t u1 = b3<kXor3>(c1, c2, h);
    const uint64_t u2 = b3<kMaj>(c1, c2, h);
    // masks are nested (m0 in m1 in m2): flip = u2 | u1 (u0 | m2) | u0 m1 | m0
    const uint64_t w1 = b3<kAandBorC>(u0, m1, m0);
    const uint64_t w2 = u0 | m2;
    const uint64_t w3 = b3<kAandBorC>(u1, w2, w1);
    if constexpr (kE) {
        // the final count is u, or 6 - u where the site flipped: the same
        // parity; bit 1 of 6 - u is XNOR(u0, u1), bit 2 is set iff u <= 2
        const uint64_t f = u2 | w3;
        f0 = u0;
        f1 = b3<kAxorBandNotC>(u1, f, u0);          // u1 ^ (f & ~u0)
        f2 = b3<kAandNotBandNotC>(f, u2, u1 & u0);  // f & ~u2 & ~(u1 & u0)
        return s ^ f;
    }
    return b3<kAxorBorC>(s, u2, w3);  // s ^ flip
}

// The same with the masks looked up for the uniform R.
template <bool kE>
__device__ __forceinline__ uint64_t site(uint64_t s, const Nb& n, uint64_t jxp, uint64_t jxm,
                                         uint64_t jyp, uint64_t jym, uint64_t up, uint64_t dn,
                                         uint32_t R, const Tables& tb, uint64_t& f0, uint64_t& f1,
                                         uint64_t& f2) {
    return site_m<kE>(s, n, jxp, jxm, jyp, jym, up, dn, lane_mask(tb, 0, R), lane_mask(tb, 1, R),
                      lane_mask(tb, 2, R), f0, f1, f2);
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

constexpr int kDeep = 12;          // per-thread counter bits
constexpr int kFlushMacros = 128;  // 128 * 24 < 2^12

// The kDeep counter planes of one thread: in registers (kInLds = false), or
// in LDS at d[k * stride] for kernels with a tight register budget.
template <bool kInLds>
struct Deep;
template <>
struct Deep<false> {
    uint64_t v[kDeep];
    __device__ __forceinline__ Deep(uint64_t*, int) {
#pragma unroll
        for (int k = 0; k < kDeep; ++k) v[k] = 0;
    }
    __device__ __forceinline__ uint64_t& at(int k) { return v[k]; }
};
template <>
struct Deep<true> {
    uint64_t* d;
    int stride;
    __device__ __forceinline__ Deep(uint64_t* base, int s) : d(base), stride(s) {}
    __device__ __forceinline__ uint64_t& at(int k) { return d[k * stride]; }
};

// deep += small (5 bits), ripple carry.  Above the five planes of the addend
// the carry rarely survives: the ripple stops once no lane of the wave
// carries.
template <bool kInLds>
__device__ __forceinline__ void add_deep(Deep<kInLds>& d, uint64_t (&a)[5]) {
    uint64_t k = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const uint64_t v = d.at(i);
        const uint64_t nk = b3<kMaj>(v, a[i], k);
        d.at(i) = b3<kXor3>(v, a[i], k);
        k = nk;
        a[i] = 0;
    }
#pragma unroll
    for (int i = 5; i < kDeep; ++i) {
        if (!__any(k != 0)) break;
        const uint64_t v = d.at(i);
        d.at(i) = v ^ k;
        k = v & k;
    }
}

// Per-lane sums of the wave's vertical counters added into Ublk[64] (the
// counters are cleared).  Plane k is transposed across the wave, so lane b
// holds bit b of every thread's plane and popcounts it.  Every lane of the
// wave takes part; only waves of a team (add) contribute.
template <bool kInLds>
__device__ __forceinline__ void flush_deep(Deep<kInLds>& d, uint32_t* Ublk, bool add) {
    const int lane = threadIdx.x & 63;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kDeep; ++k) {
        acc += (uint32_t)__popcll(wave_transpose64(d.at(k))) << k;
        d.at(k) = 0;
    }
    if (add) atomicAdd(&Ublk[lane], acc);
}

// LDS of a block (64-bit words): TT, the bucket thresholds of the shape
// (uint32, shared by the block); DEEP[kDeep][threads], the energy counters,
// only where they are kept in LDS; then one region per team: X[2 L2], Y[2 L2], ml[nk+1], MM[2 nbt] (the two
// candidate lane masks of every bucket), Ublk[64] (uint32).
__host__ __device__ inline int stream_nbt(const ShapeDev& sh) {
    return sh.bnb[0] + sh.bnb[1] + sh.bnb[2] + 3;
}
__host__ __device__ inline int stream_team_words(const ShapeDev& sh) {
    return 4 * sh.L2 + sh.nk + 1 + 2 * stream_nbt(sh) + 32;
}
__host__ __device__ inline int stream_cols(const ShapeDev& sh) { return ((sh.L2 + 63) / 64) * 64; }

// Sweep of g configurations cfg0 .. cfg0+g-1 of one shape by one block: a
// team of `cols` threads (a multiple of 64) per configuration, all teams in
// lockstep along tau (one barrier per segment; teams of one wave need none
// and run free).  Teams at or past `nlive` and threads past the last team
// run the same barriers and touch no global memory.  Segment sigma updates the colour-0 site at plane A = 2 sigma + p
// and the colour-1 site of the previous step at A - 3.
// kPacked = false: one team filling the workgroup (g = nlive = 1,
// cols = blockDim.x), so every wave is a live member.  kDeepLds: the energy
// counters live in LDS rather than registers.
template <bool kE, bool kPacked, bool kDeepLds, bool kAnti>
__device__ __forceinline__ void sweep_teams(const ShapeDev& sh, const int cfg0, const int g,
                                            const int nlive, const int cols, uint64_t* lds,
                                            const uint32_t key0, const uint32_t key1,
                                            const uint32_t t) {
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, W = sh.W;
    const int nb0 = sh.bnb[0] + 1, nb1 = sh.bnb[1] + 1, nb2 = sh.bnb[2] + 1;
    const int nbt = nb0 + nb1 + nb2;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int team = kPacked ? __builtin_amdgcn_readfirstlane(tid / cols) : 0;  // wave-uniform
    const int ttid = tid - team * cols;
    const bool member = !kPacked || team < g;
    const int lteam = member ? team : g - 1;
    const bool live = !kPacked || (member && team < nlive);
    const bool active = live && ttid < L2;

    uint32_t* TT = (uint32_t*)lds;
    uint64_t* DEEP = lds + ((nbt + 1) >> 1);
    uint64_t* X = DEEP + (kDeepLds ? kDeep * nthr : 0) + (size_t)lteam * stream_team_words(sh);
    uint64_t* Y = X + 2 * L2;
    uint64_t* ml = X + 4 * L2;
    uint64_t* MM = ml + nk + 1;
    uint32_t* Ublk = (uint32_t*)(MM + 2 * nbt);
    const int H = L2;

    const int cfg = __builtin_amdgcn_readfirstlane(cfg0 + lteam);  // ((r*nk + w)*W + j), uniform
    const int j = cfg % W;
    const int rw = cfg / W;
    const int w = rw % nk;
    const int r = rw / nk;

    if (member)
        for (int i = ttid; i <= nk; i += cols)
            ml[i] = live ? sh.mask[((size_t)(r * W + j) * nk + w) * (nk + 1) + i] : 0ull;
    if (kE && member && ttid < 64) Ublk[ttid] = 0;
    if (kE && kDeepLds)
        for (int i = 0; i < kDeep; ++i) DEEP[i * nthr + tid] = 0;
    __syncthreads();
    // entry a of the concatenated tables (u = 0, 1, 2) sits at btab[a + shift(u)]
    const int bo0 = sh.boff[0], bo1 = sh.boff[1] - nb0, bo2 = sh.boff[2] - nb0 - nb1;
    for (int a = tid; a < nbt; a += nthr)
        TT[a] = (uint32_t)sh.btab[a + (a < nb0 ? bo0 : (a < nb0 + nb1 ? bo1 : bo2))];
    if (member)
        for (int a = ttid; a < nbt; a += cols) {
            const uint64_t e = sh.btab[a + (a < nb0 ? bo0 : (a < nb0 + nb1 ? bo1 : bo2))];
            const uint32_t kb = (uint32_t)(e >> 32) & 0xFFFFu, mu = (uint32_t)(e >> 48);
            MM[2 * a] = ml[kb];
            MM[2 * a + 1] = ml[kb + mu];
        }
    Tables tb;
    tb.T[0] = TT; tb.T[1] = TT + nb0; tb.T[2] = TT + nb0 + nb1;
    tb.M[0] = MM; tb.M[1] = MM + 2 * nb0; tb.M[2] = MM + 2 * (nb0 + nb1);
    tb.sh[0] = (uint32_t)sh.bsh[0]; tb.sh[1] = (uint32_t)sh.bsh[1]; tb.sh[2] = (uint32_t)sh.bsh[2];
    tb.nb[0] = (uint32_t)sh.bnb[0]; tb.nb[1] = (uint32_t)sh.bnb[1]; tb.nb[2] = (uint32_t)sh.bnb[2];

    const uint32_t c3 = ctr_word3(sh.word_offset + (uint32_t)j, sh.sid, kTagMetro);
    const uint32_t c2_0 = (uint32_t)rw << 1, c2_1 = c2_0 | 1u;

    const int xy = active ? ttid : 0;
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
    // descriptor fields are uniform: make that explicit (a vector descriptor
    // would turn every access into a loop over lanes)
    const uint64_t base = (uint64_t)(sh.S + (size_t)cfg * Lt * L2);
    const uint32_t base_lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t base_hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    const int nbytes = __builtin_amdgcn_readfirstlane(live ? Lt * L2 * 8 : 0);
    const __amdgpu_buffer_rsrc_t spins = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(((uint64_t)base_hi << 32) | base_lo), (short)0, nbytes, kBufferWord3);
    const int voff = 8 * xy;
    const int plane = 8 * L2;      // bytes per tau plane
    const int half = Lt >> 1;      // colour-0 steps
    const int nq = Lt >> 3;        // Philox groups per colour and column
    auto wrap = [Lt](int P) { return P >= Lt ? P - Lt : (P < 0 ? P + Lt : P); };
    // a plane reached across the tau wrap (P < 0 or P >= Ltau) is read
    // complemented and stored back complemented when the boundary is
    // antiperiodic: the wrap bond then has the sign -1 (apm = all ones).
    // kAnti = false compiles the periodic kernel without any of it.
    const uint64_t apm = kAnti ? sh.apm : 0ull;
    auto across = [Lt, apm](int P) -> uint64_t { return (kAnti && (P < 0 || P >= Lt)) ? apm : 0ull; };
    // uniform plane P; planes past Lt + 1 are never used: the load is
    // clamped, not skipped
    auto ld = [&](int P) -> uint64_t {
        const int Q = min(P, Lt + 1);
        return buf_load(spins, voff, wrap(Q) * plane) ^ across(Q);
    };
    // per-lane plane P (prologue): the plane offset goes in the vector offset
    auto ld_lane = [&](int P) -> uint64_t { return buf_load(spins, voff + wrap(P) * plane, 0) ^ across(P); };

    // window: w0..w5 = planes A-4 .. A+1, pf = A+2, A+3, nx = A+4, A+5
    uint64_t w0 = 0, w1 = 0, w2 = 0, w3, w4, w5, pf0, pf1, nx0, nx1;
    w3 = ld_lane(p - 1);
    w4 = ld_lane(p);
    w5 = ld_lane(p + 1);
    pf0 = ld_lane(min(p + 2, Lt + 1));
    pf1 = ld_lane(min(p + 3, Lt + 1));
    uint64_t pu1 = ld(4);  // plane 2 sigma + 4 of the next segment for parity 0
    // steady state: planes A + 4, A + 5 of the next segment, already in flight
    const int voffp = voff + p * plane;
    uint64_t nn0 = ld_lane(p + 4), nn1 = ld_lane(p + 5);
    u32x4 G0 = 0, G1 = 0;
    uint32_t prevlast = 0;
    uint64_t sm[5] = {0, 0, 0, 0, 0};
    Deep<kDeepLds> deep(DEEP + tid, nthr);
    uint64_t f0 = 0, f1 = 0, f2 = 0;

    if (active) X[hx] = p ? w3 : w5;  // X(0)
    __syncthreads();

    // Waves outside every team (member is wave-uniform) take part in the
    // same barriers and nothing else, decided once here: a test inside the
    // segment would leave the store count unknown along the loop and force
    // waits for every outstanding load.  Stores and LDS writes of a team
    // without a configuration need no guard of their own: its buffer
    // descriptor covers 0 bytes, and its LDS region is its own.
    // A team of one wave (64 columns or fewer) needs no barrier between
    // segments: the LDS operations of one wave take effect in program order,
    // so its teams run free of each other.  Uniform over the workgroup: all
    // teams of an item are alike.
    const bool solo = kPacked && cols == 64;
    if (kPacked && !member) {
        if (!solo)
            for (int k = 0; k < 4 * nq + 2; ++k) __syncthreads();
        if (kE) __syncthreads();
        return;
    }
    const bool lane_ok = ttid < L2;  // a column of the lattice (per lane)
    auto seg_sync = [&]() {
        if (solo) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    };

    // one segment; IS = sigma & 3 is a compile-time constant
    auto segment = [&](const int sigma, const auto ISc, const auto bulkC, const bool do_c0, const bool do_c1) {
        constexpr int IS = decltype(ISc)::value;
        constexpr bool kBulk = decltype(bulkC)::value;
        if constexpr (kBulk) {
            // no plane wraps before the last group: each lane loads its own
            // parity's planes, A + 6 and A + 7, a segment ahead of their use
            // as A + 4, A + 5 (no select that would wait for them at once)
            nx0 = nn0;
            nx1 = nn1;
            nn0 = buf_load(spins, voffp, (2 * sigma + 6) * plane);
            nn1 = buf_load(spins, voffp, (2 * sigma + 7) * plane);
        } else {
            // every load instruction reads whole planes 2 sigma + 5 and
            // 2 sigma + 6 (all columns, full cache lines); a thread keeps the
            // two planes of its parity, A + 4 and A + 5
            const uint64_t u0 = ld(2 * sigma + 5), u1 = ld(2 * sigma + 6);
            nx0 = p ? u0 : pu1;
            nx1 = p ? u1 : u0;
            pu1 = u1;
        }
        if (do_c0) {
            if (IS == 0) G0 = philox_dev((uint32_t)(xy + L2 * (sigma >> 2)), t, c2_0, c3, key0, key1);
            const uint64_t* Xb = X + (IS & 1) * H;
            const Nb n{Xb[hxp], Xb[hxm], Xb[hyp], Xb[hym]};
            uint64_t d0, d1, d2;
            w4 = site<false>(w4, n, jxp, jxm, jyp, jym, w5, w3, G0[IS], tb, d0, d1, d2);
        }
        if (IS == 1) {  // colour-1 Philox group of step s = sigma - 1 (s % 4 == 0)
            prevlast = G1[3];
            int q = (sigma - 1) >> 2;
            if (q >= nq) q -= nq;
            G1 = philox_dev((uint32_t)(xy + L2 * q), t, c2_1, c3, key0, key1);
        }
        if (do_c1) {
            constexpr int S3 = (IS + 3) & 3;  // (sigma - 1) & 3
            const uint32_t R1 = p ? G1[S3] : (S3 == 0 ? prevlast : G1[(S3 + 3) & 3]);
            const uint64_t* Yb = Y + ((IS + 1) & 1) * H;
            const Nb n{Yb[hxp], Yb[hxm], Yb[hyp], Yb[hym]};
            w1 = site<kE>(w1, n, jxp, jxm, jyp, jym, w2, w0, R1, tb, f0, f1, f2);
            if (kE && lane_ok) add3v(sm, f0, f1, f2);  // padding threads count nothing
        }
        // every store instruction writes whole planes 2 sigma - 3 and 2 sigma - 2:
        // parity 0 holds colour 1 (just updated) and colour 0 (one segment
        // old) there, parity 1 colour 0 (two segments old) and colour 1
        const int P1 = 2 * sigma - 3, P2 = 2 * sigma - 2;
        const uint64_t a1 = kBulk ? 0ull : across(P1), a2 = kBulk ? 0ull : across(P2);
        if (lane_ok && P1 >= 0) buf_store((p ? w0 : w1) ^ a1, spins, voff, wrap(P1) * plane);
        if (lane_ok && P2 >= 0) buf_store((p ? w1 : w2) ^ a2, spins, voff, wrap(P2) * plane);
        if (lane_ok) {
            Y[(IS & 1) * H + hx] = p ? w2 : w4;
            X[((IS + 1) & 1) * H + hx] = p ? w5 : pf1;
        }
        seg_sync();
        w0 = w2; w1 = w3; w2 = w4; w3 = w5; w4 = pf0; w5 = pf1; pf0 = nx0; pf1 = nx1;
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;

    using B0 = std::false_type;
    using B1 = std::true_type;
    for (int gq = 0; gq < nq - 1; ++gq) {
        const int s0 = 4 * gq;
        segment(s0 + 0, I0{}, B1{}, true, gq > 0);
        segment(s0 + 1, I1{}, B1{}, true, gq > 0);
        segment(s0 + 2, I2{}, B1{}, true, true);
        segment(s0 + 3, I3{}, B1{}, true, true);
        if (kE) {
            add_deep(deep, sm);
            if ((gq % kFlushMacros) == kFlushMacros - 1) flush_deep(deep, Ublk, true);
        }
    }
    // the last group and the tail reach the tau wrap: whole-plane loads
    const int sl = 4 * (nq - 1);
    pu1 = ld(2 * sl + 4);
    segment(sl + 0, I0{}, B0{}, true, nq > 1);
    segment(sl + 1, I1{}, B0{}, true, nq > 1);
    segment(sl + 2, I2{}, B0{}, true, true);
    segment(sl + 3, I3{}, B0{}, true, true);
    if (kE) add_deep(deep, sm);  // the 5-bit counters hold at most four sites
    segment(half, I0{}, B0{}, false, true);      // colour 1, step half-1
    segment(half + 1, I1{}, B0{}, false, true);  // colour 1, step half == step 0 (tau wrap)
    if (kE) {
        add_deep(deep, sm);
        flush_deep(deep, Ublk, true);
        __syncthreads();
        if (live && ttid < 64) sh.U[((size_t)r * W * 64 + (size_t)j * 64 + ttid) * nk + w] = Ublk[ttid];
    }
}

// Helper-wave form for L^2 = 576 (nine column waves).  Waves are placed on the
// four SIMDs round-robin, so waves 0, 4 and 8 share one SIMD and would carry
// half again the work of the others.  Three helper waves (9, 10, 11, one on
// each other SIMD) take over the uniforms and the lane-mask lookups of those
// three waves: one segment ahead, helper 9 + h runs the same Philox sequence
// as column wave 4h would, lane for lane, compares each uniform with its
// bucket threshold and leaves the six mask indices of the next segment's two
// sites in LDS; the served wave reads the masks themselves.  Every role runs
// the same segments and barriers; results are bit-identical to
// k_sweep_stream.
// Loads: until the last group no tau plane wraps, so each lane loads its own
// parity's two planes directly (no select that would wait for them at once),
// one segment earlier than the whole-plane form: a load is first used two
// segments after it is issued, which hides HBM latency under full load.
constexpr int kHelpedThreads = 768;
constexpr int kColWaves = 9;
constexpr int kHelpCols = kColWaves * 64;  // 576

__host__ __device__ inline int helped_words(const ShapeDev& sh) {
    return (stream_nbt(sh) + 1) / 2 + stream_team_words(sh) + (2 * 3 * 6 * 64) / 2;
}

// The body for configuration cfg = ((r*nk + w)*W + j), by a workgroup of
// kHelpedThreads threads; lds at least helped_words(sh) words.
template <bool kE, bool kAnti, bool kOpaquePitch = false>
__device__ __forceinline__ void helped_body(const ShapeDev& sh, const int cfg, uint64_t* lds, const uint32_t key0,
                                            const uint32_t key1, const uint32_t t) {
    const int L = sh.L, L2 = sh.L2, Lt = sh.Lt, nk = sh.nk, W = sh.W;
    const int nb0 = sh.bnb[0] + 1, nb1 = sh.bnb[1] + 1, nb2 = sh.bnb[2] + 1;
    const int nbt = nb0 + nb1 + nb2;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool helper = wave >= kColWaves;
    const int h = helper ? wave - kColWaves : (wave >> 2);  // helper slot of a served wave

    uint32_t* TT = (uint32_t*)lds;
    uint64_t* X = lds + ((nbt + 1) >> 1);
    uint64_t* Y = X + 2 * L2;
    uint64_t* ml = X + 4 * L2;
    uint64_t* MM = ml + nk + 1;
    uint32_t* Ublk = (uint32_t*)(MM + 2 * nbt);
    uint32_t* HM = (uint32_t*)(MM + 2 * nbt + 32);  // [2][3][6][64] mask indices for the served waves
    // kOpaquePitch: the buffer pitch hidden from the compiler.  A caller that
    // has tested L^2 (the batched kernel) would otherwise let it fold the
    // pitch and pair each colour-0 neighbour read with the colour-1 one into
    // one wider LDS read, which issues the colour-1 reads early and measured
    // 3% slower.
    int H = L2;
    if constexpr (kOpaquePitch) asm volatile("" : "+s"(H));

    const int j = cfg % W;
    const int rw = cfg / W;
    const int w = rw % nk;
    const int r = rw / nk;

    for (int i = tid; i <= nk; i += kHelpedThreads)
        ml[i] = sh.mask[((size_t)(r * W + j) * nk + w) * (nk + 1) + i];
    if (kE && tid < 64) Ublk[tid] = 0;
    __syncthreads();
    const int bo0 = sh.boff[0], bo1 = sh.boff[1] - nb0, bo2 = sh.boff[2] - nb0 - nb1;
    for (int a = tid; a < nbt; a += kHelpedThreads) {
        const uint64_t e = sh.btab[a + (a < nb0 ? bo0 : (a < nb0 + nb1 ? bo1 : bo2))];
        const uint32_t kb = (uint32_t)(e >> 32) & 0xFFFFu, mu = (uint32_t)(e >> 48);
        TT[a] = (uint32_t)e;
        MM[2 * a] = ml[kb];
        MM[2 * a + 1] = ml[kb + mu];
    }
    Tables tb;
    tb.T[0] = TT; tb.T[1] = TT + nb0; tb.T[2] = TT + nb0 + nb1;
    tb.M[0] = MM; tb.M[1] = MM + 2 * nb0; tb.M[2] = MM + 2 * (nb0 + nb1);
    tb.sh[0] = (uint32_t)sh.bsh[0]; tb.sh[1] = (uint32_t)sh.bsh[1]; tb.sh[2] = (uint32_t)sh.bsh[2];
    tb.nb[0] = (uint32_t)sh.bnb[0]; tb.nb[1] = (uint32_t)sh.bnb[1]; tb.nb[2] = (uint32_t)sh.bnb[2];
    __syncthreads();  // tables complete: the helpers look up segment 0's masks below

    const uint32_t c3 = ctr_word3(sh.word_offset + (uint32_t)j, sh.sid, kTagMetro);
    const uint32_t c2_0 = (uint32_t)rw << 1, c2_1 = c2_0 | 1u;

    // the column of this thread: its own, or (helper) that of the served lane
    const int xy = helper ? 64 * (4 * h) + lane : tid;
    const int x = xy % L, y = xy / L;
    const int p = (x + y) & 1;
    const int hx = xy;
    const int hxp = ((x + 1) % L) + L * y;
    const int hxm = ((x + L - 1) % L) + L * y;
    const int hyp = x + L * ((y + 1) % L);
    const int hym = x + L * ((y + L - 1) % L);
    const uint64_t* Jb = sh.J + (size_t)j * 2 * L2;
    const uint64_t jxp = Jb[xy], jxm = Jb[hxm], jyp = Jb[L2 + xy], jym = Jb[L2 + hym];

    const uint64_t base = (uint64_t)(sh.S + (size_t)cfg * Lt * L2);
    const uint32_t base_lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t base_hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    const __amdgpu_buffer_rsrc_t spins = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(((uint64_t)base_hi << 32) | base_lo), (short)0, Lt * L2 * 8, kBufferWord3);
    const int voff = 8 * xy;
    const int plane = 8 * L2;
    const int voffp = voff + p * plane;  // the thread's parity plane in the vector offset
    const int half = Lt >> 1;
    const int nq = Lt >> 3;
    auto wrap = [Lt](int P) { return P >= Lt ? P - Lt : (P < 0 ? P + Lt : P); };
    // planes across the tau wrap are complemented when antiperiodic (above)
    const uint64_t apm = kAnti ? sh.apm : 0ull;
    auto across = [Lt, apm](int P) -> uint64_t { return (kAnti && (P < 0 || P >= Lt)) ? apm : 0ull; };
    auto ld = [&](int P) -> uint64_t {
        const int Q = min(P, Lt + 1);
        return buf_load(spins, voff, wrap(Q) * plane) ^ across(Q);
    };
    auto ld_lane = [&](int P) -> uint64_t { return buf_load(spins, voff + wrap(P) * plane, 0) ^ across(P); };
    // [buffer][helper][mask][lane]: lane-contiguous, so every access is conflict-free
    auto hm = [&](int buf, int k) -> uint32_t* { return HM + ((buf * 3 + h) * 6 + k) * 64 + lane; };

    uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0, pf0 = 0, pf1 = 0, nx0 = 0, nx1 = 0, pu1 = 0;
    uint64_t nn0 = 0, nn1 = 0;  // planes A + 4, A + 5 of the next segment (steady state)
    if (!helper) {
        w3 = ld_lane(p - 1);
        w4 = ld_lane(p);
        w5 = ld_lane(p + 1);
        pf0 = ld_lane(min(p + 2, Lt + 1));
        pf1 = ld_lane(min(p + 3, Lt + 1));
        pu1 = ld(4);
        nn0 = ld_lane(p + 4);
        nn1 = ld_lane(p + 5);
    }
    u32x4 G0 = 0, G1 = 0;
    uint32_t prevlast = 0;
    uint64_t sm[5] = {0, 0, 0, 0, 0};
    Deep<false> deep(nullptr, 0);  // energy counters in registers
    uint64_t f0 = 0, f1 = 0, f2 = 0;

    if (!helper) {
        X[hx] = p ? w3 : w5;  // X(0)
    } else {
        // masks of segment 0 (colour 0, group 0) for the served lane
        G0 = philox_dev((uint32_t)xy, t, c2_0, c3, key0, key1);
        *hm(0, 0) = mask_index(tb, 0, G0[0]);
        *hm(0, 1) = mask_index(tb, 1, G0[0]);
        *hm(0, 2) = mask_index(tb, 2, G0[0]);
    }
    __syncthreads();

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;

    // kRole 0: column wave that looks up its own masks; 1: column wave fed by
    // a helper; 2: helper.  All roles run the same segments and barriers.
    auto segment = [&](const int sigma, const auto ISc, const auto roleC, const auto bulkC, const bool do_c0,
                       const bool do_c1) {
            constexpr int kRole = decltype(roleC)::value;
            constexpr int IS = decltype(ISc)::value;
            constexpr bool kBulk = decltype(bulkC)::value;
            if constexpr (kRole == 2) {
                // the next segment's masks for the served lane
                constexpr int ISn = (IS + 1) & 3;
                const int sn = sigma + 1;
                if (sn < half) {
                    if (ISn == 0)
                        G0 = philox_dev((uint32_t)(xy + L2 * (sn >> 2)), t, c2_0, c3, key0, key1);
                    const uint32_t R0 = G0[ISn];
                    *hm(ISn & 1, 0) = mask_index(tb, 0, R0);
                    *hm(ISn & 1, 1) = mask_index(tb, 1, R0);
                    *hm(ISn & 1, 2) = mask_index(tb, 2, R0);
                }
                if (ISn == 1 && sn <= half + 1) {
                    prevlast = G1[3];
                    int q = (sn - 1) >> 2;
                    if (q >= nq) q -= nq;
                    G1 = philox_dev((uint32_t)(xy + L2 * q), t, c2_1, c3, key0, key1);
                }
                if (sn >= 2 && sn <= half + 1) {
                    constexpr int S3 = (ISn + 3) & 3;
                    const uint32_t R1 = p ? G1[S3] : (S3 == 0 ? prevlast : G1[(S3 + 3) & 3]);
                    *hm(ISn & 1, 3) = mask_index(tb, 0, R1);
                    *hm(ISn & 1, 4) = mask_index(tb, 1, R1);
                    *hm(ISn & 1, 5) = mask_index(tb, 2, R1);
                }
                __syncthreads();
                return;
            } else {
                // the previous segment's colour-1 count goes into the counters
                // here, right after the barrier, where it fills the wait for
                // this segment's LDS reads (zero before the first colour-1 site)
                if (kE) add3v(sm, f0, f1, f2);
                if constexpr (kBulk) {
                    // no plane wraps before the last group: each lane loads its
                    // own parity's planes, A + 6 and A + 7, a segment ahead
                    nx0 = nn0;
                    nx1 = nn1;
                    nn0 = buf_load(spins, voffp, (2 * sigma + 6) * plane);
                    nn1 = buf_load(spins, voffp, (2 * sigma + 7) * plane);
                } else {
                    // whole planes 2 sigma + 5 and 2 sigma + 6, parity selected
                    const uint64_t u0 = ld(2 * sigma + 5), u1 = ld(2 * sigma + 6);
                    nx0 = p ? u0 : pu1;
                    nx1 = p ? u1 : u0;
                    pu1 = u1;
                }
                if (do_c0) {
                    const uint64_t* Xb = X + (IS & 1) * H;
                    const Nb n{Xb[hxp], Xb[hxm], Xb[hyp], Xb[hym]};
                    uint64_t d0, d1, d2;
                    if constexpr (kRole == 0) {
                        if (IS == 0)
                            G0 = philox_dev((uint32_t)(xy + L2 * (sigma >> 2)), t, c2_0, c3, key0, key1);
                        w4 = site<false>(w4, n, jxp, jxm, jyp, jym, w5, w3, G0[IS], tb, d0, d1, d2);
                    } else {
                        w4 = site_m<false>(w4, n, jxp, jxm, jyp, jym, w5, w3, tb.M[0][*hm(IS & 1, 0)],
                                           tb.M[1][*hm(IS & 1, 1)], tb.M[2][*hm(IS & 1, 2)], d0, d1, d2);
                    }
                }
                if constexpr (kRole == 0) {
                    if (IS == 1) {  // colour-1 Philox group of step s = sigma - 1 (s % 4 == 0)
                        prevlast = G1[3];
                        int q = (sigma - 1) >> 2;
                        if (q >= nq) q -= nq;
                        G1 = philox_dev((uint32_t)(xy + L2 * q), t, c2_1, c3, key0, key1);
                    }
                }
                if (do_c1) {
                    const uint64_t* Yb = Y + ((IS + 1) & 1) * H;
                    const Nb n{Yb[hxp], Yb[hxm], Yb[hyp], Yb[hym]};
                    if constexpr (kRole == 0) {
                        constexpr int S3 = (IS + 3) & 3;  // (sigma - 1) & 3
                        const uint32_t R1 = p ? G1[S3] : (S3 == 0 ? prevlast : G1[(S3 + 3) & 3]);
                        w1 = site<kE>(w1, n, jxp, jxm, jyp, jym, w2, w0, R1, tb, f0, f1, f2);
                    } else {
                        w1 = site_m<kE>(w1, n, jxp, jxm, jyp, jym, w2, w0, tb.M[0][*hm(IS & 1, 3)],
                                        tb.M[1][*hm(IS & 1, 4)], tb.M[2][*hm(IS & 1, 5)], f0, f1, f2);
                    }
                }
                const int P1 = 2 * sigma - 3, P2 = 2 * sigma - 2;
                const uint64_t a1 = kBulk ? 0ull : across(P1), a2 = kBulk ? 0ull : across(P2);
                if (P1 >= 0) buf_store((p ? w0 : w1) ^ a1, spins, voff, wrap(P1) * plane);
                if (P2 >= 0) buf_store((p ? w1 : w2) ^ a2, spins, voff, wrap(P2) * plane);
                Y[(IS & 1) * H + hx] = p ? w2 : w4;
                X[((IS + 1) & 1) * H + hx] = p ? w5 : pf1;
                __syncthreads();
                w0 = w2; w1 = w3; w2 = w4; w3 = w5; w4 = pf0; w5 = pf1; pf0 = nx0; pf1 = nx1;
            }
        };
    using R0 = std::integral_constant<int, 0>;
    using R1 = std::integral_constant<int, 1>;
    using R2 = std::integral_constant<int, 2>;
    using B0 = std::false_type;
    using B1 = std::true_type;
    if (helper) {
        for (int gq = 0; gq < nq; ++gq) {
            const int s0 = 4 * gq;
            segment(s0 + 0, I0{}, R2{}, B0{}, true, gq > 0);
            segment(s0 + 1, I1{}, R2{}, B0{}, true, gq > 0);
            segment(s0 + 2, I2{}, R2{}, B0{}, true, true);
            segment(s0 + 3, I3{}, R2{}, B0{}, true, true);
        }
        segment(half, I0{}, R2{}, B0{}, false, true);
        segment(half + 1, I1{}, R2{}, B0{}, false, true);
    } else {
        // column waves, fed by a helper (wave 4h) or self-served.  The last
        // group and the tail reach the tau wrap: they load whole planes.
        auto columns = [&](const auto roleC) {
            for (int gq = 0; gq < nq - 1; ++gq) {
                const int s0 = 4 * gq;
                segment(s0 + 0, I0{}, roleC, B1{}, true, gq > 0);
                segment(s0 + 1, I1{}, roleC, B1{}, true, gq > 0);
                segment(s0 + 2, I2{}, roleC, B1{}, true, true);
                segment(s0 + 3, I3{}, roleC, B1{}, true, true);
                if (kE) {
                    add_deep(deep, sm);
                    if ((gq % kFlushMacros) == kFlushMacros - 1) flush_deep(deep, Ublk, true);
                }
            }
            const int s0 = 4 * (nq - 1);
            pu1 = ld(2 * s0 + 4);
            segment(s0 + 0, I0{}, roleC, B0{}, true, nq > 1);
            segment(s0 + 1, I1{}, roleC, B0{}, true, nq > 1);
            segment(s0 + 2, I2{}, roleC, B0{}, true, true);
            segment(s0 + 3, I3{}, roleC, B0{}, true, true);
            if (kE) add_deep(deep, sm);  // the 5-bit counters hold at most four sites
            segment(half, I0{}, roleC, B0{}, false, true);
            segment(half + 1, I1{}, roleC, B0{}, false, true);
            if (kE) {
                add3v(sm, f0, f1, f2);  // the last colour-1 site
                add_deep(deep, sm);
                flush_deep(deep, Ublk, true);
            }
        };
        if ((wave & 3) == 0) columns(R1{});
        else columns(R0{});
    }
    if (kE) {
        __syncthreads();
        if (tid < 64) sh.U[((size_t)r * W * 64 + (size_t)j * 64 + tid) * nk + w] = Ublk[tid];
    }
}

template <bool kE, bool kAnti>
__global__ void __launch_bounds__(kHelpedThreads)
k_sweep_helped(ShapeDev sh, uint32_t key0, uint32_t key1, const Counters* __restrict__ ctr) {
    extern __shared__ uint64_t lds[];
    helped_body<kE, kAnti>(sh, (int)blockIdx.x, lds, key0, key1, ctr->t);
}

// One configuration per workgroup (r, w, j) = blockIdx.x.
// kOcc: minimum waves per SIMD the register allocation must allow (1 = no
// constraint); a tuning knob, the results do not depend on it.  Above 1 the
// energy counters move to LDS to fit the smaller register budget.
template <bool kE, int kOcc, bool kAnti>
__global__ void __launch_bounds__(kMaxCols) __attribute__((amdgpu_waves_per_eu(kOcc)))
k_sweep_stream(ShapeDev sh, uint32_t key0, uint32_t key1, const Counters* __restrict__ ctr) {
    extern __shared__ uint64_t lds[];
    sweep_teams<kE, false, (kOcc > 1), kAnti>(sh, (int)blockIdx.x, 1, 1, (int)blockDim.x, lds, key0, key1,
                                              ctr->t);
}

// Persistent sweep of every shape of a plan in one launch.  Work items
// (shape, teams g, live teams, first configuration) are taken from a queue
// in the order the host sorted them (longest first); a block sweeps the
// item's configurations with g teams, then takes the next item.  U is
// recounted in every sweep (it is exact whichever sweep last counted it), so
// one captured graph serves every sweep.  The last block to finish rewinds
// the queue for the next launch on the stream.  kAnti: some shape of the
// plan is antiperiodic along tau (each shape's own mask then applies).
template <int kOcc, bool kAnti>
__global__ void __launch_bounds__(kMaxBatchThreads) __attribute__((amdgpu_waves_per_eu(kOcc)))
k_sweep_batch(BatchArgs a) {
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&a.q->next, 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= a.n_items) break;
        const uint64_t e = a.items[it];
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)e);
        const int cfg0 = (int)__builtin_amdgcn_readfirstlane((uint32_t)(e >> 32));
        const int s = (int)(lo & 0xFFu), g = (int)((lo >> 8) & 0xFFu), nlive = (int)((lo >> 16) & 0xFFu);
        const ShapeDev& sh = a.shapes[s];
        const uint32_t t = __builtin_amdgcn_readfirstlane(a.ctr[s].t);
        if (sh.L2 == kHelpCols && blockDim.x == kHelpedThreads)
            helped_body<true, kAnti, true>(sh, cfg0, lds, a.key0, a.key1, t);  // one configuration, helper waves
        else
            sweep_teams<true, true, false, kAnti>(sh, cfg0, g, nlive, stream_cols(sh), lds, a.key0, a.key1, t);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&a.q->done, 1u) == gridDim.x - 1) {
            atomicExch(&a.q->next, 0u);
            atomicExch(&a.q->done, 0u);
        }
    }
}

}  // namespace

size_t sweep_stream_lds_bytes(const ShapeDev& sh, int teams, int threads, bool deep_in_lds) {
    const size_t nbt = (size_t)stream_nbt(sh);
    return ((nbt + 1) / 2 + (deep_in_lds ? (size_t)kDeep * threads : 0) +
            (size_t)teams * stream_team_words(sh)) * 8;
}

int sweep_stream_cols(const ShapeDev& sh) { return stream_cols(sh); }

size_t sweep_helped_lds_bytes(const ShapeDev& sh) { return (size_t)helped_words(sh) * 8; }

bool sweep_stream_ok(const ShapeDev& sh) {
    return sh.bnb[0] >= 0 && sh.bnb[1] >= 0 && sh.bnb[2] >= 0 && sh.L2 <= kMaxCols &&
           (sh.Lt % 8) == 0 && sh.Lt >= 16;
}

// Dynamic LDS above 64 KiB must be allowed per kernel, once.
static hipError_t allow_lds(const void* fn, size_t bytes, size_t& done) {
    if (bytes <= done) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done = bytes;
    return e;
}

template <bool kE, int kOcc, bool kAnti>
static hipError_t prepare_one(const ShapeDev& sh) {
    static size_t lds_set = 0;
    return allow_lds((const void*)k_sweep_stream<kE, kOcc, kAnti>,
                     sweep_stream_lds_bytes(sh, 1, stream_cols(sh), kOcc > 1), lds_set);
}

template <bool kE, int kOcc>
static hipError_t prepare_bc(const ShapeDev& sh) {
    return sh.apm ? prepare_one<kE, kOcc, true>(sh) : prepare_one<kE, kOcc, false>(sh);
}

hipError_t prepare_sweep_stream(const ShapeDev& sh, bool energy, int occ) {
    if (occ >= 5) return energy ? prepare_bc<true, 5>(sh) : prepare_bc<false, 5>(sh);
    return energy ? prepare_bc<true, 1>(sh) : prepare_bc<false, 1>(sh);
}

template <bool kE, int kOcc, bool kAnti>
static hipError_t launch_one(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st) {
    const int nblk = sh.R * sh.nk * sh.W;
    const int threads = stream_cols(sh);
    const size_t lds = sweep_stream_lds_bytes(sh, 1, threads, kOcc > 1);
    hipError_t e = prepare_one<kE, kOcc, kAnti>(sh);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sweep_stream<kE, kOcc, kAnti>), dim3(nblk), dim3(threads), lds, st, sh,
                       (uint32_t)seed, (uint32_t)(seed >> 32), ctr);
    return hipGetLastError();
}

template <bool kE, int kOcc>
static hipError_t launch_bc(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st) {
    return sh.apm ? launch_one<kE, kOcc, true>(sh, seed, ctr, st) : launch_one<kE, kOcc, false>(sh, seed, ctr, st);
}

bool sweep_helped_ok(const ShapeDev& sh) { return sweep_stream_ok(sh) && sh.L2 == kHelpCols; }

template <bool kE, bool kAnti>
static hipError_t launch_helped_one(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st,
                                    bool launch) {
    static size_t lds_set = 0;
    const size_t lds = (size_t)helped_words(sh) * 8;
    hipError_t e = allow_lds((const void*)k_sweep_helped<kE, kAnti>, lds, lds_set);
    if (e != hipSuccess || !launch) return e;
    hipLaunchKernelGGL((k_sweep_helped<kE, kAnti>), dim3(sh.R * sh.nk * sh.W), dim3(kHelpedThreads), lds, st,
                       sh, (uint32_t)seed, (uint32_t)(seed >> 32), ctr);
    return hipGetLastError();
}

template <bool kE>
static hipError_t launch_helped_bc(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st,
                                   bool launch) {
    return sh.apm ? launch_helped_one<kE, true>(sh, seed, ctr, st, launch)
                  : launch_helped_one<kE, false>(sh, seed, ctr, st, launch);
}

hipError_t launch_sweep_helped(const ShapeDev& sh, uint64_t seed, const Counters* ctr, bool energy,
                               hipStream_t st) {
    return energy ? launch_helped_bc<true>(sh, seed, ctr, st, true)
                  : launch_helped_bc<false>(sh, seed, ctr, st, true);
}

hipError_t prepare_sweep_helped(const ShapeDev& sh, bool energy) {
    return energy ? launch_helped_bc<true>(sh, 0, nullptr, nullptr, false)
                  : launch_helped_bc<false>(sh, 0, nullptr, nullptr, false);
}

hipError_t launch_sweep_stream(const ShapeDev& sh, uint64_t seed, const Counters* ctr,
                               bool energy, int occ, hipStream_t st) {
    if (occ >= 5)
        return energy ? launch_bc<true, 5>(sh, seed, ctr, st) : launch_bc<false, 5>(sh, seed, ctr, st);
    return energy ? launch_bc<true, 1>(sh, seed, ctr, st) : launch_bc<false, 1>(sh, seed, ctr, st);
}

static const void* batch_fn(int occ, bool anti) {
    if (anti) return occ >= 2 ? (const void*)k_sweep_batch<2, true> : (const void*)k_sweep_batch<1, true>;
    return occ >= 2 ? (const void*)k_sweep_batch<2, false> : (const void*)k_sweep_batch<1, false>;
}

hipError_t sweep_batch_prepare(int occ, bool anti, size_t lds_bytes, int threads, int* blocks_per_cu) {
    static size_t set[2][2] = {{0, 0}, {0, 0}};
    hipError_t e = allow_lds(batch_fn(occ, anti), lds_bytes, set[anti ? 1 : 0][occ >= 2 ? 1 : 0]);
    if (e != hipSuccess || !blocks_per_cu) return e;
    int nb = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_fn(occ, anti), threads, lds_bytes);
    *blocks_per_cu = nb;
    return e;
}

hipError_t launch_sweep_batch(const BatchArgs& a, int occ, bool anti, int blocks, int threads,
                              size_t lds_bytes, hipStream_t st) {
    if (anti) {
        if (occ >= 2)
            hipLaunchKernelGGL((k_sweep_batch<2, true>), dim3(blocks), dim3(threads), lds_bytes, st, a);
        else
            hipLaunchKernelGGL((k_sweep_batch<1, true>), dim3(blocks), dim3(threads), lds_bytes, st, a);
    } else {
        if (occ >= 2)
            hipLaunchKernelGGL((k_sweep_batch<2, false>), dim3(blocks), dim3(threads), lds_bytes, st, a);
        else
            hipLaunchKernelGGL((k_sweep_batch<1, false>), dim3(blocks), dim3(threads), lds_bytes, st, a);
    }
    return hipGetLastError();
}

}  // namespace tfim
