// Internal declarations shared by the libtfim host runtime and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tfim {

// Philox4x32-10 purposes (fourth counter word, bits 28..31).
enum : uint32_t { kTagMetro = 0u, kTagTemper = 1u, kTagSpin = 2u, kTagCoupling = 3u };

// Everything a kernel needs to know about one shape, by value.
struct ShapeDev {
    int L, L2, Lt, nk, W, R, P;  // P = replica pairs
    uint32_t sid, word_offset;
    uint32_t pt_every;
    // all ones when the tau boundary is antiperiodic: a spin word read
    // across the tau wrap enters complemented (the wrap bond has the sign -1)
    uint64_t apm;
    uint64_t* S;            // spins  [R][nk][W][Lt][L2]
    uint64_t* J;            // couplings [W][2][L2]
    uint8_t* kidx;          // [R][W*64][nk]  k-index of walker w
    uint8_t* winv;          // [R][W*64][nk]  walker holding k-index i
    uint32_t* U;            // [R][W*64][nk]  unsatisfied bonds of walker w
    uint64_t* mask;         // [R][W][nk][nk+1] lanes whose walker w has k-index < K
    const uint32_t* Tu;     // [nk][3]  Metropolis thresholds by unsatisfied count u
    const uint32_t* Tpt;    // swap thresholds, pair i at tpt_off[i] + d - 1
    const uint32_t* tpt_off;
    const uint32_t* dmax;
    int64_t* rec;           // measurement records [nk][W*64][P][2L+3]
    int64_t* buckets;       // [nk][2][L]
    // Bucket tables for K_u(R) = #{i : Tu[i][u] > R}: for u, R falls in
    // bucket a = min(R >> bsh[u], bnb[u]); entry (btab + boff[u])[a] packs
    // Tstar (bits 0..31), Kbase (32..47), mult (48..63) so that
    // K_u(R) = Kbase + (R < Tstar ? mult : 0).  bnb[u] = -1: no table.
    const uint64_t* btab;
    int bsh[3], bnb[3], boff[3];
    // Measurement layouts (one bit per spin, one row per sample), written by
    // the transpose kernel for configuration m = (i*S + s)*R + r (k-index i,
    // sample s, replica r):
    //   Pt[(m*nc + c)*nxp + xy]  bit t = spin bit of (tau = 64c + t, xy)
    //   Px[(m*nx + g)*Lt + tau]  bit t = spin bit of (tau, xy = 64g + t)
    // nc = ceil(Lt/64), nx = ceil(L2/64), nxp = 64*nx; padding bits are 0.
    uint64_t* Pt;
    uint64_t* Px;
    int32_t* dump;  // [2*L2*L2 + Lt*Lt] debug matrices
    int nc, nx, nxp;
};

// Plan-wide device counters.
struct Counters {
    uint32_t t;         // sweeps done
    uint32_t m;         // tempering steps done
    uint32_t error;     // nonzero: a kernel detected an inconsistency
    uint32_t pad;
};

// Work queue of the persistent batched sweep; zero between launches.
struct BatchQueue {
    uint32_t next;  // next work item to hand out
    uint32_t done;  // blocks that found the queue empty
};

// Arguments of the batched sweep kernel.  The shapes travel by value in the
// kernel arguments (scalar loads, provably uniform in the kernel).
constexpr int kMaxBatchShapes = 8;
struct BatchArgs {
    ShapeDev shapes[kMaxBatchShapes];
    const uint64_t* items;   // shape | teams << 8 | live teams << 16 | first cfg << 32
    BatchQueue* q;
    const Counters* ctr;     // [n_shapes]
    uint32_t n_items, key0, key1, pad;
};

struct TemperBatchArgs {
    const ShapeDev* shapes;  // [n_shapes]
    const uint32_t* first;   // [n_shapes + 1] first block of each shape, (r, j) groups
    Counters* ctr;           // [n_shapes]
    uint32_t n_shapes, key0, key1, pad;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// two-multiplier S-box; the key advances by the Weyl increments each round.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t v[4];
};

__host__ __device__ inline U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t key0, uint32_t key1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ key0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ key1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        key0 += kWeylA;
        key1 += kWeylB;
    }
    U4 r;
    r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
    return r;
}

__host__ __device__ inline uint32_t ctr_word3(uint32_t j_global, uint32_t sid, uint32_t tag) {
    return (j_global & 0xFFFFFu) | ((sid & 0xFFu) << 20) | (tag << 28);
}

// 64x64 bit transpose across a wavefront: lane t holds row t (bit u is
// element (t, u)); afterwards lane u holds column u (bit t is element (t, u)).
// Level k swaps the off-diagonal k x k blocks of every 2k x 2k block.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t v) {
    const int lane = threadIdx.x & 63;
    const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull,
                               0x00FF00FF00FF00FFull, 0x0F0F0F0F0F0F0F0Full,
                               0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int lv = 0; lv < 6; ++lv) {
        const int k = 32 >> lv;
        const uint64_t mk = masks[lv];
        const uint64_t o = (uint64_t)__shfl_xor((long long)v, k, 64);
        v = (lane & k) ? (((o >> k) & mk) | (v & ~mk)) : ((v & mk) | ((o & mk) << k));
    }
    return v;
}

// Operands of v_mfma_i32_32x32x32_i8 built in registers from bit rows.  In K
// step ks of a 64-bit chunk word w, lane (i, h) of a block feeds row i with
// bits 8j + 4h + m (j, m < 4) of the 32-bit half ks of w, one byte each; the
// same order on both sides of a product permutes K alike, so the dot product
// is the popcount of the AND of the two rows.  x is the half already shifted
// right by 4h; byte j of dword m is bit 8j + m of x, times 4 when kTimes4.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

template <bool kTimes4>
__device__ __forceinline__ i32x4 mfma_bits_operand(uint32_t x) {
    i32x4 o;
    if constexpr (kTimes4) {
        const uint32_t x4 = x << 2;
#pragma unroll
        for (int m = 0; m < 4; ++m) o[m] = (int)((x4 >> m) & 0x04040404u);
    } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) o[m] = (int)((x >> m) & 0x01010101u);
    }
    return o;
}

// v_mfma_scale_f32_32x32x64_f8f6f4 operands: format code 4 = e2m1 (fp4) on
// both sides, four registers of 8 nibbles each; block scales are E8M0
// (2^(e - 127)): 2^4 on the row side, 1 on the column side
constexpr int kFp4 = 4;
constexpr int kScaleRow = 127 + 4;
constexpr int kScaleOne = 127;
// Bit 4j + m of x (m < 4, j < 8) as the fp4 nibble j of register m: 0 or
// 0.5; the upper four registers are not read in the fp4 form.
__device__ __forceinline__ i32x8 fp4_bits_operand(uint32_t x) {
    i32x4 o;
#pragma unroll
    for (int m = 0; m < 4; ++m) o[m] = (int)((x >> m) & 0x11111111u);
    return __builtin_shufflevector(o, o, 0, 1, 2, 3, -1, -1, -1, -1);
}

// Sixteen int8 bytes summing to v, |v| <= 1792: fifteen of floor(v / 16) and
// one of floor(v / 16) + (v mod 16).  Against sixteen ones on the other side
// of one K step it adds v to every element of a row (or column).
__device__ __forceinline__ i32x4 mfma_pieces16(int v) {
    const int q = v >> 4, r = v & 15;
    const uint32_t rep = (uint32_t)(q & 0xFF) * 0x01010101u;
    i32x4 o;
    o[0] = (int)((rep & 0xFFFFFF00u) | (uint32_t)((q + r) & 0xFF));
    o[1] = o[2] = o[3] = (int)rep;
    return o;
}

}  // namespace tfim

// Kernel launchers (defined in the .hip files, called by the runtime).
namespace tfim {
hipError_t launch_init_couplings(const ShapeDev& sh, uint64_t seed, hipStream_t st);
hipError_t launch_init_spins(const ShapeDev& sh, uint64_t seed, hipStream_t st);
hipError_t launch_labels_identity(const ShapeDev& sh, hipStream_t st);
hipError_t launch_energy(const ShapeDev& sh, hipStream_t st);
hipError_t launch_mask_rebuild(const ShapeDev& sh, hipStream_t st);
// variant 0: streaming kernel (needs bucket tables), 1: chunked kernel,
// 2: streaming kernel compiled for >= 5 waves per SIMD, 3: streaming kernel
// with helper waves where L^2 = 576 (else as 0).
// energy: also recount U (the chunked kernel always does).
hipError_t launch_sweep(const ShapeDev& sh, uint64_t seed, const Counters* ctr, int variant,
                        bool energy, hipStream_t st);
hipError_t launch_sweep_stream(const ShapeDev& sh, uint64_t seed, const Counters* ctr,
                               bool energy, int occ, hipStream_t st);
// Kernel attributes a later launch of this shape and variant needs (dynamic
// LDS above 64 KiB), set outside any stream capture.
hipError_t prepare_sweep(const ShapeDev& sh, int variant, bool energy);
hipError_t prepare_sweep_stream(const ShapeDev& sh, bool energy, int occ);
// Helper-wave form of the streaming sweep (L^2 = 576 only).
bool sweep_helped_ok(const ShapeDev& sh);
hipError_t launch_sweep_helped(const ShapeDev& sh, uint64_t seed, const Counters* ctr, bool energy,
                               hipStream_t st);
hipError_t prepare_sweep_helped(const ShapeDev& sh, bool energy);
bool sweep_stream_ok(const ShapeDev& sh);
// LDS of a streaming-sweep block of `teams` configurations and `threads`
// threads (deep_in_lds: the energy counters are kept in LDS, not registers);
// threads per configuration (L^2 rounded up to whole waves).
size_t sweep_stream_lds_bytes(const ShapeDev& sh, int teams, int threads, bool deep_in_lds);
int sweep_stream_cols(const ShapeDev& sh);
// LDS of the helper-wave workgroup (L^2 = 576, 768 threads), which the batched
// kernel also runs for such shapes when launched with 768 threads.
size_t sweep_helped_lds_bytes(const ShapeDev& sh);
// Batched persistent sweep: allow its LDS and report resident blocks per CU
// (occ: 1 or 2 = minimum waves per SIMD the kernel was compiled for).
// anti: some shape of the plan is antiperiodic along tau
hipError_t sweep_batch_prepare(int occ, bool anti, size_t lds_bytes, int threads, int* blocks_per_cu);
hipError_t launch_sweep_batch(const BatchArgs& a, int occ, bool anti, int blocks, int threads,
                              size_t lds_bytes, hipStream_t st);
// Tempering (when due, read from the counters) of every shape, then the
// counter advance t += 1, m += due.
hipError_t launch_temper_batch(const TemperBatchArgs& a, int blocks, int max_nk, hipStream_t st);
hipError_t launch_advance_batch(const TemperBatchArgs& a, hipStream_t st);
hipError_t launch_temper(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st);
hipError_t launch_advance(Counters* ctr, uint32_t dt, uint32_t dm, hipStream_t st);
// Measurement of configurations cfg0 .. cfg0+ncfg-1 (cfg = i*S + s) into the
// records (which must be zeroed first).  mode 0: batched int8-MFMA kernels;
// mode 1: plain per-sample VALU form, one launch per configuration.
hipError_t launch_transpose(const ShapeDev& sh, hipStream_t st);
hipError_t launch_measure(const ShapeDev& sh, int mode, int cfg0, int ncfg, hipStream_t st);
hipError_t launch_buckets(const ShapeDev& sh, hipStream_t st);
hipError_t launch_dump(const ShapeDev& sh, int cfg, int a, int b, hipStream_t st);
bool measure_ok(const ShapeDev& sh);
// Three-replica records (chi^(3), F^(3)) of configurations cfg0 .. cfg0+ncfg-1
// into a caller workspace: int64 records [ncfg][triples][2][L] (rec_bytes,
// 256-aligned), then the G' digit planes [ncfg][R][2][Np][Np] (g_bytes).
struct TripleLayout {
    int nb, nt, Np;  // 8x8 site blocks per edge, tiles, padded sites
    size_t rec_bytes, g_bytes;
};
TripleLayout triple_layout(const ShapeDev& sh, int ncfg);
const char* triples_unsupported(const ShapeDev& sh);  // nullptr if supported
// rec: int64 records [ncfg][triples][2][L] (cleared first); gw: the digit
// planes, g_bytes of scratch
hipError_t launch_triples(const ShapeDev& sh, int cfg0, int ncfg, int64_t* rec, int8_t* gw, hipStream_t st);
// Library-held device scratch of the entry points that allocate nothing:
// its device address on `device` (looked up once per device) and its size.
hipError_t static_scratch(int device, void** ptr, size_t* bytes);
// Two-time records (c, q2 along the periodic diagonals of H = S^T S, summed
// over replicas) of configurations cfg0 .. cfg0+ncfg-1: int64 [ncfg][2][Lt].
const char* timecorr_unsupported(const ShapeDev& sh);  // nullptr if supported
size_t timecorr_record_bytes(const ShapeDev& sh, int ncfg);
hipError_t launch_timecorr(const ShapeDev& sh, int cfg0, int ncfg, int64_t* rec, hipStream_t st);
// Transfer matrix of one plane (2 <= L <= 5): w = T v on 2^(L^2) doubles,
// and the nev = 1 or 2 largest eigenvalues of the even (odd = 0) or odd
// parity sector by power iteration (the second with the first eigenvector
// deflated) in a workspace of three vectors and reduction partials.
const char* tm_unsupported(int L);  // nullptr if supported
size_t tm_workspace_bytes(int L);
hipError_t tm_apply(int L, double k, const int8_t* Jx, const int8_t* Jy, const double* v, double* w,
                    hipStream_t st);
hipError_t tm_top(int L, double k, const int8_t* Jx, const int8_t* Jy, int odd, int nev, double tol,
                  int max_iter, void* ws, double* lambda, int* iters, hipStream_t st);
int sweep_variants();
const char* sweep_variant_name(int v);
// Plain form (one int8 per spin, one sample per configuration; ShapeDev.W
// holds the number of samples, S and J point at int8 arrays).
hipError_t plain_init_couplings(const ShapeDev& sh, uint64_t seed, hipStream_t st);
hipError_t plain_init_spins(const ShapeDev& sh, uint64_t seed, hipStream_t st);
hipError_t plain_labels_identity(const ShapeDev& sh, hipStream_t st);
hipError_t plain_energy(const ShapeDev& sh, hipStream_t st);
// colour 0, colour 1 and the energy recount of one sweep
hipError_t plain_sweep(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st);
hipError_t plain_temper(const ShapeDev& sh, uint64_t seed, const Counters* ctr, hipStream_t st);
bool plain_measure_ok(const ShapeDev& sh);
// pair records of configurations cfg0 .. cfg0+ncfg-1 (zeroed first)
hipError_t plain_measure(const ShapeDev& sh, int cfg0, int ncfg, hipStream_t st);
hipError_t plain_buckets(const ShapeDev& sh, hipStream_t st);
}  // namespace tfim
