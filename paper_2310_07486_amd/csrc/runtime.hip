// libtfim host runtime: plan creation and validation, FP64 threshold tables,
// arena layout, state import/export, launch schedules, HIP graphs, the
// autotuner and the host-side xi^(2).  Implements include/tfim.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/tfim.h"
#include "tfim_internal.h"

namespace {

thread_local std::string g_detail;

tfim_status fail(tfim_status st, const std::string& msg) {
    g_detail = msg;
    return st;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct ShapeHost {
    tfim_shape s{};
    std::vector<double> k;
    std::vector<uint32_t> Tu;       // [nk][3]
    std::vector<uint32_t> dmax;     // [nk]  (last entry 0)
    std::vector<uint32_t> tpt_off;  // [nk]
    std::vector<uint32_t> Tpt;      // concatenated
    std::vector<uint64_t> btab;     // threshold bucket tables, all u
    int bsh[3] = {0, 0, 0}, bnb[3] = {-1, -1, -1}, boff[3] = {0, 0, 0};
    // arena offsets
    size_t oS = 0, oJ = 0, oK = 0, oWinv = 0, oU = 0, oMask = 0, oTu = 0, oTpt = 0, oTptOff = 0,
           oDmax = 0, oRec = 0, oBuck = 0, oBtab = 0, oPt = 0, oPx = 0, oDump = 0;
    size_t nS = 0, nJ = 0, nLab = 0, nMask = 0, nRec = 0, nBuck = 0, nPt = 0, nPx = 0, nDump = 0;
    int nc = 0, nx = 0;
    bool J_ready = false, S_ready = false;
    int P = 0;
};

}  // namespace

struct tfim_plan {
    std::vector<ShapeHost> shapes;
    uint64_t seed = 0;
    tfim_sizes sizes{};
    size_t oCounters = 0;
    char* arena = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    bool poisoned = false;
    std::vector<uint64_t> t, m;  // host mirrors per shape
    uint32_t schedule = TFIM_SCHED_PER_SHAPE;
    int variant = 0;
    uint32_t measure_mode = 0;
    double tuned_ms = 0.0;
    std::map<uint64_t, hipGraphExec_t> graphs;  // keyed by (n, t phase) for the per-shape schedule
    // HIP-event timing of sweep-kernel launches (tfim_set_timing)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
};

namespace {

tfim::ShapeDev dev_of(const tfim_plan* pl, int i) {
    const ShapeHost& h = pl->shapes[i];
    tfim::ShapeDev d{};
    d.L = (int)h.s.L;
    d.L2 = d.L * d.L;
    d.Lt = (int)h.s.Ltau;
    d.nk = (int)h.s.n_k;
    d.W = (int)h.s.n_words;
    d.R = (int)h.s.n_replicas;
    d.P = h.P;
    d.sid = h.s.stream_id;
    d.word_offset = h.s.word_offset;
    d.pt_every = h.s.pt_every;
    char* a = pl->arena;
    d.S = (uint64_t*)(a + h.oS);
    d.J = (uint64_t*)(a + h.oJ);
    d.kidx = (uint8_t*)(a + h.oK);
    d.winv = (uint8_t*)(a + h.oWinv);
    d.U = (uint32_t*)(a + h.oU);
    d.mask = (uint64_t*)(a + h.oMask);
    d.Tu = (const uint32_t*)(a + h.oTu);
    d.Tpt = (const uint32_t*)(a + h.oTpt);
    d.tpt_off = (const uint32_t*)(a + h.oTptOff);
    d.dmax = (const uint32_t*)(a + h.oDmax);
    d.rec = (int64_t*)(a + h.oRec);
    d.buckets = (int64_t*)(a + h.oBuck);
    d.btab = (const uint64_t*)(a + h.oBtab);
    d.Pt = (uint64_t*)(a + h.oPt);
    d.Px = (uint64_t*)(a + h.oPx);
    d.dump = (int32_t*)(a + h.oDump);
    d.nc = h.nc;
    d.nx = h.nx;
    d.nxp = 64 * h.nx;
    for (int u = 0; u < 3; ++u) {
        d.bsh[u] = h.bsh[u];
        d.bnb[u] = h.bnb[u];
        d.boff[u] = h.boff[u];
    }
    return d;
}

tfim::Counters* counters_of(const tfim_plan* pl, int i) {
    return (tfim::Counters*)(pl->arena + pl->oCounters) + i;
}

tfim_status check_hip(tfim_plan* pl, hipError_t e, const char* what) {
    if (e == hipSuccess) return TFIM_OK;
    if (pl) pl->poisoned = true;
    return fail(TFIM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

tfim_status usable(tfim_plan* pl) {
    if (!pl) return fail(TFIM_EINVAL, "null plan");
    if (pl->poisoned) return fail(TFIM_ESTATE, "plan poisoned by an earlier device error");
    if (!pl->bound) return fail(TFIM_ESTATE, "plan not bound to a device arena");
    return TFIM_OK;
}

// Metropolis thresholds Tu[i][u] = floor(2^32 exp(-k_i (12 - 4u))) and the
// swap tables, FP64 with the C library exp, x 2^32 exact, floor, clamp.
uint32_t to_threshold(double p) {
    const double v = std::floor(p * 4294967296.0);
    if (v >= 4294967295.0) return 0xFFFFFFFFu;
    if (v <= 0.0) return 0u;
    return (uint32_t)v;
}

void build_tables(ShapeHost& h) {
    const int nk = (int)h.s.n_k;
    const uint64_t N = (uint64_t)h.s.L * h.s.L * h.s.Ltau;
    h.Tu.assign((size_t)nk * 3, 0);
    for (int i = 0; i < nk; ++i)
        for (int u = 0; u < 3; ++u) {
            const double dE = (double)(12 - 4 * u);
            h.Tu[(size_t)i * 3 + u] = to_threshold(std::exp(-(h.k[i] * dE)));
        }
    h.dmax.assign(nk, 0);
    h.tpt_off.assign(nk, 0);
    h.Tpt.clear();
    for (int i = 0; i + 1 < nk; ++i) {
        const double dk = h.k[i + 1] - h.k[i];
        h.tpt_off[i] = (uint32_t)h.Tpt.size();
        uint32_t d = 0;
        while ((uint64_t)d < 3 * N) {
            const uint32_t T = to_threshold(std::exp(-(dk * (double)(2 * (int64_t)(d + 1)))));
            if (T == 0) break;
            h.Tpt.push_back(T);
            ++d;
        }
        h.dmax[i] = d;
    }
    if (h.Tpt.empty()) h.Tpt.push_back(0);
}

// Bucket tables for the per-lane threshold count K_u(R) (see ShapeDev).
// For each u, the largest shift such that every bucket [a 2^sh, (a+1) 2^sh)
// holds at most one distinct threshold strictly inside it, with at most
// kMaxBuckets buckets; bnb[u] = -1 if no such shift exists.
constexpr int kMaxBuckets = 1024;

void build_buckets(ShapeHost& h) {
    const int nk = (int)h.s.n_k;
    h.btab.clear();
    for (int u = 0; u < 3; ++u) {
        std::vector<uint64_t> T(nk);
        for (int i = 0; i < nk; ++i) T[i] = h.Tu[(size_t)i * 3 + u];
        const uint64_t Tmax = *std::max_element(T.begin(), T.end());
        int chosen = -1;
        for (int sh = 31; sh >= 0; --sh) {
            const uint64_t nb = (Tmax >> sh) + 1;
            if (nb > (uint64_t)kMaxBuckets) break;
            bool ok = true;
            for (uint64_t a = 0; a <= nb && ok; ++a) {
                const uint64_t lo = a << sh, hi = (a + 1) << sh;
                uint64_t v = UINT64_MAX;
                for (int i = 0; i < nk; ++i)
                    if (T[i] > lo && T[i] < hi) {
                        if (v == UINT64_MAX) v = T[i];
                        else if (v != T[i]) { ok = false; break; }
                    }
            }
            if (ok) { chosen = sh; break; }
        }
        h.boff[u] = (int)h.btab.size();
        if (chosen < 0) {
            h.bnb[u] = -1;
            h.bsh[u] = 0;
            continue;
        }
        const uint64_t nb = (Tmax >> chosen) + 1;
        h.bsh[u] = chosen;
        h.bnb[u] = (int)nb;
        for (uint64_t a = 0; a <= nb; ++a) {
            const uint64_t lo = a << chosen, hi = (a + 1) << chosen;
            uint64_t kbase = 0, mult = 0, tstar = 0;
            for (int i = 0; i < nk; ++i) {
                if (T[i] >= hi) ++kbase;
                else if (T[i] > lo) { tstar = T[i]; ++mult; }
            }
            h.btab.push_back(tstar | (kbase << 32) | (mult << 48));
        }
    }
    if (h.btab.empty()) h.btab.push_back(0);
}

tfim_status validate(const tfim_shape* s, uint32_t n) {
    if (!s || n == 0 || n > 64) return fail(TFIM_EINVAL, "need 1..64 shapes");
    for (uint32_t i = 0; i < n; ++i) {
        const tfim_shape& a = s[i];
        char buf[160];
        if (a.L < 2 || a.L > 24 || (a.L & 1)) {
            snprintf(buf, sizeof buf, "shape %u: L=%u must be even in [2,24]", i, a.L);
            return fail(TFIM_EINVAL, buf);
        }
        if (a.Ltau < 4 || a.Ltau > 65536 || (a.Ltau & 1)) {
            snprintf(buf, sizeof buf, "shape %u: Ltau=%u must be even in [4,65536]", i, a.Ltau);
            return fail(TFIM_EINVAL, buf);
        }
        if (a.n_words == 0 || (uint64_t)a.word_offset + a.n_words > (1u << 20))
            return fail(TFIM_EINVAL, "n_words must be >= 1 and word_offset+n_words <= 2^20");
        if (a.n_replicas == 0 || a.n_replicas > 64) return fail(TFIM_EINVAL, "n_replicas in 1..64");
        if (a.n_k == 0 || a.n_k > 255 || !a.k) return fail(TFIM_EINVAL, "n_k in 1..255 with k != NULL");
        if ((uint64_t)a.n_replicas * a.n_k >= (1u << 30)) return fail(TFIM_EINVAL, "too many walkers");
        for (uint32_t q = 0; q < a.n_k; ++q) {
            if (!(a.k[q] > 0.0) || !std::isfinite(a.k[q])) return fail(TFIM_EINVAL, "k must be finite and > 0");
            if (q && !(a.k[q] > a.k[q - 1])) return fail(TFIM_EINVAL, "k ladder must be strictly increasing");
        }
        if (a.stream_id > 255) return fail(TFIM_EINVAL, "stream_id must be < 256");
        for (uint32_t q = 0; q < i; ++q)
            if (s[q].stream_id == a.stream_id) return fail(TFIM_EINVAL, "stream_id repeated in plan");
        if (a.bc_tau == TFIM_BC_ANTIPERIODIC)
            return fail(TFIM_EUNSUPPORTED, "antiperiodic tau boundary not provided");
        if (a.bc_tau != TFIM_BC_PERIODIC) return fail(TFIM_EINVAL, "unknown bc_tau");
        if (a.Ltau % 8 != 0)
            return fail(TFIM_EUNSUPPORTED, "the GPU sweep walks tau in chunks of 8: Ltau % 8 must be 0");
        // L^2 <= 1024 threads per workgroup
    }
    return TFIM_OK;
}

}  // namespace

extern "C" {

const char* tfim_strerror(tfim_status st) {
    switch (st) {
        case TFIM_OK: return "ok";
        case TFIM_EINVAL: return "invalid argument";
        case TFIM_EUNSUPPORTED: return "unsupported";
        case TFIM_EDEVICE: return "device error";
        case TFIM_ESTATE: return "invalid state";
        case TFIM_EOVERFLOW: return "counter overflow";
        default: return "unknown status";
    }
}

const char* tfim_last_error_detail(void) { return g_detail.c_str(); }

tfim_status tfim_plan_create(const tfim_shape* shapes, uint32_t n_shapes, uint64_t seed,
                             tfim_plan** out) {
    if (!out) return fail(TFIM_EINVAL, "null output pointer");
    *out = nullptr;
    tfim_status st = validate(shapes, n_shapes);
    if (st != TFIM_OK) return st;
    tfim_plan* pl = new tfim_plan();
    pl->seed = seed;
    size_t off = 0;
    size_t tot_S = 0, tot_J = 0, tot_lab = 0, tot_tab = 0, tot_meas = 0;
    for (uint32_t i = 0; i < n_shapes; ++i) {
        ShapeHost h;
        h.s = shapes[i];
        h.k.assign(shapes[i].k, shapes[i].k + shapes[i].n_k);
        h.s.k = nullptr;
        h.P = (int)(h.s.n_replicas * (h.s.n_replicas - 1) / 2);
        build_tables(h);
        build_buckets(h);
        const size_t L2 = (size_t)h.s.L * h.s.L, nk = h.s.n_k, W = h.s.n_words,
                     R = h.s.n_replicas, Lt = h.s.Ltau, S = 64 * W;
        h.nS = R * nk * W * Lt * L2 * 8;
        h.nJ = W * 2 * L2 * 8;
        h.nLab = R * S * nk;
        h.nMask = R * W * nk * (nk + 1) * 8;
        h.nRec = h.P ? nk * S * h.P * (2 * h.s.L + 3) * 8 : 0;
        h.nBuck = nk * 2 * h.s.L * 8;
        h.nc = (int)((Lt + 63) / 64);
        h.nx = (int)((L2 + 63) / 64);
        h.nPt = h.P ? nk * S * R * (size_t)h.nc * 64 * h.nx * 8 : 0;
        h.nPx = h.P ? nk * S * R * (size_t)h.nx * Lt * 8 : 0;
        h.nDump = h.P ? (2 * L2 * L2 + Lt * Lt) * 4 : 0;
        h.oS = off; off = align256(off + h.nS); tot_S += h.nS;
        h.oJ = off; off = align256(off + h.nJ); tot_J += h.nJ;
        h.oK = off; off = align256(off + h.nLab);
        h.oWinv = off; off = align256(off + h.nLab);
        h.oU = off; off = align256(off + h.nLab * 4);
        h.oMask = off; off = align256(off + h.nMask);
        tot_lab += 6 * h.nLab + h.nMask;
        h.oTu = off; off = align256(off + h.Tu.size() * 4);
        h.oTpt = off; off = align256(off + h.Tpt.size() * 4);
        h.oTptOff = off; off = align256(off + nk * 4);
        h.oDmax = off; off = align256(off + nk * 4);
        h.oBtab = off; off = align256(off + h.btab.size() * 8);
        tot_tab += (h.Tu.size() + h.Tpt.size() + 2 * nk) * 4 + h.btab.size() * 8;
        h.oRec = off; off = align256(off + h.nRec);
        h.oBuck = off; off = align256(off + h.nBuck);
        h.oPt = off; off = align256(off + h.nPt);
        h.oPx = off; off = align256(off + h.nPx);
        h.oDump = off; off = align256(off + h.nDump);
        tot_meas += h.nRec + h.nBuck + h.nPt + h.nPx + h.nDump;
        pl->shapes.push_back(std::move(h));
    }
    pl->oCounters = off;
    off = align256(off + sizeof(tfim::Counters) * n_shapes);
    tot_tab += sizeof(tfim::Counters) * n_shapes;
    pl->sizes.total = off;
    pl->sizes.spins = tot_S;
    pl->sizes.couplings = tot_J;
    pl->sizes.labels = tot_lab;
    pl->sizes.tables = tot_tab;
    pl->sizes.measure = tot_meas;
    pl->t.assign(n_shapes, 0);
    pl->m.assign(n_shapes, 0);
    *out = pl;
    return TFIM_OK;
}

static void drop_events(tfim_plan* pl) {
    for (auto* v : {&pl->ev_used, &pl->ev_free})
        for (auto& e : *v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    pl->ev_used.clear();
    pl->ev_free.clear();
}

void tfim_plan_destroy(tfim_plan* pl) {
    if (!pl) return;
    drop_events(pl);
    for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
    delete pl;
}

tfim_status tfim_plan_sizes(const tfim_plan* pl, tfim_sizes* out) {
    if (!pl || !out) return fail(TFIM_EINVAL, "null argument");
    *out = pl->sizes;
    return TFIM_OK;
}

tfim_status tfim_bind(tfim_plan* pl, void* arena, size_t bytes, void* stream) {
    if (!pl || !arena) return fail(TFIM_EINVAL, "null plan or arena");
    if (bytes < pl->sizes.total) return fail(TFIM_EINVAL, "arena smaller than tfim_sizes.total");
    if (((uintptr_t)arena & 255) != 0) return fail(TFIM_EINVAL, "arena must be 256-byte aligned");
    pl->arena = (char*)arena;
    pl->stream = (hipStream_t)stream;
    pl->bound = true;
    pl->poisoned = false;
    for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
    pl->graphs.clear();
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < pl->shapes.size() && e == hipSuccess; ++i) {
        ShapeHost& h = pl->shapes[i];
        e = hipMemcpyAsync(pl->arena + h.oTu, h.Tu.data(), h.Tu.size() * 4, hipMemcpyHostToDevice, pl->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pl->arena + h.oTpt, h.Tpt.data(), h.Tpt.size() * 4, hipMemcpyHostToDevice, pl->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pl->arena + h.oTptOff, h.tpt_off.data(), h.tpt_off.size() * 4, hipMemcpyHostToDevice, pl->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pl->arena + h.oDmax, h.dmax.data(), h.dmax.size() * 4, hipMemcpyHostToDevice, pl->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pl->arena + h.oBtab, h.btab.data(), h.btab.size() * 8, hipMemcpyHostToDevice, pl->stream);
        h.J_ready = h.S_ready = false;
    }
    std::vector<tfim::Counters> c(pl->shapes.size());
    std::memset(c.data(), 0, c.size() * sizeof(tfim::Counters));
    if (e == hipSuccess)
        e = hipMemcpyAsync(pl->arena + pl->oCounters, c.data(), c.size() * sizeof(tfim::Counters),
                           hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    std::fill(pl->t.begin(), pl->t.end(), 0);
    std::fill(pl->m.begin(), pl->m.end(), 0);
    return check_hip(pl, e, "bind");
}

static tfim_status shape_ok(tfim_plan* pl, uint32_t shape) {
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    if (shape >= pl->shapes.size()) return fail(TFIM_EINVAL, "shape index out of range");
    return TFIM_OK;
}

static tfim_status reset_counters(tfim_plan* pl) {
    std::vector<tfim::Counters> c(pl->shapes.size());
    std::memset(c.data(), 0, c.size() * sizeof(tfim::Counters));
    hipError_t e = hipMemcpyAsync(pl->arena + pl->oCounters, c.data(), c.size() * sizeof(tfim::Counters),
                                  hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    std::fill(pl->t.begin(), pl->t.end(), 0);
    std::fill(pl->m.begin(), pl->m.end(), 0);
    return check_hip(pl, e, "reset counters");
}

tfim_status tfim_init_couplings(tfim_plan* pl, uint32_t shape, const uint64_t* J_host) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    const tfim::ShapeDev d = dev_of(pl, shape);
    hipError_t e;
    if (J_host) {
        e = hipMemcpyAsync(d.J, J_host, h.nJ, hipMemcpyHostToDevice, pl->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    } else {
        e = tfim::launch_init_couplings(d, pl->seed, pl->stream);
    }
    st = check_hip(pl, e, "init couplings");
    if (st == TFIM_OK) {
        h.J_ready = true;
        h.S_ready = false;
    }
    return st;
}

static hipError_t refresh_derived(tfim_plan* pl, uint32_t shape) {
    const tfim::ShapeDev d = dev_of(pl, shape);
    hipError_t e = tfim::launch_energy(d, pl->stream);
    if (e == hipSuccess) e = tfim::launch_mask_rebuild(d, pl->stream);
    return e;
}

tfim_status tfim_init_spins(tfim_plan* pl, uint32_t shape, const uint64_t* S_host) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (!h.J_ready) return fail(TFIM_ESTATE, "couplings of this shape are not initialised");
    const tfim::ShapeDev d = dev_of(pl, shape);
    hipError_t e;
    if (S_host) {
        e = hipMemcpyAsync(d.S, S_host, h.nS, hipMemcpyHostToDevice, pl->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    } else {
        e = tfim::launch_init_spins(d, pl->seed, pl->stream);
    }
    if (e == hipSuccess) e = tfim::launch_labels_identity(d, pl->stream);
    if (e == hipSuccess) e = refresh_derived(pl, shape);
    st = check_hip(pl, e, "init spins");
    if (st != TFIM_OK) return st;
    h.S_ready = true;
    return reset_counters(pl);
}

static tfim_status all_ready(tfim_plan* pl) {
    for (auto& h : pl->shapes)
        if (!h.S_ready) return fail(TFIM_ESTATE, "every shape needs couplings and spins before sweeping");
    return TFIM_OK;
}

static hipError_t timed_sweep(tfim_plan* pl, int i, bool energy) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    hipError_t e = hipSuccess;
    if (pl->timing) {
        if (pl->ev_free.empty()) {
            e = hipEventCreate(&ev.first);
            if (e == hipSuccess) e = hipEventCreate(&ev.second);
            if (e != hipSuccess) return e;
        } else {
            ev = pl->ev_free.back();
            pl->ev_free.pop_back();
        }
        e = hipEventRecord(ev.first, pl->stream);
    }
    if (e == hipSuccess)
        e = tfim::launch_sweep(dev_of(pl, i), pl->seed, counters_of(pl, i), pl->variant, energy,
                               pl->stream);
    if (pl->timing) {
        if (e == hipSuccess) e = hipEventRecord(ev.second, pl->stream);
        pl->ev_used.push_back(ev);
    }
    return e;
}

// Enqueue one sweep of every shape (plus due tempering) with the per-shape
// schedule; the host mirrors pl->t hold each shape's sweep counter.  U is
// recounted when a tempering step follows or when the caller will see it.
static hipError_t enqueue_sweep(tfim_plan* pl, bool last) {
    hipError_t e = hipSuccess;
    const int ns = (int)pl->shapes.size();
    for (int i = 0; i < ns && e == hipSuccess; ++i) {
        const uint32_t pe = pl->shapes[i].s.pt_every;
        const bool due = pe > 0 && ((pl->t[i] + 1) % pe) == 0;
        e = timed_sweep(pl, i, due || last);
    }
    for (int i = 0; i < ns && e == hipSuccess; ++i) {
        const uint32_t pe = pl->shapes[i].s.pt_every;
        const bool due = pe > 0 && ((pl->t[i] + 1) % pe) == 0;
        if (due) e = tfim::launch_temper(dev_of(pl, i), pl->seed, counters_of(pl, i), pl->stream);
        if (e == hipSuccess) e = tfim::launch_advance(counters_of(pl, i), 1u, due ? 1u : 0u, pl->stream);
    }
    return e;
}

tfim_status tfim_sweep(tfim_plan* pl, uint64_t n) {
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    if ((st = all_ready(pl)) != TFIM_OK) return st;
    if (n == 0) return TFIM_OK;
    for (size_t i = 0; i < pl->shapes.size(); ++i)
        if (pl->t[i] + n > 0xFFFFFFFFull) return fail(TFIM_EOVERFLOW, "sweep counter would pass 2^32-1");
    hipError_t e = hipSuccess;
    for (uint64_t s = 0; s < n && e == hipSuccess; ++s) {
        e = enqueue_sweep(pl, s + 1 == n);
        if (e != hipSuccess) break;
        for (size_t i = 0; i < pl->shapes.size(); ++i) {
            const uint32_t pe = pl->shapes[i].s.pt_every;
            if (pe > 0 && ((pl->t[i] + 1) % pe) == 0) pl->m[i] += 1;
            pl->t[i] += 1;
        }
    }
    return check_hip(pl, e, "sweep");
}

tfim_status tfim_pt_swap(tfim_plan* pl) {
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    if ((st = all_ready(pl)) != TFIM_OK) return st;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < pl->shapes.size() && e == hipSuccess; ++i) {
        if (pl->m[i] + 1 > 0xFFFFFFFFull) return fail(TFIM_EOVERFLOW, "tempering counter overflow");
        e = tfim::launch_temper(dev_of(pl, (int)i), pl->seed, counters_of(pl, (int)i), pl->stream);
        if (e == hipSuccess) e = tfim::launch_advance(counters_of(pl, (int)i), 0u, 1u, pl->stream);
        pl->m[i] += 1;
    }
    return check_hip(pl, e, "pt_swap");
}

tfim_status tfim_sync(tfim_plan* pl) {
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    return check_hip(pl, hipStreamSynchronize(pl->stream), "sync");
}

static tfim_status copy_back(tfim_plan* pl, void* dst, const void* src, size_t n, const char* what) {
    hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    return check_hip(pl, e, what);
}

tfim_status tfim_export_spins(tfim_plan* pl, uint32_t shape, uint64_t* S_host) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    if (!S_host) return fail(TFIM_EINVAL, "null host pointer");
    const ShapeHost& h = pl->shapes[shape];
    return copy_back(pl, S_host, pl->arena + h.oS, h.nS, "export spins");
}

tfim_status tfim_export_couplings(tfim_plan* pl, uint32_t shape, uint64_t* J_host) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    if (!J_host) return fail(TFIM_EINVAL, "null host pointer");
    const ShapeHost& h = pl->shapes[shape];
    return copy_back(pl, J_host, pl->arena + h.oJ, h.nJ, "export couplings");
}

tfim_status tfim_get_state(tfim_plan* pl, uint32_t shape, uint8_t* kidx, uint32_t* U) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    const ShapeHost& h = pl->shapes[shape];
    if (kidx && (st = copy_back(pl, kidx, pl->arena + h.oK, h.nLab, "get kidx")) != TFIM_OK) return st;
    if (U && (st = copy_back(pl, U, pl->arena + h.oU, h.nLab * 4, "get U")) != TFIM_OK) return st;
    return TFIM_OK;
}

tfim_status tfim_get_counters(const tfim_plan* pl, uint32_t shape, uint64_t* t, uint64_t* m) {
    if (!pl) return fail(TFIM_EINVAL, "null plan");
    if (shape >= pl->shapes.size()) return fail(TFIM_EINVAL, "shape index out of range");
    if (t) *t = pl->t[shape];
    if (m) *m = pl->m[shape];
    return TFIM_OK;
}

tfim_status tfim_set_state(tfim_plan* pl, uint32_t shape, const uint64_t* S_host,
                           const uint8_t* kidx_host, uint64_t t, uint64_t m) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (!h.J_ready) return fail(TFIM_ESTATE, "couplings of this shape are not initialised");
    if (!S_host || !kidx_host) return fail(TFIM_EINVAL, "null host pointer");
    if (t > 0xFFFFFFFFull || m > 0xFFFFFFFFull) return fail(TFIM_EOVERFLOW, "counter beyond 2^32-1");
    const size_t nk = h.s.n_k;
    std::vector<uint8_t> winv(h.nLab);
    for (size_t g = 0; g < h.nLab / nk; ++g) {
        std::vector<int> seen(nk, 0);
        for (size_t w = 0; w < nk; ++w) {
            const uint8_t i = kidx_host[g * nk + w];
            if (i >= nk || seen[i]) return fail(TFIM_EINVAL, "k labels of a (replica, sample) are not a permutation");
            seen[i] = 1;
            winv[g * nk + i] = (uint8_t)w;
        }
    }
    const tfim::ShapeDev d = dev_of(pl, shape);
    hipError_t e = hipMemcpyAsync(d.S, S_host, h.nS, hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.kidx, kidx_host, h.nLab, hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.winv, winv.data(), h.nLab, hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = refresh_derived(pl, shape);
    tfim::Counters c{};
    c.t = (uint32_t)t;
    c.m = (uint32_t)m;
    if (e == hipSuccess)
        e = hipMemcpyAsync(counters_of(pl, (int)shape), &c, sizeof c, hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    st = check_hip(pl, e, "set state");
    if (st != TFIM_OK) return st;
    h.S_ready = true;
    pl->t[shape] = t;
    pl->m[shape] = m;
    return TFIM_OK;
}

tfim_status tfim_get_thresholds(const tfim_plan* pl, uint32_t shape, uint32_t* Tm, uint32_t* dmax,
                                uint32_t* Tpt, size_t cap, size_t* n_tpt) {
    if (!pl) return fail(TFIM_EINVAL, "null plan");
    if (shape >= pl->shapes.size()) return fail(TFIM_EINVAL, "shape index out of range");
    const ShapeHost& h = pl->shapes[shape];
    const size_t nk = h.s.n_k;
    size_t tot = 0;
    for (size_t i = 0; i + 1 < nk; ++i) tot += h.dmax[i];
    if (n_tpt) *n_tpt = tot;
    if (Tm) std::memcpy(Tm, h.Tu.data(), nk * 3 * 4);
    if (dmax && nk > 1) std::memcpy(dmax, h.dmax.data(), (nk - 1) * 4);
    if (Tpt) {
        if (cap < tot) return fail(TFIM_EINVAL, "Tpt capacity too small");
        if (tot) std::memcpy(Tpt, h.Tpt.data(), tot * 4);
    }
    return TFIM_OK;
}

tfim_status tfim_xi2(const int64_t* A, uint32_t L, uint32_t n_k, double* xi) {
    if (!A || !xi || L < 2) return fail(TFIM_EINVAL, "bad xi2 arguments");
    const double pi = 3.14159265358979323846;
    std::vector<double> cosv(L);
    for (uint32_t d = 0; d < L; ++d) cosv[d] = std::cos(2.0 * pi * (double)d / (double)L);
    const double s = 2.0 * std::sin(pi / (double)L);
    for (uint32_t i = 0; i < n_k; ++i) {
        // exact integer chi; F as a compensated FP64 sum
        __int128 chi_i = 0;
        double F = 0.0, comp = 0.0;
        for (uint32_t d = 0; d < L; ++d) {
            const int64_t a = A[(size_t)i * L + d];
            chi_i += a;
            const double term = (double)a * cosv[d];
            const double y = term - comp;
            const double tsum = F + y;
            comp = (tsum - F) - y;
            F = tsum;
        }
        const double chi = (double)chi_i;
        if (F <= 0.0) {
            xi[i] = INFINITY;
            continue;
        }
        const double ratio = chi / F;
        xi[i] = ratio < 1.0 ? NAN : std::sqrt(ratio - 1.0) / s;
    }
    return TFIM_OK;
}

tfim_status tfim_set_timing(tfim_plan* pl, uint32_t enable) {
    if (!pl) return fail(TFIM_EINVAL, "null plan");
    pl->timing = enable != 0;
    return TFIM_OK;
}

tfim_status tfim_get_timing(tfim_plan* pl, double* ms_total, uint64_t* launches) {
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    double tot = 0.0;
    hipError_t e = hipStreamSynchronize(pl->stream);
    for (auto& ev : pl->ev_used) {
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.first, ev.second);
        tot += ms;
        pl->ev_free.push_back(ev);
    }
    const uint64_t n = pl->ev_used.size();
    pl->ev_used.clear();
    if (ms_total) *ms_total = tot;
    if (launches) *launches = n;
    return check_hip(pl, e, "timing");
}

tfim_status tfim_set_variant(tfim_plan* pl, uint32_t variant) {
    if (!pl) return fail(TFIM_EINVAL, "null plan");
    if (variant >= (uint32_t)tfim::sweep_variants()) return fail(TFIM_EINVAL, "unknown sweep variant");
    pl->variant = (int)variant;
    return TFIM_OK;
}

tfim_status tfim_set_schedule(tfim_plan* pl, uint32_t schedule) {
    if (!pl) return fail(TFIM_EINVAL, "null plan");
    if (schedule != TFIM_SCHED_PER_SHAPE && schedule != TFIM_SCHED_BATCHED)
        return fail(TFIM_EINVAL, "unknown schedule");
    if (schedule == TFIM_SCHED_BATCHED) return fail(TFIM_EUNSUPPORTED, "batched schedule not built yet");
    pl->schedule = schedule;
    return TFIM_OK;
}

tfim_status tfim_autotune(tfim_plan* pl, uint32_t sweeps_per_trial) {
    (void)sweeps_per_trial;
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    return fail(TFIM_EUNSUPPORTED, "autotuner not built yet");
}

tfim_status tfim_get_tuning(const tfim_plan* pl, uint32_t* config_id, double* ms) {
    if (!pl) return fail(TFIM_EINVAL, "null plan");
    if (config_id) *config_id = (uint32_t)pl->variant;
    if (ms) *ms = pl->tuned_ms;
    return TFIM_OK;
}

static tfim_status measure_core(tfim_plan* pl, uint32_t shape, uint32_t mode, uint32_t cfg0,
                                uint32_t ncfg, uint32_t flags) {
    ShapeHost& h = pl->shapes[shape];
    if (!h.S_ready) return fail(TFIM_ESTATE, "spins of this shape are not initialised");
    const tfim::ShapeDev d = dev_of(pl, shape);
    if (!tfim::measure_ok(d)) return fail(TFIM_EUNSUPPORTED, "measurement needs 2..4 replicas");
    const uint64_t ncfg_all = (uint64_t)h.s.n_k * 64 * h.s.n_words;
    if ((uint64_t)cfg0 + ncfg > ncfg_all) return fail(TFIM_EINVAL, "configuration range out of bounds");
    if (mode > 1) return fail(TFIM_EINVAL, "unknown measurement mode");
    const size_t rl = (size_t)(2 * h.s.L + 3) * h.P * 8;
    hipError_t e = hipMemsetAsync(pl->arena + h.oRec + (size_t)cfg0 * rl, 0, (size_t)ncfg * rl, pl->stream);
    if (e == hipSuccess && !(flags & TFIM_MEASURE_REUSE_LAYOUT)) e = tfim::launch_transpose(d, pl->stream);
    if (e == hipSuccess) e = tfim::launch_measure(d, (int)mode, (int)cfg0, (int)ncfg, pl->stream);
    return check_hip(pl, e, "measure");
}

tfim_status tfim_measure(tfim_plan* pl, uint32_t shape, uint32_t what, void* out, size_t bytes) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (!out) return fail(TFIM_EINVAL, "null host pointer");
    const size_t S = 64 * (size_t)h.s.n_words, nk = h.s.n_k, R = h.s.n_replicas;
    if (what == TFIM_MEASURE_ENERGY) {
        if (bytes < R * S * nk * 4) return fail(TFIM_EINVAL, "output buffer too small");
        std::vector<uint8_t> winv(h.nLab);
        std::vector<uint32_t> U(h.nLab);
        if ((st = copy_back(pl, winv.data(), pl->arena + h.oWinv, h.nLab, "get winv")) != TFIM_OK) return st;
        if ((st = copy_back(pl, U.data(), pl->arena + h.oU, h.nLab * 4, "get U")) != TFIM_OK) return st;
        uint32_t* o = (uint32_t*)out;
        for (size_t g = 0; g < R * S; ++g)
            for (size_t i = 0; i < nk; ++i) o[g * nk + i] = U[g * nk + winv[g * nk + i]];
        return TFIM_OK;
    }
    if (what != TFIM_MEASURE_RECORDS && what != TFIM_MEASURE_BUCKETS)
        return fail(TFIM_EINVAL, "unknown measurement");
    const size_t need = what == TFIM_MEASURE_RECORDS ? h.nRec : h.nBuck;
    if (bytes < need) return fail(TFIM_EINVAL, "output buffer too small");
    if ((st = measure_core(pl, shape, pl->measure_mode, 0, (uint32_t)(nk * S), 0)) != TFIM_OK) return st;
    if (what == TFIM_MEASURE_BUCKETS) {
        const hipError_t e = tfim::launch_buckets(dev_of(pl, (int)shape), pl->stream);
        if ((st = check_hip(pl, e, "buckets")) != TFIM_OK) return st;
        return copy_back(pl, out, pl->arena + h.oBuck, h.nBuck, "copy buckets");
    }
    return copy_back(pl, out, pl->arena + h.oRec, h.nRec, "copy records");
}

tfim_status tfim_measure_range(tfim_plan* pl, uint32_t shape, uint32_t mode, uint32_t cfg0,
                               uint32_t ncfg, uint32_t flags, int64_t* out, size_t bytes) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    const size_t rl = (size_t)(2 * h.s.L + 3) * h.P * 8;
    if (out && bytes < (size_t)ncfg * rl) return fail(TFIM_EINVAL, "output buffer too small");
    if ((st = measure_core(pl, shape, mode, cfg0, ncfg, flags)) != TFIM_OK) return st;
    if (!out) return TFIM_OK;
    return copy_back(pl, out, pl->arena + h.oRec + (size_t)cfg0 * rl, (size_t)ncfg * rl, "copy records");
}

tfim_status tfim_set_measure_mode(tfim_plan* pl, uint32_t mode) {
    if (!pl) return fail(TFIM_EINVAL, "null plan");
    if (mode > 1) return fail(TFIM_EINVAL, "unknown measurement mode");
    pl->measure_mode = mode;
    return TFIM_OK;
}

tfim_status tfim_dump_gram(tfim_plan* pl, uint32_t shape, uint32_t i, uint32_t s, uint32_t a,
                           uint32_t b, int32_t* Ga, int32_t* Gb, int32_t* Q) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (!h.S_ready) return fail(TFIM_ESTATE, "spins of this shape are not initialised");
    const size_t S = 64 * (size_t)h.s.n_words;
    if (i >= h.s.n_k || s >= S || a >= h.s.n_replicas || b >= h.s.n_replicas)
        return fail(TFIM_EINVAL, "index out of range");
    if (h.P == 0) return fail(TFIM_EUNSUPPORTED, "needs at least two replicas");
    const tfim::ShapeDev d = dev_of(pl, shape);
    hipError_t e = tfim::launch_transpose(d, pl->stream);
    if (e == hipSuccess) e = tfim::launch_dump(d, (int)(i * S + s), (int)a, (int)b, pl->stream);
    if ((st = check_hip(pl, e, "dump")) != TFIM_OK) return st;
    const size_t n1 = (size_t)d.L2 * d.L2 * 4, n2 = (size_t)d.Lt * d.Lt * 4;
    char* base = pl->arena + h.oDump;
    if (Ga && (st = copy_back(pl, Ga, base, n1, "dump Ga")) != TFIM_OK) return st;
    if (Gb && (st = copy_back(pl, Gb, base + n1, n1, "dump Gb")) != TFIM_OK) return st;
    if (Q && (st = copy_back(pl, Q, base + 2 * n1, n2, "dump Q")) != TFIM_OK) return st;
    return TFIM_OK;
}

}  // extern "C"
