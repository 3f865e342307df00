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
    int device = 0;           // current device at tfim_bind
    bool bound = false;
    bool poisoned = false;   // sticky: set by a device error, never cleared
    uint32_t form = TFIM_FORM_MULTISPIN;
    // failure injection (TFIM_FAIL_AFTER): the n-th enqueueing call fails
    int64_t fail_after = 0;
    std::vector<uint64_t> t, m;  // host mirrors per shape
    uint32_t schedule = TFIM_SCHED_PER_SHAPE;
    int variant = 3;  // helper waves where L = 24, else the streaming kernel
    uint32_t measure_mode = 0;
    double tuned_ms = 0.0;
    // batched schedule: arena region (ShapeDev[ns], first[ns+1], queue,
    // items[]), geometry, and the graphs of 1..kGraphSweeps sweeps
    size_t oBatch = 0, oFirst = 0, oQueue = 0, oItems = 0, max_items = 0;
    uint32_t batch_threads = 0, batch_bpc = 0, batch_blocks = 0, temper_blocks = 0;
    size_t batch_lds = 0;
    std::vector<uint64_t> items;
    int max_nk = 0, n_cu = 0;
    bool any_pt = false;
    bool batch_anti = false;  // some shape is antiperiodic: the batched kernel checks the tau mask
    hipStream_t cap_stream = nullptr;
    std::vector<hipStream_t> side;                // concurrent schedule: one branch per shape
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    bool tables_up = false;                       // shape table and tempering ranges uploaded
    std::map<uint32_t, hipGraphExec_t> graphs;  // (schedule, sweeps per replay) -> graph
    // HIP-event timing (tfim_set_timing): event pairs and the launches each covers
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
    std::vector<uint32_t> ev_n;
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
    d.apm = h.s.bc_tau == TFIM_BC_ANTIPERIODIC ? ~0ull : 0ull;
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

// Failure injection: counts the calls that enqueue device work; the
// fail_after-th one enqueues nothing and fails as a device error does
// (TFIM_EDEVICE, plan poisoned).  Off when fail_after is 0.
tfim_status injected(tfim_plan* pl) {
    if (pl->fail_after <= 0) return TFIM_OK;
    if (--pl->fail_after > 0) return TFIM_OK;
    pl->poisoned = true;
    return fail(TFIM_EDEVICE, "injected device failure (TFIM_FAIL_AFTER)");
}

bool plain(const tfim_plan* pl) { return pl->form == TFIM_FORM_PLAIN_I8; }

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

tfim_status validate(const tfim_shape* s, uint32_t n, uint32_t form) {
    if (form != TFIM_FORM_MULTISPIN && form != TFIM_FORM_PLAIN_I8) return fail(TFIM_EINVAL, "unknown form");
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
        // PLAIN_I8: n_words counts samples, sample s using word word_offset + s/64
        const uint64_t words = form == TFIM_FORM_PLAIN_I8 ? ((uint64_t)a.n_words + 63) / 64 : a.n_words;
        if (a.n_words == 0 || (uint64_t)a.word_offset + words > (1u << 20))
            return fail(TFIM_EINVAL, "n_words must be >= 1 and the words used must end below 2^20");
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
        if (a.bc_tau != TFIM_BC_PERIODIC && a.bc_tau != TFIM_BC_ANTIPERIODIC)
            return fail(TFIM_EINVAL, "unknown bc_tau");
        if (a.Ltau % 8 != 0 && form == TFIM_FORM_MULTISPIN)
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
                             uint32_t form, tfim_plan** out) {
    if (!out) return fail(TFIM_EINVAL, "null output pointer");
    *out = nullptr;
    tfim_status st = validate(shapes, n_shapes, form);
    if (st != TFIM_OK) return st;
    tfim_plan* pl = new tfim_plan();
    pl->seed = seed;
    pl->form = form;
    const bool pf = form == TFIM_FORM_PLAIN_I8;
    if (const char* fa = std::getenv("TFIM_FAIL_AFTER")) pl->fail_after = std::max(0ll, std::atoll(fa));
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
                     R = h.s.n_replicas, Lt = h.s.Ltau, S = pf ? W : 64 * W;
        h.nc = (int)((Lt + 63) / 64);
        h.nx = (int)((L2 + 63) / 64);
        h.nLab = R * S * nk;
        h.nRec = h.P ? nk * S * h.P * (2 * h.s.L + 3) * 8 : 0;
        h.nBuck = nk * 2 * h.s.L * 8;
        if (pf) {
            // one byte per spin and coupling; no lane masks or bit layouts
            h.nS = R * nk * S * Lt * L2;
            h.nJ = S * 2 * L2;
        } else {
            h.nS = R * nk * W * Lt * L2 * 8;
            h.nJ = W * 2 * L2 * 8;
            h.nMask = R * W * nk * (nk + 1) * 8;
            // bit layouts for every measurement, the one-replica two-time records included
            h.nPt = nk * S * R * (size_t)h.nc * 64 * h.nx * 8;
            h.nPx = nk * S * R * (size_t)h.nx * Lt * 8;
            h.nDump = h.P ? (2 * L2 * L2 + Lt * Lt) * 4 : 0;
        }
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
    size_t nitems = 0;
    for (auto& h : pl->shapes) nitems += (size_t)h.s.n_replicas * h.s.n_k * h.s.n_words;
    pl->oBatch = off; off = align256(off + sizeof(tfim::ShapeDev) * n_shapes);
    pl->oFirst = off; off = align256(off + 4 * (size_t)(n_shapes + 1));
    pl->oQueue = off; off = align256(off + sizeof(tfim::BatchQueue));
    pl->oItems = off; off = align256(off + 8 * nitems);
    pl->max_items = nitems;
    tot_tab += sizeof(tfim::ShapeDev) * n_shapes + 4 * (n_shapes + 1) + sizeof(tfim::BatchQueue) + 8 * nitems;
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
    pl->ev_n.clear();
}

static void drop_graphs(tfim_plan* pl) {
    for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
    pl->graphs.clear();
}

void tfim_plan_destroy(tfim_plan* pl) {
    if (!pl) return;
    drop_events(pl);
    drop_graphs(pl);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    for (auto st : pl->side) (void)hipStreamDestroy(st);
    if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
    for (auto ev : pl->ev_join) (void)hipEventDestroy(ev);
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
    if (pl->poisoned) return fail(TFIM_ESTATE, "plan poisoned by an earlier device error");
    pl->arena = (char*)arena;
    pl->stream = (hipStream_t)stream;
    pl->bound = true;
    drop_graphs(pl);
    pl->batch_threads = pl->batch_bpc = pl->batch_blocks = 0;
    pl->tables_up = false;
    pl->schedule = TFIM_SCHED_PER_SHAPE;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    pl->device = dev;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&pl->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && !pl->cap_stream) e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipMemsetAsync(pl->arena + pl->oQueue, 0, sizeof(tfim::BatchQueue), pl->stream);
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

// Plain-form host arrays must hold +1 / -1 bytes only.
static bool plus_minus_one(const void* p, size_t n) {
    const int8_t* b = (const int8_t*)p;
    for (size_t i = 0; i < n; ++i)
        if (b[i] != 1 && b[i] != -1) return false;
    return true;
}

tfim_status tfim_init_couplings(tfim_plan* pl, uint32_t shape, const void* J_host) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (J_host && plain(pl) && !plus_minus_one(J_host, h.nJ))
        return fail(TFIM_EINVAL, "plain-form couplings must be +1 or -1");
    if ((st = injected(pl)) != TFIM_OK) return st;
    const tfim::ShapeDev d = dev_of(pl, shape);
    hipError_t e;
    if (J_host) {
        e = hipMemcpyAsync(d.J, J_host, h.nJ, hipMemcpyHostToDevice, pl->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    } else if (plain(pl)) {
        e = tfim::plain_init_couplings(d, pl->seed, pl->stream);
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
    if (plain(pl)) return tfim::plain_energy(d, pl->stream);
    hipError_t e = tfim::launch_energy(d, pl->stream);
    if (e == hipSuccess) e = tfim::launch_mask_rebuild(d, pl->stream);
    return e;
}

tfim_status tfim_init_spins(tfim_plan* pl, uint32_t shape, const void* S_host) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (!h.J_ready) return fail(TFIM_ESTATE, "couplings of this shape are not initialised");
    if (S_host && plain(pl) && !plus_minus_one(S_host, h.nS))
        return fail(TFIM_EINVAL, "plain-form spins must be +1 or -1");
    if ((st = injected(pl)) != TFIM_OK) return st;
    const tfim::ShapeDev d = dev_of(pl, shape);
    hipError_t e;
    if (S_host) {
        e = hipMemcpyAsync(d.S, S_host, h.nS, hipMemcpyHostToDevice, pl->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    } else if (plain(pl)) {
        e = tfim::plain_init_spins(d, pl->seed, pl->stream);
    } else {
        e = tfim::launch_init_spins(d, pl->seed, pl->stream);
    }
    if (e == hipSuccess)
        e = plain(pl) ? tfim::plain_labels_identity(d, pl->stream) : tfim::launch_labels_identity(d, pl->stream);
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

// A pair of timing events around one launch (or graph replay) covering n
// sweep launches, when timing is on.
static hipError_t timing_begin(tfim_plan* pl, std::pair<hipEvent_t, hipEvent_t>& ev) {
    ev = {nullptr, nullptr};
    if (!pl->timing) return hipSuccess;
    hipError_t e = hipSuccess;
    if (pl->ev_free.empty()) {
        e = hipEventCreate(&ev.first);
        if (e == hipSuccess) e = hipEventCreate(&ev.second);
        if (e != hipSuccess) return e;
    } else {
        ev = pl->ev_free.back();
        pl->ev_free.pop_back();
    }
    return hipEventRecord(ev.first, pl->stream);
}

static hipError_t timing_end(tfim_plan* pl, std::pair<hipEvent_t, hipEvent_t>& ev, uint32_t n,
                             hipError_t e) {
    if (!pl->timing) return e;
    if (e == hipSuccess) e = hipEventRecord(ev.second, pl->stream);
    pl->ev_used.push_back(ev);
    pl->ev_n.push_back(n);
    return e;
}

static hipError_t timed_sweep(tfim_plan* pl, int i, bool energy) {
    std::pair<hipEvent_t, hipEvent_t> ev;
    hipError_t e = timing_begin(pl, ev);
    if (e == hipSuccess && plain(pl))
        e = tfim::plain_sweep(dev_of(pl, i), pl->seed, counters_of(pl, i), pl->stream);
    else if (e == hipSuccess)
        e = tfim::launch_sweep(dev_of(pl, i), pl->seed, counters_of(pl, i), pl->variant, energy,
                               pl->stream);
    return timing_end(pl, ev, 1, e);
}

static hipError_t temper(tfim_plan* pl, int i) {
    if (plain(pl)) return tfim::plain_temper(dev_of(pl, i), pl->seed, counters_of(pl, i), pl->stream);
    return tfim::launch_temper(dev_of(pl, i), pl->seed, counters_of(pl, i), pl->stream);
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
        if (due) e = temper(pl, i);
        if (e == hipSuccess) e = tfim::launch_advance(counters_of(pl, i), 1u, due ? 1u : 0u, pl->stream);
    }
    return e;
}

// ---------------------------------------------------------------------------
// Batched schedule
// ---------------------------------------------------------------------------
constexpr uint32_t kGraphSweeps = 16;        // sweeps captured per graph
constexpr uint32_t kMaxBatchThreads = 768;   // launch bound of the batched kernel
constexpr size_t kLdsLimit = 160 * 1024 - 256;

static tfim::BatchArgs batch_args(const tfim_plan* pl) {
    tfim::BatchArgs a{};
    for (int i = 0; i < (int)pl->shapes.size() && i < tfim::kMaxBatchShapes; ++i) a.shapes[i] = dev_of(pl, i);
    a.items = (const uint64_t*)(pl->arena + pl->oItems);
    a.q = (tfim::BatchQueue*)(pl->arena + pl->oQueue);
    a.ctr = counters_of(pl, 0);
    a.n_items = (uint32_t)pl->items.size();
    a.key0 = (uint32_t)pl->seed;
    a.key1 = (uint32_t)(pl->seed >> 32);
    return a;
}

static tfim::TemperBatchArgs temper_args(const tfim_plan* pl) {
    tfim::TemperBatchArgs a{};
    a.shapes = (const tfim::ShapeDev*)(pl->arena + pl->oBatch);
    a.first = (const uint32_t*)(pl->arena + pl->oFirst);
    a.ctr = counters_of(pl, 0);
    a.n_shapes = (uint32_t)pl->shapes.size();
    a.key0 = (uint32_t)pl->seed;
    a.key1 = (uint32_t)(pl->seed >> 32);
    return a;
}

// The device shape table and the first tempering block of each shape, used
// by the all-shape tempering and counter-advance launches of the batched and
// concurrent schedules.
static tfim_status upload_tables(tfim_plan* pl) {
    const int ns = (int)pl->shapes.size();
    std::vector<tfim::ShapeDev> devs(ns);
    std::vector<uint32_t> first(ns + 1, 0);
    int max_nk = 0;
    bool any_pt = false;
    for (int i = 0; i < ns; ++i) {
        devs[i] = dev_of(pl, i);
        first[i + 1] = first[i] + (uint32_t)(devs[i].R * devs[i].W);
        max_nk = std::max(max_nk, devs[i].nk);
        any_pt = any_pt || devs[i].pt_every != 0;
    }
    hipError_t e = hipMemcpyAsync(pl->arena + pl->oBatch, devs.data(), sizeof(tfim::ShapeDev) * ns,
                                  hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pl->arena + pl->oFirst, first.data(), 4 * first.size(), hipMemcpyHostToDevice,
                           pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    if (e != hipSuccess) return check_hip(pl, e, "shape table upload");
    pl->temper_blocks = first[ns];
    pl->max_nk = max_nk;
    pl->any_pt = any_pt;
    pl->tables_up = true;
    return TFIM_OK;
}

// Branch streams and fork/join events of the concurrent schedule, and the
// kernel attributes its captured launches need.
static tfim_status concurrent_setup(tfim_plan* pl) {
    const int ns = (int)pl->shapes.size();
    hipError_t e = hipSuccess;
    while ((int)pl->side.size() < ns && e == hipSuccess) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) pl->side.push_back(st);
    }
    if (e == hipSuccess && !pl->ev_fork) e = hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming);
    while (e == hipSuccess && (int)pl->ev_join.size() < ns) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) pl->ev_join.push_back(ev);
    }
    for (int i = 0; i < ns && e == hipSuccess; ++i) e = tfim::prepare_sweep(dev_of(pl, i), pl->variant, true);
    if (e != hipSuccess) return check_hip(pl, e, "concurrent setup");
    return pl->tables_up ? TFIM_OK : upload_tables(pl);
}

// Work items and geometry of the batched launch; uploads the shape table,
// the tempering block ranges and the items, rewinds the queue.
static tfim_status batch_setup(tfim_plan* pl, uint32_t threads, uint32_t bpc) {
    const int ns = (int)pl->shapes.size();
    if (ns > tfim::kMaxBatchShapes) return fail(TFIM_EUNSUPPORTED, "batched schedule takes at most 8 shapes");
    int maxcols = 0;
    for (int i = 0; i < ns; ++i) {
        const tfim::ShapeDev d = dev_of(pl, i);
        if (!tfim::sweep_stream_ok(d))
            return fail(TFIM_EUNSUPPORTED, "batched schedule needs every shape on the streaming sweep");
        maxcols = std::max(maxcols, tfim::sweep_stream_cols(d));
    }
    if (threads == 0) threads = (uint32_t)maxcols;
    if (threads % 64 || threads < (uint32_t)maxcols || threads > kMaxBatchThreads)
        return fail(TFIM_EINVAL, "batch threads must be a multiple of 64 in [largest L^2 rounded to 64, 768]");
    struct Item { uint64_t e; int Lt; size_t order; };
    std::vector<Item> it;
    size_t lds = 0;
    std::vector<tfim::ShapeDev> devs(ns);
    std::vector<uint32_t> first(ns + 1, 0);
    int max_nk = 0;
    bool any_pt = false, any_anti = false;
    for (int i = 0; i < ns; ++i) {
        const tfim::ShapeDev d = dev_of(pl, i);
        devs[i] = d;
        const int cols = tfim::sweep_stream_cols(d);
        int g = std::min<int>((int)threads / cols, 255);
        while (g > 1 && tfim::sweep_stream_lds_bytes(d, g, (int)threads, false) > kLdsLimit) --g;
        if (tfim::sweep_stream_lds_bytes(d, g, (int)threads, false) > kLdsLimit)
            return fail(TFIM_EUNSUPPORTED, "batched workgroup does not fit in LDS");
        lds = std::max(lds, tfim::sweep_stream_lds_bytes(d, g, (int)threads, false));
        if (threads == kMaxBatchThreads && tfim::sweep_helped_ok(d)) {
            g = 1;  // the batched kernel runs these configurations with helper waves
            lds = std::max(lds, tfim::sweep_helped_lds_bytes(d));
        }
        const int ncfg = d.R * d.nk * d.W;
        for (int c0 = 0; c0 < ncfg; c0 += g) {
            const uint64_t live = (uint64_t)std::min(g, ncfg - c0);
            it.push_back({(uint64_t)i | ((uint64_t)g << 8) | (live << 16) | ((uint64_t)c0 << 32), d.Lt,
                          it.size()});
        }
        first[i + 1] = first[i] + (uint32_t)(d.R * d.W);
        max_nk = std::max(max_nk, d.nk);
        any_pt = any_pt || d.pt_every != 0;
        any_anti = any_anti || d.apm != 0;
    }
    // longest items first (a sweep of a configuration takes time ~ Ltau)
    std::stable_sort(it.begin(), it.end(), [](const Item& a, const Item& b) { return a.Lt > b.Lt; });
    int per_cu = 0;
    hipError_t e = tfim::sweep_batch_prepare(1, any_anti, lds, (int)threads, &per_cu);
    if (e != hipSuccess) return check_hip(pl, e, "batch prepare");
    if (per_cu <= 0) return fail(TFIM_EUNSUPPORTED, "batched workgroup cannot be resident");
    if (bpc) per_cu = std::min<int>(per_cu, (int)bpc);
    std::vector<uint64_t> items(it.size());
    for (size_t k = 0; k < it.size(); ++k) items[k] = it[k].e;
    tfim_status ts = upload_tables(pl);
    if (ts != TFIM_OK) return ts;
    e = hipMemcpyAsync(pl->arena + pl->oItems, items.data(), 8 * items.size(), hipMemcpyHostToDevice,
                       pl->stream);
    if (e == hipSuccess) e = hipMemsetAsync(pl->arena + pl->oQueue, 0, sizeof(tfim::BatchQueue), pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    if (e != hipSuccess) return check_hip(pl, e, "batch upload");
    drop_graphs(pl);
    pl->items = std::move(items);
    pl->batch_threads = threads;
    pl->batch_bpc = bpc;
    pl->batch_blocks = (uint32_t)std::min<size_t>((size_t)pl->n_cu * per_cu, pl->items.size());
    pl->batch_lds = lds;
    pl->batch_anti = any_anti;
    (void)first;
    (void)max_nk;
    (void)any_pt;
    return TFIM_OK;
}

// The graph of g sweeps of the batched or concurrent schedule (captured
// once on the private stream).
static hipError_t batch_graph(tfim_plan* pl, uint32_t g, hipGraphExec_t* out) {
    const uint32_t key = g + 1000u * pl->schedule + 100000u * (uint32_t)pl->variant;
    auto f = pl->graphs.find(key);
    if (f != pl->graphs.end()) {
        *out = f->second;
        return hipSuccess;
    }
    tfim::BatchArgs a = batch_args(pl);
    const tfim::TemperBatchArgs ta = temper_args(pl);
    hipError_t e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    const int ns = (int)pl->shapes.size();
    for (uint32_t s = 0; s < g && le == hipSuccess; ++s) {
        if (pl->schedule == TFIM_SCHED_CONCURRENT) {
            // fork: every shape's sweep on its own branch; join before tempering
            le = hipEventRecord(pl->ev_fork, pl->cap_stream);
            for (int i = 0; i < ns && le == hipSuccess; ++i) {
                le = hipStreamWaitEvent(pl->side[i], pl->ev_fork, 0);
                if (le == hipSuccess)
                    le = tfim::launch_sweep(dev_of(pl, i), pl->seed, counters_of(pl, i), pl->variant, true,
                                            pl->side[i]);
                if (le == hipSuccess) le = hipEventRecord(pl->ev_join[i], pl->side[i]);
                if (le == hipSuccess) le = hipStreamWaitEvent(pl->cap_stream, pl->ev_join[i], 0);
            }
        } else {
            le = tfim::launch_sweep_batch(a, 1, pl->batch_anti, (int)pl->batch_blocks, (int)pl->batch_threads,
                                          pl->batch_lds, pl->cap_stream);
        }
        if (le == hipSuccess && pl->any_pt)
            le = tfim::launch_temper_batch(ta, (int)pl->temper_blocks, pl->max_nk, pl->cap_stream);
        if (le == hipSuccess) le = tfim::launch_advance_batch(ta, pl->cap_stream);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(pl->cap_stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return le != hipSuccess ? le : e;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    pl->graphs[key] = exec;
    *out = exec;
    return hipSuccess;
}

static hipError_t enqueue_batched(tfim_plan* pl, uint64_t n) {
    hipError_t e = hipSuccess;
    while (n > 0 && e == hipSuccess) {
        const uint32_t g = (uint32_t)std::min<uint64_t>(n, kGraphSweeps);
        hipGraphExec_t ex = nullptr;
        e = batch_graph(pl, g, &ex);
        if (e != hipSuccess) break;
        std::pair<hipEvent_t, hipEvent_t> ev;
        e = timing_begin(pl, ev);
        if (e == hipSuccess) e = hipGraphLaunch(ex, pl->stream);
        e = timing_end(pl, ev, g, e);
        n -= g;
    }
    return e;
}

static tfim_status sweep_impl(tfim_plan* pl, uint64_t n) {
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    if ((st = all_ready(pl)) != TFIM_OK) return st;
    if (n == 0) return TFIM_OK;
    for (size_t i = 0; i < pl->shapes.size(); ++i)
        if (n > 0xFFFFFFFFull - pl->t[i]) return fail(TFIM_EOVERFLOW, "sweep counter would pass 2^32-1");
    if ((st = injected(pl)) != TFIM_OK) return st;
    // host mirrors of the counters: tempering after sweeps t+1 .. t+n that
    // are multiples of pt_every
    auto advance = [pl](uint64_t k) {
        for (size_t i = 0; i < pl->shapes.size(); ++i) {
            const uint64_t pe = pl->shapes[i].s.pt_every;
            if (pe > 0) pl->m[i] += (pl->t[i] + k) / pe - pl->t[i] / pe;
            pl->t[i] += k;
        }
    };
    hipError_t e = hipSuccess;
    if (pl->schedule == TFIM_SCHED_BATCHED || pl->schedule == TFIM_SCHED_CONCURRENT) {
        e = enqueue_batched(pl, n);
        if (e == hipSuccess) advance(n);
    } else {
        for (uint64_t s = 0; s < n && e == hipSuccess; ++s) {
            e = enqueue_sweep(pl, s + 1 == n);  // reads the mirrors of this sweep
            if (e == hipSuccess) advance(1);
        }
    }
    return check_hip(pl, e, "sweep");
}

tfim_status tfim_sweep(tfim_plan* pl, uint64_t n) { return sweep_impl(pl, n); }

tfim_status tfim_pt_swap(tfim_plan* pl) {
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    if ((st = all_ready(pl)) != TFIM_OK) return st;
    for (size_t i = 0; i < pl->shapes.size(); ++i)
        if (pl->m[i] >= 0xFFFFFFFFull) return fail(TFIM_EOVERFLOW, "tempering counter overflow");
    if ((st = injected(pl)) != TFIM_OK) return st;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < pl->shapes.size() && e == hipSuccess; ++i) {
        e = temper(pl, (int)i);
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

tfim_status tfim_export_spins(tfim_plan* pl, uint32_t shape, void* S_host) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    if (!S_host) return fail(TFIM_EINVAL, "null host pointer");
    const ShapeHost& h = pl->shapes[shape];
    return copy_back(pl, S_host, pl->arena + h.oS, h.nS, "export spins");
}

tfim_status tfim_export_couplings(tfim_plan* pl, uint32_t shape, void* J_host) {
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

tfim_status tfim_set_state(tfim_plan* pl, uint32_t shape, const void* S_host,
                           const uint8_t* kidx_host, uint64_t t, uint64_t m) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (!h.J_ready) return fail(TFIM_ESTATE, "couplings of this shape are not initialised");
    if (!S_host || !kidx_host) return fail(TFIM_EINVAL, "null host pointer");
    if (plain(pl) && !plus_minus_one(S_host, h.nS)) return fail(TFIM_EINVAL, "plain-form spins must be +1 or -1");
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
    if ((st = injected(pl)) != TFIM_OK) return st;
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

static tfim_status tm_args(uint32_t L, double k, const int8_t* Jx, const int8_t* Jy) {
    if (const char* why = tfim::tm_unsupported((int)L)) return fail(TFIM_EUNSUPPORTED, why);
    if (!(k > 0.0) || !std::isfinite(k)) return fail(TFIM_EINVAL, "k must be finite and > 0");
    if (!Jx || !Jy) return fail(TFIM_EINVAL, "null couplings");
    for (uint32_t i = 0; i < L * L; ++i)
        if ((Jx[i] != 1 && Jx[i] != -1) || (Jy[i] != 1 && Jy[i] != -1))
            return fail(TFIM_EINVAL, "couplings must be +1 or -1");
    return TFIM_OK;
}

tfim_status tfim_tm_workspace(uint32_t L, size_t* bytes) {
    if (!bytes) return fail(TFIM_EINVAL, "null argument");
    if (const char* why = tfim::tm_unsupported((int)L)) return fail(TFIM_EUNSUPPORTED, why);
    *bytes = tfim::tm_workspace_bytes((int)L);
    return TFIM_OK;
}

tfim_status tfim_tm_apply(uint32_t L, double k, const int8_t* Jx, const int8_t* Jy, const double* v,
                          double* w, void* hip_stream) {
    tfim_status st = tm_args(L, k, Jx, Jy);
    if (st != TFIM_OK) return st;
    if (!v || !w || v == w) return fail(TFIM_EINVAL, "v and w must be distinct device vectors");
    const hipError_t e = tfim::tm_apply((int)L, k, Jx, Jy, v, w, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(TFIM_EDEVICE, std::string("transfer matrix: ") + hipGetErrorString(e));
    return TFIM_OK;
}

tfim_status tfim_tm_top(uint32_t L, double k, const int8_t* Jx, const int8_t* Jy, uint32_t sector,
                        uint32_t n_eig, double tol, uint32_t max_iter, void* ws, size_t ws_bytes,
                        void* hip_stream, double* lambda_out, uint32_t* iters_out) {
    tfim_status st = tm_args(L, k, Jx, Jy);
    if (st != TFIM_OK) return st;
    if (sector > 1) return fail(TFIM_EINVAL, "sector must be 0 (even) or 1 (odd)");
    if (n_eig < 1 || n_eig > 2) return fail(TFIM_EINVAL, "n_eig must be 1 or 2");
    if (!(tol > 0.0) || max_iter == 0 || !lambda_out) return fail(TFIM_EINVAL, "bad iteration arguments");
    if (!ws || ((uintptr_t)ws & 255)) return fail(TFIM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < tfim::tm_workspace_bytes((int)L)) return fail(TFIM_EINVAL, "workspace too small");
    double lam[2] = {0.0, 0.0};
    int it[2] = {0, 0};
    const hipError_t e = tfim::tm_top((int)L, k, Jx, Jy, (int)sector, (int)n_eig, tol,
                                      (int)std::min<uint32_t>(max_iter, 1u << 30), ws, lam, it,
                                      (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(TFIM_EDEVICE, std::string("transfer matrix: ") + hipGetErrorString(e));
    for (uint32_t q = 0; q < n_eig; ++q) {
        lambda_out[q] = lam[q];
        if (iters_out) iters_out[q] = (uint32_t)it[q];
    }
    return TFIM_OK;
}

tfim_status tfim_xi3(const int64_t* rec, uint32_t L, uint32_t n_k, uint32_t n_per_k,
                     uint32_t direction, double* xi) {
    if (!rec || !xi || L < 2 || direction > 2) return fail(TFIM_EINVAL, "bad xi3 arguments");
    const double pi = 3.14159265358979323846;
    const double s = 2.0 * std::sin(pi / (double)L);
    std::vector<__int128> A(L);
    for (uint32_t i = 0; i < n_k; ++i) {
        // exact bucket sums over records, then chi and a compensated F
        std::fill(A.begin(), A.end(), (__int128)0);
        for (uint32_t n = 0; n < n_per_k; ++n) {
            const int64_t* r = rec + ((size_t)i * n_per_k + n) * 2 * L;
            for (uint32_t d = 0; d < L; ++d) {
                if (direction != 1) A[d] += r[d];
                if (direction != 0) A[d] += r[L + d];
            }
        }
        __int128 chi_i = 0;
        double F = 0.0, comp = 0.0;
        for (uint32_t d = 0; d < L; ++d) {
            chi_i += A[d];
            const double term = (double)A[d] * std::cos(2.0 * pi * (double)d / (double)L);
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

tfim_status tfim_binder(const int64_t* rec, uint32_t L, uint32_t Ltau, uint32_t n_k,
                        uint32_t n_per_k, double* B) {
    if (!rec || !B || L < 2 || Ltau < 2) return fail(TFIM_EINVAL, "bad binder arguments");
    const size_t rl = 2 * (size_t)L + 3;
    for (uint32_t i = 0; i < n_k; ++i) {
        __int128 q2 = 0, q4 = 0;
        for (uint32_t n = 0; n < n_per_k; ++n) {
            const int64_t* r = rec + ((size_t)i * n_per_k + n) * rl;
            q2 += r[2 * L + 1];
            q4 += r[2 * L + 2];
        }
        if (q2 == 0) {
            B[i] = NAN;
            continue;
        }
        const long double lq2 = (long double)q2;
        B[i] = (double)((long double)Ltau * Ltau * n_per_k * (long double)q4 / (lq2 * lq2));
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
    uint64_t n = 0;
    for (uint32_t c : pl->ev_n) n += c;
    pl->ev_used.clear();
    pl->ev_n.clear();
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
    if (schedule != TFIM_SCHED_PER_SHAPE && schedule != TFIM_SCHED_BATCHED &&
        schedule != TFIM_SCHED_CONCURRENT)
        return fail(TFIM_EINVAL, "unknown schedule");
    if (schedule != TFIM_SCHED_PER_SHAPE && plain(pl))
        return fail(TFIM_EUNSUPPORTED, "the plain form runs the per-shape schedule only");
    if (schedule == TFIM_SCHED_BATCHED) {
        tfim_status st = usable(pl);
        if (st != TFIM_OK) return st;
        if (pl->batch_threads == 0 && (st = batch_setup(pl, 0, 0)) != TFIM_OK) return st;
    }
    if (schedule == TFIM_SCHED_CONCURRENT) {
        tfim_status st = usable(pl);
        if (st != TFIM_OK) return st;
        if ((st = concurrent_setup(pl)) != TFIM_OK) return st;
    }
    pl->schedule = schedule;
    return TFIM_OK;
}

tfim_status tfim_set_batch(tfim_plan* pl, uint32_t threads, uint32_t blocks_per_cu) {
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    if (plain(pl)) return fail(TFIM_EUNSUPPORTED, "the plain form runs the per-shape schedule only");
    return batch_setup(pl, threads, blocks_per_cu);
}

}  // extern "C"

namespace {

struct Choice {
    uint32_t schedule = TFIM_SCHED_PER_SHAPE, variant = 0, threads = 0, bpc = 0;
    double ms = 0.0;
};

// Cache key: device and every shape's geometry (results never depend on it).
std::string tune_key(const tfim_plan* pl) {
    std::string k;
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        k = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
    for (auto& h : pl->shapes) {
        char b[128];
        snprintf(b, sizeof b, "|%u,%u,%u,%u,%u,%u", h.s.L, h.s.Ltau, h.s.n_words, h.s.n_replicas, h.s.n_k,
                 h.s.pt_every);
        k += b;
    }
    return k;
}

// One JSON object per line: {"key": "...", "schedule": S, "variant": V,
// "threads": T, "blocks_per_cu": B, "ms_per_sweep": M}
bool read_field(const std::string& line, const char* name, double* v) {
    const std::string pat = std::string("\"") + name + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    return sscanf(line.c_str() + p + pat.size(), " %lf", v) == 1;
}

bool cache_lookup(const char* path, const std::string& key, Choice* c) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    const std::string want = "{\"key\": \"" + key + "\",";
    char buf[4096];
    bool found = false;
    while (fgets(buf, sizeof buf, f)) {
        const std::string line(buf);
        if (line.compare(0, want.size(), want) != 0) continue;
        double s, v, t, b, m;
        if (read_field(line, "schedule", &s) && read_field(line, "variant", &v) &&
            read_field(line, "threads", &t) && read_field(line, "blocks_per_cu", &b) &&
            read_field(line, "ms_per_sweep", &m)) {
            c->schedule = (uint32_t)s; c->variant = (uint32_t)v; c->threads = (uint32_t)t;
            c->bpc = (uint32_t)b; c->ms = m;
            found = true;
        }
    }
    fclose(f);
    return found;
}

bool cache_store(const char* path, const std::string& key, const Choice& c) {
    std::vector<std::string> keep;
    const std::string mine = "{\"key\": \"" + key + "\",";
    if (FILE* f = fopen(path, "r")) {
        char buf[4096];
        while (fgets(buf, sizeof buf, f)) {
            std::string line(buf);
            if (line.compare(0, mine.size(), mine) != 0 && line.size() > 1) keep.push_back(line);
        }
        fclose(f);
    }
    char b[256];
    snprintf(b, sizeof b, " \"schedule\": %u, \"variant\": %u, \"threads\": %u, \"blocks_per_cu\": %u, "
             "\"ms_per_sweep\": %.6f}\n", c.schedule, c.variant, c.threads, c.bpc, c.ms);
    keep.push_back(mine + b);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    for (auto& l : keep) fputs(l.c_str(), f);
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

static tfim_status apply_choice(tfim_plan* pl, const Choice& c) {
    if (c.variant >= (uint32_t)tfim::sweep_variants()) return fail(TFIM_EINVAL, "unknown sweep variant");
    pl->variant = (int)c.variant;
    tfim_status st = TFIM_OK;
    if (c.schedule == TFIM_SCHED_BATCHED) st = batch_setup(pl, c.threads, c.bpc);
    else if (c.schedule == TFIM_SCHED_CONCURRENT) st = concurrent_setup(pl);
    if (st != TFIM_OK) return st;
    pl->schedule = c.schedule;
    return TFIM_OK;
}

tfim_status tfim_autotune(tfim_plan* pl, uint32_t sweeps_per_trial, const char* cache_path,
                          uint64_t* sweeps_done) {
    tfim_status st = usable(pl);
    if (st != TFIM_OK) return st;
    if ((st = all_ready(pl)) != TFIM_OK) return st;
    if (sweeps_per_trial == 0) return fail(TFIM_EINVAL, "sweeps_per_trial must be >= 1");
    if (sweeps_done) *sweeps_done = 0;
    if (plain(pl)) return fail(TFIM_EUNSUPPORTED, "the plain form has one launch configuration");
    const std::string key = tune_key(pl);
    Choice c;
    if (cache_path && cache_lookup(cache_path, key, &c)) {
        if ((st = apply_choice(pl, c)) != TFIM_OK) return st;
        pl->tuned_ms = c.ms;
        return TFIM_OK;
    }
    // candidates
    std::vector<Choice> cand;
    bool stream_all = true;
    int maxcols = 0;
    for (int i = 0; i < (int)pl->shapes.size(); ++i) {
        const tfim::ShapeDev d = dev_of(pl, i);
        stream_all = stream_all && tfim::sweep_stream_ok(d);
        maxcols = std::max(maxcols, tfim::sweep_stream_cols(d));
    }
    for (uint32_t sched : {(uint32_t)TFIM_SCHED_PER_SHAPE, (uint32_t)TFIM_SCHED_CONCURRENT}) {
        if (sched == TFIM_SCHED_CONCURRENT && pl->shapes.size() < 2) continue;  // same as per-shape
        for (uint32_t v : {3u, 0u, 2u}) {
            Choice p;
            p.schedule = sched;
            p.variant = v;
            cand.push_back(p);
            if (!stream_all) break;  // the other variants fall back to the same kernel
        }
    }
    if (stream_all) {
        // workgroup sizes from the largest team upwards: one per distinct
        // packing of the shapes' teams
        std::vector<std::vector<int>> seen;
        for (uint32_t t = (uint32_t)maxcols; t <= kMaxBatchThreads; t += 64) {
            std::vector<int> pack;
            for (int i = 0; i < (int)pl->shapes.size(); ++i)
                pack.push_back((int)t / tfim::sweep_stream_cols(dev_of(pl, i)));
            if (std::find(seen.begin(), seen.end(), pack) != seen.end()) continue;
            seen.push_back(pack);
            Choice b;
            b.schedule = TFIM_SCHED_BATCHED;
            b.threads = t;
            cand.push_back(b);
        }
    }
    const bool timing = pl->timing;
    pl->timing = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    uint64_t done = 0;
    double best = -1.0;
    Choice pick;
    for (auto& cd : cand) {
        if (e != hipSuccess) break;
        st = apply_choice(pl, cd);
        if (st == TFIM_EUNSUPPORTED) continue;  // geometry does not fit: not a candidate
        if (st != TFIM_OK) break;
        if ((st = sweep_impl(pl, 1)) != TFIM_OK) break;
        done += 1;
        e = hipEventRecord(e0, pl->stream);
        if (e != hipSuccess) break;
        if ((st = sweep_impl(pl, sweeps_per_trial)) != TFIM_OK) break;
        done += sweeps_per_trial;
        e = hipEventRecord(e1, pl->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        cd.ms = ms / sweeps_per_trial;
        if (best < 0.0 || cd.ms < best) {
            best = cd.ms;
            pick = cd;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    pl->timing = timing;
    if (sweeps_done) *sweeps_done = done;
    if (e != hipSuccess) return check_hip(pl, e, "autotune");
    if (st != TFIM_OK && st != TFIM_EUNSUPPORTED) return st;
    if (best < 0.0) return fail(TFIM_EUNSUPPORTED, "no launch configuration fits these shapes");
    if ((st = apply_choice(pl, pick)) != TFIM_OK) return st;
    pl->tuned_ms = best;
    if (cache_path && !cache_store(cache_path, key, pick))
        return fail(TFIM_EINVAL, std::string("cannot write tuning cache ") + cache_path);
    return TFIM_OK;
}

tfim_status tfim_get_tuning(const tfim_plan* pl, tfim_tuning* out) {
    if (!pl || !out) return fail(TFIM_EINVAL, "null argument");
    out->schedule = pl->schedule;
    out->variant = (uint32_t)pl->variant;
    out->batch_threads = pl->batch_threads;
    out->batch_blocks_per_cu = pl->batch_bpc;
    out->batch_blocks = pl->batch_blocks;
    out->batch_items = (uint32_t)pl->items.size();
    out->ms_per_sweep = pl->tuned_ms;
    return TFIM_OK;
}

static uint64_t samples_of(const tfim_plan* pl, const ShapeHost& h) {
    return plain(pl) ? (uint64_t)h.s.n_words : 64ull * h.s.n_words;
}

static tfim_status measure_core(tfim_plan* pl, uint32_t shape, uint32_t mode, uint32_t cfg0,
                                uint32_t ncfg, uint32_t flags) {
    ShapeHost& h = pl->shapes[shape];
    if (!h.S_ready) return fail(TFIM_ESTATE, "spins of this shape are not initialised");
    const tfim::ShapeDev d = dev_of(pl, shape);
    const uint64_t ncfg_all = (uint64_t)h.s.n_k * samples_of(pl, h);
    if (mode > 1) return fail(TFIM_EINVAL, "unknown measurement mode");
    if (plain(pl)) {
        if (!tfim::plain_measure_ok(d)) return fail(TFIM_EUNSUPPORTED, "measurement needs 2..6 replicas");
        if (mode != 1) return fail(TFIM_EUNSUPPORTED, "the plain form measures in the plain per-sample mode (1)");
        if ((uint64_t)cfg0 + ncfg > ncfg_all) return fail(TFIM_EINVAL, "configuration range out of bounds");
        tfim_status st = injected(pl);
        if (st != TFIM_OK) return st;
        return check_hip(pl, tfim::plain_measure(d, (int)cfg0, (int)ncfg, pl->stream), "measure");
    }
    if (!tfim::measure_ok(d)) return fail(TFIM_EUNSUPPORTED, "measurement needs 2..6 replicas and L <= 32");
    if ((uint64_t)cfg0 + ncfg > ncfg_all) return fail(TFIM_EINVAL, "configuration range out of bounds");
    tfim_status st = injected(pl);
    if (st != TFIM_OK) return st;
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
    const size_t S = samples_of(pl, h), nk = h.s.n_k, R = h.s.n_replicas;
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
    const uint32_t mode = plain(pl) ? 1u : pl->measure_mode;
    if ((st = measure_core(pl, shape, mode, 0, (uint32_t)(nk * S), 0)) != TFIM_OK) return st;
    if (what == TFIM_MEASURE_BUCKETS) {
        const tfim::ShapeDev d = dev_of(pl, (int)shape);
        const hipError_t e = plain(pl) ? tfim::plain_buckets(d, pl->stream) : tfim::launch_buckets(d, pl->stream);
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

tfim_status tfim_triples_workspace(const tfim_plan* pl, uint32_t shape, uint32_t ncfg,
                                   size_t* bytes) {
    if (!pl || !bytes) return fail(TFIM_EINVAL, "null argument");
    if (shape >= pl->shapes.size()) return fail(TFIM_EINVAL, "shape index out of range");
    if (plain(pl)) return fail(TFIM_EUNSUPPORTED, "three-replica records need the multispin form");
    const tfim::ShapeDev d = dev_of(pl, shape);
    if (const char* why = tfim::triples_unsupported(d)) return fail(TFIM_EUNSUPPORTED, why);
    const tfim::TripleLayout lay = tfim::triple_layout(d, (int)ncfg);
    *bytes = lay.rec_bytes + lay.g_bytes;
    return TFIM_OK;
}

tfim_status tfim_measure_triples(tfim_plan* pl, uint32_t shape, uint32_t cfg0, uint32_t ncfg,
                                 uint32_t flags, void* ws, size_t ws_bytes, int64_t* out,
                                 size_t out_bytes) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (plain(pl)) return fail(TFIM_EUNSUPPORTED, "three-replica records need the multispin form");
    if (!h.S_ready) return fail(TFIM_ESTATE, "spins of this shape are not initialised");
    const tfim::ShapeDev d = dev_of(pl, shape);
    if (const char* why = tfim::triples_unsupported(d)) return fail(TFIM_EUNSUPPORTED, why);
    const uint64_t ncfg_all = (uint64_t)h.s.n_k * 64 * h.s.n_words;
    if ((uint64_t)cfg0 + ncfg > ncfg_all) return fail(TFIM_EINVAL, "configuration range out of bounds");
    const tfim::TripleLayout lay = tfim::triple_layout(d, (int)ncfg);
    if (!ws || ((uintptr_t)ws & 255)) return fail(TFIM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < lay.rec_bytes + lay.g_bytes) return fail(TFIM_EINVAL, "workspace too small");
    const uint32_t R = h.s.n_replicas;
    const size_t rec_used = (size_t)ncfg * (R * (R - 1) * (R - 2) / 6) * 2 * h.s.L * 8;
    if (out && out_bytes < rec_used) return fail(TFIM_EINVAL, "output buffer too small");
    if (ncfg == 0) return TFIM_OK;
    if ((st = injected(pl)) != TFIM_OK) return st;
    hipError_t e = hipSuccess;
    if (!(flags & TFIM_MEASURE_REUSE_LAYOUT)) e = tfim::launch_transpose(d, pl->stream);
    if (e == hipSuccess)
        e = tfim::launch_triples(d, (int)cfg0, (int)ncfg, (int64_t*)ws, (int8_t*)ws + lay.rec_bytes, pl->stream);
    if ((st = check_hip(pl, e, "triples")) != TFIM_OK) return st;
    if (!out) return TFIM_OK;
    return copy_back(pl, out, (const char*)ws, rec_used, "copy triple records");
}

tfim_status tfim_measure_triples_noalloc(tfim_plan* pl, uint32_t shape, uint32_t cfg0, uint32_t ncfg,
                                         uint32_t flags, int64_t* rec_dev, size_t rec_bytes) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (plain(pl)) return fail(TFIM_EUNSUPPORTED, "three-replica records need the multispin form");
    if (!h.S_ready) return fail(TFIM_ESTATE, "spins of this shape are not initialised");
    const tfim::ShapeDev d = dev_of(pl, shape);
    if (const char* why = tfim::triples_unsupported(d)) return fail(TFIM_EUNSUPPORTED, why);
    const uint64_t ncfg_all = (uint64_t)h.s.n_k * 64 * h.s.n_words;
    if ((uint64_t)cfg0 + ncfg > ncfg_all) return fail(TFIM_EINVAL, "configuration range out of bounds");
    const uint32_t R = h.s.n_replicas;
    const size_t rec_used = (size_t)ncfg * (R * (R - 1) * (R - 2) / 6) * 2 * h.s.L * 8;
    if (!rec_dev || ((uintptr_t)rec_dev & 7)) return fail(TFIM_EINVAL, "records need an 8-byte aligned device buffer");
    if (rec_bytes < rec_used) return fail(TFIM_EINVAL, "record buffer too small");
    void* scr = nullptr;
    size_t scr_bytes = 0;
    if ((st = check_hip(pl, tfim::static_scratch(pl->device, &scr, &scr_bytes), "static scratch")) != TFIM_OK)
        return st;
    const tfim::TripleLayout lay = tfim::triple_layout(d, (int)ncfg);
    if (lay.g_bytes > scr_bytes) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "%u configurations need %zu bytes of digit planes; the library's scratch holds %zu "
                 "(at most %zu configurations of this shape per call)",
                 ncfg, lay.g_bytes, scr_bytes, scr_bytes / (lay.g_bytes / std::max<uint32_t>(ncfg, 1)));
        return fail(TFIM_EINVAL, buf);
    }
    if (ncfg == 0) return TFIM_OK;
    if ((st = injected(pl)) != TFIM_OK) return st;
    hipError_t e = hipSuccess;
    if (!(flags & TFIM_MEASURE_REUSE_LAYOUT)) e = tfim::launch_transpose(d, pl->stream);
    if (e == hipSuccess) e = tfim::launch_triples(d, (int)cfg0, (int)ncfg, rec_dev, (int8_t*)scr, pl->stream);
    return check_hip(pl, e, "triples (library scratch)");
}

tfim_status tfim_measure_time(tfim_plan* pl, uint32_t shape, uint32_t cfg0, uint32_t ncfg,
                              uint32_t flags, void* ws, size_t ws_bytes, int64_t* out,
                              size_t out_bytes) {
    tfim_status st = shape_ok(pl, shape);
    if (st != TFIM_OK) return st;
    ShapeHost& h = pl->shapes[shape];
    if (plain(pl)) return fail(TFIM_EUNSUPPORTED, "two-time records need the multispin form");
    if (!h.S_ready) return fail(TFIM_ESTATE, "spins of this shape are not initialised");
    const tfim::ShapeDev d = dev_of(pl, shape);
    if (const char* why = tfim::timecorr_unsupported(d)) return fail(TFIM_EUNSUPPORTED, why);
    const uint64_t ncfg_all = (uint64_t)h.s.n_k * 64 * h.s.n_words;
    if ((uint64_t)cfg0 + ncfg > ncfg_all) return fail(TFIM_EINVAL, "configuration range out of bounds");
    const size_t need = tfim::timecorr_record_bytes(d, (int)ncfg);
    if (!ws || ((uintptr_t)ws & 255)) return fail(TFIM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(TFIM_EINVAL, "workspace too small");
    if (out && out_bytes < need) return fail(TFIM_EINVAL, "output buffer too small");
    if (ncfg == 0) return TFIM_OK;
    if ((st = injected(pl)) != TFIM_OK) return st;
    hipError_t e = hipSuccess;
    if (!(flags & TFIM_MEASURE_REUSE_LAYOUT)) e = tfim::launch_transpose(d, pl->stream);
    if (e == hipSuccess) e = tfim::launch_timecorr(d, (int)cfg0, (int)ncfg, (int64_t*)ws, pl->stream);
    if ((st = check_hip(pl, e, "two-time records")) != TFIM_OK) return st;
    if (!out) return TFIM_OK;
    return copy_back(pl, out, (const char*)ws, need, "copy two-time records");
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
    if (plain(pl)) return fail(TFIM_EUNSUPPORTED, "the debug dump needs the multispin form");
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
