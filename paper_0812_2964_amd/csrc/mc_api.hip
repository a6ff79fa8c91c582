// mc_api.hip -- host side of the C ABI declared in include/mc.h: argument
// validation, device state of a context, and the order of kernel launches for
// Algorithm steps 1-5 and eq. (new_weight) of arXiv 0812.2964.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <array>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "../../include/mc.h"
#include "mc_internal.h"

using namespace mcgpu;

namespace {

thread_local std::string g_err;

mc_status fail(mc_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

struct HostSize {
    mc_size cfg;
    SizeDev dev;
    SizePlan plan;     // how its sweeps are launched
    int64_t pending;   // configurations added to histograms since the last update
    int64_t last_M;    // sweeps of the last complete round, 0 after its joint
    int64_t part_ld;   // a round run in parts (mc_run_chains_part): its length,
    int64_t part_done; //   and the sweeps of it made so far (0: no round in parts)
    uint64_t g_host;   // host mirror of the device's global sweep index (Ctl.g)
    uint64_t r_host;   // host mirror of the joint round index (Ctl.r)
};

// The random words of sweep g and joint round r are keyed by the 32-bit
// counters g and r, so a size may make at most 2^32 sweeps and 2^32 joints
// in its lifetime: beyond that its random words would repeat.
constexpr uint64_t kCounterLimit = 0x100000000ull;

}  // namespace

struct mc_ctx {
    int device = 0;
    int n_cu = 256;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;  // created on first graph capture
    bool broken = false;
    std::vector<HostSize> sizes;
    // batched launch of all sizes (when every size keeps its lattices in LDS)
    bool batched = false;
    Tile *tiles_dev = nullptr;
    int32_t *counter_dev = nullptr;
    int n_tiles = 0;
    int batch_grid = 0;
    size_t batch_lds = 0;
    int live_graphs = 0;  // graphs hold the tile buffer and the state pointers
    double *thermo_buf = nullptr;  // mc_thermo: [thermo_cap] betas + [4 * thermo_cap] results
    int thermo_cap = 0;
    double *thermo_static = nullptr;  // mc_thermo_static: the device's static array (not owned)
};

struct mc_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    mc_ctx *ctx = nullptr;
    uint64_t sweeps = 0;  // sweeps and joint rounds one replay advances each size by
    uint64_t rounds = 0;
};

namespace {

mc_status hip_fail(mc_ctx *ctx, hipError_t e, const char *what) {
    if (ctx) ctx->broken = true;
    return fail(MC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_OR_FAIL(ctx, call)                                        \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);      \
    } while (0)

mc_status check_ctx(mc_ctx *ctx) {
    if (!ctx) return fail(MC_EINVAL, "null context");
    if (ctx->broken) return fail(MC_EHIP, "context is broken by an earlier HIP error");
    return MC_OK;
}

mc_status check_size(mc_ctx *ctx, int32_t i) {
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    if (i < 0 || i >= (int32_t)ctx->sizes.size()) return fail(MC_EINVAL, "size index %d out of range", i);
    return MC_OK;
}

void free_size(SizeDev &d) {
    if (d.lat) (void)hipFree(d.lat);
    if (d.lev) (void)hipFree(d.lev);
    if (d.lnW) (void)hipFree(d.lnW);
    if (d.tab) (void)hipFree(d.tab);
    if (d.tabc) (void)hipFree(d.tabc);
    if (d.ctl) (void)hipFree(d.ctl);
    if (d.scratch_cut) (void)hipFree(d.scratch_cut);
    if (d.join_order) (void)hipFree(d.join_order);
    if (d.hist64) (void)hipFree(d.hist64);
    if (d.n_bad) (void)hipFree(d.n_bad);
    if (d.ord) (void)hipFree(d.ord);
    d = SizeDev{};
}

// Default launch: for large lattices the quad-speculative streamed-row kernel
// (per-bin thresholds in LDS where they fit), 16 chains per workgroup when
// one workgroup per compute unit then holds every chain, else 32 (two
// consumer waves) so that they stay resident; for 8 <= L <= 64 the
// quad-speculative kernel; otherwise the producer/consumer pair kernel with
// the most chains per workgroup that fits, then the one-wave kernels.
SizePlan default_plan(const SizeDev &d, int n_cu) {
    if (d.L > 64) {
        const int cpb = (int64_t)d.P > 16ll * n_cu ? 32 : 16;
        SizePlan q = plan_sweeps(d, cpb, true);
        if (q.kind == kSweepBigQ || q.kind == kSweepBigQGlb) return q;
        q = plan_sweeps(d, 64, true);
        if (q.kind == kSweepBig || q.kind == kSweepBigGlb) return q;
    }
    if (d.L >= 8 && d.L <= 64) {
        // the quad-speculative kernel at 16 chains per workgroup: fastest at
        // every size measured (L = 16, 32, 64)
        SizePlan q = plan_sweeps(d, 16, true);
        if (q.kind == kSweepPCQ) return q;
    }
    for (int cpb = 64; cpb >= 8; cpb /= 2) {
        SizePlan q = plan_sweeps(d, cpb, true);
        if (q.kind == kSweepPC) return q;
    }
    SizePlan p = plan_sweeps(d, 64, false);
    for (int cpb = 32; p.kind == kSweepLds && cpb >= 16; cpb /= 2) {
        SizePlan q = plan_sweeps(d, cpb, false);
        if (q.kind == kSweepLdsTab) p = q;
    }
    return p;
}

// (Re)build the launch configuration after the plans changed.  Not allowed
// while capturing (it copies to the device and sets kernel attributes).
hipError_t rebuild_launch(mc_ctx *ctx) {
    for (auto &h : ctx->sizes) {
        hipError_t e = prepare_sweeps(h.dev, h.plan);
        if (e != hipSuccess) return e;
    }
    ctx->batched = ctx->sizes.size() > 1;
    for (auto &h : ctx->sizes) ctx->batched = ctx->batched && batchable(h.plan);
    if (!ctx->batched) return hipSuccess;
    // tiles, largest lattice first so the longest work starts first
    std::vector<int> order(ctx->sizes.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ctx->sizes[a].dev.N > ctx->sizes[b].dev.N; });
    std::vector<Tile> tiles;
    size_t lds = 0;
    for (int i : order) {
        const HostSize &h = ctx->sizes[i];
        for (int c0 = 0; c0 < h.dev.P; c0 += h.plan.cpb) tiles.push_back(Tile{i, c0});
        lds = std::max(lds, h.plan.lds_bytes);
    }
    if (ctx->tiles_dev) (void)hipFree(ctx->tiles_dev);
    ctx->tiles_dev = nullptr;
    hipError_t e = hipMalloc((void **)&ctx->tiles_dev, tiles.size() * sizeof(Tile));
    if (e != hipSuccess) return e;
    e = hipMemcpy(ctx->tiles_dev, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    if (!ctx->counter_dev) {
        e = hipMalloc((void **)&ctx->counter_dev, sizeof(int32_t));
        if (e != hipSuccess) return e;
    }
    ctx->n_tiles = (int)tiles.size();
    ctx->batch_lds = lds;
    const int per_cu = std::max(1, (int)((160 * 1024) / std::max<size_t>(lds, 1)));
    ctx->batch_grid = std::min(ctx->n_tiles, ctx->n_cu * std::min(per_cu, 8));
    return prepare_batched(lds);
}

// Sweeps of every size (Algorithm step 2), one launch when batched; sweep k of
// chain c goes to trace[s][c * ld + k].
hipError_t enqueue_sweeps(mc_ctx *ctx, hipStream_t st, int64_t M, int64_t ld, void *const *trace,
                          int32_t *const *hist) {
    const int n = (int)ctx->sizes.size();
    hipError_t e = hipSuccess;
    if (ctx->batched) {
        std::vector<SizeDev> devs(n);
        std::vector<SizePlan> plans(n);
        for (int i = 0; i < n; ++i) {
            devs[i] = ctx->sizes[i].dev;
            plans[i] = ctx->sizes[i].plan;
        }
        e = launch_sweeps_batched(devs.data(), plans.data(), n, ctx->tiles_dev, ctx->n_tiles, ctx->counter_dev,
                                  ctx->batch_grid, ctx->batch_lds, M, ld, trace, hist, st);
    } else {
        for (int i = 0; i < n && e == hipSuccess; ++i)
            e = launch_sweeps(ctx->sizes[i].dev, ctx->sizes[i].plan, M, ld, trace[i], hist[i], st);
    }
    for (int i = 0; i < n && e == hipSuccess; ++i) e = launch_advance(ctx->sizes[i].dev, M, st);
    return e;
}

// Copies of the chain state of every size and buffers for their traces, so
// that probe launches leave the chains untouched.
struct ScratchSizes {
    std::vector<SizeDev> dev;
    std::vector<void *> trace;
    std::vector<int32_t *> hist;

    hipError_t alloc(const mc_ctx *ctx, int64_t M) {
        for (const auto &h : ctx->sizes) {
            SizeDev d = h.dev;
            d.lat = nullptr;
            d.lev = nullptr;
            d.ctl = nullptr;
            void *tr = nullptr;
            int32_t *hs = nullptr;
            hipError_t e = hipMalloc((void **)&d.lat, (size_t)d.L * d.W * d.P * 4);
            if (e == hipSuccess) e = hipMalloc((void **)&d.lev, (size_t)d.P * 4);
            if (e == hipSuccess) e = hipMalloc((void **)&d.ctl, sizeof(Ctl));
            if (e == hipSuccess) e = hipMalloc(&tr, (size_t)d.P * M * d.trace_bytes);
            if (e == hipSuccess) e = hipMalloc((void **)&hs, (size_t)d.n_bins * 4);
            dev.push_back(d);
            trace.push_back(tr);
            hist.push_back(hs);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t refresh(const mc_ctx *ctx, hipStream_t st) {
        for (size_t i = 0; i < dev.size(); ++i) {
            const SizeDev &d = ctx->sizes[i].dev;
            hipError_t e = hipMemcpyAsync(dev[i].lat, d.lat, (size_t)d.L * d.W * d.P * 4, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(dev[i].lev, d.lev, (size_t)d.P * 4, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(dev[i].ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    ~ScratchSizes() {
        for (size_t i = 0; i < dev.size(); ++i) {
            if (dev[i].lat) (void)hipFree(dev[i].lat);
            if (dev[i].lev) (void)hipFree(dev[i].lev);
            if (dev[i].ctl) (void)hipFree(dev[i].ctl);
            if (trace[i]) (void)hipFree(trace[i]);
            if (hist[i]) (void)hipFree(hist[i]);
        }
    }
};

// Sizes that run batched share one persistent launch, whose time depends on
// how many chains run at once as well as on each size's own speed.  Time the
// batched launch for 16, 32 and 64 chains per workgroup everywhere and, with
// at most six sizes, for every mix of each size's own best plan and its
// widest one (most chains per workgroup); keep the fastest.
hipError_t autotune_batched(mc_ctx *ctx, int64_t probe_sweeps, hipEvent_t e0, hipEvent_t e1) {
    const int n = (int)ctx->sizes.size();
    std::vector<SizePlan> own(n), wide(n), best(n);
    for (int i = 0; i < n; ++i) {
        own[i] = best[i] = ctx->sizes[i].plan;
        wide[i] = own[i];
        for (int cpb : {64, 32, 16}) {
            const SizePlan q = plan_sweeps(ctx->sizes[i].dev, cpb, true);
            if (batchable(q)) {
                wide[i] = q;
                break;
            }
        }
    }
    std::vector<std::vector<SizePlan>> cands;
    for (int cpb : {16, 32, 64}) {
        std::vector<SizePlan> c(n);
        for (int i = 0; i < n; ++i) c[i] = plan_sweeps(ctx->sizes[i].dev, cpb, true);
        cands.push_back(c);
    }
    if (n <= 6)
        for (int mask = 0; mask < (1 << n); ++mask) {
            std::vector<SizePlan> c(n);
            for (int i = 0; i < n; ++i) c[i] = ((mask >> i) & 1) ? wide[i] : own[i];
            cands.push_back(c);
        }
    else
        cands.push_back(own);
    ScratchSizes scr;
    hipError_t e = scr.alloc(ctx, probe_sweeps);
    float best_ms = 1e30f;
    for (size_t k = 0; k < cands.size() && e == hipSuccess; ++k) {
        bool ok = true;
        for (int i = 0; i < n; ++i) {
            ctx->sizes[i].plan = cands[k][i];
            ok = ok && batchable(ctx->sizes[i].plan);
        }
        if (!ok) continue;
        e = rebuild_launch(ctx);
        if (e != hipSuccess || !ctx->batched) break;
        std::vector<SizePlan> plans(n);
        for (int i = 0; i < n; ++i) plans[i] = ctx->sizes[i].plan;
        float t_min = 1e30f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            e = scr.refresh(ctx, ctx->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
            if (e == hipSuccess)
                e = launch_sweeps_batched(scr.dev.data(), plans.data(), n, ctx->tiles_dev, ctx->n_tiles,
                                          ctx->counter_dev, ctx->batch_grid, ctx->batch_lds, probe_sweeps,
                                          probe_sweeps, scr.trace.data(), scr.hist.data(), ctx->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            t_min = std::min(t_min, ms);
        }
        if (e == hipSuccess && t_min < best_ms) {
            best_ms = t_min;
            best = plans;
        }
    }
    for (int i = 0; i < n; ++i) ctx->sizes[i].plan = best[i];
    return e;
}

}  // namespace

// CRC-32 of the IEEE 802.3 / zlib definition (reflected polynomial
// 0xEDB88320, initial and final complement), table driven.
static uint32_t crc32_of(const unsigned char *p, size_t n) {
    // built once; the initialisation of a function-local static is thread-safe
    static const std::array<uint32_t, 256> table = [] {
        std::array<uint32_t, 256> t{};
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int k = 0; k < 8; ++k) c = (c & 1u) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
            t[i] = c;
        }
        return t;
    }();
    uint32_t c = 0xFFFFFFFFu;
    for (size_t i = 0; i < n; ++i) c = table[(c ^ p[i]) & 0xFFu] ^ (c >> 8);
    return c ^ 0xFFFFFFFFu;
}

// State blob: a 24-byte header {"MCS1", version, crc, n_sizes, total bytes}
// and per size {L, n_chains, seed, bin_shift, W, n_bins, chain_offset, pending, last_M,
// the Ctl counters field by field, lattice words, levels, ln w}, all
// little-endian; the CRC-32 covers the whole blob with its crc field zero.
constexpr uint32_t kStateVersion = 1;
constexpr size_t kStateHeader = 24;

static size_t state_size_of(const SizeDev &d) {
    return 7 * 4 + 2 * 8 + (4 * 4 + 2 * 8 + 2 * 4) + (size_t)d.L * d.W * d.P * 4 + (size_t)d.P * 4 +
           (size_t)d.n_bins * 8;
}

// Check the chain state of one size in a blob before it reaches the kernels,
// which index the threshold tables and histograms by level: every site bit
// beyond L in a row's last word is zero (as the kernels keep it), and each
// chain's level is half its number of broken bonds (Sec. 4.1, J = 1: level
// (E + 2N)/4).  lat: [L*W][P] words, chain-interleaved; lev: [P].  Returns the
// first chain that fails, or -1.
static int64_t bad_chain(const SizeDev &d, const unsigned char *lat, const unsigned char *lev, int32_t *why) {
    const int L = d.L, W = d.W, P = d.P;
    const int nb = L - 32 * (W - 1);  // site bits in a row's last word
    const uint32_t last_mask = nb == 32 ? 0xFFFFFFFFu : (1u << nb) - 1u;
    auto word = [&](int row, int w, int c) {
        uint32_t v;
        std::memcpy(&v, lat + ((size_t)(row * W + w) * P + c) * 4, 4);
        return v;
    };
    std::vector<uint32_t> cur((size_t)W), first((size_t)W);
    for (int c = 0; c < P; ++c) {
        int64_t broken = 0;
        for (int w = 0; w < W; ++w) first[w] = word(0, w, c);
        for (int y = 0; y < L; ++y) {
            for (int w = 0; w < W; ++w) cur[w] = word(y, w, c);
            if (cur[W - 1] & ~last_mask) {
                *why = 1;
                return c;
            }
            for (int w = 0; w < W; ++w) {
                // right neighbours of the word's sites: the next site bit,
                // wrapping from site L-1 to site 0
                uint32_t right, mask = 0xFFFFFFFFu;
                if (w < W - 1) {
                    right = (cur[w] >> 1) | (cur[w + 1] << 31);
                } else {
                    right = (cur[w] >> 1) | ((cur[0] & 1u) << (nb - 1));
                    mask = last_mask;
                }
                const uint32_t down = y + 1 < L ? word(y + 1, w, c) : first[w];
                broken += __builtin_popcount((cur[w] ^ right) & mask) + __builtin_popcount((cur[w] ^ down) & mask);
            }
        }
        int32_t m;
        std::memcpy(&m, lev + (size_t)c * 4, 4);
        if ((int64_t)m * 2 != broken) {
            *why = 2;
            return c;
        }
    }
    return -1;
}

void mcgpu::set_last_error(const char *msg) { g_err = msg; }

extern "C" {

const char *mc_last_error(void) { return g_err.c_str(); }

mc_status mc_create(const mc_size *sizes, int32_t n_sizes, void *hip_stream, mc_ctx **out) {
    if (!out) return fail(MC_EINVAL, "null output pointer");
    *out = nullptr;
    if (!sizes || n_sizes < 1 || n_sizes > 16) return fail(MC_EINVAL, "n_sizes must be 1..16");
    for (int i = 0; i < n_sizes; ++i) {
        const mc_size &c = sizes[i];
        if (c.L < 4 || c.L > 256 || (c.L & 1)) return fail(MC_EINVAL, "size %d: L=%d must be even, 4..256", i, c.L);
        if (c.n_chains < 1 || c.n_chains > (1 << 20))
            return fail(MC_EINVAL, "size %d: n_chains=%d must be 1..2^20", i, c.n_chains);
        if (c.bin_shift < 0 || c.bin_shift > 1) return fail(MC_EINVAL, "size %d: bin_shift must be 0 or 1", i);
        if ((uint64_t)c.chain_offset + (uint64_t)c.n_chains > 0x100000000ull)
            return fail(MC_EINVAL, "size %d: chain_offset + n_chains must not exceed 2^32", i);
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(MC_ENODEV, "no HIP device available");
    }
    mc_ctx *ctx = new mc_ctx();
    ctx->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return fail(MC_ENODEV, "hipGetDevice failed");
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) == hipSuccess && ncu > 0)
        ctx->n_cu = ncu;
    // the device address of mc_thermo_static's array, looked up with this device current
    if (thermo_scratch_address(ctx->device, &ctx->thermo_static) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return fail(MC_EHIP, "device address of the static reweighting array");
    }
    ctx->sizes.resize(n_sizes);
    mc_status st = MC_OK;
    for (int i = 0; i < n_sizes && st == MC_OK; ++i) {
        HostSize &h = ctx->sizes[i];
        h.cfg = sizes[i];
        h.pending = 0;
        h.last_M = 0;
        h.part_ld = 0;
        h.part_done = 0;
        h.g_host = 0;
        h.r_host = 0;
        SizeDev &d = h.dev;
        d = SizeDev{};
        d.L = h.cfg.L;
        d.N = d.L * d.L;
        d.W = (d.L + 31) / 32;
        d.P = h.cfg.n_chains;
        d.bin_shift = h.cfg.bin_shift;
        d.n_bins = (d.N >> d.bin_shift) + 1;
        d.seed = h.cfg.seed;
        d.c_off = h.cfg.chain_offset;
        d.trace_bytes = (d.L <= 254) ? 2 : 4;
        d.tab_r = d.bin_shift == 0 ? 2 : 1;
        const size_t lat_b = (size_t)d.L * d.W * d.P * 4;
        if (hipMalloc((void **)&d.lat, lat_b) != hipSuccess || hipMalloc((void **)&d.lev, (size_t)d.P * 4) != hipSuccess ||
            hipMalloc((void **)&d.lnW, (size_t)d.n_bins * 8) != hipSuccess ||
            hipMalloc((void **)&d.tab, (size_t)(d.N + 1) * 8 * 4) != hipSuccess ||
            hipMalloc((void **)&d.tabc, (size_t)d.n_bins * (2 * d.tab_r + 1) * 4) != hipSuccess ||
            hipMalloc((void **)&d.ctl, sizeof(Ctl)) != hipSuccess ||
            hipMalloc((void **)&d.scratch_cut, (size_t)d.P * 4) != hipSuccess ||
            hipMalloc((void **)&d.join_order, (size_t)d.P * 4) != hipSuccess ||
            hipMalloc((void **)&d.hist64, (size_t)d.n_bins * 8) != hipSuccess ||
            hipMalloc((void **)&d.n_bad, sizeof(int64_t)) != hipSuccess ||
            hipMalloc((void **)&d.ord, order_scratch_ints(d.N, d.P) * 4) != hipSuccess) {
            (void)hipGetLastError();
            st = fail(MC_ENOMEM, "device allocation failed for size %d", i);
            break;
        }
        Ctl c0{};
        c0.sigma = -1;
        std::vector<double> zeros((size_t)d.n_bins, 0.0);
        hipError_t e = hipMemcpyAsync(d.ctl, &c0, sizeof c0, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d.lnW, zeros.data(), zeros.size() * 8, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipMemsetAsync(d.hist64, 0, (size_t)d.n_bins * 8, ctx->stream);
        if (e == hipSuccess) e = launch_init(d, ctx->stream);
        if (e == hipSuccess) e = launch_tabulate(d, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = hip_fail(nullptr, e, "context initialisation");
        h.plan = default_plan(d, ctx->n_cu);
    }
    if (st == MC_OK) {
        hipError_t e = rebuild_launch(ctx);
        if (e != hipSuccess) st = hip_fail(nullptr, e, "launch configuration");
    }
    if (st != MC_OK) {
        for (auto &h : ctx->sizes) free_size(h.dev);
        if (ctx->tiles_dev) (void)hipFree(ctx->tiles_dev);
        if (ctx->counter_dev) (void)hipFree(ctx->counter_dev);
        delete ctx;
        return st;
    }
    *out = ctx;
    return MC_OK;
}

mc_status mc_destroy(mc_ctx *ctx) {
    if (!ctx) return MC_OK;
    if (ctx->live_graphs > 0) return fail(MC_ESTATE, "destroy the context's graphs first");
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &h : ctx->sizes) free_size(h.dev);
    if (ctx->tiles_dev) (void)hipFree(ctx->tiles_dev);
    if (ctx->counter_dev) (void)hipFree(ctx->counter_dev);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->thermo_buf) (void)hipFree(ctx->thermo_buf);
    delete ctx;
    return MC_OK;
}

int32_t mc_n_bins(const mc_ctx *ctx, int32_t i) {
    if (!ctx || i < 0 || i >= (int32_t)ctx->sizes.size()) return -1;
    return ctx->sizes[i].dev.n_bins;
}

int32_t mc_trace_elem_bytes(const mc_ctx *ctx, int32_t i) {
    if (!ctx || i < 0 || i >= (int32_t)ctx->sizes.size()) return -1;
    return ctx->sizes[i].dev.trace_bytes;
}

int32_t mc_lattice_words(const mc_ctx *ctx, int32_t i) {
    if (!ctx || i < 0 || i >= (int32_t)ctx->sizes.size()) return -1;
    return ctx->sizes[i].dev.L * ctx->sizes[i].dev.W;
}

mc_status mc_init_weights(mc_ctx *ctx, int32_t i, const double *lnW_host, int32_t n_bins) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    SizeDev &d = ctx->sizes[i].dev;
    if (n_bins != d.n_bins) return fail(MC_EINVAL, "n_bins=%d, size %d has %d bins", n_bins, i, d.n_bins);
    std::vector<double> w((size_t)d.n_bins, 0.0);
    if (lnW_host) {
        for (int b = 0; b < d.n_bins; ++b) {
            if (!std::isfinite(lnW_host[b])) return fail(MC_EINVAL, "ln w[%d] is not finite", b);
            w[b] = lnW_host[b];
        }
    }
    HIP_OR_FAIL(ctx, hipMemcpyAsync(d.lnW, w.data(), w.size() * 8, hipMemcpyHostToDevice, ctx->stream));
    HIP_OR_FAIL(ctx, launch_tabulate(d, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

mc_status mc_run_chains(mc_ctx *ctx, int64_t n_sweeps, void *const *trace_dev, int32_t *const *hist_dev) {
    return mc_run_chains_part(ctx, n_sweeps, 0, n_sweeps, trace_dev, hist_dev);
}

mc_status mc_run_chains_part(mc_ctx *ctx, int64_t n_sweeps, int64_t col, int64_t row_len, void *const *trace_dev,
                             int32_t *const *hist_dev) {
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    if (n_sweeps < 1 || n_sweeps > 0x7FFFFFFF) return fail(MC_EINVAL, "n_sweeps=%lld must be 1..2^31-1", (long long)n_sweeps);
    if (row_len < 1 || row_len > 0x7FFFFFFF) return fail(MC_EINVAL, "row_len=%lld must be 1..2^31-1", (long long)row_len);
    if (col < 0 || col + n_sweeps > row_len)
        return fail(MC_EINVAL, "columns %lld..%lld do not fit rows of %lld", (long long)col,
                    (long long)(col + n_sweeps - 1), (long long)row_len);
    if (!trace_dev || !hist_dev) return fail(MC_EINVAL, "null trace/hist pointer array");
    const int n = (int)ctx->sizes.size();
    for (int i = 0; i < n; ++i) {
        HostSize &h = ctx->sizes[i];
        if (!trace_dev[i] || !hist_dev[i]) return fail(MC_EINVAL, "size %d: null trace or hist", i);
        if (col > 0 && (h.part_ld != row_len || h.part_done != col))
            return fail(MC_ESTATE, "size %d: columns from %lld continue no round in parts (%lld of %lld made)", i,
                        (long long)col, (long long)h.part_done, (long long)h.part_ld);
        const int64_t add = (int64_t)h.dev.P * n_sweeps;
        if (h.pending + add > 0x7FFFFFFFll)
            return fail(MC_EOVERFLOW, "size %d: %lld configurations would exceed the int32 histogram", i,
                        (long long)(h.pending + add));
        if (h.g_host + (uint64_t)n_sweeps > kCounterLimit)
            return fail(MC_EOVERFLOW, "size %d: sweeps %llu..%llu would pass the 2^32 sweep counter of the random "
                        "words", i, (unsigned long long)h.g_host, (unsigned long long)(h.g_host + n_sweeps - 1));
    }
    std::vector<void *> tr((size_t)n);
    for (int i = 0; i < n; ++i)
        tr[i] = (char *)trace_dev[i] + (size_t)col * (size_t)ctx->sizes[i].dev.trace_bytes;
    HIP_OR_FAIL(ctx, enqueue_sweeps(ctx, ctx->stream, n_sweeps, row_len, tr.data(), hist_dev));
    for (int i = 0; i < n; ++i) {
        HostSize &h = ctx->sizes[i];
        h.pending += (int64_t)h.dev.P * n_sweeps;
        h.g_host += (uint64_t)n_sweeps;
        if (col + n_sweeps == row_len) {
            h.last_M = row_len;  // the round is complete: it can be joined
            h.part_ld = h.part_done = 0;
        } else {
            h.last_M = 0;
            h.part_ld = row_len;
            h.part_done = col + n_sweeps;
        }
    }
    return MC_OK;
}

mc_status mc_join(mc_ctx *ctx, int32_t i, const void *trace_dev, int64_t n_sweeps, int32_t *cut_dev, int32_t *hist_dev,
                  int32_t mode) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    HostSize &h = ctx->sizes[i];
    if (!trace_dev || !cut_dev || !hist_dev) return fail(MC_EINVAL, "null trace, cut or hist");
    if (mode < 0 || mode > 2) return fail(MC_EINVAL, "mode must be 0, 1 or 2");
    if (h.last_M == 0) return fail(MC_ESTATE, "size %d: no complete round of mc_run_chains to join", i);
    if (h.r_host + 1 > kCounterLimit)
        return fail(MC_EOVERFLOW, "size %d: the 2^32 joint rounds of the random words are used up", i);
    if (n_sweeps != h.last_M)
        return fail(MC_EINVAL, "n_sweeps=%lld differs from the last run (%lld)", (long long)n_sweeps, (long long)h.last_M);
    const int32_t *order = nullptr;
    if (mode == 2) {
        HIP_OR_FAIL(ctx, launch_energy_order(h.dev, trace_dev, n_sweeps, ctx->stream));
        order = h.dev.join_order;
    }
    HIP_OR_FAIL(ctx, launch_join(h.dev, trace_dev, n_sweeps, cut_dev, hist_dev, mode == 2 ? 0 : mode, order,
                                 ctx->stream));
    h.last_M = 0;
    h.r_host += 1;
    return MC_OK;
}

mc_status mc_update_weights(mc_ctx *ctx, int32_t i, int32_t *hist_dev, double *lnW_out_host, int32_t *is_flat,
                            int64_t *retained) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    HostSize &h = ctx->sizes[i];
    if (!hist_dev) return fail(MC_EINVAL, "null hist");
    HIP_OR_FAIL(ctx, launch_update(h.dev, hist_dev, ctx->stream));
    h.pending = 0;
    h.part_ld = h.part_done = 0;
    if (lnW_out_host || is_flat || retained) {
        Ctl c{};
        HIP_OR_FAIL(ctx, hipMemcpyAsync(&c, h.dev.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
        if (lnW_out_host)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(lnW_out_host, h.dev.lnW, (size_t)h.dev.n_bins * 8, hipMemcpyDeviceToHost,
                                            ctx->stream));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
        if (is_flat) *is_flat = c.flat;
        if (retained) *retained = c.retained_last;
    }
    return MC_OK;
}

mc_status mc_iterate_topup(mc_ctx *ctx, int64_t m_total, int64_t m_max, int32_t max_rounds, void *trace_dev,
                           int32_t *hist_dev, int32_t *cut_dev, int32_t mode, int32_t *rounds_out, int64_t *sweeps_out,
                           int64_t *retained_out, int32_t *is_flat) {
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    if (ctx->sizes.size() != 1) return fail(MC_EINVAL, "mc_iterate_topup needs a context of one size");
    HostSize &h = ctx->sizes[0];
    const SizeDev &d = h.dev;
    if (!trace_dev || !hist_dev || !cut_dev) return fail(MC_EINVAL, "null trace, hist or cut");
    if (m_total < 1) return fail(MC_EINVAL, "m_total must be positive");
    if (m_max < 1 || m_max > 0x7FFFFFFF) return fail(MC_EINVAL, "m_max must be 1..2^31-1");
    if (max_rounds < 1 || max_rounds > 1000000) return fail(MC_EINVAL, "max_rounds must be 1..10^6");
    if (mode < 0 || mode > 2) return fail(MC_EINVAL, "mode must be 0, 1 or 2");
    if ((int64_t)d.P * m_max > 0x7FFFFFFFll)
        return fail(MC_EOVERFLOW, "%d chains x %lld sweeps exceed the int32 histogram of one round", d.P,
                    (long long)m_max);
    if (h.pending != 0 || h.last_M != 0 || h.part_ld != 0)
        return fail(MC_ESTATE, "mc_iterate_topup must start after a weight update");
    Ctl c{};
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&c, d.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t kept0 = c.retained;
    int64_t kept = 0, swept = 0;
    int rounds = 0;
    for (;;) {
        // Algorithm step 6: the next round covers the shortfall at the rate seen so far
        int64_t m = m_max;
        if (rounds > 0 && kept > 0) {
            const int64_t need = m_total - kept;
            const __int128 q = ((__int128)need * swept + kept - 1) / kept;
            m = q > m_max ? m_max : std::max<int64_t>(1, (int64_t)q);
        }
        void *tr[1] = {trace_dev};
        int32_t *hs[1] = {hist_dev};
        st = mc_run_chains(ctx, m, tr, hs);
        if (st != MC_OK) return st;
        st = mc_join(ctx, 0, trace_dev, m, cut_dev, hist_dev, mode);
        if (st != MC_OK) return st;
        HIP_OR_FAIL(ctx, launch_fold_hist(d, hist_dev, ctx->stream));
        h.pending = 0;
        HIP_OR_FAIL(ctx, hipMemcpyAsync(&c, d.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
        kept = c.retained - kept0;
        swept += m;
        rounds += 1;
        if (kept >= m_total || rounds >= max_rounds) break;
    }
    HIP_OR_FAIL(ctx, launch_update64(d, ctx->stream));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&c, d.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    if (rounds_out) *rounds_out = rounds;
    if (sweeps_out) *sweeps_out = swept;
    if (retained_out) *retained_out = c.retained_last;
    if (is_flat) *is_flat = c.flat;
    return MC_OK;
}

mc_status mc_get_levels(mc_ctx *ctx, int32_t i, int32_t *levels_host) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    if (!levels_host) return fail(MC_EINVAL, "null output");
    const SizeDev &d = ctx->sizes[i].dev;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(levels_host, d.lev, (size_t)d.P * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

mc_status mc_get_lattice(mc_ctx *ctx, int32_t i, int32_t chain, uint32_t *words_host, int32_t n_words) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    const SizeDev &d = ctx->sizes[i].dev;
    if (!words_host || n_words != d.L * d.W) return fail(MC_EINVAL, "need %d words", d.L * d.W);
    if (chain < 0 || chain >= d.P) return fail(MC_EINVAL, "chain %d out of range", chain);
    // word w of the chain sits at lat[w*P + chain]: a strided 2D copy
    HIP_OR_FAIL(ctx, hipMemcpy2DAsync(words_host, 4, d.lat + chain, (size_t)d.P * 4, 4, (size_t)n_words,
                                      hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

mc_status mc_get_counters(mc_ctx *ctx, int32_t i, int32_t *seam, uint32_t *round, uint32_t *sweep) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    Ctl c{};
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&c, ctx->sizes[i].dev.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    if (seam) *seam = c.sigma;
    if (round) *round = c.r;
    if (sweep) *sweep = c.g;
    return MC_OK;
}

mc_status mc_set_seam(mc_ctx *ctx, int32_t i, int32_t seam) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    HostSize &h = ctx->sizes[i];
    if (seam < -1 || seam > h.dev.N) return fail(MC_EINVAL, "seam=%d must be -1..%d", seam, h.dev.N);
    Ctl c{};
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&c, h.dev.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    c.sigma = seam;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(h.dev.ctl, &c, sizeof c, hipMemcpyHostToDevice, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

mc_status mc_sync(mc_ctx *ctx) {
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

mc_status mc_get_weights(mc_ctx *ctx, int32_t i, double *lnW_host, int32_t n_bins) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    const SizeDev &d = ctx->sizes[i].dev;
    if (!lnW_host || n_bins != d.n_bins) return fail(MC_EINVAL, "need %d bins", d.n_bins);
    HIP_OR_FAIL(ctx, hipMemcpyAsync(lnW_host, d.lnW, (size_t)d.n_bins * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

mc_status mc_get_state(mc_ctx *ctx, void *buf, size_t *len) {
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    if (!len) return fail(MC_EINVAL, "null length pointer");
    for (size_t i = 0; i < ctx->sizes.size(); ++i)
        if (ctx->sizes[i].part_ld != 0)
            return fail(MC_ESTATE, "size %zu: a round is partly run (mc_run_chains_part); finish it first", i);
    size_t need = kStateHeader;
    for (const auto &h : ctx->sizes) need += state_size_of(h.dev);
    if (!buf) {
        *len = need;
        return MC_OK;
    }
    if (*len < need) return fail(MC_EINVAL, "the state needs %zu bytes, the buffer has %zu", need, *len);
    unsigned char *o = (unsigned char *)buf;
    size_t at = 0;
    auto put = [&](const void *v, size_t n) {
        std::memcpy(o + at, v, n);
        at += n;
    };
    auto put32 = [&](uint32_t v) { put(&v, 4); };
    auto put64 = [&](uint64_t v) { put(&v, 8); };
    put("MCS1", 4);
    put32(kStateVersion);
    put32(0u);  // crc, filled in below
    put32((uint32_t)ctx->sizes.size());
    put64((uint64_t)need);
    for (const auto &h : ctx->sizes) {
        const SizeDev &d = h.dev;
        Ctl c{};
        HIP_OR_FAIL(ctx, hipMemcpyAsync(&c, d.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
        const size_t lat_b = (size_t)d.L * d.W * d.P * 4;
        const size_t base = at + 7 * 4 + 2 * 8 + (4 * 4 + 2 * 8 + 2 * 4);
        HIP_OR_FAIL(ctx, hipMemcpyAsync(o + base, d.lat, lat_b, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(o + base + lat_b, d.lev, (size_t)d.P * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(o + base + lat_b + (size_t)d.P * 4, d.lnW, (size_t)d.n_bins * 8,
                                        hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
        put32((uint32_t)d.L);
        put32((uint32_t)d.P);
        put32(d.seed);
        put32((uint32_t)d.bin_shift);
        put32((uint32_t)d.W);
        put32((uint32_t)d.n_bins);
        put32(d.c_off);
        put64((uint64_t)h.pending);
        put64((uint64_t)h.last_M);
        put32(c.g);
        put32(c.r);
        put32((uint32_t)c.sigma);
        put32((uint32_t)c.flat);
        put64((uint64_t)c.retained);
        put64((uint64_t)c.retained_last);
        put32((uint32_t)c.iter);
        put32((uint32_t)c.flat_iter);
        at = base + lat_b + (size_t)d.P * 4 + (size_t)d.n_bins * 8;
    }
    const uint32_t crc = crc32_of(o, need);
    std::memcpy(o + 8, &crc, 4);
    *len = need;
    return MC_OK;
}

mc_status mc_set_state(mc_ctx *ctx, const void *buf, size_t len) {
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    if (!buf) return fail(MC_EINVAL, "null state");
    const unsigned char *b = (const unsigned char *)buf;
    if (len < kStateHeader || std::memcmp(b, "MCS1", 4) != 0) return fail(MC_ECORRUPT, "not a state blob");
    uint32_t version, crc, n_sizes;
    uint64_t total;
    std::memcpy(&version, b + 4, 4);
    std::memcpy(&crc, b + 8, 4);
    std::memcpy(&n_sizes, b + 12, 4);
    std::memcpy(&total, b + 16, 8);
    if (version != kStateVersion) return fail(MC_ECORRUPT, "state version %u, expected %u", version, kStateVersion);
    if (total != len) return fail(MC_ECORRUPT, "state length %zu, the blob says %llu", len, (unsigned long long)total);
    std::vector<unsigned char> copy(b, b + len);
    std::memset(copy.data() + 8, 0, 4);
    if (crc32_of(copy.data(), len) != crc) return fail(MC_ECORRUPT, "state checksum mismatch");
    if (n_sizes != ctx->sizes.size())
        return fail(MC_EINVAL, "the state has %u sizes, the context %zu", n_sizes, ctx->sizes.size());
    // validate every size before touching any
    size_t at = kStateHeader;
    auto get32 = [&](size_t pos) {
        uint32_t v;
        std::memcpy(&v, b + pos, 4);
        return v;
    };
    auto get64 = [&](size_t pos) {
        uint64_t v;
        std::memcpy(&v, b + pos, 8);
        return v;
    };
    for (const auto &h : ctx->sizes) {
        const SizeDev &d = h.dev;
        if (at + 28 > len) return fail(MC_ECORRUPT, "state too short");
        if ((int)get32(at) != d.L || (int)get32(at + 4) != d.P || get32(at + 8) != d.seed ||
            (int)get32(at + 12) != d.bin_shift || (int)get32(at + 16) != d.W || (int)get32(at + 20) != d.n_bins ||
            get32(at + 24) != d.c_off)
            return fail(MC_EINVAL, "the state's sizes differ from the context's");
        if (at + state_size_of(d) > len) return fail(MC_ECORRUPT, "state too short");
        const int64_t pending = (int64_t)get64(at + 28), last_M = (int64_t)get64(at + 36);
        const int32_t sigma = (int32_t)get32(at + 52), flat = (int32_t)get32(at + 56);
        const int64_t retained = (int64_t)get64(at + 60), retained_last = (int64_t)get64(at + 68);
        const int32_t iter = (int32_t)get32(at + 76), flat_iter = (int32_t)get32(at + 80);
        if (pending < 0 || pending > 0x7FFFFFFFll || last_M < 0 || last_M > 0x7FFFFFFFll || sigma < -1 ||
            sigma > d.N || (flat != 0 && flat != 1) || retained < 0 || retained_last < 0 || iter < 0 ||
            flat_iter < 0 || flat_iter > iter)
            return fail(MC_ECORRUPT, "the state's counters are out of range");
        const size_t lat_at = at + 84, lev_at = lat_at + (size_t)d.L * d.W * d.P * 4;
        int32_t why = 0;
        const int64_t c = bad_chain(d, b + lat_at, b + lev_at, &why);
        if (c >= 0)
            return fail(MC_ECORRUPT, why == 1 ? "chain %lld: lattice bits set beyond L" :
                                                "chain %lld: level does not match its lattice", (long long)c);
        const size_t lnw = at + state_size_of(d) - (size_t)d.n_bins * 8;
        for (int k = 0; k < d.n_bins; ++k) {
            double v;
            std::memcpy(&v, b + lnw + (size_t)k * 8, 8);
            if (!std::isfinite(v)) return fail(MC_ECORRUPT, "ln w[%d] in the state is not finite", k);
        }
        at += state_size_of(d);
    }
    if (at != len) return fail(MC_ECORRUPT, "state length does not match its sizes");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    at = kStateHeader;
    for (auto &h : ctx->sizes) {
        SizeDev &d = h.dev;
        Ctl c{};
        c.g = get32(at + 44);
        c.r = get32(at + 48);
        c.sigma = (int32_t)get32(at + 52);
        c.flat = (int32_t)get32(at + 56);
        c.retained = (int64_t)get64(at + 60);
        c.retained_last = (int64_t)get64(at + 68);
        c.iter = (int32_t)get32(at + 76);
        c.flat_iter = (int32_t)get32(at + 80);
        const size_t base = at + 84;
        const size_t lat_b = (size_t)d.L * d.W * d.P * 4;
        HIP_OR_FAIL(ctx, hipMemcpyAsync(d.ctl, &c, sizeof c, hipMemcpyHostToDevice, ctx->stream));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(d.lat, b + base, lat_b, hipMemcpyHostToDevice, ctx->stream));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(d.lev, b + base + lat_b, (size_t)d.P * 4, hipMemcpyHostToDevice, ctx->stream));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(d.lnW, b + base + lat_b + (size_t)d.P * 4, (size_t)d.n_bins * 8,
                                        hipMemcpyHostToDevice, ctx->stream));
        HIP_OR_FAIL(ctx, hipMemsetAsync(d.hist64, 0, (size_t)d.n_bins * 8, ctx->stream));
        HIP_OR_FAIL(ctx, launch_tabulate(d, ctx->stream));
        HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
        h.pending = (int64_t)get64(at + 28);
        h.last_M = (int64_t)get64(at + 36);
        h.part_ld = h.part_done = 0;
        h.g_host = c.g;
        h.r_host = c.r;
        at += state_size_of(d);
    }
    return MC_OK;
}

mc_status mc_thermo(mc_ctx *ctx, int32_t i, const double *beta_host, int32_t n_beta, double *out_host) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    if (!beta_host || !out_host) return fail(MC_EINVAL, "null pointer");
    if (n_beta < 1 || n_beta > kThermoMaxBetas) return fail(MC_EINVAL, "n_beta must be 1..%d", kThermoMaxBetas);
    for (int k = 0; k < n_beta; ++k)
        if (!(beta_host[k] > 0.0) || !std::isfinite(beta_host[k]))
            return fail(MC_EINVAL, "beta[%d] must be positive and finite", k);
    if (n_beta > ctx->thermo_cap) {
        HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->thermo_buf) (void)hipFree(ctx->thermo_buf);
        ctx->thermo_buf = nullptr;
        ctx->thermo_cap = 0;
        if (hipMalloc((void **)&ctx->thermo_buf, (size_t)5 * n_beta * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MC_ENOMEM, "device allocation failed");
        }
        ctx->thermo_cap = n_beta;
    }
    double *beta_dev = ctx->thermo_buf, *out_dev = ctx->thermo_buf + n_beta;
    const SizeDev &d = ctx->sizes[i].dev;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(beta_dev, beta_host, (size_t)n_beta * 8, hipMemcpyHostToDevice, ctx->stream));
    HIP_OR_FAIL(ctx, launch_thermo(d, beta_dev, n_beta, out_dev, ctx->stream));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(out_host, out_dev, (size_t)4 * n_beta * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

mc_status mc_thermo_static(mc_ctx *ctx, int32_t i, const double *beta_host, int32_t n_beta, double *out_host) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    if (!beta_host || !out_host) return fail(MC_EINVAL, "null pointer");
    if (n_beta < 1 || n_beta > kThermoStaticMaxBetas)
        return fail(MC_EINVAL, "n_beta=%d must be 1..%d (the static array's capacity)", n_beta, kThermoStaticMaxBetas);
    for (int k = 0; k < n_beta; ++k)
        if (!(beta_host[k] > 0.0) || !std::isfinite(beta_host[k]))
            return fail(MC_EINVAL, "beta[%d] must be positive and finite", k);
    if (!ctx->thermo_static) return fail(MC_EHIP, "no static array on this device");
    // betas at [0, n_beta), results at [n_beta, 5 n_beta) of the array
    double *beta_dev = ctx->thermo_static, *out_dev = ctx->thermo_static + n_beta;
    const SizeDev &d = ctx->sizes[i].dev;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(beta_dev, beta_host, (size_t)n_beta * 8, hipMemcpyHostToDevice, ctx->stream));
    HIP_OR_FAIL(ctx, launch_thermo(d, beta_dev, n_beta, out_dev, ctx->stream));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(out_host, out_dev, (size_t)4 * n_beta * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

mc_status mc_get_progress(mc_ctx *ctx, int32_t i, int32_t *updates, int32_t *first_flat, int32_t *last_flat,
                          int64_t *retained_last) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    Ctl c{};
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&c, ctx->sizes[i].dev.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    if (updates) *updates = c.iter;
    if (first_flat) *first_flat = c.flat_iter;
    if (last_flat) *last_flat = c.flat;
    if (retained_last) *retained_last = c.retained_last;
    return MC_OK;
}

mc_status mc_set_chains_per_block(mc_ctx *ctx, int32_t i, int32_t chains_per_block) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    if (chains_per_block < 1 || chains_per_block > 64) return fail(MC_EINVAL, "chains_per_block must be 1..64");
    if (ctx->live_graphs > 0) return fail(MC_ESTATE, "the launch configuration is fixed while graphs exist");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    ctx->sizes[i].plan = plan_sweeps(ctx->sizes[i].dev, chains_per_block);
    HIP_OR_FAIL(ctx, rebuild_launch(ctx));
    return MC_OK;
}

mc_status mc_set_launch(mc_ctx *ctx, int32_t i, int32_t kind, int32_t chains_per_block) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    if (chains_per_block < 1 || chains_per_block > 64) return fail(MC_EINVAL, "chains_per_block must be 1..64");
    if (kind < 0 || kind > kSweepBigQGlb) return fail(MC_EINVAL, "kind must be 0..%d", (int)kSweepBigQGlb);
    if (ctx->live_graphs > 0) return fail(MC_ESTATE, "the launch configuration is fixed while graphs exist");
    const SizePlan p = plan_kind(ctx->sizes[i].dev, kind, chains_per_block);
    if (p.kind != kind || p.cpb != chains_per_block)
        return fail(MC_EINVAL, "size %d: kind %d does not run L=%d at %d chains per workgroup", i, kind,
                    ctx->sizes[i].dev.L, chains_per_block);
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    ctx->sizes[i].plan = p;
    HIP_OR_FAIL(ctx, rebuild_launch(ctx));
    return MC_OK;
}

mc_status mc_get_launch(mc_ctx *ctx, int32_t i, int32_t *chains_per_block, int32_t *kind, int32_t *batched) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    if (chains_per_block) *chains_per_block = ctx->sizes[i].plan.cpb;
    if (kind) *kind = ctx->sizes[i].plan.kind;
    if (batched) *batched = ctx->batched ? 1 : 0;
    return MC_OK;
}

mc_status mc_autotune(mc_ctx *ctx, int64_t probe_sweeps, int32_t *chains_per_block_out) {
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    if (probe_sweeps < 1 || probe_sweeps > 100000) return fail(MC_EINVAL, "probe_sweeps must be 1..100000");
    if (ctx->live_graphs > 0) return fail(MC_ESTATE, "the launch configuration is fixed while graphs exist");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    hipEvent_t e0, e1;
    HIP_OR_FAIL(ctx, hipEventCreate(&e0));
    HIP_OR_FAIL(ctx, hipEventCreate(&e1));
    const int cands[6] = {16, 32, 64, 16, 32, 64};  // producer/consumer kernel first, then single-wave
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < ctx->sizes.size() && e == hipSuccess; ++i) {
        HostSize &h = ctx->sizes[i];
        const SizeDev &d = h.dev;
        // probes run on copies of the chain state, so the chains are untouched
        SizeDev scr = d;
        scr.lat = nullptr;
        scr.lev = nullptr;
        scr.ctl = nullptr;
        void *tr = nullptr;
        int32_t *hs = nullptr;
        const size_t lat_b = (size_t)d.L * d.W * d.P * 4;
        e = hipMalloc((void **)&scr.lat, lat_b);
        if (e == hipSuccess) e = hipMalloc((void **)&scr.lev, (size_t)d.P * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&scr.ctl, sizeof(Ctl));
        if (e == hipSuccess) e = hipMalloc(&tr, (size_t)d.P * probe_sweeps * d.trace_bytes);
        if (e == hipSuccess) e = hipMalloc((void **)&hs, (size_t)d.n_bins * 4);
        float best = 1e30f;
        SizePlan best_plan = h.plan;
        for (int k = 0; k < 6 && e == hipSuccess; ++k) {
            const SizePlan cand = plan_sweeps(d, cands[k], k < 3);
            if (cand.kind == kSweepGeneric) break;
            e = prepare_sweeps(d, cand);
            float t_min = 1e30f;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                e = hipMemcpyAsync(scr.lat, d.lat, lat_b, hipMemcpyDeviceToDevice, ctx->stream);
                if (e == hipSuccess) e = hipMemcpyAsync(scr.lev, d.lev, (size_t)d.P * 4, hipMemcpyDeviceToDevice, ctx->stream);
                if (e == hipSuccess) e = hipMemcpyAsync(scr.ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToDevice, ctx->stream);
                if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
                if (e == hipSuccess) e = launch_sweeps(scr, cand, probe_sweeps, probe_sweeps, tr, hs, ctx->stream);
                if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                t_min = std::min(t_min, ms);
            }
            if (e == hipSuccess && t_min < best) {
                best = t_min;
                best_plan = cand;
            }
        }
        if (scr.lat) (void)hipFree(scr.lat);
        if (scr.lev) (void)hipFree(scr.lev);
        if (scr.ctl) (void)hipFree(scr.ctl);
        if (tr) (void)hipFree(tr);
        if (hs) (void)hipFree(hs);
        if (e == hipSuccess) h.plan = best_plan;
        if (chains_per_block_out) chains_per_block_out[i] = h.plan.cpb;
    }
    if (e == hipSuccess && ctx->sizes.size() > 1) e = autotune_batched(ctx, probe_sweeps, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune");
    HIP_OR_FAIL(ctx, rebuild_launch(ctx));
    if (chains_per_block_out)
        for (size_t i = 0; i < ctx->sizes.size(); ++i) chains_per_block_out[i] = ctx->sizes[i].plan.cpb;
    return MC_OK;
}

mc_status mc_graph_create(mc_ctx *ctx, int64_t n_sweeps, int32_t n_iters, void *const *trace_dev,
                          int32_t *const *hist_dev, int32_t *const *cut_dev, int32_t mode, mc_graph **out) {
    if (!out) return fail(MC_EINVAL, "null output pointer");
    *out = nullptr;
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    if (n_sweeps < 1 || n_sweeps > 0x7FFFFFFF) return fail(MC_EINVAL, "n_sweeps must be 1..2^31-1");
    if (n_iters < 1 || n_iters > 100000) return fail(MC_EINVAL, "n_iters must be 1..100000");
    if (mode < 0 || mode > 2) return fail(MC_EINVAL, "mode must be 0, 1 or 2");
    if (!trace_dev || !hist_dev || !cut_dev) return fail(MC_EINVAL, "null pointer array");
    const int n = (int)ctx->sizes.size();
    for (int i = 0; i < n; ++i) {
        const HostSize &h = ctx->sizes[i];
        if (!trace_dev[i] || !hist_dev[i] || !cut_dev[i]) return fail(MC_EINVAL, "size %d: null buffer", i);
        if (h.pending != 0 || h.last_M != 0)
            return fail(MC_ESTATE, "size %d: a graph must start after a weight update", i);
        if ((int64_t)h.dev.P * n_sweeps > 0x7FFFFFFFll)
            return fail(MC_EOVERFLOW, "size %d: one iteration exceeds the int32 histogram", i);
        if (h.part_ld != 0) return fail(MC_ESTATE, "size %d: a round is partly run", i);
        if ((uint64_t)n_sweeps * (uint64_t)n_iters > kCounterLimit || (uint64_t)n_iters > kCounterLimit)
            return fail(MC_EOVERFLOW, "size %d: %d iterations of %lld sweeps pass the 2^32 counters", i, n_iters,
                        (long long)n_sweeps);
    }
    if (!ctx->capture_stream)
        HIP_OR_FAIL(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    hipStream_t cs = ctx->capture_stream;
    HIP_OR_FAIL(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int it = 0; it < n_iters && e == hipSuccess; ++it) {
        e = enqueue_sweeps(ctx, cs, n_sweeps, n_sweeps, trace_dev, hist_dev);
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            const SizeDev &d = ctx->sizes[i].dev;
            if (mode == 2) e = launch_energy_order(d, trace_dev[i], n_sweeps, cs);
            if (e == hipSuccess)
                e = launch_join(d, trace_dev[i], n_sweeps, cut_dev[i], hist_dev[i], mode == 2 ? 0 : mode,
                                mode == 2 ? d.join_order : nullptr, cs);
        }
        for (int i = 0; i < n && e == hipSuccess; ++i) e = launch_update(ctx->sizes[i].dev, hist_dev[i], cs);
    }
    hipGraph_t graph = nullptr;
    hipError_t e_end = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = e_end;
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(ctx, e, "graph capture");
    }
    mc_graph *g = new mc_graph();
    g->graph = graph;
    g->ctx = ctx;
    g->sweeps = (uint64_t)n_sweeps * (uint64_t)n_iters;
    g->rounds = (uint64_t)n_iters;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return hip_fail(ctx, e, "graph instantiation");
    }
    ctx->live_graphs += 1;
    *out = g;
    return MC_OK;
}

mc_status mc_graph_launch(mc_ctx *ctx, mc_graph *g) {
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    if (!g || g->ctx != ctx) return fail(MC_EINVAL, "graph does not belong to this context");
    for (size_t i = 0; i < ctx->sizes.size(); ++i) {
        const HostSize &h = ctx->sizes[i];
        if (h.pending != 0 || h.last_M != 0 || h.part_ld != 0)
            return fail(MC_ESTATE, "a graph must start after a weight update");
        if (h.g_host + g->sweeps > kCounterLimit || h.r_host + g->rounds > kCounterLimit)
            return fail(MC_EOVERFLOW, "size %zu: a replay would pass the 2^32 sweep or round counters", i);
    }
    HIP_OR_FAIL(ctx, hipGraphLaunch(g->exec, ctx->stream));
    for (auto &h : ctx->sizes) {
        h.g_host += g->sweeps;
        h.r_host += g->rounds;
    }
    return MC_OK;
}

mc_status mc_graph_destroy(mc_graph *g) {
    if (!g) return MC_OK;
    if (g->ctx) {
        (void)hipStreamSynchronize(g->ctx->stream);
        g->ctx->live_graphs -= 1;
    }
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return MC_OK;
}

mc_status mc_get_stats(mc_ctx *ctx, int32_t i, mc_stats *out) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    if (!out) return fail(MC_EINVAL, "null output");
    Ctl c{};
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&c, ctx->sizes[i].dev.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    mc_stats o{};
    o.updates = c.iter;
    o.first_flat = c.flat_iter;
    o.last_flat = c.flat;
    o.retained_last = c.retained_last;
    o.hist_sum = c.upd_h_sum;
    o.hist_min = c.upd_h_min;
    o.n_reach_bins = c.upd_n_reach;
    o.lnw_min = c.iter > 0 ? c.upd_lnw_lo : 0.0;
    o.lnw_max = c.iter > 0 ? c.upd_lnw_hi : 0.0;
    o.join_none = c.join_none;
    o.join_cut_max = c.join_cut_max;
    o.join_cut_sum = c.join_cut_sum;
    o.sweep_index = c.g;
    o.round_index = c.r;
    o.seam = c.sigma;
    *out = o;
    return MC_OK;
}

mc_status mc_check_levels(mc_ctx *ctx, int32_t i, int64_t *n_bad) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    const SizeDev &d = ctx->sizes[i].dev;
    int64_t bad = 0;
    HIP_OR_FAIL(ctx, launch_check_levels(d, ctx->stream));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&bad, d.n_bad, sizeof bad, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    if (n_bad) *n_bad = bad;
    if (bad != 0)
        return fail(MC_EINTERNAL, "size %d: %lld chains hold a level that is not half their broken bonds", i,
                    (long long)bad);
    return MC_OK;
}

}  // extern "C"

