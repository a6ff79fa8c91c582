// mc_api.hip -- host side of the C ABI declared in include/mc.h: argument
// validation, device state of a context, and the order of kernel launches for
// Algorithm steps 1-5 and eq. (new_weight) of arXiv 0812.2964.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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
    int64_t pending;   // configurations added to histograms since the last update
    int64_t last_M;    // sweeps of the last mc_run_chains, 0 after its joint
};

}  // namespace

struct mc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool broken = false;
    int chains_per_block = 64;
    std::vector<HostSize> sizes;
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
    if (d.ctl) (void)hipFree(d.ctl);
    if (d.scratch_cut) (void)hipFree(d.scratch_cut);
    d = SizeDev{};
}

}  // namespace

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
    ctx->sizes.resize(n_sizes);
    mc_status st = MC_OK;
    for (int i = 0; i < n_sizes && st == MC_OK; ++i) {
        HostSize &h = ctx->sizes[i];
        h.cfg = sizes[i];
        h.pending = 0;
        h.last_M = 0;
        SizeDev &d = h.dev;
        d = SizeDev{};
        d.L = h.cfg.L;
        d.N = d.L * d.L;
        d.W = (d.L + 31) / 32;
        d.P = h.cfg.n_chains;
        d.bin_shift = h.cfg.bin_shift;
        d.n_bins = (d.N >> d.bin_shift) + 1;
        d.seed = h.cfg.seed;
        d.trace_bytes = (d.L <= 254) ? 2 : 4;
        const size_t lat_b = (size_t)d.L * d.W * d.P * 4;
        if (hipMalloc((void **)&d.lat, lat_b) != hipSuccess || hipMalloc((void **)&d.lev, (size_t)d.P * 4) != hipSuccess ||
            hipMalloc((void **)&d.lnW, (size_t)d.n_bins * 8) != hipSuccess ||
            hipMalloc((void **)&d.tab, (size_t)(d.N + 1) * 8 * 4) != hipSuccess ||
            hipMalloc((void **)&d.ctl, sizeof(Ctl)) != hipSuccess ||
            hipMalloc((void **)&d.scratch_cut, (size_t)d.P * 4) != hipSuccess) {
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
        if (e == hipSuccess) e = launch_init(d, ctx->stream);
        if (e == hipSuccess) e = launch_tabulate(d, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = hip_fail(nullptr, e, "context initialisation");
    }
    if (st != MC_OK) {
        for (auto &h : ctx->sizes) free_size(h.dev);
        delete ctx;
        return st;
    }
    *out = ctx;
    return MC_OK;
}

mc_status mc_destroy(mc_ctx *ctx) {
    if (!ctx) return MC_OK;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &h : ctx->sizes) free_size(h.dev);
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
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    if (n_sweeps < 1 || n_sweeps > 0x7FFFFFFF) return fail(MC_EINVAL, "n_sweeps=%lld must be 1..2^31-1", (long long)n_sweeps);
    if (!trace_dev || !hist_dev) return fail(MC_EINVAL, "null trace/hist pointer array");
    const int n = (int)ctx->sizes.size();
    std::vector<SizeDev> devs(n);
    for (int i = 0; i < n; ++i) {
        HostSize &h = ctx->sizes[i];
        if (!trace_dev[i] || !hist_dev[i]) return fail(MC_EINVAL, "size %d: null trace or hist", i);
        const int64_t add = (int64_t)h.dev.P * n_sweeps;
        if (h.pending + add > 0x7FFFFFFFll)
            return fail(MC_EOVERFLOW, "size %d: %lld configurations would exceed the int32 histogram", i,
                        (long long)(h.pending + add));
        devs[i] = h.dev;
    }
    HIP_OR_FAIL(ctx, launch_sweeps(devs.data(), n, n_sweeps, trace_dev, hist_dev, ctx->chains_per_block, ctx->stream));
    for (int i = 0; i < n; ++i) {
        ctx->sizes[i].pending += (int64_t)ctx->sizes[i].dev.P * n_sweeps;
        ctx->sizes[i].last_M = n_sweeps;
    }
    return MC_OK;
}

mc_status mc_join(mc_ctx *ctx, int32_t i, const void *trace_dev, int64_t n_sweeps, int32_t *cut_dev, int32_t *hist_dev,
                  int32_t mode) {
    mc_status st = check_size(ctx, i);
    if (st != MC_OK) return st;
    HostSize &h = ctx->sizes[i];
    if (!trace_dev || !cut_dev || !hist_dev) return fail(MC_EINVAL, "null trace, cut or hist");
    if (mode != 0 && mode != 1) return fail(MC_EINVAL, "mode must be 0 or 1");
    if (h.last_M == 0) return fail(MC_ESTATE, "size %d: no mc_run_chains to join", i);
    if (n_sweeps != h.last_M)
        return fail(MC_EINVAL, "n_sweeps=%lld differs from the last run (%lld)", (long long)n_sweeps, (long long)h.last_M);
    HIP_OR_FAIL(ctx, launch_join(h.dev, trace_dev, n_sweeps, cut_dev, hist_dev, mode, ctx->stream));
    h.last_M = 0;
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

mc_status mc_sync(mc_ctx *ctx) {
    mc_status st = check_ctx(ctx);
    if (st != MC_OK) return st;
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

}  // extern "C"
