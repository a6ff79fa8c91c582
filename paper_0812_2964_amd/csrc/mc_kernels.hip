// mc_kernels.hip -- HIP kernels (gfx950) of the parallel multicanonical method
// of arXiv 0812.2964 on the periodic 2D Ising model.
//
//   k_init        Algorithm step 1: random initial spins, level of each chain
//   k_tabulate    Metropolis thresholds of the current weight (Sec. 4.2)
//   k_sweep_*     Algorithm step 2: one chain per lane, typewriter sweeps
//   k_join_*      Algorithm steps 3-5: detailed-balance joints between chains
//   k_update      eq. (new_weight) in logarithms + flatness test
//
// Lattice layout: each row of a chain is W = ceil(L/32) 32-bit words (bit x%32
// of word x/32 is site x, 1 = spin up); word w of row y of chain c lives at
// lat[(y*W + w)*P + c], so that consecutive lanes (chains) touch consecutive
// words.
#include "mc_internal.h"
#include "mc_math.h"

namespace mcgpu {

// ---------------------------------------------------------------------------
// Algorithm step 1.
// ---------------------------------------------------------------------------
__global__ void k_init(SizeDev s) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= s.P) return;
    const int L = s.L, W = s.W;
    for (int y = 0; y < L; ++y) {
        for (int w = 0; w < W; ++w) {
            uint32_t word = 0;
            for (int b = 0; b < 32; ++b) {
                const int x = w * 32 + b;
                if (x >= L) break;
                const uint32_t j = (uint32_t)(y * L + x);
                const uint4 blk = philox10(make_uint4(j >> 2, 0u, (uint32_t)c, kDomInit), s.seed, (uint32_t)L);
                word |= (word_of(blk, j & 3u) >> 31) << b;
            }
            s.lat[(size_t)(y * W + w) * s.P + c] = word;
        }
    }
    // level = (number of broken bonds) / 2, each bond counted once (right, down)
    int broken = 0;
    for (int y = 0; y < L; ++y) {
        const int yd = (y + 1) % L;
        for (int x = 0; x < L; ++x) {
            const int xr = (x + 1) % L;
            const uint32_t sv = (s.lat[(size_t)(y * W + (x >> 5)) * s.P + c] >> (x & 31)) & 1u;
            const uint32_t sr = (s.lat[(size_t)(y * W + (xr >> 5)) * s.P + c] >> (xr & 31)) & 1u;
            const uint32_t sd = (s.lat[(size_t)(yd * W + (x >> 5)) * s.P + c] >> (x & 31)) & 1u;
            broken += (int)(sv ^ sr) + (int)(sv ^ sd);
        }
    }
    s.lev[c] = broken / 2;
}

hipError_t launch_init(const SizeDev &s, hipStream_t st) {
    const int bs = 64;
    hipLaunchKernelGGL(k_init, dim3((s.P + bs - 1) / bs), dim3(bs), 0, st, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Thresholds: entry (m, a) = tau(ln w[b(m + a - 2)] - ln w[b(m)]) for a = 0..4
// with the target level inside [0, N]; every other entry is 0 (never used).
// ---------------------------------------------------------------------------
__global__ void k_tabulate(SizeDev s) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m > s.N) return;
    const double w0 = s.lnW[m >> s.bin_shift];
    for (int a = 0; a < 8; ++a) {
        const int mt = m + a - 2;
        uint32_t t = 0u;
        if (a <= 4 && mt >= 0 && mt <= s.N) t = tau_of(s.lnW[mt >> s.bin_shift] - w0);
        s.tab[(size_t)m * 8 + a] = t;
    }
}

hipError_t launch_tabulate(const SizeDev &s, hipStream_t st) {
    const int bs = 256;
    hipLaunchKernelGGL(k_tabulate, dim3((s.N + 1 + bs - 1) / bs), dim3(bs), 0, st, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Algorithm step 2.  One chain per lane; CPB chains per 64-lane block.
// ---------------------------------------------------------------------------
struct SweepParams {
    SizeDev s;
    int64_t M;
    void *trace;
    int32_t *hist;
    int32_t cpb;
    int32_t lds_hist;
};

template <int L>
struct Row {
    uint32_t w[(L + 31) / 32];
};

template <int L>
__device__ __forceinline__ uint32_t bit_at(const Row<L> &r, int x) {
    return (r.w[x >> 5] >> (x & 31)) & 1u;
}

// Row r' with r'_x = r_{(x+1) mod L} (bit x of the result is the right-hand
// neighbour of site x).  Padding bits above L stay zero.
template <int L>
__device__ __forceinline__ Row<L> ring_next(const Row<L> &c) {
    constexpr int W = (L + 31) / 32;
    Row<L> r;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        r.w[w] = c.w[w] >> 1;
        if (w + 1 < W) r.w[w] |= c.w[w + 1] << 31;
    }
    r.w[W - 1] |= (c.w[0] & 1u) << ((L - 1) & 31);
    return r;
}

// One row of typewriter Metropolis attempts (Sec. 2 step 2 with the energy of
// Sec. 4.1 and the Metropolis rule of Sec. 4.2).
//
// Level bookkeeping: mi = 8 m + 4, so the threshold of a flip with `anti`
// anti-aligned neighbours (level change a - 2 = 2 - anti) sits at tab[mi - anti]
// and an accepted flip moves mi by D = 16 - 8 anti.
//
// The number of anti-aligned neighbours of site x is fixed at the start of the
// row except for its left neighbour x-1, which may have flipped just before
// (and, for x = L-1, its right neighbour 0).  So while the test at site x is
// being decided, both thresholds site x+1 can need -- site x rejected (level
// unchanged, left bond as at row start) or accepted (level moved by D, left
// bond toggled) -- are already being read from LDS; the decision then only
// selects one.  xu, xd, hb: bits x of (row ^ up), (row ^ down), (row ^ right
// neighbour), all at row start.
template <int L>
__device__ __forceinline__ void sweep_row(uint32_t y, uint32_t g, uint32_t c, uint32_t k0, uint32_t k1, Row<L> &cur,
                                          const Row<L> &up, const Row<L> &dn, int &mi, const uint32_t *tab) {
    constexpr int W = (L + 31) / 32;
    Row<L> xu, xd, hb;
    const Row<L> nx = ring_next<L>(cur);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        xu.w[w] = cur.w[w] ^ up.w[w];
        xd.w[w] = cur.w[w] ^ dn.w[w];
        hb.w[w] = cur.w[w] ^ nx.w[w];
    }
    // site 0: every neighbour is as at row start (its left neighbour L-1 comes last)
    int anti = (int)(bit_at<L>(xu, 0) + bit_at<L>(xd, 0) + bit_at<L>(hb, 0) + bit_at<L>(hb, L - 1));
    uint32_t t = tab[mi - anti];
    int D = 16 - 8 * anti;
    uint32_t f0 = 0;
    uint4 rnd = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int x = 0; x < L; ++x) {
        if ((x & 3) == 0)
            rnd = philox10(make_uint4(y * (uint32_t)(L / 4) + (uint32_t)(x >> 2), g, c, kDomSweep), k0, k1);
        const uint32_t u = (x & 3) == 0 ? rnd.x : (x & 3) == 1 ? rnd.y : (x & 3) == 2 ? rnd.z : rnd.w;
        int an0 = 0, an1 = 0;
        uint32_t t0n = 0, t1n = 0;
        if (x + 1 < L) {
            const int xn = x + 1;
            const uint32_t left = bit_at<L>(hb, x);  // bond (x, x+1) at row start
            uint32_t right = bit_at<L>(hb, xn);      // bond (x+1, x+2)
            if (xn == L - 1) right ^= f0;            // its right neighbour is site 0
            an0 = (int)(bit_at<L>(xu, xn) + bit_at<L>(xd, xn) + right + left);
            an1 = an0 + 1 - 2 * (int)left;
            t0n = tab[mi - an0];
            t1n = tab[mi + D - an1];
        }
        const bool acc = u <= t;
        if (x == 0) f0 = acc ? 1u : 0u;
        cur.w[x >> 5] ^= (acc ? 1u : 0u) << (x & 31);
        mi = acc ? mi + D : mi;
        if (x + 1 < L) {
            anti = acc ? an1 : an0;
            t = acc ? t1n : t0n;
            D = 16 - 8 * anti;
        }
    }
}

// Lattice and (optionally) thresholds in LDS.  LDS layout:
//   [L*W*cpb] lattice words, word (row*W + w) of local chain l at (row*W+w)*cpb + l
//   [(N+1)*8] thresholds           (TAB_LDS)
//   [n_bins]  histogram            (lds_hist)
template <int L, bool TAB_LDS>
__global__ __launch_bounds__(64) void k_sweep_lds(SweepParams p) {
    constexpr int W = (L + 31) / 32;
    constexpr int N = L * L;
    extern __shared__ uint32_t smem[];
    const SizeDev &s = p.s;
    const int cpb = p.cpb;
    const int lane = threadIdx.x;
    const int c = blockIdx.x * cpb + lane;
    const bool active = lane < cpb && c < s.P;
    uint32_t *slat = smem;
    uint32_t *stab = smem + L * W * cpb;
    int32_t *shist = (int32_t *)(stab + (TAB_LDS ? (N + 1) * 8 : 0));
    const uint32_t *tab = TAB_LDS ? stab : s.tab;
    if (TAB_LDS)
        for (int i = lane; i < (N + 1) * 8; i += blockDim.x) stab[i] = s.tab[i];
    if (p.lds_hist)
        for (int i = lane; i < s.n_bins; i += blockDim.x) shist[i] = 0;
    if (active)
        for (int w = 0; w < L * W; ++w) slat[w * cpb + lane] = s.lat[(size_t)w * s.P + c];
    __syncthreads();

    if (active) {
        int mi = 8 * s.lev[c] + 4;
        const uint32_t g0 = s.ctl->g;
        const uint32_t k0 = s.seed, k1 = (uint32_t)L;
        auto load = [&](int y) {
            Row<L> r;
#pragma unroll
            for (int w = 0; w < W; ++w) r.w[w] = slat[(y * W + w) * cpb + lane];
            return r;
        };
        auto store = [&](int y, const Row<L> &r) {
#pragma unroll
            for (int w = 0; w < W; ++w) slat[(y * W + w) * cpb + lane] = r.w[w];
        };
        for (int64_t k = 0; k < p.M; ++k) {
            const uint32_t g = g0 + (uint32_t)k;
            Row<L> up = load(L - 1);
            Row<L> cur = load(0);
            Row<L> dn = load(1);
            for (int y = 0; y < L; ++y) {
                sweep_row<L>((uint32_t)y, g, (uint32_t)c, k0, k1, cur, up, dn, mi, tab);
                store(y, cur);
                up = cur;
                cur = dn;
                dn = load(y + 2 < L ? y + 2 : y + 2 - L);
            }
            const int m = mi >> 3;
            const int ev = m - N / 2;
            if (s.trace_bytes == 2)
                ((int16_t *)p.trace)[(size_t)c * p.M + k] = (int16_t)ev;
            else
                ((int32_t *)p.trace)[(size_t)c * p.M + k] = ev;
            if (p.lds_hist)
                atomicAdd(&shist[m >> s.bin_shift], 1);
            else
                atomicAdd(&p.hist[m >> s.bin_shift], 1);
        }
        s.lev[c] = mi >> 3;
    }
    __syncthreads();
    if (active)
        for (int w = 0; w < L * W; ++w) s.lat[(size_t)w * s.P + c] = slat[w * cpb + lane];
    if (p.lds_hist)
        for (int i = lane; i < s.n_bins; i += blockDim.x)
            if (shist[i]) atomicAdd(&p.hist[i], shist[i]);
}

// Lattice rows streamed from global memory (large L); thresholds from global.
template <int L>
__global__ __launch_bounds__(64) void k_sweep_glb(SweepParams p) {
    constexpr int W = (L + 31) / 32;
    constexpr int N = L * L;
    const SizeDev &s = p.s;
    const int lane = threadIdx.x;
    const int c = blockIdx.x * p.cpb + lane;
    if (lane >= p.cpb || c >= s.P) return;
    uint32_t *lat = s.lat;
    const size_t P = (size_t)s.P;
    auto load = [&](int y) {
        Row<L> r;
#pragma unroll
        for (int w = 0; w < W; ++w) r.w[w] = lat[(size_t)(y * W + w) * P + c];
        return r;
    };
    auto store = [&](int y, const Row<L> &r) {
#pragma unroll
        for (int w = 0; w < W; ++w) lat[(size_t)(y * W + w) * P + c] = r.w[w];
    };
    int mi = 8 * s.lev[c] + 4;
    const uint32_t g0 = s.ctl->g;
    const uint32_t k0 = s.seed, k1 = (uint32_t)L;
    for (int64_t k = 0; k < p.M; ++k) {
        const uint32_t g = g0 + (uint32_t)k;
        Row<L> up = load(L - 1);
        Row<L> cur = load(0);
        Row<L> dn = load(1);
        for (int y = 0; y < L; ++y) {
            sweep_row<L>((uint32_t)y, g, (uint32_t)c, k0, k1, cur, up, dn, mi, s.tab);
            store(y, cur);
            up = cur;
            cur = dn;
            dn = load(y + 2 < L ? y + 2 : y + 2 - L);
        }
        const int m = mi >> 3;
        const int ev = m - N / 2;
        if (s.trace_bytes == 2)
            ((int16_t *)p.trace)[(size_t)c * p.M + k] = (int16_t)ev;
        else
            ((int32_t *)p.trace)[(size_t)c * p.M + k] = ev;
        atomicAdd(&p.hist[m >> s.bin_shift], 1);
    }
    s.lev[c] = mi >> 3;
}

// Any even L (also L not a multiple of 4): bit-by-bit from global memory.
__global__ __launch_bounds__(64) void k_sweep_generic(SweepParams p) {
    const SizeDev &s = p.s;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= s.P) return;
    const int L = s.L, W = s.W, N = s.N;
    const size_t P = (size_t)s.P;
    auto word = [&](int y, int x) -> uint32_t & { return s.lat[(size_t)(y * W + (x >> 5)) * P + c]; };
    auto spin = [&](int y, int x) -> uint32_t { return (word(y, x) >> (x & 31)) & 1u; };
    int m = s.lev[c];
    const uint32_t g0 = s.ctl->g;
    for (int64_t k = 0; k < p.M; ++k) {
        const uint32_t g = g0 + (uint32_t)k;
        uint4 blk = make_uint4(0, 0, 0, 0);
        for (int j = 0; j < N; ++j) {
            if ((j & 3) == 0)
                blk = philox10(make_uint4((uint32_t)j >> 2, g, (uint32_t)c, kDomSweep), s.seed, (uint32_t)L);
            const uint32_t u = word_of(blk, (uint32_t)j & 3u);
            const int x = j % L, y = j / L;
            const uint32_t sv = spin(y, x);
            const uint32_t anti = (sv ^ spin(y, (x + 1) % L)) + (sv ^ spin(y, (x + L - 1) % L)) +
                                  (sv ^ spin((y + 1) % L, x)) + (sv ^ spin((y + L - 1) % L, x));
            const uint32_t a = 4u - anti;
            if (u <= s.tab[(size_t)m * 8 + a]) {
                word(y, x) ^= 1u << (x & 31);
                m += (int)a - 2;
            }
        }
        const int ev = m - N / 2;
        if (s.trace_bytes == 2)
            ((int16_t *)p.trace)[(size_t)c * p.M + k] = (int16_t)ev;
        else
            ((int32_t *)p.trace)[(size_t)c * p.M + k] = ev;
        atomicAdd(&p.hist[m >> s.bin_shift], 1);
    }
    s.lev[c] = m;
}

__global__ void k_advance_sweeps(Ctl *ctl, uint32_t M) { ctl->g += M; }

template <int L>
static hipError_t launch_sweep_L(const SweepParams &p0, hipStream_t st) {
    constexpr int W = (L + 31) / 32;
    constexpr int N = L * L;
    SweepParams p = p0;
    const int cpb = p.cpb;
    const size_t lat_b = (size_t)L * W * cpb * 4;
    const size_t tab_b = (size_t)(N + 1) * 8 * 4;
    const size_t hist_b = (size_t)p.s.n_bins * 4;
    const size_t lds_max = 160 * 1024;
    const dim3 grid((p.s.P + cpb - 1) / cpb), block(64);
    if (L <= 64 && lat_b + tab_b + hist_b <= lds_max) {
        p.lds_hist = 1;
        const size_t bytes = lat_b + tab_b + hist_b;
        auto kern = k_sweep_lds<L, true>;
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, grid, block, bytes, st, p);
    } else if (L <= 64 && lat_b + hist_b <= lds_max) {
        p.lds_hist = 1;
        const size_t bytes = lat_b + hist_b;
        auto kern = k_sweep_lds<L, false>;
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, grid, block, bytes, st, p);
    } else {
        p.lds_hist = 0;
        hipLaunchKernelGGL(k_sweep_glb<L>, grid, block, 0, st, p);
    }
    return hipGetLastError();
}

hipError_t launch_sweeps(const SizeDev *sizes, int n_sizes, int64_t M, void *const *trace, int32_t *const *hist,
                         int chains_per_block, hipStream_t st) {
    for (int i = 0; i < n_sizes; ++i) {
        SweepParams p{};
        p.s = sizes[i];
        p.M = M;
        p.trace = trace[i];
        p.hist = hist[i];
        p.cpb = chains_per_block;
        p.lds_hist = 0;
        hipError_t e = hipSuccess;
        switch (p.s.L) {
        case 4: e = launch_sweep_L<4>(p, st); break;
        case 8: e = launch_sweep_L<8>(p, st); break;
        case 12: e = launch_sweep_L<12>(p, st); break;
        case 16: e = launch_sweep_L<16>(p, st); break;
        case 20: e = launch_sweep_L<20>(p, st); break;
        case 24: e = launch_sweep_L<24>(p, st); break;
        case 32: e = launch_sweep_L<32>(p, st); break;
        case 40: e = launch_sweep_L<40>(p, st); break;
        case 48: e = launch_sweep_L<48>(p, st); break;
        case 64: e = launch_sweep_L<64>(p, st); break;
        case 128: e = launch_sweep_L<128>(p, st); break;
        case 256: e = launch_sweep_L<256>(p, st); break;
        default:
            hipLaunchKernelGGL(k_sweep_generic, dim3((p.s.P + 63) / 64), dim3(64), 0, st, p);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_advance_sweeps, dim3(1), dim3(1), 0, st, p.s.ctl, (uint32_t)M);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Algorithm steps 3-5.
//  (1) k_join_spec: one wave per chain i finds its first accepted position
//      against the seam it would see if chain i-1 kept something (the level
//      of chain i-1's last configuration; for i = 0 the carried seam), testing
//      64 positions per step.
//  (2) k_join_fix: one wave walks the chains in order with the true seam and
//      re-tests only chains whose true seam lies in another bin than the
//      speculated one (the test depends on the seam only through ln w of its
//      bin, and its random words do not depend on the seam at all).
//  (3) k_join_hist: the discarded prefixes are taken out of the histogram.
// ---------------------------------------------------------------------------
struct JoinParams {
    SizeDev s;
    const void *trace;
    int64_t M;
    int32_t *cut;
    int32_t *hist;
    int32_t mode;
};

template <typename TT>
__device__ int join_scan(const SizeDev &s, const TT *row, int64_t M, int sigma, uint32_t r, uint32_t i) {
    const int lane = threadIdx.x & 63;
    const int half = s.N / 2;
    const double ws = s.lnW[sigma >> s.bin_shift];
    for (int64_t k0 = 0; k0 < M; k0 += 64) {
        const int64_t k = k0 + lane;
        bool acc = false;
        if (k < M) {
            const int mk = min(max((int)row[k] + half, 0), s.N);  // traces come from the sweeps; clamp anyway
            const uint32_t t = tau_of(s.lnW[mk >> s.bin_shift] - ws);
            const uint4 blk = philox10(make_uint4((uint32_t)k >> 2, r, i, kDomJoin), s.seed, (uint32_t)s.L);
            acc = word_of(blk, (uint32_t)k & 3u) <= t;
        }
        const unsigned long long bal = __ballot(acc);
        if (bal) return (int)(k0 + __ffsll(bal)); /* 1-based */
    }
    return -1;
}

template <typename TT>
__global__ __launch_bounds__(64) void k_join_spec(JoinParams p) {
    const SizeDev &s = p.s;
    const int i = blockIdx.x;
    const TT *tr = (const TT *)p.trace;
    const int half = s.N / 2;
    const int sigma =
        (i == 0) ? s.ctl->sigma : min(max((int)tr[(size_t)(i - 1) * p.M + (p.M - 1)] + half, 0), s.N);
    int cut;
    if (p.mode == 1 || sigma < 0)
        cut = 1;
    else
        cut = join_scan<TT>(s, tr + (size_t)i * p.M, p.M, sigma, s.ctl->r, (uint32_t)i);
    if (threadIdx.x == 0) s.scratch_cut[i] = cut;
}

template <typename TT>
__global__ __launch_bounds__(64) void k_join_fix(JoinParams p) {
    constexpr int CH = 1024;
    __shared__ int s_cut[CH];
    __shared__ int s_last[CH + 1];
    const SizeDev &s = p.s;
    const TT *tr = (const TT *)p.trace;
    const int half = s.N / 2;
    const int lane = threadIdx.x;
    const uint32_t r = s.ctl->r;
    int sigma = s.ctl->sigma;
    int64_t kept = 0;
    for (int c0 = 0; c0 < s.P; c0 += CH) {
        const int n = min(CH, s.P - c0);
        __syncthreads();
        for (int t = lane; t < n; t += 64) {
            s_cut[t] = s.scratch_cut[c0 + t];
            s_last[t + 1] = min(max((int)tr[(size_t)(c0 + t) * p.M + (p.M - 1)] + half, 0), s.N);
        }
        if (lane == 0)
            s_last[0] = c0 > 0 ? min(max((int)tr[(size_t)(c0 - 1) * p.M + (p.M - 1)] + half, 0), s.N) : s.ctl->sigma;
        __syncthreads();
        for (int t = 0; t < n; ++t) {
            const int i = c0 + t;
            int cut = s_cut[t];
            const int spec = s_last[t];  // seam assumed by k_join_spec
            if (p.mode == 0 && i > 0 && sigma >= 0 && (sigma >> s.bin_shift) != (spec >> s.bin_shift))
                cut = join_scan<TT>(s, tr + (size_t)i * p.M, p.M, sigma, r, (uint32_t)i);
            if (lane == 0) p.cut[i] = cut;
            if (cut > 0) {
                kept += p.M - cut + 1;
                sigma = s_last[t + 1];
            }
        }
    }
    if (lane == 0) {
        s.ctl->sigma = sigma;
        s.ctl->retained += kept;
        s.ctl->r = r + 1;
    }
}

template <typename TT>
__global__ __launch_bounds__(256) void k_join_hist(JoinParams p) {
    extern __shared__ uint32_t smem[];
    int32_t *sh = (int32_t *)smem;
    const SizeDev &s = p.s;
    const int i = blockIdx.x;
    const int cut = p.cut[i];
    const int64_t ndisc = cut > 0 ? (int64_t)cut - 1 : p.M;
    if (ndisc == 0) return;
    const TT *row = (const TT *)p.trace + (size_t)i * p.M;
    const int half = s.N / 2;
    const bool use_lds = ndisc > 256 && s.n_bins <= 16384;
    if (use_lds) {
        for (int b = threadIdx.x; b < s.n_bins; b += blockDim.x) sh[b] = 0;
        __syncthreads();
        for (int64_t k = threadIdx.x; k < ndisc; k += blockDim.x)
            atomicAdd(&sh[min(max((int)row[k] + half, 0), s.N) >> s.bin_shift], 1);
        __syncthreads();
        for (int b = threadIdx.x; b < s.n_bins; b += blockDim.x)
            if (sh[b]) atomicSub(&p.hist[b], sh[b]);
    } else {
        for (int64_t k = threadIdx.x; k < ndisc; k += blockDim.x)
            atomicSub(&p.hist[min(max((int)row[k] + half, 0), s.N) >> s.bin_shift], 1);
    }
}

template <typename TT>
static hipError_t launch_join_T(const JoinParams &p, hipStream_t st) {
    hipLaunchKernelGGL(k_join_spec<TT>, dim3(p.s.P), dim3(64), 0, st, p);
    hipLaunchKernelGGL(k_join_fix<TT>, dim3(1), dim3(64), 0, st, p);
    const size_t lds = p.s.n_bins <= 16384 ? (size_t)p.s.n_bins * 4 : 0;
    if (lds > 64 * 1024) {
        hipError_t e =
            hipFuncSetAttribute((const void *)k_join_hist<TT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_join_hist<TT>, dim3(p.s.P), dim3(256), lds, st, p);
    return hipGetLastError();
}

hipError_t launch_join(const SizeDev &s, const void *trace, int64_t M, int32_t *cut, int32_t *hist, int mode,
                       hipStream_t st) {
    JoinParams p{s, trace, M, cut, hist, mode};
    return s.trace_bytes == 2 ? launch_join_T<int16_t>(p, st) : launch_join_T<int32_t>(p, st);
}

// ---------------------------------------------------------------------------
// eq. (new_weight): ln w(b) -= ln h(b) where h(b) > 0; flatness over the bins
// holding a reachable level (every level except 1 and N-1); h := 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool bin_reachable(int b, int bin_shift, int N) {
    for (int m = b << bin_shift; m < ((b + 1) << bin_shift) && m <= N; ++m)
        if (m != 1 && m != N - 1) return true;
    return false;
}

__global__ __launch_bounds__(1024) void k_update(SizeDev s, int32_t *hist) {
    __shared__ long long s_min[16], s_sum[16];
    __shared__ int s_n[16];
    long long mn = 0x7FFFFFFFFFFFFFFFll, sum = 0;
    int n = 0;
    for (int b = threadIdx.x; b < s.n_bins; b += blockDim.x) {
        const int h = hist[b];
        if (h > 0) s.lnW[b] = s.lnW[b] - det_log((int64_t)h);
        if (bin_reachable(b, s.bin_shift, s.N)) {
            n += 1;
            sum += h;
            mn = h < mn ? h : mn;
        }
        hist[b] = 0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const long long omn = __shfl_xor(mn, off, 64);
        mn = omn < mn ? omn : mn;
        sum += __shfl_xor(sum, off, 64);
        n += __shfl_xor(n, off, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_min[wv] = mn;
        s_sum[wv] = sum;
        s_n[wv] = n;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        long long tmn = s_min[0], tsum = 0;
        int tn = 0;
        for (int i = 0; i < nw; ++i) {
            tmn = s_min[i] < tmn ? s_min[i] : tmn;
            tsum += s_sum[i];
            tn += s_n[i];
        }
        const int flat = (tn > 0 && tsum > 0 && 5ll * tn * tmn >= 4ll * tsum) ? 1 : 0;
        Ctl *ctl = s.ctl;
        ctl->flat = flat;
        ctl->iter += 1;
        if (flat && ctl->flat_iter == 0) ctl->flat_iter = ctl->iter;
        ctl->retained_last = ctl->retained;
        ctl->retained = 0;
    }
}

hipError_t launch_update(const SizeDev &s, int32_t *hist, hipStream_t st) {
    hipLaunchKernelGGL(k_update, dim3(1), dim3(1024), 0, st, s, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tabulate(s, st);
}

}  // namespace mcgpu
