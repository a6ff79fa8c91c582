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
                const uint4 blk = philox10(make_uint4(j >> 2, 0u, (uint32_t)c + s.c_off, kDomInit), s.seed, (uint32_t)L);
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

// The same thresholds per bin (used by the large-lattice sweeps): bin b has
// K = 2r + 1 entries, entry j for a move into bin b + j - r (a flip changes the
// level by at most 2, so r = 2 with one level per bin and r = 1 otherwise).
// The threshold of a move from level m to m' is entry K (m >> bs) +
// (m' >> bs) - (m >> bs) + r, at byte 4 r + 8 r (m >> bs) + 4 (m' >> bs).
// Entries of bins outside [0, n_bins) are 0 and never used.
__global__ void k_tabulate_compact(SizeDev s) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= s.n_bins) return;
    const int r = s.tab_r, K = 2 * r + 1;
    const double w0 = s.lnW[b];
    for (int j = 0; j < K; ++j) {
        const int bt = b + j - r;
        uint32_t t = 0u;
        if (bt >= 0 && bt < s.n_bins) t = tau_of(s.lnW[bt] - w0);
        s.tabc[(size_t)b * K + j] = t;
    }
}

hipError_t launch_tabulate(const SizeDev &s, hipStream_t st) {
    const int bs = 256;
    hipLaunchKernelGGL(k_tabulate, dim3((s.N + 1 + bs - 1) / bs), dim3(bs), 0, st, s);
    hipLaunchKernelGGL(k_tabulate_compact, dim3((s.n_bins + bs - 1) / bs), dim3(bs), 0, st, s);
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
    // fully unrolled up to L = 64 (the row's words and bit positions become
    // constants); larger rows by 32 sites, within the instruction cache
    constexpr int kUnrollSites = L <= 64 ? L : 32;
#pragma unroll kUnrollSites
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

// Sweeps of the chains c0 .. c0+cpb-1 of one size, lane l = chain c0 + l,
// with the lattices and (TAB_LDS) the thresholds held in LDS.  LDS layout:
//   [L*W*cpb] lattice words, word (row*W + w) of local chain l at (row*W+w)*cpb + l
//   [(N+1)*8] thresholds           (TAB_LDS)
//   [n_bins]  histogram            (lds_hist)
// Must be called by all 64 threads of the block (it synchronises).
template <int L, bool TAB_LDS>
__device__ __forceinline__ void sweep_tile_lds(const SizeDev &s, int c0, int cpb, int64_t M, void *trace,
                                               int32_t *hist, bool lds_hist, uint32_t *smem) {
    constexpr int W = (L + 31) / 32;
    constexpr int N = L * L;
    const int lane = threadIdx.x;
    const int c = c0 + lane;
    const bool active = lane < cpb && c < s.P;
    uint32_t *slat = smem;
    uint32_t *stab = smem + L * W * cpb;
    int32_t *shist = (int32_t *)(stab + (TAB_LDS ? (N + 1) * 8 : 0));
    const uint32_t *tab = TAB_LDS ? stab : s.tab;
    if (TAB_LDS)
        for (int i = lane; i < (N + 1) * 8; i += blockDim.x) stab[i] = s.tab[i];
    if (lds_hist)
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
        for (int64_t k = 0; k < M; ++k) {
            const uint32_t g = g0 + (uint32_t)k;
            Row<L> up = load(L - 1);
            Row<L> cur = load(0);
            Row<L> dn = load(1);
            for (int y = 0; y < L; ++y) {
                sweep_row<L>((uint32_t)y, g, (uint32_t)c + s.c_off, k0, k1, cur, up, dn, mi, tab);
                store(y, cur);
                up = cur;
                cur = dn;
                dn = load(y + 2 < L ? y + 2 : y + 2 - L);
            }
            const int m = mi >> 3;
            const int ev = m - N / 2;
            if (s.trace_bytes == 2)
                ((int16_t *)trace)[(size_t)c * s.tld + k] = (int16_t)ev;
            else
                ((int32_t *)trace)[(size_t)c * s.tld + k] = ev;
            if (lds_hist)
                atomicAdd(&shist[m >> s.bin_shift], 1);
            else
                atomicAdd(&hist[m >> s.bin_shift], 1);
        }
        s.lev[c] = mi >> 3;
    }
    __syncthreads();
    if (active)
        for (int w = 0; w < L * W; ++w) s.lat[(size_t)w * s.P + c] = slat[w * cpb + lane];
    if (lds_hist)
        for (int i = lane; i < s.n_bins; i += blockDim.x)
            if (shist[i]) atomicAdd(&hist[i], shist[i]);
    __syncthreads();
}

template <int L, bool TAB_LDS>
__global__ __launch_bounds__(64) void k_sweep_lds(SweepParams p) {
    extern __shared__ __align__(16) uint32_t smem[];
    sweep_tile_lds<L, TAB_LDS>(p.s, blockIdx.x * p.cpb, p.cpb, p.M, p.trace, p.hist, p.lds_hist != 0, smem);
}

// ---------------------------------------------------------------------------
// Producer/consumer sweeps (L <= 64).  A chain's attempts are strictly serial,
// so a chain advances at most one instruction of its wave per issue slot; the
// random words, which do not depend on the chain, are therefore generated by
// the other waves of the workgroup (on other SIMDs) into an LDS double buffer,
// R rows of every chain at a time, while the first wave consumes the previous
// R rows.  The waves meet at one barrier per chunk.
//
// LDS layout (bytes, 16-aligned parts):
//   [L*W*cpb u32]            lattice words, word (row*W + w) of chain l at (row*W+w)*cpb + l
//   [(N+1)*5 u32]            thresholds, entry a of level m at 5m + a
//   [n_bins i32]             histogram
//   [64 uint4]               site-pair table (pair_table)
//   [2][R][L/4][cpb] uint4   random words, group q of row r of chain l
// ---------------------------------------------------------------------------
__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Bytes per level of the LDS threshold table.
constexpr int kLevelBytes = 20;

struct PcLayout {
    size_t lat, tab, hist, pair, ubuf, total;
};

__host__ __device__ inline PcLayout pc_layout(int L, int W, int N, int n_bins, int cpb, int R) {
    PcLayout o;
    o.lat = 0;
    o.tab = align16((size_t)L * W * cpb * 4);
    o.hist = o.tab + align16((size_t)(N + 1) * kLevelBytes);
    o.pair = o.hist + align16((size_t)n_bins * 4);
    o.ubuf = o.pair + 64 * 16;
    o.total = o.ubuf + (size_t)2 * R * (L / 4) * cpb * 16;
    return o;
}

typedef __attribute__((address_space(3))) const uint32_t lds_u32;

// Read a 32-bit word at a byte address of LDS.
__device__ __forceinline__ uint32_t lds_load(uint32_t addr) { return *(lds_u32 *)(size_t)addr; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const u32x4 lds_u32x4;

// Read 16 bytes at a (16-aligned) byte address of LDS.
__device__ __forceinline__ uint4 lds_load128(uint32_t addr) {
    const u32x4 v = *(lds_u32x4 *)(size_t)addr;
    return make_uint4(v.x, v.y, v.z, v.w);
}

typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef __attribute__((address_space(3))) const u32x3 lds_u32x3;

// Read the first 12 bytes of a 16-byte table entry (a narrower read, so that no
// register of the result is dead while the read is in flight).
__device__ __forceinline__ uint4 lds_load96(uint32_t addr) {
    const u32x3 v = *(lds_u32x3 *)(size_t)addr;
    return make_uint4(v.x, v.y, v.z, 0u);
}

// Signed byte k of w.
__device__ __forceinline__ int32_t sbyte(uint32_t w, int k) { return (int32_t)(w << (24 - 8 * k)) >> 24; }

// Site-pair table.  The consumer decides sites x and x+1 (x even) together.
// With q = (up bond) + (down bond) + (right bond) broken at row start and h the
// left bond at row start, site x has anti = q_x + (h_x ^ a) anti-aligned
// neighbours, a = 1 iff its left neighbour x-1 flipped just before, and site
// x+1 has an0 = q_{x+1} + h_{x+1} or an1 = q_{x+1} + (h_{x+1} ^ 1) after x was
// rejected or accepted.  Entry i, for i = P0_x | P0_{x+1} << 1 | P1_x << 2 |
// P1_{x+1} << 3 | h_x << 4 | h_{x+1} << 5 (q = P0 + 2 P1), holds as signed bytes
// the byte offsets, from the threshold address of the current level (entry
// a = 4 of that level), of
//   .x = { threshold of x+1 if x rejected, 0, 0, level move if only x+1 accepted }
//   .y = { threshold of x, threshold of x+1 if x accepted, level move if only x
//          accepted, level move if both accepted }  for a = 0
//   .z = the same for a = 1.
__device__ void build_pair_table(uint4 *tbl, int tid, int nthreads) {
    auto pack = [](int b0, int b1, int b2, int b3) {
        return (uint32_t)(b0 & 255) | ((uint32_t)(b1 & 255) << 8) | ((uint32_t)(b2 & 255) << 16) |
               ((uint32_t)(b3 & 255) << 24);
    };
    for (int i = tid; i < 64; i += nthreads) {
        const int qx = (i & 1) + 2 * ((i >> 2) & 1);
        const int qx1 = ((i >> 1) & 1) + 2 * ((i >> 3) & 1);
        const int hx = (i >> 4) & 1, hx1 = (i >> 5) & 1;
        const int an0 = qx1 + hx1, an1 = qx1 + (hx1 ^ 1);
        uint32_t v[2];
        for (int a = 0; a < 2; ++a) {
            const int ax = qx + (hx ^ a);
            const int dx = kLevelBytes * (2 - ax);
            v[a] = pack(-4 * ax, dx - 4 * an1, dx, dx + kLevelBytes * (2 - an1));
        }
        tbl[i] = make_uint4(pack(-4 * an0, 0, 0, kLevelBytes * (2 - an0)), v[0], v[1], 0u);
    }
}

// The same table for the quad-speculative consumer, with bytes 1 and 2 of .y
// and .z swapped:
//   .y / .z = { threshold of x, level move if only x accepted, threshold of
//               x+1 if x accepted, level move if both accepted },
// so that all three level moves sit at odd bytes (1 and 3 of .y / .z, 3 of
// .x) and a lane picks the move of its assumed outcome, sign-extended, with
// one byte permute (v_perm_b32 sign codes exist for bytes 1, 3, 5, 7 only).
__device__ void build_pair_table_q(uint4 *tbl, int tid, int nthreads) {
    auto pack = [](int b0, int b1, int b2, int b3) {
        return (uint32_t)(b0 & 255) | ((uint32_t)(b1 & 255) << 8) | ((uint32_t)(b2 & 255) << 16) |
               ((uint32_t)(b3 & 255) << 24);
    };
    for (int i = tid; i < 64; i += nthreads) {
        const int qx = (i & 1) + 2 * ((i >> 2) & 1);
        const int qx1 = ((i >> 1) & 1) + 2 * ((i >> 3) & 1);
        const int hx = (i >> 4) & 1, hx1 = (i >> 5) & 1;
        const int an0 = qx1 + hx1, an1 = qx1 + (hx1 ^ 1);
        uint32_t v[2];
        for (int a = 0; a < 2; ++a) {
            const int ax = qx + (hx ^ a);
            const int dx = kLevelBytes * (2 - ax);
            v[a] = pack(-4 * ax, dx, dx - 4 * an1, dx + kLevelBytes * (2 - an1));
        }
        tbl[i] = make_uint4(pack(-4 * an0, 0, 0, kLevelBytes * (2 - an0)), v[0], v[1], 0u);
    }
}

// v_perm_b32 selectors over {.x (bytes 4-7), V = .y or .z (bytes 0-3)} of a
// build_pair_table_q entry giving, sign-extended, the level move of pair
// outcome j = (x accepted) + 2 (x+1 accepted): 0; byte 1 of V; byte 3 of .x
// (byte 7); byte 3 of V.  Codes 8, 9, 11 repeat the sign bit of bytes 1, 3, 7;
// code 12 gives a zero byte.
__device__ __forceinline__ uint32_t quad_move_selector(uint32_t j) {
    return j == 0 ? 0x0C0C0C0Cu : j == 1 ? 0x08080801u : j == 2 ? 0x0B0B0B07u : 0x09090903u;
}

// One row of the consumer, two sites at a time.  mib is the LDS byte address of
// entry a = 4 of the current level of the threshold table, so the threshold of
// a flip with `anti` anti-aligned neighbours is at mib - 4 anti and an accepted
// flip moves mib by kLevelBytes (2 - anti).  The three thresholds a pair can
// need are read at once from the level at the start of the pair; the two
// decisions then only select.
template <int L>
__device__ __forceinline__ void pc_row(Row<L> &cur, const Row<L> &up, const Row<L> &dn, uint32_t &mib,
                                       uint32_t pair_addr, const uint4 *urow, int cpb) {
    constexpr int W = (L + 31) / 32;
    constexpr int wl = (L - 1) >> 5, bl = (L - 1) & 31;
    Row<L> xu, xd, hb, P0, P1, hs, fl;
    const Row<L> nx = ring_next<L>(cur);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        xu.w[w] = cur.w[w] ^ up.w[w];
        xd.w[w] = cur.w[w] ^ dn.w[w];
        hb.w[w] = cur.w[w] ^ nx.w[w];
        P0.w[w] = __builtin_amdgcn_bitop3_b32(xu.w[w], xd.w[w], hb.w[w], 0x96);  // parity
        P1.w[w] = __builtin_amdgcn_bitop3_b32(xu.w[w], xd.w[w], hb.w[w], 0xE8);  // majority
        fl.w[w] = 0u;
    }
    // hs: bit x is the left bond of site x, i.e. bond (x-1, x), cyclically
#pragma unroll
    for (int w = 0; w < W; ++w) hs.w[w] = (hb.w[w] << 1) | (w > 0 ? hb.w[w - 1] >> 31 : 0u);
    hs.w[0] |= (hb.w[wl] >> bl) & 1u;
    auto entry = [&](int p) {
        const int w = (2 * p) >> 5, b = (2 * p) & 31;
        const uint32_t idx =
            ((P0.w[w] >> b) & 3u) | (((P1.w[w] >> b) & 3u) << 2) | (((hs.w[w] >> b) & 3u) << 4);
        return lds_load128(pair_addr + idx * 16u);
    };
    bool aprev = false;
    uint4 u4 = make_uint4(0, 0, 0, 0);
    uint4 en = entry(0);
#pragma unroll
    for (int p = 0; p < L / 2; ++p) {
        const int x = 2 * p, w = x >> 5, b = x & 31;
        if (p == 1) {
            // the right neighbour of site L-1 is site 0, decided in the first pair
            const uint32_t hl = hb.w[wl] ^ ((fl.w[0] & 1u) << bl);
            P0.w[wl] = __builtin_amdgcn_bitop3_b32(xu.w[wl], xd.w[wl], hl, 0x96);
            P1.w[wl] = __builtin_amdgcn_bitop3_b32(xu.w[wl], xd.w[wl], hl, 0xE8);
        }
        // entries are read one pair ahead; with two pairs per row the last one
        // is read again after the fix above
        const uint4 e = (L / 2 == 2 && p == 1) ? entry(1) : en;
        if (p + 1 < L / 2) en = entry(p + 1);
        if ((p & 1) == 0) u4 = urow[(p >> 1) * cpb];
        const uint32_t ux = (p & 1) ? u4.z : u4.x;
        const uint32_t ux1 = (p & 1) ? u4.w : u4.y;
        const uint32_t V = aprev ? e.z : e.y;
        const uint32_t tx = lds_load(mib + sbyte(V, 0));
        const uint32_t t0 = lds_load(mib + sbyte(e.x, 0));
        const uint32_t t1 = lds_load(mib + sbyte(V, 1));
        const uint32_t m10 = mib + sbyte(V, 2), m11 = mib + sbyte(V, 3), m01 = mib + sbyte(e.x, 3);
        const bool ax = ux <= tx;
        const uint32_t tn = ax ? t1 : t0;
        const uint32_t mA = ax ? m11 : m01, mB = ax ? m10 : mib;
        const bool ax1 = ux1 <= tn;
        mib = ax1 ? mA : mB;
        fl.w[w] |= (ax ? 1u << b : 0u) | (ax1 ? 2u << b : 0u);
        aprev = ax1;
    }
#pragma unroll
    for (int w = 0; w < W; ++w) cur.w[w] ^= fl.w[w];
}

// Random words of one chunk: rows y0 .. y0+R-1 of sweep g for every chain of
// the block, item it = rq * cpb + l (word group rq of the chunk, chain l; the
// words are those of global chain cg0 + l).
// Producer thread pt of np takes items pt, pt + np, ..., two independent
// Philox calls at a time; lanes whose chain is beyond P write words that are
// never read.
template <int L>
__device__ __forceinline__ void pc_produce(uint4 *ub, int R, uint32_t y0, uint32_t g, uint32_t cg0, int cpb,
                                           uint32_t k0, uint32_t k1, int pt, int np) {
    constexpr int NQ = L / 4;
    const int items = R * NQ * cpb;
    const int dl = np % cpb, drq = np / cpb;
    int l = pt % cpb, rq = pt / cpb;
    const uint32_t ctr0 = y0 * (uint32_t)NQ;
    auto step = [&](int &ll, int &rr) {
        ll += dl;
        rr += drq;
        if (ll >= cpb) {
            ll -= cpb;
            ++rr;
        }
    };
    for (int it = pt; it < items; it += 2 * np) {
        int l1 = l, rq1 = rq;
        step(l1, rq1);
        const uint4 v0 = philox10(make_uint4(ctr0 + (uint32_t)rq, g, cg0 + (uint32_t)l, kDomSweep), k0, k1);
        const uint4 v1 = philox10(make_uint4(ctr0 + (uint32_t)rq1, g, cg0 + (uint32_t)l1, kDomSweep), k0, k1);
        ub[it] = v0;
        if (it + np < items) ub[it + np] = v1;
        l = l1;
        rq = rq1;
        step(l, rq);
    }
}

struct PcParams {
    SizeDev s;
    int64_t M;
    void *trace;
    int32_t *hist;
    int32_t cpb;
    int32_t R;
};

// Sweeps of chains c0 .. c0+cpb-1; wave 0 consumes, waves 1.. produce.
template <int L>
__device__ __forceinline__ void sweep_tile_pc(const SizeDev &s, int c0, int cpb, int R, int64_t M, void *trace,
                                              int32_t *hist, uint32_t *smem) {
    constexpr int W = (L + 31) / 32;
    constexpr int N = L * L;
    const PcLayout lay = pc_layout(L, W, N, s.n_bins, cpb, R);
    char *lds = (char *)smem;
    uint32_t *slat = (uint32_t *)(lds + lay.lat);
    uint32_t *stab = (uint32_t *)(lds + lay.tab);
    int32_t *shist = (int32_t *)(lds + lay.hist);
    uint4 *ptbl = (uint4 *)(lds + lay.pair);
    uint4 *ubuf = (uint4 *)(lds + lay.ubuf);
    const int chunk_words = R * (L / 4) * cpb;  // uint4 per buffer
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = c0 + lane;
    const bool consumer = wave == 0;
    const bool active = consumer && lane < cpb && c < s.P;
    const uint32_t k0 = s.seed, k1 = (uint32_t)L;
    const uint32_t g0 = s.ctl->g;
    for (int i = threadIdx.x; i < (N + 1) * 5; i += blockDim.x) {
        const int m = i / 5;
        stab[i] = s.tab[(size_t)m * 8 + (i - 5 * m)];
    }
    for (int i = threadIdx.x; i < s.n_bins; i += blockDim.x) shist[i] = 0;
    build_pair_table(ptbl, threadIdx.x, blockDim.x);
    if (active)
        for (int w = 0; w < L * W; ++w) slat[w * cpb + lane] = s.lat[(size_t)w * s.P + c];
    const int np = blockDim.x - 64, pt = threadIdx.x - 64;
    const int per_sweep = L / R;
    const int64_t n_chunks = M * per_sweep;
    if (!consumer) pc_produce<L>(ubuf, R, 0u, g0, (uint32_t)c0 + s.c_off, cpb, k0, k1, pt, np);
    __syncthreads();

    uint32_t mib = 0;
    Row<L> up, cur, dn;
    // absolute LDS byte address (dynamic LDS starts at address 0 of the workgroup's LDS)
    const uint32_t tab_addr = (uint32_t)(size_t)(lds_u32 *)(stab);
    const uint32_t pair_addr = (uint32_t)(size_t)(lds_u32 *)(ptbl);
    if (active) mib = tab_addr + (uint32_t)kLevelBytes * (uint32_t)s.lev[c] + 16u;
    for (int64_t i = 0; i < n_chunks; ++i) {
        const int64_t k = i / per_sweep;
        const int y0 = (int)(i - k * per_sweep) * R;
        if (active) {
            const uint4 *ub = ubuf + (size_t)(i & 1) * chunk_words;
            auto load = [&](int y) {
                Row<L> r;
#pragma unroll
                for (int w = 0; w < W; ++w) r.w[w] = slat[(y * W + w) * cpb + lane];
                return r;
            };
            if (y0 == 0) {
                up = load(L - 1);
                cur = load(0);
                dn = load(1);
            }
            for (int r = 0; r < R; ++r) {
                const int y = y0 + r;
                pc_row<L>(cur, up, dn, mib, pair_addr, ub + (size_t)r * (L / 4) * cpb + lane, cpb);
#pragma unroll
                for (int w = 0; w < W; ++w) slat[(y * W + w) * cpb + lane] = cur.w[w];
                up = cur;
                cur = dn;
                dn = load(y + 2 < L ? y + 2 : y + 2 - L);
            }
            if (y0 + R == L) {
                const int m = (int)((mib - tab_addr - 16u) / (uint32_t)kLevelBytes);
                const int ev = m - N / 2;
                if (s.trace_bytes == 2)
                    ((int16_t *)trace)[(size_t)c * s.tld + k] = (int16_t)ev;
                else
                    ((int32_t *)trace)[(size_t)c * s.tld + k] = ev;
                atomicAdd(&shist[m >> s.bin_shift], 1);
            }
        } else if (!consumer && i + 1 < n_chunks) {
            const int64_t k1s = (i + 1) / per_sweep;
            const int y1 = (int)(i + 1 - k1s * per_sweep) * R;
            pc_produce<L>(ubuf + (size_t)((i + 1) & 1) * chunk_words, R, (uint32_t)y1, g0 + (uint32_t)k1s, (uint32_t)c0 + s.c_off, cpb,
                          k0, k1, pt, np);
        }
        __syncthreads();
    }
    if (active) {
        s.lev[c] = (int)((mib - tab_addr - 16u) / (uint32_t)kLevelBytes);
        for (int w = 0; w < L * W; ++w) s.lat[(size_t)w * s.P + c] = slat[w * cpb + lane];
    }
    for (int i = threadIdx.x; i < s.n_bins; i += blockDim.x)
        if (shist[i]) atomicAdd(&hist[i], shist[i]);
    __syncthreads();
}

// 256 threads: one consumer wave and three producer waves.
constexpr int kPcThreads = 256;
// Chains per workgroup of the quad-speculative kernel (four lanes each).
constexpr int kPcqMaxChains = 16;

template <int L>
__global__ __launch_bounds__(kPcThreads) void k_sweep_pc(PcParams p) {
    extern __shared__ __align__(16) uint32_t smem[];
    sweep_tile_pc<L>(p.s, blockIdx.x * p.cpb, p.cpb, p.R, p.M, p.trace, p.hist, smem);
}

// ---------------------------------------------------------------------------
// Quad-speculative sweeps (8 <= L <= 64).  Each chain gets the four lanes of a
// DPP quad.  Per step the quad decides four sites, pairs p and p+1: every lane
// decides pair p from the chain's state and, at the same time, pair p+1 from
// the state pair p would leave under one of its four outcomes (lane j assumes
// site x accepted iff j & 1 and site x+1 accepted iff j & 2).  The six
// thresholds do not depend on each other's outcome, and the lane whose
// assumption was right hands its result to the quad.  Producer waves, tables
// and buffers are those of the producer/consumer kernel.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ uint32_t quad_bcast(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

// One row of the quad consumer (pair table of build_pair_table_q).  selh: the
// byte-permute selector of the level move of the lane's assumed outcome of
// pair p (quad_move_selector); hym: all ones in lanes that assume site x+1 of
// pair p accepted; jq: the lane's place in its quad; hf0 / hf1: its result
// flags (jq, its assumed outcome of pair p, in bits 28-29, plus bit 30 when
// pair p+1's first site is accepted), so that the word selected for the quad
// carries the step's four flips in bits 28-31.  TREAD selects where the six
// thresholds come from: 0, the level table (the sweeps); 1 and 2 exist for
// the step-timing probe only (k_quad_step_probe): 1 reads six words of the
// pair table instead, at addresses formed from the entries alone, and folds
// the state in afterwards; 2 reads nothing and makes the thresholds from the
// state with arithmetic.
template <int L, int TREAD = 0>
__device__ __forceinline__ void pcq_row(Row<L> &cur, const Row<L> &up, const Row<L> &dn, uint32_t &mib,
                                        uint32_t pair_addr, const uint4 *urow, int cpb, uint32_t selh, uint32_t hym,
                                        uint32_t jq, uint32_t hf0, uint32_t hf1) {
    static_assert(L >= 8 && L % 4 == 0, "two pairs per step, site 0 decided before the last step");
    constexpr int W = (L + 31) / 32;
    constexpr int wl = (L - 1) >> 5, bl = (L - 1) & 31;
    constexpr int NS = L / 4;  // steps of four sites
    Row<L> xu, xd, hb, P0, P1, hs, fl;
    const Row<L> nx = ring_next<L>(cur);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        xu.w[w] = cur.w[w] ^ up.w[w];
        xd.w[w] = cur.w[w] ^ dn.w[w];
        hb.w[w] = cur.w[w] ^ nx.w[w];
        P0.w[w] = __builtin_amdgcn_bitop3_b32(xu.w[w], xd.w[w], hb.w[w], 0x96);  // parity
        P1.w[w] = __builtin_amdgcn_bitop3_b32(xu.w[w], xd.w[w], hb.w[w], 0xE8);  // majority
        fl.w[w] = 0u;
    }
#pragma unroll
    for (int w = 0; w < W; ++w) hs.w[w] = (hb.w[w] << 1) | (w > 0 ? hb.w[w - 1] >> 31 : 0u);
    hs.w[0] |= (hb.w[wl] >> bl) & 1u;
    // The table addresses of the row's pairs, shared out over the quad: lane jq
    // holds those of pairs 4k + jq (k = 0 .. NK-1); a step takes the ones it
    // needs from their lanes with a DPP broadcast.
    constexpr int NK = (L / 2 + 3) / 4;
    uint32_t own[NK];
    auto addr_of = [&](int k) {
        const int w = (8 * k) >> 5;
        const uint32_t b = (uint32_t)((8 * k) & 31) + 2u * jq;
        const uint32_t idx = __builtin_amdgcn_ubfe(P0.w[w], b, 2) | (__builtin_amdgcn_ubfe(P1.w[w], b, 2) << 2) |
                             (__builtin_amdgcn_ubfe(hs.w[w], b, 2) << 4);
        return pair_addr + idx * 16u;
    };
#pragma unroll
    for (int k = 0; k < NK; ++k) own[k] = addr_of(k);
    auto entry = [&](int p) {
        const uint32_t v = own[p >> 2];
        const uint32_t a = (p & 3) == 0 ? quad_bcast<0x00>(v) : (p & 3) == 1 ? quad_bcast<0x55>(v)
                         : (p & 3) == 2 ? quad_bcast<0xAA>(v) : quad_bcast<0xFF>(v);
        return lds_load96(a);
    };
    bool aprev = false;
    uint4 n0 = entry(0), n1 = entry(1);
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        const int p = 2 * st, x = 4 * st, w = x >> 5, b = x & 31;
        if (st == 1) {
            // the right neighbour of site L-1 is site 0, decided in the first step
            const uint32_t hl = hb.w[wl] ^ ((fl.w[0] & 1u) << bl);
            P0.w[wl] = __builtin_amdgcn_bitop3_b32(xu.w[wl], xd.w[wl], hl, 0x96);
            P1.w[wl] = __builtin_amdgcn_bitop3_b32(xu.w[wl], xd.w[wl], hl, 0xE8);
            own[(L / 2 - 1) >> 2] = addr_of((L / 2 - 1) >> 2);
        }
        const uint4 ea = n0;
        // with two steps per row the last pair's entry is read after the fix above
        const uint4 eb = (NS == 2 && st == 1) ? entry(3) : n1;
        if (st + 1 < NS) {
            n0 = entry(p + 2);
            n1 = entry(p + 3);
        }
        const uint4 u4 = urow[st * cpb];
        // pair p from the chain's state
        const uint32_t V = aprev ? ea.z : ea.y;
        // pair p+1 from the state left by the assumed outcome of pair p: the
        // level move is byte 3 of V (both accepted), byte 3 of ea.x (only x+1),
        // byte 1 of V (only x) or 0, picked by the lane's selector
        const uint32_t mh = mib + __builtin_amdgcn_perm(ea.x, V, selh);
        const uint32_t Vq = (eb.z & hym) | (eb.y & ~hym);
        uint32_t tx, t0, t1, qx, q0, q1;
        if constexpr (TREAD == 0) {
            tx = lds_load(mib + sbyte(V, 0));
            t0 = lds_load(mib + sbyte(ea.x, 0));
            t1 = lds_load(mib + sbyte(V, 2));
            qx = lds_load(mh + sbyte(Vq, 0));
            q0 = lds_load(mh + sbyte(eb.x, 0));
            q1 = lds_load(mh + sbyte(Vq, 2));
        } else if constexpr (TREAD == 1) {
            tx = lds_load(pair_addr + 64 + sbyte(V, 0)) ^ mib;
            t0 = lds_load(pair_addr + 128 + sbyte(ea.x, 0)) ^ mib;
            t1 = lds_load(pair_addr + 192 + sbyte(V, 2)) ^ mib;
            qx = lds_load(pair_addr + 256 + sbyte(Vq, 0)) ^ mh;
            q0 = lds_load(pair_addr + 320 + sbyte(eb.x, 0)) ^ mh;
            q1 = lds_load(pair_addr + 384 + sbyte(Vq, 2)) ^ mh;
        } else {
            tx = mib * 0x9E3779B9u;
            t0 = tx ^ 0x55555555u;
            t1 = tx ^ 0x33333333u;
            qx = mh * 0x9E3779B9u;
            q0 = qx ^ 0x55555555u;
            q1 = qx ^ 0x33333333u;
        }
        const bool bx = u4.z <= qx;
        const uint32_t qn = bx ? q1 : q0;
        const uint32_t nA = mh + (uint32_t)(bx ? sbyte(Vq, 3) : sbyte(eb.x, 3));
        const uint32_t nB = mh + (uint32_t)(bx ? sbyte(Vq, 1) : 0);
        const bool bx1 = u4.w <= qn;
        // result of the assumption: next state, the assumed outcome of pair p
        // in bits 28-29 and the two decisions of pair p+1 in bits 30, 31
        const uint32_t res = (bx1 ? nA : nB) | (bx ? hf1 : hf0) | (bx1 ? 1u << 31 : 0u);
        const uint32_t r0 = quad_bcast<0x00>(res), r1 = quad_bcast<0x55>(res);
        const uint32_t r2 = quad_bcast<0xAA>(res), r3 = quad_bcast<0xFF>(res);
        const bool ax = u4.x <= tx;
        const uint32_t tn = ax ? t1 : t0;
        const uint32_t rA = ax ? r3 : r2, rB = ax ? r1 : r0;
        const bool ax1 = u4.y <= tn;
        const uint32_t sel = ax1 ? rA : rB;
        // the selected lane assumed the true outcome: bits 28-31 are the step's four flips
        mib = sel & 0x0FFFFFFFu;
        fl.w[w] |= (sel >> 28) << b;
        aprev = (sel >> 31) != 0u;
    }
#pragma unroll
    for (int w = 0; w < W; ++w) cur.w[w] ^= fl.w[w];
}

// Sweeps of chains c0 .. c0+cpb-1 (cpb <= 16); the chain of consumer lane l is
// c0 + l/4.  Wave 0 consumes, waves 1.. produce.
template <int L>
__device__ __forceinline__ void sweep_tile_pcq(const SizeDev &s, int c0, int cpb, int R, int64_t M, void *trace,
                                               int32_t *hist, uint32_t *smem) {
    constexpr int W = (L + 31) / 32;
    constexpr int N = L * L;
    const PcLayout lay = pc_layout(L, W, N, s.n_bins, cpb, R);
    char *lds = (char *)smem;
    uint32_t *slat = (uint32_t *)(lds + lay.lat);
    uint32_t *stab = (uint32_t *)(lds + lay.tab);
    int32_t *shist = (int32_t *)(lds + lay.hist);
    uint4 *ptbl = (uint4 *)(lds + lay.pair);
    uint4 *ubuf = (uint4 *)(lds + lay.ubuf);
    const int chunk_words = R * (L / 4) * cpb;  // uint4 per buffer
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cl = lane >> 2, j = lane & 3;
    const int c = c0 + cl;
    const bool consumer = wave == 0;
    const bool active = consumer && cl < cpb && c < s.P;
    const bool lead = active && j == 0;  // one lane per chain for the global writes and atomics
    const uint32_t selh = quad_move_selector((uint32_t)j), hym = 0u - (uint32_t)((j >> 1) & 1);
    const uint32_t hf0 = (uint32_t)j << 28, hf1 = hf0 | (1u << 30);
    const uint32_t k0 = s.seed, k1 = (uint32_t)L;
    const uint32_t g0 = s.ctl->g;
    for (int i = threadIdx.x; i < (N + 1) * 5; i += blockDim.x) {
        const int m = i / 5;
        stab[i] = s.tab[(size_t)m * 8 + (i - 5 * m)];
    }
    for (int i = threadIdx.x; i < s.n_bins; i += blockDim.x) shist[i] = 0;
    build_pair_table_q(ptbl, threadIdx.x, blockDim.x);
    if (lead)
        for (int w = 0; w < L * W; ++w) slat[w * cpb + cl] = s.lat[(size_t)w * s.P + c];
    const int np = blockDim.x - 64, pt = threadIdx.x - 64;
    const int per_sweep = L / R;
    const int64_t n_chunks = M * per_sweep;
    if (!consumer) pc_produce<L>(ubuf, R, 0u, g0, (uint32_t)c0 + s.c_off, cpb, k0, k1, pt, np);
    __syncthreads();

    uint32_t mib = 0;
    Row<L> up, cur, dn;
    const uint32_t tab_addr = (uint32_t)(size_t)(lds_u32 *)(stab);
    const uint32_t pair_addr = (uint32_t)(size_t)(lds_u32 *)(ptbl);
    if (active) mib = tab_addr + (uint32_t)kLevelBytes * (uint32_t)s.lev[c] + 16u;
    for (int64_t i = 0; i < n_chunks; ++i) {
        const int64_t k = i / per_sweep;
        const int y0 = (int)(i - k * per_sweep) * R;
        if (active) {
            const uint4 *ub = ubuf + (size_t)(i & 1) * chunk_words;
            auto load = [&](int y) {
                Row<L> r;
#pragma unroll
                for (int w = 0; w < W; ++w) r.w[w] = slat[(y * W + w) * cpb + cl];
                return r;
            };
            if (y0 == 0) {
                up = load(L - 1);
                cur = load(0);
                dn = load(1);
            }
            for (int r = 0; r < R; ++r) {
                const int y = y0 + r;
                pcq_row<L>(cur, up, dn, mib, pair_addr, ub + (size_t)r * (L / 4) * cpb + cl, cpb, selh, hym,
                           (uint32_t)j, hf0, hf1);
                // the four lanes of the quad hold the same row
#pragma unroll
                for (int w = 0; w < W; ++w) slat[(y * W + w) * cpb + cl] = cur.w[w];
                up = cur;
                cur = dn;
                dn = load(y + 2 < L ? y + 2 : y + 2 - L);
            }
            if (y0 + R == L && lead) {
                const int m = (int)((mib - tab_addr - 16u) / (uint32_t)kLevelBytes);
                const int ev = m - N / 2;
                if (s.trace_bytes == 2)
                    ((int16_t *)trace)[(size_t)c * s.tld + k] = (int16_t)ev;
                else
                    ((int32_t *)trace)[(size_t)c * s.tld + k] = ev;
                atomicAdd(&shist[m >> s.bin_shift], 1);
            }
        } else if (!consumer && i + 1 < n_chunks) {
            const int64_t k1s = (i + 1) / per_sweep;
            const int y1 = (int)(i + 1 - k1s * per_sweep) * R;
            pc_produce<L>(ubuf + (size_t)((i + 1) & 1) * chunk_words, R, (uint32_t)y1, g0 + (uint32_t)k1s, (uint32_t)c0 + s.c_off, cpb,
                          k0, k1, pt, np);
        }
        __syncthreads();
    }
    if (lead) {
        s.lev[c] = (int)((mib - tab_addr - 16u) / (uint32_t)kLevelBytes);
        for (int w = 0; w < L * W; ++w) s.lat[(size_t)w * s.P + c] = slat[w * cpb + cl];
    }
    for (int i = threadIdx.x; i < s.n_bins; i += blockDim.x)
        if (shist[i]) atomicAdd(&hist[i], shist[i]);
    __syncthreads();
}

template <int L>
__global__ __launch_bounds__(kPcThreads) void k_sweep_pcq(PcParams p) {
    extern __shared__ __align__(16) uint32_t smem[];
    sweep_tile_pcq<L>(p.s, blockIdx.x * p.cpb, p.cpb, p.R, p.M, p.trace, p.hist, smem);
}

// ---------------------------------------------------------------------------
// Timing probe of the quad step (mc_probe kinds 9-11; a measurement, not a
// step of the method): one wave holding 16 chains of L = 32 with hashed spins,
// a level table of hashed thresholds (a flip that keeps the level is always
// accepted) and hashed random words, times `rows` rows of pcq_row with the
// shader clock, with nothing else on the compute unit: no producer waves, no
// barriers, no global memory.  The levels are those of the lattices, tracked
// exactly, so every table read stays inside the table.  out[c] receives chain
// c's final level, *cyc the cycles of the timed rows.
// ---------------------------------------------------------------------------
constexpr int kProbeL = 32, kProbeChains = 16, kProbeR = 8;

__host__ __device__ inline PcLayout quad_probe_layout() {
    return pc_layout(kProbeL, 1, kProbeL * kProbeL, kProbeL * kProbeL / 2 + 1, kProbeChains, kProbeR);
}

__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

template <int TREAD>
__global__ __launch_bounds__(64) void k_quad_step_probe(int rows, int64_t *cyc, uint32_t *out) {
    constexpr int L = kProbeL, N = L * L, cpb = kProbeChains, R = kProbeR;
    extern __shared__ __align__(16) uint32_t smem[];
    const PcLayout lay = quad_probe_layout();
    char *lds = (char *)smem;
    uint32_t *slat = (uint32_t *)(lds + lay.lat);
    uint32_t *stab = (uint32_t *)(lds + lay.tab);
    uint4 *ptbl = (uint4 *)(lds + lay.pair);
    uint4 *ubuf = (uint4 *)(lds + lay.ubuf);
    const int lane = (int)threadIdx.x, cl = lane >> 2, j = lane & 3;
    for (int i = lane; i < (N + 1) * 5; i += 64) stab[i] = i % 5 == 2 ? 0xFFFFFFFFu : probe_hash(77u * i + 1u);
    build_pair_table_q(ptbl, lane, 64);
    for (int i = lane; i < R * (L / 4) * cpb * 4; i += 64) ((uint32_t *)ubuf)[i] = probe_hash((uint32_t)i + 12345u);
    for (int i = lane; i < L * cpb; i += 64) slat[i] = probe_hash(0x51EDu + (uint32_t)i);
    __syncthreads();
    // level = half the broken bonds (right and down neighbours, periodic)
    uint32_t broken = 0;
    for (int y = 0; y < L; ++y) {
        const uint32_t r = slat[y * cpb + cl], d = slat[((y + 1) % L) * cpb + cl];
        broken += __popc(r ^ ((r >> 1) | (r << 31))) + __popc(r ^ d);
    }
    const uint32_t selh = quad_move_selector((uint32_t)j), hym = 0u - (uint32_t)((j >> 1) & 1);
    const uint32_t hf0 = (uint32_t)j << 28, hf1 = hf0 | (1u << 30);
    const uint32_t tab_addr = (uint32_t)(size_t)(lds_u32 *)(stab);
    const uint32_t pair_addr = (uint32_t)(size_t)(lds_u32 *)(ptbl);
    uint32_t mib = tab_addr + (uint32_t)kLevelBytes * (broken / 2) + 16u;
    Row<L> up, cur, dn;
    up.w[0] = slat[(L - 1) * cpb + cl];
    cur.w[0] = slat[cl];
    dn.w[0] = slat[cpb + cl];
    const long long t0 = clock64();
    for (int r = 0; r < rows; ++r) {
        const int y = r % L;
        pcq_row<L, TREAD>(cur, up, dn, mib, pair_addr, ubuf + (size_t)(r % R) * (L / 4) * cpb + cl, cpb, selh, hym,
                          (uint32_t)j, hf0, hf1);
        slat[y * cpb + cl] = cur.w[0];  // the four lanes of the quad hold the same row
        up = cur;
        cur = dn;
        dn.w[0] = slat[((y + 2) % L) * cpb + cl];
    }
    const long long t1 = clock64();
    if (lane == 0) *cyc = t1 - t0;
    if (j == 0) out[cl] = (mib - tab_addr - 16u) / (uint32_t)kLevelBytes;
}

hipError_t launch_quad_step_probe(int mode, int rows, int64_t *cyc, uint32_t *out, hipStream_t st) {
    const size_t bytes = quad_probe_layout().total;
    if (mode == 0)
        hipLaunchKernelGGL(k_quad_step_probe<0>, dim3(1), dim3(64), bytes, st, rows, cyc, out);
    else if (mode == 1)
        hipLaunchKernelGGL(k_quad_step_probe<1>, dim3(1), dim3(64), bytes, st, rows, cyc, out);
    else
        hipLaunchKernelGGL(k_quad_step_probe<2>, dim3(1), dim3(64), bytes, st, rows, cyc, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Large lattices (L = 128, 256): the producer/consumer scheme with each row
// streamed from global memory one 32-bit word at a time (the next word is read
// while the current one is swept) and the thresholds in the compact per-bin
// table, held in LDS when it fits (TAB_LDS) and read from global memory
// otherwise.
//
// LDS layout (bytes):
//   [n_bins*(2r+1) u32]      compact thresholds (TAB_LDS)
//   [64 uint4]               site-pair table in level units (pair_levels)
//   [2][R][L/4][cpb] uint4   random words, as for the producer/consumer kernel
// ---------------------------------------------------------------------------
struct BigLayout {
    size_t tab, pair, ubuf, total;
};

__host__ __device__ inline BigLayout big_layout(int L, int n_bins, int r, int cpb, int R, bool tab_lds) {
    BigLayout o;
    o.tab = 0;
    o.pair = tab_lds ? align16((size_t)n_bins * (2 * r + 1) * 4) : 0;
    o.ubuf = o.pair + 128 * 16;  // room for build_pair_parity_q (128 uint4); the others use 64
    o.total = o.ubuf + (size_t)2 * R * (L / 4) * cpb * 16;
    return o;
}

// The site-pair table of pair_table with level changes instead of byte
// offsets: for d = 2 - anti (the level change of a flip),
//   .x = { d of x+1 if x rejected }
//   .y = { d of x, (d of x) + (d of x+1 if x accepted) }  for a = 0
//   .z = the same for a = 1.
__device__ void build_pair_levels(uint4 *tbl, int tid, int nthreads) {
    auto pack = [](int b0, int b1) { return (uint32_t)(b0 & 255) | ((uint32_t)(b1 & 255) << 8); };
    for (int i = tid; i < 64; i += nthreads) {
        const int qx = (i & 1) + 2 * ((i >> 2) & 1);
        const int qx1 = ((i >> 1) & 1) + 2 * ((i >> 3) & 1);
        const int hx = (i >> 4) & 1, hx1 = (i >> 5) & 1;
        const int d0 = 2 - (qx1 + hx1), d1 = 2 - (qx1 + (hx1 ^ 1));
        uint32_t v[2];
        for (int a = 0; a < 2; ++a) {
            const int dx = 2 - (qx + (hx ^ a));
            v[a] = pack(dx, dx + d1);
        }
        tbl[i] = make_uint4(pack(d0, 0), v[0], v[1], 0u);
    }
}

// Thresholds of the compact table at a byte offset: from LDS (the offset is an
// absolute LDS address) or from global memory (relative to tabc).
template <bool TAB_LDS>
__device__ __forceinline__ uint32_t big_threshold(const uint32_t *tabc, uint32_t off) {
    if (TAB_LDS) return lds_load(off);
    return *(const uint32_t *)((const char *)tabc + off);
}

// One row of a large lattice.  State: m, the level, and Bm = B0 + 8 r (m >> bs),
// the byte offset of bin m >> bs in the compact table plus 4 r, so that the
// threshold of a move to level m' is at Bm + 4 (m' >> bs).
template <int L, bool TAB_LDS>
__device__ __forceinline__ void big_row(uint32_t *lat, size_t P, int c, int y, int &m, uint32_t &Bm, int bs,
                                        uint32_t B0, int sB, const uint32_t *tabc, uint32_t pair_addr,
                                        const uint4 *urow, int cpb) {
    constexpr int W = L / 32;
    const int yu = y == 0 ? L - 1 : y - 1, yd = y + 1 == L ? 0 : y + 1;
    auto word = [&](int yy, int w) { return lat + (size_t)(yy * W + w) * P + c; };
    uint32_t cn = *word(y, 0), un = *word(yu, 0), dn = *word(yd, 0), cnn = *word(y, 1);
    // bond (L-1, 0) at row start: the left bond of site 0
    uint32_t carry = ((*word(y, W - 1) >> 31) ^ cn) & 1u;
    uint32_t c0new = 0u;
    bool aprev = false;
    for (int w = 0; w < W; ++w) {
        const uint32_t cw = cn, uw = un, dw = dn;
        // right neighbours of the word; for the last word bit 31 is site 0 as
        // it is now (it was decided at the start of the row)
        const uint32_t cw1 = w + 1 < W ? cnn : c0new;
        if (w + 1 < W) {
            cn = cnn;
            un = *word(yu, w + 1);
            dn = *word(yd, w + 1);
            if (w + 2 < W) cnn = *word(y, w + 2);
        }
        const uint32_t xu = cw ^ uw, xd = cw ^ dw, hb = cw ^ ((cw >> 1) | (cw1 << 31));
        const uint32_t P0 = __builtin_amdgcn_bitop3_b32(xu, xd, hb, 0x96);
        const uint32_t P1 = __builtin_amdgcn_bitop3_b32(xu, xd, hb, 0xE8);
        const uint32_t hs = (hb << 1) | carry;  // left bonds
        carry = hb >> 31;
        const uint4 *uw4 = urow + (size_t)w * 8 * cpb;
        auto entry = [&](int p) {
            const uint32_t idx = ((P0 >> (2 * p)) & 3u) | (((P1 >> (2 * p)) & 3u) << 2) | (((hs >> (2 * p)) & 3u) << 4);
            return lds_load128(pair_addr + idx * 16u);
        };
        uint32_t fw = 0u;
        uint4 u4 = make_uint4(0, 0, 0, 0);
        uint4 en = entry(0);
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            const uint4 e = en;
            if (p + 1 < 16) en = entry(p + 1);
            if ((p & 1) == 0) u4 = uw4[(p >> 1) * cpb];
            const uint32_t ux = (p & 1) ? u4.z : u4.x;
            const uint32_t ux1 = (p & 1) ? u4.w : u4.y;
            const uint32_t V = aprev ? e.z : e.y;
            const int mx = m + sbyte(V, 0), m0 = m + sbyte(e.x, 0), m11 = m + sbyte(V, 1);
            const uint32_t bx = (uint32_t)(mx >> bs), b0 = (uint32_t)(m0 >> bs), b11 = (uint32_t)(m11 >> bs);
            const uint32_t Bx = B0 + (bx << sB), Bb0 = B0 + (b0 << sB), B11 = B0 + (b11 << sB);
            const uint32_t tx = big_threshold<TAB_LDS>(tabc, Bm + 4u * bx);
            const uint32_t t0 = big_threshold<TAB_LDS>(tabc, Bm + 4u * b0);
            const uint32_t t1 = big_threshold<TAB_LDS>(tabc, Bx + 4u * b11);
            const bool ax = ux <= tx;
            const uint32_t tn = ax ? t1 : t0;
            const int mA = ax ? m11 : m0, mB = ax ? mx : m;
            const uint32_t BA = ax ? B11 : Bb0, BB = ax ? Bx : Bm;
            const bool ax1 = ux1 <= tn;
            m = ax1 ? mA : mB;
            Bm = ax1 ? BA : BB;
            fw |= (ax ? 1u << (2 * p) : 0u) | (ax1 ? 2u << (2 * p) : 0u);
            aprev = ax1;
        }
        const uint32_t cnew = cw ^ fw;
        *word(y, w) = cnew;
        if (w == 0) c0new = cnew;
    }
}

// Sweeps of chains c0 .. c0+cpb-1 of a large lattice; wave 0 consumes, the
// other waves produce random words.
template <int L, bool TAB_LDS>
__device__ __forceinline__ void sweep_tile_big(const SizeDev &s, int c0, int cpb, int R, int64_t M, void *trace,
                                               int32_t *hist, uint32_t *smem) {
    constexpr int N = L * L;
    const int r = s.tab_r, K = 2 * r + 1;
    const BigLayout lay = big_layout(L, s.n_bins, r, cpb, R, TAB_LDS);
    char *lds = (char *)smem;
    uint32_t *stab = (uint32_t *)(lds + lay.tab);
    uint4 *ptbl = (uint4 *)(lds + lay.pair);
    uint4 *ubuf = (uint4 *)(lds + lay.ubuf);
    const int chunk_words = R * (L / 4) * cpb;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = c0 + lane;
    const bool consumer = wave == 0;
    const bool active = consumer && lane < cpb && c < s.P;
    const uint32_t k0 = s.seed, k1 = (uint32_t)L;
    const uint32_t g0 = s.ctl->g;
    if (TAB_LDS)
        for (int i = threadIdx.x; i < s.n_bins * K; i += blockDim.x) stab[i] = s.tabc[i];
    build_pair_levels(ptbl, threadIdx.x, blockDim.x);
    const int np = blockDim.x - 64, pt = threadIdx.x - 64;
    const int per_sweep = L / R;
    const int64_t n_chunks = M * per_sweep;
    if (!consumer) pc_produce<L>(ubuf, R, 0u, g0, (uint32_t)c0 + s.c_off, cpb, k0, k1, pt, np);
    __syncthreads();

    const uint32_t B0 = (TAB_LDS ? (uint32_t)(size_t)(lds_u32 *)(stab) : 0u) + 4u * (uint32_t)r;
    const int sB = r == 1 ? 3 : 4;  // log2(8 r)
    const int bs = s.bin_shift;
    const uint32_t pair_addr = (uint32_t)(size_t)(lds_u32 *)(ptbl);
    int m = 0;
    uint32_t Bm = 0u;
    if (active) {
        m = s.lev[c];
        Bm = B0 + ((uint32_t)(m >> bs) << sB);
    }
    for (int64_t i = 0; i < n_chunks; ++i) {
        const int64_t k = i / per_sweep;
        const int y0 = (int)(i - k * per_sweep) * R;
        if (active) {
            const uint4 *ub = ubuf + (size_t)(i & 1) * chunk_words;
            for (int rr = 0; rr < R; ++rr)
                big_row<L, TAB_LDS>(s.lat, (size_t)s.P, c, y0 + rr, m, Bm, bs, B0, sB, s.tabc, pair_addr,
                                    ub + (size_t)rr * (L / 4) * cpb + lane, cpb);
            if (y0 + R == L) {
                const int ev = m - N / 2;
                if (s.trace_bytes == 2)
                    ((int16_t *)trace)[(size_t)c * s.tld + k] = (int16_t)ev;
                else
                    ((int32_t *)trace)[(size_t)c * s.tld + k] = ev;
                atomicAdd(&hist[m >> bs], 1);
            }
        } else if (!consumer && i + 1 < n_chunks) {
            const int64_t k1s = (i + 1) / per_sweep;
            const int y1 = (int)(i + 1 - k1s * per_sweep) * R;
            pc_produce<L>(ubuf + (size_t)((i + 1) & 1) * chunk_words, R, (uint32_t)y1, g0 + (uint32_t)k1s, (uint32_t)c0 + s.c_off, cpb,
                          k0, k1, pt, np);
        }
        __syncthreads();
    }
    if (active) s.lev[c] = m;
}

template <int L, bool TAB_LDS>
__global__ __launch_bounds__(kPcThreads) void k_sweep_big(PcParams p) {
    extern __shared__ __align__(16) uint32_t smem[];
    sweep_tile_big<L, TAB_LDS>(p.s, blockIdx.x * p.cpb, p.cpb, p.R, p.M, p.trace, p.hist, smem);
}

// ---------------------------------------------------------------------------
// Quad-speculative sweeps of large lattices (L = 128, 256): the rows streamed
// as in k_sweep_big, each chain on the four lanes of a DPP quad deciding four
// sites per step as in k_sweep_pcq, the thresholds from the per-bin table.
// ---------------------------------------------------------------------------

// v_perm_b32 selectors for the signed level change of a pair whose outcome is
// k = (first site accepted) + 2 (second site accepted), from {S0 = .x,
// S1 = .y or .z} of a build_pair_levels_q entry: 0 (code 12 gives zero
// bytes), dx (byte 1 of S1), d0 (byte 1 of S0, i.e. byte 5), dx + d1 (byte 3
// of S1); codes 8, 10, 9 repeat the sign bits of bytes 1, 5, 3.
constexpr uint32_t kSelMove0 = 0x0C0C0C0Cu, kSelMove1 = 0x08080801u, kSelMove2 = 0x0A0A0A05u,
                   kSelMove3 = 0x09090903u;

__device__ __forceinline__ int pair_move(uint32_t ex, uint32_t v, uint32_t sel) {
    return (int)__builtin_amdgcn_perm(ex, v, sel);
}

// build_pair_levels with every level change at an odd byte:
//   .x = {0, d0, 0, 0},  .y / .z = {0, dx, 0, dx + d1} for a left neighbour
//   that did not / did flip
// (d = 2 - anti: d0 of site x+1 if x was rejected, dx of site x, d1 of x+1 if
// x was accepted).
__device__ void build_pair_levels_q(uint4 *tbl, int tid, int nthreads) {
    auto pack = [](int b1, int b3) { return ((uint32_t)(b1 & 255) << 8) | ((uint32_t)(b3 & 255) << 24); };
    for (int i = tid; i < 64; i += nthreads) {
        const int qx = (i & 1) + 2 * ((i >> 2) & 1);
        const int qx1 = ((i >> 1) & 1) + 2 * ((i >> 3) & 1);
        const int hx = (i >> 4) & 1, hx1 = (i >> 5) & 1;
        const int d0 = 2 - (qx1 + hx1), d1 = 2 - (qx1 + (hx1 ^ 1));
        uint32_t v[2];
        for (int a = 0; a < 2; ++a) {
            const int dx = 2 - (qx + (hx ^ a));
            v[a] = pack(dx, dx + d1);
        }
        tbl[i] = make_uint4(pack(d0, 0), v[0], v[1], 0u);
    }
}

// The three thresholds a pair can need from level m (entry e, left-neighbour
// variant V): site x, site x+1 after x was rejected, after x was accepted.
template <bool TAB_LDS>
__device__ __forceinline__ void bigq_thresholds(int m, uint32_t ex, uint32_t V, int bs, uint32_t B0, int sB,
                                                const uint32_t *tabc, uint32_t &tx, uint32_t &t0, uint32_t &t1) {
    const int mx = m + sbyte(V, 1), m0 = m + sbyte(ex, 1), m11 = m + sbyte(V, 3);
    const uint32_t Bm = B0 + ((uint32_t)(m >> bs) << sB), Bx = B0 + ((uint32_t)(mx >> bs) << sB);
    tx = big_threshold<TAB_LDS>(tabc, Bm + 4u * (uint32_t)(mx >> bs));
    t0 = big_threshold<TAB_LDS>(tabc, Bm + 4u * (uint32_t)(m0 >> bs));
    t1 = big_threshold<TAB_LDS>(tabc, Bx + 4u * (uint32_t)(m11 >> bs));
}

// One row of a large lattice on a chain's quad.  Lane j assumes outcome j of
// each step's first pair (bit 0: its first site accepted, bit 1: its second);
// hym is all ones when j & 2, sel_h selects its assumed level change, f0 / f1
// its result flags (j in bits 28-29, plus bit 30 when the second pair's first
// site is accepted).  The word a lane hands to its quad is {next level, the
// four decisions in bits 28-31}.  Every lane of the quad stores the row words
// it computed (the same values), so that each lane's later reads of them
// follow its own store.
template <int L, bool TAB_LDS>
__device__ __forceinline__ void bigq_row(uint32_t *lat, size_t P, int c, int y, int &m, int bs, uint32_t B0, int sB,
                                         const uint32_t *tabc, uint32_t pair_addr, const uint4 *urow, int cpb,
                                         uint32_t hym, uint32_t sel_h, uint32_t f0, uint32_t f1) {
    static_assert(L % 4 == 0 && L > 64, "steps of four sites; at least three words per row");
    constexpr int W = (L + 31) / 32;
    constexpr int NB = L - 32 * (W - 1);  // sites in the last word (32 unless L % 32 != 0)
    const int yu = y == 0 ? L - 1 : y - 1, yd = y + 1 == L ? 0 : y + 1;
    auto word = [&](int yy, int w) { return lat + (size_t)(yy * W + w) * P + c; };
    uint32_t cn = *word(y, 0), un = *word(yu, 0), dn = *word(yd, 0), cnn = *word(y, 1);
    // bond (L-1, 0) at row start: the left bond of site 0
    uint32_t carry = ((*word(y, W - 1) >> (NB - 1)) ^ cn) & 1u;
    uint32_t c0new = 0u;
    bool aprev = false;
    for (int w = 0; w < W; ++w) {
        const uint32_t cw = cn, uw = un, dw = dn;
        // right neighbours of the word; for the last word bit 31 is site 0 as
        // it is now (it was decided at the start of the row)
        const uint32_t cw1 = w + 1 < W ? cnn : c0new;
        if (w + 1 < W) {
            cn = cnn;
            un = *word(yu, w + 1);
            dn = *word(yd, w + 1);
            if (w + 2 < W) cnn = *word(y, w + 2);
        }
        // the right neighbour of the word's last site: bit 0 of the next word, or
        // for the last word (NB sites) site 0 of the row
        const int nb = w + 1 < W ? 32 : NB;
        const uint32_t xu = cw ^ uw, xd = cw ^ dw, hb = cw ^ ((cw >> 1) | ((cw1 & 1u) << (nb - 1)));
        const uint32_t P0 = __builtin_amdgcn_bitop3_b32(xu, xd, hb, 0x96);
        const uint32_t P1 = __builtin_amdgcn_bitop3_b32(xu, xd, hb, 0xE8);
        const uint32_t hs = (hb << 1) | carry;  // left bonds
        carry = (hb >> 31) & 1u;  // (a partial word is the last one: its carry is not used)
        const uint4 *uw4 = urow + (size_t)w * 8 * cpb;
        // (sharing these indices over the quad, as pcq_row does, was measured
        // slower here: 124 against 124 cycles at L = 128, 141 against 127 at 256)
        auto entry = [&](int p) {
            const uint32_t idx = ((P0 >> (2 * p)) & 3u) | (((P1 >> (2 * p)) & 3u) << 2) | (((hs >> (2 * p)) & 3u) << 4);
            return lds_load96(pair_addr + idx * 16u);
        };
        uint32_t fw = 0u;
        uint4 n0 = entry(0), n1 = entry(1);
        const int nst = nb / 4;  // steps of four sites in this word
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            if (st >= nst) break;
            const int p = 2 * st;
            const uint4 ea = n0, eb = n1;
            if (st + 1 < nst) {
                n0 = entry(p + 2);
                n1 = entry(p + 3);
            }
            const uint4 u4 = uw4[st * cpb];
            // pair p from the chain's state
            const uint32_t V = aprev ? ea.z : ea.y;
            uint32_t tx, t0, t1;
            bigq_thresholds<TAB_LDS>(m, ea.x, V, bs, B0, sB, tabc, tx, t0, t1);
            // pair p+1 from the state the assumed outcome of pair p leaves
            const int mh = m + pair_move(ea.x, V, sel_h);
            const uint32_t Vq = (eb.z & hym) | (eb.y & ~hym);
            uint32_t qx, q0, q1;
            bigq_thresholds<TAB_LDS>(mh, eb.x, Vq, bs, B0, sB, tabc, qx, q0, q1);
            const bool bx = u4.z <= qx;
            const uint32_t qn = bx ? q1 : q0;
            const uint32_t sA = bx ? kSelMove3 : kSelMove2, sB2 = bx ? kSelMove1 : kSelMove0;
            const bool bx1 = u4.w <= qn;
            const uint32_t nxt = (uint32_t)(mh + pair_move(eb.x, Vq, bx1 ? sA : sB2));
            const uint32_t res = nxt | (bx ? f1 : f0) | (bx1 ? 1u << 31 : 0u);
            const uint32_t r0 = quad_bcast<0x00>(res), r1 = quad_bcast<0x55>(res);
            const uint32_t r2 = quad_bcast<0xAA>(res), r3 = quad_bcast<0xFF>(res);
            const bool ax = u4.x <= tx;
            const uint32_t tn = ax ? t1 : t0;
            const uint32_t rA = ax ? r3 : r2, rB = ax ? r1 : r0;
            const bool ax1 = u4.y <= tn;
            const uint32_t sel = ax1 ? rA : rB;
            m = (int)(sel & 0x0FFFFFFFu);
            fw |= (sel >> 28) << (4 * st);
            aprev = (sel >> 31) != 0u;
        }
        const uint32_t cnew = cw ^ fw;
        *word(y, w) = cnew;
        if (w == 0) c0new = cnew;
    }
}

// ---- parity-state quad rows (bin_shift 1) ----------------------------------
// With two levels per bin, a flip's threshold and the state it leads to depend
// on the level only through its bin b and its parity p (m = 2b + p): a move by
// d (|d| <= 2) goes to bin b + floor((p + d)/2).  The state is therefore kept
// as S = B0 + 12 b + 2 p, the byte address of bin b's row {down, same, up} of
// the per-bin table plus twice the parity (bit 1 of S is p; rows are
// 4-aligned).  The threshold of a move by d from S is at
// S - 2p + 4 (floor((p + d)/2) + 1), and the move takes S to
// S + 12 floor((p + d)/2) + 2 ((p + d) & 1) - 2p: both are fixed offsets once
// p is known, so the site-pair table holds them for p = 0 and p = 1 and a step
// needs no bin arithmetic.

// Byte offset, from S, of the threshold of a move by d from a level of parity p.
__host__ __device__ constexpr int par_thr(int p, int d) {
    return 4 * (((p + d + 4) >> 1) - 2 + 1) - 2 * p;
}
// Change of S when a move by d from parity p is accepted.
__host__ __device__ constexpr int par_move(int p, int d) {
    return 12 * (((p + d + 4) >> 1) - 2) + 2 * ((p + d) & 1) - 2 * p;
}

// Site-pair table of the parity-state step: entry i (the index of
// build_pair_table) is 32 bytes, {X0, Y0, Z0, 0, X1, Y1, Z1, 0}: for a level
// of parity p, Xp = {threshold of x+1 if x rejected, 0, 0, move if only x+1
// accepted} and Yp / Zp (left neighbour x-1 not flipped / flipped) =
// {threshold of x, move if only x accepted, threshold of x+1 if x accepted,
// move if both accepted}, as signed byte offsets of S (the moves at odd bytes
// for quad_move_selector's byte permutes).
__device__ void build_pair_parity_q(uint4 *tbl, int tid, int nthreads) {
    auto pack = [](int b0, int b1, int b2, int b3) {
        return (uint32_t)(b0 & 255) | ((uint32_t)(b1 & 255) << 8) | ((uint32_t)(b2 & 255) << 16) |
               ((uint32_t)(b3 & 255) << 24);
    };
    for (int e = tid; e < 128; e += nthreads) {
        const int i = e >> 1, p = e & 1;
        const int qx = (i & 1) + 2 * ((i >> 2) & 1);
        const int qx1 = ((i >> 1) & 1) + 2 * ((i >> 3) & 1);
        const int hx = (i >> 4) & 1, hx1 = (i >> 5) & 1;
        const int d0 = 2 - (qx1 + hx1), d1 = 2 - (qx1 + (hx1 ^ 1));
        uint32_t v[2];
        for (int a = 0; a < 2; ++a) {
            const int dx = 2 - (qx + (hx ^ a));
            const int p1 = (p + dx) & 1;  // parity after x accepted
            const int mx = par_move(p, dx);
            v[a] = pack(par_thr(p, dx), mx, mx + par_thr(p1, d1), mx + par_move(p1, d1));
        }
        tbl[e] = make_uint4(pack(par_thr(p, d0), 0, 0, par_move(p, d0)), v[0], v[1], 0u);
    }
}

// One row of a large lattice on a chain's quad, in the parity state (bin_shift
// 1): the streamed words and quad exchange of bigq_row, with the thresholds
// and moves of each pair taken at fixed offsets of S from the variant of its
// entry for S's parity (the first pair of a step: the chain's parity; the
// second: the parity each lane's assumed outcome of the first leaves).
template <int L, bool TAB_LDS>
__device__ __forceinline__ void bigq_row_p(uint32_t *lat, size_t P, int c, int y, uint32_t &S,
                                           const uint32_t *tabc, uint32_t pair_addr, const uint4 *urow, int cpb,
                                           uint32_t hym, uint32_t sel_h, uint32_t f0, uint32_t f1, uint32_t jq) {
    static_assert(L % 4 == 0 && L > 64, "steps of four sites; at least three words per row");
    constexpr int W = (L + 31) / 32;
    constexpr int NB = L - 32 * (W - 1);
    const int yu = y == 0 ? L - 1 : y - 1, yd = y + 1 == L ? 0 : y + 1;
    auto word = [&](int yy, int w) { return lat + (size_t)(yy * W + w) * P + c; };
    auto thr = [&](uint32_t off) { return big_threshold<TAB_LDS>(tabc, off); };
    uint32_t cn = *word(y, 0), un = *word(yu, 0), dn = *word(yd, 0), cnn = *word(y, 1);
    uint32_t carry = ((*word(y, W - 1) >> (NB - 1)) ^ cn) & 1u;
    uint32_t c0new = 0u;
    bool aprev = false;
    for (int w = 0; w < W; ++w) {
        const uint32_t cw = cn, uw = un, dw = dn;
        const uint32_t cw1 = w + 1 < W ? cnn : c0new;
        if (w + 1 < W) {
            cn = cnn;
            un = *word(yu, w + 1);
            dn = *word(yd, w + 1);
            if (w + 2 < W) cnn = *word(y, w + 2);
        }
        const int nb = w + 1 < W ? 32 : NB;
        const uint32_t xu = cw ^ uw, xd = cw ^ dw, hb = cw ^ ((cw >> 1) | ((cw1 & 1u) << (nb - 1)));
        const uint32_t P0 = __builtin_amdgcn_bitop3_b32(xu, xd, hb, 0x96);
        const uint32_t P1 = __builtin_amdgcn_bitop3_b32(xu, xd, hb, 0xE8);
        const uint32_t hs = (hb << 1) | carry;
        carry = (hb >> 31) & 1u;
        const uint4 *uw4 = urow + (size_t)w * 8 * cpb;
        // the entry addresses of the word's 16 pairs, shared out over the
        // quad as in the L <= 64 kernel: lane jq forms those of pairs 4k + jq,
        // and a step takes the two it needs from their lanes with a DPP
        // broadcast (pairs past the word's last site are formed, never read)
        uint32_t own[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t bq = (uint32_t)(8 * k) + 2u * jq;
            const uint32_t idx = __builtin_amdgcn_ubfe(P0, bq, 2) | (__builtin_amdgcn_ubfe(P1, bq, 2) << 2) |
                                 (__builtin_amdgcn_ubfe(hs, bq, 2) << 4);
            own[k] = pair_addr + idx * 32u;
        }
        auto entry = [&](int p, uint4 &h0, uint4 &h1) {
            const uint32_t v = own[p >> 2];
            const uint32_t a = (p & 3) == 0 ? quad_bcast<0x00>(v) : (p & 3) == 1 ? quad_bcast<0x55>(v)
                             : (p & 3) == 2 ? quad_bcast<0xAA>(v) : quad_bcast<0xFF>(v);
            h0 = lds_load96(a);
            h1 = lds_load96(a + 16u);
        };
        uint32_t fw = 0u;
        uint4 n0a, n0b, n1a, n1b;
        entry(0, n0a, n0b);
        entry(1, n1a, n1b);
        const int nst = nb / 4;
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            if (st >= nst) break;
            const int p = 2 * st;
            const uint4 ea0 = n0a, ea1 = n0b, eb0 = n1a, eb1 = n1b;
            if (st + 1 < nst) {
                entry(p + 2, n0a, n0b);
                entry(p + 3, n1a, n1b);
            }
            const uint4 u4 = uw4[st * cpb];
            // the second pair's variants for this lane's assumed left neighbour
            const uint32_t Yq0 = (eb0.z & hym) | (eb0.y & ~hym), Yq1 = (eb1.z & hym) | (eb1.y & ~hym);
            // pair p from the chain's state
            const bool pb = (S & 2u) != 0u;
            const uint32_t ex = pb ? ea1.x : ea0.x;
            const uint32_t V = aprev ? (pb ? ea1.z : ea0.z) : (pb ? ea1.y : ea0.y);
            const uint32_t tx = thr(S + sbyte(V, 0));
            const uint32_t t0 = thr(S + sbyte(ex, 0));
            const uint32_t t1 = thr(S + sbyte(V, 2));
            // pair p+1 from the state the assumed outcome of pair p leaves
            const uint32_t mh = S + __builtin_amdgcn_perm(ex, V, sel_h);
            const bool ph = (mh & 2u) != 0u;
            const uint32_t exq = ph ? eb1.x : eb0.x;
            const uint32_t Vq = ph ? Yq1 : Yq0;
            const uint32_t qx = thr(mh + sbyte(Vq, 0));
            const uint32_t q0 = thr(mh + sbyte(exq, 0));
            const uint32_t q1 = thr(mh + sbyte(Vq, 2));
            const bool bx = u4.z <= qx;
            const uint32_t qn = bx ? q1 : q0;
            const uint32_t nA = mh + (uint32_t)(bx ? sbyte(Vq, 3) : sbyte(exq, 3));
            const uint32_t nB = mh + (uint32_t)(bx ? sbyte(Vq, 1) : 0);
            const bool bx1 = u4.w <= qn;
            const uint32_t res = (bx1 ? nA : nB) | (bx ? f1 : f0) | (bx1 ? 1u << 31 : 0u);
            const uint32_t r0 = quad_bcast<0x00>(res), r1 = quad_bcast<0x55>(res);
            const uint32_t r2 = quad_bcast<0xAA>(res), r3 = quad_bcast<0xFF>(res);
            const bool ax = u4.x <= tx;
            const uint32_t tn = ax ? t1 : t0;
            const uint32_t rA = ax ? r3 : r2, rB = ax ? r1 : r0;
            const bool ax1 = u4.y <= tn;
            const uint32_t sel = ax1 ? rA : rB;
            S = sel & 0x0FFFFFFFu;
            fw |= (sel >> 28) << (4 * st);
            aprev = (sel >> 31) != 0u;
        }
        const uint32_t cnew = cw ^ fw;
        *word(y, w) = cnew;
        if (w == 0) c0new = cnew;
    }
}

// Chains per workgroup of the quad large-lattice kernel: up to two consumer
// waves of 16 chains (the other waves produce), so that 8192 chains of L = 128
// stay resident with the per-bin table in LDS.
constexpr int kBigqMaxChains = 32;

// Sweeps of chains c0 .. c0+cpb-1 (cpb <= 32) of a large lattice.  Waves
// 0 .. nc-1 consume (nc = ceil(cpb / 16); the chain of lane l of consumer wave
// q is c0 + 16 q + l/4), the other waves produce.
template <int L, bool TAB_LDS>
__device__ __forceinline__ void sweep_tile_bigq(const SizeDev &s, int c0, int cpb, int R, int64_t M, void *trace,
                                                int32_t *hist, uint32_t *smem) {
    constexpr int N = L * L;
    const int r = s.tab_r, K = 2 * r + 1;
    const BigLayout lay = big_layout(L, s.n_bins, r, cpb, R, TAB_LDS);
    char *lds = (char *)smem;
    uint32_t *stab = (uint32_t *)(lds + lay.tab);
    uint4 *ptbl = (uint4 *)(lds + lay.pair);
    uint4 *ubuf = (uint4 *)(lds + lay.ubuf);
    const int chunk_words = R * (L / 4) * cpb;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nc = (cpb + 15) >> 4;
    const int cl = wave * 16 + (lane >> 2), j = lane & 3;
    const int c = c0 + cl;
    const bool consumer = wave < nc;
    const bool active = consumer && cl < cpb && c < s.P;
    const bool lead = active && j == 0;  // one lane per chain for the trace, histogram and level
    const uint32_t hym = 0u - (uint32_t)((j >> 1) & 1);
    // two levels per bin: the parity-state step (no bin arithmetic on the
    // chain's path); one level per bin: levels and per-bin rows
    const bool par = s.bin_shift == 1;
    const uint32_t sel_h = par ? quad_move_selector((uint32_t)j)
                               : j == 0 ? kSelMove0 : j == 1 ? kSelMove1 : j == 2 ? kSelMove2 : kSelMove3;
    const uint32_t f0 = (uint32_t)j << 28, f1 = f0 | (1u << 30);
    const uint32_t k0 = s.seed, k1 = (uint32_t)L;
    const uint32_t g0 = s.ctl->g;
    if (TAB_LDS)
        for (int i = threadIdx.x; i < s.n_bins * K; i += blockDim.x) stab[i] = s.tabc[i];
    if (par)
        build_pair_parity_q(ptbl, threadIdx.x, blockDim.x);
    else
        build_pair_levels_q(ptbl, threadIdx.x, blockDim.x);
    const int np = (int)blockDim.x - 64 * nc, pt = (int)threadIdx.x - 64 * nc;
    const int per_sweep = L / R;
    const int64_t n_chunks = M * per_sweep;
    if (!consumer) pc_produce<L>(ubuf, R, 0u, g0, (uint32_t)c0 + s.c_off, cpb, k0, k1, pt, np);
    __syncthreads();

    const uint32_t B0 = (TAB_LDS ? (uint32_t)(size_t)(lds_u32 *)(stab) : 0u) + 4u * (uint32_t)r;
    const int sB = r == 1 ? 3 : 4;  // log2(8 r)
    const int bs = s.bin_shift;
    const uint32_t pair_addr = (uint32_t)(size_t)(lds_u32 *)(ptbl);
    // parity state S = T0 + 12 b + 2 p of level m = 2 b + p (T0: the table's
    // byte address in LDS, or 0 for the table in global memory)
    const uint32_t T0 = TAB_LDS ? (uint32_t)(size_t)(lds_u32 *)(stab) : 0u;
    auto level_of = [&](uint32_t S) { return 2 * (int)((S - T0) / 12u) + (int)((S >> 1) & 1u); };
    int m = 0;
    uint32_t S = 0u;
    if (active) {
        m = s.lev[c];
        S = T0 + 12u * (uint32_t)(m >> 1) + 2u * (uint32_t)(m & 1);
    }
    for (int64_t i = 0; i < n_chunks; ++i) {
        const int64_t k = i / per_sweep;
        const int y0 = (int)(i - k * per_sweep) * R;
        if (active) {
            const uint4 *ub = ubuf + (size_t)(i & 1) * chunk_words;
            for (int rr = 0; rr < R; ++rr) {
                const uint4 *urow = ub + (size_t)rr * (L / 4) * cpb + cl;
                if (par)
                    bigq_row_p<L, TAB_LDS>(s.lat, (size_t)s.P, c, y0 + rr, S, s.tabc, pair_addr, urow, cpb, hym,
                                           sel_h, f0, f1, (uint32_t)j);
                else
                    bigq_row<L, TAB_LDS>(s.lat, (size_t)s.P, c, y0 + rr, m, bs, B0, sB, s.tabc, pair_addr, urow,
                                         cpb, hym, sel_h, f0, f1);
            }
            if (par && y0 + R == L) m = level_of(S);
            if (y0 + R == L && lead) {
                const int ev = m - N / 2;
                if (s.trace_bytes == 2)
                    ((int16_t *)trace)[(size_t)c * s.tld + k] = (int16_t)ev;
                else
                    ((int32_t *)trace)[(size_t)c * s.tld + k] = ev;
                atomicAdd(&hist[m >> bs], 1);
            }
        } else if (!consumer && i + 1 < n_chunks) {
            const int64_t k1s = (i + 1) / per_sweep;
            const int y1 = (int)(i + 1 - k1s * per_sweep) * R;
            pc_produce<L>(ubuf + (size_t)((i + 1) & 1) * chunk_words, R, (uint32_t)y1, g0 + (uint32_t)k1s, (uint32_t)c0 + s.c_off, cpb,
                          k0, k1, pt, np);
        }
        __syncthreads();
    }
    if (lead) s.lev[c] = m;
}

template <int L, bool TAB_LDS>
__global__ __launch_bounds__(kPcThreads) void k_sweep_bigq(PcParams p) {
    extern __shared__ __align__(16) uint32_t smem[];
    sweep_tile_bigq<L, TAB_LDS>(p.s, blockIdx.x * p.cpb, p.cpb, p.R, p.M, p.trace, p.hist, smem);
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
            sweep_row<L>((uint32_t)y, g, (uint32_t)c + s.c_off, k0, k1, cur, up, dn, mi, s.tab);
            store(y, cur);
            up = cur;
            cur = dn;
            dn = load(y + 2 < L ? y + 2 : y + 2 - L);
        }
        const int m = mi >> 3;
        const int ev = m - N / 2;
        if (s.trace_bytes == 2)
            ((int16_t *)p.trace)[(size_t)c * p.s.tld + k] = (int16_t)ev;
        else
            ((int32_t *)p.trace)[(size_t)c * p.s.tld + k] = ev;
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
                blk = philox10(make_uint4((uint32_t)j >> 2, g, (uint32_t)c + s.c_off, kDomSweep), s.seed, (uint32_t)L);
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
            ((int16_t *)p.trace)[(size_t)c * p.s.tld + k] = (int16_t)ev;
        else
            ((int32_t *)p.trace)[(size_t)c * p.s.tld + k] = ev;
        atomicAdd(&p.hist[m >> s.bin_shift], 1);
    }
    s.lev[c] = m;
}

__global__ void k_advance_sweeps(Ctl *ctl, uint32_t M) { ctl->g += M; }

hipError_t launch_advance(const SizeDev &s, int64_t M, hipStream_t st) {
    hipLaunchKernelGGL(k_advance_sweeps, dim3(1), dim3(1), 0, st, s.ctl, (uint32_t)M);
    return hipGetLastError();
}

// Dynamic LDS a launch may use: a CU's 160 KB less room for the kernels'
// static LDS.
constexpr size_t kLdsMax = 160 * 1024 - 256;

static bool big_size(int L) { return L == 128 || L == 256; }      // one lane per chain (kinds 5, 6)
static bool bigq_size(int L) { return L == 100 || L == 128 || L == 256; }  // quad streamed rows (kinds 8, 9)

static bool compiled_size(int L) {
    switch (L) {
    case 4: case 8: case 12: case 16: case 20: case 24: case 32: case 40: case 48: case 64: case 100: case 128:
    case 256:
        return true;
    default:
        return false;
    }
}

SizePlan plan_sweeps(const SizeDev &s, int cpb, bool allow_pc) {
    SizePlan p{};
    p.cpb = cpb < 1 ? 1 : (cpb > 64 ? 64 : cpb);
    p.R = 0;
    if (!compiled_size(s.L)) {
        p.kind = kSweepGeneric;
        p.cpb = 64;
        return p;
    }
    if (allow_pc && bigq_size(s.L) && p.cpb <= kBigqMaxChains) {
        for (int pass = 0; pass < 2; ++pass) {
            const bool tab_lds = pass == 0;
            for (int R = 4; R >= 1; R /= 2) {
                const BigLayout lay = big_layout(s.L, s.n_bins, s.tab_r, p.cpb, R, tab_lds);
                if (lay.total <= kLdsMax) {
                    p.kind = tab_lds ? kSweepBigQ : kSweepBigQGlb;
                    p.R = R;
                    p.lds_bytes = lay.total;
                    return p;
                }
            }
        }
    }
    if (allow_pc && big_size(s.L)) {
        for (int pass = 0; pass < 2; ++pass) {
            const bool tab_lds = pass == 0;
            for (int R = 4; R >= 1; R /= 2) {
                const BigLayout lay = big_layout(s.L, s.n_bins, s.tab_r, p.cpb, R, tab_lds);
                if (lay.total <= kLdsMax) {
                    p.kind = tab_lds ? kSweepBig : kSweepBigGlb;
                    p.R = R;
                    p.lds_bytes = lay.total;
                    return p;
                }
            }
        }
    }
    if (allow_pc && s.L >= 8 && s.L <= 64 && s.L % 4 == 0 && p.cpb <= kPcqMaxChains) {
        for (int R = 8; R >= 1; R /= 2) {
            if (s.L % R) continue;
            const PcLayout lay = pc_layout(s.L, s.W, s.N, s.n_bins, p.cpb, R);
            if (lay.total <= kLdsMax) {
                p.kind = kSweepPCQ;
                p.R = R;
                p.lds_bytes = lay.total;
                return p;
            }
        }
    }
    if (allow_pc && s.L <= 64 && s.L % 4 == 0) {
        for (int R = 8; R >= 1; R /= 2) {
            if (s.L % R) continue;
            const PcLayout lay = pc_layout(s.L, s.W, s.N, s.n_bins, p.cpb, R);
            if (lay.total <= kLdsMax) {
                p.kind = kSweepPC;
                p.R = R;
                p.lds_bytes = lay.total;
                return p;
            }
        }
    }
    const size_t lat_b = (size_t)s.L * s.W * p.cpb * 4;
    const size_t tab_b = (size_t)(s.N + 1) * 8 * 4;
    const size_t hist_b = (size_t)s.n_bins * 4;
    if (s.L <= 64 && lat_b + tab_b + hist_b <= kLdsMax) {
        p.kind = kSweepLdsTab;
        p.lds_bytes = lat_b + tab_b + hist_b;
    } else if (s.L <= 64 && lat_b + hist_b <= kLdsMax) {
        p.kind = kSweepLds;
        p.lds_bytes = lat_b + hist_b;
    } else {
        p.kind = kSweepGlobal;
        p.lds_bytes = 0;
    }
    return p;
}

SizePlan plan_kind(const SizeDev &s, int kind, int cpb) {
    // the one-wave kinds come from the plan without producer waves
    SizePlan p = plan_sweeps(s, cpb, kind != kSweepLdsTab && kind != kSweepLds && kind != kSweepGlobal);
    if (p.kind == kind || !compiled_size(s.L)) return p;
    // kinds the default plan passes over for a faster one at this size and cpb
    SizePlan q = p;
    auto first_fit = [&](int k, auto layout_total) {
        for (int R = 8; R >= 1; R /= 2) {
            if (s.L % R) continue;
            const size_t total = layout_total(R);
            if (total <= kLdsMax) {
                q.kind = k;
                q.R = R;
                q.lds_bytes = total;
                return true;
            }
        }
        return false;
    };
    if (kind == kSweepPC && s.L <= 64 && s.L % 4 == 0) {
        if (first_fit(kind, [&](int R) { return pc_layout(s.L, s.W, s.N, s.n_bins, p.cpb, R).total; })) return q;
    } else if ((kind == kSweepBig || kind == kSweepBigGlb) && big_size(s.L)) {
        const bool tl = kind == kSweepBig;
        if (first_fit(kind, [&](int R) { return R <= 4 ? big_layout(s.L, s.n_bins, s.tab_r, p.cpb, R, tl).total
                                                        : kLdsMax + 1; }))
            return q;
    } else if (kind == kSweepBigQGlb && bigq_size(s.L) && p.cpb <= kBigqMaxChains) {
        if (first_fit(kind, [&](int R) { return R <= 4 ? big_layout(s.L, s.n_bins, s.tab_r, p.cpb, R, false).total
                                                        : kLdsMax + 1; }))
            return q;
    } else if (kind == kSweepLds && s.L <= 64) {
        const size_t total = (size_t)s.L * s.W * p.cpb * 4 + (size_t)s.n_bins * 4;
        if (total <= kLdsMax) {
            q.kind = kSweepLds;
            q.R = 0;
            q.lds_bytes = total;
            return q;
        }
    } else if (kind == kSweepGlobal && s.L <= 64) {
        q.kind = kSweepGlobal;
        q.R = 0;
        q.lds_bytes = 0;
        return q;
    }
    return p;
}

bool batchable(const SizePlan &p) {
    return p.kind == kSweepLdsTab || p.kind == kSweepLds || p.kind == kSweepPC || p.kind == kSweepPCQ;
}

// Raise a kernel's dynamic-LDS limit to at least `bytes` (never lower it: one
// kernel can serve several sizes with different plans).
static hipError_t allow_lds(const void *kernel, size_t &allowed, size_t bytes) {
    if (bytes <= allowed) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) allowed = bytes;
    return e;
}

template <int L>
static hipError_t prepare_L(const SizePlan &p) {
    static size_t allowed_tab = 0, allowed_notab = 0, allowed_pc = 0, allowed_big = 0, allowed_bigg = 0;
    if constexpr (L >= 128 && L % 32 == 0) {
        if (p.kind == kSweepBig) return allow_lds((const void *)k_sweep_big<L, true>, allowed_big, p.lds_bytes);
        if (p.kind == kSweepBigGlb)
            return allow_lds((const void *)k_sweep_big<L, false>, allowed_bigg, p.lds_bytes);
    }
    if constexpr (L > 64 && L % 4 == 0) {
        static size_t allowed_bq = 0, allowed_bqg = 0;
        if (p.kind == kSweepBigQ) return allow_lds((const void *)k_sweep_bigq<L, true>, allowed_bq, p.lds_bytes);
        if (p.kind == kSweepBigQGlb)
            return allow_lds((const void *)k_sweep_bigq<L, false>, allowed_bqg, p.lds_bytes);
    }
    if constexpr (L >= 8 && L <= 64 && L % 4 == 0) {
        static size_t allowed_pcq = 0;
        if (p.kind == kSweepPCQ) return allow_lds((const void *)k_sweep_pcq<L>, allowed_pcq, p.lds_bytes);
    }
    if (p.kind == kSweepPC) return allow_lds((const void *)k_sweep_pc<L>, allowed_pc, p.lds_bytes);
    if (p.kind == kSweepLdsTab) return allow_lds((const void *)k_sweep_lds<L, true>, allowed_tab, p.lds_bytes);
    if (p.kind == kSweepLds) return allow_lds((const void *)k_sweep_lds<L, false>, allowed_notab, p.lds_bytes);
    return hipSuccess;
}

template <int L>
static hipError_t launch_L(const SweepParams &p0, const SizePlan &pl, hipStream_t st) {
    SweepParams p = p0;
    const dim3 grid((p.s.P + pl.cpb - 1) / pl.cpb), block(64);
    if constexpr (L >= 128 && L % 32 == 0) {
        if (pl.kind == kSweepBig || pl.kind == kSweepBigGlb) {
            PcParams q{p.s, p.M, p.trace, p.hist, pl.cpb, pl.R};
            if (pl.kind == kSweepBig)
                hipLaunchKernelGGL((k_sweep_big<L, true>), grid, dim3(kPcThreads), pl.lds_bytes, st, q);
            else
                hipLaunchKernelGGL((k_sweep_big<L, false>), grid, dim3(kPcThreads), pl.lds_bytes, st, q);
            return hipGetLastError();
        }
    }
    if constexpr (L > 64 && L % 4 == 0) {
        if (pl.kind == kSweepBigQ || pl.kind == kSweepBigQGlb) {
            PcParams q{p.s, p.M, p.trace, p.hist, pl.cpb, pl.R};
            if (pl.kind == kSweepBigQ)
                hipLaunchKernelGGL((k_sweep_bigq<L, true>), grid, dim3(kPcThreads), pl.lds_bytes, st, q);
            else
                hipLaunchKernelGGL((k_sweep_bigq<L, false>), grid, dim3(kPcThreads), pl.lds_bytes, st, q);
            return hipGetLastError();
        }
    }
    if constexpr (L >= 8 && L <= 64 && L % 4 == 0) {
        if (pl.kind == kSweepPCQ) {
            PcParams q{p.s, p.M, p.trace, p.hist, pl.cpb, pl.R};
            hipLaunchKernelGGL(k_sweep_pcq<L>, grid, dim3(kPcThreads), pl.lds_bytes, st, q);
            return hipGetLastError();
        }
    }
    if (pl.kind == kSweepPC) {
        PcParams q{p.s, p.M, p.trace, p.hist, pl.cpb, pl.R};
        hipLaunchKernelGGL(k_sweep_pc<L>, grid, dim3(kPcThreads), pl.lds_bytes, st, q);
        return hipGetLastError();
    }
    if (pl.kind == kSweepLdsTab) {
        p.lds_hist = 1;
        hipLaunchKernelGGL((k_sweep_lds<L, true>), grid, block, pl.lds_bytes, st, p);
    } else if (pl.kind == kSweepLds) {
        p.lds_hist = 1;
        hipLaunchKernelGGL((k_sweep_lds<L, false>), grid, block, pl.lds_bytes, st, p);
    } else {
        p.lds_hist = 0;
        hipLaunchKernelGGL(k_sweep_glb<L>, grid, block, 0, st, p);
    }
    return hipGetLastError();
}

#define MC_FOR_EACH_SIZE(X) X(4) X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(100) X(128) X(256)

hipError_t prepare_sweeps(const SizeDev &s, const SizePlan &p) {
    switch (s.L) {
#define MC_CASE(LL) \
    case LL: return prepare_L<LL>(p);
        MC_FOR_EACH_SIZE(MC_CASE)
#undef MC_CASE
    default:
        return hipSuccess;
    }
}

hipError_t launch_sweeps(const SizeDev &s, const SizePlan &pl, int64_t M, int64_t ld, void *trace, int32_t *hist,
                         hipStream_t st) {
    if (ld < M) return hipErrorInvalidValue;
    SweepParams p{};
    p.s = s;
    p.s.tld = ld;
    p.M = M;
    p.trace = trace;
    p.hist = hist;
    p.cpb = pl.cpb;
    p.lds_hist = 0;
    if (pl.kind == kSweepGeneric) {
        hipLaunchKernelGGL(k_sweep_generic, dim3((s.P + 63) / 64), dim3(64), 0, st, p);
        return hipGetLastError();
    }
    switch (s.L) {
#define MC_CASE(LL) \
    case LL: return launch_L<LL>(p, pl, st);
        MC_FOR_EACH_SIZE(MC_CASE)
#undef MC_CASE
    default:
        return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Batched sweeps: every size of a context in one persistent launch.  Blocks
// take tiles (a size and a run of its chains) from a queue ordered largest
// lattice first and sweep them exactly as the single-size kernel does, so a
// chain's trajectory does not depend on how it is batched (its random words
// are keyed by its own size and index).
// ---------------------------------------------------------------------------
struct BatchParams {
    SizeDev sizes[kMaxSizes];
    void *trace[kMaxSizes];
    int32_t *hist[kMaxSizes];
    int32_t cpb[kMaxSizes];
    int32_t kind[kMaxSizes];
    int32_t R[kMaxSizes];
    const Tile *tiles;
    int32_t n_tiles;
    int32_t *counter;
    int64_t M;
};

template <int L>
__device__ __forceinline__ void batched_tile(const BatchParams &p, int si, int c0, uint32_t *smem) {
    if constexpr (L >= 8) {
        if (p.kind[si] == kSweepPCQ) {
            sweep_tile_pcq<L>(p.sizes[si], c0, p.cpb[si], p.R[si], p.M, p.trace[si], p.hist[si], smem);
            return;
        }
    }
    if (p.kind[si] == kSweepPC)
        sweep_tile_pc<L>(p.sizes[si], c0, p.cpb[si], p.R[si], p.M, p.trace[si], p.hist[si], smem);
    else if (p.kind[si] == kSweepLdsTab)
        sweep_tile_lds<L, true>(p.sizes[si], c0, p.cpb[si], p.M, p.trace[si], p.hist[si], true, smem);
    else
        sweep_tile_lds<L, false>(p.sizes[si], c0, p.cpb[si], p.M, p.trace[si], p.hist[si], true, smem);
}

// kPcThreads threads: waves 1.. produce random words for producer/consumer
// tiles and idle on the others.
__global__ __launch_bounds__(kPcThreads) void k_sweep_batched(BatchParams p) {
    // The dynamic LDS follows this kernel's static s_tile; without the
    // alignment it would start at byte 4, and every 12- and 16-byte read of
    // the tile buffers (random words, pair table) would be misaligned, which
    // costs the dependent chain of a sweep about a quarter of its speed.
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int s_tile;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_tile = atomicAdd(p.counter, 1);
        __syncthreads();
        const int t = s_tile;
        if (t >= p.n_tiles) break;  // every block leaves once the queue is empty
        const Tile tl = p.tiles[t];
        switch (p.sizes[tl.size].L) {
#define MC_CASE(LL) \
    case LL: batched_tile<LL>(p, tl.size, tl.c0, smem); break;
            MC_CASE(4) MC_CASE(8) MC_CASE(12) MC_CASE(16) MC_CASE(20) MC_CASE(24) MC_CASE(32) MC_CASE(40) MC_CASE(48)
            MC_CASE(64)
#undef MC_CASE
        default:
            break;
        }
    }
}

__global__ void k_reset_counter(int32_t *c) { *c = 0; }

hipError_t prepare_batched(size_t lds_bytes) {
    static size_t allowed = 0;
    if (lds_bytes > kLdsMax) return hipErrorInvalidValue;
    return allow_lds((const void *)k_sweep_batched, allowed, lds_bytes);
}

hipError_t launch_sweeps_batched(const SizeDev *sizes, const SizePlan *plans, int n_sizes, const Tile *tiles_dev,
                                 int n_tiles, int32_t *counter_dev, int grid, size_t lds_bytes, int64_t M, int64_t ld,
                                 void *const *trace, int32_t *const *hist, hipStream_t st) {
    if (n_sizes > kMaxSizes || ld < M) return hipErrorInvalidValue;
    BatchParams p{};
    for (int i = 0; i < n_sizes; ++i) {
        p.sizes[i] = sizes[i];
        p.sizes[i].tld = ld;
        p.trace[i] = trace[i];
        p.hist[i] = hist[i];
        p.cpb[i] = plans[i].cpb;
        p.kind[i] = plans[i].kind;
        p.R[i] = plans[i].R;
    }
    p.tiles = tiles_dev;
    p.n_tiles = n_tiles;
    p.counter = counter_dev;
    p.M = M;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, counter_dev);
    hipLaunchKernelGGL(k_sweep_batched, dim3(grid), dim3(kPcThreads), lds_bytes, st, p);
    return hipGetLastError();
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
// "In order" means by position t = 0 .. P-1; the chain at position t is
// order[t] (the energy ordering of the chains, Sec. 2), or t without an order.
// A chain's tests draw their words from its own index, whatever its position.
// ---------------------------------------------------------------------------
struct JoinParams {
    SizeDev s;
    const void *trace;
    int64_t M;
    int32_t *cut;
    int32_t *hist;
    int32_t mode;
    const int32_t *order;  // nullptr: index order
};

__device__ __forceinline__ int join_chain(const JoinParams &p, int t) { return p.order ? p.order[t] : t; }

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
            const uint4 blk = philox10(make_uint4((uint32_t)k >> 2, r, i + s.c_off, kDomJoin), s.seed, (uint32_t)s.L);
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
    const int t = blockIdx.x;  // position
    const int i = join_chain(p, t);
    const TT *tr = (const TT *)p.trace;
    const int half = s.N / 2;
    const int sigma = (t == 0) ? s.ctl->sigma
                               : min(max((int)tr[(size_t)join_chain(p, t - 1) * p.M + (p.M - 1)] + half, 0), s.N);
    int cut;
    if (p.mode == 1 || sigma < 0)
        cut = 1;
    else
        cut = join_scan<TT>(s, tr + (size_t)i * p.M, p.M, sigma, s.ctl->r, (uint32_t)i);
    if (threadIdx.x == 0) s.scratch_cut[t] = cut;
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
    int64_t kept = 0, cut_sum = 0;
    int n_none = 0, cut_max = 0;
    for (int c0 = 0; c0 < s.P; c0 += CH) {
        const int n = min(CH, s.P - c0);
        __syncthreads();
        for (int t = lane; t < n; t += 64) {
            s_cut[t] = s.scratch_cut[c0 + t];
            s_last[t + 1] = min(max((int)tr[(size_t)join_chain(p, c0 + t) * p.M + (p.M - 1)] + half, 0), s.N);
        }
        if (lane == 0)
            s_last[0] = c0 > 0 ? min(max((int)tr[(size_t)join_chain(p, c0 - 1) * p.M + (p.M - 1)] + half, 0), s.N)
                               : s.ctl->sigma;
        __syncthreads();
        for (int t = 0; t < n; ++t) {
            const int pos = c0 + t;
            const int i = join_chain(p, pos);
            int cut = s_cut[t];
            const int spec = s_last[t];  // seam assumed by k_join_spec
            if (p.mode == 0 && pos > 0 && sigma >= 0 && (sigma >> s.bin_shift) != (spec >> s.bin_shift))
                cut = join_scan<TT>(s, tr + (size_t)i * p.M, p.M, sigma, r, (uint32_t)i);
            if (lane == 0) p.cut[i] = cut;
            if (cut > 0) {
                kept += p.M - cut + 1;
                sigma = s_last[t + 1];
                cut_sum += cut;
                cut_max = max(cut_max, cut);
            } else {
                n_none += 1;
            }
        }
    }
    if (lane == 0) {
        s.ctl->sigma = sigma;
        s.ctl->retained += kept;
        s.ctl->r = r + 1;
        s.ctl->join_none = n_none;
        s.ctl->join_cut_max = cut_max;
        s.ctl->join_cut_sum = cut_sum;
    }
}

template <typename TT>
__global__ __launch_bounds__(256) void k_join_hist(JoinParams p) {
    extern __shared__ __align__(16) uint32_t smem[];
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

// ---------------------------------------------------------------------------
// The energy ordering of the chains for a joint (Sec. 2 suggests ordering the
// nodes by the energies of their configurations and leaves the rule open): a
// greedy chain of nearest levels.  Starting from the seam (with none, chain 0
// goes first), each position takes the chain not yet placed whose first
// configuration's level is nearest to the level the chain before it ended on,
// ties to the lower level, then the lower index.  Built on the device, so a
// joint in energy order needs no host round trip and can be captured in a
// graph.  One workgroup:
//   (1) every chain's first and last level; counts of first levels and their
//       prefix sums, the runs of a list of chains sorted by (first level,
//       index);
//   (2) the list, filled in index order a chunk at a time (a chain's place in
//       its level's run is the number of earlier chains of that level);
//   (3) a two-level bitmap (in LDS) of the levels that still hold unplaced
//       chains;
//   (4) one thread walks the positions: the nearest level at or above the
//       reference and the nearest one below it come from the bitmaps; the
//       pick takes the next chain of that level's run.
// ---------------------------------------------------------------------------
constexpr int kOrderThreads = 256;
constexpr int kOrderMaxWords = (kMaxLevels + 64) / 64;

template <typename TT>
__global__ __launch_bounds__(kOrderThreads) void k_energy_order(SizeDev s, const TT *tr, int64_t M) {
    const int N = s.N, P = s.P, half = N / 2, t = threadIdx.x;
    int32_t *nextp = s.ord, *endp = s.ord + (N + 1), *list = s.ord + 2 * (N + 1);
    int32_t *firstl = list + P, *lastl = firstl + P;
    const int NW = order_bitmap_words(N), NSUM = order_summary_words(N);
    __shared__ uint64_t bm[kOrderMaxWords];
    __shared__ uint64_t sm[(kOrderMaxWords + 63) / 64];
    __shared__ int32_t sh[kOrderThreads];
    __shared__ int32_t sf[kOrderThreads];
    for (int m = t; m <= N; m += kOrderThreads) nextp[m] = 0;
    for (int c = t; c < P; c += kOrderThreads) {
        firstl[c] = min(max((int)tr[(size_t)c * M] + half, 0), N);
        lastl[c] = min(max((int)tr[(size_t)c * M + (M - 1)] + half, 0), N);
    }
    __syncthreads();
    for (int c = t; c < P; c += kOrderThreads) atomicAdd(&nextp[firstl[c]], 1);
    __syncthreads();
    // exclusive prefix sums of the counts, each thread over a contiguous range
    const int per = (N + 1 + kOrderThreads - 1) / kOrderThreads;
    const int m0 = min(N + 1, t * per), m1 = min(N + 1, m0 + per);
    int tot = 0;
    for (int m = m0; m < m1; ++m) tot += nextp[m];
    sh[t] = tot;
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int i = 0; i < kOrderThreads; ++i) {
            const int v = sh[i];
            sh[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int acc = sh[t];
    for (int m = m0; m < m1; ++m) {
        const int v = nextp[m];
        nextp[m] = acc;
        endp[m] = acc + v;
        acc += v;
    }
    __syncthreads();
    // the sorted list, stable in the chain index
    for (int c0 = 0; c0 < P; c0 += kOrderThreads) {
        const int c = c0 + t;
        const int f = c < P ? firstl[c] : -1;
        sf[t] = f;
        __syncthreads();
        int rank = 0;
        bool lastof = true;
        if (f >= 0) {
            for (int u = 0; u < kOrderThreads; ++u) {
                if (sf[u] != f) continue;
                if (u < t) ++rank;
                if (u > t) lastof = false;
            }
            list[nextp[f] + rank] = c;
        }
        __syncthreads();
        if (f >= 0 && lastof) nextp[f] += rank + 1;
        __syncthreads();
    }
    // back to the start of every run (runs are contiguous in level order)
    for (int m = t; m <= N; m += kOrderThreads) nextp[m] = m > 0 ? endp[m - 1] : 0;
    for (int w = t; w < NW; w += kOrderThreads) {
        uint64_t bits = 0;
        for (int k = 0; k < 64; ++k) {
            const int m = 64 * w + k;
            if (m <= N && endp[m] > (m > 0 ? endp[m - 1] : 0)) bits |= 1ull << k;
        }
        bm[w] = bits;
    }
    __syncthreads();
    for (int w = t; w < NSUM; w += kOrderThreads) {
        uint64_t bits = 0;
        for (int k = 0; k < 64; ++k)
            if (64 * w + k < NW && bm[64 * w + k]) bits |= 1ull << k;
        sm[w] = bits;
    }
    __syncthreads();
    if (t != 0) return;
    auto take = [&](int m) {
        const int c = list[nextp[m]];
        nextp[m] += 1;
        if (nextp[m] == endp[m]) {
            const int w = m >> 6;
            bm[w] &= ~(1ull << (m & 63));
            if (!bm[w]) sm[w >> 6] &= ~(1ull << (w & 63));
        }
        return c;
    };
    // smallest level >= m that holds unplaced chains, or -1
    auto at_or_above = [&](int m) {
        if (m > N) return -1;
        int w = m >> 6;
        const uint64_t b = bm[w] & (~0ull << (m & 63));
        if (b) return 64 * w + __ffsll((unsigned long long)b) - 1;
        const int w1 = w + 1;
        int sw = w1 >> 6;
        if (sw >= NSUM) return -1;
        uint64_t sb = sm[sw] & (~0ull << (w1 & 63));
        while (!sb) {
            if (++sw >= NSUM) return -1;
            sb = sm[sw];
        }
        w = 64 * sw + __ffsll((unsigned long long)sb) - 1;
        return 64 * w + __ffsll((unsigned long long)bm[w]) - 1;
    };
    // largest level <= m that holds unplaced chains, or -1
    auto at_or_below = [&](int m) {
        if (m < 0) return -1;
        int w = m >> 6;
        const int k = m & 63;
        const uint64_t b = bm[w] & (k == 63 ? ~0ull : ((1ull << (k + 1)) - 1));
        if (b) return 64 * w + 63 - __clzll((long long)b);
        const int w1 = w - 1;
        if (w1 < 0) return -1;
        int sw = w1 >> 6;
        const int k1 = w1 & 63;
        uint64_t sb = sm[sw] & (k1 == 63 ? ~0ull : ((1ull << (k1 + 1)) - 1));
        while (!sb) {
            if (--sw < 0) return -1;
            sb = sm[sw];
        }
        w = 64 * sw + 63 - __clzll((long long)sb);
        return 64 * w + 63 - __clzll((long long)bm[w]);
    };
    int pos = 0, ref = s.ctl->sigma;
    if (ref < 0 && P > 0) {
        const int c = take(firstl[0]);  // chain 0 heads its level's run
        s.join_order[pos++] = c;
        ref = lastl[c];
    }
    for (; pos < P; ++pos) {
        const int up = at_or_above(ref);
        const int dn = at_or_below(ref - 1);
        const int pick = (dn >= 0 && (up < 0 || ref - dn <= up - ref)) ? dn : up;
        const int c = take(pick);
        s.join_order[pos] = c;
        ref = lastl[c];
    }
}

hipError_t launch_energy_order(const SizeDev &s, const void *trace, int64_t M, hipStream_t st) {
    if (s.N > kMaxLevels - 1) return hipErrorInvalidValue;
    if (s.trace_bytes == 2)
        hipLaunchKernelGGL(k_energy_order<int16_t>, dim3(1), dim3(kOrderThreads), 0, st, s, (const int16_t *)trace, M);
    else
        hipLaunchKernelGGL(k_energy_order<int32_t>, dim3(1), dim3(kOrderThreads), 0, st, s, (const int32_t *)trace, M);
    return hipGetLastError();
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
                       const int32_t *order, hipStream_t st) {
    JoinParams p{s, trace, M, cut, hist, mode, order};
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

template <typename HT>
__global__ __launch_bounds__(1024) void k_update(SizeDev s, HT *hist) {
    __shared__ long long s_min[16], s_sum[16];
    __shared__ int s_n[16];
    __shared__ double s_lo[16], s_hi[16];
    long long mn = 0x7FFFFFFFFFFFFFFFll, sum = 0;
    int n = 0;
    double lo = INFINITY, hi = -INFINITY;
    for (int b = threadIdx.x; b < s.n_bins; b += blockDim.x) {
        const long long h = hist[b];
        double w = s.lnW[b];
        if (h > 0) {
            w = w - det_log((int64_t)h);
            s.lnW[b] = w;
        }
        if (bin_reachable(b, s.bin_shift, s.N)) {
            n += 1;
            sum += h;
            mn = h < mn ? h : mn;
            lo = fmin(lo, w);
            hi = fmax(hi, w);
        }
        hist[b] = 0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const long long omn = __shfl_xor(mn, off, 64);
        mn = omn < mn ? omn : mn;
        sum += __shfl_xor(sum, off, 64);
        n += __shfl_xor(n, off, 64);
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_min[wv] = mn;
        s_sum[wv] = sum;
        s_n[wv] = n;
        s_lo[wv] = lo;
        s_hi[wv] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        long long tmn = s_min[0], tsum = 0;
        int tn = 0;
        double tlo = s_lo[0], thi = s_hi[0];
        for (int i = 0; i < nw; ++i) {
            tmn = s_min[i] < tmn ? s_min[i] : tmn;
            tsum += s_sum[i];
            tn += s_n[i];
            tlo = fmin(tlo, s_lo[i]);
            thi = fmax(thi, s_hi[i]);
        }
        const int flat = (tn > 0 && tsum > 0 && 5ll * tn * tmn >= 4ll * tsum) ? 1 : 0;
        Ctl *ctl = s.ctl;
        ctl->upd_h_sum = tsum;
        ctl->upd_h_min = tn > 0 ? tmn : 0;
        ctl->upd_n_reach = tn;
        ctl->upd_lnw_lo = tlo;
        ctl->upd_lnw_hi = thi;
        ctl->flat = flat;
        ctl->iter += 1;
        if (flat && ctl->flat_iter == 0) ctl->flat_iter = ctl->iter;
        ctl->retained_last = ctl->retained;
        ctl->retained = 0;
    }
}

// A chain's level is half the number of its broken bonds (level m = (E + 2N)/4
// with E = -(bonds) + 2 (broken bonds) over the 2N bonds, J = 1); the sweeps
// track it incrementally, so a disagreement means the state is corrupt.  One
// thread per chain counts broken right and down bonds of its bit-packed rows
// (a row's last word holds L - 32 (W - 1) sites; the right neighbour of site
// L-1 is site 0, the row below row L-1 is row 0).
__global__ __launch_bounds__(256) void k_check_levels(SizeDev s) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= s.P) return;
    const int L = s.L, W = s.W;
    const size_t P = (size_t)s.P;
    const int nb = L - 32 * (W - 1);
    const uint32_t last_mask = nb == 32 ? 0xFFFFFFFFu : (1u << nb) - 1u;
    int64_t broken = 0;
    for (int y = 0; y < L; ++y) {
        const int yd = y + 1 < L ? y + 1 : 0;
        for (int w = 0; w < W; ++w) {
            const uint32_t cur = s.lat[(size_t)(y * W + w) * P + c];
            const uint32_t down = s.lat[(size_t)(yd * W + w) * P + c];
            uint32_t right, mask = 0xFFFFFFFFu;
            if (w + 1 < W) {
                right = (cur >> 1) | (s.lat[(size_t)(y * W + w + 1) * P + c] << 31);
            } else {
                const uint32_t first = s.lat[(size_t)(y * W) * P + c];
                right = (cur >> 1) | ((first & 1u) << (nb - 1));
                mask = last_mask;
            }
            broken += __popc((cur ^ right) & mask) + __popc((cur ^ down) & mask);
        }
    }
    if (2ll * s.lev[c] != broken) atomicAdd((unsigned long long *)s.n_bad, 1ull);
}

__global__ void k_zero64(int64_t *p) { *p = 0; }

hipError_t launch_check_levels(const SizeDev &s, hipStream_t st) {
    hipLaunchKernelGGL(k_zero64, dim3(1), dim3(1), 0, st, s.n_bad);
    hipLaunchKernelGGL(k_check_levels, dim3((s.P + 255) / 256), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_update(const SizeDev &s, int32_t *hist, hipStream_t st) {
    hipLaunchKernelGGL(k_update<int32_t>, dim3(1), dim3(1024), 0, st, s, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tabulate(s, st);
}

// Algorithm step 6 keeps the joined histogram of several rounds: each round's
// int32 histogram is added to the size's int64 one and cleared.
__global__ void k_fold_hist(int64_t *acc, int32_t *hist, int n) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) {
        acc[b] += hist[b];
        hist[b] = 0;
    }
}

hipError_t launch_fold_hist(const SizeDev &s, int32_t *hist, hipStream_t st) {
    hipLaunchKernelGGL(k_fold_hist, dim3((s.n_bins + 255) / 256), dim3(256), 0, st, s.hist64, hist, s.n_bins);
    return hipGetLastError();
}

hipError_t launch_update64(const SizeDev &s, hipStream_t st) {
    hipLaunchKernelGGL(k_update<int64_t>, dim3(1), dim3(1024), 0, st, s, s.hist64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tabulate(s, st);
}

}  // namespace mcgpu
