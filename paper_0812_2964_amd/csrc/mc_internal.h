// mc_internal.h -- device-side state layout and kernel launchers of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcgpu {

// Per-size control block in device memory.  Counters advance on the device,
// so a captured sequence of launches stays correct when replayed.
struct Ctl {
    uint32_t g;             // global index of the next sweep (random-word domain 0)
    uint32_t r;             // index of the next joint round (domain 2)
    int32_t sigma;          // seam level, -1 = none yet
    int32_t flat;           // flatness of the last update
    int64_t retained;       // configurations kept by joints since the last update
    int64_t retained_last;  // the same, frozen by the last update
    int32_t iter;           // updates done so far
    int32_t flat_iter;      // first update (1-based) that was flat, 0 = none
    // Statistics of the last joint and of the last update (read by
    // mc_get_stats; not part of a checkpoint).
    int32_t join_none;      // chains of the last joint that kept nothing
    int32_t join_cut_max;   // largest cut point of the last joint
    int64_t join_cut_sum;   // sum of its cut points over the chains that kept something
    int64_t upd_h_sum;      // configurations in bins holding a reachable level, at the last update
    int64_t upd_h_min;      // fewest of them in one such bin
    int32_t upd_n_reach;    // number of such bins
    int32_t pad_;
    double upd_lnw_lo;      // smallest and largest ln w over those bins after the update
    double upd_lnw_hi;
};

// Device view of one lattice size.
struct SizeDev {
    int32_t L, N, W;        // W = 32-bit words per lattice row
    int32_t P;              // chains
    int32_t bin_shift, n_bins;
    uint32_t seed;
    uint32_t c_off;         // global index of chain 0 (the random words are keyed by the global index)
    int32_t trace_bytes;    // 2 (int16) or 4 (int32)
    int64_t tld;            // row length of the trace a sweep launch writes (set per launch)
    uint32_t *lat;          // [L*W][P] chain-interleaved bit-packed rows
    int32_t *lev;           // [P] current level of each chain
    double *lnW;            // [n_bins]
    uint32_t *tab;          // [(N+1)*8] thresholds, entry (m, a) at m*8 + a, a = dm + 2
    uint32_t *tabc;         // [n_bins*(2*tab_r+1)] the same thresholds per bin (k_tabulate_compact)
    int32_t tab_r;          // 2 with one level per bin, else 1
    Ctl *ctl;
    int32_t *scratch_cut;   // [P] speculative cut points of the joint
    int32_t *join_order;    // [P] chain at each position of an energy-ordered joint
    int64_t *hist64;        // [n_bins] joined histogram of Algorithm step 6's rounds
    int64_t *n_bad;         // [1] chains whose level disagrees with their lattice (mc_check_levels)
    int32_t *ord;           // [order_scratch_ints(N, P)] scratch of the energy ordering (k_energy_order)
};

// Scratch of the device-side energy ordering of one size: per level the next
// and the end position of its run (2 (N+1)), the chains sorted by first level
// and index, every chain's first and last level (3 P), then, 8-aligned, the
// bitmap of levels with unplaced chains and its summary (uint64 words).
__host__ __device__ inline int order_bitmap_words(int N) { return (N + 64) / 64; }
__host__ __device__ inline int order_summary_words(int N) { return (order_bitmap_words(N) + 63) / 64; }
__host__ __device__ inline size_t order_bitmap_at(int N, int P) {
    return ((size_t)2 * (N + 1) + (size_t)3 * P + 1) & ~(size_t)1;  // in int32 units, 8-byte aligned
}
__host__ __device__ inline size_t order_scratch_ints(int N, int P) {
    return order_bitmap_at(N, P) + 2 * (size_t)(order_bitmap_words(N) + order_summary_words(N));
}

// How the sweeps of one size are launched.
enum SweepKind : int32_t {
    kSweepLdsTab = 0,   // lattice and thresholds in LDS
    kSweepLds = 1,      // lattice in LDS, thresholds read from global memory
    kSweepGlobal = 2,   // lattice rows streamed from global memory (large L)
    kSweepGeneric = 3,  // any even L, bit by bit (L not among the compiled sizes)
    kSweepPC = 4,       // lattice and thresholds in LDS, random words from producer waves
    kSweepBig = 5,      // L >= 128: rows streamed from global memory, per-bin thresholds in LDS
    kSweepBigGlb = 6,   // the same with the per-bin thresholds read from global memory
    kSweepPCQ = 7,      // as kSweepPC with four lanes per chain deciding four sites per step (8 <= L <= 64)
    kSweepBigQ = 8,     // as kSweepBig with four lanes per chain deciding four sites per step
    kSweepBigQGlb = 9,  // the same with the per-bin thresholds read from global memory
};

struct SizePlan {
    int32_t cpb;        // chains per 64-lane block
    int32_t kind;       // SweepKind
    int32_t R;          // rows per chunk of random words (producer/consumer kinds)
    size_t lds_bytes;   // dynamic LDS per block
};

constexpr int kMaxSizes = 16;
// Levels of the largest lattice (L = 256: N + 1).
constexpr int kMaxLevels = 256 * 256 + 1;

// One unit of work of the batched launch: chains c0 .. c0+cpb-1 of size `size`.
struct Tile {
    int32_t size;
    int32_t c0;
};

// Kernel launchers (mc_kernels.hip).  All enqueue on `st` and return the
// launch status.
SizePlan plan_sweeps(const SizeDev &s, int chains_per_block, bool allow_pc = true);
// The plan a kernel kind would get at chains_per_block (its kind differs from
// `kind` when that kind cannot run the size at that many chains per block).
SizePlan plan_kind(const SizeDev &s, int kind, int chains_per_block);
bool batchable(const SizePlan &p);
hipError_t prepare_sweeps(const SizeDev &s, const SizePlan &p);  // kernel attributes; call outside capture
hipError_t prepare_batched(size_t lds_bytes);
hipError_t launch_init(const SizeDev &s, hipStream_t st);
hipError_t launch_tabulate(const SizeDev &s, hipStream_t st);
// M sweeps; sweep k of chain c goes to trace[c * ld + k] (ld >= M).
hipError_t launch_sweeps(const SizeDev &s, const SizePlan &p, int64_t M, int64_t ld, void *trace, int32_t *hist,
                         hipStream_t st);
hipError_t launch_sweeps_batched(const SizeDev *sizes, const SizePlan *plans, int n_sizes, const Tile *tiles_dev,
                                 int n_tiles, int32_t *counter_dev, int grid, size_t lds_bytes, int64_t M, int64_t ld,
                                 void *const *trace, int32_t *const *hist, hipStream_t st);
hipError_t launch_advance(const SizeDev &s, int64_t M, hipStream_t st);
// The energy ordering of a round's chains into s.join_order (k_energy_order).
hipError_t launch_energy_order(const SizeDev &s, const void *trace, int64_t M, hipStream_t st);
// order: the chain at each position of the joint, or nullptr for index order.
hipError_t launch_join(const SizeDev &s, const void *trace, int64_t M, int32_t *cut, int32_t *hist, int mode,
                       const int32_t *order, hipStream_t st);
hipError_t launch_update(const SizeDev &s, int32_t *hist, hipStream_t st);
// Add a round's int32 histogram to s.hist64 and clear it; the update from
// s.hist64 (which it then clears).
hipError_t launch_fold_hist(const SizeDev &s, int32_t *hist, hipStream_t st);
hipError_t launch_update64(const SizeDev &s, hipStream_t st);
hipError_t launch_thermo(const SizeDev &s, const double *beta_dev, int n_beta, double *out_dev, hipStream_t st);
// Count, into s.n_bad, the chains whose level is not half their broken bonds.
hipError_t launch_check_levels(const SizeDev &s, hipStream_t st);
// Step-timing probe of the quad step (mc_probe kinds 9-11): mode 0 the sweeps'
// step, 1 its threshold reads moved to the pair table, 2 no threshold reads.
hipError_t launch_quad_step_probe(int mode, int rows, int64_t *cyc, uint32_t *out, hipStream_t st);

// Most inverse temperatures one mc_thermo call takes.
constexpr int kThermoMaxBetas = 1 << 20;
// Most inverse temperatures one mc_thermo_static call takes (its device array
// holds 5 doubles per inverse temperature: 320 KB per GPU).
constexpr int kThermoStaticMaxBetas = 8192;
constexpr int kMaxDevices = 64;
// Device address of mc_thermo_static's array on `device` (which must be the
// current device on the first call for it); looked up once per device.
hipError_t thermo_scratch_address(int device, double **out);

// Message returned by mc_last_error() on this thread (mc_api.hip).
void set_last_error(const char *msg);

}  // namespace mcgpu
