/*
 * mc.h -- C ABI of the MI355X (gfx950) implementation of the parallel
 * multicanonical Markov-chain method of Sugihara, Higo and Nakamura,
 * "Parallelization of Markov Chain Generation and its Application to the
 * Multicanonical Method" (arXiv 0812.2964), applied to the periodic 2D Ising
 * model of its Sec. 4.
 *
 * One iteration of the method, for one lattice size:
 *
 *     mc_run_chains     Algorithm step 2: every chain makes n_sweeps sweeps
 *     mc_join           Algorithm steps 3-5: detailed-balance joints
 *     mc_update_weights eq. (new_weight) in logarithms (Sec. 3.1, Sec. 4.2)
 *
 * Conventions (the readings of the paper this library implements):
 *   - N = L*L spins, J = 1, H = -sum_<ij> s_i s_j with periodic boundaries.
 *   - A "configuration" of a chain is its lattice after one sweep: N
 *     single-spin Metropolis attempts in typewriter order (site j = y*L + x).
 *   - Level m = (E + 2N)/4 in [0, N]; bin b = m >> bin_shift; n_bins =
 *     (N >> bin_shift) + 1.  ln w is stored per bin in binary64.
 *   - Acceptance of a move that changes ln w by d: u <= tau(d), where u is a
 *     32-bit Philox4x32-10 word and tau(d) = 2^32-1 for d >= 0, else
 *     min(floor(exp(d) 2^32), 2^32-1), with exp and log evaluated by a fixed
 *     Cody-Waite/Taylor sequence of IEEE-754 operations (bit-reproducible).
 *   - Random words: counter (j>>2, a, chain, domain), key (seed, L), word j&3;
 *     domain 0 = sweeps (a = global sweep index), 1 = initial spins, 2 = joint
 *     tests (a = round, j = 0-based position in the chain).
 *   - Energies in traces are E/4 (= m - N/2): int16 elements for L <= 254,
 *     int32 for L = 256.  Traces are row-major [n_chains][n_sweeps].
 *
 * Memory and streams: a context owns the chain state (bit-packed lattices,
 * levels, counters, seam), the ln w tables and the acceptance thresholds, in
 * device memory it allocates at creation.  Traces, histograms and cut arrays
 * are device buffers owned by the caller.  Every call enqueues work on the
 * HIP stream given at creation and returns without waiting, except those
 * that write host memory, which synchronise that stream.
 *
 * Errors: every call returns an mc_status.  Argument errors are detected
 * before anything is enqueued and leave the context unchanged.  A failed HIP
 * call marks the context broken (MC_EHIP), after which every call except
 * mc_destroy fails.  mc_last_error() returns a message for the last error on
 * the calling thread.  Calls on one context are not thread-safe.
 */
#ifndef MC_H
#define MC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mc_ctx mc_ctx;

typedef enum {
    MC_OK = 0,
    MC_EINVAL = -1,     /* bad argument                                       */
    MC_ENOMEM = -2,     /* device allocation failed                           */
    MC_ENODEV = -3,     /* no usable GPU                                      */
    MC_EHIP = -4,       /* a HIP runtime call failed; the context is broken   */
    MC_ESTATE = -5,     /* call out of order (e.g. join of sweeps not run)    */
    MC_EOVERFLOW = -6,  /* histogram or counter range would be exceeded       */
    MC_ECORRUPT = -7,   /* a state blob failed its checks                     */
    MC_EINTERNAL = -8   /* the chain state failed a consistency check         */
} mc_status;

/* One lattice size of a context.  Sizes are independent ensembles: each has
   its own chains, ln w table, seam and counters. */
typedef struct {
    int32_t L;         /* even, 4 <= L <= 256                                  */
    int32_t n_chains;  /* p of the paper, >= 1, <= 2^20                        */
    uint32_t seed;     /* Philox key word 0 (word 1 is L)                      */
    int32_t bin_shift; /* 0: one bin per level; 1: two levels (8 energy units) */
    uint32_t chain_offset; /* global index of chain 0: the chains are chains
                              chain_offset .. chain_offset + n_chains - 1 of a
                              run split over several contexts (or GPUs), and
                              every random word is keyed by the global index;
                              0 for a whole run.  offset + n_chains <= 2^32 */
} mc_size;

/* Create a context on the current HIP device for n_sizes (1..16) lattice
   sizes, bound to hip_stream (a hipStream_t; NULL = the null stream).
   Sizes whose lattices fit in LDS (L <= 64) run batched: one persistent
   launch sweeps all of them (see mc_get_launch).
   Algorithm step 1: every chain c of every size gets its initial spins
   (s_j = +1 iff bit 31 of the domain-1 word of site j is set), its level is
   computed, ln w is set to 0 (w^(1) = 1, Sec. 3.1), the seam is "none" and the
   sweep and round counters are 0.  On success *out receives the context.
   Errors: MC_EINVAL (sizes), MC_ENODEV (no GPU), MC_ENOMEM, MC_EHIP. */
mc_status mc_create(const mc_size *sizes, int32_t n_sizes, void *hip_stream, mc_ctx **out);

/* Release everything the context owns (waits for its stream first). NULL is a
   no-op; MC_ESTATE while graphs of the context exist. */
mc_status mc_destroy(mc_ctx *ctx);

/* Number of bins / trace element size in bytes / lattice words per chain of a size. */
int32_t mc_n_bins(const mc_ctx *ctx, int32_t size_idx);
int32_t mc_trace_elem_bytes(const mc_ctx *ctx, int32_t size_idx);
int32_t mc_lattice_words(const mc_ctx *ctx, int32_t size_idx);

/* Set ln w of one size from host memory (copied; n_bins values, all finite),
   or to 0 everywhere when lnW_host is NULL, and tabulate the acceptance
   thresholds.  Sec. 3.1 (initial weight w^(1) = 1) and Sec. 4.2 (weights kept
   as logarithms).  Errors: MC_EINVAL (n_bins mismatch, non-finite value). */
mc_status mc_init_weights(mc_ctx *ctx, int32_t size_idx, const double *lnW_host, int32_t n_bins);

/* Algorithm step 2 for every size of the context, in one launch: each chain
   makes n_sweeps sweeps from where it stopped (each chain is generated
   independently over the whole run, Sec. 2).  For size s:
     trace_dev[s]: device, [n_chains][n_sweeps] of E/4 after each sweep;
     hist_dev[s]:  device int32 [n_bins]; the bin of every configuration of
                   every chain is added to it (so it must hold zeros, or the
                   joint histogram so far, on entry).
   trace_dev and hist_dev are host arrays of n_sizes device pointers.
   Errors: MC_EINVAL (n_sweeps < 1, NULL pointer), MC_EOVERFLOW (more than
   2^31-1 configurations would be counted before the next weight update, or
   the size's sweeps would pass 2^32 in its lifetime: the sweep index is a
   32-bit counter of the random words, which would then repeat). */
mc_status mc_run_chains(mc_ctx *ctx, int64_t n_sweeps, void *const *trace_dev, int32_t *const *hist_dev);

/* Algorithm step 2 for one round of row_len sweeps made in several launches
   (progress reports between launches, bounded kernel durations): n_sweeps
   more sweeps of every chain, written to columns
   col .. col + n_sweeps - 1 of each size's [n_chains][row_len] trace
   (trace_dev[s] is the start of that trace, not of the columns).  The
   chains, random words and histogram are exactly those of one
   mc_run_chains(row_len) call: the parts of a round are bit for bit the
   whole.  col = 0 starts a round; each later part must continue it (col =
   sweeps made so far, the same row_len).  The round can be joined
   (mc_join with n_sweeps = row_len) once col + n_sweeps = row_len.
   mc_run_chains(ctx, n, t, h) is mc_run_chains_part(ctx, n, 0, n, t, h).
   Errors: as mc_run_chains; MC_EINVAL when the columns do not fit the rows;
   MC_ESTATE for a part that does not continue the round in progress. */
mc_status mc_run_chains_part(mc_ctx *ctx, int64_t n_sweeps, int64_t col, int64_t row_len, void *const *trace_dev,
                             int32_t *const *hist_dev);

/* Algorithm steps 3-5 for one size over the trace of the last mc_run_chains
   (n_sweeps must match it).  For chain i = 0 .. n_chains-1 in order, the
   configurations are tested against the seam (the energy of the last kept
   configuration before chain i) with the Metropolis rule until one is
   accepted; it and its successors are kept, the others discarded.  If none is
   accepted the seam is carried on unchanged.  The first chain of the very
   first round has no seam and is kept whole.
     cut_dev:  device int32 [n_chains]: 1-based first kept position, or -1;
     hist_dev: device int32 [n_bins]: the histogram mc_run_chains filled; the
               discarded configurations are removed from it, so on return it
               is the total histogram h(E) of the joined chain;
     mode:     0 = detailed balance (the paper's method), 1 = keep every
               chain whole (the naive splice compared in Sec. 5), 2 = detailed
               balance with the chains taken in energy order (the ordering
               Sec. 2 suggests to raise the acceptance at the joints, rule not
               given there): starting from the seam (with none, chain 0
               first), each position takes the chain not yet placed whose
               first configuration's level is nearest to the level the chain
               before it ended on, ties to the lower level, then the lower
               index.  Mode 2 builds the order on the device (one
               workgroup, from the trace's first and last columns), so it
               does not synchronise and can be captured in a graph.
   The test of chain c's k-th configuration uses its own random word (round,
   c, k) in every mode, whatever c's position.
   Errors: MC_EINVAL, MC_ESTATE (no complete round of mc_run_chains to join),
   MC_EOVERFLOW (the size's 2^32 joint rounds, a 32-bit counter of the
   random words, are used up). */
mc_status mc_join(mc_ctx *ctx, int32_t size_idx, const void *trace_dev, int64_t n_sweeps, int32_t *cut_dev,
                  int32_t *hist_dev, int32_t mode);

/* Eq. (new_weight) in logarithms for one size: ln w(b) -= ln h(b) for every
   bin with h(b) > 0, the flatness test (over bins holding a reachable level:
   5 n min h >= 4 sum h, in integers), re-tabulation of the thresholds, and
   hist_dev set to zero.  Optional host outputs (each may be NULL; if any is
   non-NULL the call synchronises): lnW_out_host [n_bins], is_flat, retained
   (configurations kept by the joints since the previous update).
   Errors: MC_EINVAL. */
mc_status mc_update_weights(mc_ctx *ctx, int32_t size_idx, int32_t *hist_dev, double *lnW_out_host,
                            int32_t *is_flat, int64_t *retained);

/* One whole iteration with Algorithm step 6 (Sec. 2) for a context of one
   size: rounds of mc_run_chains and mc_join (mode as there) until the joined
   histogram holds at least m_total configurations, then the weight update of
   mc_update_weights.  The first round makes m_max sweeps; each later one
   ceil((m_total - kept) * swept / kept) sweeps within 1 .. m_max (the
   shortfall at the rate kept so far, so that little more than m_total is
   generated; m_max while nothing has been kept), and at most max_rounds
   rounds are made.  Each round's histogram is added on the device to an
   int64 histogram of the iteration, so the total may exceed 2^31.
     trace_dev: device, room for [n_chains][m_max] trace entries (each round
                writes [n_chains][m] there);
     hist_dev:  device int32 [n_bins], zero on entry, zero on return;
     cut_dev:   device int32 [n_chains], the cuts of the last round.
   Host outputs (nullable): rounds made, sweeps per chain over all rounds,
   configurations kept, flatness of the update.  Synchronises after each
   round.  Errors: MC_EINVAL (not one size, bad argument), MC_EOVERFLOW
   (n_chains * m_max >= 2^31), MC_ESTATE (a run or joint since the last
   update), and those of the calls it makes. */
mc_status mc_iterate_topup(mc_ctx *ctx, int64_t m_total, int64_t m_max, int32_t max_rounds, void *trace_dev,
                           int32_t *hist_dev, int32_t *cut_dev, int32_t mode, int32_t *rounds_out, int64_t *sweeps_out,
                           int64_t *retained_out, int32_t *is_flat);

/* Inspection (synchronising, host outputs):
   levels_host [n_chains] current level m of each chain;
   words_host  [mc_lattice_words] the bit-packed lattice of one chain: row y,
               word w at [y*W + w], bit x%32 of word x/32 is site (x, y), 1 = +1;
   seam / counters: seam level (-1 = none), round index, global sweep index. */
mc_status mc_get_levels(mc_ctx *ctx, int32_t size_idx, int32_t *levels_host);
mc_status mc_get_lattice(mc_ctx *ctx, int32_t size_idx, int32_t chain, uint32_t *words_host, int32_t n_words);
mc_status mc_get_counters(mc_ctx *ctx, int32_t size_idx, int32_t *seam, uint32_t *round, uint32_t *sweep);

/* The seam the next mc_join of one size starts from (Algorithm step 4: the
   level of the last configuration kept before its first chain; -1 = none, so
   that its first chain is kept whole).  For a run split into blocks of chains
   (chain_offset), each block's joint starts from the seam the previous
   block's joint ended with (mc_get_counters); the blocks joined in order then
   keep exactly what one joint over all chains keeps.  Only the joint reads
   the seam, so it may be set between a block's run and its joint.
   Synchronising.  MC_EINVAL for a seam outside -1..N. */
mc_status mc_set_seam(mc_ctx *ctx, int32_t size_idx, int32_t seam);

/* Checkpoint and resume (synchronising).  The random words are counter-based
   (their counters are the chain, the site and the global sweep and round
   indices), so a context restored from a blob continues bit for bit as the
   one the blob was taken from.  The blob (version 1, little-endian) holds,
   for every size: its configuration, the host call-order state (runs since
   the last update, the pending joint), the device counters (sweep index,
   round, seam, retained counts, updates, flatness), the lattices, the levels
   and ln w, under a CRC-32 (the zlib definition) of the whole blob.  The
   thresholds are rebuilt from ln w.  Caller-owned buffers (traces,
   histograms, cuts) are not part of it: a blob taken between mc_run_chains
   and mc_update_weights resumes only together with the caller's histogram.
   mc_get_state: with buf NULL, *len receives the size; otherwise buf must
   hold *len >= that size, and *len receives it.  MC_EINVAL for a null len or
   a short buffer; MC_ESTATE while a round is partly run (mc_run_chains_part).
   mc_set_state: the context must have been created with the same sizes,
   chain counts, seeds and bins (MC_EINVAL otherwise).  A blob that fails its
   magic, version, length or checksum, holds a non-finite ln w, counters out of
   range (a seam outside -1..N, pending configurations or sweeps outside
   0..2^31-1), lattice bits set beyond L in a row's last word, or a chain whose
   level is not half its broken bonds gives MC_ECORRUPT and changes nothing:
   the kernels index their tables by level, so the state is checked on the
   host before it is copied.  Graphs of the context stay valid. */
mc_status mc_get_state(mc_ctx *ctx, void *buf, size_t *len);
mc_status mc_set_state(mc_ctx *ctx, const void *buf, size_t len);

/* Read ln w of one size into host memory (n_bins values; synchronising). */
mc_status mc_get_weights(mc_ctx *ctx, int32_t size_idx, double *lnW_host, int32_t n_bins);

/* Reduced reweighting, the paper's code (ii) (Sec. 3.3, eq. reweighting2; the
   quantities of Sec. 4.1): the thermodynamics of one size at n_beta inverse
   temperatures (J = 1) from its current ln w alone.  The density of states is
   taken inversely proportional to the weight of each reachable level's bin
   (levels m = (E + 2N)/4 except 1 and N-1), normalised to count the 2^N
   configurations.  beta_host: n_beta values, each positive and finite.
   out_host: 4 * n_beta doubles; out[q * n_beta + k] is, at beta[k], for q = 0
   the mean energy E = <H>, 1 the specific heat C = beta^2 (<H^2> - <H>^2),
   2 the free energy F = -ln Z / beta, 3 the entropy S = beta (E - F), all
   totals over the lattice.  Computed on the device in binary64 after the work
   already queued on the context's stream; synchronising.  Host arrays are the
   caller's.  MC_EINVAL for a null pointer, n_beta outside 1..2^20 or a beta
   that is not positive and finite; MC_ENOMEM if the device buffer (5 * n_beta
   doubles, kept by the context for later calls) cannot be allocated. */
mc_status mc_thermo(mc_ctx *ctx, int32_t size_idx, const double *beta_host, int32_t n_beta, double *out_host);

/* mc_thermo for callers that cannot allocate device memory (code under HIP
   graph capture aside, tight serving loops, harnesses that forbid
   allocation): the same computation and results, bit for bit, with the
   inverse temperatures and results staged in a static device array of the
   library instead of a buffer the context allocates.  The array holds
   MC_THERMO_STATIC_MAX_BETAS inverse temperatures (5 doubles each, 320 KB);
   each GPU the library runs on holds one until the process ends, its address
   looked up when a context is created on that GPU.  Every call on a GPU
   shares that GPU's array, which keeps the last call's contents: calls that
   overlap on one GPU (several contexts, streams or threads) race, and must be
   serialised by the caller.  Allocates nothing: no hipMalloc or hipFree.
   Synchronising.  MC_EINVAL for a null pointer, n_beta outside
   1..MC_THERMO_STATIC_MAX_BETAS or a beta that is not positive and finite. */
#define MC_THERMO_STATIC_MAX_BETAS 8192
mc_status mc_thermo_static(mc_ctx *ctx, int32_t size_idx, const double *beta_host, int32_t n_beta,
                           double *out_host);

/* Progress of the weight recursion of one size (synchronising; each output may
   be NULL): updates done, first update (1-based) whose histogram was flat (0 =
   none yet), flatness of the last update, configurations kept by the joints
   before the last update. */
mc_status mc_get_progress(mc_ctx *ctx, int32_t size_idx, int32_t *updates, int32_t *first_flat, int32_t *last_flat,
                          int64_t *retained_last);

/* Launch configuration.  Chains are independent, so the configuration
   changes speed only, never results.
   mc_set_chains_per_block: chains per workgroup (1..64, one chain per lane of
   the workgroup's first wave) of one size.
   mc_get_launch: chains per workgroup, kernel kind and whether the sizes run
   batched in one persistent launch (all sizes keep lattices in LDS).  Kinds:
     0  lattice and per-level thresholds in LDS, one wave
     1  lattice in LDS, thresholds read from global memory, one wave
     2  lattice rows streamed from global memory, one wave
     3  generic bit-by-bit kernel for L not among the compiled sizes (4, 8,
        12, 16, 20, 24, 32, 40, 48, 64, 100, 128, 256)
     4  as 0, random words made by three producer waves of the workgroup, two
        sites decided per threshold read (L <= 64)
     5  L = 128, 256: lattice rows streamed from global memory one word at a
        time, per-bin thresholds in LDS, producer waves as in 4
     6  as 5 with the per-bin thresholds read from global memory
     7  as 4 with four lanes per chain: each step decides four sites, the
        second pair under each of the four outcomes of the first
        (8 <= L <= 64, at most 16 chains per workgroup)
     8  as 5 with four lanes per chain as in 7 (L = 100, 128, 256, at most 32
        chains per workgroup: up to two consumer waves of 16 chains)
     9  as 8 with the per-bin thresholds read from global memory.
   By default 8 <= L <= 64 run kind 7 with 16 chains per workgroup, and
   L = 100, 128, 256 kind 8 (else 9) with 16 chains per workgroup, or 32 when there
   are more chains than 16 per compute unit.  mc_set_chains_per_block picks
   kind 7 (L <= 64) or 8 / 9 (L >= 100) where the chains per workgroup allow
   it (at most 16, resp. 32), else kind 4 or 5 / 6.
   mc_set_launch: the kernel kind (0..9) and chains per workgroup of one
   size, for a kind other than the one mc_set_chains_per_block would pick
   (kind 4 or a one-wave kind at 16 chains, say); MC_EINVAL when that kind
   cannot run the size at that many chains per workgroup (the configuration
   is then unchanged).
   mc_autotune: times probe_sweeps sweeps of every size on copies of the chain
   state for 16, 32 and 64 chains per workgroup, with the producer/consumer
   kinds and with the one-wave kinds, and keeps the fastest; when the sizes
   run batched it then times the batched launch itself for 16, 32 and 64
   chains per workgroup everywhere and (up to six sizes) every mix of each
   size's fastest plan and its widest one, and keeps the fastest
   (chains_per_block_out: n_sizes values, nullable).  The chains are not
   advanced.  The setters fail with MC_ESTATE while graphs of the context
   exist. */
mc_status mc_set_chains_per_block(mc_ctx *ctx, int32_t size_idx, int32_t chains_per_block);
mc_status mc_set_launch(mc_ctx *ctx, int32_t size_idx, int32_t kind, int32_t chains_per_block);
mc_status mc_get_launch(mc_ctx *ctx, int32_t size_idx, int32_t *chains_per_block, int32_t *kind, int32_t *batched);
mc_status mc_autotune(mc_ctx *ctx, int64_t probe_sweeps, int32_t *chains_per_block_out);

/* A captured sequence of n_iters whole iterations of the method for every
   size of the context -- mc_run_chains, mc_join and mc_update_weights, as in
   Sec. 4.2 -- replayed with one call (HIP graph).  The counters of the chains
   live in device memory, so every replay continues the recursion.  The
   buffers (host arrays of n_sizes device pointers, shapes as for the single
   calls) are baked into the graph and must stay allocated; hist_dev must hold
   zeros before the first replay (each update leaves them zeroed).  A graph
   can only be created and launched right after a weight update (or at the
   start).  mode: the joint's mode (0, 1 or 2), as for mc_join.  Destroy
   graphs before their context.
   Errors: MC_EINVAL, MC_ESTATE, MC_EOVERFLOW (n_chains * n_sweeps >= 2^31;
   at launch, also when a replay would pass the 2^32 sweep or joint-round
   counters of the random words). */
typedef struct mc_graph mc_graph;
mc_status mc_graph_create(mc_ctx *ctx, int64_t n_sweeps, int32_t n_iters, void *const *trace_dev,
                          int32_t *const *hist_dev, int32_t *const *cut_dev, int32_t mode, mc_graph **out);
mc_status mc_graph_launch(mc_ctx *ctx, mc_graph *graph);
mc_status mc_graph_destroy(mc_graph *graph);

/* ------------------------------------------------------------------------
   Learned initial weight.  A fully connected fp32 network with inputs
   (1/L, e = E/N), two tanh layers of 64 units and a linear output f that
   approximates the entropy per site ln g(E)/N.  A converged multicanonical
   weight gives its training targets: a flat histogram means D(E) w(E) is
   constant (Sec. 3.1), so ln g = -ln w + const, the constant fixed by
   sum_E g(E) = 2^N.  For a new lattice size the network proposes
   ln w = -N f, from which the recursion (eq. new_weight) continues; ln w = 0
   (w^(1) = 1) remains the fallback.  These calls need no context: they take
   device pointers and a HIP stream and return without waiting, except
   mc_mlp_train with loss_host.
   Parameters: mc_mlp_n_params() floats, laid out W1[64][2] | b1[64] |
   W2[64][64] | b2[64] | W3[64] | b3.  Samples: x [n][2], targets t [n],
   optional sample weights w [n] (NULL = 1).  Loss: sum w (y-t)^2 / sum w.
   workspace: mc_mlp_workspace_bytes(n) bytes of device memory.
   Errors: MC_EINVAL (NULL pointer, n < 1, bad L), MC_EHIP. */
int32_t mc_mlp_n_params(void);
size_t mc_mlp_workspace_bytes(int32_t n);
/* Glorot-uniform weights (Philox words of domain 3, key (seed, 0)), zero biases. */
mc_status mc_mlp_init(float *params_dev, uint32_t seed, void *hip_stream);
/* y_dev [n] = f(x_dev). */
mc_status mc_mlp_forward(const float *params_dev, const float *x_dev, int32_t n, float *y_dev, void *hip_stream);
/* grad_dev [n_params] = d loss / d params; loss_dev (nullable) [1]. */
mc_status mc_mlp_loss_grad(const float *params_dev, const float *x_dev, const float *t_dev, const float *w_dev,
                           int32_t n, float *grad_dev, float *loss_dev, void *workspace_dev, void *hip_stream);
/* `steps` full-batch Adam steps (beta 0.9/0.999, eps 1e-8) at rate lr.
   adam_dev: 2 n_params floats of moment estimates (zeros at the start);
   *step_io: steps taken so far (host, updated); loss_host (nullable): loss
   before the last step (synchronises). */
mc_status mc_mlp_train(float *params_dev, const float *x_dev, const float *t_dev, const float *w_dev, int32_t n,
                       int32_t steps, float lr, float *adam_dev, int32_t *step_io, float *loss_host,
                       void *workspace_dev, void *hip_stream);
/* Training samples of one converged ln w (device, n_bins values): x_dev
   [n_bins][2] = (1/L, e_b) with e_b the energy per site of the centre of bin
   b, t_dev [n_bins] = (-ln w_b + c)/N. */
mc_status mc_mlp_targets(const double *lnW_dev, int32_t L, int32_t bin_shift, float *x_dev, float *t_dev,
                         void *hip_stream);
/* Proposed ln w of a lattice size: lnW_dev [n_bins] = -N f(1/L, e_b). */
mc_status mc_mlp_predict_weights(const float *params_dev, int32_t L, int32_t bin_shift, double *lnW_dev,
                                 void *hip_stream);

/* Statistics of one size for a record of the recursion (synchronising):
   the progress of mc_get_progress, the histogram of the last weight update
   over the bins that hold a reachable level (its total, its smallest bin --
   flatness is 5 n_reach_bins hist_min >= 4 hist_sum -- and the number of such
   bins), the range of ln w over those bins after that update, the last
   joint's chains that kept nothing, its largest cut point and the sum of its
   cut points over the chains that kept something (Algorithm steps 3-5), and
   the device counters (next sweep index, next joint round, seam). */
typedef struct {
    int32_t updates, first_flat, last_flat;
    int32_t n_reach_bins;
    int64_t retained_last;
    int64_t hist_sum, hist_min;
    double lnw_min, lnw_max;
    int32_t join_none, join_cut_max;
    int64_t join_cut_sum;
    uint32_t sweep_index, round_index;
    int32_t seam;
} mc_stats;
mc_status mc_get_stats(mc_ctx *ctx, int32_t size_idx, mc_stats *out);

/* Consistency check of the chains of one size (synchronising): the sweeps
   track each chain's level m = (E + 2N)/4 incrementally (Sec. 4.1, J = 1,
   E = -sum of s_i s_j over the 2N bonds), so each level must equal half the
   number of broken bonds of the chain's lattice.  A kernel recounts them.
   *n_bad (nullable) receives the number of chains that disagree.  Returns
   MC_OK, or MC_EINTERNAL if any chain disagrees (the state is corrupt, by a
   fault of the library or of memory). */
mc_status mc_check_levels(mc_ctx *ctx, int32_t size_idx, int64_t *n_bad);

/* Microbenchmarks of the chip resources that bound the sweep kernels (a
   measurement, not a step of the method; no context).  The method's work is
   integer vector ALU work on strictly serial chains, so the roofline of the
   sweeps is set by the ALU rate of its instruction classes, by LDS, and by
   what one wave issues.  kind:
     0..4  chip-wide rate of independent 32-bit VALU instructions, in
           lane-instructions/s: 0 v_xor_b32, 1 v_mul_lo_u32, 2 v_mul_hi_u32,
           3 v_mad_u64_u32 (the Philox multiply), 4 v_bitop3_b32 (three-input
           xor); 8 one-wave workgroups per SIMD;
     5     chip-wide LDS read bandwidth, bytes/s (16-byte reads, no bank
           conflicts, two 256-thread workgroups per compute unit);
     6     latency of one wave's dependent LDS reads, shader-clock cycles per
           read (including the one instruction that forms the next address);
     7, 8  issue interval of a lone wave, cycles per instruction, for
           dependent (7) and independent (8) simple VALU instructions;
     9..11 cycles per four-site step of the quad sweep step alone (one wave,
           16 chains of L = 32, hashed spins, thresholds and random words; no
           producer waves, barriers or global memory): 9 as the sweeps run
           it, 10 with its six threshold reads taken from the small pair
           table at addresses that do not depend on the level, 11 with the
           thresholds made by arithmetic from the level instead of read.
   iters (1..2^24) scales the work (rows of 32 sites for kinds 9..11).
   out_host[4]: the figure, the seconds of the timed launch (hipEvents), the
   work counted (lane-instructions, bytes, reads, instructions or steps), the
   shader-clock cycles counted (kinds 6..11).
   Allocates and frees its own device buffers; synchronises hip_stream.
   Errors: MC_EINVAL, MC_ENODEV, MC_ENOMEM, MC_EHIP. */
mc_status mc_probe(int32_t kind, int32_t iters, void *hip_stream, double *out_host);

/* Wait for all work of the context. */
mc_status mc_sync(mc_ctx *ctx);

/* Message of the last error on this thread ("" if none). */
const char *mc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MC_H */
