/*
 * mc_oracle.c -- plain, serial, fp64 CPU oracle of the parallel multicanonical
 * Markov-chain method of Sugihara, Higo and Nakamura, "Parallelization of
 * Markov Chain Generation and its Application to the Multicanonical Method"
 * (arXiv 0812.2964).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant with
 * the GPU library: everything below is written from the paper and from the
 * published definitions it relies on.
 *
 * Everything is deliberately unoptimised: spins are one int8 per site, the
 * neighbour sum is taken with modular index arithmetic, and every random word
 * is a fresh Philox call.
 *
 * What is followed where:
 *   - chain generation (Metropolis, one configuration per sweep): Sec. 2,
 *     Algorithm step 2; the Metropolis rule is the one named in Sec. 4.2.
 *   - the joint between chains: Sec. 2, Algorithm steps 1-5 and Sec. 4.2.
 *   - the weight recursion w <- w/h (h > 0): Sec. 3.1, eq. (new_weight), kept in
 *     logarithms as Sec. 4.2 prescribes.
 *   - the Ising energy: Sec. 4.1 (periodic L x L square lattice, J = 1).
 *
 * Readings of the paper that are not spelled out there (each is listed in the
 * design notes of the repository):
 *   R1 one "configuration" is the lattice after one sweep of N single-spin
 *      Metropolis attempts in typewriter order (site j = y*L + x, x fastest);
 *   R2 level m = (E + 2N)/4 in [0, N]; bin b = m >> bin_shift;
 *   R3 acceptance of a move with log-weight change d: u <= tau(d) with u a
 *      uniform 32-bit word and tau(d) = 2^32-1 for d >= 0, otherwise
 *      min(floor(exp(d) * 2^32), 2^32-1) (probability (tau+1)/2^32);
 *   R4 random words: Philox4x32-10 with counter (j>>2, a, c, dom), key
 *      (seed, L), word j&3; dom 0 = sweep (a = global sweep index), 1 = initial
 *      spins (a = 0), 2 = joint test (a = round, j = 0-based position);
 *   R5 exp and log are the deterministic Cody-Waite/Taylor forms below, so that
 *      the thresholds are reproducible bit for bit on any IEEE-754 machine;
 *   R6 the seam is only the energy of the last kept configuration; a chain
 *      whose configurations are all rejected keeps its own lattice and the seam
 *      is carried unchanged.  The very first seam is "none": the first chain of
 *      the first round is kept whole.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).                        */
/* One round: (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2,                          */
/*            c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0).                 */
/* The key is bumped by the Weyl constants between rounds.                   */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Reading R4: the word used for position j of stream (dom, a) of chain c. */
uint32_t orc_uniform(uint32_t seed, int32_t L, uint32_t dom, uint32_t a, uint32_t c, uint32_t j)
{
    uint32_t ctr[4] = {j >> 2, a, c, dom};
    uint32_t key[2] = {seed, (uint32_t)L};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[j & 3u];
}

/* ------------------------------------------------------------------------- */
/* Reading R5: deterministic exp and log in IEEE binary64, using only +,-,*, */
/* /, fma, rint, frexp and ldexp.                                            */
/* exp: Cody-Waite reduction x = k ln2 + r (ln 2 split into a rounded head   */
/*      and its rounded remainder), Taylor polynomial of degree 13 in r.     */
/* log: h = f 2^e with f in [sqrt(1/2), sqrt(2)), s = (f-1)/(f+1),            */
/*      ln f = 2 s sum_{i>=0} s^(2i)/(2i+1) truncated after s^22.            */
/* ------------------------------------------------------------------------- */
static double orc_ln2_head(void) { return 0x1.62e42fefa39efp-1; }  /* RN(ln 2)            */
static double orc_ln2_tail(void) { return 0x1.abc9e3b39803fp-56; } /* RN(ln 2 - RN(ln 2)) */
static double orc_inv_ln2(void) { return 0x1.71547652b82fep+0; }  /* RN(1/ln 2)          */

double orc_exp(double x)
{
    if (x < -745.0) return 0.0;
    /* Taylor coefficients 1/i!, each the correctly rounded quotient 1/i!
       (i! is exact in binary64 for i <= 13). */
    double coef[14];
    double fact = 1.0;
    for (int i = 0; i < 14; ++i) {
        if (i > 0) fact *= (double)i;
        coef[i] = 1.0 / fact;
    }
    double k = rint(x * orc_inv_ln2());
    double r = fma(-k, orc_ln2_head(), x);
    r = fma(-k, orc_ln2_tail(), r);
    double p = coef[13];
    for (int i = 12; i >= 0; --i) p = fma(p, r, coef[i]);
    return ldexp(p, (int)k);
}

double orc_log(int64_t h)
{
    /* h >= 1 (a histogram count). */
    int e;
    double f = frexp((double)h, &e);
    if (f < 0x1.6a09e667f3bcdp-1) { /* RN(sqrt(1/2)) */
        f = f * 2.0;
        e = e - 1;
    }
    double s = (f - 1.0) / (f + 1.0);
    double z = s * s;
    double q = 1.0 / 23.0;
    for (int i = 10; i >= 1; --i) q = fma(q, z, 1.0 / (double)(2 * i + 1));
    double s2 = s + s;
    double lnf = fma(s2 * z, q, s2);
    double de = (double)e;
    return fma(de, orc_ln2_head(), fma(de, orc_ln2_tail(), lnf));
}

/* Reading R3. */
uint32_t orc_threshold(double d)
{
    if (d >= 0.0) return 0xFFFFFFFFu;
    if (d < -23.0) return 0u; /* exp(-23) 2^32 < 1: the floor is 0 there anyway */
    double v = floor(orc_exp(d) * 4294967296.0);
    if (v >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)v;
}

int orc_accept(uint32_t tau, uint32_t u) { return u <= tau ? 1 : 0; }

/* ------------------------------------------------------------------------- */
/* The 2D Ising model of Sec. 4.1: H = -sum_<ij> s_i s_j, periodic L x L.     */
/* Each bond is counted once, as (site, right neighbour) and (site, down).    */
/* ------------------------------------------------------------------------- */
int64_t orc_energy(int32_t L, const int8_t *s)
{
    int64_t e = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            int j = y * L + x;
            int right = y * L + (x + 1) % L;
            int down = ((y + 1) % L) * L + x;
            e -= (int64_t)s[j] * (s[right] + s[down]);
        }
    return e;
}

int32_t orc_level_of_energy(int32_t L, int64_t e) { return (int32_t)((e + 2 * (int64_t)L * L) / 4); }

/* Algorithm step 1: random initial configuration, Philox domain 1. */
void orc_init_chain(int32_t L, uint32_t seed, uint32_t c, int8_t *s)
{
    int N = L * L;
    for (int j = 0; j < N; ++j) s[j] = (orc_uniform(seed, L, 1u, 0u, c, (uint32_t)j) >> 31) ? 1 : -1;
}

/* Reachable levels of the periodic lattice (even L): every m in [0, N] except
   m = 1 and m = N - 1 (E = -2N + 4 would need a single broken bond). */
int orc_level_reachable(int32_t L, int32_t m)
{
    int N = L * L;
    if (m < 0 || m > N) return 0;
    return (m != 1 && m != N - 1) ? 1 : 0;
}

/* Threshold table for a fixed weight: T[m*5 + a], a = dm + 2 in 0..4 the change
   of level a flip causes.  Entries whose target lies outside [0, N] cannot be
   reached and are 0. */
void orc_tabulate(int32_t L, int32_t bin_shift, const double *lnW, uint32_t *T)
{
    int N = L * L;
    for (int m = 0; m <= N; ++m)
        for (int a = 0; a < 5; ++a) {
            int mt = m + a - 2;
            if (mt < 0 || mt > N) {
                T[m * 5 + a] = 0u;
                continue;
            }
            double d = lnW[mt >> bin_shift] - lnW[m >> bin_shift];
            T[m * 5 + a] = orc_threshold(d);
        }
}

/* Algorithm step 2 for one chain: n_sweeps sweeps starting at global sweep
   index g0.  After every sweep the configuration's energy is recorded as E/4
   in trace[k] and counted in hist[bin]. *m_io is the current level. */
void orc_sweeps(int32_t L, uint32_t seed, int32_t bin_shift, uint32_t c, int8_t *s, int32_t *m_io,
                uint32_t g0, int64_t n_sweeps, const uint32_t *T, int32_t *trace, int64_t *hist)
{
    int N = L * L;
    int32_t m = *m_io;
    for (int64_t k = 0; k < n_sweeps; ++k) {
        uint32_t g = g0 + (uint32_t)k;
        for (int j = 0; j < N; ++j) {
            int x = j % L, y = j / L;
            int right = y * L + (x + 1) % L;
            int left = y * L + (x + L - 1) % L;
            int down = ((y + 1) % L) * L + x;
            int up = ((y + L - 1) % L) * L + x;
            int h = s[right] + s[left] + s[down] + s[up];
            int dE = 2 * s[j] * h; /* energy change of flipping site j */
            int dm = dE / 4;
            uint32_t tau = T[m * 5 + dm + 2];
            uint32_t u = orc_uniform(seed, L, 0u, g, c, (uint32_t)j);
            if (orc_accept(tau, u)) {
                s[j] = (int8_t)-s[j];
                m += dm;
            }
        }
        if (trace) trace[k] = m - N / 2;
        if (hist) hist[m >> bin_shift] += 1;
    }
    *m_io = m;
}

/* Algorithm steps 3-5 for one round r over p chains.  trace holds p rows of
   M values E/4.  *sigma_io is the seam level (-1 = none).  cut[c] is the
   1-based first kept position of chain c or -1.  Kept configurations are
   added to H; their number to *retained.
   order: NULL for the chains in index order, else the chain taken at each
   position (a permutation of 0..p-1, the energy ordering of Sec. 2's remark;
   see orc_energy_order).  The test of chain c's k-th configuration draws its
   word from (round r, chain c_off + c, position k), whatever its place in the
   order: c_off is the global index of chain 0 when a run is split into blocks
   of chains, each joined in turn from the seam the block before ended with.
   mode 0: detailed balance at the joints (the paper's method);
   mode 1: every chain kept whole (the naive splice compared in Sec. 5). */
void orc_join(int32_t L, int32_t bin_shift, uint32_t seed, uint32_t c_off, int32_t p, int64_t M,
              const int32_t *trace, const double *lnW, int32_t *sigma_io, uint32_t r, int32_t mode, const int32_t *order,
              int32_t *cut, int64_t *H, int64_t *retained)
{
    int N = L * L;
    int32_t sigma = *sigma_io;
    for (int t = 0; t < p; ++t) {
        const int c = order ? order[t] : t;
        const int32_t *tr = trace + (int64_t)c * M;
        int64_t kstar = -1;
        if (mode == 1 || sigma < 0) {
            kstar = 0;
        } else {
            for (int64_t k = 0; k < M; ++k) {
                int32_t mk = tr[k] + N / 2;
                double d = lnW[mk >> bin_shift] - lnW[sigma >> bin_shift];
                uint32_t u = orc_uniform(seed, L, 2u, r, c_off + (uint32_t)c, (uint32_t)k);
                if (orc_accept(orc_threshold(d), u)) {
                    kstar = k;
                    break;
                }
            }
        }
        if (kstar >= 0) {
            for (int64_t k = kstar; k < M; ++k) H[(tr[k] + N / 2) >> bin_shift] += 1;
            *retained += M - kstar;
            sigma = tr[M - 1] + N / 2;
            cut[c] = (int32_t)(kstar + 1);
        } else {
            cut[c] = -1;
        }
    }
    *sigma_io = sigma;
}

/* The energy ordering of the chains for one round (the paper suggests
   ordering the nodes by the energies of their configurations to raise the
   acceptance at the joints, Sec. 2, and leaves the rule open).  Reading: a
   greedy chain of nearest levels.  first[c] and last[c] are the levels of
   chain c's first and last configuration of the round.  Starting from the
   seam sigma (or, with no seam, from chain 0 placed first), each position
   takes the chain not yet placed whose first level is nearest to the last
   level of the chain placed before it (or to the seam); ties go to the lower
   level, then to the lower chain index.  O(p^2), for the test-suite. */
void orc_energy_order(int32_t p, const int32_t *first, const int32_t *last, int32_t sigma, int32_t *order)
{
    char *used = (char *)calloc((size_t)p, 1);
    int t = 0;
    int32_t ref = sigma;
    if (ref < 0 && p > 0) {
        order[t++] = 0;
        used[0] = 1;
        ref = last[0];
    }
    for (; t < p; ++t) {
        int best = -1;
        for (int c = 0; c < p; ++c) {
            if (used[c]) continue;
            if (best < 0) {
                best = c;
                continue;
            }
            int dc = abs(first[c] - ref), db = abs(first[best] - ref);
            if (dc < db || (dc == db && first[c] < first[best])) best = c;
        }
        order[t] = best;
        used[best] = 1;
        ref = last[best];
    }
    free(used);
}

/* Eq. (new_weight) in logarithms: ln w <- ln w - ln h where h > 0.
   Flatness (the stopping test of the iteration): over the bins that hold a
   reachable level, 5 * n * min h >= 4 * sum h.  Returns the flat flag. */
int orc_update(int32_t L, int32_t bin_shift, const int64_t *H, double *lnW)
{
    int N = L * L;
    int n_bins = (N >> bin_shift) + 1;
    for (int b = 0; b < n_bins; ++b)
        if (H[b] > 0) lnW[b] = lnW[b] - orc_log(H[b]);
    int64_t n = 0, mn = -1, sum = 0;
    for (int b = 0; b < n_bins; ++b) {
        int reach = 0;
        for (int m = b << bin_shift; m < ((b + 1) << bin_shift) && m <= N; ++m) reach |= orc_level_reachable(L, m);
        if (!reach) continue;
        n += 1;
        sum += H[b];
        if (mn < 0 || H[b] < mn) mn = H[b];
    }
    return (n > 0 && sum > 0 && 5 * n * mn >= 4 * sum) ? 1 : 0;
}

/* One round for p chains (chains c0 .. c0+p-1), each continuing from its own
   state: spins[p][N], m[p].  Wraps orc_sweeps chain by chain. */
void orc_run_round(int32_t L, uint32_t seed, int32_t bin_shift, uint32_t c0, int32_t p, int64_t M, uint32_t g0,
                   const double *lnW, int8_t *spins, int32_t *m, int32_t *trace, int64_t *hist)
{
    int N = L * L;
    uint32_t *T = (uint32_t *)malloc(sizeof(uint32_t) * 5 * (size_t)(N + 1));
    orc_tabulate(L, bin_shift, lnW, T);
    for (int i = 0; i < p; ++i)
        orc_sweeps(L, seed, bin_shift, c0 + (uint32_t)i, spins + (int64_t)i * N, m + i, g0, M, T,
                   trace ? trace + (int64_t)i * M : NULL, hist);
    free(T);
}
