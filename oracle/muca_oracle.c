/*
 * Reference (oracle) implementation of parallel multicanonical sampling of the
 * three-dimensional Blume-Capel model, after Zierenberg, Fytas and Janke,
 * "Parallel multicanonical study of the three-dimensional Blume-Capel model".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the GPU path: its Philox
 * generator, its lattice helpers, its threshold tables, its sweep and its
 * weight recursion are all written here, plainly and slowly.
 *
 * Everything is sequential and in the order the method states it: one walker
 * after another (threads only split the independent walkers), one site visit
 * after another, one Philox block evaluated per site visit.
 *
 * Conventions (the paper is silent on these; each is restated at the function
 * that uses it):
 *   site index      i = x + L*(y + L*z), periodic neighbours x+-1, y+-1, z+-1
 *   colour-major    visiting order (even L: 2 colours, odd L: 3 colours)
 *   proposal        sigma' = b-th of the two other values, ascending
 *   random numbers  Philox4x32-10, key (seed lo, seed hi),
 *                   sweep draw counter (p>>2, w, s, 0), word p&3,
 *                   initial spins counter (i>>2, w, 0, 1), word i&3
 *   acceptance      (double)u31 < B'[dEJ+12] * R_d[E_Delta]
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the definition in Salmon, Moraes, Dror and Shaw,      */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two  */
/* 32x32->64 multiplications, each round followed by a Weyl bump of the key. */
/* ------------------------------------------------------------------------ */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One 32-bit draw: word `word` of the Philox block at counter (c0,c1,c2,c3). */
static uint32_t orc_draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         unsigned word)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[word & 3u];
}

/* ------------------------------------------------------------------------ */
/* Lattice: L^3 simple cubic, periodic boundaries (Sec. I, Eq. (1)).          */
/* ------------------------------------------------------------------------ */
static int orc_site(int L, int x, int y, int z) { return x + L * (y + L * z); }

/* Colour of a site.  Even L: (x+y+z) mod 2.  Odd L: with f(t) = t mod 2 for
 * t <= L-2 and f(L-1) = 2, colour (f(x)+f(y)+f(z)) mod 3.  Both are proper
 * colourings of the periodic lattice: neighbours never share a colour. */
static int orc_colour(int L, int x, int y, int z)
{
    if (L % 2 == 0)
        return (x + y + z) % 2;
    int fx = (x == L - 1) ? 2 : x % 2;
    int fy = (y == L - 1) ? 2 : y % 2;
    int fz = (z == L - 1) ? 2 : z % 2;
    return (fx + fy + fz) % 3;
}

int orc_num_colours(int L) { return (L % 2 == 0) ? 2 : 3; }

/* Colour-major visiting order: for colour c ascending, then z, y, x ascending,
 * the sites of colour c.  order[p] = site index visited at position p. */
void orc_order(int L, int32_t *order)
{
    int p = 0;
    for (int c = 0; c < orc_num_colours(L); c++)
        for (int z = 0; z < L; z++)
            for (int y = 0; y < L; y++)
                for (int x = 0; x < L; x++)
                    if (orc_colour(L, x, y, z) == c)
                        order[p++] = orc_site(L, x, y, z);
}

/* Sum of the six neighbour spins of site i (with multiplicity when L == 2). */
static int orc_neighbour_sum(int L, const int8_t *s, int i)
{
    int x = i % L, y = (i / L) % L, z = i / (L * L);
    int xp = (x + 1) % L, xm = (x + L - 1) % L;
    int yp = (y + 1) % L, ym = (y + L - 1) % L;
    int zp = (z + 1) % L, zm = (z + L - 1) % L;
    return s[orc_site(L, xp, y, z)] + s[orc_site(L, xm, y, z)] +
           s[orc_site(L, x, yp, z)] + s[orc_site(L, x, ym, z)] +
           s[orc_site(L, x, y, zp)] + s[orc_site(L, x, y, zm)];
}

/* Energies of Eq. (1) with J = 1: E_J = -sum over the 3V forward bonds of
 * sigma_i sigma_j, E_Delta = sum sigma_i^2; also the magnetisation M. */
void orc_energies(int L, const int8_t *s, int64_t out[3])
{
    int64_t ej = 0, ed = 0, m = 0;
    for (int z = 0; z < L; z++)
        for (int y = 0; y < L; y++)
            for (int x = 0; x < L; x++) {
                int i = orc_site(L, x, y, z);
                int si = s[i];
                ej -= si * (s[orc_site(L, (x + 1) % L, y, z)] +
                            s[orc_site(L, x, (y + 1) % L, z)] +
                            s[orc_site(L, x, y, (z + 1) % L)]);
                ed += si * si;
                m += si;
            }
    out[0] = ej; out[1] = ed; out[2] = m;
}

/* Initial lattice of walker w: sigma_i = floor(3 x / 2^32) - 1 with x the word
 * i&3 of the Philox block at counter (i>>2, w, 0, 1).  Spins are site-indexed. */
void orc_init_walker(int L, uint64_t seed, uint32_t w, int8_t *s)
{
    int V = L * L * L;
    for (int i = 0; i < V; i++) {
        uint32_t x = orc_draw(seed, (uint32_t)(i >> 2), w, 0u, 1u, (unsigned)(i & 3));
        s[i] = (int8_t)((int)(((uint64_t)x * 3u) >> 32) - 1);
    }
}

/* ------------------------------------------------------------------------ */
/* Acceptance thresholds (Sec. II: MUCA weights W(E_Delta) at fixed beta).    */
/* Metropolis acceptance of sigma -> sigma' is                                */
/*   min(1, exp(-beta dE_J) W(E_Delta + d) / W(E_Delta)),  d = sigma'^2-sigma^2*/
/* compared against u31 / 2^31.  Scaled by 2^31:                              */
/*   Bp[k+12] = 2^31 exp(-beta k)             k = dE_J in [-12, 12]           */
/*   Rp[E]    = exp(lnW[E+1] - lnW[E])         (d = +1), Rp[V] = 0            */
/*   Rm[E]    = exp(lnW[E-1] - lnW[E])         (d = -1), Rm[0] = 0            */
/* ------------------------------------------------------------------------ */
void orc_tables(int V, double beta, const double *lnW, double *Bp, double *Rp, double *Rm)
{
    for (int k = -12; k <= 12; k++)
        Bp[k + 12] = ldexp(exp(-(beta * (double)k)), 31);
    for (int E = 0; E <= V; E++) {
        Rp[E] = (E < V) ? exp(lnW[E + 1] - lnW[E]) : 0.0;
        Rm[E] = (E > 0) ? exp(lnW[E - 1] - lnW[E]) : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Window (a job's Delta range confines its walkers to E_Delta in [lo, hi];  */
/* the paper runs MUCA over all of [0, V], so this is an added reading).     */
/* Inside the window the chain is the same Metropolis chain with the moves   */
/* that would leave the window rejected: R_+[hi] = 0, R_-[lo] = 0.  Outside   */
/* it the weights are walls falling by kappa = 12 beta + ln(2V) + 1 per bin */
/* away from the window.  A walker outside then accepts every proposal that  */
/* moves it towards the window (|dE_J| <= 12 and the wall factor e^kappa     */
/* beats exp(-12 beta)), and accepts one away from it with probability at   */
/* most 1/(2eV), which outweighs the at most V proposals per sweep that the  */
/* entropy of E_Delta offers in that direction: it enters in a few sweeps,  */
/* and once inside it never leaves.  With [lo, hi] = [0, V] nothing changes. */
/* ------------------------------------------------------------------------ */
void orc_tables_window(int V, double beta, const double *lnW, int lo, int hi, double *Bp, double *Rp,
                       double *Rm)
{
    orc_tables(V, beta, lnW, Bp, Rp, Rm);
    Rp[hi] = 0.0;
    Rm[lo] = 0.0;
}

void orc_window_walls(int V, double beta, int lo, int hi, double *lnW)
{
    double kappa = 12.0 * beta + log(2.0 * (double)V) + 1.0;
    for (int E = hi + 1; E <= V; E++)
        lnW[E] = lnW[hi] - kappa * (double)(E - hi);
    for (int E = lo - 1; E >= 0; E--)
        lnW[E] = lnW[lo] - kappa * (double)(lo - E);
}

/* Decision for one proposal: one double product, one compare. */
int orc_accept(uint32_t u31, int dEJ, int d, int E, const double *Bp, const double *Rp,
               const double *Rm)
{
    double threshold = Bp[dEJ + 12];
    if (d > 0)
        threshold = threshold * Rp[E];
    else if (d < 0)
        threshold = threshold * Rm[E];
    return (double)u31 < threshold;
}

/* Proposal: the b-th (ascending) of the two values in {-1,0,+1} other than s. */
static int orc_propose(int s, int b)
{
    int others[2];
    int n = 0;
    for (int v = -1; v <= 1; v++)
        if (v != s)
            others[n++] = v;
    return others[b];
}

/* ------------------------------------------------------------------------ */
/* Walkers, sweeps and measurements.                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int L, V;
    uint64_t seed;
    const int32_t *order;
    const double *Bp, *Rp, *Rm;
    int64_t n_sweeps;
    int record;
    int8_t *spins;          /* n_walkers x V, site-indexed */
    int64_t *state;         /* n_walkers x 4: E_J, E_Delta, M, sweeps done */
    int w_begin, w_end;     /* local walker indices [w_begin, w_end) */
    int w_first;            /* global index of local walker 0 */
    int lo, hi;             /* window: production sums record only E_Delta in [lo, hi] */
    int64_t *hist;          /* V+1, private to the thread */
    int64_t *acc;           /* 5 x (V+1): H, SJ, SJJ, SA, SM2, private */
    unsigned __int128 *sm4; /* V+1, private */
} orc_task;

/* One sweep of walker w: V single-spin-flip Metropolis attempts in
 * colour-major order.  The attempt at position p of sweep s uses word p&3 of
 * the Philox block at counter (p>>2, w, s, 0): bit 0 picks the proposal, the
 * upper 31 bits are the uniform u31. */
static void orc_sweep(const orc_task *t, int w, int8_t *s, int64_t *st)
{
    uint32_t sweep = (uint32_t)st[3];
    for (int p = 0; p < t->V; p++) {
        int i = t->order[p];
        uint32_t x = orc_draw(t->seed, (uint32_t)(p >> 2), (uint32_t)w, sweep, 0u,
                              (unsigned)(p & 3));
        int b = (int)(x & 1u);
        uint32_t u31 = x >> 1;
        int old = s[i];
        int proposed = orc_propose(old, b);
        int h = orc_neighbour_sum(t->L, s, i);
        int dEJ = -(proposed - old) * h;
        int d = proposed * proposed - old * old;
        if (orc_accept(u31, dEJ, d, (int)st[1], t->Bp, t->Rp, t->Rm)) {
            s[i] = (int8_t)proposed;
            st[0] += dEJ;
            st[1] += d;
            st[2] += proposed - old;
        }
    }
    st[3] += 1;
}

/* After every sweep each walker adds one entry at its E_Delta to the
 * histogram; when recording, also to the per-bin sums of E_J, E_J^2, |M|,
 * M^2 and M^4 used by time-series reweighting (Sec. II). */
static void *orc_worker(void *arg)
{
    orc_task *t = (orc_task *)arg;
    for (int w = t->w_begin; w < t->w_end; w++) {
        int8_t *s = t->spins + (size_t)w * t->V;
        int64_t *st = t->state + 4 * (size_t)w;
        for (int64_t n = 0; n < t->n_sweeps; n++) {
            orc_sweep(t, t->w_first + w, s, st);
            int64_t ej = st[0], ed = st[1], m = st[2];
            t->hist[ed] += 1;
            if (t->record && ed >= t->lo && ed <= t->hi) {
                int64_t am = m < 0 ? -m : m;
                t->acc[0 * (t->V + 1) + ed] += 1;
                t->acc[1 * (t->V + 1) + ed] += ej;
                t->acc[2 * (t->V + 1) + ed] += ej * ej;
                t->acc[3 * (t->V + 1) + ed] += am;
                t->acc[4 * (t->V + 1) + ed] += m * m;
                t->sm4[ed] += (unsigned __int128)(m * m) * (unsigned __int128)(m * m);
            }
        }
    }
    return NULL;
}

/* Run n_sweeps sweeps of walkers [w_first, w_first + n_walkers) (global
 * walker indices; spins and state hold these walkers in order) under the weights lnW at
 * inverse temperature beta, confined to the window [lo, hi] of E_Delta
 * (0, V: no window).  hist (V+1) and, when record != 0, acc
 * (5 x (V+1): H, SJ, SJJ, SA, SM2) and sm4_lo/sm4_hi (V+1 each, the low and
 * high 64 bits of the 128-bit sums of M^4) are added to, not cleared; the
 * production sums take only measurements inside the window (a walker still
 * on its way in is not in equilibrium under the walls).
 * Walkers are independent between weight updates, so they are split over
 * n_threads threads (0: one per online core); integer sums do not depend on
 * the split.  Returns the number of threads used. */
int orc_run(int L, double beta, uint64_t seed, int w_first, int n_walkers, int8_t *spins, int64_t *state,
            const double *lnW, int lo, int hi, int64_t n_sweeps, int record, int64_t *hist, int64_t *acc,
            uint64_t *sm4_lo, uint64_t *sm4_hi, int n_threads)
{
    int V = L * L * L;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * V);
    double *Bp = (double *)malloc(sizeof(double) * 25);
    double *Rp = (double *)malloc(sizeof(double) * (V + 1));
    double *Rm = (double *)malloc(sizeof(double) * (V + 1));
    orc_order(L, order);
    orc_tables_window(V, beta, lnW, lo, hi, Bp, Rp, Rm);

    if (n_threads <= 0)
        n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads > n_walkers)
        n_threads = n_walkers;
    if (n_threads < 1)
        n_threads = 1;

    orc_task *tasks = (orc_task *)calloc((size_t)n_threads, sizeof(orc_task));
    pthread_t *tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    for (int k = 0; k < n_threads; k++) {
        orc_task *t = &tasks[k];
        t->L = L; t->V = V; t->seed = seed; t->order = order;
        t->Bp = Bp; t->Rp = Rp; t->Rm = Rm;
        t->n_sweeps = n_sweeps; t->record = record; t->w_first = w_first;
        t->lo = lo; t->hi = hi;
        t->spins = spins; t->state = state;
        t->w_begin = (int)((int64_t)n_walkers * k / n_threads);
        t->w_end = (int)((int64_t)n_walkers * (k + 1) / n_threads);
        t->hist = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
        t->acc = (int64_t *)calloc(5 * ((size_t)V + 1), sizeof(int64_t));
        t->sm4 = (unsigned __int128 *)calloc((size_t)V + 1, sizeof(unsigned __int128));
    }
    for (int k = 1; k < n_threads; k++)
        pthread_create(&tids[k], NULL, orc_worker, &tasks[k]);
    orc_worker(&tasks[0]);
    for (int k = 1; k < n_threads; k++)
        pthread_join(tids[k], NULL);

    for (int k = 0; k < n_threads; k++) {
        orc_task *t = &tasks[k];
        for (int E = 0; E <= V; E++) {
            hist[E] += t->hist[E];
            if (record) {
                for (int q = 0; q < 5; q++)
                    acc[q * (V + 1) + E] += t->acc[q * (V + 1) + E];
                unsigned __int128 total =
                    ((unsigned __int128)sm4_hi[E] << 64) | (unsigned __int128)sm4_lo[E];
                total += t->sm4[E];
                sm4_lo[E] = (uint64_t)total;
                sm4_hi[E] = (uint64_t)(total >> 64);
            }
        }
        free(t->hist); free(t->acc); free(t->sm4);
    }
    free(tasks); free(tids); free(order); free(Bp); free(Rp); free(Rm);
    return n_threads;
}

/* Initialise walkers [w_first, w_first + n_walkers): spins from
 * orc_init_walker, energies by full recomputation, sweep counter 0. */
void orc_init(int L, uint64_t seed, int w_first, int n_walkers, int8_t *spins, int64_t *state)
{
    int V = L * L * L;
    for (int w = 0; w < n_walkers; w++) {
        int8_t *s = spins + (size_t)w * V;
        orc_init_walker(L, seed, (uint32_t)(w_first + w), s);
        int64_t e[3];
        orc_energies(L, s, e);
        state[4 * (size_t)w + 0] = e[0];
        state[4 * (size_t)w + 1] = e[1];
        state[4 * (size_t)w + 2] = e[2];
        state[4 * (size_t)w + 3] = 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Weight recursion (Sec. II: W(E_Delta) adapted iteratively towards a flat   */
/* E_Delta histogram; the plain multicanonical recursion W <- W / H):         */
/*   lnW[E] <- lnW[E] - log(H[E])  for H[E] > 0, unchanged otherwise.         */
/* Flatness min_E H[E] / mean_E H[E] over the full range [0, V] is returned.   */
/* ------------------------------------------------------------------------ */
double orc_update_weights(int V, const int64_t *hist, double *lnW)
{
    int64_t total = 0, least = hist[0];
    for (int E = 0; E <= V; E++) {
        total += hist[E];
        if (hist[E] < least)
            least = hist[E];
    }
    for (int E = 0; E <= V; E++)
        if (hist[E] > 0)
            lnW[E] = lnW[E] - log((double)hist[E]);
    if (total == 0)
        return 0.0;
    return (double)least / ((double)total / (double)(V + 1));
}

/* ------------------------------------------------------------------------ */
/* Faster weight convergence (the recursion variants the paper cites, after  */
/* Berg's multicanonical recursion as presented by Janke; not printed in the */
/* paper, so the exact form below is this implementation's reading).         */
/*                                                                          */
/* flags & 1 (accumulated): the log-weight differences d(E) = lnW(E+1) -     */
/*   lnW(E) of neighbouring bins are updated with the statistics of every    */
/*   iteration so far, each iteration weighted by its significance           */
/*   k_n(E) = H(E) H(E+1) / (H(E) + H(E+1)):                                 */
/*     K(E) += k_n(E);  d(E) += (k_n(E) / K(E)) * (log H(E) - log H(E+1))   */
/*   for pairs with both bins visited.  A pair with one bin visited takes the */
/*   plain step (the empty side counts as one entry); a pair with none keeps  */
/*   d.  The weights are rebuilt from d upwards from bin 0, whose value is    */
/*   kept.  With K starting at 0 the first iteration is the plain recursion.  */
/*   K restarts at 0 whenever an iteration reaches a bin no earlier one did: */
/*   the estimates gathered before were sampled while part of the range was  */
/*   out of reach, and averaging them in freezes their bias (measured: at    */
/*   T < 1.1 it multiplied the iterations to flatness several times).  K     */
/*   also restarts when an iteration leaves a bin unvisited between the      */
/*   lowest and highest bins visited so far: the walkers stopped reaching    */
/*   part of the range, the few entries near its edge barely move d against  */
/*   the statistics gathered before, and the visited part would keep         */
/*   shrinking (measured on windows spanning a first-order transition).      */
/* flags & 2 (extrapolate): bins outside the range [lo, hi] of bins visited  */
/*   in any iteration so far continue the slope of lnW over the last         */
/*   k = min(8, hi - lo) bins inside the range, at each end.                  */
/* kacc (V doubles) and seen (V+1 bytes) carry the state between iterations. */
/* With a window [lo, hi] (see orc_tables_window) all of this acts on the    */
/* bins of the window only, as if it were the whole range: the flatness is   */
/* min / mean over [lo, hi], the pairs are those inside it, the visited range */
/* and its extrapolation stay inside it, and the walls outside are rebuilt  */
/* from the new edge values.                                                */
/* Returns the flatness of hist over [lo, hi].                               */
/* ------------------------------------------------------------------------ */
double orc_update_weights_window(int V, double beta, int lo, int hi, const int64_t *hist, double *lnW,
                                 unsigned flags, double *kacc, uint8_t *seen)
{
    int64_t total = 0, least = hist[lo];
    int any_seen = 0, reached_new = 0;
    for (int E = lo; E <= hi; E++)
        if (seen[E])
            any_seen = 1;
    for (int E = lo; E <= hi; E++) {
        total += hist[E];
        if (hist[E] < least)
            least = hist[E];
        if (hist[E] > 0) {
            if (!seen[E])
                reached_new = 1;
            seen[E] = 1;
        }
    }
    /* a bin left unvisited inside the range visited so far */
    int lost = 0;
    {
        int slo = -1, shi = -1;
        for (int E = lo; E <= hi; E++)
            if (seen[E]) {
                if (slo < 0)
                    slo = E;
                shi = E;
            }
        for (int E = slo; slo >= 0 && E <= shi; E++)
            if (hist[E] == 0)
                lost = 1;
    }
    if ((flags & 1u) && any_seen && (reached_new || lost))
        for (int E = lo; E < hi; E++)
            kacc[E] = 0.0;
    if (flags & 1u) {
        double *d = (double *)malloc(sizeof(double) * (size_t)(V > 0 ? V : 1));
        for (int E = lo; E < hi; E++)
            d[E] = lnW[E + 1] - lnW[E];
        for (int E = lo; E < hi; E++) {
            int64_t a = hist[E], b = hist[E + 1];
            if (a > 0 && b > 0) {
                double ha = (double)a, hb = (double)b;
                double k = ha * hb / (ha + hb);
                kacc[E] = kacc[E] + k;
                d[E] = d[E] + (k / kacc[E]) * (log(ha) - log(hb));
            } else if (a > 0) {
                d[E] = d[E] + log((double)a);
            } else if (b > 0) {
                d[E] = d[E] - log((double)b);
            }
        }
        for (int E = lo; E < hi; E++)
            lnW[E + 1] = lnW[E] + d[E];
        free(d);
    } else {
        for (int E = lo; E <= hi; E++)
            if (hist[E] > 0)
                lnW[E] = lnW[E] - log((double)hist[E]);
    }
    if (flags & 2u) {
        int slo = -1, shi = -1;
        for (int E = lo; E <= hi; E++)
            if (seen[E]) {
                if (slo < 0)
                    slo = E;
                shi = E;
            }
        if (slo >= 0 && shi > slo) {
            int k = shi - slo < 8 ? shi - slo : 8;
            double s_hi = (lnW[shi] - lnW[shi - k]) / (double)k;
            double s_lo = (lnW[slo + k] - lnW[slo]) / (double)k;
            for (int E = shi + 1; E <= hi; E++)
                lnW[E] = lnW[shi] + (double)(E - shi) * s_hi;
            for (int E = slo - 1; E >= lo; E--)
                lnW[E] = lnW[slo] - (double)(slo - E) * s_lo;
        }
    }
    orc_window_walls(V, beta, lo, hi, lnW);
    if (total == 0)
        return 0.0;
    return (double)least / ((double)total / (double)(hi - lo + 1));
}

/* The recursion over the whole range [0, V] (no window, no walls). */
double orc_update_weights_ex(int V, const int64_t *hist, double *lnW, unsigned flags, double *kacc,
                             uint8_t *seen)
{
    return orc_update_weights_window(V, 0.0, 0, V, hist, lnW, flags, kacc, seen);
}
