/*
 * muca.h -- C ABI of libmuca: parallel multicanonical (MUCA) sampling of the
 * three-dimensional Blume-Capel model on one AMD Instinct MI355X (gfx950).
 *
 * Method: J. Zierenberg, N. G. Fytas, W. Janke, "Parallel multicanonical study
 * of the three-dimensional Blume-Capel model".
 *   Sec. I, Eq. (1)  model H = -J sum_<ij> s_i s_j + Delta sum_i s_i^2 = E_J + Delta E_Delta,
 *                    s_i in {-1, 0, +1}, L^3 simple cubic lattice, periodic, J = k_B = 1.
 *   Sec. II          multicanonical weights W(E_Delta) at fixed beta replace
 *                    exp(-beta Delta E_Delta); W is adapted iteratively to a flat
 *                    E_Delta histogram (E_Delta is an integer in [0, V]); many
 *                    independent walkers share W and merge their histograms
 *                    (parallel MUCA); time-series reweighting gives canonical
 *                    expectation values at any Delta.
 *   Eq. (FieldDerivative), Eq. (sph)  field derivatives, C(Delta) = d<E_J>/dDelta.
 *
 * Conventions fixed where the paper is silent (identical in the test oracle;
 * the walker index w below is the global one, first_walker + local index):
 *   site i = x + L(y + Lz); colour-major visiting order (even L: colour (x+y+z) mod 2;
 *   odd L: f(t) = t mod 2 for t <= L-2, f(L-1) = 2, colour (f(x)+f(y)+f(z)) mod 3;
 *   colours ascending, then z, y, x ascending); proposal = the b-th (ascending) of the
 *   two other spin values; Philox4x32-10 with key (seed lo32, seed hi32): the attempt
 *   at position p of sweep s of walker w uses word p&3 of block (p>>2, w, s, 0),
 *   b = bit 0, u31 = bits 1..31; initial spin of site i: word i&3 of block
 *   (i>>2, w, 0, 1), s_i = floor(3x / 2^32) - 1; accept iff
 *   (double)u31 < B'[dE_J + 12] * R_d[E_Delta] with B'[k] = 2^31 exp(-beta k),
 *   R_+[E] = exp(lnW[E+1] - lnW[E]), R_-[E] = exp(lnW[E-1] - lnW[E]), R_0 = 1.
 *
 * General rules:
 *   - Every call returns int: MUCA_OK (0) or a negative MUCA_E_* code.  No
 *     exception or abort crosses the ABI.  muca_strerror() describes a code; after
 *     MUCA_E_DEVICE it also carries the HIP error of the failing call.
 *   - Device memory is allocated by the caller (e.g. PyTorch) and borrowed: sizes
 *     come from muca_query_sizes, the pointers must stay valid until muca_free and
 *     are never freed by the library.  Device buffers need 256-byte alignment.
 *   - Host arrays belong to the caller; the library copies from or into them during
 *     the call and keeps no reference.
 *   - All device work of a job is ordered on the caller's HIP stream given to
 *     muca_init.  Calls return after enqueueing, except those marked "synchronises".
 *   - A job must not be used from two threads at once; distinct jobs are independent.
 */
#ifndef MUCA_H
#define MUCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MUCA_OK 0
#define MUCA_E_INVAL (-1)       /* bad argument: L, T, n_walkers, null pointer, range */
#define MUCA_E_UNSUPPORTED (-2) /* valid request the library does not implement */
#define MUCA_E_SIZE (-3)        /* buffer too small / too large for a fixed limit */
#define MUCA_E_STATE (-4)       /* call out of order (e.g. reweight with no recorded data) */
#define MUCA_E_OVERFLOW (-5)    /* a counter would overflow (n_sweeps per call) */
#define MUCA_E_DEVICE (-6)      /* a HIP call failed or a kernel reported an error */

#define MUCA_L_MIN 2
#define MUCA_L_MAX 32
#define MUCA_MAX_SWEEPS_PER_CALL ((int64_t)1 << 40)

/* muca_sweep flags */
#define MUCA_RECORD 1u /* also accumulate the per-bin production sums used by muca_reweight */

typedef struct muca_job muca_job;

typedef struct {
    int32_t L;         /* MUCA_L_MIN..MUCA_L_MAX; V = L^3 */
    double T;          /* temperature > 0, or +INFINITY for beta = 0; beta = 1.0 / T in FP64 */
    int32_t n_walkers; /* >= 1 independent walkers sharing one weight function */
    uint64_t seed;     /* Philox key: k0 = low 32 bits, k1 = high 32 bits */
    int32_t max_delta; /* largest n_delta a muca_reweight call may ask for, 0..65536 */
    int32_t first_walker; /* global index of the job's walker 0 (>= 0): the job holds walkers
                             [first_walker, first_walker + n_walkers) of a larger run with the same
                             seed, so a run split into such sub-jobs (one per device, say) replays
                             exactly the chains of the whole run and its merged histogram is the sum
                             of theirs; 0 for a whole job */
} muca_params;

/* Caller-owned device buffers, sized by muca_query_sizes (bytes, 256-aligned). */
typedef struct {
    void *lattice;      /* spins, n_walkers x Vp int8 (Vp = V rounded up to 16), colour-major order */
    void *walker_state; /* n_walkers x 4 int32: E_J, E_Delta, M, sweeps done (uint32) */
    void *hist;         /* V+1 uint64: E_Delta histogram of the current iteration */
    void *tables;       /* thresholds B'[25], R_-/R_+[V+1], lnW[V+1], neighbour and site tables */
    void *accum;        /* 7 x (V+1) uint64 per-bin production sums: H, SJ, SJJ, S|M|, SM2, SM4 lo, SM4 hi */
    void *obs;          /* reweighting scratch: Delta values, observables, ln P(E_Delta), per-bin sums */
} muca_dev_buffers;

/* Observables of one reweighting point (Sec. II; Eqs. (FieldDerivative), (sph)). */
#define MUCA_N_OBS 15
typedef struct {
    double delta;     /* the crystal field Delta */
    double mean_EJ;   /* <E_J> */
    double mean_ED;   /* <E_Delta> */
    double mean_E;    /* <E_J + Delta E_Delta> */
    double mean_EJ2;  /* <E_J^2> */
    double var_EJ;    /* <E_J^2> - <E_J>^2 */
    double var_ED;    /* <E_Delta^2> - <E_Delta>^2 */
    double C_field;   /* C(Delta) = d<E_J>/dDelta = -beta (<E_J E_Delta> - <E_J><E_Delta>), Eq. (sph) */
    double dC_dDelta; /* dC/dDelta = beta^2 <(E_J - <E_J>)(E_Delta - <E_Delta>)^2> */
    double cV;        /* beta^2 Var(E) / V, E = E_J + Delta E_Delta */
    double mean_absM; /* <|M|> */
    double mean_M2;   /* <M^2> */
    double mean_M4;   /* <M^4> */
    double binder_U4; /* 1 - <M^4> / (3 <M^2>^2); NaN when <M^2> = 0 */
    double edge_weight; /* reweighted probability of the first + last visited E_Delta bin */
} muca_obs;

/* Byte sizes of the six device buffers for params.  Returns MUCA_E_INVAL on bad
 * params.  Any size pointer may be NULL. */
int muca_query_sizes(const muca_params *params, size_t *lattice_bytes, size_t *state_bytes,
                     size_t *hist_bytes, size_t *tables_bytes, size_t *accum_bytes,
                     size_t *obs_bytes);

/* Create a job (steps "init" and "tables", Sec. I-II).  Draws the initial
 * lattices on the device (Philox, counter tag 1), computes E_J, E_Delta, M by
 * full recomputation, zeroes hist and accum, and uploads the threshold tables
 * for lnW_host (V+1 doubles, copied; NULL = flat, lnW = 0).  stream is a
 * hipStream_t (NULL = default stream).  On success *out owns host resources
 * released by muca_free.  Synchronises. */
int muca_init(const muca_params *params, const muca_dev_buffers *buffers, const double *lnW_host,
              void *stream, muca_job **out);

/* Step "sweep" + "measure" (Sec. II): n_sweeps (0..MUCA_MAX_SWEEPS_PER_CALL)
 * sweeps of every walker, V single-spin-flip Metropolis attempts each under
 * exp(-beta E_J) W(E_Delta); after each sweep every walker adds one entry at its
 * E_Delta to hist.  With MUCA_RECORD, the per-bin production sums are added to as
 * well.  Asynchronous on the job's stream. */
int muca_sweep(muca_job *job, int64_t n_sweeps, uint32_t flags);

/* Step "reduce" (Sec. II, parallel MUCA merge): copy the walker-summed histogram
 * (V+1 int64) to hist_host; if reset != 0 zero it on the device afterwards.
 * Synchronises; reports MUCA_E_DEVICE if a kernel flagged an internal error. */
int muca_reduce_hist(muca_job *job, int64_t *hist_host, int32_t reset);

/* Step "update" (Sec. II, iterative weights): lnW[E] -= log(H[E]) where H[E] > 0
 * (plain recursion W <- W / H; muca_set_recursion selects a variant) on the
 * job's weights, then re-upload the threshold tables.
 * hist (V+1, non-negative) is the merged histogram of the
 * iteration; lnW_out (V+1, may be NULL) receives the new weights; flatness_out
 * (may be NULL) receives min_E H[E] / mean_E H[E] over [0, V] of hist.  The
 * production sums are cleared (they belong to the weights they were sampled
 * under).  Host FP64; the upload is asynchronous. */
int muca_update_weights(muca_job *job, const int64_t *hist, double *lnW_out, double *flatness_out);

/* Weight recursion used by muca_update_weights from now on (flags below; 0,
 * the default, is the plain recursion W <- W / H on the visited bins).  The
 * paper adapts W iteratively and cites the multicanonical recursions of Berg
 * and of Janke without printing one (Sec. II); these are the variants:
 *   MUCA_REC_ACCUMULATED: the log-weight differences d(E) = lnW(E+1) - lnW(E)
 *     take the mean of every iteration's estimate d(E) + ln H(E) - ln H(E+1),
 *     weighted by its inverse Poisson variance H(E)H(E+1)/(H(E)+H(E+1)); a
 *     pair with one visited bin takes the plain step; lnW(0) is kept and the
 *     rest rebuilt from the differences.  The accumulated statistics restart
 *     whenever an iteration reaches a bin no earlier iteration did, or leaves
 *     a bin unvisited between the lowest and highest bins visited so far
 *     (walkers that stopped reaching part of the range, e.g. across a
 *     first-order barrier, would otherwise leave it with steps too small to
 *     bring them back).
 *   MUCA_REC_EXTRAPOLATE: bins outside the range visited in any iteration so
 *     far continue the mean slope of the last min(8, width) differences inside
 *     it, at each end.
 * Resets the accumulated statistics and the visited range.  MUCA_E_INVAL on
 * unknown flags.  Host only. */
#define MUCA_REC_ACCUMULATED 1u
#define MUCA_REC_EXTRAPOLATE 2u
int muca_set_recursion(muca_job *job, uint32_t flags);

/* Replace the job's weights by lnW (V+1 finite doubles) and re-upload the
 * thresholds; clears the production sums.  For weights carried over from an
 * earlier run, a checkpoint, or a start tilted towards some Delta. */
int muca_set_weights(muca_job *job, const double *lnW);

/* State of the weight recursion, for an exact checkpoint of a job iterating
 * with MUCA_REC_ACCUMULATED or MUCA_REC_EXTRAPOLATE: kacc (V doubles, the
 * accumulated pair weights) and seen (V+1 bytes, 1 for the bins any iteration
 * since muca_set_recursion has reached).  get copies them out; set restores
 * them (after muca_set_recursion, muca_set_window and muca_set_weights, which
 * reset them).  Either pointer may be NULL (not copied).  MUCA_E_INVAL on a
 * negative or non-finite kacc or a seen byte other than 0 or 1. */
int muca_get_recursion_state(const muca_job *job, double *kacc, uint8_t *seen);
int muca_set_recursion_state(muca_job *job, const double *kacc, const uint8_t *seen);

/* Copy the job's current weights (V+1 doubles) to lnW_out. */
int muca_get_weights(const muca_job *job, double *lnW_out);

/* Order the job's later device work on stream (a hipStream_t, NULL = default
 * stream) instead of the one given to muca_init, e.g. to move a job created
 * on one stream into a batch on another.  Waits for the work already queued on
 * the old stream.  A job in a batch must not change stream while the batch
 * exists. */
int muca_set_stream(muca_job *job, void *stream);

/* Confine the job's walkers to the E_Delta window [lo, hi] (0 <= lo < hi <=
 * V).  The paper iterates the weights over all of [0, V] (Sec. II); a job
 * that only needs Delta in some range (its canonical E_Delta distributions
 * lie inside the window) converges over the window alone:
 *   - moves that would leave the window are rejected (R_+[hi] = R_-[lo] = 0),
 *     so inside it the chain is the Metropolis chain of exp(-beta E_J) W(E_Delta)
 *     restricted to the window;
 *   - the weights outside become walls falling by kappa = 12 beta + ln(2V) + 1
 *     per bin away from the window: a walker outside accepts every move towards
 *     it and enters in a few sweeps, then stays;
 *   - muca_update_weights updates, extrapolates and measures flatness over the
 *     window only (entries outside it are not used) and rebuilds the walls;
 *     muca_set_weights keeps the window and rebuilds the walls;
 *   - MUCA_RECORD adds to the production sums only measurements inside it.
 * The window [0, V] (the default) changes nothing.  Clears the recursion
 * statistics and the production sums.  MUCA_E_INVAL on a bad range. */
int muca_set_window(muca_job *job, int32_t lo, int32_t hi);

/* The job's window (lo, hi); either pointer may be NULL. */
int muca_get_window(const muca_job *job, int32_t *lo, int32_t *hi);

/* Step "reweight" (Sec. II time-series reweighting; Eqs. (FieldDerivative),
 * (sph)): canonical expectation values at (beta, delta[k]) for k < n_delta from
 * the production sums and the weights they were recorded under.  Runs one
 * device block per Delta.  n_delta in 1..max_delta.  MUCA_E_STATE when nothing
 * has been recorded.  Synchronises. */
int muca_reweight(muca_job *job, const double *delta, int32_t n_delta, muca_obs *out);

/* Reweighting of caller-supplied per-bin sums (e.g. a jackknife subset of the
 * production measurements, Sec. II-III): sums (5 x (V+1) int64: H, SJ, SJJ,
 * S|M|, SM2) and sm4 (2 x (V+1) uint64: low, high words of the 128-bit sums of
 * M^4), recorded under the job's current weights.  Otherwise as muca_reweight.
 * MUCA_E_STATE if sums holds no measurement.  Synchronises. */
int muca_reweight_sums(muca_job *job, const int64_t *sums, const uint64_t *sm4, const double *delta,
                       int32_t n_delta, muca_obs *out);

/* Reweighted distribution of E_Delta at (beta, delta) from the production
 * histogram and the weights it was recorded under (Sec. II: the measurements
 * of bin E carry weight exp(-beta delta E) / W(E)): lnP_out[E] = ln P(E) for
 * E = 0..V, normalised to sum 1, -INFINITY where nothing was recorded.  One
 * device block.  MUCA_E_STATE when nothing has been recorded.  Synchronises. */
int muca_reweight_hist(muca_job *job, double delta, double *lnP_out);

/* Reweighted distribution of E_Delta as muca_reweight_hist, from a
 * caller-supplied histogram hist (V+1 non-negative int64, e.g. the production
 * histogram with one time block left out, for jackknife errors of the
 * equal-height field, Sec. II-III) recorded under the job's current weights.
 * MUCA_E_INVAL on a negative entry, MUCA_E_STATE if hist holds no entry.
 * Uses the job's obs buffer as staging.  Synchronises. */
int muca_reweight_hist_sums(muca_job *job, const int64_t *hist, double delta, double *lnP_out);

/* Copy walker state to the host: spins (n_walkers x V int8, site-indexed
 * i = x + L(y + Lz), may be NULL) and state (n_walkers x 4 int64: E_J, E_Delta,
 * M, sweeps done; may be NULL).  Synchronises. */
int muca_read_state(muca_job *job, int8_t *spins, int64_t *state);

/* Overwrite walker state from the host (checkpoint resume).  spins as in
 * muca_read_state with values in {-1,0,1}; state's E_J, E_Delta, M must equal
 * the energies of the spins (not checked on the device) and sweeps done < 2^32.
 * Synchronises. */
int muca_write_state(muca_job *job, const int8_t *spins, const int64_t *state);

/* Copy the production sums to the host: sums (5 x (V+1) int64: H, SJ, SJJ, S|M|,
 * SM2) and sm4 (2 x (V+1) uint64: low words, then high words of the 128-bit
 * sums of M^4); either may be NULL.  Synchronises. */
int muca_read_accum(muca_job *job, int64_t *sums, uint64_t *sm4);

/* Zero the production sums.  Asynchronous. */
int muca_reset_accum(muca_job *job);

/* Overwrite the production sums from the host (checkpoint resume), in the
 * layout muca_read_accum returns; marks them as recorded when they hold any
 * measurement.  Synchronises. */
int muca_write_accum(muca_job *job, const int64_t *sums, const uint64_t *sm4);

/* Launch shape of the sweep kernel (results do not depend on it):
 * waves_per_walker in {1, 2, 4} (64, 128 or 256 lanes cooperate on one walker),
 * blocks_per_lane in {1, 2} (4 or 8 consecutive sites per lane per pass),
 * lds_tables: 1 = thresholds and neighbour table in LDS, 0 = read through the
 * caches, -1 = automatic; packing: 1 = lattices held in LDS as 2-bit codes (a
 * quarter of the bytes, one more field extract per neighbour read; needs
 * blocks_per_lane 1), 0 = one byte per site, -1 = automatic (packed when that
 * raises the blocks resident on a compute unit).  The histogram of the
 * iteration is kept in LDS unless that lowers the resident blocks.
 * MUCA_E_INVAL on a bad value, MUCA_E_SIZE if the shape needs more LDS than a
 * block may use. */
int muca_set_launch(muca_job *job, int32_t waves_per_walker, int32_t blocks_per_lane,
                    int32_t lds_tables, int32_t packing);

/* Current launch shape (packing as resolved: 0 or 1) and its LDS bytes per
 * block.  Any pointer may be NULL. */
int muca_get_launch(const muca_job *job, int32_t *waves_per_walker, int32_t *blocks_per_lane,
                    int32_t *lds_tables, int32_t *packing, int32_t *lds_bytes);

/* Diagnostics: when enabled, the sweep kernel counts passes (colour-class
 * groups of sites handled together), rounds of the exact E_Delta resolution,
 * and accepted moves.  Off by default; a few atomics per pass. */
int muca_set_stats(muca_job *job, int32_t enable);

/* out[0] = passes, out[1] = fixed-point decision rounds (summed over the
 * waves that share a walker), out[2] = accepted moves, summed over walkers
 * since the last reset (3 int64).  reset != 0 zeroes them afterwards.
 * Synchronises. */
int muca_read_stats(muca_job *job, int64_t *out, int32_t reset);

/* ---------------------------------------------------------------------------
 * Batched persistent launch: the walkers of several jobs (different L, T and
 * weights) swept by one kernel launch.  Blocks pull work tiles (walkers of one
 * job) from a device work counter, heaviest jobs first, so jobs of uneven size
 * share the device.  Every walker runs exactly the chain it runs under
 * muca_sweep on its own job: results do not depend on the batching.
 * ------------------------------------------------------------------------- */
typedef struct muca_batch muca_batch;

/* Device bytes the batch needs for its job table and work list (for jobs[0..n)). */
int muca_batch_query_size(muca_job *const *jobs, int32_t n_jobs, size_t *bytes);

/* Create a batch over n_jobs (>= 1) distinct jobs created on the same device
 * with the same stream.  dev_buffer: caller-owned device memory of at least
 * muca_batch_query_size bytes, 256-aligned, valid until muca_batch_free.  The
 * jobs stay owned by the caller and must outlive the batch.  Synchronises. */
int muca_batch_create(muca_job *const *jobs, int32_t n_jobs, void *dev_buffer, size_t bytes,
                      muca_batch **out);

/* Launch shape of the batched kernel (results do not depend on it):
 * waves_per_walker in {0, 1, 2, 4}, blocks_per_lane in {1, 2}; blocks <= 0
 * fills the device (occupancy query); packing as for muca_set_launch.  The
 * default is one wave per walker for every job (two or four when four
 * lattices of the largest job do not fit in the LDS of a block even packed)
 * and automatic packing.  waves_per_walker 0 picks per job: four waves per
 * walker for the jobs whose walkers would otherwise set the length of the
 * launch (large lattices, few waves in the batch), one for the rest; it pays
 * while the weights are smooth.  MUCA_E_SIZE if the lattice slots of the
 * largest tile do not fit in LDS. */
int muca_batch_set_launch(muca_batch *batch, int32_t waves_per_walker, int32_t blocks_per_lane,
                          int32_t blocks, int32_t packing);

/* The launch shape in use: the waves per walker of each job's tiles
 * (waves_per_walker[k] for the k-th job passed to muca_batch_create, so an
 * array of n_jobs), the Philox blocks per lane, the packing (0 or 1) and the
 * LDS bytes per block.  Any pointer may be NULL.  MUCA_E_INVAL for a NULL
 * batch. */
int muca_batch_get_launch(const muca_batch *batch, int32_t *waves_per_walker, int32_t *blocks_per_lane,
                          int32_t *packing, int32_t *lds_bytes);

/* n_sweeps (0..MUCA_MAX_SWEEPS_PER_CALL) sweeps of every walker of every job in
 * the batch, in one persistent launch per at most 2^26 sweeps; flags as for
 * muca_sweep.  Each job's histogram (and production sums with MUCA_RECORD) is
 * added to as by muca_sweep.  Asynchronous on the jobs' stream. */
int muca_batch_sweep(muca_batch *batch, int64_t n_sweeps, uint32_t flags);

/* Asynchronous iterations.  Every job's histogram is merged and its weights
 * updated by the host between iterations (Sec. II); batches on different
 * streams iterate independently, so the jobs of a short-lattice batch need
 * not wait for those of a long one.  submit: muca_batch_sweep, then mark the
 * batch's completion point on its stream (returns at once).  poll: *done = 1
 * when everything submitted to the batch so far has finished, else 0; never
 * blocks.  finish: wait for it.  MUCA_E_DEVICE on a failed launch. */
int muca_batch_submit(muca_batch *batch, int64_t n_sweeps, uint32_t flags);
int muca_batch_poll(muca_batch *batch, int32_t *done);
int muca_batch_finish(muca_batch *batch);

/* Release the batch's host resources (waits for queued work).  NULL ignored. */
void muca_batch_free(muca_batch *batch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the batched
 * sweep of muca_batch_create + muca_batch_sweep in one call, in the default
 * launch shape of muca_batch_create, with the job table, the work list and the
 * work counter in a static device array owned by the library instead of a
 * caller buffer.  The array holds MUCA_STATIC_MAX_JOBS jobs and
 * MUCA_STATIC_MAX_TILES tiles (a tile is the walkers of one block: 4 walkers of
 * one job at one wave each, or 2 or 1 when 4 lattices do not fit in LDS), so
 * at least 65536 walkers: 540 KiB per device, held until the process ends.  Its device address is taken once per device when the first job is
 * created there (muca_init).  jobs: n_jobs distinct jobs created on one device
 * with one stream; n_sweeps and flags as for muca_batch_sweep, with the same
 * results.  The call allocates nothing; it copies the job table from host
 * memory the library owns and waits for the previous call's copy first.
 * Every call on a device shares that device's array and rewrites it: calls
 * that overlap on one device (two streams, or two threads) race.
 * MUCA_E_SIZE beyond the limits, MUCA_E_INVAL on a bad list, MUCA_E_DEVICE if
 * the array's address could not be taken.  Asynchronous on the jobs' stream. */
#define MUCA_STATIC_MAX_JOBS 256
#define MUCA_STATIC_MAX_TILES 65536
int muca_batch_sweep_static(muca_job *const *jobs, int32_t n_jobs, int64_t n_sweeps, uint32_t flags);

/* Host-only: flatness min / mean of hist[lo..hi] (inclusive bins, 0 <= lo <= hi),
 * the convergence measure of the weight iteration restricted to a window of
 * E_Delta; 0 when the window holds no entries. */
int muca_flatness(const int64_t *hist, int32_t lo, int32_t hi, double *flatness_out);

/* Host-only: the threshold tables of the acceptance rule for (L, T, lnW) and
 * the window [lo, hi] (0, V: none): Bp (25), Rp (V+1) and Rm (V+1) doubles.
 * Used to check that the tables are bitwise identical to an independent
 * implementation on the same host. */
int muca_host_tables(int32_t L, double T, const double *lnW, int32_t lo, int32_t hi, double *Bp, double *Rp,
                     double *Rm);

/* Host-only: replace lnW (V+1 doubles) outside the window [lo, hi] by the walls
 * muca_set_window uses. */
int muca_host_walls(int32_t L, double T, int32_t lo, int32_t hi, double *lnW);

/* Host-only: the colour-major visiting order, order[p] = site index (V int32). */
int muca_host_order(int32_t L, int32_t *order);

/* Human-readable description of an error code (static storage; thread-local
 * detail for MUCA_E_DEVICE). */
const char *muca_strerror(int code);

/* Release the job's host resources.  Waits for the job's queued work first.
 * NULL is ignored.  The caller's device buffers are not touched. */
void muca_free(muca_job *job);

#ifdef __cplusplus
}
#endif

#endif /* MUCA_H */
