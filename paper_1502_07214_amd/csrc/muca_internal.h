// Internal declarations shared by the host side (muca_host.cpp) and the device
// kernels (muca_kernels.hip) of libmuca.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace muca {

constexpr int kBlock = 256;          // threads per block of every kernel: 4 wave64
constexpr int kMaxClasses = 3;       // colours of the visiting order
constexpr int kLdsFixed = 384;       // B'[32] doubles + scan scratch at the start of LDS
constexpr int kMaxSweepsPerLaunch = 1 << 26;
constexpr int kMaxCachedPasses = 4;  // passes per sweep whose neighbour positions stay in registers
constexpr int kRPad = 8;             // threshold-table entries padded below E = 0 and above E = V (>= sites per lane - 1)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Everything that depends only on L: sizes of the device buffers and offsets of
// the sub-tables inside the tables buffer.
struct Layout {
    int L, V, Vp, C;
    int cls[kMaxClasses + 1];  // colour class c covers positions [cls[c], cls[c+1])
    int n_walkers, max_delta;
    size_t lattice_bytes, state_bytes, hist_bytes, tables_bytes, accum_bytes, obs_bytes;
    size_t off_bp, off_r, off_lnw, off_nb, off_nb2, off_site;  // byte offsets inside tables
    size_t off_obs_lnp, off_obs_sums;                 // byte offsets inside obs
};

// Arguments of the sweep kernel.
struct SweepArgs {
    int8_t *lattice;               // n_walkers x Vp, colour-major positions
    int32_t *wstate;               // n_walkers x 4: E_J, E_Delta, M, sweeps done
    unsigned long long *hist;      // V+1
    const double *bp;              // 25 (+pad) thresholds 2^31 exp(-beta k)
    const double *r;               // (V+1+2*kRPad) x 2: [E+kRPad][0] = R_-, [E+kRPad][1] = R_+
    const uint16_t *nb;            // 6 x Vp neighbour positions
    const uint16_t *nb2;           // the same, doubled (packed lattices: bit offset of a 2-bit code)
    unsigned long long *acc;       // 7 x (V+1) production sums
    int *err;                      // device error word (the tail of the hist buffer)
    unsigned long long *stats;     // null, or [passes, rounds, accepted moves]
    int V, Vp, n_walkers, n_classes;
    int cls[kMaxClasses + 1];
    int n_pass;                    // > 0: a sweep is exactly these passes (blocks_per_lane 1)
    int pass_p0[kMaxCachedPasses], pass_p1[kMaxCachedPasses], pass_jbase[kMaxCachedPasses];
    unsigned pass_sync;            // bit k: synchronise after pass k (end of a colour class)
    uint32_t k0, k1;
    int rec_lo, rec_hi;            // production sums record only E_Delta in [rec_lo, rec_hi]
    int w0;                        // global index of walker 0 (Philox counter word 1)
    int n_sweeps;
    int lds_hist;                  // 1: histogram in LDS, flushed at the end
    int lds_off_hist, lds_off_lat, lds_off_r, lds_off_nb;
};

struct InitArgs {
    int8_t *lattice;
    int32_t *wstate;
    const uint16_t *nb;
    const uint16_t *site;
    int V, Vp, n_walkers;
    uint32_t k0, k1;
    int w0;                          // global index of walker 0
};

struct LogHistArgs {
    const unsigned long long *hist;  // V+1 counts
    const double *lnw;               // V+1
    double *lnp;                     // V+1 output
    int V;
    double bd;                       // beta * Delta
};

struct ReweightArgs {
    const unsigned long long *acc;  // 7 x (V+1)
    const double *lnw;              // V+1
    const double *delta;            // n_delta
    double *obs;                    // n_delta x 15
    int V;
    double beta;
};

// One job of a batched launch (device-resident table).
struct BatchJob {
    int8_t *lattice;
    int32_t *wstate;
    unsigned long long *hist;
    const double *bp;
    const double *r;
    const uint16_t *nb;
    const uint16_t *nb2;
    unsigned long long *acc;
    int *err;
    int V, Vp, n_walkers, n_classes;
    int cls[kMaxClasses + 1];
    uint32_t k0, k1;
    int rec_lo, rec_hi;      // production sums record only E_Delta in [rec_lo, rec_hi]
    int w0;                  // global index of walker 0
    int lds_tables;          // 1: thresholds and neighbour table staged in LDS for this job's tiles
    int wpw;                 // waves per walker of this job's tiles (1 or 4) in a per-job launch
};

struct BatchArgs {
    const BatchJob *jobs;
    const int2 *tiles;       // (job, first walker), heaviest first
    int n_tiles;
    unsigned *counter;       // work counter, zero at launch
    int n_sweeps;
    int lds_off_lat;         // LDS offset of the lattice slots (sized for the largest job)
    int lds_off_tab;         // LDS offset of the staged tables (jobs with lds_tables)
};

// Launchers (muca_kernels.hip).  Return the hipError_t of the launch.
hipError_t launch_init(const InitArgs &a, hipStream_t s);
// pack: lattices as 2-bit codes in LDS (blocks_per_lane 1 only)
hipError_t launch_sweep(const SweepArgs &a, int waves_per_walker, int blocks_per_lane, bool record,
                        bool lds_tables, bool pack, size_t lds_bytes, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_reweight(const ReweightArgs &a, int n_delta, hipStream_t s);
hipError_t launch_log_hist(const LogHistArgs &a, hipStream_t s);
// blocks <= 0: as many blocks as fit on the device at once
hipError_t launch_batch(const BatchArgs &b, int wpw, int bpl, bool record, bool pack, size_t lds, int blocks,
                        hipStream_t s);

}  // namespace muca
