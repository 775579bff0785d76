// Device kernels of libmuca for gfx950 (CDNA4, wave64).
//
// The sweep kernel runs the multicanonical Markov chain of the Blume-Capel model
// (Sec. II of the paper: single-site Metropolis under exp(-beta E_J) W(E_Delta))
// with several lanes cooperating on one walker without changing the chain:
//
//  * Sites are visited in colour-major order.  Inside one colour class no two
//    sites are neighbours, so every lane can evaluate its sites' neighbour sums,
//    proposals, Philox words and E_J changes at once.
//  * The only sequential coupling inside a class is E_Delta: the acceptance of
//    a move that creates or removes a vacancy reads W at the walker's current
//    E_Delta.  It is resolved exactly by a fixed-point iteration: each site
//    guesses the E_Delta it will see, decides, a walker-wide prefix sum of the
//    accepted E_Delta steps gives new guesses, and the loop stops when no guess
//    changes.  Iteration k fixes at least the first k sites of the chain, so it
//    ends after at most (sites in the pass + 1) rounds.  When several waves
//    share a walker, each wave iterates its own chunk without barriers and
//    the waves exchange only chunk totals between such inner iterations.
//  * Lattices live in LDS in colour-major position order, as one int8 per site
//    or (PACK) as 2-bit two's-complement codes, four sites per byte, a quarter
//    of the LDS (more resident walkers when lattices bound occupancy, at one
//    extra field extract per neighbour read).  A lane owns 4 consecutive
//    positions (one Philox block) per group, so spin writes are whole dwords
//    (int8) or bytes (packed) with no atomics.  In HBM lattices are always
//    int8; a packed launch packs them on the way in and unpacks them on the
//    way out.  Thresholds B', R_+-, and the neighbour table sit in LDS when
//    they fit, else are read through L1/L2.
//  * Histograms: one LDS atomic per walker per sweep, flushed to HBM with one
//    64-bit atomic per nonzero bin at the end of the launch (when the histogram
//    fits in LDS next to the lattices; otherwise, and in batched launches, one
//    64-bit HBM atomic per walker per sweep).
#include <hip/hip_runtime.h>

#include "muca_internal.h"
#include "muca_philox.h"

namespace muca {

// ---------------------------------------------------------------------------
// Wave64 cross-lane helpers (DPP row shifts and row broadcasts of GFX9).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned wave_incl_sum(unsigned x)
{
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

__device__ __forceinline__ unsigned wave_total(unsigned incl)
{
    return (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// min(max(x, 0), hi) in one instruction.
__device__ __forceinline__ int clamp0(int x, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return r;
}

// 2-bit codes of a packed lattice: site p is the sign-extended field at bit
// 2p mod 32 of dword p / 16 (-1 = 0b11, 0 = 0b00, +1 = 0b01).  The packed
// neighbour table holds 2p, whose low five bits are that field's offset.
__device__ __forceinline__ int code_field(unsigned word, unsigned off2)
{
    return __builtin_amdgcn_sbfe((int)word, off2, 2u);
}

// 16 int8 spins -> one dword of 2-bit codes, and back.
__device__ __forceinline__ unsigned pack16(uint4 v)
{
    const unsigned w[4] = {v.x, v.y, v.z, v.w};
    unsigned out = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) out |= ((w[i] >> (8 * t)) & 3u) << (2 * (4 * i + t));
    return out;
}

__device__ __forceinline__ uint4 unpack16(unsigned x)
{
    unsigned w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        unsigned d = 0u;
#pragma unroll
        for (int t = 0; t < 4; ++t) d |= ((unsigned)code_field(x, 2u * (4 * i + t)) & 0xffu) << (8 * t);
        w[i] = d;
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Proposal: the b-th (ascending) of the two spin values other than s.  Over
// the six cases that is b - 1, raised by one when s < b (s = -1: b; s = 0:
// 2b - 1; s = +1: b - 1), one compare and an add with carry.
__device__ __forceinline__ int propose(int s, int b)
{
    return b - 1 + (s < b ? 1 : 0);
}

// ---------------------------------------------------------------------------
// One pass: the sites of one colour class whose Philox blocks start at jbase,
// BPL consecutive blocks (4*BPL positions) per lane, GL lanes per walker.
// ---------------------------------------------------------------------------
template <int WPW, int BPL, bool PACK>
struct Walker {
    static constexpr int GL = 64 * WPW;  // lanes per walker
    static constexpr int NS = 4 * BPL;   // sites per lane per pass
    static constexpr int WPB = 4 / WPW;  // walkers per block
    static_assert(!PACK || BPL == 1, "packed lattices are read one Philox block per lane");
    int8_t *lat;                         // this walker's lattice in LDS (PACK: 2-bit codes)
    const double *R;                     // [E][0] = R_-, [E][1] = R_+
    const double *sBp;                   // B' in LDS, mirrored: sBp[12 + k] = B'(dE_J = -k)
    int *sX;                             // [2][4] per-wave exchange words
    int V, wave, lane, slot, wi, lg;
    uint32_t w32, k0, k1;
    uint32_t rk[WPW == 4 ? 20 : 1];      // round keys in vector registers (four waves per walker)
    int ED;                              // E_Delta of the walker (uniform)
    int parity;                          // exchange buffer in use (alternates)
    unsigned myEJ, myM;                  // this lane's accepted E_J and M changes (mod 2^32)
    unsigned rounds, accepted;           // diagnostics of the last pass (this wave)

    // nq[q][dir]: neighbour positions of the 4 sites of block q (two per uint2).
    __device__ __forceinline__ void pass(int P0, int P1, int jbase, uint32_t sweep, const uint2 (&nq)[BPL][6],
                                         int *err)
    {
        const int j1 = ((P1 - 1) >> 2) + 1;
        const int j0 = P0 >> 2;
        const int jb0 = jbase + lg * BPL;
        // ---- independent part: Philox words, neighbour sums, proposals ----
        double u[NS], bp[NS];
        int dd[NS], ndej[NS], dsg[NS], snew[NS], sold[NS];
        bool valid[NS];
        // spins first: their LDS latency overlaps the generator's rounds
        int words[BPL];
        int nbs[BPL][6][4];
#pragma unroll
        for (int q = 0; q < BPL; ++q) {
            const int jb = jb0 + q;
            const int jbc = jb < j1 ? jb : j0;
            if constexpr (PACK) {
                // the four sites of block jbc are byte jbc; neighbours hold 2p
                const unsigned *lat32 = reinterpret_cast<const unsigned *>(lat);
                words[q] = (int)reinterpret_cast<const uint8_t *>(lat)[jbc];
#pragma unroll
                for (int dir = 0; dir < 6; ++dir) {
                    const unsigned x = nq[q][dir].x, y = nq[q][dir].y;
                    nbs[q][dir][0] = code_field(lat32[(x >> 5) & 0x7ffu], x);
                    nbs[q][dir][1] = code_field(lat32[x >> 21], x >> 16);
                    nbs[q][dir][2] = code_field(lat32[(y >> 5) & 0x7ffu], y);
                    nbs[q][dir][3] = code_field(lat32[y >> 21], y >> 16);
                }
            } else {
                words[q] = *reinterpret_cast<const int *>(lat + 4 * jbc);
#pragma unroll
                for (int dir = 0; dir < 6; ++dir) {
                    nbs[q][dir][0] = lat[nq[q][dir].x & 0xffffu];
                    nbs[q][dir][1] = lat[nq[q][dir].x >> 16];
                    nbs[q][dir][2] = lat[nq[q][dir].y & 0xffffu];
                    nbs[q][dir][3] = lat[nq[q][dir].y >> 16];
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // the round keys are cheap to rebuild; keeping them live across
        // passes would only spill them
        // Walkers of four waves (latency-bound: one wave per SIMD) take the
        // round keys from vector registers; the others rebuild them here, as
        // keeping them live across passes would only spill them.
        uint32_t kk0 = 0u, kk1 = 0u;
        if constexpr (WPW != 4) {
            kk0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)k0);
            kk1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)k1);
            asm volatile("" : "+s"(kk0), "+s"(kk1));
        }
#pragma unroll
        for (int q = 0; q < BPL; ++q) {
            const int jb = jb0 + q;
            const bool blk = jb < j1;
            const int jbc = blk ? jb : j0;
            Ctr4 x;
            if constexpr (WPW == 4)
                x = philox10_rk((uint32_t)jbc, w32, sweep, 0u, rk);
            else
                x = philox10((uint32_t)jbc, w32, sweep, 0u, kk0, kk1);
            const int word = words[q];
            int h[4] = {0, 0, 0, 0};
#pragma unroll
            for (int dir = 0; dir < 6; ++dir)
#pragma unroll
                for (int t = 0; t < 4; ++t) h[t] += nbs[q][dir][t];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = 4 * q + t;
                const int p = 4 * jbc + t;
                valid[k] = blk && p >= P0 && p < P1;
                const int s = PACK ? code_field((unsigned)word, 2u * t) : (int)(int8_t)(word >> (8 * t));
                const uint32_t xw = x.v[t];
                const int sn = propose(s, (int)(xw & 1u));
                u[k] = (double)(xw >> 1);
                sold[k] = s;
                snew[k] = sn;
                dsg[k] = sn - s;
                ndej[k] = (sn - s) * h[t];  // -dE_J
                dd[k] = sn * sn - s * s;
                bp[k] = sBp[ndej[k] + 12];
            }
        }
        // ---- sequential part: exact fixed point over E_Delta ----
        // Round 0 decides every site at the walker's E_Delta.  A later round
        // decides each site at the E_Delta implied by the previous decisions of
        // the sites before it (a prefix sum); round t reproduces at least the
        // first t sites of the sequential chain, so the rounds stop at the
        // chain's own result.  Every site does the same work (all threshold
        // loads of a round issue together) and loop exits are wave-uniform.
        // A round's decisions are kept as wave masks (one bit per lane and
        // site): the guesses are a fixed point exactly when no decision that
        // moves E_Delta (a valid site with d != 0) differs from the previous
        // round's, so the test is scalar and needs no guess comparison.
        //
        // With several waves per walker the iteration is two-level.  Each wave
        // iterates its own chunk of the pass to a fixed point, wave-locally and
        // without barriers, from an assumed E_Delta at the chunk's start; the
        // waves then exchange chunk totals once (one barrier), which gives every
        // chunk a new start.  The walker is done when no start changes: every
        // chunk then holds the exact chain from the exact E_Delta before it.
        // Chunk 0 always starts right, so after k exchanges the first k chunks
        // do, and at most WPW + 1 exchanges happen (the first one after round 0).
        static_assert(NS - 1 <= kRPad, "guesses of a lane's later sites must stay inside the padded table");
        int ddv[NS], ridx[NS];
        unsigned acc0 = 0u;  // bit k: the decision of site k where d == 0
        uint64_t SENS[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            ddv[k] = valid[k] ? dd[k] : 0;   // E_Delta step if accepted
            ridx[k] = dd[k] > 0 ? 1 : 0;     // 0: R_-, 1: R_+
            acc0 |= (valid[k] && u[k] < bp[k] ? 1u : 0u) << k;
            SENS[k] = __ballot(ddv[k] != 0);
        }
        bool c[NS];      // this lane's decisions of the last round
        uint64_t S[NS];  // the same as wave masks
        {
            const double rm = R[2 * ED], rpl = R[2 * ED + 1];
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                c[k] = u[k] < bp[k] * (ridx[k] ? rpl : rm);
                S[k] = __ballot(c[k]);
            }
        }
        int ex[NS];
        int laneOff;
        unsigned incl;
        auto scan = [&]() {
            int run = 0;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                ex[k] = run;
                run += c[k] ? ddv[k] : 0;
            }
            incl = wave_incl_sum((unsigned)run);
            laneOff = (int)incl - run;
        };
        // Exchange of chunk totals: start offsets (relative to the walker's
        // E_Delta) of all four waves of the block, and the walkers' totals.
        int off[4] = {0, 0, 0, 0};
        int wsum = 0;
        auto write_spins = [&]() {
#pragma unroll
            for (int q = 0; q < BPL; ++q) {
                const int jb = jb0 + q;
                unsigned nw = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 4 * q + t;
                    const bool a = ddv[k] != 0 ? c[k] : ((acc0 >> k) & 1u) != 0u;
                    if (PACK)
                        nw |= ((unsigned)(a ? snew[k] : sold[k]) & 3u) << (2 * t);
                    else
                        nw |= ((unsigned)(a ? snew[k] : sold[k]) & 0xffu) << (8 * t);
                }
                if (jb < j1) {
                    if (PACK)
                        reinterpret_cast<uint8_t *>(lat)[jb] = (uint8_t)nw;
                    else
                        *reinterpret_cast<unsigned *>(lat + 4 * jb) = nw;
                }
            }
        };
        auto exchange = [&](int (&no)[4]) {
            if (lane == 63) sX[4 * parity + wave] = (int)incl;
            __syncthreads();
            const int4 xw = *reinterpret_cast<const int4 *>(sX + 4 * parity);
            parity ^= 1;
            const int xs[4] = {xw.x, xw.y, xw.z, xw.w};
            int before = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (v % WPW == 0) before = 0;
                no[v] = before;
                before += xs[v];
                if (v / WPW == slot) wsum = before;
            }
        };
        scan();
        if (WPW > 1) exchange(off);
        int base = ED + off[wave];
        // eb: the guess at the lane's first site; site k is guessed at eb + ex[k].
        // One clamp per lane keeps the table reads in bounds (the padding covers
        // ex); at the fixed point every guess is a true E_Delta and untouched.
        int eb = base + laneOff;
        uint64_t moved = 0;
#pragma unroll
        for (int k = 0; k < NS; ++k) moved |= __ballot(eb + ex[k] != ED) & SENS[k];
        // round 0 decided at E_Delta itself: done unless a guess moved
        bool again = moved != 0;
        // the pass's spins in LDS lag its decisions (uniform): with several
        // waves per walker they are written before an exchange whenever they
        // changed, so the exchange that ends the pass also orders them before
        // the next pass reads them
        bool dirty = true;
        unsigned nround = 1;
        int outer = 0;
        const int cap = 64 * NS + 2;
        for (;;) {
            // wave-local fixed point of this chunk from the start `base`
            int inner = 0;
            while (again) {
                double r[NS];
                const int ce = clamp0(eb, V);
#pragma unroll
                for (int k = 0; k < NS; ++k) r[k] = R[2 * (ce + ex[k]) + ridx[k]];
                uint64_t diff = 0;
#pragma unroll
                for (int k = 0; k < NS; ++k) {
                    c[k] = u[k] < bp[k] * r[k];
                    const uint64_t m = __ballot(c[k]);
                    diff |= (m ^ S[k]) & SENS[k];
                    S[k] = m;
                }
                ++nround;
                if (diff == 0) break;
                dirty = true;
                scan();
                eb = base + laneOff;
                if (++inner > cap) {
                    if (lane == 0) atomicOr(err, 1);
                    break;
                }
            }
            if (WPW == 1) {
                wsum = (int)wave_total(incl);
                break;
            }
            if (dirty) {
                write_spins();
                dirty = false;
            }
            int no[4];
            exchange(no);
            const bool stable = no[0] == off[0] && no[1] == off[1] && no[2] == off[2] && no[3] == off[3];
            if (stable) break;  // block-uniform: every wave read the same words
            if (++outer > WPW) {
                if (lane == 0) atomicOr(err, 1);
                break;
            }
            const int shift = __builtin_amdgcn_readfirstlane(no[wave] - off[wave]);
#pragma unroll
            for (int v = 0; v < 4; ++v) off[v] = no[v];
            base += shift;
            eb += shift;
            again = shift != 0;
        }
        const int total = wsum;
        bool acc[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) acc[k] = ddv[k] != 0 ? c[k] : ((acc0 >> k) & 1u) != 0u;
        rounds = nround;
        // ---- apply the accepted moves ----
        if (dirty) write_spins();
        unsigned nacc = 0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            myEJ -= acc[k] ? (unsigned)ndej[k] : 0u;
            myM += acc[k] ? (unsigned)dsg[k] : 0u;
            nacc += acc[k] ? 1u : 0u;
        }
        accepted = nacc;
        ED += total;
    }
};

// ---------------------------------------------------------------------------
// Sweep kernel.
//   WPW: waves per walker (1, 2, 4); BPL: Philox blocks (4 sites) per lane per
//   pass; RECORD: accumulate production sums; LDS_TABLES: R (and, without
//   register caching, the neighbour table) staged in LDS; NCP > 0: a sweep is
//   exactly the NCP passes listed in the arguments and each lane keeps the
//   neighbour positions of its sites in registers for the whole launch.
// ---------------------------------------------------------------------------
template <int WPW, int BPL, bool RECORD, bool LDS_TABLES, int NCP, bool PACK>
__device__ __forceinline__ void sweep_tile(const SweepArgs &a, int walker_base, unsigned char *smem)
{
    using W = Walker<WPW, BPL, PACK>;
    constexpr int LAT_DIV = PACK ? 4 : 1;  // LDS bytes per site: 1 / LAT_DIV

    double *sBp = reinterpret_cast<double *>(smem);
    int *sX = reinterpret_cast<int *>(smem + 256);                   // [8] exchange words
    unsigned *sRed = reinterpret_cast<unsigned *>(smem + 256 + 80);  // [8] per-wave E_J / M sums
    unsigned *sHist = reinterpret_cast<unsigned *>(smem + a.lds_off_hist);
    int8_t *sLat = reinterpret_cast<int8_t *>(smem + a.lds_off_lat);

    const int V = a.V, Vp = a.Vp;
    const int tid = threadIdx.x;
    W wk;
    wk.wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave, held in a scalar register
    wk.lane = tid & 63;
    wk.slot = wk.wave / WPW;
    wk.wi = wk.wave % WPW;
    wk.lg = wk.wi * 64 + wk.lane;
    const int walker = walker_base + wk.slot;
    const bool live = walker < a.n_walkers;
    const int lg = wk.lg, lane = wk.lane, wave = wk.wave, slot = wk.slot;

    // ---- stage tables and lattices in LDS ----
    // mirrored, so that a lane indexes it with -dE_J = (s' - s) h directly
    for (int k = tid; k < 32; k += kBlock) sBp[k] = (k < 25) ? a.bp[24 - k] : 0.0;
    if (a.lds_hist)
        for (int e = tid; e <= V; e += kBlock) sHist[e] = 0u;
    const double *R = a.r + 2 * kRPad;  // R[2E + 1] = R_+(E), R[2E] = R_-(E), E in [-kRPad, V + kRPad]
    const uint16_t *NB = PACK ? a.nb2 : a.nb;  // positions, or twice the positions for packed lattices
    if (LDS_TABLES) {
        double *sR = reinterpret_cast<double *>(smem + a.lds_off_r);
        const int nr = 2 * (V + 1 + 2 * kRPad);
        for (int k = tid; k < nr; k += kBlock) sR[k] = a.r[k];
        R = sR + 2 * kRPad;
        if (NCP == 0) {
            uint16_t *sNB = reinterpret_cast<uint16_t *>(smem + a.lds_off_nb);
            const uint4 *gnb = reinterpret_cast<const uint4 *>(NB);
            uint4 *lnb = reinterpret_cast<uint4 *>(sNB);
            const int nq = (6 * Vp * 2) / 16;
            for (int k = tid; k < nq; k += kBlock) lnb[k] = gnb[k];
            NB = sNB;
        }
    }
    int8_t *lat = sLat + (size_t)slot * (Vp / LAT_DIV);
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.lattice + (size_t)(live ? walker : 0) * Vp);
        if (PACK) {
            unsigned *dst = reinterpret_cast<unsigned *>(lat);
            for (int k = lg; k < Vp / 16; k += W::GL) dst[k] = live ? pack16(src[k]) : 0u;
        } else {
            uint4 *dst = reinterpret_cast<uint4 *>(lat);
            for (int k = lg; k < Vp / 16; k += W::GL) dst[k] = live ? src[k] : make_uint4(0, 0, 0, 0);
        }
    }
    int EJ0 = 0, M0 = 0;
    uint32_t sweep = 0;
    wk.ED = 0;
    if (live) {
        const int4 st = reinterpret_cast<const int4 *>(a.wstate)[walker];
        EJ0 = st.x;
        wk.ED = st.y;
        M0 = st.z;
        sweep = (uint32_t)st.w;
    }
    if (tid < 8) sX[tid] = 0;
    wk.parity = 0;
    wk.lat = lat;
    wk.R = R;
    wk.sBp = sBp;
    wk.sX = sX;
    wk.V = V;
    wk.w32 = (uint32_t)(a.w0 + walker);  // the global walker index keys the chain
    wk.k0 = a.k0;
    wk.k1 = a.k1;
    if constexpr (WPW == 4) philox_round_keys(a.k0, a.k1, wk.rk);
    wk.myEJ = 0u;
    wk.myM = 0u;

    // neighbour positions of this lane's sites, for the cached passes
    uint2 nbc[NCP > 0 ? NCP : 1][BPL][6];
    if (NCP > 0) {
#pragma unroll
        for (int cp = 0; cp < (NCP > 0 ? NCP : 1); ++cp) {
            const int j1 = ((a.pass_p1[cp] - 1) >> 2) + 1;
#pragma unroll
            for (int q = 0; q < BPL; ++q) {
                const int jb = a.pass_jbase[cp] + lg * BPL + q;
                const int jbc = jb < j1 ? jb : (a.pass_p0[cp] >> 2);
#pragma unroll
                for (int dir = 0; dir < 6; ++dir)
                    nbc[cp][q][dir] = *reinterpret_cast<const uint2 *>(NB + dir * Vp + 4 * jbc);
            }
        }
    }
    __syncthreads();

    // diagnostics (off unless requested: they cost three atomics per wave and pass)
    auto stats_after_pass = [&]() {
        if (a.stats != nullptr) {
            const unsigned n = wave_total(wave_incl_sum(wk.accepted));
            if (live && lane == 0) {
                atomicAdd(&a.stats[2], (unsigned long long)n);
                atomicAdd(&a.stats[1], (unsigned long long)wk.rounds);
                if (lg == 0) atomicAdd(&a.stats[0], 1ull);
            }
        }
    };

    for (int n = 0; n < a.n_sweeps; ++n) {
        if (NCP > 0) {
#pragma unroll
            for (int cp = 0; cp < (NCP > 0 ? NCP : 1); ++cp) {
                wk.pass(a.pass_p0[cp], a.pass_p1[cp], a.pass_jbase[cp], sweep, nbc[cp], a.err);
                stats_after_pass();
                // with several waves per walker the pass ended on a barrier
                if (WPW == 1 && ((a.pass_sync >> cp) & 1u)) wave_sync_lds();
            }
        } else {
            for (int c = 0; c < a.n_classes; ++c) {
                const int P0 = a.cls[c], P1 = a.cls[c + 1];
                const int j0 = P0 >> 2, j1 = ((P1 - 1) >> 2) + 1;
                for (int jbase = j0; jbase < j1; jbase += W::GL * BPL) {
                    uint2 nq[BPL][6];
#pragma unroll
                    for (int q = 0; q < BPL; ++q) {
                        const int jb = jbase + lg * BPL + q;
                        const int jbc = jb < j1 ? jb : j0;
#pragma unroll
                        for (int dir = 0; dir < 6; ++dir)
                            nq[q][dir] = *reinterpret_cast<const uint2 *>(NB + dir * Vp + 4 * jbc);
                    }
                    wk.pass(P0, P1, jbase, sweep, nq, a.err);
                    stats_after_pass();
                }
                if (WPW == 1) wave_sync_lds();
            }
        }
        sweep += 1u;
        // ---- measurement after the sweep ----
        if (RECORD) {
            unsigned ej = wave_total(wave_incl_sum(wk.myEJ));
            unsigned m = wave_total(wave_incl_sum(wk.myM));
            if (WPW > 1) {
                if (lane == 0) {
                    sRed[2 * wave] = ej;
                    sRed[2 * wave + 1] = m;
                }
                __syncthreads();
                ej = 0u;
                m = 0u;
#pragma unroll
                for (int v = 0; v < WPW; ++v) {
                    ej += sRed[2 * (slot * WPW + v)];
                    m += sRed[2 * (slot * WPW + v) + 1];
                }
            }
            if (live && lg == 0 && wk.ED >= a.rec_lo && wk.ED <= a.rec_hi) {
                const int ED = wk.ED;
                const long long EJ = (long long)(int)((unsigned)EJ0 + ej);
                const long long M = (long long)(int)((unsigned)M0 + m);
                const int V1 = V + 1;
                unsigned long long *acc = a.acc;
                const unsigned long long m2 = (unsigned long long)(M * M);
                const unsigned long long m4 = m2 * m2;
                atomicAdd(&acc[0 * V1 + ED], 1ull);
                atomicAdd(&acc[1 * V1 + ED], (unsigned long long)EJ);
                atomicAdd(&acc[2 * V1 + ED], (unsigned long long)(EJ * EJ));
                atomicAdd(&acc[3 * V1 + ED], (unsigned long long)(M < 0 ? -M : M));
                atomicAdd(&acc[4 * V1 + ED], m2);
                const unsigned long long old = atomicAdd(&acc[5 * V1 + ED], m4);
                if (old + m4 < old) atomicAdd(&acc[6 * V1 + ED], 1ull);
            }
        }
        if (live && lg == 0) {
            if (a.lds_hist)
                atomicAdd(&sHist[wk.ED], 1u);
            else
                atomicAdd(&a.hist[wk.ED], 1ull);
        }
    }

    // ---- write back ----
    unsigned ej = wave_total(wave_incl_sum(wk.myEJ));
    unsigned m = wave_total(wave_incl_sum(wk.myM));
    __syncthreads();  // every wave is done with sRed and sHist of the last sweep
    if (lane == 0) {
        sRed[2 * wave] = ej;
        sRed[2 * wave + 1] = m;
    }
    __syncthreads();
    ej = 0u;
    m = 0u;
#pragma unroll
    for (int v = 0; v < WPW; ++v) {
        ej += sRed[2 * (slot * WPW + v)];
        m += sRed[2 * (slot * WPW + v) + 1];
    }
    if (live) {
        uint4 *dst = reinterpret_cast<uint4 *>(a.lattice + (size_t)walker * Vp);
        if (PACK) {
            const unsigned *src = reinterpret_cast<const unsigned *>(lat);
            for (int k = lg; k < Vp / 16; k += W::GL) dst[k] = unpack16(src[k]);
        } else {
            const uint4 *src = reinterpret_cast<const uint4 *>(lat);
            for (int k = lg; k < Vp / 16; k += W::GL) dst[k] = src[k];
        }
        if (lg == 0)
            reinterpret_cast<int4 *>(a.wstate)[walker] =
                make_int4((int)((unsigned)EJ0 + ej), wk.ED, (int)((unsigned)M0 + m), (int)sweep);
    }
    if (a.lds_hist)
        for (int e = tid; e <= V; e += kBlock) {
            const unsigned cnt = sHist[e];
            if (cnt) atomicAdd(&a.hist[e], (unsigned long long)cnt);
        }
}

template <int WPW, int BPL, bool RECORD, bool LDS_TABLES, int NCP, bool PACK>
__global__ __launch_bounds__(kBlock) void muca_sweep_kernel(SweepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_tile<WPW, BPL, RECORD, LDS_TABLES, NCP, PACK>(a, (int)blockIdx.x * (4 / WPW), smem);
}

// ---------------------------------------------------------------------------
// Batched persistent sweep: walkers of many jobs (different L, T, weights) in
// one launch.  Blocks pull tiles (4 / WPW walkers of one job) from a work
// counter until the list is exhausted; the host orders the list heaviest
// first.  Spins are staged in LDS; thresholds and neighbour tables too for
// the jobs whose tables fit the batch's LDS budget (else they are read through
// the caches); histograms go straight to each job's buffer.  Each walker
// runs exactly the chain it runs in its own job's launch.  WPW == 0 takes the
// waves per walker from each tile's job (1 or 4), so the walkers of large
// lattices get a whole block while small ones share one.
// ---------------------------------------------------------------------------
template <int WPW, int BPL, bool RECORD, bool PACK>
__device__ __forceinline__ void batch_tile(const BatchArgs &b, const BatchJob &J, SweepArgs &a, int walker0,
                                           unsigned char *smem)
{
    if (J.lds_tables) {
        a.lds_off_r = b.lds_off_tab;
        a.lds_off_nb = b.lds_off_tab + ((16 * (J.V + 1 + 2 * kRPad) + 15) & ~15);
        sweep_tile<WPW, BPL, RECORD, true, 0, PACK>(a, walker0, smem);
    } else {
        a.lds_off_r = 0;
        a.lds_off_nb = 0;
        sweep_tile<WPW, BPL, RECORD, false, 0, PACK>(a, walker0, smem);
    }
}

template <int WPW, int BPL, bool RECORD, bool PACK>
__global__ __launch_bounds__(kBlock) void muca_batch_kernel(BatchArgs b)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int sTile;
    for (;;) {
        if (threadIdx.x == 0) sTile = (int)atomicAdd(b.counter, 1u);
        __syncthreads();
        const int t = sTile;
        __syncthreads();
        if (t >= b.n_tiles) break;
        const int2 tile = b.tiles[t];
        const BatchJob &J = b.jobs[tile.x];
        SweepArgs a;
        a.lattice = J.lattice;
        a.wstate = J.wstate;
        a.hist = J.hist;
        a.bp = J.bp;
        a.r = J.r;
        a.nb = J.nb;
        a.nb2 = J.nb2;
        a.acc = J.acc;
        a.err = J.err;
        a.stats = nullptr;
        a.V = J.V;
        a.Vp = J.Vp;
        a.n_walkers = J.n_walkers;
        a.n_classes = J.n_classes;
#pragma unroll
        for (int c = 0; c <= kMaxClasses; ++c) a.cls[c] = J.cls[c];
        a.n_pass = 0;
        a.pass_sync = 0u;
        a.k0 = J.k0;
        a.k1 = J.k1;
        a.rec_lo = J.rec_lo;
        a.rec_hi = J.rec_hi;
        a.w0 = J.w0;
        a.n_sweeps = b.n_sweeps;
        a.lds_hist = 0;
        a.lds_off_hist = kLdsFixed;
        a.lds_off_lat = b.lds_off_lat;
        if constexpr (WPW == 0) {
            if (J.wpw == 4)
                batch_tile<4, BPL, RECORD, PACK>(b, J, a, tile.y, smem);
            else
                batch_tile<1, BPL, RECORD, PACK>(b, J, a, tile.y, smem);
        } else {
            batch_tile<WPW, BPL, RECORD, PACK>(b, J, a, tile.y, smem);
        }
    }
}

// ---------------------------------------------------------------------------
// Initial lattices: spin at position p (site i = site[p]) from word i&3 of the
// Philox block (i>>2, w, 0, 1), w the global walker index: s = floor(3 x / 2^32) - 1.
// Padding bytes are 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void muca_init_lattice_kernel(InitArgs a)
{
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (size_t)a.n_walkers * a.Vp) return;
    const int w = (int)(idx / (size_t)a.Vp);
    const int p = (int)(idx % (size_t)a.Vp);
    int v = 0;
    if (p < a.V) {
        const int i = a.site[p];
        const Ctr4 x = philox10((uint32_t)(i >> 2), (uint32_t)(a.w0 + w), 0u, 1u, a.k0, a.k1);
        const uint32_t xw = x.v[i & 3];
        v = (int)(((uint64_t)xw * 3u) >> 32) - 1;
    }
    a.lattice[idx] = (int8_t)v;
}

// E_J = -(1/2) sum_p s_p h_p (each bond twice), E_Delta = sum s^2, M = sum s.
__global__ __launch_bounds__(kBlock) void muca_init_energy_kernel(InitArgs a)
{
    __shared__ int red[3][kBlock];
    const int w = blockIdx.x;
    const int8_t *lat = a.lattice + (size_t)w * a.Vp;
    int sh = 0, s2 = 0, s1 = 0;
    for (int p = threadIdx.x; p < a.V; p += kBlock) {
        const int s = lat[p];
        int h = 0;
        for (int dir = 0; dir < 6; ++dir) h += lat[a.nb[dir * a.Vp + p]];
        sh += s * h;
        s2 += s * s;
        s1 += s;
    }
    red[0][threadIdx.x] = sh;
    red[1][threadIdx.x] = s2;
    red[2][threadIdx.x] = s1;
    __syncthreads();
    for (int half = kBlock / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        reinterpret_cast<int4 *>(a.wstate)[w] = make_int4(-red[0][0] / 2, red[1][0], red[2][0], 0);
}

__global__ __launch_bounds__(kBlock) void muca_zero_kernel(uint4 *p, size_t n16)
{
    for (size_t k = blockIdx.x * (size_t)kBlock + threadIdx.x; k < n16; k += (size_t)gridDim.x * kBlock)
        p[k] = make_uint4(0, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Reweighting, one block per Delta (Sec. II time-series reweighting grouped per
// E_Delta bin; Eqs. (FieldDerivative), (sph)).  Fixed-order block reductions in
// FP64; within-bin variances from exact 128-bit integers.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double (*sh)[kBlock])
{
#pragma unroll
    for (int k = 0; k < N; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int half = kBlock / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half)
#pragma unroll
            for (int k = 0; k < N; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + half];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = sh[k][0];
    __syncthreads();
}

__device__ __forceinline__ double u128_to_double(unsigned long long hi, unsigned long long lo)
{
    return (double)hi * 18446744073709551616.0 + (double)lo;
}

__global__ __launch_bounds__(kBlock) void muca_reweight_kernel(ReweightArgs a)
{
    __shared__ double sh[8][kBlock];
    __shared__ int shi[2][kBlock];
    const int V = a.V, V1 = V + 1;
    const unsigned long long *H = a.acc;
    const long long *SJ = reinterpret_cast<const long long *>(a.acc + V1);
    const long long *SJJ = reinterpret_cast<const long long *>(a.acc + 2 * V1);
    const unsigned long long *SA = a.acc + 3 * V1;
    const unsigned long long *SM2 = a.acc + 4 * V1;
    const unsigned long long *SM4lo = a.acc + 5 * V1;
    const unsigned long long *SM4hi = a.acc + 6 * V1;
    const double delta = a.delta[blockIdx.x];
    const double bd = a.beta * delta;

    // pass 1: max exponent, first and last visited bin
    double amax = -INFINITY;
    int first = V1, last = -1;
    for (int e = threadIdx.x; e <= V; e += kBlock)
        if (H[e] > 0) {
            amax = fmax(amax, -bd * (double)e - a.lnw[e]);
            first = min(first, e);
            last = max(last, e);
        }
    sh[0][threadIdx.x] = amax;
    shi[0][threadIdx.x] = first;
    shi[1][threadIdx.x] = last;
    __syncthreads();
    for (int half = kBlock / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) {
            sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + half]);
            shi[0][threadIdx.x] = min(shi[0][threadIdx.x], shi[0][threadIdx.x + half]);
            shi[1][threadIdx.x] = max(shi[1][threadIdx.x], shi[1][threadIdx.x + half]);
        }
        __syncthreads();
    }
    amax = sh[0][0];
    first = shi[0][0];
    last = shi[1][0];
    __syncthreads();

    // pass 2: normalisation and first moments
    double s1[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // Z, SJ, E, SJJ, SA, SM2, SM4, edge
    for (int e = threadIdx.x; e <= V; e += kBlock) {
        const unsigned long long h = H[e];
        if (h == 0) continue;
        const double w = exp(-bd * (double)e - a.lnw[e] - amax);
        const double hw = w * (double)h;
        s1[0] += hw;
        s1[1] += w * (double)SJ[e];
        s1[2] += hw * (double)e;
        s1[3] += w * (double)SJJ[e];
        s1[4] += w * (double)SA[e];
        s1[5] += w * (double)SM2[e];
        s1[6] += w * u128_to_double(SM4hi[e], SM4lo[e]);
        if (e == first || e == last) s1[7] += hw;
    }
    block_sum<8>(s1, sh);
    const double Z = s1[0];
    const double eJ = s1[1] / Z, eD = s1[2] / Z, eJJ = s1[3] / Z;
    const double eA = s1[4] / Z, eM2 = s1[5] / Z, eM4 = s1[6] / Z, edge = s1[7] / Z;

    // pass 3: central moments (between-bin + exact within-bin variance)
    double s2[4] = {0, 0, 0, 0};  // var_EJ, var_ED, cov, third
    for (int e = threadIdx.x; e <= V; e += kBlock) {
        const unsigned long long h = H[e];
        if (h == 0) continue;
        const double w = exp(-bd * (double)e - a.lnw[e] - amax);
        const double hw = w * (double)h;
        const double hd = (double)h;
        const double mJ = (double)SJ[e] / hd;
        const __int128 num = (__int128)(long long)h * (__int128)SJJ[e] - (__int128)SJ[e] * (__int128)SJ[e];
        const double within = (double)num / (hd * hd);
        const double dJ = mJ - eJ, dD = (double)e - eD;
        s2[0] += hw * (within + dJ * dJ);
        s2[1] += hw * dD * dD;
        s2[2] += hw * dJ * dD;
        s2[3] += hw * dJ * dD * dD;
    }
    block_sum<4>(s2, sh);
    if (threadIdx.x == 0) {
        const double beta = a.beta;
        const double varJ = s2[0] / Z, varD = s2[1] / Z, cov = s2[2] / Z, third = s2[3] / Z;
        const double varE = varJ + 2.0 * delta * cov + delta * delta * varD;
        double *o = a.obs + (size_t)blockIdx.x * 15;
        o[0] = delta;
        o[1] = eJ;
        o[2] = eD;
        o[3] = eJ + delta * eD;
        o[4] = eJJ;
        o[5] = varJ;
        o[6] = varD;
        o[7] = -beta * cov;
        o[8] = beta * beta * third;
        o[9] = beta * beta * varE / (double)V;
        o[10] = eA;
        o[11] = eM2;
        o[12] = eM4;
        o[13] = eM2 > 0.0 ? 1.0 - eM4 / (3.0 * eM2 * eM2) : __builtin_nan("");
        o[14] = edge;
    }
}

// ---------------------------------------------------------------------------
// Reweighted ln P(E_Delta) at one Delta (one block): a(E) = -beta Delta E -
// lnW(E) + ln H(E) over the recorded bins, normalised by a log-sum-exp.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void muca_log_hist_kernel(LogHistArgs a)
{
    __shared__ double sh[1][kBlock];
    const int V = a.V;
    double amax = -INFINITY;
    for (int e = threadIdx.x; e <= V; e += kBlock)
        if (a.hist[e] > 0) amax = fmax(amax, -a.bd * (double)e - a.lnw[e] + log((double)a.hist[e]));
    sh[0][threadIdx.x] = amax;
    __syncthreads();
    for (int half = kBlock / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + half]);
        __syncthreads();
    }
    amax = sh[0][0];
    __syncthreads();
    double z[1] = {0.0};
    for (int e = threadIdx.x; e <= V; e += kBlock)
        if (a.hist[e] > 0) z[0] += exp(-a.bd * (double)e - a.lnw[e] + log((double)a.hist[e]) - amax);
    block_sum<1>(z, sh);
    const double lz = amax + log(z[0]);
    for (int e = threadIdx.x; e <= V; e += kBlock)
        a.lnp[e] = a.hist[e] > 0 ? -a.bd * (double)e - a.lnw[e] + log((double)a.hist[e]) - lz : -INFINITY;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_init(const InitArgs &a, hipStream_t s)
{
    const size_t n = (size_t)a.n_walkers * a.Vp;
    hipLaunchKernelGGL(muca_init_lattice_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(muca_init_energy_kernel, dim3((unsigned)a.n_walkers), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    size_t blocks = (n16 + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(muca_zero_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       reinterpret_cast<uint4 *>(p), n16);
    return hipGetLastError();
}

hipError_t launch_log_hist(const LogHistArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(muca_log_hist_kernel, dim3(1), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reweight(const ReweightArgs &a, int n_delta, hipStream_t s)
{
    hipLaunchKernelGGL(muca_reweight_kernel, dim3((unsigned)n_delta), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int WPW, int BPL, bool RECORD, bool LDS_TABLES, int NCP, bool PACK>
static hipError_t launch_sweep_t(const SweepArgs &a, size_t lds, hipStream_t s)
{
    auto kern = muca_sweep_kernel<WPW, BPL, RECORD, LDS_TABLES, NCP, PACK>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    constexpr int WPB = 4 / WPW;
    const unsigned blocks = (unsigned)((a.n_walkers + WPB - 1) / WPB);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

template <int WPW, int BPL, bool RECORD, bool LDS_TABLES, bool PACK>
static hipError_t launch_sweep_n(const SweepArgs &a, size_t lds, hipStream_t s)
{
    if constexpr (BPL == 1) {
        switch (a.n_pass) {
        case 2: return launch_sweep_t<WPW, BPL, RECORD, LDS_TABLES, 2, PACK>(a, lds, s);
        case 3: return launch_sweep_t<WPW, BPL, RECORD, LDS_TABLES, 3, PACK>(a, lds, s);
        case 4: return launch_sweep_t<WPW, BPL, RECORD, LDS_TABLES, 4, PACK>(a, lds, s);
        default: break;
        }
    }
    return launch_sweep_t<WPW, BPL, RECORD, LDS_TABLES, 0, PACK>(a, lds, s);
}

template <int WPW, int BPL, bool PACK>
static hipError_t launch_sweep_b(const SweepArgs &a, bool record, bool lds_tables, size_t lds, hipStream_t s)
{
    if (record)
        return lds_tables ? launch_sweep_n<WPW, BPL, true, true, PACK>(a, lds, s)
                          : launch_sweep_n<WPW, BPL, true, false, PACK>(a, lds, s);
    return lds_tables ? launch_sweep_n<WPW, BPL, false, true, PACK>(a, lds, s)
                      : launch_sweep_n<WPW, BPL, false, false, PACK>(a, lds, s);
}

template <int WPW, int BPL, bool RECORD, bool PACK>
static hipError_t launch_batch_t(const BatchArgs &b, size_t lds, int blocks, hipStream_t s)
{
    auto kern = muca_batch_kernel<WPW, BPL, RECORD, PACK>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (blocks <= 0) {
        int per_cu = 0, dev = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern), kBlock, lds);
        if (e != hipSuccess) return e;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        blocks = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 256);
        if (blocks > b.n_tiles) blocks = b.n_tiles;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlock), lds, s, b);
    return hipGetLastError();
}

template <int WPW>
static hipError_t launch_batch_w(const BatchArgs &b, int bpl, bool record, bool pack, size_t lds, int blocks,
                                 hipStream_t s)
{
    if (bpl == 1) {
        if (pack)
            return record ? launch_batch_t<WPW, 1, true, true>(b, lds, blocks, s)
                          : launch_batch_t<WPW, 1, false, true>(b, lds, blocks, s);
        return record ? launch_batch_t<WPW, 1, true, false>(b, lds, blocks, s)
                      : launch_batch_t<WPW, 1, false, false>(b, lds, blocks, s);
    }
    return record ? launch_batch_t<WPW, 2, true, false>(b, lds, blocks, s)
                  : launch_batch_t<WPW, 2, false, false>(b, lds, blocks, s);
}

// pack: packed lattices (only with bpl == 1; the host never asks otherwise)
hipError_t launch_batch(const BatchArgs &b, int wpw, int bpl, bool record, bool pack, size_t lds, int blocks,
                        hipStream_t s)
{
    if (pack && bpl != 1) return hipErrorInvalidValue;
    switch (wpw) {
    case 0: return launch_batch_w<0>(b, bpl, record, pack, lds, blocks, s);
    case 1: return launch_batch_w<1>(b, bpl, record, pack, lds, blocks, s);
    case 2: return launch_batch_w<2>(b, bpl, record, pack, lds, blocks, s);
    default: return launch_batch_w<4>(b, bpl, record, pack, lds, blocks, s);
    }
}

template <int WPW>
static hipError_t launch_sweep_w(const SweepArgs &a, int bpl, bool record, bool lds_tables, bool pack, size_t lds,
                                 hipStream_t s)
{
    if (bpl == 1)
        return pack ? launch_sweep_b<WPW, 1, true>(a, record, lds_tables, lds, s)
                    : launch_sweep_b<WPW, 1, false>(a, record, lds_tables, lds, s);
    return launch_sweep_b<WPW, 2, false>(a, record, lds_tables, lds, s);
}

hipError_t launch_sweep(const SweepArgs &a, int wpw, int bpl, bool record, bool lds_tables, bool pack, size_t lds,
                        hipStream_t s)
{
    if (pack && bpl != 1) return hipErrorInvalidValue;
    if (wpw == 1) return launch_sweep_w<1>(a, bpl, record, lds_tables, pack, lds, s);
    if (wpw == 2) return launch_sweep_w<2>(a, bpl, record, lds_tables, pack, lds, s);
    return launch_sweep_w<4>(a, bpl, record, lds_tables, pack, lds, s);
}

}  // namespace muca
