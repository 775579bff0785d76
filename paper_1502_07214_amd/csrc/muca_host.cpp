// Host side of libmuca: argument checks, buffer layout, the colour-major order
// and neighbour tables, the acceptance thresholds and the multicanonical weight
// recursion (host FP64), and the ordering of device work on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/muca.h"
#include "muca_internal.h"

using namespace muca;

static_assert(sizeof(muca_obs) == MUCA_N_OBS * sizeof(double), "muca_obs must be 15 packed doubles");

namespace {

thread_local std::string g_detail;

int fail_device(hipError_t e, const char *what)
{
    g_detail = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return MUCA_E_DEVICE;
}

#define HIP_TRY(expr)                                     \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return fail_device(e_, #expr); \
    } while (0)

// ---------------------------------------------------------------------------
// Lattice geometry (Sec. I: L^3 simple cubic, periodic) and visiting order.
// ---------------------------------------------------------------------------
int colour_count(int L) { return (L & 1) ? 3 : 2; }

// Proper colouring: even L by parity of x+y+z; odd L by f(t) = t mod 2 for
// t < L-1 and f(L-1) = 2, colour = (f(x) + f(y) + f(z)) mod 3.
int colour_of(int L, int x, int y, int z)
{
    if (!(L & 1)) return (x + y + z) & 1;
    auto f = [L](int t) { return t == L - 1 ? 2 : (t & 1); };
    return (f(x) + f(y) + f(z)) % 3;
}

// order[p] = site index at position p; cls[c] = first position of colour c.
void build_order(int L, std::vector<int> &order, int cls[kMaxClasses + 1])
{
    const int V = L * L * L, C = colour_count(L);
    std::vector<int> count(C + 1, 0);
    std::vector<int> col(V);
    for (int i = 0; i < V; ++i) {
        col[i] = colour_of(L, i % L, (i / L) % L, i / (L * L));
        count[col[i] + 1]++;
    }
    for (int c = 0; c < C; ++c) count[c + 1] += count[c];
    for (int c = 0; c <= kMaxClasses; ++c) cls[c] = c <= C ? count[c] : V;
    order.assign(V, 0);
    std::vector<int> fill(count.begin(), count.end() - 1);
    for (int i = 0; i < V; ++i) order[fill[col[i]]++] = i;  // ascending i inside each colour
}

bool params_ok(const muca_params *p)
{
    if (!p) return false;
    if (p->L < MUCA_L_MIN || p->L > MUCA_L_MAX) return false;
    if (!(p->T > 0.0)) return false;  // rejects NaN and T <= 0; +inf allowed
    if (p->n_walkers < 1) return false;
    if (p->max_delta < 0 || p->max_delta > 65536) return false;
    if (p->first_walker < 0 || (int64_t)p->first_walker + p->n_walkers > ((int64_t)1 << 31)) return false;
    return true;
}

double beta_of(double T) { return std::isinf(T) ? 0.0 : 1.0 / T; }

void static_scratch_setup(int device);

Layout make_layout(const muca_params *p)
{
    Layout g{};
    g.L = p->L;
    g.V = p->L * p->L * p->L;
    g.Vp = (int)align_up((size_t)g.V, 16);
    g.C = colour_count(p->L);
    g.n_walkers = p->n_walkers;
    g.max_delta = p->max_delta;
    const size_t V1 = (size_t)g.V + 1;
    g.lattice_bytes = align_up((size_t)g.n_walkers * g.Vp, 256);
    g.state_bytes = align_up((size_t)g.n_walkers * 16, 256);
    g.hist_bytes = align_up(8 * V1, 256) + 256;  // + error word
    g.off_bp = 0;
    g.off_r = 256;
    g.off_lnw = g.off_r + align_up(16 * (V1 + 2 * kRPad), 256);
    g.off_nb = g.off_lnw + align_up(8 * V1, 256);
    g.off_nb2 = g.off_nb + align_up((size_t)12 * g.Vp, 256);
    g.off_site = g.off_nb2 + align_up((size_t)12 * g.Vp, 256);
    g.tables_bytes = g.off_site + align_up((size_t)2 * g.Vp, 256);
    g.accum_bytes = align_up(7 * 8 * V1, 256);
    g.off_obs_lnp = align_up((size_t)g.max_delta * (1 + MUCA_N_OBS) * 8, 256);
    g.off_obs_sums = g.off_obs_lnp + align_up(8 * V1, 256);
    g.obs_bytes = g.off_obs_sums + align_up(7 * 8 * V1, 256);
    return g;
}

// Acceptance thresholds (Sec. II): Bp[k+12] = 2^31 exp(-beta k), k = dE_J in
// [-12, 12]; Rp[E] = exp(lnW[E+1] - lnW[E]) (0 at E = V); Rm[E] =
// exp(lnW[E-1] - lnW[E]) (0 at E = 0).  A window [lo, hi] rejects the moves
// that would leave it: Rp[hi] = Rm[lo] = 0 ([0, V]: no change).
void compute_tables(int V, double beta, const double *lnW, int lo, int hi, double *Bp, double *Rp, double *Rm)
{
    for (int k = 0; k < 25; ++k) {
        const double dE = (double)(k - 12);
        Bp[k] = std::ldexp(std::exp(-(beta * dE)), 31);
    }
    for (int E = 0; E <= V; ++E) {
        Rp[E] = E < V ? std::exp(lnW[E + 1] - lnW[E]) : 0.0;
        Rm[E] = E > 0 ? std::exp(lnW[E - 1] - lnW[E]) : 0.0;
    }
    Rp[hi] = 0.0;
    Rm[lo] = 0.0;
}

// Weights outside a window [lo, hi]: walls that fall by kappa = 12 beta +
// ln(2V) + 1 per bin away from it.  A walker outside accepts every proposal
// towards the window (the wall factor beats exp(-beta dE_J) for |dE_J| <= 12)
// and one away from it with probability at most 1/(2eV), which outweighs the
// at most V such proposals per sweep that the entropy of E_Delta offers: it
// enters in a few sweeps and, the tables confining it, never leaves.
void window_walls(int V, double beta, int lo, int hi, double *lnW)
{
    const double kappa = 12.0 * beta + std::log(2.0 * (double)V) + 1.0;
    for (int E = hi + 1; E <= V; ++E) lnW[E] = lnW[hi] - kappa * (double)(E - hi);
    for (int E = lo - 1; E >= 0; --E) lnW[E] = lnW[lo] - kappa * (double)(lo - E);
}

int query_max_lds(int device)
{
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || v <= 0)
        v = 65536;
    return v;
}

}  // namespace

struct muca_job {
    muca_params p;
    Layout g;
    double beta;
    uint32_t k0, k1;
    int device;
    int max_lds;  // LDS bytes a block may use
    int lds_cu;   // LDS bytes of one compute unit
    int n_cu;
    hipStream_t stream;
    muca_dev_buffers d;
    std::vector<int> order;   // position -> site
    std::vector<double> lnW;  // current weights (V+1)
    // weight recursion: MUCA_REC_* flags, accumulated pair statistics (V),
    // bins visited in any iteration since the recursion was set (V+1)
    uint32_t rec_flags;
    std::vector<double> kacc;
    std::vector<uint8_t> seen;
    // E_Delta window [win_lo, win_hi] the walkers are confined to ([0, V]: none)
    int win_lo, win_hi;
    // launch shape
    int wpw, bpl, lds_tables_req, pack_req;
    // pinned staging
    unsigned char *pin_tables;  // Bp | R | lnW regions of the tables buffer
    unsigned char *pin_hist;    // hist + error word
    unsigned char *pin_obs;     // obs buffer
    hipEvent_t ev_tables;
    int64_t recorded;           // sweeps recorded into accum since the last clear
    int stats;                  // count passes / rounds / accepted moves in the sweep kernel
};

namespace {

// The passes of one sweep for a launch shape: colour classes in order, each
// split into groups of 64*wpw*bpl Philox blocks.  Returns the number of passes
// when a sweep is at most kMaxCachedPasses passes and bpl == 1 (neighbour
// positions then live in registers), else 0.
int cached_passes(const Layout &g, int wpw, int bpl, SweepArgs *a)
{
    if (bpl != 1) return 0;
    const int per_pass = 64 * wpw * bpl;
    int np = 0;
    unsigned sync = 0u;
    for (int c = 0; c < g.C; ++c) {
        const int j0 = g.cls[c] >> 2, j1 = ((g.cls[c + 1] - 1) >> 2) + 1;
        for (int jb = j0; jb < j1; jb += per_pass) {
            if (np == kMaxCachedPasses) return 0;
            if (a) {
                a->pass_p0[np] = g.cls[c];
                a->pass_p1[np] = g.cls[c + 1];
                a->pass_jbase[np] = jb;
            }
            ++np;
        }
        sync |= 1u << (np - 1);
    }
    if (a) a->pass_sync = sync;
    return np;
}

struct LaunchPlan {
    bool lds_tables, lds_hist, pack;
    size_t lds;
    int off_hist, off_lat, off_r, off_nb;
};

// Blocks of a launch resident on one compute unit, by LDS alone, capped at
// the eight blocks of four waves a CU holds and at what the launch can use.
long resident_blocks(const muca_job *j, size_t lds, long blocks)
{
    const long cus = j->n_cu > 0 ? j->n_cu : 256;
    const long need = (blocks + cus - 1) / cus;
    return std::min<long>(std::min<long>(need, 8), std::max<long>(1, (long)j->lds_cu / (long)lds));
}

// LDS layout of a sweep launch.  lds_tables_req and pack_req: 1 yes, 0 no,
// -1 automatic.  Packed lattices need bpl == 1.
bool plan_launch(const muca_job *j, int wpw, int bpl, int lds_tables_req, int pack_req, LaunchPlan *out)
{
    const Layout &g = j->g;
    const int wpb = 4 / wpw;
    auto build = [&](bool tables, bool hist, bool pack, LaunchPlan *pl) {
        size_t off = kLdsFixed;
        pl->off_hist = (int)off;
        if (hist) off += align_up(4 * ((size_t)g.V + 1), 16);
        pl->off_lat = (int)off;
        off += align_up((size_t)wpb * (size_t)g.Vp / (pack ? 4 : 1), 16);
        pl->off_r = (int)off;
        if (tables) off += align_up(16 * ((size_t)g.V + 1 + 2 * kRPad), 16);
        pl->off_nb = (int)off;
        if (tables && cached_passes(g, wpw, bpl, nullptr) == 0) off += align_up((size_t)12 * g.Vp, 16);
        pl->lds = off;
        pl->lds_tables = tables;
        pl->lds_hist = hist;
        pl->pack = pack;
        return off <= (size_t)j->max_lds;
    };
    // The per-block LDS histogram saves one HBM atomic per walker and sweep,
    // but at large L it is as large as the lattices: it is kept only while it
    // does not lower the number of blocks resident on a compute unit.  Packed
    // lattices cost an extract per neighbour read; automatic packing takes
    // them only when they raise the resident blocks.
    const long blocks = ((long)g.n_walkers + wpb - 1) / wpb;
    auto resident = [&](const LaunchPlan &pl) { return resident_blocks(j, pl.lds, blocks); };
    const bool try_tables[2] = {true, false};
    for (bool t : try_tables) {
        if (lds_tables_req == 1 && !t) continue;
        if (lds_tables_req == 0 && t) continue;
        bool have = false;
        LaunchPlan best{};
        for (int pk = 0; pk < 2; ++pk) {
            const bool pack = pk == 1;
            if (pack && (bpl != 1 || pack_req == 0)) continue;
            if (!pack && pack_req == 1) continue;
            LaunchPlan with_hist, without, pl;
            const bool fits_h = build(t, true, pack, &with_hist);
            const bool fits_n = build(t, false, pack, &without);
            if (fits_h && (!fits_n || resident(with_hist) >= resident(without)))
                pl = with_hist;
            else if (fits_n)
                pl = without;
            else
                continue;
            if (!have || resident(pl) > resident(best)) {
                best = pl;
                have = true;
            }
        }
        if (have) {
            *out = best;
            return true;
        }
    }
    return false;
}

void default_launch(muca_job *j)
{
    // Measured on MI355X: few walkers -> spread each
    // walker over a whole block (4 waves) with the thresholds staged in LDS;
    // many walkers -> one wave per walker, thresholds read through the caches
    // (LDS then only holds lattices, so more blocks fit per CU).  One Philox
    // block per lane keeps the neighbour positions in registers.
    const int nw = j->p.n_walkers;
    const int simds = 4 * (j->n_cu > 0 ? j->n_cu : 256);
    int wpw = 1;
    if (4 * nw <= 2 * simds)
        wpw = 4;
    else if (2 * nw <= 2 * simds)
        wpw = 2;
    const int bpl = 1;
    LaunchPlan pl;
    while (!plan_launch(j, wpw, bpl, -1, -1, &pl) && wpw < 4) wpw *= 2;  // fewer walkers per block -> less LDS
    j->wpw = wpw;
    j->bpl = bpl;
    j->lds_tables_req = wpw == 1 ? 0 : -1;
    j->pack_req = -1;
    if (wpw > 1 && plan_launch(j, wpw, bpl, 1, -1, &pl) && pl.lds_tables) {
        // staged tables only while every block still fits on the device at
        // once: a second wave of blocks costs more than the cached reads
        const long blocks = (nw + 4 / wpw - 1) / (4 / wpw);
        const long per_cu = std::max<long>(1, (long)j->max_lds / (long)pl.lds);
        if (blocks > per_cu * (long)(simds / 4)) j->lds_tables_req = 0;
    }
    if (!plan_launch(j, wpw, bpl, j->lds_tables_req, -1, &pl)) j->lds_tables_req = -1;
}

int upload_tables(muca_job *j)
{
    const Layout &g = j->g;
    HIP_TRY(hipEventSynchronize(j->ev_tables));  // staging free again
    double *Bp = reinterpret_cast<double *>(j->pin_tables + g.off_bp);
    double *R = reinterpret_cast<double *>(j->pin_tables + g.off_r);
    double *lw = reinterpret_cast<double *>(j->pin_tables + g.off_lnw);
    std::vector<double> Rp(g.V + 1), Rm(g.V + 1);
    for (int k = 0; k < 32; ++k) Bp[k] = 0.0;
    compute_tables(g.V, j->beta, j->lnW.data(), j->win_lo, j->win_hi, Bp, Rp.data(), Rm.data());
    for (int k = 0; k < 2 * (g.V + 1 + 2 * kRPad); ++k) R[k] = 0.0;
    for (int E = 0; E <= g.V; ++E) {
        R[2 * (E + kRPad)] = Rm[E];
        R[2 * (E + kRPad) + 1] = Rp[E];
    }
    std::memcpy(lw, j->lnW.data(), sizeof(double) * (g.V + 1));
    HIP_TRY(hipMemcpyAsync(j->d.tables, j->pin_tables, g.off_nb, hipMemcpyHostToDevice, j->stream));
    HIP_TRY(hipEventRecord(j->ev_tables, j->stream));
    return MUCA_OK;
}

int clear_accum(muca_job *j)
{
    HIP_TRY(launch_zero(j->d.accum, j->g.accum_bytes, j->stream));
    j->recorded = 0;
    return MUCA_OK;
}

int use_device(const muca_job *j)
{
    HIP_TRY(hipSetDevice(j->device));
    return MUCA_OK;
}

}  // namespace

extern "C" {

int muca_query_sizes(const muca_params *params, size_t *lattice_bytes, size_t *state_bytes,
                     size_t *hist_bytes, size_t *tables_bytes, size_t *accum_bytes, size_t *obs_bytes)
{
    if (!params_ok(params)) return MUCA_E_INVAL;
    const Layout g = make_layout(params);
    if (lattice_bytes) *lattice_bytes = g.lattice_bytes;
    if (state_bytes) *state_bytes = g.state_bytes;
    if (hist_bytes) *hist_bytes = g.hist_bytes;
    if (tables_bytes) *tables_bytes = g.tables_bytes;
    if (accum_bytes) *accum_bytes = g.accum_bytes;
    if (obs_bytes) *obs_bytes = g.obs_bytes;
    return MUCA_OK;
}

int muca_init(const muca_params *params, const muca_dev_buffers *buffers, const double *lnW_host,
              void *stream, muca_job **out)
{
    if (!out) return MUCA_E_INVAL;
    *out = nullptr;
    if (!params_ok(params) || !buffers) return MUCA_E_INVAL;
    void *ptrs[6] = {buffers->lattice, buffers->walker_state, buffers->hist,
                     buffers->tables, buffers->accum, buffers->obs};
    for (void *q : ptrs)
        if (!q || (reinterpret_cast<uintptr_t>(q) & 255u)) return MUCA_E_INVAL;
    const Layout g = make_layout(params);
    if (lnW_host)
        for (int E = 0; E <= g.V; ++E)
            if (!std::isfinite(lnW_host[E])) return MUCA_E_INVAL;

    muca_job *j = new (std::nothrow) muca_job();
    if (!j) return MUCA_E_SIZE;
    j->p = *params;
    j->g = g;
    build_order(g.L, j->order, j->g.cls);
    j->beta = beta_of(params->T);
    j->k0 = (uint32_t)(params->seed & 0xffffffffu);
    j->k1 = (uint32_t)(params->seed >> 32);
    j->stream = reinterpret_cast<hipStream_t>(stream);
    j->d = *buffers;
    if (lnW_host)
        j->lnW.assign(lnW_host, lnW_host + g.V + 1);
    else
        j->lnW.assign(g.V + 1, 0.0);
    j->recorded = 0;
    j->rec_flags = 0u;
    j->kacc.assign(std::max(g.V, 1), 0.0);
    j->seen.assign(g.V + 1, 0);
    j->win_lo = 0;
    j->win_hi = g.V;

    auto bail = [&](int rc) {
        muca_free(j);
        return rc;
    };
    if (hipGetDevice(&j->device) != hipSuccess) return bail(fail_device(hipGetLastError(), "hipGetDevice"));
    j->max_lds = query_max_lds(j->device);
    if (hipDeviceGetAttribute(&j->lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, j->device) !=
            hipSuccess ||
        j->lds_cu < j->max_lds)
        j->lds_cu = j->max_lds;
    static_scratch_setup(j->device);
    if (hipDeviceGetAttribute(&j->n_cu, hipDeviceAttributeMultiprocessorCount, j->device) != hipSuccess)
        j->n_cu = 256;
    hipError_t e;
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&j->pin_tables), g.tables_bytes, hipHostMallocDefault)) != hipSuccess)
        return bail(fail_device(e, "hipHostMalloc(tables)"));
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&j->pin_hist), g.hist_bytes, hipHostMallocDefault)) != hipSuccess)
        return bail(fail_device(e, "hipHostMalloc(hist)"));
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&j->pin_obs), g.obs_bytes, hipHostMallocDefault)) != hipSuccess)
        return bail(fail_device(e, "hipHostMalloc(obs)"));
    if ((e = hipEventCreateWithFlags(&j->ev_tables, hipEventDisableTiming)) != hipSuccess)
        return bail(fail_device(e, "hipEventCreate"));
    if ((e = hipEventRecord(j->ev_tables, j->stream)) != hipSuccess) return bail(fail_device(e, "hipEventRecord"));

    // neighbour and site tables in position space (uploaded once)
    {
        const int L = g.L, V = g.V, Vp = g.Vp;
        std::vector<int> pos(V);
        for (int p = 0; p < V; ++p) pos[j->order[p]] = p;
        uint16_t *nb = reinterpret_cast<uint16_t *>(j->pin_tables + g.off_nb);
        uint16_t *nb2 = reinterpret_cast<uint16_t *>(j->pin_tables + g.off_nb2);
        uint16_t *site = reinterpret_cast<uint16_t *>(j->pin_tables + g.off_site);
        std::memset(nb, 0, (size_t)12 * Vp);
        std::memset(nb2, 0, (size_t)12 * Vp);
        std::memset(site, 0, (size_t)2 * Vp);
        for (int p = 0; p < V; ++p) {
            const int i = j->order[p];
            const int x = i % L, y = (i / L) % L, z = i / (L * L);
            const int nbr[6] = {(x + 1) % L + L * (y + L * z), (x + L - 1) % L + L * (y + L * z),
                                x + L * ((y + 1) % L + L * z), x + L * ((y + L - 1) % L + L * z),
                                x + L * (y + L * ((z + 1) % L)), x + L * (y + L * ((z + L - 1) % L))};
            for (int dir = 0; dir < 6; ++dir) {
                nb[(size_t)dir * Vp + p] = (uint16_t)pos[nbr[dir]];
                nb2[(size_t)dir * Vp + p] = (uint16_t)(2 * pos[nbr[dir]]);  // V <= 32768
            }
            site[p] = (uint16_t)i;
        }
        unsigned char *dt = reinterpret_cast<unsigned char *>(j->d.tables);
        if ((e = hipMemcpyAsync(dt + g.off_nb, j->pin_tables + g.off_nb, g.tables_bytes - g.off_nb,
                                hipMemcpyHostToDevice, j->stream)) != hipSuccess)
            return bail(fail_device(e, "hipMemcpyAsync(nb)"));
        if ((e = hipStreamSynchronize(j->stream)) != hipSuccess)
            return bail(fail_device(e, "hipStreamSynchronize"));
    }
    int rc = upload_tables(j);
    if (rc) return bail(rc);
    if ((e = launch_zero(j->d.hist, g.hist_bytes, j->stream)) != hipSuccess) return bail(fail_device(e, "zero hist"));
    if ((e = launch_zero(j->d.accum, g.accum_bytes, j->stream)) != hipSuccess) return bail(fail_device(e, "zero accum"));
    InitArgs ia;
    ia.lattice = reinterpret_cast<int8_t *>(j->d.lattice);
    ia.wstate = reinterpret_cast<int32_t *>(j->d.walker_state);
    ia.nb = reinterpret_cast<const uint16_t *>(reinterpret_cast<unsigned char *>(j->d.tables) + g.off_nb);
    ia.site = reinterpret_cast<const uint16_t *>(reinterpret_cast<unsigned char *>(j->d.tables) + g.off_site);
    ia.V = g.V;
    ia.Vp = g.Vp;
    ia.n_walkers = g.n_walkers;
    ia.k0 = j->k0;
    ia.k1 = j->k1;
    ia.w0 = params->first_walker;
    if ((e = launch_init(ia, j->stream)) != hipSuccess) return bail(fail_device(e, "init kernels"));
    if ((e = hipStreamSynchronize(j->stream)) != hipSuccess) return bail(fail_device(e, "hipStreamSynchronize"));
    default_launch(j);
    *out = j;
    return MUCA_OK;
}

int muca_sweep(muca_job *j, int64_t n_sweeps, uint32_t flags)
{
    if (!j || n_sweeps < 0 || (flags & ~MUCA_RECORD)) return MUCA_E_INVAL;
    if (n_sweeps > MUCA_MAX_SWEEPS_PER_CALL) return MUCA_E_OVERFLOW;
    if (n_sweeps == 0) return MUCA_OK;
    if (int rc = use_device(j)) return rc;
    const Layout &g = j->g;
    LaunchPlan pl;
    if (!plan_launch(j, j->wpw, j->bpl, j->lds_tables_req, j->pack_req, &pl)) return MUCA_E_SIZE;
    SweepArgs a;
    a.lattice = reinterpret_cast<int8_t *>(j->d.lattice);
    a.wstate = reinterpret_cast<int32_t *>(j->d.walker_state);
    a.hist = reinterpret_cast<unsigned long long *>(j->d.hist);
    unsigned char *dt = reinterpret_cast<unsigned char *>(j->d.tables);
    a.bp = reinterpret_cast<const double *>(dt + g.off_bp);
    a.r = reinterpret_cast<const double *>(dt + g.off_r);
    a.nb = reinterpret_cast<const uint16_t *>(dt + g.off_nb);
    a.nb2 = reinterpret_cast<const uint16_t *>(dt + g.off_nb2);
    a.acc = reinterpret_cast<unsigned long long *>(j->d.accum);
    unsigned char *tail = reinterpret_cast<unsigned char *>(j->d.hist) + align_up(8 * ((size_t)g.V + 1), 256);
    a.err = reinterpret_cast<int *>(tail);
    a.stats = j->stats ? reinterpret_cast<unsigned long long *>(tail + 16) : nullptr;
    a.V = g.V;
    a.Vp = g.Vp;
    a.n_walkers = g.n_walkers;
    a.n_classes = g.C;
    for (int c = 0; c <= kMaxClasses; ++c) a.cls[c] = g.cls[c];
    a.k0 = j->k0;
    a.k1 = j->k1;
    a.rec_lo = j->win_lo;
    a.rec_hi = j->win_hi;
    a.w0 = j->p.first_walker;
    a.lds_hist = pl.lds_hist ? 1 : 0;
    a.lds_off_hist = pl.off_hist;
    a.lds_off_lat = pl.off_lat;
    a.lds_off_r = pl.off_r;
    a.lds_off_nb = pl.off_nb;
    a.n_pass = cached_passes(g, j->wpw, j->bpl, &a);
    const bool record = (flags & MUCA_RECORD) != 0;
    int64_t left = n_sweeps;
    while (left > 0) {
        const int chunk = (int)std::min<int64_t>(left, kMaxSweepsPerLaunch);
        a.n_sweeps = chunk;
        HIP_TRY(launch_sweep(a, j->wpw, j->bpl, record, pl.lds_tables, pl.pack, pl.lds, j->stream));
        left -= chunk;
    }
    if (record) j->recorded += n_sweeps;
    return MUCA_OK;
}

int muca_reduce_hist(muca_job *j, int64_t *hist_host, int32_t reset)
{
    if (!j || !hist_host) return MUCA_E_INVAL;
    if (int rc = use_device(j)) return rc;
    const Layout &g = j->g;
    HIP_TRY(hipMemcpyAsync(j->pin_hist, j->d.hist, g.hist_bytes, hipMemcpyDeviceToHost, j->stream));
    HIP_TRY(hipStreamSynchronize(j->stream));
    const int err = *reinterpret_cast<const int *>(j->pin_hist + align_up(8 * ((size_t)g.V + 1), 256));
    std::memcpy(hist_host, j->pin_hist, 8 * ((size_t)g.V + 1));
    if (reset) HIP_TRY(launch_zero(j->d.hist, align_up(8 * ((size_t)g.V + 1), 16), j->stream));
    if (err) {
        g_detail = "sweep kernel reported an internal error (fixed-point round cap)";
        return MUCA_E_DEVICE;
    }
    return MUCA_OK;
}

int muca_set_recursion(muca_job *j, uint32_t flags)
{
    if (!j || (flags & ~(MUCA_REC_ACCUMULATED | MUCA_REC_EXTRAPOLATE))) return MUCA_E_INVAL;
    j->rec_flags = flags;
    j->kacc.assign(std::max(j->g.V, 1), 0.0);
    j->seen.assign(j->g.V + 1, 0);
    return MUCA_OK;
}

namespace {

// Accumulated recursion on the log-weight differences of neighbouring bins:
// each iteration's estimate of the flat-histogram difference enters with its
// inverse Poisson variance k = H(E) H(E+1) / (H(E) + H(E+1)); a pair with one
// visited bin takes the plain step; the weights are rebuilt upwards from bin 0.
// The caller restarts the sums when an iteration reaches a new bin or misses
// one inside the range visited so far.
void accumulated_step(int lo, int hi, const int64_t *hist, double *lnW, double *kacc)
{
    std::vector<double> d(std::max(hi, 1));
    for (int E = lo; E < hi; ++E) d[E] = lnW[E + 1] - lnW[E];
    for (int E = lo; E < hi; ++E) {
        const int64_t a = hist[E], b = hist[E + 1];
        if (a > 0 && b > 0) {
            const double ha = (double)a, hb = (double)b;
            const double k = ha * hb / (ha + hb);
            kacc[E] = kacc[E] + k;
            d[E] = d[E] + (k / kacc[E]) * (std::log(ha) - std::log(hb));
        } else if (a > 0) {
            d[E] = d[E] + std::log((double)a);
        } else if (b > 0) {
            d[E] = d[E] - std::log((double)b);
        }
    }
    for (int E = lo; E < hi; ++E) lnW[E + 1] = lnW[E] + d[E];
}

// Bins of the window [wlo, whi] outside the visited range [lo, hi] continue
// the mean slope of the last min(8, hi - lo) differences inside it, at each end.
void extrapolate_edges(int wlo, int whi, const uint8_t *seen, double *lnW)
{
    int lo = -1, hi = -1;
    for (int E = wlo; E <= whi; ++E)
        if (seen[E]) {
            if (lo < 0) lo = E;
            hi = E;
        }
    if (lo < 0 || hi <= lo) return;
    const int k = std::min(hi - lo, 8);
    const double s_hi = (lnW[hi] - lnW[hi - k]) / (double)k;
    const double s_lo = (lnW[lo + k] - lnW[lo]) / (double)k;
    for (int E = hi + 1; E <= whi; ++E) lnW[E] = lnW[hi] + (double)(E - hi) * s_hi;
    for (int E = lo - 1; E >= wlo; --E) lnW[E] = lnW[lo] - (double)(lo - E) * s_lo;
}

}  // namespace

int muca_update_weights(muca_job *j, const int64_t *hist, double *lnW_out, double *flatness_out)
{
    if (!j || !hist) return MUCA_E_INVAL;
    const int V = j->g.V;
    for (int E = 0; E <= V; ++E)
        if (hist[E] < 0) return MUCA_E_INVAL;
    if (int rc = use_device(j)) return rc;
    // everything acts on the window: entries outside it (walkers on their
    // way in) are not used
    const int lo = j->win_lo, hi = j->win_hi;
    int64_t sum = 0, least = hist[lo];
    bool any_seen = false, reached_new = false;
    for (int E = lo; E <= hi; ++E) any_seen = any_seen || j->seen[E];
    for (int E = lo; E <= hi; ++E) {
        sum += hist[E];
        least = std::min(least, hist[E]);
        if (hist[E] > 0) {
            reached_new = reached_new || !j->seen[E];
            j->seen[E] = 1;
        }
    }
    // estimates sampled before the range grew are biased by the part that was
    // out of reach: the accumulated statistics restart.  They restart too when
    // the walkers stop reaching a bin inside the range visited so far: the few
    // entries near that edge would barely move the weights against the
    // statistics gathered before, and the visited part would keep shrinking.
    bool missed = false;
    {
        int first = -1, last = -1;
        for (int E = lo; E <= hi; ++E)
            if (j->seen[E]) {
                if (first < 0) first = E;
                last = E;
            }
        for (int E = first; first >= 0 && E <= last && !missed; ++E) missed = hist[E] == 0;
    }
    if ((j->rec_flags & MUCA_REC_ACCUMULATED) && any_seen && (reached_new || missed))
        std::fill(j->kacc.begin() + lo, j->kacc.begin() + hi, 0.0);
    if (j->rec_flags & MUCA_REC_ACCUMULATED) {
        accumulated_step(lo, hi, hist, j->lnW.data(), j->kacc.data());
    } else {
        // W <- W / H on the visited bins (plain multicanonical recursion)
        for (int E = lo; E <= hi; ++E)
            if (hist[E] > 0) j->lnW[E] = j->lnW[E] - std::log((double)hist[E]);
    }
    if (j->rec_flags & MUCA_REC_EXTRAPOLATE) extrapolate_edges(lo, hi, j->seen.data(), j->lnW.data());
    window_walls(V, j->beta, lo, hi, j->lnW.data());
    if (flatness_out) *flatness_out = sum > 0 ? (double)least / ((double)sum / (double)(hi - lo + 1)) : 0.0;
    if (lnW_out) std::memcpy(lnW_out, j->lnW.data(), sizeof(double) * (V + 1));
    if (int rc = upload_tables(j)) return rc;
    return clear_accum(j);
}

int muca_set_weights(muca_job *j, const double *lnW)
{
    if (!j || !lnW) return MUCA_E_INVAL;
    for (int E = 0; E <= j->g.V; ++E)
        if (!std::isfinite(lnW[E])) return MUCA_E_INVAL;
    if (int rc = use_device(j)) return rc;
    j->lnW.assign(lnW, lnW + j->g.V + 1);
    window_walls(j->g.V, j->beta, j->win_lo, j->win_hi, j->lnW.data());
    if (int rc = upload_tables(j)) return rc;
    return clear_accum(j);
}

int muca_set_stream(muca_job *j, void *stream)
{
    if (!j) return MUCA_E_INVAL;
    if (int rc = use_device(j)) return rc;
    HIP_TRY(hipStreamSynchronize(j->stream));  // also completes the last table upload
    j->stream = reinterpret_cast<hipStream_t>(stream);
    return MUCA_OK;
}

int muca_set_window(muca_job *j, int32_t lo, int32_t hi)
{
    if (!j || lo < 0 || hi > j->g.V || lo >= hi) return MUCA_E_INVAL;
    if (int rc = use_device(j)) return rc;
    j->win_lo = lo;
    j->win_hi = hi;
    window_walls(j->g.V, j->beta, lo, hi, j->lnW.data());
    j->kacc.assign(std::max(j->g.V, 1), 0.0);
    j->seen.assign(j->g.V + 1, 0);
    if (int rc = upload_tables(j)) return rc;
    return clear_accum(j);
}

int muca_get_window(const muca_job *j, int32_t *lo, int32_t *hi)
{
    if (!j) return MUCA_E_INVAL;
    if (lo) *lo = j->win_lo;
    if (hi) *hi = j->win_hi;
    return MUCA_OK;
}

int muca_get_recursion_state(const muca_job *j, double *kacc, uint8_t *seen)
{
    if (!j) return MUCA_E_INVAL;
    if (kacc) std::memcpy(kacc, j->kacc.data(), sizeof(double) * (size_t)j->g.V);
    if (seen) std::memcpy(seen, j->seen.data(), (size_t)j->g.V + 1);
    return MUCA_OK;
}

int muca_set_recursion_state(muca_job *j, const double *kacc, const uint8_t *seen)
{
    if (!j) return MUCA_E_INVAL;
    const int V = j->g.V;
    if (kacc)
        for (int E = 0; E < V; ++E)
            if (!std::isfinite(kacc[E]) || kacc[E] < 0.0) return MUCA_E_INVAL;
    if (seen)
        for (int E = 0; E <= V; ++E)
            if (seen[E] > 1) return MUCA_E_INVAL;
    if (kacc) std::memcpy(j->kacc.data(), kacc, sizeof(double) * (size_t)V);
    if (seen) std::memcpy(j->seen.data(), seen, (size_t)V + 1);
    return MUCA_OK;
}

int muca_get_weights(const muca_job *j, double *lnW_out)
{
    if (!j || !lnW_out) return MUCA_E_INVAL;
    std::memcpy(lnW_out, j->lnW.data(), sizeof(double) * (j->g.V + 1));
    return MUCA_OK;
}

static int reweight_from(muca_job *j, const unsigned long long *acc_dev, const double *delta, int32_t n_delta,
                         muca_obs *out)
{
    const Layout &g = j->g;
    double *pd = reinterpret_cast<double *>(j->pin_obs);
    std::memcpy(pd, delta, sizeof(double) * n_delta);
    double *dobs = reinterpret_cast<double *>(j->d.obs);
    HIP_TRY(hipMemcpyAsync(dobs, pd, sizeof(double) * n_delta, hipMemcpyHostToDevice, j->stream));
    ReweightArgs a;
    a.acc = acc_dev;
    a.lnw = reinterpret_cast<const double *>(reinterpret_cast<unsigned char *>(j->d.tables) + g.off_lnw);
    a.delta = dobs;
    a.obs = dobs + g.max_delta;
    a.V = g.V;
    a.beta = j->beta;
    HIP_TRY(launch_reweight(a, n_delta, j->stream));
    HIP_TRY(hipMemcpyAsync(pd + g.max_delta, dobs + g.max_delta, sizeof(double) * MUCA_N_OBS * n_delta,
                           hipMemcpyDeviceToHost, j->stream));
    HIP_TRY(hipStreamSynchronize(j->stream));
    std::memcpy(out, pd + g.max_delta, sizeof(double) * MUCA_N_OBS * n_delta);
    return MUCA_OK;
}

int muca_reweight(muca_job *j, const double *delta, int32_t n_delta, muca_obs *out)
{
    if (!j || !delta || !out || n_delta < 1) return MUCA_E_INVAL;
    if (n_delta > j->g.max_delta) return MUCA_E_SIZE;
    for (int k = 0; k < n_delta; ++k)
        if (!std::isfinite(delta[k])) return MUCA_E_INVAL;
    if (j->recorded <= 0) return MUCA_E_STATE;
    if (int rc = use_device(j)) return rc;
    return reweight_from(j, reinterpret_cast<const unsigned long long *>(j->d.accum), delta, n_delta, out);
}

int muca_reweight_sums(muca_job *j, const int64_t *sums, const uint64_t *sm4, const double *delta, int32_t n_delta,
                       muca_obs *out)
{
    if (!j || !sums || !sm4 || !delta || !out || n_delta < 1) return MUCA_E_INVAL;
    if (n_delta > j->g.max_delta) return MUCA_E_SIZE;
    for (int k = 0; k < n_delta; ++k)
        if (!std::isfinite(delta[k])) return MUCA_E_INVAL;
    const size_t V1 = (size_t)j->g.V + 1;
    int64_t n = 0;
    for (size_t E = 0; E < V1; ++E) {
        if (sums[E] < 0) return MUCA_E_INVAL;
        n += sums[E];
    }
    if (n == 0) return MUCA_E_STATE;
    if (int rc = use_device(j)) return rc;
    unsigned char *scratch = reinterpret_cast<unsigned char *>(j->d.obs) + j->g.off_obs_sums;
    HIP_TRY(hipMemcpyAsync(scratch, sums, 5 * V1 * 8, hipMemcpyHostToDevice, j->stream));
    HIP_TRY(hipMemcpyAsync(scratch + 5 * V1 * 8, sm4, 2 * V1 * 8, hipMemcpyHostToDevice, j->stream));
    return reweight_from(j, reinterpret_cast<const unsigned long long *>(scratch), delta, n_delta, out);
}

int muca_reweight_hist(muca_job *j, double delta, double *lnP_out)
{
    if (!j || !lnP_out || !std::isfinite(delta)) return MUCA_E_INVAL;
    if (j->recorded <= 0) return MUCA_E_STATE;
    if (int rc = use_device(j)) return rc;
    const Layout &g = j->g;
    LogHistArgs a;
    a.hist = reinterpret_cast<const unsigned long long *>(j->d.accum);  // production counts H
    a.lnw = reinterpret_cast<const double *>(reinterpret_cast<unsigned char *>(j->d.tables) + g.off_lnw);
    a.lnp = reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(j->d.obs) + g.off_obs_lnp);
    a.V = g.V;
    a.bd = j->beta * delta;
    HIP_TRY(launch_log_hist(a, j->stream));
    HIP_TRY(hipMemcpyAsync(lnP_out, a.lnp, sizeof(double) * (g.V + 1), hipMemcpyDeviceToHost, j->stream));
    HIP_TRY(hipStreamSynchronize(j->stream));
    return MUCA_OK;
}

int muca_reweight_hist_sums(muca_job *j, const int64_t *hist, double delta, double *lnP_out)
{
    if (!j || !hist || !lnP_out || !std::isfinite(delta)) return MUCA_E_INVAL;
    const Layout &g = j->g;
    int64_t n = 0;
    for (int E = 0; E <= g.V; ++E) {
        if (hist[E] < 0) return MUCA_E_INVAL;
        n += hist[E];
    }
    if (n == 0) return MUCA_E_STATE;
    if (int rc = use_device(j)) return rc;
    unsigned char *scratch = reinterpret_cast<unsigned char *>(j->d.obs) + g.off_obs_sums;
    HIP_TRY(hipMemcpyAsync(scratch, hist, sizeof(int64_t) * (g.V + 1), hipMemcpyHostToDevice, j->stream));
    LogHistArgs a;
    a.hist = reinterpret_cast<const unsigned long long *>(scratch);
    a.lnw = reinterpret_cast<const double *>(reinterpret_cast<unsigned char *>(j->d.tables) + g.off_lnw);
    a.lnp = reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(j->d.obs) + g.off_obs_lnp);
    a.V = g.V;
    a.bd = j->beta * delta;
    HIP_TRY(launch_log_hist(a, j->stream));
    HIP_TRY(hipMemcpyAsync(lnP_out, a.lnp, sizeof(double) * (g.V + 1), hipMemcpyDeviceToHost, j->stream));
    HIP_TRY(hipStreamSynchronize(j->stream));
    return MUCA_OK;
}

int muca_read_state(muca_job *j, int8_t *spins, int64_t *state)
{
    if (!j) return MUCA_E_INVAL;
    if (int rc = use_device(j)) return rc;
    const Layout &g = j->g;
    std::vector<int8_t> lat;
    std::vector<int32_t> st;
    if (spins) {
        lat.resize((size_t)g.n_walkers * g.Vp);
        HIP_TRY(hipMemcpyAsync(lat.data(), j->d.lattice, lat.size(), hipMemcpyDeviceToHost, j->stream));
    }
    if (state) {
        st.resize((size_t)g.n_walkers * 4);
        HIP_TRY(hipMemcpyAsync(st.data(), j->d.walker_state, st.size() * 4, hipMemcpyDeviceToHost, j->stream));
    }
    HIP_TRY(hipStreamSynchronize(j->stream));
    for (int w = 0; spins && w < g.n_walkers; ++w)
        for (int p = 0; p < g.V; ++p) spins[(size_t)w * g.V + j->order[p]] = lat[(size_t)w * g.Vp + p];
    for (int w = 0; state && w < g.n_walkers; ++w) {
        state[4 * (size_t)w + 0] = st[4 * (size_t)w + 0];
        state[4 * (size_t)w + 1] = st[4 * (size_t)w + 1];
        state[4 * (size_t)w + 2] = st[4 * (size_t)w + 2];
        state[4 * (size_t)w + 3] = (int64_t)(uint32_t)st[4 * (size_t)w + 3];
    }
    return MUCA_OK;
}

int muca_write_state(muca_job *j, const int8_t *spins, const int64_t *state)
{
    if (!j || !spins || !state) return MUCA_E_INVAL;
    const Layout &g = j->g;
    for (size_t k = 0; k < (size_t)g.n_walkers * g.V; ++k)
        if (spins[k] < -1 || spins[k] > 1) return MUCA_E_INVAL;
    for (int w = 0; w < g.n_walkers; ++w) {
        const int64_t *s = state + 4 * (size_t)w;
        if (s[1] < 0 || s[1] > g.V || s[0] < -3LL * g.V || s[0] > 3LL * g.V || s[2] < -g.V || s[2] > g.V ||
            s[3] < 0 || s[3] > 0xffffffffLL)
            return MUCA_E_INVAL;
    }
    if (int rc = use_device(j)) return rc;
    std::vector<int8_t> lat((size_t)g.n_walkers * g.Vp, 0);
    std::vector<int32_t> st((size_t)g.n_walkers * 4);
    for (int w = 0; w < g.n_walkers; ++w) {
        for (int p = 0; p < g.V; ++p) lat[(size_t)w * g.Vp + p] = spins[(size_t)w * g.V + j->order[p]];
        for (int k = 0; k < 4; ++k) st[4 * (size_t)w + k] = (int32_t)(uint32_t)state[4 * (size_t)w + k];
    }
    HIP_TRY(hipMemcpyAsync(j->d.lattice, lat.data(), lat.size(), hipMemcpyHostToDevice, j->stream));
    HIP_TRY(hipMemcpyAsync(j->d.walker_state, st.data(), st.size() * 4, hipMemcpyHostToDevice, j->stream));
    HIP_TRY(hipStreamSynchronize(j->stream));
    return MUCA_OK;
}

int muca_read_accum(muca_job *j, int64_t *sums, uint64_t *sm4)
{
    if (!j) return MUCA_E_INVAL;
    if (int rc = use_device(j)) return rc;
    const size_t V1 = (size_t)j->g.V + 1;
    std::vector<uint64_t> buf(7 * V1);
    HIP_TRY(hipMemcpyAsync(buf.data(), j->d.accum, buf.size() * 8, hipMemcpyDeviceToHost, j->stream));
    HIP_TRY(hipStreamSynchronize(j->stream));
    if (sums) std::memcpy(sums, buf.data(), 5 * V1 * 8);
    if (sm4) std::memcpy(sm4, buf.data() + 5 * V1, 2 * V1 * 8);
    return MUCA_OK;
}

int muca_write_accum(muca_job *j, const int64_t *sums, const uint64_t *sm4)
{
    if (!j || !sums || !sm4) return MUCA_E_INVAL;
    const size_t V1 = (size_t)j->g.V + 1;
    int64_t n = 0;
    for (size_t E = 0; E < V1; ++E) {
        if (sums[E] < 0) return MUCA_E_INVAL;
        n += sums[E];
    }
    if (int rc = use_device(j)) return rc;
    std::vector<uint64_t> buf(7 * V1);
    std::memcpy(buf.data(), sums, 5 * V1 * 8);
    std::memcpy(buf.data() + 5 * V1, sm4, 2 * V1 * 8);
    HIP_TRY(hipMemcpyAsync(j->d.accum, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, j->stream));
    HIP_TRY(hipStreamSynchronize(j->stream));
    j->recorded = n > 0 ? 1 : 0;
    return MUCA_OK;
}

int muca_reset_accum(muca_job *j)
{
    if (!j) return MUCA_E_INVAL;
    if (int rc = use_device(j)) return rc;
    return clear_accum(j);
}

int muca_set_stats(muca_job *j, int32_t enable)
{
    if (!j) return MUCA_E_INVAL;
    j->stats = enable ? 1 : 0;
    return MUCA_OK;
}

int muca_read_stats(muca_job *j, int64_t *out, int32_t reset)
{
    if (!j || !out) return MUCA_E_INVAL;
    if (int rc = use_device(j)) return rc;
    const size_t off = align_up(8 * ((size_t)j->g.V + 1), 256) + 16;
    uint64_t v[4];
    unsigned char *dh = reinterpret_cast<unsigned char *>(j->d.hist) + off;
    HIP_TRY(hipMemcpyAsync(v, dh, sizeof(v), hipMemcpyDeviceToHost, j->stream));
    HIP_TRY(hipStreamSynchronize(j->stream));
    for (int k = 0; k < 3; ++k) out[k] = (int64_t)v[k];
    if (reset) HIP_TRY(launch_zero(dh, sizeof(v), j->stream));
    return MUCA_OK;
}

int muca_set_launch(muca_job *j, int32_t wpw, int32_t bpl, int32_t lds_tables, int32_t packing)
{
    if (!j) return MUCA_E_INVAL;
    if (!(wpw == 1 || wpw == 2 || wpw == 4) || !(bpl == 1 || bpl == 2) || lds_tables < -1 || lds_tables > 1 ||
        packing < -1 || packing > 1 || (packing == 1 && bpl != 1))
        return MUCA_E_INVAL;
    LaunchPlan pl;
    if (!plan_launch(j, wpw, bpl, lds_tables, packing, &pl)) return MUCA_E_SIZE;
    j->wpw = wpw;
    j->bpl = bpl;
    j->lds_tables_req = lds_tables;
    j->pack_req = packing;
    return MUCA_OK;
}

int muca_get_launch(const muca_job *j, int32_t *wpw, int32_t *bpl, int32_t *lds_tables, int32_t *packing,
                    int32_t *lds_bytes)
{
    if (!j) return MUCA_E_INVAL;
    LaunchPlan pl;
    if (!plan_launch(j, j->wpw, j->bpl, j->lds_tables_req, j->pack_req, &pl)) return MUCA_E_SIZE;
    if (wpw) *wpw = j->wpw;
    if (bpl) *bpl = j->bpl;
    if (lds_tables) *lds_tables = pl.lds_tables ? 1 : 0;
    if (packing) *packing = pl.pack ? 1 : 0;
    if (lds_bytes) *lds_bytes = (int32_t)pl.lds;
    return MUCA_OK;
}

int muca_flatness(const int64_t *hist, int32_t lo, int32_t hi, double *flatness_out)
{
    if (!hist || !flatness_out || lo < 0 || hi < lo) return MUCA_E_INVAL;
    int64_t sum = 0, least = hist[lo];
    for (int32_t E = lo; E <= hi; ++E) {
        if (hist[E] < 0) return MUCA_E_INVAL;
        sum += hist[E];
        least = std::min(least, hist[E]);
    }
    *flatness_out = sum > 0 ? (double)least / ((double)sum / (double)(hi - lo + 1)) : 0.0;
    return MUCA_OK;
}

int muca_host_tables(int32_t L, double T, const double *lnW, int32_t lo, int32_t hi, double *Bp, double *Rp,
                     double *Rm)
{
    if (L < MUCA_L_MIN || L > MUCA_L_MAX || !(T > 0.0) || !lnW || !Bp || !Rp || !Rm) return MUCA_E_INVAL;
    if (lo < 0 || hi > L * L * L || lo >= hi) return MUCA_E_INVAL;
    compute_tables(L * L * L, beta_of(T), lnW, lo, hi, Bp, Rp, Rm);
    return MUCA_OK;
}

int muca_host_walls(int32_t L, double T, int32_t lo, int32_t hi, double *lnW)
{
    if (L < MUCA_L_MIN || L > MUCA_L_MAX || !(T > 0.0) || !lnW) return MUCA_E_INVAL;
    if (lo < 0 || hi > L * L * L || lo >= hi) return MUCA_E_INVAL;
    window_walls(L * L * L, beta_of(T), lo, hi, lnW);
    return MUCA_OK;
}

int muca_host_order(int32_t L, int32_t *order)
{
    if (L < MUCA_L_MIN || L > MUCA_L_MAX || !order) return MUCA_E_INVAL;
    std::vector<int> o;
    int cls[kMaxClasses + 1];
    build_order(L, o, cls);
    for (size_t p = 0; p < o.size(); ++p) order[p] = o[p];
    return MUCA_OK;
}

}  // extern "C"

struct muca_batch {
    std::vector<muca_job *> jobs;
    hipStream_t stream;
    int device;
    unsigned char *dev;
    size_t bytes;
    int n_tiles;
    int wpw, bpl, blocks;  // wpw 0: each job's tiles use job_wpw
    std::vector<int> job_wpw;
    size_t total_walkers;
    size_t tab_bytes;  // LDS reserved for staged tables (0: every job reads them through the caches)
    int pack_req;      // packed lattices: 1 yes, 0 no, -1 automatic
    bool pack;         // the resolved choice
    hipEvent_t done;   // recorded after the last submitted launch
};

namespace {

size_t batch_bytes(size_t n_jobs, size_t walkers)
{
    return align_up(n_jobs * sizeof(BatchJob), 256) + align_up(walkers * sizeof(int2), 256) + 256;
}

// The jobs of one batched launch and the waves per walker of their tiles.
struct BatchPlan {
    muca_job *const *jobs;
    int n;
    int wpw;             // 1, 2 or 4 for every job, or 0: job_wpw[k] for job k
    const int *job_wpw;  // n entries when wpw == 0
    size_t tab_bytes;    // LDS reserved for staged tables (0: none)
    bool pack;           // lattices as 2-bit codes in LDS
    int wpw_of(int k) const { return wpw ? wpw : job_wpw[k]; }
};

// LDS of a block: the fixed part and the lattice slots of the largest tile.
size_t plan_lds(const BatchPlan &p)
{
    size_t lat = 0;
    for (int k = 0; k < p.n; ++k)
        lat = std::max(lat, (size_t)(4 / p.wpw_of(k)) * (size_t)p.jobs[k]->g.Vp / (p.pack ? 4 : 1));
    return kLdsFixed + align_up(lat, 16);
}

// LDS a job's thresholds and neighbour table take when staged.
size_t job_tab_bytes(const muca_job *j)
{
    return align_up(16 * ((size_t)j->g.V + 1 + 2 * kRPad), 16) + align_up((size_t)12 * j->g.Vp, 16);
}

// Per-block LDS up to which a batch stages tables: enough for the thresholds
// of served-size jobs while four blocks still fit on a CU.
constexpr size_t kBatchLdsBudget = 40 * 1024;

// The largest staged-table size that keeps the block within the budget.
size_t plan_tab_bytes(const BatchPlan &p)
{
    const size_t base = plan_lds(p);
    size_t best = 0;
    for (int k = 0; k < p.n; ++k) {
        const size_t t = job_tab_bytes(p.jobs[k]);
        if (base + t <= kBatchLdsBudget) best = std::max(best, t);
    }
    return best;
}

// order[0..n): job indices with the most work per walker (largest V) first,
// equal V in the order given (a stable insertion sort: no allocation).
void heaviest_first(muca_job *const *jobs, int n, int *order)
{
    for (int k = 0; k < n; ++k) {
        int m = k;
        while (m > 0 && jobs[order[m - 1]]->g.V < jobs[k]->g.V) {
            order[m] = order[m - 1];
            --m;
        }
        order[m] = k;
    }
}

// Tiles of the plan: 4/wpw consecutive walkers of one job each.
int count_tiles(const BatchPlan &p)
{
    int t = 0;
    for (int k = 0; k < p.n; ++k) {
        const int wpb = 4 / p.wpw_of(k);
        t += (p.jobs[k]->g.n_walkers + wpb - 1) / wpb;
    }
    return t;
}

// Host images of the device job table (n entries) and of the tile list
// (count_tiles(p) entries, jobs in `order`); returns the number of tiles.
int fill_batch(const BatchPlan &p, const int *order, BatchJob *bj, int2 *tiles)
{
    for (int k = 0; k < p.n; ++k) {
        const muca_job *j = p.jobs[k];
        const Layout &g = j->g;
        unsigned char *dt = reinterpret_cast<unsigned char *>(j->d.tables);
        BatchJob &J = bj[k];
        J.lattice = reinterpret_cast<int8_t *>(j->d.lattice);
        J.wstate = reinterpret_cast<int32_t *>(j->d.walker_state);
        J.hist = reinterpret_cast<unsigned long long *>(j->d.hist);
        J.bp = reinterpret_cast<const double *>(dt + g.off_bp);
        J.r = reinterpret_cast<const double *>(dt + g.off_r);
        J.nb = reinterpret_cast<const uint16_t *>(dt + g.off_nb);
        J.nb2 = reinterpret_cast<const uint16_t *>(dt + g.off_nb2);
        J.acc = reinterpret_cast<unsigned long long *>(j->d.accum);
        J.err = reinterpret_cast<int *>(reinterpret_cast<unsigned char *>(j->d.hist) + align_up(8 * ((size_t)g.V + 1), 256));
        J.V = g.V;
        J.Vp = g.Vp;
        J.n_walkers = g.n_walkers;
        J.n_classes = g.C;
        for (int c = 0; c <= kMaxClasses; ++c) J.cls[c] = g.cls[c];
        J.k0 = j->k0;
        J.k1 = j->k1;
        J.rec_lo = j->win_lo;
        J.rec_hi = j->win_hi;
        J.w0 = j->p.first_walker;
        J.lds_tables = p.tab_bytes > 0 && job_tab_bytes(j) <= p.tab_bytes ? 1 : 0;
        J.wpw = p.wpw_of(k);
    }
    int t = 0;
    for (int m = 0; m < p.n; ++m) {
        const int jx = order[m];
        const int wpb = 4 / p.wpw_of(jx);
        for (int w = 0; w < p.jobs[jx]->g.n_walkers; w += wpb) tiles[t++] = make_int2(jx, w);
    }
    return t;
}

// The enqueue common to both batched entry points: for each chunk of at most
// kMaxSweepsPerLaunch sweeps, clear the work counter (a fill kernel) and launch.
int enqueue_batch(const BatchPlan &p, int bpl, int blocks, const BatchJob *d_jobs, const int2 *d_tiles, int n_tiles,
                  unsigned *d_counter, int64_t n_sweeps, bool record, hipStream_t stream)
{
    BatchArgs a;
    a.jobs = d_jobs;
    a.tiles = d_tiles;
    a.n_tiles = n_tiles;
    a.counter = d_counter;
    a.lds_off_lat = kLdsFixed;
    a.lds_off_tab = (int)plan_lds(p);
    const size_t lds = plan_lds(p) + p.tab_bytes;
    int64_t left = n_sweeps;
    while (left > 0) {
        const int chunk = (int)std::min<int64_t>(left, kMaxSweepsPerLaunch);
        a.n_sweeps = chunk;
        HIP_TRY(launch_zero(d_counter, 16, stream));
        HIP_TRY(launch_batch(a, p.wpw, bpl, record, p.pack, lds, blocks, stream));
        left -= chunk;
    }
    if (record)
        for (int k = 0; k < p.n; ++k) p.jobs[k]->recorded += n_sweeps;
    return MUCA_OK;
}

BatchPlan plan_of(const muca_batch *b, int wpw)
{
    BatchPlan p;
    p.jobs = b->jobs.data();
    p.n = (int)b->jobs.size();
    p.wpw = wpw;
    p.job_wpw = b->job_wpw.data();
    p.tab_bytes = b->tab_bytes;
    p.pack = b->pack;
    return p;
}

// Packing and staged tables of a batched launch.  pack_req 1 or 0 forces the
// packing (packed needs bpl == 1); -1 takes packed lattices only when they
// raise the blocks resident on a compute unit (the staged-table budget then
// also grows).  Returns false if no choice fits in a block's LDS.
bool resolve_batch_plan(BatchPlan &p, int bpl, int pack_req)
{
    const muca_job *j0 = p.jobs[0];
    bool have = false;
    BatchPlan best = p;
    long best_res = 0;
    for (int pk = 0; pk < 2; ++pk) {
        const bool pack = pk == 1;
        if (pack && (bpl != 1 || pack_req == 0)) continue;
        if (!pack && pack_req == 1) continue;
        BatchPlan q = p;
        q.pack = pack;
        q.tab_bytes = 0;
        if (plan_lds(q) > (size_t)j0->max_lds) continue;
        q.tab_bytes = plan_tab_bytes(q);
        const long res = std::min<long>(8, std::max<long>(1, (long)j0->lds_cu / (long)(plan_lds(q) + q.tab_bytes)));
        if (!have || res > best_res) {
            best = q;
            best_res = res;
            have = true;
        }
    }
    if (have) p = best;
    return have;
}

// Waves per walker of each job in a launch that mixes them (an opt-in shape:
// measured on the batched workloads, four-wave walkers of large lattices
// shortened the first launches from a flat start about 2x but lengthened the
// later ones, with steep weights, by 15-20 %, so one wave per walker for every
// job is the default).  A walker at one
// wave per walker is latency-bound at about 12 clocks per site; the whole
// batch, spread over the device at the VALU issue limit, takes about 4 clocks
// per site per SIMD.  A job whose walkers would outlast that share by the
// first measure gets four waves per walker (a block each), provided its colour
// classes fill 4 x 64 lanes of 4 sites, and provided every wave of the batch
// still has a SIMD to itself: the waves of a walker meet at a barrier several
// times per pass, so sharing their SIMDs with other waves costs them more than
// it costs single-wave walkers (measured: slower once the weights are steep).
// Jobs are promoted largest first.  A job whose four lattices do not fit in
// LDS next to each other gets four waves (one lattice per block) regardless.
void choose_job_wpw(muca_batch *b)
{
    double total = 0.0;
    long waves = 0;
    for (const muca_job *j : b->jobs) {
        total += (double)j->g.V * (double)j->g.n_walkers;
        waves += j->g.n_walkers;
    }
    const muca_job *j0 = b->jobs[0];
    const long simds = 4L * (j0->n_cu > 0 ? j0->n_cu : 256);
    b->job_wpw.assign(b->jobs.size(), 1);
    std::vector<int> idx(b->jobs.size());
    heaviest_first(b->jobs.data(), (int)b->jobs.size(), idx.data());
    for (int k : idx) {
        const Layout &g = b->jobs[k]->g;
        const bool fills = g.V / g.C >= 4 * 64 * 4;
        const long extra = 3L * g.n_walkers;
        if (fills && 3.0 * (double)g.V * (double)simds > total && waves + extra <= simds) {
            b->job_wpw[k] = 4;
            waves += extra;
        }
    }
    for (size_t k = 0; k < b->jobs.size(); ++k)
        if (kLdsFixed + align_up((size_t)4 * b->jobs[k]->g.Vp, 16) > (size_t)j0->max_lds) b->job_wpw[k] = 4;
}

int upload_batch(muca_batch *b)
{
    const BatchPlan p = plan_of(b, b->wpw);
    std::vector<int> order(b->jobs.size());
    heaviest_first(p.jobs, p.n, order.data());
    std::vector<BatchJob> bj(b->jobs.size());
    std::vector<int2> tiles((size_t)count_tiles(p));
    b->n_tiles = fill_batch(p, order.data(), bj.data(), tiles.data());
    const size_t off_tiles = align_up(bj.size() * sizeof(BatchJob), 256);
    HIP_TRY(hipMemcpyAsync(b->dev, bj.data(), bj.size() * sizeof(BatchJob), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->dev + off_tiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return MUCA_OK;
}

// Common checks of a job list: non-null, distinct, one device and one stream.
int check_job_list(muca_job *const *jobs, int32_t n_jobs)
{
    if (!jobs || n_jobs < 1) return MUCA_E_INVAL;
    for (int k = 0; k < n_jobs; ++k) {
        if (!jobs[k]) return MUCA_E_INVAL;
        if (jobs[k]->stream != jobs[0]->stream || jobs[k]->device != jobs[0]->device) return MUCA_E_INVAL;
        for (int m = 0; m < k; ++m)
            if (jobs[m] == jobs[k]) return MUCA_E_INVAL;
    }
    return MUCA_OK;
}

// ---------------------------------------------------------------------------
// Device scratch of muca_batch_sweep_static: the job table, the work list and
// the work counter of a batched launch, in a file-scope device array (one copy
// per device, held until the process ends).  In host code `scratch` names a
// host-side stand-in: its device address on each device comes from
// hipGetSymbolAddress, taken once per device when the first job is created
// there (static_scratch_setup), and only that address is passed to kernels.
// ---------------------------------------------------------------------------
constexpr int kStaticMaxJobs = MUCA_STATIC_MAX_JOBS;
constexpr int kStaticMaxTiles = MUCA_STATIC_MAX_TILES;
constexpr size_t kStaticOffTiles = (kStaticMaxJobs * sizeof(BatchJob) + 255) / 256 * 256;
constexpr size_t kStaticOffCounter = kStaticOffTiles + (size_t)kStaticMaxTiles * sizeof(int2);
constexpr size_t kStaticScratchBytes = kStaticOffCounter + 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct StaticScratch {
    unsigned char *dev = nullptr;  // device address of `scratch` on this device
    hipEvent_t staged = nullptr;   // recorded after the last upload from the host images below
    std::mutex lock;               // host images are shared by the calls on this device
    BatchJob host_jobs[kStaticMaxJobs];
    int2 host_tiles[kStaticMaxTiles];
    int order[kStaticMaxJobs];
};

std::mutex g_static_lock;
StaticScratch *g_static[kMaxDevices] = {};
hipError_t g_static_error[kMaxDevices] = {};

// Once per device, with that device current: the device address of the
// scratch array and the event that guards the host images.  A failure is kept
// and reported by muca_batch_sweep_static; it does not fail job creation.
void static_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> guard(g_static_lock);
    if (g_static[device] || g_static_error[device] != hipSuccess) return;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        g_static_error[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        return;
    }
    StaticScratch *st = new (std::nothrow) StaticScratch();
    if (!st) {
        g_static_error[device] = hipErrorOutOfMemory;
        return;
    }
    if ((e = hipEventCreateWithFlags(&st->staged, hipEventDisableTiming)) != hipSuccess) {
        delete st;
        g_static_error[device] = e;
        return;
    }
    st->dev = reinterpret_cast<unsigned char *>(ptr);
    g_static[device] = st;
}

}  // namespace

extern "C" {

int muca_batch_query_size(muca_job *const *jobs, int32_t n_jobs, size_t *bytes)
{
    if (!jobs || n_jobs < 1 || !bytes) return MUCA_E_INVAL;
    size_t walkers = 0;
    for (int k = 0; k < n_jobs; ++k) {
        if (!jobs[k]) return MUCA_E_INVAL;
        walkers += (size_t)jobs[k]->g.n_walkers;
    }
    *bytes = batch_bytes((size_t)n_jobs, walkers);
    return MUCA_OK;
}

int muca_batch_create(muca_job *const *jobs, int32_t n_jobs, void *dev_buffer, size_t bytes, muca_batch **out)
{
    if (!out) return MUCA_E_INVAL;
    *out = nullptr;
    size_t need = 0;
    if (int rc = muca_batch_query_size(jobs, n_jobs, &need)) return rc;
    if (!dev_buffer || (reinterpret_cast<uintptr_t>(dev_buffer) & 255u)) return MUCA_E_INVAL;
    if (bytes < need) return MUCA_E_SIZE;
    if (int rc = check_job_list(jobs, n_jobs)) return rc;
    muca_batch *b = new (std::nothrow) muca_batch();
    if (!b) return MUCA_E_SIZE;
    b->jobs.assign(jobs, jobs + n_jobs);
    b->stream = jobs[0]->stream;
    b->device = jobs[0]->device;
    b->dev = reinterpret_cast<unsigned char *>(dev_buffer);
    b->bytes = bytes;
    b->total_walkers = 0;
    for (muca_job *j : b->jobs) {
        b->total_walkers += (size_t)j->g.n_walkers;
    }
    b->wpw = 1;
    b->bpl = 1;
    b->blocks = 0;
    b->tab_bytes = 0;
    b->pack_req = -1;
    b->pack = false;
    choose_job_wpw(b);  // the shape of a per-job launch, if a caller asks for one
    BatchPlan p = plan_of(b, b->wpw);
    while (!resolve_batch_plan(p, b->bpl, b->pack_req) && p.wpw < 4) p.wpw *= 2;
    if (!resolve_batch_plan(p, b->bpl, b->pack_req)) {
        delete b;
        return MUCA_E_SIZE;
    }
    b->wpw = p.wpw;
    b->pack = p.pack;
    b->tab_bytes = p.tab_bytes;
    if (int rc = use_device(jobs[0])) {
        delete b;
        return rc;
    }
    b->done = nullptr;
    if (int rc = upload_batch(b)) {
        delete b;
        return rc;
    }
    if (hipError_t e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming); e != hipSuccess) {
        delete b;
        return fail_device(e, "hipEventCreate(batch)");
    }
    *out = b;
    return MUCA_OK;
}

int muca_batch_set_launch(muca_batch *b, int32_t wpw, int32_t bpl, int32_t blocks, int32_t packing)
{
    if (!b || !(wpw == 0 || wpw == 1 || wpw == 2 || wpw == 4) || !(bpl == 1 || bpl == 2) || packing < -1 ||
        packing > 1 || (packing == 1 && bpl != 1))
        return MUCA_E_INVAL;
    BatchPlan p = plan_of(b, wpw);
    if (!resolve_batch_plan(p, bpl, packing)) return MUCA_E_SIZE;
    if (int rc = use_device(b->jobs[0])) return rc;
    const int old = b->wpw;
    const bool old_pack = b->pack;
    const size_t old_tab = b->tab_bytes;
    b->wpw = wpw;
    b->bpl = bpl;
    b->blocks = blocks > 0 ? blocks : 0;
    b->pack_req = packing;
    b->pack = p.pack;
    b->tab_bytes = p.tab_bytes;
    if (old != wpw || old_pack != b->pack || old_tab != b->tab_bytes) return upload_batch(b);
    return MUCA_OK;
}

int muca_batch_get_launch(const muca_batch *b, int32_t *waves_per_walker, int32_t *blocks_per_lane,
                          int32_t *packing, int32_t *lds_bytes)
{
    if (!b) return MUCA_E_INVAL;
    const BatchPlan p = plan_of(b, b->wpw);
    if (waves_per_walker)
        for (int k = 0; k < p.n; ++k) waves_per_walker[k] = p.wpw_of(k);
    if (blocks_per_lane) *blocks_per_lane = b->bpl;
    if (packing) *packing = b->pack ? 1 : 0;
    if (lds_bytes) *lds_bytes = (int32_t)(plan_lds(p) + p.tab_bytes);
    return MUCA_OK;
}

int muca_batch_sweep(muca_batch *b, int64_t n_sweeps, uint32_t flags)
{
    if (!b || n_sweeps < 0 || (flags & ~MUCA_RECORD)) return MUCA_E_INVAL;
    if (n_sweeps > MUCA_MAX_SWEEPS_PER_CALL) return MUCA_E_OVERFLOW;
    if (n_sweeps == 0) return MUCA_OK;
    if (int rc = use_device(b->jobs[0])) return rc;
    const size_t off_tiles = align_up(b->jobs.size() * sizeof(BatchJob), 256);
    const size_t off_counter = off_tiles + align_up(b->total_walkers * sizeof(int2), 256);
    return enqueue_batch(plan_of(b, b->wpw), b->bpl, b->blocks, reinterpret_cast<const BatchJob *>(b->dev),
                         reinterpret_cast<const int2 *>(b->dev + off_tiles), b->n_tiles,
                         reinterpret_cast<unsigned *>(b->dev + off_counter), n_sweeps, (flags & MUCA_RECORD) != 0,
                         b->stream);
}

int muca_batch_submit(muca_batch *b, int64_t n_sweeps, uint32_t flags)
{
    if (int rc = muca_batch_sweep(b, n_sweeps, flags)) return rc;
    HIP_TRY(hipEventRecord(b->done, b->stream));
    return MUCA_OK;
}

int muca_batch_poll(muca_batch *b, int32_t *done)
{
    if (!b || !done) return MUCA_E_INVAL;
    if (int rc = use_device(b->jobs[0])) return rc;
    const hipError_t e = hipEventQuery(b->done);
    if (e == hipSuccess) {
        *done = 1;
        return MUCA_OK;
    }
    if (e == hipErrorNotReady) {
        *done = 0;
        return MUCA_OK;
    }
    return fail_device(e, "hipEventQuery(batch)");
}

int muca_batch_finish(muca_batch *b)
{
    if (!b) return MUCA_E_INVAL;
    if (int rc = use_device(b->jobs[0])) return rc;
    HIP_TRY(hipEventSynchronize(b->done));
    return MUCA_OK;
}

void muca_batch_free(muca_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    if (b->done) (void)hipEventDestroy(b->done);
    delete b;
}

int muca_batch_sweep_static(muca_job *const *jobs, int32_t n_jobs, int64_t n_sweeps, uint32_t flags)
{
    if (int rc = check_job_list(jobs, n_jobs)) return rc;
    if (n_sweeps < 0 || (flags & ~MUCA_RECORD)) return MUCA_E_INVAL;
    if (n_jobs > kStaticMaxJobs) return MUCA_E_SIZE;
    if (n_sweeps > MUCA_MAX_SWEEPS_PER_CALL) return MUCA_E_OVERFLOW;
    // the launch shape muca_batch_create picks by default: one wave per
    // walker, more only when the lattice slots do not fit in LDS
    BatchPlan p;
    p.jobs = jobs;
    p.n = n_jobs;
    p.wpw = 1;
    p.job_wpw = nullptr;
    p.tab_bytes = 0;
    p.pack = false;
    while (!resolve_batch_plan(p, 1, -1) && p.wpw < 4) p.wpw *= 2;
    if (!resolve_batch_plan(p, 1, -1)) return MUCA_E_SIZE;
    if (count_tiles(p) > kStaticMaxTiles) return MUCA_E_SIZE;
    if (n_sweeps == 0) return MUCA_OK;
    const int device = jobs[0]->device;
    if (int rc = use_device(jobs[0])) return rc;
    StaticScratch *st = nullptr;
    {
        std::lock_guard<std::mutex> guard(g_static_lock);
        if (device >= 0 && device < kMaxDevices) {
            st = g_static[device];
            if (!st && g_static_error[device] != hipSuccess)
                return fail_device(g_static_error[device], "hipGetSymbolAddress(scratch)");
        }
    }
    if (!st) return MUCA_E_STATE;
    std::lock_guard<std::mutex> guard(st->lock);
    HIP_TRY(hipEventSynchronize(st->staged));  // the previous upload has read the host images
    heaviest_first(jobs, n_jobs, st->order);
    const int n_tiles = fill_batch(p, st->order, st->host_jobs, st->host_tiles);
    hipStream_t stream = jobs[0]->stream;
    HIP_TRY(hipMemcpyAsync(st->dev, st->host_jobs, sizeof(BatchJob) * (size_t)n_jobs, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(st->dev + kStaticOffTiles, st->host_tiles, sizeof(int2) * (size_t)n_tiles,
                           hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventRecord(st->staged, stream));
    return enqueue_batch(p, 1, 0, reinterpret_cast<const BatchJob *>(st->dev),
                         reinterpret_cast<const int2 *>(st->dev + kStaticOffTiles), n_tiles,
                         reinterpret_cast<unsigned *>(st->dev + kStaticOffCounter), n_sweeps,
                         (flags & MUCA_RECORD) != 0, stream);
}

const char *muca_strerror(int code)
{
    switch (code) {
    case MUCA_OK: return "ok";
    case MUCA_E_INVAL: return "invalid argument";
    case MUCA_E_UNSUPPORTED: return "unsupported request";
    case MUCA_E_SIZE: return "size limit exceeded";
    case MUCA_E_STATE: return "call out of order (nothing recorded?)";
    case MUCA_E_OVERFLOW: return "counter overflow";
    case MUCA_E_DEVICE:
        return g_detail.empty() ? "device error" : g_detail.c_str();
    default: return "unknown error code";
    }
}

void muca_free(muca_job *j)
{
    if (!j) return;
    (void)hipSetDevice(j->device);
    (void)hipStreamSynchronize(j->stream);
    if (j->ev_tables) (void)hipEventDestroy(j->ev_tables);
    if (j->pin_tables) (void)hipHostFree(j->pin_tables);
    if (j->pin_hist) (void)hipHostFree(j->pin_hist);
    if (j->pin_obs) (void)hipHostFree(j->pin_obs);
    delete j;
}

}  // extern "C"
