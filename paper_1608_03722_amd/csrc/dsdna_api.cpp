// dsdna_api.cpp -- host runtime of libdsdna: the C ABI of include/dsdna.h.
//
// The context owns every device buffer.  The state machine of a context:
//   NONE       topology set, no positions yet
//   FULL       full-step state uploaded (set_sites / set_state /
//              thermalize / set_velocities): the next step first evaluates
//              the forces of this state (MODE_FIRST)
//   RESUME     full-step state plus its site forces (set_resume): the next
//              step starts from the stored forces (MODE_FROM_FORCES)
//   LEAPFROG   after dsdna_step: positions one step ahead and half-step
//              velocities live in the device buffers; the full-step state is
//              the previous position buffer plus the full-step velocities
//              the last step wrote
//   HALTED     a step raised an error: only getters and setters work
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dsdna.h"
#include "dsdna_dev.h"

using namespace dsdna;

namespace {

enum Phase { PH_NONE = 0, PH_FULL, PH_RESUME, PH_LEAPFROG, PH_HALTED };

constexpr double TWO_16 = 1.12246204830937298143;  // 2^(1/6)
constexpr double DEFAULT_SKIN = 0.5;
constexpr double LIST_SLACK = 1e-4;

// Longest rebuild interval, and steps between two reads of the control block
// (each read waits for the queued work: an outrun or a full list is caught
// there, and the interval adapted): SYNC_FIRST after a state change, then
// twice as many each time up to SYNC_STEPS.
constexpr int K_MAX = 256;
constexpr int64_t SYNC_FIRST = 64;
constexpr int64_t SYNC_STEPS = 500;
// The interval aims at rebuilds when the farthest bead has covered this
// fraction of half the skin.
constexpr double SCHEDULE_FRACTION = 0.95;
// Instantiated step graphs kept per context.
constexpr int GRAPH_CACHE = 6;

}  // namespace

struct dsdna_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    dsdna_params prm{};
    std::string err;

    int32_t n_rep = 0;
    std::vector<int32_t> n_bp;
    std::vector<int64_t> off;
    int64_t N = 0, n_bp_total = 0;
    std::vector<RepInfo> rep_h;
    std::vector<Tile> tiles_h;

    StepArgs a{};  // buffers, physics, grid (host copy)
    StepArgs *dA = nullptr;  // device copy read by the kernels
    StepArgs up{};           // contents of dA as last uploaded
    bool up_valid = false;
    Phase phase = PH_NONE;
    int full_par = 0;
    int64_t full_step = 0;
    int binned_buf = -1;  // buffer the cell list describes, -1 if none
    int cur_par = 0;      // host mirror of ctl.par
    int64_t cur_step = 0; // host mirror of ctl.step
    int64_t state_step = 0;  // step counter at the last state change

    // instantiated step graphs, keyed by their length and rebuild interval:
    // the interval moves between neighbouring values as displacements
    // fluctuate, and each graph is captured once (least recently used first
    // out)
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        int steps = 0;
        int K = 0;
        uint64_t used = 0;
    };
    StepGraph graphs[GRAPH_CACHE];
    uint64_t graph_clock = 0;

    // neighbour-list schedule: a rebuild follows every K-th step kernel;
    // `age` step kernels have run since the last rebuild
    int K = 4;
    int age = 0;
    int64_t outruns = 0;   // beads that outran the schedule since the last state change
    int64_t sync_batch = 64;  // steps until the next read of the control block
    bool rebuilt = false;     // a scheduled rebuild ran since the last read

    // curve sets of the linking-number kernels (one per replica of at least
    // two base pairs) and their scratch, built at the first linking call
    // after a change of topology or ring flags
    std::vector<CurveSet> sets_h;
    std::vector<int32_t> set_rep;   // replica of each set
    CurveSet *d_sets = nullptr;
    int2 *d_lkblk = nullptr;
    double *d_curves = nullptr, *d_lkpart = nullptr, *d_lkout = nullptr;
    int lk_blocks = 0, lk_pts = 0;
    bool lk_stale = true;
    hipEvent_t lk_ev[2] = {nullptr, nullptr};

    // per-replica energies, and the bubble statistics' scratch and results
    // (sized for bub_nhist bins)
    double *d_rep_e = nullptr;
    int32_t *d_bub_hist = nullptr;
    int4 *d_bub_info = nullptr;
    double *d_bub_frac = nullptr;
    int64_t *d_bub_out = nullptr;
    int bub_nhist = 0;

    // the context's own full-step velocity buffers while the caller's arrays
    // are bound in their place (null when nothing is bound)
    double *own_Vf = nullptr, *own_Lf = nullptr;
};

static bool is_bound(const dsdna_ctx *c) { return c->own_Vf != nullptr; }

// ------------------------------------------------------------------ helpers

// Last failure of a context-free call on this thread.
static thread_local std::string g_free_error = "null context";

void dsdna::set_free_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_free_error = buf;
}

static dsdna_status fail(dsdna_ctx *c, dsdna_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

#define HIPCHK(c, expr)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail((c), DSDNA_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

template <typename T>
static hipError_t dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

static void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

static void free_curves(dsdna_ctx *c)
{
    dfree(c->d_sets); dfree(c->d_lkblk); dfree(c->d_curves); dfree(c->d_lkpart); dfree(c->d_lkout);
    c->d_sets = nullptr; c->d_lkblk = nullptr; c->d_curves = c->d_lkpart = c->d_lkout = nullptr;
    c->sets_h.clear();
    c->set_rep.clear();
    c->lk_blocks = c->lk_pts = 0;
    c->lk_stale = true;
}

static void free_bubbles(dsdna_ctx *c)
{
    dfree(c->d_bub_hist); dfree(c->d_bub_info); dfree(c->d_bub_frac); dfree(c->d_bub_out);
    c->d_bub_hist = nullptr;
    c->d_bub_info = nullptr;
    c->d_bub_frac = nullptr;
    c->d_bub_out = nullptr;
    c->bub_nhist = 0;
}

static void free_state(dsdna_ctx *c)
{
    free_curves(c);
    free_bubbles(c);
    dfree(c->d_rep_e);
    c->d_rep_e = nullptr;
    Bufs &b = c->a.b;
    if (is_bound(c)) {  // the bound arrays are the caller's
        b.Vf = c->own_Vf;
        b.Lf = c->own_Lf;
        c->own_Vf = c->own_Lf = nullptr;
    }
    for (int k = 0; k < 2; ++k) {
        dfree(b.R[k]); dfree(b.u[k]); dfree(b.V[k]); dfree(b.L[k]);
    }
    dfree(b.Vf); dfree(b.Lf); dfree(b.Fb); dfree(b.Fp);
    dfree(b.rec); dfree(b.rcell); dfree(b.key); dfree(b.slot); dfree(b.srec); dfree(b.sid); dfree(b.scell);
    dfree(b.fex); dfree(b.cmask); dfree(b.eex); dfree(b.plist); dfree(b.vmax);
    dfree(b.rep); dfree(b.tiles); dfree(b.eacc); dfree(b.open);
    dfree(b.diag_fb); dfree(b.diag_fp);
    dfree(b.k2bp);
    Ctl *ctl = b.ctl;
    uint32_t *count = b.count;
    int32_t *start = b.start, *bsum = b.bsum;
    std::memset(&b, 0, sizeof b);
    b.ctl = ctl;
    b.count = count; b.start = start; b.bsum = bsum;
}

static void free_grid(dsdna_ctx *c)
{
    dfree(c->a.b.count); dfree(c->a.b.start); dfree(c->a.b.bsum);
    c->a.b.count = nullptr;
    c->a.b.start = c->a.b.bsum = nullptr;
}

// Upload the argument block if it changed since the last upload.  Never
// called during graph capture: a captured graph reads the block through dA.
static dsdna_status sync_args(dsdna_ctx *c)
{
    if (!c->dA) {
        HIPCHK(c, dalloc(&c->dA, 1));
        c->up_valid = false;
    }
    if (c->up_valid && std::memcmp(&c->up, &c->a, sizeof(StepArgs)) == 0) return DSDNA_OK;
    std::memcpy(&c->up, &c->a, sizeof(StepArgs));
    HIPCHK(c, hipMemcpyAsync(c->dA, &c->up, sizeof(StepArgs), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->up_valid = true;
    return DSDNA_OK;
}

static void drop_graph(dsdna_ctx *c)
{
    for (auto &g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = dsdna_ctx::StepGraph{};
    }
}

static void fill_phys(dsdna_ctx *c)
{
    const dsdna_params &p = c->prm;
    Phys &h = c->a.ph;
    h.K1 = p.K1; h.R0 = p.R0; h.eps_bb = p.eps_bb; h.sig_bb = p.sig_bb;
    h.K2 = p.K2; h.r0_hb = p.r0_hb; h.rc_hb = p.rc_hb;
    h.eps = p.eps; h.sig_s = p.sig_s; h.sig_x = p.sig_x;
    h.K3 = p.K3; h.d_dih = p.d_dih; h.K4 = p.K4; h.lam = p.lam; h.r0_m = p.r0_m;
    h.K5 = p.K5; h.a0 = p.a0; h.K6 = p.K6;
    h.ell = p.ell; h.m_bead = p.m_bead; h.m_patch = p.m_patch;
    h.gamma = p.gamma; h.kT = p.kT; h.dt = p.dt;
    h.M = p.m_bead + p.m_patch;
    h.I = p.m_bead * p.m_patch / h.M * p.ell * p.ell;
    h.db = p.ell * p.m_patch / h.M;
    h.dp = p.ell * p.m_bead / h.M;
    h.noise_amp = std::sqrt(2.0 * p.gamma * p.kT / p.dt);
    const double w = (p.r0_hb - p.rc_hb) * (p.r0_hb - p.rc_hb);
    h.hb_pref = p.hb_depth_convention == 0 ? p.K2 / (2.0 * w) : p.K2 / w;
    h.rc_bb = TWO_16 * p.sig_bb;
    h.rc_s = TWO_16 * p.sig_s;
    h.rc_x = TWO_16 * p.sig_x;
    h.cos_d = std::cos(p.d_dih);
    h.sin_d = std::sin(p.d_dih);
    h.cos_a0 = std::cos(p.a0);
    h.sin_a0 = std::sin(p.a0);
    h.kick = 0.5 * p.dt;
    h.skin = p.skin > 0.0 ? p.skin : DEFAULT_SKIN;
    // list cutoffs carry a slack for their FP32 evaluation on the fixed-point
    // records; the stale threshold is as much below half the skin, so a pair
    // left out of the list cannot come within its cutoff before a rebuild
    h.rl2_s = (h.rc_s + h.skin + LIST_SLACK) * (h.rc_s + h.skin + LIST_SLACK);
    h.rl2_x = (h.rc_x + h.skin + LIST_SLACK) * (h.rc_x + h.skin + LIST_SLACK);
    h.half_skin2 = (float)((0.5 * h.skin - LIST_SLACK) * (0.5 * h.skin - LIST_SLACK));
    h.inv_I = 1.0 / h.I;
    h.kick_M = h.kick / h.M;
    h.inv_R0sq = 1.0 / (p.R0 * p.R0);
    h.seed = p.seed;
    h.noise_kind = p.noise_kind;
    h.ssdna_rule = p.ssdna_rule;
    h.fene_clamp = p.fene_clamp;
    h.dihedral_damping = p.dihedral_damping;
    h.planarity_both = p.planarity_both;
}

// Reach of the neighbour search: the largest WCA cutoff plus the skin.
static double rc_max(const dsdna_ctx *c)
{
    return TWO_16 * std::max(c->prm.sig_s, c->prm.sig_x) + c->a.ph.skin + LIST_SLACK;
}

static double cell_edge(const dsdna_ctx *c)
{
    // default: just above the search reach (fewest candidates per bead)
    return c->prm.cell_size > 0.0 ? c->prm.cell_size : rc_max(c) * 1.001;
}

// The 27 cells around any cell must hash to 27 distinct buckets, also across
// periodic wraps: check every coordinate difference two such cells can have.
static bool hash_separates(uint32_t A, uint32_t B, uint32_t mask, const std::vector<RepInfo> &reps)
{
    for (const RepInfo &r : reps) {
        std::vector<int64_t> D[3];
        for (int k = 0; k < 3; ++k) {
            const bool per = r.flags & (REP_PER_X << k);
            for (int d = -2; d <= 2; ++d) {
                if (!per) { D[k].push_back(d); continue; }
                const int64_t n = r.ncell[k];
                for (int w = -1; w <= 1; ++w) {
                    const int64_t v = d + w * n;
                    if (v > -n && v < n) D[k].push_back(v);
                }
            }
            std::sort(D[k].begin(), D[k].end());
            D[k].erase(std::unique(D[k].begin(), D[k].end()), D[k].end());
        }
        for (int64_t dx : D[0])
            for (int64_t dy : D[1])
                for (int64_t dz : D[2]) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    const uint32_t k = ((uint32_t)dx + A * (uint32_t)dy + B * (uint32_t)dz) & mask;
                    if (k == 0) return false;
                }
    }
    return true;
}

// Choose the cell edge, per-replica cell counts, bucket count and hash for
// the replicas `reps` (the context's, or a candidate set of them).  The new
// replica table and grid are built in local copies and become the context's
// only when every check and allocation has succeeded, so a failure leaves the
// context as it was.
static dsdna_status configure_grid_for(dsdna_ctx *c, std::vector<RepInfo> reps)
{
    const double h = cell_edge(c);
    const double reach = rc_max(c);
    if (!(h >= reach * (1.0 + 1e-6)))
        return fail(c, DSDNA_EINVAL, "cell_size %g is below the search reach %g (largest WCA cutoff plus skin)", h,
                    reach);
    bool all_per_same = c->n_rep > 0;
    for (int r = 0; r < c->n_rep; ++r) {
        RepInfo &ri = reps[r];
        for (int k = 0; k < 3; ++k) {
            if (ri.flags & (REP_PER_X << k)) {
                const int64_t n = (int64_t)std::floor(ri.len[k] / h);
                if (n < 3)
                    return fail(c, DSDNA_EINVAL, "replica %d: periodic edge %g holds fewer than 3 cells of %g", r,
                                ri.len[k], h);
                if (n > (1 << 20)) return fail(c, DSDNA_EINVAL, "replica %d: periodic edge too long", r);
                // cells are cut on the 32-bit coordinates (unit L / 2^32): a
                // cell must stay wider than the reach plus a few units
                if (ri.len[k] / (double)n < reach + 4.0 * ri.len[k] / 4294967296.0)
                    return fail(c, DSDNA_EINVAL, "replica %d: periodic edge %g too long for cell %g", r, ri.len[k], h);
                ri.ncell[k] = (int32_t)n;
                ri.inv_h[k] = (double)n / ri.len[k];
            } else {
                ri.ncell[k] = 0;
                ri.inv_h[k] = 1.0 / h;
                all_per_same = false;
            }
        }
        if (r > 0)
            for (int k = 0; k < 3; ++k) all_per_same = all_per_same && ri.ncell[k] == reps[0].ncell[k];
    }
    int lg = c->prm.hash_log2;
    if (lg <= 0) {
        // about four buckets per bead: few records of far cells share the
        // buckets of a bead's neighbourhood
        int64_t want = std::max<int64_t>(SCAN_CHUNK, 4 * c->N);
        lg = 12;
        while ((int64_t(1) << lg) < want && lg < 24) ++lg;
    }
    if (lg < 12 || lg > 28) return fail(c, DSDNA_EINVAL, "hash_log2 %d out of [12, 28]", lg);
    // bucket counters are 16 bits: keep the mean load far below that
    if (c->N > ((int64_t)1 << lg) * 4096)
        return fail(c, DSDNA_EINVAL, "hash_log2 %d too small for %lld nucleotides", lg, (long long)c->N);
    const uint32_t nb = 1u << lg, mask = nb - 1u;
    uint32_t A = 1031u, B = 1031u * 1031u;
    if (all_per_same) {
        A = (uint32_t)reps[0].ncell[0];
        B = A * (uint32_t)reps[0].ncell[1];
    }
    // fall back to other odd multipliers if the first choice folds two
    // neighbouring cells into one bucket
    uint64_t x = 0x9E3779B97F4A7C15ull;
    int tries = 0;
    while (!hash_separates(A, B, mask, reps)) {
        if (++tries > 1000) return fail(c, DSDNA_EINVAL, "no cell hash separates neighbours with 2^%d buckets", lg);
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;
        A = ((uint32_t)x | 1u) & 0xFFFFu;
        if (A < 17) A += 17;
        B = (uint32_t)(x >> 32) | 1u;
    }
    Grid g = c->a.g;
    g.A = A;
    g.B = B;
    g.C = all_per_same ? B * (uint32_t)reps[0].ncell[2] : B * 1031u + 7u;
    g.mask = mask;
    g.h = h;
    g.any_open = 0;
    for (int r = 0; r < c->n_rep; ++r)
        for (int k = 0; k < 3; ++k) g.any_open |= (reps[r].flags & (REP_PER_X << k)) ? 0 : 1;
    g.fast_screen = c->n_rep == 1;
    for (int r = 0; r < c->n_rep; ++r) {
        RepInfo &ri = reps[r];
        for (int k = 0; k < 3; ++k)
            ri.qlen[k] = (ri.flags & (REP_PER_X << k)) ? (float)(ri.len[k] / 4294967296.0) : (float)(1.0 / OPEN_QINV);
        g.fast_screen = g.fast_screen && ri.qlen[0] == ri.qlen[1] && ri.qlen[1] == ri.qlen[2];
    }
    const bool new_buckets = c->a.g.nbucket != (int32_t)nb || !c->a.b.count;
    uint32_t *count = nullptr;
    int32_t *start = nullptr, *bsum = nullptr;
    const auto drop = [&] { dfree(count); dfree(start); dfree(bsum); };
    if (new_buckets) {
        if (dalloc(&count, (size_t)nb / 2) != hipSuccess || dalloc(&start, (size_t)nb + 1) != hipSuccess ||
            dalloc(&bsum, (size_t)nb / SCAN_CHUNK) != hipSuccess) {
            drop();
            return fail(c, DSDNA_ENOMEM, "cell-list allocation for 2^%d buckets failed", lg);
        }
    }
    hipError_t e = hipSuccess;
    if (new_buckets) e = hipMemsetAsync(count, 0, sizeof(uint32_t) * (nb / 2), c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->a.b.rep, reps.data(), sizeof(RepInfo) * c->n_rep, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        drop();
        // the device table may be partly written: put the previous one back
        (void)hipMemcpyAsync(c->a.b.rep, c->rep_h.data(), sizeof(RepInfo) * c->n_rep, hipMemcpyHostToDevice,
                             c->stream);
        (void)hipStreamSynchronize(c->stream);
        return fail(c, DSDNA_EDEVICE, "grid upload failed: %s", hipGetErrorString(e));
    }
    if (new_buckets) {
        free_grid(c);
        c->a.b.count = count;
        c->a.b.start = start;
        c->a.b.bsum = bsum;
        g.nbucket = (int32_t)nb;
    }
    c->rep_h = std::move(reps);
    c->a.g = g;
    c->binned_buf = -1;
    drop_graph(c);
    return DSDNA_OK;
}

static dsdna_status configure_grid(dsdna_ctx *c) { return configure_grid_for(c, c->rep_h); }

// Clear the cell histogram and the sparse excluded-volume accumulators (a
// halted step or evaluation may leave entries behind).  Not used during graph
// capture.
static dsdna_status clear_accumulators(dsdna_ctx *c)
{
    Bufs &b = c->a.b;
    HIPCHK(c, hipMemsetAsync(b.count, 0, sizeof(uint32_t) * ((size_t)c->a.g.nbucket / 2), c->stream));
    HIPCHK(c, hipMemsetAsync(b.fex, 0, sizeof(unsigned long long) * FEX_WORDS * (size_t)c->N, c->stream));
    HIPCHK(c, hipMemsetAsync(b.cmask, 0, sizeof(uint32_t) * CMASK_WORDS * (size_t)c->a.n_tiles, c->stream));
    return DSDNA_OK;
}

static dsdna_status upload_reps(dsdna_ctx *c)
{
    HIPCHK(c, hipMemcpyAsync(c->a.b.rep, c->rep_h.data(), sizeof(RepInfo) * c->n_rep, hipMemcpyHostToDevice,
                             c->stream));
    return DSDNA_OK;
}

static dsdna_status write_ctl(dsdna_ctx *c, int64_t step, int par)
{
    Ctl h{};
    h.step = step;
    h.par = par;
    h.done_step = step - 1;
    h.done_par = par ^ 1;
    HIPCHK(c, hipMemcpyAsync(c->a.b.ctl, &h, sizeof h, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->cur_step = step;
    c->cur_par = par;
    c->state_step = step;
    c->outruns = 0;
    c->sync_batch = SYNC_FIRST;
    return DSDNA_OK;
}

static dsdna_status read_ctl(dsdna_ctx *c, Ctl *h)
{
    HIPCHK(c, hipMemcpyAsync(h, c->a.b.ctl, sizeof *h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DSDNA_OK;
}

// Copy on the context's stream and wait for it (the stream does not
// synchronise with the legacy default stream).
static dsdna_status copy(dsdna_ctx *c, void *dst, const void *src, size_t bytes, hipMemcpyKind kind)
{
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, kind, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DSDNA_OK;
}

// SoA device [3][N] <-> host [N][3]
static dsdna_status up3(dsdna_ctx *c, double *dst, const double *src)
{
    std::vector<double> t(3 * (size_t)c->N);
    for (int64_t i = 0; i < c->N; ++i)
        for (int k = 0; k < 3; ++k) t[k * c->N + i] = src[3 * i + k];
    return copy(c, dst, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice);
}

static dsdna_status down3(dsdna_ctx *c, double *dst, const double *src)
{
    std::vector<double> t(3 * (size_t)c->N);
    dsdna_status st = copy(c, t.data(), src, sizeof(double) * t.size(), hipMemcpyDeviceToHost);
    if (st) return st;
    for (int64_t i = 0; i < c->N; ++i)
        for (int k = 0; k < 3; ++k) dst[3 * i + k] = t[k * c->N + i];
    return DSDNA_OK;
}

static dsdna_status check_ready(dsdna_ctx *c, bool need_state)
{
    if (!c) return DSDNA_EINVAL;
    if (c->n_rep == 0) return fail(c, DSDNA_ESTATE, "set_topology has not been called");
    if (need_state && c->phase == PH_NONE) return fail(c, DSDNA_ESTATE, "no positions: call set_sites or set_state");
    return DSDNA_OK;
}

// Enlarge the neighbour-list buffer to hold at least `need` pairs.
static dsdna_status grow_list(dsdna_ctx *c, int64_t need)
{
    const int64_t cap = std::max<int64_t>(need + need / 4 + 64, 2 * c->a.list_cap);
    PairRec *p = nullptr;
    if (dalloc(&p, (size_t)cap) != hipSuccess)
        return fail(c, DSDNA_ENOMEM, "neighbour list of %lld pairs: allocation failed", (long long)cap);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c->a.b.plist);
    c->a.b.plist = p;
    c->a.list_cap = cap;
    return sync_args(c);
}

// Rebuild the neighbour list from the positions of buffer `which`: bin,
// scan, scatter, search.  A list larger than its buffer is rebuilt into a
// larger one.  Clears a stale mark and restarts the rebuild schedule.
static dsdna_status rebin(dsdna_ctx *c, int which)
{
    dsdna_status st = sync_args(c);
    if (st) return st;
    Ctl h;
    if ((st = read_ctl(c, &h))) return st;
    if (h.halt_step != 0) {
        h.halt_step = 0;
        if ((st = copy(c, c->a.b.ctl, &h, sizeof h, hipMemcpyHostToDevice))) return st;
    }
    for (;;) {
        // the histogram is cleared by the search that ends a rebuild, which an
        // error may have cut short
        HIPCHK(c, hipMemsetAsync(c->a.b.count, 0, sizeof(uint32_t) * ((size_t)c->a.g.nbucket / 2), c->stream));
        HIPCHK(c, launch_bin(c->a, c->dA, which, c->stream));
        HIPCHK(c, launch_scan(c->a, c->stream));
        HIPCHK(c, launch_scatter(c->a, c->stream));
        HIPCHK(c, launch_build(c->a, c->dA, c->stream));
        if ((st = read_ctl(c, &h))) return st;
        if (h.code != 0) break;  // the caller reads the error
        if (h.list_n > (uint64_t)c->a.list_cap) {
            if ((st = grow_list(c, (int64_t)h.list_n))) return st;
            h.halt_step = 0;
            if ((st = copy(c, c->a.b.ctl, &h, sizeof h, hipMemcpyHostToDevice))) return st;
            continue;
        }
        c->binned_buf = which;
        c->age = 0;
        return DSDNA_OK;
    }
    c->binned_buf = -1;
    return DSDNA_OK;
}

// Make buffer 0 the full-step state at `step`: the next step starts from a
// force evaluation there.
static dsdna_status start_from_buffer0(dsdna_ctx *c, int64_t step)
{
    dsdna_status st;
    // a halted step may have left histogram or accumulator entries behind
    if ((st = clear_accumulators(c))) return st;
    if ((st = write_ctl(c, step, 0))) return st;
    c->full_par = 0;
    c->full_step = step;
    c->binned_buf = -1;
    c->phase = PH_FULL;
    return DSDNA_OK;
}

// Copy the full-step positions and axes of buffer p into the bound arrays
// (their velocities are the full-step buffers themselves), and with
// `velocities` also the buffer's own velocities.
static dsdna_status mirror_bound(dsdna_ctx *c, int p, bool velocities)
{
    if (!is_bound(c)) return DSDNA_OK;
    Bufs &b = c->a.b;
    const size_t n = sizeof(double) * 3 * (size_t)c->N;
    HIPCHK(c, hipMemcpyAsync(b.Rf, b.R[p], n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b.uf, b.u[p], n, hipMemcpyDeviceToDevice, c->stream));
    if (velocities) {
        HIPCHK(c, hipMemcpyAsync(b.Vf, b.V[p], n, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(b.Lf, b.L[p], n, hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DSDNA_OK;
}

static dsdna_status upload_full_state(dsdna_ctx *c, const double *R, const double *V, const double *u,
                                      const double *L, int64_t step)
{
    Bufs &b = c->a.b;
    dsdna_status st;
    if ((st = up3(c, b.R[0], R)) || (st = up3(c, b.u[0], u))) return st;
    if (V) {
        if ((st = up3(c, b.V[0], V))) return st;
    } else {
        HIPCHK(c, hipMemsetAsync(b.V[0], 0, sizeof(double) * 3 * c->N, c->stream));
    }
    if (L) {
        if ((st = up3(c, b.L[0], L))) return st;
    } else {
        HIPCHK(c, hipMemsetAsync(b.L[0], 0, sizeof(double) * 3 * c->N, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(b.Vf, b.V[0], sizeof(double) * 3 * c->N, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b.Lf, b.L[0], sizeof(double) * 3 * c->N, hipMemcpyDeviceToDevice, c->stream));
    if ((st = mirror_bound(c, 0, false))) return st;
    return start_from_buffer0(c, step);
}

// Bring a LEAPFROG context back to its full-step state in buffer full_par so
// that velocities can be replaced.
static dsdna_status to_full(dsdna_ctx *c)
{
    if (c->phase != PH_LEAPFROG && c->phase != PH_RESUME && c->phase != PH_HALTED) return DSDNA_OK;
    Bufs &b = c->a.b;
    const int p = c->full_par;
    if (c->phase != PH_HALTED) {  // halted: the buffer keeps its own velocities
        HIPCHK(c, hipMemcpyAsync(b.V[p], b.Vf, sizeof(double) * 3 * c->N, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(b.L[p], b.Lf, sizeof(double) * 3 * c->N, hipMemcpyDeviceToDevice, c->stream));
    }
    dsdna_status st = clear_accumulators(c);
    if (st) return st;
    st = write_ctl(c, c->full_step, p);
    if (st) return st;
    c->binned_buf = -1;
    c->phase = PH_FULL;
    return DSDNA_OK;
}

static dsdna_status status_from_ctl(dsdna_ctx *c, const Ctl &h)
{
    if (h.code == 0) return DSDNA_OK;
    c->phase = PH_HALTED;
    c->full_par = h.par;
    c->full_step = h.step;
    // bound arrays show the state the error left, velocities included
    const dsdna_status ms = mirror_bound(c, h.par, true);
    if (ms) return ms;
    const char *what = h.code == DSDNA_EBOND    ? "backbone bond reached R0 (FENE energy infinite)"
                       : h.code == DSDNA_ENAN   ? "non-finite position or orientation"
                       : h.code == DSDNA_EWALL  ? "bead reached the anchoring wall"
                       : h.code == DSDNA_EDOMAIN ? "bead left the representable coordinate range"
                       : h.code == DSDNA_ECELL  ? "more than 65535 beads in one cell-list bucket (raise hash_log2)"
                                                 : "device error";
    return fail(c, (dsdna_status)h.code, "%s at step %lld, nucleotide %lld", what, (long long)h.err_step,
                (long long)h.err_id);
}

// One step: the neighbour-list pairs and the step kernel, then, when the
// schedule says so, the kernels of a rebuild from the new positions.  `ev`
// (7 events, or null) brackets the kernels: pairs, step, bin, scan,
// scatter, build.
static hipError_t enqueue_step(dsdna_ctx *c, int mode, int write_full, int rebuild_after, int age, hipStream_t s,
                               hipEvent_t *ev = nullptr)
{
    hipError_t e = hipSuccess;
    auto mark = [&](int k) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[k], s);
    };
    mark(0);
    // the pair kernel publishes the step; a resume from stored forces
    // evaluates no forces in its first launch
    e = launch_pairs(c->a, c->dA, -1, 0, mode == MODE_FROM_FORCES ? PAIRS_PUBLISH : PAIRS_STEP, s);
    mark(1);
    if (e == hipSuccess) e = launch_step(c->a, c->dA, c->prm.force_fp64, mode, write_full, rebuild_after, age, s);
    mark(2);
    if (rebuild_after) {
        // the step kernel has binned its new beads
        mark(3);
        if (e == hipSuccess) e = launch_scan(c->a, s);
        mark(4);
        if (e == hipSuccess) e = launch_scatter(c->a, s);
        mark(5);
        if (e == hipSuccess) e = launch_build(c->a, c->dA, s);
    } else {
        mark(3);
        mark(4);
        mark(5);
    }
    mark(6);
    return e;
}

// A graph of `steps` steps (a multiple of the rebuild interval K) that starts
// right after a rebuild: rebuilds follow its K-th, 2K-th, ... step.  Taken
// from the cache when there, else captured into the least recently used slot.
static dsdna_status step_graph(dsdna_ctx *c, int steps, int K, hipGraphExec_t *out)
{
    dsdna_ctx::StepGraph *slot = &c->graphs[0];
    for (auto &g : c->graphs) {
        if (g.exec && g.steps == steps && g.K == K) {
            g.used = ++c->graph_clock;
            *out = g.exec;
            return DSDNA_OK;
        }
        if (!g.exec || (slot->exec && g.used < slot->used)) slot = &g;
    }
    if (slot->exec) (void)hipGraphExecDestroy(slot->exec);
    *slot = dsdna_ctx::StepGraph{};
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < steps && e == hipSuccess; ++k)
        e = enqueue_step(c, MODE_NORMAL, 0, (k + 1) % K == 0, k % K + 1, c->stream);
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c, DSDNA_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, DSDNA_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    slot->exec = x;
    slot->steps = steps;
    slot->K = K;
    slot->used = ++c->graph_clock;
    *out = x;
    return DSDNA_OK;
}

// Kernel classes timed by dsdna_profile_kernels, in the order enqueue_step
// brackets them.
static const int PROF_CLASS[6] = {DSDNA_KERNEL_EXCL, DSDNA_KERNEL_STEP, DSDNA_KERNEL_BIN,
                                  DSDNA_KERNEL_SCAN, DSDNA_KERNEL_SCATTER, DSDNA_KERNEL_BUILD};

// Rebuild interval from the largest displacement of a bead over an interval
// since the last read (the per-tile maxima, which are then cleared): scaled
// by SCHEDULE_FRACTION of half the skin over that displacement, at most
// doubled or halved at a time.  Displacements grow at most linearly with
// the interval, so the scaling approaches the target from either side.
static dsdna_status adapt_interval(dsdna_ctx *c)
{
    if (!c->rebuilt) return DSDNA_OK;  // nothing measured since the last read
    c->rebuilt = false;
    std::vector<float> v((size_t)c->a.n_tiles);
    dsdna_status st = copy(c, v.data(), c->a.b.vmax, sizeof(float) * v.size(), hipMemcpyDeviceToHost);
    if (st) return st;
    HIPCHK(c, hipMemsetAsync(c->a.b.vmax, 0, sizeof(float) * v.size(), c->stream));
    float d2 = 0.0f;
    for (float x : v) d2 = std::max(d2, x);
    const double half = 0.5 * c->a.ph.skin - LIST_SLACK;
    double k = 2.0 * c->K;
    if (d2 > 0.0f) k = std::min(k, std::floor(c->K * SCHEDULE_FRACTION * half / std::sqrt((double)d2)));
    c->K = (int)std::max(1.0, std::min((double)K_MAX, std::max(k, (double)(c->K / 2))));
    return DSDNA_OK;
}

// Run n_steps; with `prof`, eager launches with events around every kernel
// and the mean duration per step of each kernel class.
static dsdna_status run_steps(dsdna_ctx *c, int64_t n_steps, std::vector<double> *prof)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (n_steps < 0) return fail(c, DSDNA_EINVAL, "n_steps < 0");
    if (c->phase == PH_HALTED) return fail(c, DSDNA_ESTATE, "halted by an earlier error; set a state first");
    if (n_steps == 0) return DSDNA_OK;
    if ((st = sync_args(c))) return st;
    if (c->binned_buf != c->cur_par) {
        if ((st = rebin(c, c->cur_par))) return st;
    }
    int64_t launches = n_steps;
    int first_mode = MODE_NORMAL;
    if (c->phase == PH_FULL) { first_mode = MODE_FIRST; launches += 1; }
    if (c->phase == PH_RESUME) { first_mode = MODE_FROM_FORCES; launches += 1; }
    const int64_t step0 = c->cur_step;
    if (prof) prof->assign(DSDNA_NKERNELS, 0.0);
    std::vector<hipEvent_t> evs;
    const auto free_events = [&] {
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
        evs.clear();
    };
    const auto give_up = [&](dsdna_status code) {
        free_events();
        return code;
    };
    // one eager launch, following the schedule
    const auto one = [&](int64_t k) -> hipError_t {
        const int rebuild_after = c->age + 1 >= c->K;
        hipEvent_t *ev = nullptr;
        if (prof) {
            const size_t e0 = evs.size();
            evs.resize(e0 + 7, nullptr);
            for (int q = 0; q < 7; ++q) {
                const hipError_t e = hipEventCreate(&evs[e0 + q]);
                if (e != hipSuccess) return e;
            }
            ev = &evs[e0];
        }
        const hipError_t e = enqueue_step(c, k == 0 ? first_mode : MODE_NORMAL, k == launches - 1, rebuild_after,
                                          c->age + 1, c->stream, ev);
        c->age = rebuild_after ? 0 : c->age + 1;
        c->rebuilt = c->rebuilt || rebuild_after;
        return e;
    };
    int64_t k = 0;  // launches done
    Ctl h;
    while (k < launches) {
        int64_t end = std::min(launches, k + c->sync_batch);
        c->sync_batch = std::min(SYNC_STEPS, 2 * c->sync_batch);
        const auto launch_fail = [&](hipError_t e) {
            return give_up(fail(c, DSDNA_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e)));
        };
        hipError_t e = hipSuccess;
        if (k == 0 && first_mode != MODE_NORMAL) {
            if ((e = one(k)) != hipSuccess) return launch_fail(e);
            ++k;
        }
        const int G0 = c->prm.graph_steps;
        if (!prof && G0 > 0) {
            // graphs end before the run's last launch, which writes the
            // full-step state; eager steps up to the next rebuild, then whole
            // graphs.  Short of the run's end the batch is stretched to a
            // whole number of graphs, so that the next starts on a rebuild.
            const int64_t gend = end == launches ? end - 1 : end;
            while (c->age != 0 && k < gend) {
                if ((e = one(k)) != hipSuccess) return launch_fail(e);
                ++k;
            }
            const int G = (G0 + c->K - 1) / c->K * c->K;
            int64_t n_g = (gend - k) / G;
            if (end != launches) n_g = std::min((gend - k + G - 1) / G, (launches - 1 - k) / G);
            if (c->age == 0 && n_g > 0) {
                hipGraphExec_t gx = nullptr;
                if ((st = step_graph(c, G, c->K, &gx))) return st;
                for (int64_t q = 0; q < n_g; ++q) {
                    if ((e = hipGraphLaunch(gx, c->stream)) != hipSuccess) return launch_fail(e);
                    k += G;
                    c->rebuilt = true;
                }
                end = std::max(end, k);
            }
        }
        for (; k < end; ++k)
            if ((e = one(k)) != hipSuccess) return launch_fail(e);
        if ((st = read_ctl(c, &h))) return give_up(st);
        if (h.code != 0) break;  // an error: reported below
        if ((st = adapt_interval(c))) return give_up(st);
        if (h.halt_step != 0) {
            // a bead outran the schedule, or a rebuild outgrew the list: every
            // kernel after the step kernel that wrote the positions of
            // halt_step returned at once, and those positions and half-step
            // velocities are intact.  Rebuild the list there and go on from
            // the launch that did not run.
            k = h.done_step + 1 - step0;
            const bool full = h.list_n > (uint64_t)c->a.list_cap;
            if (full && (st = grow_list(c, (int64_t)h.list_n))) return give_up(st);
            if (!full) {
                c->K = std::max(1, std::min(c->K, (c->K + 1) / 2));
                ++c->outruns;
            }
            h.halt_step = 0;
            if ((st = copy(c, c->a.b.ctl, &h, sizeof h, hipMemcpyHostToDevice))) return give_up(st);
            if ((st = rebin(c, h.done_par ^ 1))) return give_up(st);
        }
    }
    if (prof) {
        for (size_t q = 0; q + 6 < evs.size(); q += 7)
            for (int m = 0; m < 6; ++m) {
                float t = 0.0f;
                if (hipEventElapsedTime(&t, evs[q + m], evs[q + m + 1]) == hipSuccess) (*prof)[PROF_CLASS[m]] += t;
            }
        for (auto &x : *prof) x /= (double)launches;
        free_events();
    }
    if ((st = read_ctl(c, &h))) return st;
    if (h.code != 0) {
        // the state stays at the step the failing kernels worked on
        c->cur_step = h.step;
        c->cur_par = h.par;
        return status_from_ctl(c, h);
    }
    // the last step kernel wrote the positions one step ahead
    c->cur_step = h.done_step + 1;
    c->cur_par = h.done_par ^ 1;
    c->binned_buf = c->cur_par;
    c->full_par = h.done_par;
    c->full_step = h.done_step;
    c->phase = PH_LEAPFROG;
    return DSDNA_OK;
}

// Buffer holding the full-step positions.
static int full_buffer(const dsdna_ctx *c) { return c->phase == PH_LEAPFROG ? c->full_par : c->cur_par; }

// Run the diagnostic kernel on the full-step positions.
static dsdna_status run_diag(dsdna_ctx *c, uint32_t mask)
{
    dsdna_status st;
    const int which = full_buffer(c);
    if ((st = sync_args(c))) return st;
    if (c->binned_buf != which) {
        if ((st = rebin(c, which))) return st;
    }
    HIPCHK(c, hipMemsetAsync(c->a.b.eex, 0, sizeof(double) * (size_t)c->N, c->stream));
    HIPCHK(c, launch_pairs(c->a, c->dA, which, 1, PAIRS_DIAG, c->stream));
    // the full-step velocities (a halted context keeps them in its buffer)
    const Bufs &b = c->a.b;
    const bool halted = c->phase == PH_HALTED;
    HIPCHK(c, launch_diag(c->a, c->dA, which, c->prm.force_fp64, mask, halted ? b.V[which] : b.Vf,
                          halted ? b.L[which] : b.Lf, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Ctl h;
    if ((st = read_ctl(c, &h))) return st;
    if (h.code != 0) {
        // a diagnostic evaluation found an invalid state: report it, but do
        // not leave the error latched for the stepping kernels
        dsdna_status code = (dsdna_status)h.code;
        Ctl clr = h;
        clr.code = 0;
        if ((st = copy(c, c->a.b.ctl, &clr, sizeof clr, hipMemcpyHostToDevice))) return st;
        // the failed evaluation may have left histogram or accumulator entries
        if ((st = clear_accumulators(c))) return st;
        c->binned_buf = -1;
        return fail(c, code, "invalid state: error %d at nucleotide %lld", (int)code, (long long)h.err_id);
    }
    return DSDNA_OK;
}

// ------------------------------------------------------------ tuning cache

// Key of an autotuner choice: what the best neighbour-search settings depend
// on (the size and kind of the workload and the force precision).
static std::string tune_key(const dsdna_ctx *c)
{
    bool open = false;
    double vol = 0.0;
    for (const RepInfo &r : c->rep_h) {
        const bool per = (r.flags & (REP_PER_X | REP_PER_Y | REP_PER_Z)) == (REP_PER_X | REP_PER_Y | REP_PER_Z);
        open = open || !per;
        if (per) vol += r.len[0] * r.len[1] * r.len[2];
    }
    char buf[160];
    snprintf(buf, sizeof buf, "nt=%lld rep=%d fp64=%d open=%d density=%.3g", (long long)c->N, c->n_rep,
             c->prm.force_fp64, open ? 1 : 0, open || vol <= 0.0 ? 0.0 : (double)c->N / vol);
    return buf;
}

static std::mutex g_tune_mutex;
static std::map<std::string, dsdna_tune_result> g_tune;
static bool g_tune_file_read = false;

// The cache file: one choice per line, "key<TAB>skin<TAB>cell<TAB>hash_log2<TAB>interval".
static void tune_cache_load_file()
{
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char *path = std::getenv("DSDNA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char *tab = std::strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        dsdna_tune_result r{};
        if (std::sscanf(tab + 1, "%lf\t%lf\t%d\t%d", &r.skin, &r.cell_size, &r.hash_log2, &r.interval) == 4)
            g_tune[line] = r;
    }
    std::fclose(f);
}

static bool tune_cache_find(const std::string &key, dsdna_tune_result *out)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    tune_cache_load_file();
    const auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

static void tune_cache_store(const std::string &key, const dsdna_tune_result &r)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    tune_cache_load_file();
    g_tune[key] = r;
    const char *path = std::getenv("DSDNA_TUNE_CACHE");
    if (!path || !*path) return;
    if (FILE *f = std::fopen(path, "a")) {
        std::fprintf(f, "%s\t%.17g\t%.17g\t%d\t%d\n", key.c_str(), r.skin, r.cell_size, r.hash_log2, r.interval);
        std::fclose(f);
    }
}

// ----------------------------------------------------------------- C ABI

extern "C" {

dsdna_status dsdna_default_params(dsdna_params *p)
{
    if (!p) return DSDNA_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->K1 = 30.0; p->R0 = 0.6825; p->eps_bb = 1.0; p->sig_bb = 0.4430;
    p->K2 = 6.0; p->r0_hb = 0.0; p->rc_hb = 0.3;
    p->eps = 1.0; p->sig_s = 1.0; p->sig_x = 0.5;
    p->K3 = 50.0; p->d_dih = -144.0 * M_PI / 180.0;
    p->K4 = 30.0; p->lam = 8.0; p->r0_m = 0.34;
    p->K5 = 200.0; p->a0 = 90.0 * M_PI / 180.0;
    p->K6 = 52.0;
    p->ell = 0.5; p->m_bead = 1.0; p->m_patch = 1.0;
    p->gamma = 1.0; p->kT = 1.0; p->dt = 0.005;
    p->seed = 0;
    p->noise_kind = 0; p->force_fp64 = 0; p->ssdna_rule = 0; p->hb_depth_convention = 0;
    p->cell_size = 0.0; p->hash_log2 = 0; p->graph_steps = 0;
    return DSDNA_OK;
}

dsdna_status dsdna_create(dsdna_ctx **out, const dsdna_params *params, int device, void *hip_stream)
{
    if (!out || !params) return DSDNA_EINVAL;
    *out = nullptr;
    if (params->dt <= 0 || params->ell <= 0 || params->m_bead <= 0 || params->m_patch <= 0 || params->gamma < 0 ||
        params->kT < 0 || params->R0 <= 0 || params->rc_hb <= params->r0_hb || !(params->skin == 0.0 || params->skin >= 1e-3) ||
        params->list_capacity < 0)
        return DSDNA_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DSDNA_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return DSDNA_EDEVICE;
    dsdna_ctx *c = new dsdna_ctx();
    c->device = device;
    c->prm = *params;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return DSDNA_EDEVICE;
        }
        c->own_stream = true;
    }
    if (dalloc(&c->a.b.ctl, 1) != hipSuccess) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return DSDNA_ENOMEM;
    }
    fill_phys(c);
    *out = c;
    return DSDNA_OK;
}

dsdna_status dsdna_destroy(dsdna_ctx *c)
{
    if (!c) return DSDNA_EINVAL;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    free_state(c);
    free_grid(c);
    dfree(c->a.b.ctl);
    dfree(c->dA);
    for (hipEvent_t e : c->lk_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return DSDNA_OK;
}

const char *dsdna_last_error(const dsdna_ctx *c) { return c ? c->err.c_str() : g_free_error.c_str(); }

static dsdna_status build_topology(dsdna_ctx *c, int32_t n_rep, const int32_t *n_bp, int64_t N);

dsdna_status dsdna_set_topology(dsdna_ctx *c, int32_t n_rep, const int32_t *n_bp)
{
    if (!c) return DSDNA_EINVAL;
    if (n_rep <= 0 || !n_bp) return fail(c, DSDNA_EINVAL, "need n_rep >= 1 and n_bp");
    int64_t N = 0;
    for (int r = 0; r < n_rep; ++r) {
        if (n_bp[r] < 1) return fail(c, DSDNA_EINVAL, "replica %d has %d base pairs", r, n_bp[r]);
        N += 2 * (int64_t)n_bp[r];
    }
    if (N >= (int64_t(1) << 31) || n_rep >= (1 << 29)) return fail(c, DSDNA_EINVAL, "too many nucleotides");
    const dsdna_status st = build_topology(c, n_rep, n_bp, N);
    if (st) {
        // a half-built context is not left behind: it has no topology
        const std::string msg = c->err;
        free_state(c);
        c->n_rep = 0;
        c->phase = PH_NONE;
        c->tiles_h.clear();
        c->rep_h.clear();
        c->err = msg;
    }
    return st;
}

static dsdna_status build_topology(dsdna_ctx *c, int32_t n_rep, const int32_t *n_bp, int64_t N)
{
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    free_state(c);
    c->n_rep = n_rep;
    c->n_bp.assign(n_bp, n_bp + n_rep);
    c->off.resize(n_rep);
    c->N = N;
    c->n_bp_total = N / 2;
    c->rep_h.assign(n_rep, RepInfo{});
    c->tiles_h.clear();
    int64_t o = 0;
    for (int r = 0; r < n_rep; ++r) {
        c->off[r] = o;
        RepInfo &ri = c->rep_h[r];
        ri.off = o;
        ri.n_bp = n_bp[r];
        ri.flags = 0;
        ri.k2_scale = 1.0;
        for (int k = 0; k < 3; ++k) {
            ri.lo[k] = 0.0;
            ri.len[k] = 1.0;
            ri.inv_len[k] = 1.0;
        }
        ri.tile0 = (int32_t)c->tiles_h.size();
        for (int n0 = 0; n0 < n_bp[r]; n0 += TILE_BP) c->tiles_h.push_back(Tile{r, n0, n_bp[r], 0});
        o += 2 * (int64_t)n_bp[r];
    }
    StepArgs &a = c->a;
    a.n_nt = N;
    a.n_tiles = (int32_t)c->tiles_h.size();
    a.n_tiles_pad = (a.n_tiles + 7) / 8 * 8;
    Bufs &b = a.b;
    const size_t n3 = 3 * (size_t)N;
    for (int k = 0; k < 2; ++k) {
        HIPCHK(c, dalloc(&b.R[k], n3)); HIPCHK(c, dalloc(&b.u[k], n3));
        HIPCHK(c, dalloc(&b.V[k], n3)); HIPCHK(c, dalloc(&b.L[k], n3));
    }
    HIPCHK(c, dalloc(&b.Vf, n3)); HIPCHK(c, dalloc(&b.Lf, n3));
    HIPCHK(c, dalloc(&b.Fb, n3)); HIPCHK(c, dalloc(&b.Fp, n3));
    HIPCHK(c, dalloc(&b.key, (size_t)N)); HIPCHK(c, dalloc(&b.slot, (size_t)N));
    HIPCHK(c, dalloc(&b.rec, (size_t)N)); HIPCHK(c, dalloc(&b.rcell, (size_t)N));
    HIPCHK(c, dalloc(&b.srec, (size_t)N)); HIPCHK(c, dalloc(&b.sid, (size_t)N)); HIPCHK(c, dalloc(&b.scell, (size_t)N));
    HIPCHK(c, dalloc(&b.fex, FEX_WORDS * (size_t)N));
    HIPCHK(c, dalloc(&b.cmask, CMASK_WORDS * (size_t)a.n_tiles));
    HIPCHK(c, dalloc(&b.eex, (size_t)N));
    // the list holds the non-local pairs within the cutoffs plus the skin: a
    // few per thousand beads in a relaxed duplex; it grows when needed
    a.list_cap = c->prm.list_capacity > 0 ? c->prm.list_capacity : std::max<int64_t>(4096, N / 8);
    HIPCHK(c, dalloc(&b.plist, (size_t)a.list_cap));
    HIPCHK(c, dalloc(&b.vmax, (size_t)a.n_tiles));
    HIPCHK(c, hipMemsetAsync(b.vmax, 0, sizeof(float) * (size_t)a.n_tiles, c->stream));
    HIPCHK(c, dalloc(&b.rep, (size_t)n_rep));
    HIPCHK(c, dalloc(&b.tiles, c->tiles_h.size()));
    HIPCHK(c, dalloc(&b.eacc, (size_t)a.n_tiles * DSDNA_NENERGY));
    HIPCHK(c, dalloc(&c->d_rep_e, (size_t)n_rep * DSDNA_NENERGY));
    HIPCHK(c, dalloc(&b.open, (size_t)c->n_bp_total));
    HIPCHK(c, dalloc(&b.diag_fb, n3)); HIPCHK(c, dalloc(&b.diag_fp, n3));
    c->phase = PH_NONE;
    dsdna_status st0 = copy(c, b.tiles, c->tiles_h.data(), sizeof(Tile) * c->tiles_h.size(), hipMemcpyHostToDevice);
    if (st0) return st0;
    dsdna_status st = configure_grid(c);
    if (st) return st;
    return write_ctl(c, 0, 0);
}

dsdna_status dsdna_set_box(dsdna_ctx *c, const double *lo_hi, const uint8_t *periodic)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (!lo_hi || !periodic) return fail(c, DSDNA_EINVAL, "null box");
    // the new boxes go into a copy of the replica table, which replaces the
    // context's only if the grid can be built for it
    std::vector<RepInfo> reps = c->rep_h;
    for (int r = 0; r < c->n_rep; ++r) {
        RepInfo &ri = reps[r];
        ri.flags &= ~(uint32_t)(REP_PER_X | REP_PER_Y | REP_PER_Z);
        for (int k = 0; k < 3; ++k) {
            const double lo = lo_hi[6 * r + k], hi = lo_hi[6 * r + 3 + k];
            if (!(hi > lo) || !std::isfinite(hi - lo))
                return fail(c, DSDNA_EINVAL, "replica %d: empty box along %d", r, k);
            ri.lo[k] = lo;
            ri.len[k] = hi - lo;
            ri.inv_len[k] = 1.0 / (hi - lo);
            if (periodic[3 * r + k]) ri.flags |= (REP_PER_X << k);
        }
    }
    return configure_grid_for(c, std::move(reps));
}

dsdna_status dsdna_set_external(dsdna_ctx *c, int32_t rep, const double F[3], const double G[3], int32_t tether,
                                double wall_z)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (rep < 0 || rep >= c->n_rep) return fail(c, DSDNA_EINVAL, "replica %d out of range", rep);
    RepInfo &ri = c->rep_h[rep];
    const bool any = tether || (F && (F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0)) ||
                     (G && (G[0] != 0.0 || G[1] != 0.0 || G[2] != 0.0));
    if ((ri.flags & REP_RING) && any)
        return fail(c, DSDNA_EINVAL, "replica %d is a ring: it has no end to anchor, pull or twist", rep);
    ri.flags &= ~(uint32_t)(REP_TETHER | REP_PULL | REP_TORQUE);
    for (int k = 0; k < 3; ++k) {
        ri.pull[k] = F ? F[k] : 0.0;
        ri.torque[k] = G ? G[k] : 0.0;
    }
    if (ri.pull[0] != 0.0 || ri.pull[1] != 0.0 || ri.pull[2] != 0.0) ri.flags |= REP_PULL;
    if (ri.torque[0] != 0.0 || ri.torque[1] != 0.0 || ri.torque[2] != 0.0) ri.flags |= REP_TORQUE;
    if (tether) ri.flags |= REP_TETHER;
    ri.wall_z = wall_z;
    return upload_reps(c);
}

dsdna_status dsdna_set_k2_scale(dsdna_ctx *c, const double *scale)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (!scale) return fail(c, DSDNA_EINVAL, "null scale");
    for (int r = 0; r < c->n_rep; ++r) c->rep_h[r].k2_scale = scale[r];
    return upload_reps(c);
}

dsdna_status dsdna_set_k2_bp(dsdna_ctx *c, const double *scale)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Bufs &b = c->a.b;
    if (!scale) {
        dfree(b.k2bp);
        b.k2bp = nullptr;
        return DSDNA_OK;
    }
    for (int64_t n = 0; n < c->n_bp_total; ++n)
        if (!(scale[n] >= 0.0 && std::isfinite(scale[n])))
            return fail(c, DSDNA_EINVAL, "K2 multiplier of base pair %lld is %g", (long long)n, scale[n]);
    if (!b.k2bp) HIPCHK(c, dalloc(&b.k2bp, (size_t)c->n_bp_total));
    if ((st = copy(c, b.k2bp, scale, sizeof(double) * c->n_bp_total, hipMemcpyHostToDevice))) {
        // a partly written table is not left behind
        dfree(b.k2bp);
        b.k2bp = nullptr;
    }
    return st;
}

dsdna_status dsdna_set_circular(dsdna_ctx *c, const uint8_t *circular)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (!circular) return fail(c, DSDNA_EINVAL, "null circular");
    for (int r = 0; r < c->n_rep; ++r) {
        if (!circular[r]) continue;
        const int nb = c->n_bp[r];
        if (nb < 9 || nb % 3 != 0)
            return fail(c, DSDNA_EINVAL,
                        "ring %d has %d base pairs: a ring needs at least 9 (the chain-local excluded-volume pairs, "
                        "up to 3 base pairs either way, must be distinct) and a multiple of 3 (steric beads every "
                        "third base pair on both sides of the seam)", r, nb);
        if (c->rep_h[r].flags & (REP_TETHER | REP_PULL | REP_TORQUE))
            return fail(c, DSDNA_EINVAL, "replica %d carries external loads and cannot be a ring", r);
    }
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<RepInfo> reps = c->rep_h;
    std::vector<Tile> tiles = c->tiles_h;
    for (int r = 0; r < c->n_rep; ++r) {
        reps[r].flags &= ~(uint32_t)REP_RING;
        if (circular[r]) reps[r].flags |= REP_RING;
    }
    for (Tile &t : tiles) t.ring = (reps[t.rep].flags & REP_RING) ? 1 : 0;
    std::swap(reps, c->rep_h);
    std::swap(tiles, c->tiles_h);
    if ((st = copy(c, c->a.b.tiles, c->tiles_h.data(), sizeof(Tile) * c->tiles_h.size(), hipMemcpyHostToDevice)) ||
        (st = upload_reps(c))) {
        // the previous flags stay (on the device as well, once they upload)
        std::swap(reps, c->rep_h);
        std::swap(tiles, c->tiles_h);
        const std::string msg = c->err;
        (void)copy(c, c->a.b.tiles, c->tiles_h.data(), sizeof(Tile) * c->tiles_h.size(), hipMemcpyHostToDevice);
        (void)upload_reps(c);
        c->err = msg;
        return st;
    }
    free_curves(c);
    return DSDNA_OK;
}

// Relaxed rise (Sec. 2) and the extension length of an open duplex's strands
// in its closure, in relaxed contour lengths (far from the molecule, so the
// closing segment stays clear of it).
constexpr double RISE_NM = 0.34;
constexpr double CLOSURE_CONTOURS = 10.0;

// The curve sets of every replica of at least two base pairs, their blocks
// and scratch (appendix on the closure procedure).
static dsdna_status build_curves(dsdna_ctx *c)
{
    std::vector<CurveSet> sets;
    std::vector<int32_t> set_rep;
    std::vector<int2> blk;
    int64_t pts = 0;
    for (int r = 0; r < c->n_rep; ++r) {
        const RepInfo &ri = c->rep_h[r];
        if (ri.n_bp < 2) continue;
        const bool ring = (ri.flags & REP_RING) != 0;
        CurveSet g;
        g.off = ri.off;
        g.n_bp = ri.n_bp;
        g.open = ring ? 0 : 1;
        g.reach = ring ? 0.0 : CLOSURE_CONTOURS * RISE_NM * ri.n_bp;
        g.n_str = ring ? ri.n_bp : ri.n_bp + 2;
        g.pt0 = (int32_t)pts;
        g.blk0 = (int32_t)blk.size();
        g.n_blk = (g.n_str + LK_THREADS - 1) / LK_THREADS;
        for (int b = 0; b < g.n_blk; ++b) blk.push_back(int2{(int)sets.size(), b * LK_THREADS});
        sets.push_back(g);
        set_rep.push_back(r);
        pts += g.n_str;
    }
    if (pts >= (int64_t(1) << 31)) return fail(c, DSDNA_EINVAL, "too many curve points");
    free_curves(c);
    if (sets.empty()) {
        c->lk_stale = false;
        return DSDNA_OK;
    }
    if (dalloc(&c->d_sets, sets.size()) != hipSuccess || dalloc(&c->d_lkblk, blk.size()) != hipSuccess ||
        dalloc(&c->d_curves, 9 * (size_t)pts) != hipSuccess || dalloc(&c->d_lkpart, 2 * blk.size()) != hipSuccess ||
        dalloc(&c->d_lkout, 2 * sets.size()) != hipSuccess) {
        free_curves(c);
        return fail(c, DSDNA_ENOMEM, "device allocation for the curves of %zu replicas failed", sets.size());
    }
    dsdna_status st;
    if ((st = copy(c, c->d_sets, sets.data(), sizeof(CurveSet) * sets.size(), hipMemcpyHostToDevice)) ||
        (st = copy(c, c->d_lkblk, blk.data(), sizeof(int2) * blk.size(), hipMemcpyHostToDevice))) {
        free_curves(c);
        return st;
    }
    c->sets_h = std::move(sets);
    c->set_rep = std::move(set_rep);
    c->lk_blocks = (int)blk.size();
    c->lk_pts = (int)pts;
    c->lk_stale = false;
    return DSDNA_OK;
}

dsdna_status dsdna_get_linking(dsdna_ctx *c, double *lk, double *wr, double *pair_ms)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (!lk || !wr) return fail(c, DSDNA_EINVAL, "null lk or wr");
    const double nan = std::numeric_limits<double>::quiet_NaN();
    std::fill(lk, lk + c->n_rep, nan);
    std::fill(wr, wr + c->n_rep, nan);
    if (pair_ms) *pair_ms = 0.0;
    HIPCHK(c, hipSetDevice(c->device));
    if (c->lk_stale && (st = build_curves(c))) return st;
    if (c->sets_h.empty()) return DSDNA_OK;
    if ((st = sync_args(c))) return st;
    if (pair_ms)
        for (hipEvent_t &e : c->lk_ev)
            if (!e) HIPCHK(c, hipEventCreate(&e));
    // the full-step positions (a stepping context holds them in the buffer
    // behind the device's current one)
    HIPCHK(c, launch_linking(c->dA, full_buffer(c), c->d_sets, (int)c->sets_h.size(), c->d_lkblk, c->lk_blocks,
                             c->lk_pts, c->d_curves, c->d_lkpart, c->d_lkout, c->stream,
                             pair_ms ? c->lk_ev[0] : nullptr, pair_ms ? c->lk_ev[1] : nullptr));
    std::vector<double> out(2 * c->sets_h.size());
    if ((st = copy(c, out.data(), c->d_lkout, sizeof(double) * out.size(), hipMemcpyDeviceToHost))) return st;
    for (size_t k = 0; k < c->sets_h.size(); ++k) {
        lk[c->set_rep[k]] = out[2 * k];
        wr[c->set_rep[k]] = out[2 * k + 1];
    }
    if (pair_ms) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->lk_ev[0], c->lk_ev[1]));
        *pair_ms = ms;
    }
    return DSDNA_OK;
}

dsdna_status dsdna_get_tiling(dsdna_ctx *c, int32_t *tile_bp, int32_t *wg_threads, int64_t *n_tiles)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (tile_bp) *tile_bp = TILE_BP;
    if (wg_threads) *wg_threads = WG_THREADS;
    if (n_tiles) *n_tiles = c->a.n_tiles;
    return DSDNA_OK;
}

dsdna_status dsdna_set_temperature(dsdna_ctx *c, double kT)
{
    if (!c) return DSDNA_EINVAL;
    if (!(kT >= 0)) return fail(c, DSDNA_EINVAL, "kT < 0");
    c->prm.kT = kT;
    fill_phys(c);
    drop_graph(c);
    return DSDNA_OK;
}

dsdna_status dsdna_set_sites(dsdna_ctx *c, const double *bead, const double *patch)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (!bead || !patch) return fail(c, DSDNA_EINVAL, "null sites");
    const double M = c->prm.m_bead + c->prm.m_patch;
    std::vector<double> R(3 * c->N), u(3 * c->N);
    for (int64_t i = 0; i < c->N; ++i) {
        double d[3], l2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            d[k] = patch[3 * i + k] - bead[3 * i + k];
            l2 += d[k] * d[k];
        }
        const double l = std::sqrt(l2);
        if (!(l > 0.0) || !std::isfinite(l)) return fail(c, DSDNA_EINVAL, "nucleotide %lld: bead and patch coincide", (long long)i);
        for (int k = 0; k < 3; ++k) {
            u[3 * i + k] = d[k] * (1.0 / l);
            R[3 * i + k] = (bead[3 * i + k] * c->prm.m_bead + patch[3 * i + k] * c->prm.m_patch) * (1.0 / M);
        }
    }
    return upload_full_state(c, R.data(), nullptr, u.data(), nullptr, 0);
}

dsdna_status dsdna_set_velocities(dsdna_ctx *c, const double *V, const double *L)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (!V || !L) return fail(c, DSDNA_EINVAL, "null velocities");
    if ((st = to_full(c))) return st;
    std::vector<double> u(3 * c->N), Lp(3 * c->N);
    if ((st = down3(c, u.data(), c->a.b.u[c->full_par]))) return st;
    for (int64_t i = 0; i < c->N; ++i) {
        const double dl = L[3 * i] * u[3 * i] + L[3 * i + 1] * u[3 * i + 1] + L[3 * i + 2] * u[3 * i + 2];
        for (int k = 0; k < 3; ++k) Lp[3 * i + k] = L[3 * i + k] - u[3 * i + k] * dl;
    }
    Bufs &b = c->a.b;
    if ((st = up3(c, b.V[c->full_par], V)) || (st = up3(c, b.L[c->full_par], Lp.data()))) return st;
    HIPCHK(c, hipMemcpyAsync(b.Vf, b.V[c->full_par], sizeof(double) * 3 * c->N, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b.Lf, b.L[c->full_par], sizeof(double) * 3 * c->N, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->phase = PH_FULL;
    return DSDNA_OK;
}

dsdna_status dsdna_thermalize(dsdna_ctx *c, double kT, uint64_t seed)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (!(kT >= 0)) return fail(c, DSDNA_EINVAL, "kT < 0");
    if ((st = to_full(c))) return st;
    if ((st = sync_args(c))) return st;
    HIPCHK(c, launch_thermalize(c->a, c->dA, kT, seed, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->phase = PH_FULL;
    return DSDNA_OK;
}

dsdna_status dsdna_step(dsdna_ctx *c, int64_t n_steps)
{
    if (!c) return DSDNA_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, DSDNA_EDEVICE, "hipSetDevice failed");
    return run_steps(c, n_steps, nullptr);
}

dsdna_status dsdna_get_state(dsdna_ctx *c, double *R, double *V, double *u, double *L, int64_t *step)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    const int p = full_buffer(c);
    Bufs &b = c->a.b;
    const bool halted = c->phase == PH_HALTED;
    if (R && (st = down3(c, R, b.R[p]))) return st;
    if (u && (st = down3(c, u, b.u[p]))) return st;
    if (V && (st = down3(c, V, halted ? b.V[p] : b.Vf))) return st;
    if (L && (st = down3(c, L, halted ? b.L[p] : b.Lf))) return st;
    if (step) *step = c->full_step;
    return DSDNA_OK;
}

dsdna_status dsdna_set_state(dsdna_ctx *c, const double *R, const double *V, const double *u, const double *L,
                             int64_t step)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (!R || !u) return fail(c, DSDNA_EINVAL, "null R or u");
    if (step < 0) return fail(c, DSDNA_EINVAL, "step < 0");
    return upload_full_state(c, R, V, u, L, step);
}

// A caller's array: device memory of the context's device with at least
// `bytes` from `p` to the end of its allocation.
static dsdna_status check_device_array(dsdna_ctx *c, const void *p, size_t bytes, const char *name)
{
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(c, DSDNA_EINVAL, "%s is not device memory", name);
    }
    if (at.device != c->device) return fail(c, DSDNA_EINVAL, "%s is on device %d, not %d", name, at.device, c->device);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, DSDNA_EINVAL, "%s: no allocation range", name);
    }
    const size_t used = (size_t)((const char *)p - (const char *)base);
    if (used > size || size - used < bytes)
        return fail(c, DSDNA_EINVAL, "%s: %zu bytes needed, %zu available", name, bytes, size - used);
    return DSDNA_OK;
}

dsdna_status dsdna_bind_device(dsdna_ctx *c, double *R, double *V, double *u, double *L)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    HIPCHK(c, hipSetDevice(c->device));
    Bufs &b = c->a.b;
    const size_t n = sizeof(double) * 3 * (size_t)c->N;
    if (!R && !V && !u && !L) {
        // unbind: the full-step velocities go back to the context's buffers
        if (!is_bound(c)) return DSDNA_OK;
        HIPCHK(c, hipMemcpyAsync(c->own_Vf, b.Vf, n, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->own_Lf, b.Lf, n, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        b.Vf = c->own_Vf;
        b.Lf = c->own_Lf;
        b.Rf = b.uf = nullptr;
        c->own_Vf = c->own_Lf = nullptr;
        return DSDNA_OK;
    }
    if (!R || !V || !u || !L) return fail(c, DSDNA_EINVAL, "bind R, V, u and L together (or pass none to unbind)");
    double *arr[4] = {R, V, u, L};
    const char *names[4] = {"R", "V", "u", "L"};
    for (int k = 0; k < 4; ++k) {
        if ((st = check_device_array(c, arr[k], n, names[k]))) return st;
        for (int q = 0; q < k; ++q) {
            const char *a0 = (const char *)arr[k], *a1 = (const char *)arr[q];
            if (a0 < a1 + n && a1 < a0 + n) return fail(c, DSDNA_EINVAL, "%s and %s overlap", names[q], names[k]);
        }
    }
    // finish queued work that may still write the full-step buffers
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!is_bound(c)) {
        c->own_Vf = b.Vf;
        c->own_Lf = b.Lf;
    }
    b.Rf = R;
    b.uf = u;
    b.Vf = V;
    b.Lf = L;
    // the arrays' contents become the state; the step counter goes on
    const int64_t step = c->phase == PH_NONE ? 0 : c->full_step;
    HIPCHK(c, hipMemcpyAsync(b.R[0], R, n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b.u[0], u, n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b.V[0], V, n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b.L[0], L, n, hipMemcpyDeviceToDevice, c->stream));
    if ((st = start_from_buffer0(c, step))) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DSDNA_OK;
}

dsdna_status dsdna_get_resume(dsdna_ctx *c, double *R, double *V, double *u, double *L, double *fb, double *fp,
                              int64_t *step)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (c->phase != PH_LEAPFROG && c->phase != PH_RESUME)
        return fail(c, DSDNA_ESTATE, "no site forces yet: take at least one step first");
    if ((st = dsdna_get_state(c, R, V, u, L, step))) return st;
    if (fb && (st = down3(c, fb, c->a.b.Fb))) return st;
    if (fp && (st = down3(c, fp, c->a.b.Fp))) return st;
    return DSDNA_OK;
}

dsdna_status dsdna_set_resume(dsdna_ctx *c, const double *R, const double *V, const double *u, const double *L,
                              const double *fb, const double *fp, int64_t step)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (!R || !V || !u || !L || !fb || !fp) return fail(c, DSDNA_EINVAL, "null argument");
    if ((st = upload_full_state(c, R, V, u, L, step))) return st;
    if ((st = up3(c, c->a.b.Fb, fb)) || (st = up3(c, c->a.b.Fp, fp))) return st;
    c->phase = PH_RESUME;
    return DSDNA_OK;
}

dsdna_status dsdna_get_sites(dsdna_ctx *c, double *bead, double *patch)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    std::vector<double> R(3 * c->N), u(3 * c->N);
    if ((st = dsdna_get_state(c, R.data(), nullptr, u.data(), nullptr, nullptr))) return st;
    const double db = c->a.ph.db, dp = c->a.ph.dp;
    for (int64_t i = 0; i < 3 * c->N; ++i) {
        if (bead) bead[i] = R[i] - u[i] * db;
        if (patch) patch[i] = R[i] + u[i] * dp;
    }
    return DSDNA_OK;
}

dsdna_status dsdna_get_forces(dsdna_ctx *c, int32_t term, double *fb, double *fp)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (term < -1 || term >= DSDNA_NTERMS) return fail(c, DSDNA_EINVAL, "term %d out of range", term);
    const uint32_t mask = term < 0 ? (1u << DSDNA_NTERMS) - 1u : (1u << term);
    if ((st = run_diag(c, mask))) return st;
    if (fb && (st = copy(c, fb, c->a.b.diag_fb, sizeof(double) * 3 * c->N, hipMemcpyDeviceToHost))) return st;
    if (fp && (st = copy(c, fp, c->a.b.diag_fp, sizeof(double) * 3 * c->N, hipMemcpyDeviceToHost))) return st;
    return DSDNA_OK;
}

dsdna_status dsdna_get_energies(dsdna_ctx *c, double *E)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (!E) return fail(c, DSDNA_EINVAL, "null E");
    if ((st = run_diag(c, (1u << DSDNA_NTERMS) - 1u))) return st;
    HIPCHK(c, launch_rep_energy(c->a, c->dA, c->d_rep_e, c->n_rep, c->stream));
    return copy(c, E, c->d_rep_e, sizeof(double) * (size_t)c->n_rep * DSDNA_NENERGY, hipMemcpyDeviceToHost);
}

dsdna_status dsdna_get_bp_open(dsdna_ctx *c, uint8_t *open)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (!open) return fail(c, DSDNA_EINVAL, "null open");
    if ((st = run_diag(c, 1u << DSDNA_TERM_HBOND))) return st;
    if ((st = copy(c, open, c->a.b.open, (size_t)c->n_bp_total, hipMemcpyDeviceToHost))) return st;
    return DSDNA_OK;
}

dsdna_status dsdna_get_bubbles(dsdna_ctx *c, int32_t nhist, double *frac, int64_t *hist)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (nhist < 2 || nhist > 4096 || !frac || !hist)
        return fail(c, DSDNA_EINVAL, "need 2 <= nhist <= 4096, frac and hist");
    if ((st = run_diag(c, 1u << DSDNA_TERM_HBOND))) return st;
    if (nhist > c->bub_nhist) {
        free_bubbles(c);
        if (dalloc(&c->d_bub_hist, (size_t)c->a.n_tiles * nhist) != hipSuccess ||
            dalloc(&c->d_bub_info, (size_t)c->a.n_tiles) != hipSuccess ||
            dalloc(&c->d_bub_frac, (size_t)c->n_rep) != hipSuccess ||
            dalloc(&c->d_bub_out, (size_t)c->n_rep * nhist) != hipSuccess) {
            free_bubbles(c);
            return fail(c, DSDNA_ENOMEM, "bubble statistics: allocation failed");
        }
        c->bub_nhist = nhist;
    }
    HIPCHK(c, launch_bubbles(c->a, c->dA, nhist, c->d_bub_hist, c->d_bub_info, c->d_bub_frac, c->d_bub_out, c->n_rep,
                             c->stream));
    if ((st = copy(c, frac, c->d_bub_frac, sizeof(double) * (size_t)c->n_rep, hipMemcpyDeviceToHost))) return st;
    return copy(c, hist, c->d_bub_out, sizeof(int64_t) * (size_t)c->n_rep * nhist, hipMemcpyDeviceToHost);
}

dsdna_status dsdna_profile_kernels(dsdna_ctx *c, int64_t n_steps, double *ms)
{
    if (!c || !ms) return DSDNA_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, DSDNA_EDEVICE, "hipSetDevice failed");
    std::vector<double> prof;
    dsdna_status st = run_steps(c, n_steps, &prof);
    if (st) return st;
    for (int k = 0; k < DSDNA_NKERNELS; ++k) ms[k] = prof.empty() ? 0.0 : prof[k];
    return DSDNA_OK;
}

dsdna_status dsdna_get_sizes(dsdna_ctx *c, int32_t *n_rep, int64_t *n_nt, int64_t *n_bp_total)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (n_rep) *n_rep = c->n_rep;
    if (n_nt) *n_nt = c->N;
    if (n_bp_total) *n_bp_total = c->n_bp_total;
    return DSDNA_OK;
}

dsdna_status dsdna_get_neighbour_stats(dsdna_ctx *c, int64_t *rebuilds, int64_t *steps, int64_t *outruns,
                                       int64_t *pairs, double *skin, int32_t *interval)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    HIPCHK(c, hipSetDevice(c->device));
    Ctl h;
    if ((st = read_ctl(c, &h))) return st;
    if (rebuilds) *rebuilds = h.rebuilds;
    if (steps) *steps = c->phase == PH_LEAPFROG ? h.done_step - c->state_step : 0;
    if (pairs) *pairs = std::min<int64_t>((int64_t)h.list_n, c->a.list_cap);
    if (skin) *skin = c->a.ph.skin;
    if (outruns) *outruns = c->outruns;
    if (interval) *interval = c->K;
    return DSDNA_OK;
}

dsdna_status dsdna_get_grid(dsdna_ctx *c, double *cell_size, int64_t *n_buckets, int32_t *cells)
{
    dsdna_status st = check_ready(c, false);
    if (st) return st;
    if (cell_size) *cell_size = c->a.g.h;
    if (n_buckets) *n_buckets = c->a.g.nbucket;
    if (cells)
        for (int k = 0; k < 3; ++k) cells[k] = c->rep_h[0].ncell[k];
    return DSDNA_OK;
}

dsdna_status dsdna_autotune(dsdna_ctx *c, const dsdna_tune_space *sp, dsdna_tune_result *best)
{
    dsdna_status st = check_ready(c, true);
    if (st) return st;
    if (!sp || !best || sp->trial_steps < 1 || sp->warm_steps < 0 || sp->n_skins < 0 || sp->n_cell_factors < 0 ||
        sp->n_hash_log2s < 0)
        return fail(c, DSDNA_EINVAL, "autotune needs a space, a result and trial_steps >= 1");
    const std::vector<double> skins = sp->n_skins > 0 && sp->skins
                                          ? std::vector<double>(sp->skins, sp->skins + sp->n_skins)
                                          : std::vector<double>{c->a.ph.skin};
    const std::vector<double> facs = sp->n_cell_factors > 0 && sp->cell_factors
                                         ? std::vector<double>(sp->cell_factors, sp->cell_factors + sp->n_cell_factors)
                                         : std::vector<double>{1.001};
    const std::vector<int32_t> lgs = sp->n_hash_log2s > 0 && sp->hash_log2s
                                         ? std::vector<int32_t>(sp->hash_log2s, sp->hash_log2s + sp->n_hash_log2s)
                                         : std::vector<int32_t>{c->prm.hash_log2};
    for (double x : skins)
        if (!(x >= 1e-3)) return fail(c, DSDNA_EINVAL, "autotune: skin %g below 1e-3", x);
    for (double f : facs)
        if (!(f >= 1.001)) return fail(c, DSDNA_EINVAL, "autotune: cell factor %g below 1.001", f);
    std::memset(best, 0, sizeof *best);
    const std::string key = tune_key(c);
    const dsdna_params prm0 = c->prm;
    const int K0 = c->K;
    // on any failure the parameters and the grid they give are put back
    const auto restore = [&](dsdna_status code) {
        const std::string msg = c->err;
        c->prm = prm0;
        fill_phys(c);
        (void)configure_grid(c);
        c->K = K0;
        c->err = msg;
        return code;
    };
    const auto apply = [&](double skin, double cell, int32_t lg) -> dsdna_status {
        c->prm.skin = skin;
        c->prm.cell_size = cell;
        c->prm.hash_log2 = lg;
        fill_phys(c);
        return configure_grid(c);
    };
    dsdna_tune_result hit;
    if (sp->use_cache && tune_cache_find(key, &hit)) {
        if ((st = apply(hit.skin, hit.cell_size, hit.hash_log2))) return restore(st);
        *best = hit;
        best->from_cache = 1;
        best->ms_per_step = 0.0;
        best->candidates = 0;
        return DSDNA_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const auto done = [&](dsdna_status code) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return code == DSDNA_OK ? code : restore(code);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return done(fail(c, DSDNA_EDEVICE, "hipEventCreate failed"));
    double best_ms = 1e300;
    for (double skin : skins)
        for (double f : facs)
            for (int32_t lg : lgs) {
                const double cell = f * (TWO_16 * std::max(c->prm.sig_s, c->prm.sig_x) + skin + LIST_SLACK);
                if ((st = apply(skin, cell, lg))) return done(st);
                c->sync_batch = SYNC_FIRST;
                if ((st = run_steps(c, std::max<int64_t>(1, sp->warm_steps), nullptr))) return done(st);
                float t = 0.0f;
                if (hipEventRecord(e0, c->stream) != hipSuccess) return done(fail(c, DSDNA_EDEVICE, "event failed"));
                if ((st = run_steps(c, sp->trial_steps, nullptr))) return done(st);
                if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess)
                    return done(fail(c, DSDNA_EDEVICE, "event failed"));
                const double ms = t / (double)sp->trial_steps;
                ++best->candidates;
                if (ms < best_ms) {
                    best_ms = ms;
                    best->skin = skin;
                    best->cell_size = cell;
                    best->hash_log2 = c->a.g.nbucket > 0 ? (int32_t)std::lround(std::log2((double)c->a.g.nbucket)) : lg;
                    best->interval = c->K;
                    best->ms_per_step = ms;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    e0 = e1 = nullptr;
    if ((st = apply(best->skin, best->cell_size, best->hash_log2))) return restore(st);
    c->K = best->interval;
    if (sp->use_cache) tune_cache_store(key, *best);
    return DSDNA_OK;
}

}  // extern "C"
