// dsdna_dev.h -- internal layout shared by the HIP kernels and the host
// runtime of libdsdna.  Not part of the public ABI (include/dsdna.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsdna {

// Base pairs per tile: one workgroup of WG_THREADS threads owns the
// nucleotides of TILE_BP consecutive base pairs of one replica, and its spare
// threads stage a halo of HALO_BP base pairs on either side.  Three base
// pairs of halo hold every site a tile's terms reach: bending reaches two
// base pairs away, and the chain-local excluded-volume pairs (LOCAL_BP) three.
// TILE_NT is a multiple of 16 sites, so that the tiles of a replica that
// starts on a 128-byte boundary read and write whole 128-byte lines of each
// FP64 component array (12 halo sites then take 12 of the 16 spare threads,
// and 4 stay idle; at 1 Mbp this is 3% faster per tile than 122 bp tiles,
// which occupy every thread).
constexpr int WG_THREADS = 256;
constexpr int HALO_BP = 3;
constexpr int TILE_BP = 120;
constexpr int TILE_NT = 2 * TILE_BP;
static_assert(TILE_NT + 4 * HALO_BP <= WG_THREADS, "a tile and its halo fit the workgroup");
// Bead pairs whose base pairs lie at most LOCAL_BP apart along the chain
// (cyclically on a ring) are evaluated by the step kernel from the tile's
// staged sites; all others come from the neighbour list.
constexpr int LOCAL_BP = 3;
static_assert(LOCAL_BP <= HALO_BP, "local pairs must lie inside the staged halo");
constexpr int CMASK_WORDS = WG_THREADS / 32;  // contact-bit words per tile
constexpr int SCAN_CHUNK = 4096;  // histogram entries per scan workgroup

// Physics constants as the kernels use them (double; the force precision is
// chosen per kernel instantiation).  Derived values are filled by the host.
struct Phys {
    double K1, R0, eps_bb, sig_bb;
    double K2, r0_hb, rc_hb;
    double eps, sig_s, sig_x;
    double K3, d_dih, K4, lam, r0_m, K5, a0, K6;
    double ell, m_bead, m_patch, gamma, kT, dt;
    // derived
    double M, I, db, dp;      // body mass, moment of inertia, |bead-R|, |patch-R|
    double noise_amp;         // sqrt(2 gamma kT / dt)
    double hb_pref;           // H-bond prefactor before the per-replica scale
    double rc_bb, rc_s, rc_x; // WCA cutoffs 2^(1/6) sigma
    double cos_d, sin_d;      // cos and sin of the dihedral phase
    double cos_a0, sin_a0;    // cos and sin of the planarity angle
    double kick;              // dt / 2
    double skin;              // neighbour-list skin
    double rl2_s, rl2_x;      // squared list cutoffs (rc + skin + slack) for
                              // same-strand steric pairs and cross-strand pairs
    float half_skin2;         // squared displacement that makes the list stale
    double inv_I, kick_M;     // 1 / I, (dt / 2) / M
    double inv_R0sq;          // 1 / R0^2
    uint64_t seed;
    int32_t noise_kind, ssdna_rule;
    int32_t fene_clamp, dihedral_damping;
    int32_t planarity_both;
};

enum : uint32_t {
    REP_TETHER = 1u,
    REP_PER_X = 2u,
    REP_PER_Y = 4u,
    REP_PER_Z = 8u,
    REP_PULL = 16u,
    REP_TORQUE = 32u,
    REP_RING = 64u,   // closed ring: bp n_bp-1 is bonded to bp 0
};

struct RepInfo {
    int64_t off;        // first nucleotide
    int32_t n_bp;
    uint32_t flags;     // REP_*
    double lo[3];       // box low corner: origin of the cell grid
    double len[3];      // box edge (periodic dims)
    double inv_len[3];
    double pull[3], torque[3];
    double wall_z, k2_scale;
    int32_t ncell[3];   // cells per periodic dim (0 for open dims)
    int32_t tile0;      // index of the replica's first tile
    double inv_h[3];    // cells per unit length per dim
    float qlen[3];      // length of one fixed-point coordinate unit
    int32_t pad2;
};

// A bead in the cell list: 32-bit fixed-point coordinates and a tag word
// (bit 0 strand, bit 1 steric, bits 2..31 replica).  Periodic dims map the
// box edge onto the full 32-bit range, so the wrapped difference of two
// coordinates is the minimum image; open dims use 2^-24 length units, so
// differences of beads less than 128 apart are exact.
struct alignas(16) BeadRec {
    uint32_t x, y, z, tag;
};
constexpr double OPEN_QINV = 16777216.0;  // 2^24

struct Tile {
    int32_t rep;
    int32_t n0;    // first base pair of the tile within its replica
    int32_t n_bp;  // base pairs of the replica
    int32_t ring;  // 1 if the replica is a ring (REP_RING)
};

// Control block in device memory.  (step, par) is the step index of the
// positions in buffer par that the current step integrates, and (done_step,
// done_par) those of the last step kernel that started; kernels read them at
// launch, so captured graphs replay without argument changes.  The first
// kernel of a step (the pair kernel) publishes step = done_step + 1 and par =
// done_par ^ 1, and block 0 of the step kernel records done_step = step at
// its start: each field is written by one thread of a kernel that does not
// read it, so no kernel sees a value change under it.  The neighbour list is
// rebuilt on a schedule the host chooses.  halt_step (0: none) stops the run
// so that the host can rebuild the list there and continue: a step kernel
// that finds a bead half the skin from where the list last saw it (on a step
// not followed by a rebuild) sets it to the index of the new positions, a
// rebuild that outgrows the list buffer to that of the positions it binned;
// every kernel of that step or later returns at once, after the pair kernel
// has published the step.
struct Ctl {
    int64_t step;
    int32_t par;
    int32_t code;      // first error (dsdna_status), 0 if none
    int64_t err_step;
    int64_t err_id;
    int64_t done_step;
    int32_t done_par;
    uint32_t list_n;   // pairs in the neighbour list (may exceed its capacity)
    int64_t halt_step;
    int64_t rebuilds;  // neighbour-list builds since the counter was reset
};

// A pair of beads of the neighbour list: nucleotides i and j (i's record
// precedes j's in cell order), their replica, and whether they are on the
// same strand (same-strand pairs are steric-steric).
struct PairRec {
    int32_t i, j, rep, same;
};

// Hash of cell (cx, cy, cz) of replica r into [0, nbucket): linear in the
// cell coordinates so that the three cells cx-1, cx, cx+1 of a row are three
// consecutive buckets.  The host chooses A, B, C such that the 27 cells
// around any cell fall in 27 distinct buckets.  The bucket is the counting
// sort key.
struct Grid {
    uint32_t A, B, C, mask;  // mask = nbucket - 1
    double h;                // cell edge for open dims
    int32_t nbucket;
    int32_t any_open;        // some replica has an open edge
    int32_t fast_screen;     // one replica, the same fixed-point unit along x, y, z
};

// Device buffers of one context.
struct Bufs {
    double *R[2], *u[2], *V[2], *L[2];  // SoA [3][N] (x block, y block, z block)
    double *Vf, *Lf;                    // full-step velocities of the last step
    double *Rf, *uf;                    // caller-bound full-step R and u, or null
    double *Fb, *Fp;                    // full-step site forces (SoA [3][N])
    BeadRec *rec;                       // bead record per nucleotide
    int4 *rcell;                        // cell (x, y, z) of each bead (open edges only)
    int32_t *key, *slot;                // counting-sort key and slot of each bead
    BeadRec *srec;                      // records in key order (counting sort)
    int32_t *sid;                       // nucleotide of each sorted record
    int4 *scell;                        // cell of each sorted record (open edges only)
    // histogram: two 16-bit bucket counts per word (bucket k in bits
    // 16 (k & 1) .. 16 (k & 1) + 15 of word k >> 1)
    uint32_t *count;
    int32_t *start, *bsum;              // per key (start: nbucket + 1); per scan chunk
    // excluded-volume force of the neighbour-list pairs per nt as exact
    // fixed-point sums (FEX_WORDS per nt: FIX_HI and FIX_LO parts of x, y,
    // z), zero except beads with contacts; consumers read and clear the
    // entries whose contact bit is set
    unsigned long long *fex;
    // contact bits, CMASK_WORDS words per tile: bit t of the tile's mask is
    // set when tile thread t's nucleotide (2 (n - n0) + s) has a fex entry
    uint32_t *cmask;
    double *eex;                        // list-pair excluded-volume energy per nt (diagnostics)
    PairRec *plist;                     // neighbour list (non-local bead pairs)
    // per tile: the largest squared displacement of a bead over a rebuild
    // interval (measured on the steps a rebuild follows) since the host last
    // cleared it
    float *vmax;
    RepInfo *rep;
    Tile *tiles;
    Ctl *ctl;
    double *eacc;                       // per tile energy partials
    uint8_t *open;                      // per bp open flags (diagnostics)
    double *k2bp;                       // per bp K2 multiplier, null if unset
    double *diag_fb, *diag_fp;          // per-term diagnostic forces (AoS [N][3])
};

enum StepMode : int { MODE_NORMAL = 0, MODE_FIRST = 1, MODE_FROM_FORCES = 2 };

// Exact, order-independent sums of the neighbour-list contact forces: each
// force component f is split into a coarse part (an integer number of
// FIX_HI units) and the remainder (an integer number of FIX_LO units, |.| <=
// 2^31), and the two are summed in separate 64-bit integers.  The total is
// resolved to 2^-40 force units whatever its size; a pair force of
// PAIR_FORCE_MAX or more (or not finite) is an error.
constexpr double FIX_HI = 256.0;              // 2^8 per force unit
constexpr double FIX_LO = 1099511627776.0;    // 2^40 per force unit
constexpr double PAIR_FORCE_MAX = 1099511627776.0;  // 2^40 (|fx| + |fy| + |fz|)
constexpr int FEX_WORDS = 8;  // per nucleotide: coarse x, y, z, unused; fine x, y, z, unused

// Everything the kernels read that does not change from launch to launch.
// The host keeps a copy in device memory and passes its address, so the
// large block is loaded through the scalar cache on demand instead of
// occupying scalar registers.
struct StepArgs {
    Phys ph;
    Grid g;
    Bufs b;
    int64_t n_nt;
    int32_t n_tiles;
    int32_t n_tiles_pad;   // launched workgroups (multiple of 8)
    int64_t list_cap;      // capacity of b.plist
};

// The curves of one replica for the linking-number kernels (appendix on the
// closure procedure).  A ring's two strands and centreline are closed
// polygons of n_bp points.  An open duplex's strands are closed by two extra
// points each (n_str = n_bp + 2: the last bead pushed out along its end
// tangent by `reach`, then the first bead pushed out likewise, the closing
// segment between them), while its centreline stays an open polygon of n_bp
// points.  pt0: first point slot of the set in each of the three curve
// blocks (n_str slots per set); workgroups: blocks of LK_THREADS rows,
// first at blk0.
constexpr int LK_THREADS = 256;
struct CurveSet {
    int64_t off;      // first nucleotide
    double reach;     // extension length of an open duplex's strands
    int32_t n_bp;
    int32_t open;     // 1: open duplex, 0: ring
    int32_t n_str;    // points of each strand curve
    int32_t pt0;
    int32_t blk0;
    int32_t n_blk;
};

// Launchers (defined in dsdna_kernels.hip).  `a` is the host copy (grid
// sizes), `dA` the device copy the kernels read.
//
// One step is launch_pairs and launch_step, followed on the steps the host
// schedules a rebuild by the kernels of a neighbour-list rebuild from the
// positions the step kernel has just written and binned (launch_scan,
// launch_scatter, launch_build).  rebuild_after: a rebuild follows this step
// kernel, which then bins its new beads; age: steps since the last rebuild,
// this one included.  launch_bin bins a given buffer (a rebuild outside the
// steps).
hipError_t launch_step(const StepArgs &a, const StepArgs *dA, int fp64, int mode, int write_full, int rebuild_after,
                       int age, hipStream_t s);
// Excluded-volume force of every neighbour-list pair within its cutoff at the
// positions of buffer `which` (-1: the control block's current buffer),
// accumulated into b.fex / b.cmask (and with `energy`, half of each pair's
// energy into b.eex of both beads).  mode PAIRS_STEP: the first kernel of a
// step (publishes the step; which is ignored); PAIRS_PUBLISH: only
// publishes it (a step that starts from stored forces); PAIRS_DIAG: for the
// diagnostics, at the control block's step.
enum PairsMode : int { PAIRS_DIAG = 0, PAIRS_STEP = 1, PAIRS_PUBLISH = 2 };
hipError_t launch_pairs(const StepArgs &a, const StepArgs *dA, int which, int energy, int mode, hipStream_t s);
// Counting-sort count phase: record, cell, key and slot of every bead of
// buffer `which` (-1: the positions the last step kernel wrote).
hipError_t launch_bin(const StepArgs &a, const StepArgs *dA, int which, hipStream_t s);
hipError_t launch_scan(const StepArgs &a, hipStream_t s);
hipError_t launch_scatter(const StepArgs &a, hipStream_t s);
// Neighbour search over the sorted records: every non-local bead pair within
// its cutoff plus the skin goes to b.plist; clears the histogram.
hipError_t launch_build(const StepArgs &a, const StepArgs *dA, hipStream_t s);
hipError_t launch_thermalize(const StepArgs &a, const StepArgs *dA, double kT, uint64_t seed, hipStream_t s);
// term_mask: bit t selects term t; writes per-term forces (AoS doubles) to
// b.diag_fb / b.diag_fp, energies per tile to b.eacc[tile][DSDNA_NENERGY]
// (the kinetic ones from the velocities Vk, Lk, SoA [3][N]) and open flags
// per bp to b.open.
hipError_t launch_diag(const StepArgs &a, const StepArgs *dA, int which, int fp64, uint32_t term_mask,
                       const double *Vk, const double *Lk, hipStream_t s);
// Per replica: the tiles' energy partials summed in a fixed order into
// out[n_rep][DSDNA_NENERGY] (device).
hipError_t launch_rep_energy(const StepArgs &a, const StepArgs *dA, double *out, int n_rep, hipStream_t s);
// Bubble statistics (Sec. 5) of the open flags in b.open: frac[n_rep] and
// out[n_rep][nhist] (device); hist_tiles[n_tiles][nhist] and info[n_tiles]
// are scratch.
hipError_t launch_bubbles(const StepArgs &a, const StepArgs *dA, int nhist, int32_t *hist_tiles, int4 *info,
                          double *frac, int64_t *out, int n_rep, hipStream_t s);
// Linking number of the strands and writhe of the centreline of every curve
// set (a ring, or an open duplex closed by extension) from the positions in
// buffer `which`: curves (3 curves x n_pts point slots x 3 doubles) and
// partial ([n_blocks][2]) are scratch, out[n_sets][2] receives (Lk, Wr).
// blocks[n_blocks] = (set, first row).  ev0/ev1 (may be null) bracket the
// pair kernel.
hipError_t launch_linking(const StepArgs *dA, int which, const CurveSet *sets, int n_sets, const int2 *blocks,
                          int n_blocks, int n_pts, double *curves, double *partial, double *out, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1);
// The same for one ring given as three closed curves A, B, C of n points
// ([n][3] doubles each, device memory): partial holds 2 ceil(n /
// LK_THREADS) doubles, out[2] receives (Lk(A, B), Wr(C)).
hipError_t launch_linking_curves(const double *A, const double *B, const double *C, int n, double *partial,
                                 double *out, hipStream_t s);
// Message of the last failure of a context-free call on this thread (read by
// dsdna_last_error(NULL)); printf-style.
void set_free_error(const char *fmt, ...);

}  // namespace dsdna
