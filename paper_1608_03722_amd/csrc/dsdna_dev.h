// dsdna_dev.h -- internal layout shared by the HIP kernels and the host
// runtime of libdsdna.  Not part of the public ABI (include/dsdna.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsdna {

// Base pairs per tile: one workgroup of WG_THREADS threads owns the
// nucleotides of TILE_BP consecutive base pairs of one replica.  124 base
// pairs keep every per-tile phase (sites with halo, backbone steps, bending
// centres) within one item per thread.
constexpr int WG_THREADS = 256;
constexpr int TILE_BP = 124;
constexpr int TILE_NT = 2 * TILE_BP;
constexpr int HALO_BP = 2;  // bending reaches two base pairs away
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
    double inv_I, kick_M;     // 1 / I, (dt / 2) / M
    double inv_R0sq;          // 1 / R0^2
    uint64_t seed;
    int32_t noise_kind, ssdna_rule;
    int32_t fene_clamp, dihedral_damping;
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

// Control block in device memory.  `step` is the step index of the positions
// in buffer `par`; kernels read both at launch so that captured graphs replay
// without argument changes.
struct Ctl {
    int64_t step;
    int32_t par;
    int32_t code;      // first error (dsdna_status), 0 if none
    int64_t err_step;
    int64_t err_id;
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
};

// Device buffers of one context.
struct Bufs {
    double *R[2], *u[2], *V[2], *L[2];  // SoA [3][N] (x block, y block, z block)
    double *Vf, *Lf;                    // full-step velocities of the last step
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
    // excluded-volume force per nt as exact fixed-point sums (x, y, z, unused;
    // units FIX32_UNIT or FIX64_UNIT), zero except beads with contacts;
    // consumers read and clear the entries whose contact bit is set
    unsigned long long *fex;
    // contact bits, CMASK_WORDS words per tile: bit t of the tile's mask is
    // set when tile thread t's nucleotide (2 (n - n0) + s) has a fex entry
    uint32_t *cmask;
    double *eex;                        // excluded-volume energy per nt (diagnostics)
    RepInfo *rep;
    Tile *tiles;
    Ctl *ctl;
    double *eacc;                       // per tile energy partials
    uint8_t *open;                      // per bp open flags (diagnostics)
    double *k2bp;                       // per bp K2 multiplier, null if unset
    double *diag_fb, *diag_fp;          // per-term diagnostic forces (AoS [N][3])
};

enum StepMode : int { MODE_NORMAL = 0, MODE_FIRST = 1, MODE_FROM_FORCES = 2 };

// Units of the fixed-point excluded-volume sums: 2^24 per force unit with
// FP32 forces, 2^36 with FP64 forces.
constexpr double FIX32_UNIT = 16777216.0;
constexpr double FIX64_UNIT = 68719476736.0;

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
};

// A ring for the linking-number kernels: its first nucleotide, length,
// first point in the curve buffers and its workgroups (blocks of LK_THREADS
// base pairs, first at blk0).
constexpr int LK_THREADS = 256;
struct RingSeg {
    int64_t off;
    int32_t n_bp;
    int32_t pt0;
    int32_t blk0;
    int32_t n_blk;
};

// Launchers (defined in dsdna_kernels.hip).  `a` is the host copy (grid
// sizes), `dA` the device copy the kernels read.
hipError_t launch_bin(const StepArgs &a, const StepArgs *dA, int which, hipStream_t s);
hipError_t launch_scan(const StepArgs &a, hipStream_t s);
hipError_t launch_scatter(const StepArgs &a, int inc_step, hipStream_t s);
hipError_t launch_step(const StepArgs &a, const StepArgs *dA, int fp64, int mode, int write_full, hipStream_t s);
// Excluded-volume force (and with `energy`, energy) of every bead from the
// sorted records, written to b.fex (b.eex) by nucleotide.  `which`: position
// buffer the records describe (-1: the control block's current buffer).
hipError_t launch_excl(const StepArgs &a, const StepArgs *dA, int fp64, int energy, int which, hipStream_t s);
hipError_t launch_thermalize(const StepArgs &a, const StepArgs *dA, double kT, uint64_t seed, hipStream_t s);
// term_mask: bit t selects term t; writes per-term forces (AoS doubles) to
// b.diag_fb / b.diag_fp, energies per tile to b.eacc[tile][DSDNA_NTERMS] and
// open flags per bp to b.open.
hipError_t launch_diag(const StepArgs &a, const StepArgs *dA, int which, int fp64, uint32_t term_mask,
                       hipStream_t s);
// Linking number of the strands and writhe of the centreline of every ring
// from the positions in buffer `which`: curves (3 curves x n_pts points x 3
// doubles) and partial ([n_blocks][2]) are scratch, out[n_rings][2]
// receives (Lk, Wr).  blocks[n_blocks] = (ring, first bp).  ev0/ev1 (may be
// null) bracket the pair kernel.
hipError_t launch_linking(const StepArgs *dA, int which, const RingSeg *rings, int n_rings, const int2 *blocks,
                          int n_blocks, int n_pts, double *curves, double *partial, double *out, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1);

}  // namespace dsdna
