/*
 * dsdna.h -- C ABI of the MI355X (gfx950) Langevin hot path of the
 * single-nucleotide double-stranded DNA model of Fosado, Michieletto, Allan,
 * Brackley, Henrich and Marenduzzo (arXiv:1608.03722).
 *
 * One time step follows Appendix A of the paper: the Langevin equation of
 * motion with the potentials of Sec. 2 and Appendix A (Table 2 parameters),
 * integrated by NVT velocity-Verlet with dt = 0.005 tau_Br.  Each nucleotide
 * is the rigid bead+patch body of Sec. 2.  Per step the library bins beads
 * into a counting-sort cell list, evaluates the excluded volume (WCA with the
 * steric/ghost rule of Sec. 2) and the fixed-topology terms (FENE backbone,
 * Morse stacking, hydrogen bond, helical-twist dihedral, planarity,
 * Kratky-Porod bending, Appendix A), adds the external loads of Sec. 4 and
 * the Langevin friction and counter-based noise, and integrates.
 *
 * Conventions
 *   - Reduced units of Table 3: length sigma = 1 nm, energy k_B T, force
 *     k_B T / nm = 4.1419 pN, time tau_Br.
 *   - Replica r holds n_bp[r] base pairs.  Nucleotide (strand s, base pair n)
 *     of replica r has global index off[r] + 2 n + s, off[r] = 2 sum_{q<r}
 *     n_bp[q] ("base-pair-major" order).  Replicas never interact.
 *   - Every array argument is a HOST pointer, caller-owned, read or written
 *     during the call only.  Vectors are packed [count][3] (x, y, z) doubles.
 *   - The context owns all device memory; it is freed by dsdna_destroy.
 *   - Work is enqueued on the context's HIP stream.  Calls on one context are
 *     not thread-safe.  Functions that return data synchronise the stream.
 *   - Every function returns a dsdna_status; DSDNA_OK is 0.  On failure
 *     dsdna_last_error() describes the cause (with step and nucleotide for
 *     DSDNA_EBOND, DSDNA_ENAN, DSDNA_EWALL, DSDNA_EDOMAIN, DSDNA_ECELL).
 *   - Call order: create -> set_topology -> (set_box, set_circular,
 *     set_external, set_k2_scale, set_k2_bp) -> set_sites or set_state ->
 *     (thermalize or set_velocities) -> step ...  Out-of-order calls return
 *     DSDNA_ESTATE.
 */
#ifndef DSDNA_H
#define DSDNA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DSDNA_OK = 0,
    DSDNA_EINVAL = 1,   /* bad argument                                      */
    DSDNA_ENOMEM = 2,   /* device or host allocation failed                  */
    DSDNA_EDEVICE = 3,  /* HIP runtime error                                 */
    DSDNA_EBOND = 4,    /* backbone bond reached R0: the FENE energy is
                           infinite (Appendix A, U_bb for r >= R0)           */
    DSDNA_ENAN = 5,     /* non-finite position or orientation, or an
                           excluded-volume contact force that is not finite
                           or exceeds 2^40 kT/nm (beads on top of each
                           other)                                           */
    DSDNA_ESTATE = 6,   /* call out of order                                 */
    DSDNA_EWALL = 7,    /* a bead of a tethered replica reached its wall     */
    DSDNA_EDOMAIN = 8,  /* a bead left the representable coordinate range   */
    DSDNA_ECELL = 9     /* more than 65535 beads in one cell-list bucket
                           (raise hash_log2)                                 */
} dsdna_status;

/* Slots of the per-term force and energy arrays. */
enum {
    DSDNA_TERM_EXCL = 0,   /* bead excluded volume, WCA (Sec. 2, App. A)     */
    DSDNA_TERM_BOND = 1,   /* backbone FENE + its WCA core (App. A, U_bb)    */
    DSDNA_TERM_STACK = 2,  /* Morse between consecutive patches (U_morse)    */
    DSDNA_TERM_HBOND = 3,  /* truncated harmonic between paired patches      */
    DSDNA_TERM_TWIST = 4,  /* dihedral (bead n, patch n, patch n+1, bead n+1) */
    DSDNA_TERM_PLANAR = 5, /* harmonic angle at patch n+1 (patch n, bead n+1) */
    DSDNA_TERM_BEND = 6,   /* Kratky-Porod on three consecutive patches      */
    DSDNA_TERM_EXT = 7,    /* anchoring wall, pulling force, end torque      */
    DSDNA_NTERMS = 8
};
/* dsdna_get_energies writes DSDNA_NENERGY values per replica: the
 * DSDNA_NTERMS potential terms, then translational and rotational kinetic
 * energy of the full-step velocities. */
#define DSDNA_NENERGY (DSDNA_NTERMS + 2)

/* Kernels timed by dsdna_profile_kernels.  The last four make up a rebuild
 * of the neighbour list and do their work only on the steps that need one;
 * their means are per step, so they include the rebuild frequency. */
enum {
    DSDNA_KERNEL_STEP = 0,    /* bonded + chain-local excluded volume +
                                 loads + Langevin + integrate + skin test    */
    DSDNA_KERNEL_SCAN = 1,    /* exclusive scan of the cell histogram (2 kernels) */
    DSDNA_KERNEL_SCATTER = 2, /* counting-sort scatter into cell order       */
    DSDNA_KERNEL_EXCL = 3,    /* excluded volume of the neighbour-list pairs */
    DSDNA_KERNEL_BIN = 4,     /* cell of every bead (counting-sort count)    */
    DSDNA_KERNEL_BUILD = 5,   /* neighbour search into the list              */
    DSDNA_NKERNELS = 6
};

typedef struct dsdna_ctx dsdna_ctx; /* opaque */

typedef struct {
    /* Table 2 (Appendix A), simulation units; angles in radians */
    double K1, R0, eps_bb, sig_bb;  /* FENE spring, max length, its WCA core */
    double K2, r0_hb, rc_hb;        /* H-bond strength, rest length, break   */
    double eps, sig_s, sig_x;       /* steric WCA: same-strand sigma (steric
                                       beads), cross-strand sigma (all beads) */
    double K3, d_dih;               /* dihedral strength and phase d         */
    double K4, lam, r0_m;           /* Morse depth, width, rest length       */
    double K5, a0;                  /* planarity stiffness, rest angle       */
    double K6;                      /* Kratky-Porod stiffness                */
    /* Sec. 2: rigid nucleotide: bead-patch distance and site masses */
    double ell, m_bead, m_patch;
    /* Appendix A: friction per site, temperature, time step */
    double gamma, kT, dt;
    uint64_t seed;                  /* key of the Philox noise               */
    int32_t noise_kind;             /* 0: Gaussian (Box-Muller), 1: uniform
                                       with the same variance               */
    int32_t force_fp64;             /* 0: forces in FP32 (positions and the
                                       integrator always FP64); 1: FP64     */
    int32_t ssdna_rule;             /* 1: drop dihedral and bending terms
                                       inside bubbles > 2 bp (Sec. 5)        */
    int32_t hb_depth_convention;    /* 0: H-bond prefactor K2/(2(r0-rc)^2)
                                       as printed; 1: K2/(r0-rc)^2           */
    double cell_size;               /* cell edge of the neighbour search; 0:
                                       1.001 x (largest cutoff + skin)       */
    int32_t hash_log2;              /* log2 of cell-hash buckets; 0: the
                                       power of two >= 4 x nucleotides,
                                       within [12, 24]                      */
    int32_t graph_steps;            /* steps per captured HIP graph; 0 = off */
    int32_t fene_clamp;             /* 0: a backbone bond reaching R0 stops
                                       the run (DSDNA_EBOND); 1: once
                                       1 - r^2/R0^2 falls below 0.1 it is held
                                       there (the force keeps growing with r,
                                       the energy is capped), and only a bond
                                       of 2 R0 stops the run               */
    int32_t dihedral_damping;       /* 0: dihedral as printed; 1: multiplied
                                       by sin^3 of both of its bond angles
                                       (finite gradient at collinear bonds;
                                       1 at the ideal helix)               */
    double skin;                    /* neighbour-list skin: bead pairs more
                                       than 3 base pairs apart are listed
                                       when closer than their WCA cutoff plus
                                       the skin, and the list is rebuilt
                                       once a bead has moved skin/2; 0: 0.5,
                                       else at least 1e-3.
                                       Results do not depend on it.        */
    int64_t list_capacity;          /* initial pairs the neighbour list holds;
                                       0: max(4096, nucleotides / 8).  The
                                       list grows by itself when a rebuild
                                       finds more pairs.                    */
    int32_t planarity_both;         /* 0: one planarity angle per backbone
                                       step and strand, at patch n+1 between
                                       patch n and bead n+1; 1: also the
                                       angle at patch n between patch n+1
                                       and bead n (both triples of the step,
                                       same potential)                     */
} dsdna_params;

/* Table 2 values plus the defaults for what the paper leaves open: unit
 * masses, gamma = 1 (tau_Br = sigma^2/D with D = kT/gamma, Table 3),
 * dt = 0.005 (Appendix A), Gaussian noise, FP32 forces, rule off. */
dsdna_status dsdna_default_params(dsdna_params *out);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on (e.g. a torch stream handle); NULL makes the context create and
 * own a default-priority stream. */
dsdna_status dsdna_create(dsdna_ctx **out, const dsdna_params *params, int device,
                          void *hip_stream);
dsdna_status dsdna_destroy(dsdna_ctx *ctx);
/* Description of the last failure on this context ("" if none); with NULL,
 * of the last failed context-free call on this thread. */
const char *dsdna_last_error(const dsdna_ctx *ctx);

/* Sizes of the current topology: replicas, nucleotides (2 sum n_bp) and base
 * pairs (sum n_bp); any pointer may be NULL.  DSDNA_ESTATE before
 * dsdna_set_topology. */
dsdna_status dsdna_get_sizes(dsdna_ctx *ctx, int32_t *n_rep, int64_t *n_nt, int64_t *n_bp_total);

/* Replica lengths n_bp[n_rep] (each >= 1).  Allocates device memory for
 * sum 2 n_bp nucleotides.  Resets boxes to open, loads to zero, K2 scales
 * to 1. */
dsdna_status dsdna_set_topology(dsdna_ctx *ctx, int32_t n_rep, const int32_t *n_bp);

/* Per-replica box lo_hi[n_rep][6] (lo x, y, z, hi x, y, z) and periodic
 * flags periodic[n_rep][3] (0/1).  Periodic dimensions wrap pair distances
 * (minimum image); positions are kept unwrapped.  For open dimensions lo
 * is the origin of single-precision neighbour coordinates (beads must stay
 * within 8192 of it).  A periodic edge must hold at least 3 cells. */
dsdna_status dsdna_set_box(dsdna_ctx *ctx, const double *lo_hi, const uint8_t *periodic);

/* External loads of replica `rep` (Sec. 4): pulling force F[3] on the last
 * base pair (half on each patch), torque G[3] applied as a couple on the two
 * beads of the last base pair, and anchoring (tether != 0: the first base
 * pair is fixed and every bead feels a WCA wall, sigma = sig_s, at z = wall_z). */
dsdna_status dsdna_set_external(dsdna_ctx *ctx, int32_t rep, const double F[3],
                                const double G[3], int32_t tether, double wall_z);

/* Sequence-specific base pairing (Sec. 5, K2(AT) < K2(CG)): scale[n_bp_total]
 * multiplies K2 of each base pair, in replica order then bp order, on top of
 * the per-replica dsdna_set_k2_scale.  NULL removes the table (every base
 * pair then has multiplier 1).  Entries must be finite and >= 0
 * (DSDNA_EINVAL).  The table is copied; set_topology removes it, and so does
 * a failed copy. */
dsdna_status dsdna_set_k2_bp(dsdna_ctx *ctx, const double *scale);

/* Close replicas into rings (Sec. 4.2, circular DNA): circular[n_rep], 1 for
 * a ring, in which base pair n_bp-1 is bonded to base pair 0 on both
 * strands.  Every backbone step (FENE + core, stacking, dihedral,
 * planarity) then includes the seam step n_bp-1 -> 0, there is a bending
 * triple centred on every base pair, and the single-strand rule reads
 * bubbles cyclically.  A ring needs n_bp >= 6 and n_bp a multiple of 3 (the
 * steric beads, every third base pair, stay every third across the seam)
 * and takes no external loads; either is DSDNA_EINVAL.  The flag of every
 * replica is replaced by this call; set_topology clears all of them.  On
 * any failure the previous rings stay as they were.
 * Placing the sites so that the ring closes is the caller's concern. */
dsdna_status dsdna_set_circular(dsdna_ctx *ctx, const uint8_t *circular);

/* Topology of every replica from the current state (appendix on the
 * closure procedure, Gauss's double integral): lk[n_rep] = linking number of
 * the closed curves of the strand 0 and strand 1 beads, both oriented along
 * increasing base pair (a relaxed right-handed duplex has Lk ~ +n_bp/10);
 * wr[n_rep] = writhe of the centreline through the midpoints of the paired
 * patches (Sec. 3.1).  The twist is Lk - Wr.  A ring's curves are closed by
 * its seam.  A linear replica's strands are closed as the appendix
 * describes: each is extended outwards from both ends along the unit
 * tangent of its terminal bead pair by ten relaxed contour lengths
 * (10 x 0.34 nm x n_bp) and the two far points are joined by a straight
 * segment; its centreline is left open (wr is the integral over the open
 * polygon's pairs of segments).  Both are computed exactly for the polygons
 * (the sum over segment pairs of signed solid angles, FP64), so lk is an
 * integer up to rounding while the closed strands do not cross.  A replica
 * of one base pair gets NaN.  pair_ms (may be NULL) receives the duration of
 * the segment-pair kernel in milliseconds.  Runs on the context's stream
 * after the steps already queued.  The curve buffers (72 bytes per base
 * pair) are allocated at the first call after set_topology or
 * set_circular: DSDNA_ENOMEM if that fails. */
dsdna_status dsdna_get_linking(dsdna_ctx *ctx, double *lk, double *wr, double *pair_ms);

/* The tiling of the step kernel: base pairs per tile, threads per workgroup
 * (one per site of the tile plus its halo, a build constant) and the number
 * of tiles of the current topology (a replica starts a new tile).  Any
 * pointer may be NULL.  DSDNA_ESTATE before set_topology. */
dsdna_status dsdna_get_tiling(dsdna_ctx *ctx, int32_t *tile_bp, int32_t *wg_threads, int64_t *n_tiles);

/* Multiply K2 of each replica by scale[n_rep] (denaturation, Sec. 5). */
dsdna_status dsdna_set_k2_scale(dsdna_ctx *ctx, const double *scale);

/* Temperature kT used by the noise from the next step on. */
dsdna_status dsdna_set_temperature(dsdna_ctx *ctx, double kT);

/* Positions of all beads and patches (bead[N][3], patch[N][3]).  Each body
 * gets R = centre of mass and u = unit vector bead -> patch; the sites are
 * then placed ell apart on u.  Velocities are set to zero and the step
 * counter to 0. */
dsdna_status dsdna_set_sites(dsdna_ctx *ctx, const double *bead, const double *patch);

/* Body velocities V[N][3] and angular momenta L[N][3] at the current step
 * (the component of L along the body axis is removed). */
dsdna_status dsdna_set_velocities(dsdna_ctx *ctx, const double *V, const double *L);

/* Maxwell-Boltzmann velocities at kT from noise stream 1 keyed by `seed`:
 * V ~ N(0, kT/M) per component, L ~ N(0, I kT) per component minus its
 * part along u.  Anchored bodies get zero. */
dsdna_status dsdna_thermalize(dsdna_ctx *ctx, double kT, uint64_t seed);

/* Advance n_steps >= 0 time steps.  Enqueued on the stream; returns after
 * reading the device status word once.  On DSDNA_EBOND / DSDNA_ENAN /
 * DSDNA_EWALL / DSDNA_EDOMAIN / DSDNA_ECELL the remaining steps are skipped and
 * the state is left at the step where the error was found. */
dsdna_status dsdna_step(dsdna_ctx *ctx, int64_t n_steps);

/* Current full-step state: body centres R, velocities V, axes u, angular
 * momenta L ([N][3] each, any may be NULL) and the step counter. */
dsdna_status dsdna_get_state(dsdna_ctx *ctx, double *R, double *V, double *u, double *L,
                             int64_t *step);
/* Replace the full-step state (arrays as in dsdna_get_state).  The next step
 * evaluates forces at this state first (friction from V). */
dsdna_status dsdna_set_state(dsdna_ctx *ctx, const double *R, const double *V, const double *u,
                             const double *L, int64_t step);

/* Bind caller-owned device arrays as the full-step state (App. A: centres
 * R, velocities V, axes u, angular momenta L of the rigid nucleotides), so
 * that device memory from another allocator (torch tensors, say) holds the
 * state with no host copy.
 *   R, V, u, L: FP64 device memory of the context's device, each 3N doubles,
 *     component-major: element k * N + i is component k of nucleotide i (a
 *     contiguous (3, N) array, the layout the step kernel works in); four
 *     distinct, non-overlapping arrays.
 *   Binding makes the arrays' contents the state (as dsdna_set_state, keeping
 *   the step counter): the next step starts from a force evaluation there.
 *   From then on every call that changes the state (dsdna_step, _thermalize,
 *   _set_velocities, _set_state, _set_sites, _set_resume) leaves the
 *   full-step state in the arrays before it returns, also when a step fails
 *   with DSDNA_EBOND etc. (the state the error left).  The step kernel writes
 *   the full-step velocities straight into V and L, and R and u on the last
 *   step of each call.  After writing into the arrays, bind them again (the
 *   same pointers will do) for the context to take the new contents.
 *   All four NULL: unbind; the context keeps the current state.
 *   Ownership: the arrays stay the caller's; they must outlive the binding
 *   (dsdna_set_topology and dsdna_destroy end it).  Work on other streams
 *   that touches them must be ordered with the context's stream by the caller.
 * Errors: DSDNA_EINVAL when only some pointers are NULL, when an array is not
 * device memory of the context's device, has fewer than 3N doubles up to the
 * end of its allocation, or overlaps another; nothing is changed then. */
dsdna_status dsdna_bind_device(dsdna_ctx *ctx, double *R, double *V, double *u, double *L);

/* Exact resume point: the full-step state plus the total site forces
 * (f_bead, f_patch [N][3], including the Langevin forces) that the next half
 * kick uses.  Restoring it with dsdna_set_resume continues the trajectory
 * bit for bit.  Needs at least one step since the last set_state/set_sites. */
dsdna_status dsdna_get_resume(dsdna_ctx *ctx, double *R, double *V, double *u, double *L,
                              double *f_bead, double *f_patch, int64_t *step);
dsdna_status dsdna_set_resume(dsdna_ctx *ctx, const double *R, const double *V,
                              const double *u, const double *L, const double *f_bead,
                              const double *f_patch, int64_t step);

/* Site positions of the current state (bead[N][3], patch[N][3]). */
dsdna_status dsdna_get_sites(dsdna_ctx *ctx, double *bead, double *patch);

/* Conservative and external site forces of one term (DSDNA_TERM_*), or of
 * all terms summed (term = -1), at the current positions, computed by the
 * same device code as the step in the context's precision. */
dsdna_status dsdna_get_forces(dsdna_ctx *ctx, int32_t term, double *f_bead, double *f_patch);

/* Energies E[n_rep][DSDNA_NENERGY] at the current state: the potential
 * terms and the kinetic energies of the full-step velocities, each summed
 * per replica on the device in a fixed order. */
dsdna_status dsdna_get_energies(dsdna_ctx *ctx, double *E);

/* Open flags (H-bond beyond r_c) of every base pair, open[sum n_bp]. */
dsdna_status dsdna_get_bp_open(dsdna_ctx *ctx, uint8_t *open);

/* Bubble statistics of Sec. 5 per replica, computed on the device: frac[n_rep]
 * = fraction of open base pairs; hist[n_rep][nhist] = number of maximal open
 * runs of length k (k < nhist; longer runs counted in nhist-1); on a ring
 * runs are cyclic and an all-open ring is one run.  2 <= nhist <= 4096. */
dsdna_status dsdna_get_bubbles(dsdna_ctx *ctx, int32_t nhist, double *frac, int64_t *hist);

/* Run n_steps steps with a HIP event pair around every kernel launch and
 * return the mean duration in milliseconds of each DSDNA_KERNEL_* class
 * (ms[DSDNA_NKERNELS]).  The steps advance the state like dsdna_step. */
dsdna_status dsdna_profile_kernels(dsdna_ctx *ctx, int64_t n_steps, double *ms);

/* Neighbour list (Sec. 6: short-range neighbour search without O(N^2)
 * loops): bead pairs more than 3 base pairs apart along the chain within
 * their WCA cutoff plus the skin, rebuilt from a counting-sort cell list
 * every `interval` steps.  The interval adapts so that no bead moves three
 * quarters of half the skin between rebuilds; a bead that moves half the
 * skin before its rebuild (an outrun) stops the queued steps, and the list
 * is rebuilt there and the run continues (the results do not depend on the
 * skin or the interval).  Since the last state change (set_sites, set_state,
 * thermalize, ...): rebuilds (including the one that preceded the first
 * step), steps taken, outruns; and now: pairs in the list, the skin, the
 * interval.  Any pointer may be NULL. */
dsdna_status dsdna_get_neighbour_stats(dsdna_ctx *ctx, int64_t *rebuilds, int64_t *steps, int64_t *outruns,
                                       int64_t *pairs, double *skin, int32_t *interval);

/* Sizes chosen for the cell list: cell edge, number of hash buckets and
 * cells per periodic dimension of replica 0 (cells[3], 0 for open). */
dsdna_status dsdna_get_grid(dsdna_ctx *ctx, double *cell_size, int64_t *n_buckets,
                            int32_t *cells);

/* Autotuner of the neighbour search (Sec. 6): every combination of a skin,
 * a cell edge (a factor >= 1.001 times the search reach, the largest WCA
 * cutoff plus the skin) and a bucket count is run for warm_steps untimed
 * steps (the rebuild interval settles) and trial_steps timed ones on the
 * current state, and the fastest is kept.  NULL or 0-length lists mean the
 * context's current value.  The trial steps advance the state.  With
 * use_cache, the choice is remembered for the rest of the process, keyed by
 * (nucleotides, replicas, bead density of periodic boxes, open or periodic,
 * force precision), and a later call with the same key takes it without
 * trials; if the environment variable DSDNA_TUNE_CACHE names a file, choices
 * are also read from and appended to it.  On failure the previous settings
 * are restored. */
typedef struct {
    int32_t n_skins;
    const double *skins;
    int32_t n_cell_factors;
    const double *cell_factors;
    int32_t n_hash_log2s;
    const int32_t *hash_log2s;
    int64_t warm_steps;
    int64_t trial_steps;
    int32_t use_cache;
} dsdna_tune_space;

typedef struct {
    double skin;
    double cell_size;
    int32_t hash_log2;
    int32_t interval;       /* rebuild interval at the end of the winner's trial */
    double ms_per_step;     /* the winner's trial (0 when taken from the cache) */
    int32_t candidates;     /* combinations timed */
    int32_t from_cache;     /* 1: taken from the cache, no trials */
} dsdna_tune_result;

dsdna_status dsdna_autotune(dsdna_ctx *ctx, const dsdna_tune_space *space, dsdna_tune_result *best);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * linking number and writhe of one ring given as three closed curves, the
 * computation dsdna_get_linking performs for the rings of a context, with no
 * context and no allocation.  Its per-workgroup partial sums live in a fixed
 * device array inside the library (2 doubles per 256 points, at most
 * DSDNA_NOALLOC_MAX_POINTS points: 64 KiB per GPU, held until the process
 * ends).
 *   A, B: DEVICE pointers to the two strand curves, C: to the centreline,
 *         each n points [n][3] of FP64, closed (point n-1 joins point 0);
 *   out:  DEVICE pointer to 2 doubles, receives Lk(A, B) and Wr(C) as
 *         dsdna_get_linking defines them;
 *   stream: hipStream_t of the current device (NULL: the null stream).
 * Runs on the current HIP device, asynchronously on `stream`; the caller
 * keeps the buffers alive until the work completes.  Calls whose work
 * overlaps on one GPU share the fixed array and race: serialise them (one
 * stream, or events).  The first call on each device resolves the array's
 * address; make it outside a stream capture.  n outside [3,
 * DSDNA_NOALLOC_MAX_POINTS] or a NULL pointer is DSDNA_EINVAL,
 * dsdna_last_error(NULL) describes the failure. */
#define DSDNA_NOALLOC_MAX_POINTS 1048576
dsdna_status dsdna_linking_curves_noalloc(const double *A, const double *B, const double *C, int64_t n,
                                          double *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DSDNA_H */
